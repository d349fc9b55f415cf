/* Modified Stokes double-layer operator on the MAC grid (gfx950).
 *
 * Sec. 3.3 (eq. ms-bie): the flow part of a time step is the double-layer potential
 * D phi = (D_u phi, D_p phi) of a vector density phi on the interface, for the modified
 * Stokes operator (Delta - c^2) u - grad p, div u = 0 with the Green's function that
 * vanishes on the box; the density solves -phi/2 + D_u phi = -u1 on the interface.
 * As in Sec. 4.1, D phi is evaluated through its equivalent interface problem (App. A.2
 * with [u] = phi, [T(u, p)] = 0, no forcing, zero velocity on the box), discretised by the
 * corrected MAC scheme of Sec. 4.2.2 (eq. crc-mac-fds), with the jumps of App. A.2, and
 * the velocity traces at the markers by the corrected interpolation of Sec. 4.3 applied
 * to each velocity component on its own staggered grid.
 *
 * The MAC system is solved exactly (to a relative residual tolerance) by preconditioned
 * conjugate gradients on the pressure Schur complement: velocity solves by sine
 * transforms (DST-I along the normal direction, DST-II along the tangential one), the
 * Cahouet-Chabard preconditioner c^2 L^-1 + I with L the cell Laplacian of zero normal
 * flux (DCT-II in both directions).  The paper uses geometric multigrid instead.
 *
 * Grid (Sec. 4.2.2): h = side / N; u at (x0 + i h, y0 + (j - 1/2) h), i = 0..N, j = 1..N;
 * v at (x0 + (i - 1/2) h, y0 + j h), i = 1..N, j = 0..N; p at cell centres, i, j = 1..N.
 * Markers as in kfbi.h: X_k at a_k = 2 pi k / M, counter-clockwise, [w] = w(inside) -
 * w(outside), outward normal; every marker at least 3h from the box boundary.
 *
 * All arrays are caller-owned device memory (FP64) unless noted; calls are ordered on the
 * context's stream and return KFBI_OK or a KFBI_E_* code (kfbi.h) with the message in
 * kfbi_last_error().  stokes_create and stokes_set_interface allocate; the other calls
 * allocate nothing. */
#ifndef STOKES_H
#define STOKES_H

#include "kfbi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stokes_ctx stokes_ctx;

typedef struct {
  double x0, y0, side; /* box [x0, x0 + side] x [y0, y0 + side] */
  int N;               /* intervals per side, a power of two, 32 <= N <= 1024 */
  double c2;           /* c^2 >= 0 of (Delta - c^2) */
  int max_markers;     /* largest M of stokes_set_interface, <= 2048 */
  void* stream;        /* hipStream_t, or NULL for the null stream */
  double solve_tol;    /* relative residual of the Schur-complement CG (e.g. 1e-13) */
  int solve_maxit;     /* its iteration limit */
} stokes_params;

typedef struct {
  int M;                /* markers of the installed interface */
  int n_crossings;      /* interface crossings with the lines of the half-spacing grid */
  int cg_iters;         /* CG iterations of the last apply */
  double cg_relres;     /* its final relative residual */
} stokes_info;

/* KFBI_E_INVALID for parameters outside the ranges above (or c2 < 0, side <= 0,
 * solve_tol <= 0, solve_maxit < 1); KFBI_E_HIP when a device or pinned host allocation
 * fails.  *out is NULL on error. */
int stokes_create(const stokes_params* p, stokes_ctx** out);
int stokes_destroy(stokes_ctx* st);

/* Install the interface: xy_dev [2][M] (x then y), M even, 16 <= M <= max_markers.
 * Builds labels and crossings of the half-spacing grid (whose nodes are the u, v and p
 * points) and the marker geometry.  KFBI_E_GEOMETRY for markers closer than 3h to the
 * box or a curve the grid does not resolve. */
int stokes_set_interface(stokes_ctx* st, int M, const double* xy_dev);

/* D phi for phi_dev [2][M] (phi_1 at the markers, then phi_2): the velocity traces from
 * inside (u_plus_dev [2][M]) and from outside (u_minus_dev [2][M]); either may be NULL.
 * The MAC fields of the solution stay in the context (stokes_fields). */
int stokes_apply(stokes_ctx* st, const double* phi_dev, double* u_plus_dev,
                 double* u_minus_dev);
/* Errors of stokes_apply (and of stokes_operator, stokes_gmres_solve): KFBI_E_STATE with no
 * interface installed; KFBI_E_NOCONV when the CG reaches solve_maxit iterations above
 * solve_tol (stokes_get_info reports the iterations and the residual reached);
 * KFBI_E_NONFINITE for a non-finite CG residual; KFBI_E_GEOMETRY when a MAC stencil pair and
 * the interface crossings disagree.  The call returns after the GPU work has finished. */

/* The MAC fields of the last apply: u_dev [N][N+1] (row j - 1, column i = 0..N), v_dev
 * [N+1][N] (row j = 0..N, column i - 1), p_dev [N][N] (row j - 1, column i - 1, mean
 * zero); any may be NULL. */
int stokes_fields(stokes_ctx* st, double* u_dev, double* v_dev, double* p_dev);

/* Left-hand side of eq. ms-bie, y = -x/2 + D_u x = trace of D x from outside, for
 * x_dev, y_dev [2M] (component 1 at the markers, then component 2). */
int stokes_operator(stokes_ctx* st, const double* x_dev, double* y_dev);

/* Solve -phi/2 + D_u phi = rhs (eq. ms-bie) by restarted GMRES (FP64; opts->precision
 * must be KFBI_FP64) from the initial guess in x_dev [2M]; kfbi_gmres_stats as in kfbi.h. */
int stokes_gmres_solve(stokes_ctx* st, const double* rhs_dev, double* x_dev,
                       const kfbi_gmres_opts* opts, kfbi_gmres_stats* stats);

int stokes_get_info(const stokes_ctx* st, stokes_info* info);

#ifdef __cplusplus
}
#endif
#endif /* STOKES_H */
