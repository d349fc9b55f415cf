/*
 * thetal.h -- C ABI of the theta-L / small-scale-decomposition interface evolution for
 * the Hele-Shaw problem on MI355X (gfx950), built on kfbi.h.
 *
 * Model (Sec. 2.1 and 3.1): the pressure outside the bubble is p = v + w with the
 * injection part v = -J ln|x| and w = D phi + int phi ds, where the double-layer density
 * phi solves the boundary integral equation (eq. bie-HS)
 *      -phi/2 + D phi + int phi ds = -sigma kappa - v      on Gamma,
 * discretised by the KFBI apply with the free-space box data (Sec. 4.1) and solved by
 * matrix-free GMRES.  The normal velocity is U = J (x.n)/|x|^2 - d_n(D phi).
 * Evolution (Sec. 5.1-5.3): the curve is held in equal-arclength theta-L variables,
 * eta = theta - alpha, length L and centroid Xbar; V is the tangential velocity that
 * keeps the parametrisation equal in arclength (eq. L-evo, the-evo); the stiff
 * surface-tension term lambda2 (2 pi/L)^3 H[theta_aaa] is treated by an integrating
 * factor in Fourier space with second-order Adams-Bashforth for the rest
 * (eq. Fourier-theta2); L and Xbar advance by Adams-Bashforth 2.  The first step uses
 * the integrating-factor forward Euler step.
 *
 * Readings where the text is silent or inconsistent (the same in the CPU reference):
 *  - theta_t follows eq. the-evo (the form in which L_2 damps);
 *  - L and Xbar use L^{n+1} = L^n + (tau/2)(3 M^n - M^{n-1}) with M = int theta_a U;
 *  - U uses the average of the two one-sided normal derivatives of D phi;
 *  - the reconstruction X = Xbar + (L/2pi) * mean-free antiderivative of
 *    (cos theta, sin theta); Nyquist modes are zeroed in every spectral operation.
 *
 * Adaptive marker refinement (Sec. 6.1, long-time computation): with refine > 0, after
 * a step whose new length gives a marker spacing L/M above refine * h, M is doubled (up
 * to max_M); eta, the last two densities and the history of the explicit term are
 * carried to the doubled parameter grid by trigonometric interpolation (zero padding in
 * Fourier space).  The paper fixes only the criterion (refine = 1.5 there).
 *
 * Every spectral operation runs in FP64 on the GPU (single-workgroup LDS FFTs); the
 * pressure solve uses kfbi_gmres_solve with the options given at creation (its FP32
 * inner mode keeps the FP64 residual tolerance).  Conventions as in kfbi.h: *_dev are
 * caller-owned device pointers, structs are host memory, status codes are KFBI_*.
 */
#ifndef THETAL_H
#define THETAL_H

#include "kfbi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct thetaL thetaL;

typedef struct {
  kfbi_grid grid;        /* box and grid of the pressure solve: box_bc must be
                            KFBI_BOX_FREESPACE and c2 = 0 (Laplace); grid.max_markers is
                            ignored (M is used)                                          */
  int M;                 /* markers: a power of two, 16 <= M <= 2048                     */
  double sigma;          /* surface tension                                              */
  double J;              /* injection rate                                               */
  double tau;            /* time step                                                    */
  double lambda2;        /* SSD constant of the stiff term; a negative value selects sigma */
  kfbi_gmres_opts gmres; /* options of the per-step GMRES solve                          */
  double refine;         /* marker refinement ratio (0 = off; > 0: double M when
                            L/M > refine * h)                                           */
  int max_M;             /* largest M refinement may reach (a power of two, M <= max_M
                            <= 2048; 0 = M)                                             */
} thetaL_params;

/* Per-step record (host).  area and length describe the curve at the start of the step
 * (the curve the pressure was solved on).  ms_geometry and ms_gmres are host wall clock
 * (each ends with a stream synchronisation); ms_apply (the velocity apply) and ms_update
 * are GPU time between events, since the step runs them back to back without a host
 * synchronisation. */
typedef struct {
  int step;              /* index n of the step just taken, from 0                       */
  double t;              /* time after the step                                          */
  int iters;             /* GMRES Arnoldi steps of the pressure solve                    */
  int applies64, applies32;
  double relres;         /* final true FP64 relative residual                            */
  double area, length;
  double ms_geometry, ms_gmres, ms_apply, ms_update;
  int M;                 /* markers of this step                                         */
  int M_next;            /* markers after it (2M when the step ended with a refinement)  */
} thetaL_stats;

/* Checkpoint of the evolution.  Arrays are caller-owned device arrays sized for the
 * current M (thetaL_size); scal is host. */
typedef struct {
  double* eta_dev;       /* [M] eta = theta - alpha                                      */
  double* phi_prev_dev;  /* [M] density of the last solve (next initial guess)            */
  double* phi_prev2_dev; /* [M] density of the solve before it (zero if none)              */
  double* nhat_prev_dev; /* [2M] DFT of the last explicit term, (re, im) interleaved      */
  double scal[8];        /* L, Xbar_x, Xbar_y, t, L_prev, M_prev, Qbar_prev_x, Qbar_prev_y */
  int n;                 /* steps taken                                                  */
  int M;                 /* markers of the state (set_state: 0 = the current M; else a
                            power of two in [16, max_M])                                 */
} thetaL_state;

/* Create an evolution object (and its KFBI context).  KFBI_E_INVALID on bad params. */
int thetaL_create(const thetaL_params* params, thetaL** out);
int thetaL_destroy(thetaL* th);

/* Start from a closed counter-clockwise curve sampled at Mi equispaced parameter values
 * (xy_dev: x[0..Mi) then y[0..Mi), Mi even, 16 <= Mi <= 4096): resample to M points
 * equispaced in arclength (Newton on the trigonometric interpolant of the arclength
 * function), set eta, L, Xbar, time 0, step count 0, zero previous density.  Syncs. */
int thetaL_init(thetaL* th, int Mi, const double* xy_dev);

/* Current number of markers (changes only by refinement, thetaL_init keeps it). */
int thetaL_size(const thetaL* th, int* M);

/* One time step.  x0_dev: initial guess of the pressure density (M doubles) or NULL for
 * the previous step's density (zero at the first step); GMRES always runs to the same
 * FP64 residual tolerance, so the guess changes the iteration count only.  Re-installs
 * the interface in the KFBI context (its geometry workspaces may grow), solves, applies
 * once more for d_n(D phi), advances the state, then refines the markers if due.
 * Synchronises.  Errors: KFBI_E_NOCONV
 * (the state is left unchanged), KFBI_E_GEOMETRY (curve not resolvable, unchanged),
 * KFBI_E_NONFINITE (the new state is not finite). */
int thetaL_step(thetaL* th, const double* x0_dev, thetaL_stats* stats);

/* nsteps steps with the previous-density initial guess; stats: nsteps records or NULL.
 * Stops at the first failing step and returns its status. */
int thetaL_run(thetaL* th, int nsteps, thetaL_stats* stats);

/* Current markers X(alpha_k) (xy_dev: 2M doubles, x then y), and the density of the last
 * solve (phi_dev: M doubles).  Asynchronous. */
int thetaL_markers(thetaL* th, double* xy_dev);
int thetaL_density(const thetaL* th, double* phi_dev);

/* The KFBI context used for the pressure solves (owned by th). */
kfbi_ctx* thetaL_kfbi(thetaL* th);

/* Checkpoint / restart: copy the state out to / in from caller arrays.  Synchronises. */
int thetaL_get_state(const thetaL* th, thetaL_state* st);
int thetaL_set_state(thetaL* th, const thetaL_state* st);

#ifdef __cplusplus
}
#endif
#endif /* THETAL_H */
