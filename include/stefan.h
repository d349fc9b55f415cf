/*
 * stefan.h -- C ABI of the Stefan problem (solidification with a Gibbs-Thomson interface)
 * on MI355X (gfx950), built on kfbi.h and the theta-L evolution of thetal.h.
 *
 * Model (Sec. 2.2 and 3.2): solid Omega+ inside the interface, undercooled liquid Omega-
 * outside, heat equation in both phases, zero normal derivative of the temperature on the
 * box.  Each step discretises the heat equation in time,
 *     backward Euler  (Delta - 1/tau) T^{n+1} = -T^n / tau,
 *     BDF2            (Delta - 3/(2 tau)) T^{n+1} = (T^{n-1} - 4 T^n) / (2 tau),
 * (c^2 the constant on the left; BDF2 starts with T^{-1} = T^0) and splits
 * T^{n+1} = T1 + T2: T1 solves the five-point problem on the box with the right-hand side
 * above, T2 = -S psi is the single layer of the box Green's function (KFBI_BOX_NEUMANN) with
 * psi = [d_n T] = U, the normal velocity.  The Gibbs-Thomson relation gives
 *     eps_V psi - S psi = -eps_C kappa - T1       on Gamma     (eq. bie-GT),
 * solved by kfbi_gmres_solve with {SINGLE, AVG, a_marker = eps_V, b = -1, q = 0}.  The
 * interface then moves with U by the theta-L equations (Sec. 5.1) with the small-scale
 * decomposition of Sec. 5.2.2: ssd = 1 treats lambda_1 (2pi/L)^2 theta_aa implicitly
 * (eps_V = O(1)), ssd = 2 lambda_2 (2pi/L)^3 H[theta_aaa] (eps_V << 1), both by the
 * integrating factor of eq. Fourier-theta1/2 with Adams-Bashforth 2 (Euler first step).
 *
 * Readings (the same in the CPU reference): the equation of step n is posed on the
 * interface of step n; T1 at the markers is the Sec. 4.3 six-point interpolation with zero
 * jumps; anisotropy eps(n) = e0 (1 + e1 cos(m (phi - phi0)) + e2 cos(2 m (phi - phi0))) of
 * the angle phi of the outward normal; lambda_1 = max |eps_C / eps_V| and
 * lambda_2 = max |2 eps_C| over phi sampled at 4096 equispaced angles.
 *
 * The temperature is held as cosine coefficients along x for every grid row (the layout of
 * the column solve), so that the T1 solve is one column solve of a dense right-hand side
 * and T^{n+1} one column solve of that right-hand side plus the interface corrections; the
 * grid values are formed only on request (stefan_temperature).
 * Conventions as in kfbi.h (device pointers *_dev, host structs, KFBI_* status codes).
 */
#ifndef STEFAN_H
#define STEFAN_H

#include "thetal.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stefan stefan;

typedef struct {
  double e0, e1, e2;     /* eps(phi) = e0 (1 + e1 cos(m (phi - phi0)) + e2 cos(2m (phi - phi0))) */
  int m;
  double phi0;
} stefan_aniso;

typedef struct {
  double x0, y0, side;   /* box [x0, x0+side]^2                                            */
  int N;                 /* grid intervals per side (power of two, 64..2048)                */
  int M;                 /* markers: a power of two, 16 <= M <= 2048                        */
  double tau;            /* time step                                                       */
  int bdf2;              /* 1: BDF2 (c^2 = 3/(2 tau)), 0: backward Euler (c^2 = 1/tau)       */
  int ssd;               /* 1 or 2: the implicit term (see above)                           */
  double lambda;         /* SSD constant; <= 0 selects the frozen-coefficient maximum       */
  stefan_aniso eps_c;    /* surface tension eps_C                                           */
  stefan_aniso eps_v;    /* kinetic coefficient eps_V (e0 > 0 with ssd = 1)                  */
  kfbi_gmres_opts gmres; /* options of the per-step GMRES solve                             */
  void* stream;          /* hipStream_t (NULL = default stream)                             */
  double refine;         /* marker refinement ratio as thetaL_params.refine (0 = off)        */
  int max_M;             /* refinement limit (power of two, M..2048; 0 = M)                 */
} stefan_params;

typedef struct {
  int step;              /* index n of the step just taken                                  */
  double t;              /* time after the step                                             */
  int iters, applies64, applies32;
  double relres;         /* final true FP64 relative residual of eq. bie-GT                 */
  double area, length;   /* of the interface the step was solved on                         */
  double ms_geometry, ms_temperature, ms_gmres, ms_update;  /* geometry, GMRES: host
                            wall clock (GMRES also waits for the temperature kernels queued
                            before it); temperature (T1 and its trace) and update (T^{n+1},
                            theta-L): GPU time between events                               */
  int M, M_next;         /* markers of the step and after it (refinement doubles M)        */
} stefan_stats;

int stefan_create(const stefan_params* params, stefan** out);
int stefan_destroy(stefan* st);

/* Start: the interface from a closed counter-clockwise curve sampled at Mi equispaced
 * parameter values (as thetaL_init), the temperature from T0_dev ((N+1)^2 grid values,
 * row-major j (N+1) + i), or, with T0_dev NULL, the seed field: 0 at the nodes inside the
 * (resampled) curve and St outside.  Synchronises. */
int stefan_init(stefan* st, int Mi, const double* xy_dev, const double* T0_dev, double St);

/* One step (x0_dev: initial guess of psi, M doubles, or NULL for the last density).
 * Synchronises.  Errors as thetaL_step. */
int stefan_step(stefan* st, const double* x0_dev, stefan_stats* stats);
int stefan_run(stefan* st, int nsteps, stefan_stats* stats);

/* Grid temperature ((N+1)^2 doubles, row-major) of the current state; asynchronous. */
int stefan_temperature(stefan* st, double* grid_dev);
/* Markers (2M doubles) and the last density psi = U (M doubles); asynchronous. */
int stefan_markers(stefan* st, double* xy_dev);
int stefan_density(const stefan* st, double* psi_dev);
/* eta, L, Xbar and the time of the interface state (eta_dev: M doubles; scal_host: L, Xbar_x,
 * Xbar_y, t).  Synchronises. */
int stefan_interface(const stefan* st, double* eta_dev, double* scal_host);
/* The SSD constant in use, and the squared operator constant c^2 of the temperature step. */
int stefan_constants(const stefan* st, double* lambda, double* c2);
/* Current number of markers. */
int stefan_size(const stefan* st, int* M);
/* The theta-L state of the interface, owned by st: pass it to kfbi_ws_predict (before
 * stefan_step, whose x0_dev then takes the guess) and kfbi_ws_record (after it) of
 * warmstart.h for the learned initial guess of psi (the densities of the previous steps
 * play the part of the Hele-Shaw phi). */
thetaL* stefan_thetal(stefan* st);

#ifdef __cplusplus
}
#endif
#endif /* STEFAN_H */
