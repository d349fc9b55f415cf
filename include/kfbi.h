/*
 * kfbi.h -- C ABI of the MI355X (gfx950) kernel-free boundary integral library.
 *
 * Method: Zhou, Li, Ying, "A Cartesian grid-based boundary integral method for moving
 * interface problems".  A boundary integral operator (single/double layer of the
 * Laplace or modified-Helmholtz operator Delta - c^2) is applied by solving its
 * equivalent interface problem on a fixed Cartesian grid (Sec. 4.1, eq. kfbi-ifp and
 * Table 2): jump-corrected five-point right-hand sides at irregular nodes (Sec. 4.2.1,
 * eq. modified-fdm, jumps from App. A.1), a fast solve, and jump-corrected polynomial
 * interpolation of the one-sided traces (Sec. 4.3).  The discrete boundary integral
 * equation is solved by matrix-free GMRES (Sec. 4, opening), and the interface evolves
 * by the theta-L / small-scale decomposition scheme (Sec. 5).
 *
 * Conventions for every entry point:
 *  - Array arguments named *_dev are caller-owned DEVICE pointers (e.g. the data_ptr()
 *    of a torch tensor on the same GPU); the library never frees them.  Structs
 *    (grid, options, statistics, state) live in HOST memory.
 *  - All device work is enqueued on the context's HIP stream (kfbi_grid.stream; NULL
 *    = the default stream).  kfbi_apply is asynchronous; kfbi_set_interface,
 *    kfbi_gmres_solve and thetaL_step synchronise that stream before returning.
 *  - The library owns its workspaces: they are allocated in kfbi_create (the GMRES
 *    Krylov basis for max_markers and the largest restart among them) and grown only
 *    in kfbi_set_interface; kfbi_apply and kfbi_gmres_solve allocate nothing.
 *  - Errors: every call returns a KFBI_* status; no exception crosses the ABI; outputs
 *    are unspecified on error; kfbi_last_error() gives a thread-local message.
 *  - A context is used by one host thread at a time.
 */
#ifndef KFBI_H
#define KFBI_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define KFBI_OK 0
#define KFBI_E_INVALID 1    /* bad argument (null pointer, size out of range, ...)      */
#define KFBI_E_GEOMETRY 2   /* interface not resolvable on the grid (see set_interface) */
#define KFBI_E_NOCONV 3     /* GMRES hit maxit before the tolerance                    */
#define KFBI_E_HIP 4        /* a HIP runtime call failed                                */
#define KFBI_E_NOMEM 5      /* device allocation failed                                 */
#define KFBI_E_NONFINITE 6  /* NaN/Inf met in a residual or state                       */
#define KFBI_E_STATE 7      /* call order violated (e.g. apply before set_interface)    */

/* layer potentials (Table 2: S -> jumps (0, -psi), D -> jumps (phi, 0)) */
#define KFBI_SINGLE 0
#define KFBI_DOUBLE 1
/* which boundary value enters the operator (Sec. 4.3: boundary operator = average) */
#define KFBI_PLUS 0         /* limit from the interior Omega+ */
#define KFBI_MINUS 1        /* limit from the exterior Omega- */
#define KFBI_AVG 2          /* (v+ + v-)/2                    */
/* box boundary data */
#define KFBI_BOX_ZERO 0      /* homogeneous Dirichlet box (box Green's function)              */
#define KFBI_BOX_USER 1      /* caller supplies the box values with each apply               */
#define KFBI_BOX_FREESPACE 2 /* free-space layer potential on the box by the trapezoidal rule
                                (Sec. 4.1, Hele-Shaw); requires c2 == 0                     */
#define KFBI_BOX_NEUMANN 3   /* zero normal derivative on the box (the Stefan problem's box
                                Green's function, Sec. 3.2): the five-point scheme holds at
                                every node (i, j = 0..N) with ghost values mirrored across
                                the box, solved by the cosine transform; requires c2 > 0.
                                The grid output then holds the solution on the box too. */
/* arithmetic of the grid stages (jumps, corrections, solve, interpolation) */
#define KFBI_FP64 0
#define KFBI_FP32 1
/* GMRES only: FP64 GMRES whose operator applies switch to FP32 as the residual falls */
#define KFBI_MIXED 2

typedef struct kfbi_ctx kfbi_ctx;

/* The box [x0, x0+side] x [y0, y0+side] with N intervals per side, h = side/N,
 * nodes (i, j), i, j = 0..N (Sec. 4.2).  N a power of two, 64 <= N <= 2048; the operator is
 * Delta - c2 (c2 >= 0).  max_markers bounds M (even, 16 <= M <= 4096).  max_batch bounds
 * the densities of one kfbi_apply_batch call (0 is taken as 1; at most 64); the grid
 * workspaces are allocated max_batch times. */
typedef struct {
  double x0, y0, side;
  int N;
  double c2;
  int box_bc;
  int max_markers;
  void* stream; /* hipStream_t */
  int max_batch;
} kfbi_grid;

/* Sizes of the current interface discretisation (host struct, filled on request). */
typedef struct {
  int M;            /* markers                                            */
  int n_cross_h;    /* crossings with grid rows y = y_j                   */
  int n_cross_v;    /* crossings with grid columns x = x_i                */
  int n_arms;       /* irregular stencil arms P -> Q (Sec. 4.2.1)         */
  int n_nodes;      /* distinct interpolation-stencil nodes (Sec. 4.3)    */
  int n_rows;       /* grid rows holding stencil nodes                    */
  int row_lo, row_hi; /* band of grid rows written by the fast solve      */
  int n_parts;      /* row parts (at most 16 arms of one row each) of the
                       row sine transform                                */
  int sub_batch;    /* densities per launch of kfbi_apply_batch: a larger
                       batch runs as consecutive launches of at most this
                       many, so that each launch's row-transform output and
                       band stay within the last-level cache              */
  long long workspace_bytes; /* device memory the context holds (all its
                       workspaces); unchanged by apply and GMRES calls   */
} kfbi_info;

/* Outputs of one apply.  Each pointer is a device array or NULL (not computed).
 *  v_plus/v_minus  [M]: one-sided limits v+-(X_k) of the layer potential (Sec. 4.3)
 *  dn_plus/dn_minus[M]: n . grad v+- with the outward normal n = (y_a, -x_a)/s_a
 *  grid [(N+1)*(N+1)]: grid solution, row-major index j*(N+1)+i, box values on the
 *                      ring.  Requesting the grid switches to the full-grid solve. */
typedef struct {
  double* v_plus;
  double* v_minus;
  double* dn_plus;
  double* dn_minus;
  double* grid;
} kfbi_out;

/* Thread-local message describing the last failing call of this thread. */
const char* kfbi_last_error(void);

/* Create a context on the current HIP device; allocates the grid workspaces and the
 * GMRES workspace (Krylov basis of max_markers x 65 doubles, Hessenberg matrix, events). */
int kfbi_create(const kfbi_grid* grid, kfbi_ctx** out);
int kfbi_destroy(kfbi_ctx* ctx);

/* Install the interface Gamma: xy_dev holds 2*M doubles, x[0..M) then y[0..M), the
 * markers X_k at equispaced parameters a_k = 2 pi k/M, counter-clockwise (Omega+ is
 * the bounded interior).  Runs the per-step geometry on the GPU: spectral derivatives
 * (Sec. 5.3 remark), grid-line crossings (6-point Lagrange interpolation between
 * markers, safeguarded Newton), inside/outside labels, the irregular-arm list with
 * App. A jump coefficients, the Sec. 4.3 interpolation stencils and their weights.
 * A column crossing within 1e-9 h of a grid node is assigned to the column segment
 * where the row-based labels change (interface through a node up to rounding).
 * Synchronises the stream.  Returns KFBI_E_GEOMETRY if a marker is within 3h of the
 * box boundary, a grid segment is cut twice, labels and crossings disagree, or the
 * interface has more row parts than the column solve can hold in the LDS of one
 * workgroup (the message gives both numbers). */
int kfbi_set_interface(kfbi_ctx* ctx, int M, const double* xy_dev);
int kfbi_get_info(const kfbi_ctx* ctx, kfbi_info* info);

/* One operator apply (Sec. 4): v = S psi (layer KFBI_SINGLE) or D phi (KFBI_DOUBLE)
 * with density_dev [M] (doubles), evaluated through the equivalent interface problem;
 * writes the requested outputs.  ring_dev: with KFBI_BOX_USER, 4*(N+1) doubles of box
 * values in the order bottom (j=0, i=0..N), top (j=N), left (i=0, j=0..N), right
 * (i=N); otherwise NULL (corner nodes are taken from the left/right arrays in the grid
 * output; they never enter the five-point stencils).  precision KFBI_FP64 or KFBI_FP32 (grid stages in FP32,
 * inputs/outputs stay FP64).  Asynchronous on the context stream. */
int kfbi_apply(kfbi_ctx* ctx, int layer, int precision, const double* density_dev,
               const double* ring_dev, const kfbi_out* out);

/* B independent applies of the same layer on the installed interface, in one launch per
 * stage (the densities share the geometry; Sec. 4 for each of them).  density_dev
 * [B][M] (row b = density b); ring_dev [B][4(N+1)] (KFBI_BOX_USER) or NULL; the outputs
 * v_plus, v_minus, dn_plus, dn_minus are [B][M] device arrays or NULL, and out->grid must
 * be NULL.  Each result equals, bit for bit, kfbi_apply on that density alone.
 * 1 <= B <= max_batch of the context (else KFBI_E_INVALID).  Batches larger than
 * kfbi_info.sub_batch run as consecutive launches of at most that many densities.
 * Asynchronous. */
int kfbi_apply_batch(kfbi_ctx* ctx, int layer, int precision, int B, const double* density_dev,
                     const double* ring_dev, const kfbi_out* out);

/* Discrete boundary integral operator A x = a x + b * trace_side(layer[x])
 *                                          + q * sum_k x_k s_a,k (2 pi / M).
 * Hele-Shaw (Sec. 3.1, eq. bie-HS): {DOUBLE, MINUS, a=0, b=1, q=1} with the free-space
 * box; interior Dirichlet: {DOUBLE, PLUS, 0, 1, 0}; Gibbs-Thomson (eq. bie-GT):
 * {SINGLE, AVG, eps_V, -1, 0} with the zero-normal-derivative box.  a_marker: NULL, or
 * a device array of M doubles that replaces a by one value per marker (an anisotropic
 * eps_V); it must stay valid while the operator is in use. */
typedef struct {
  int layer;
  int side;
  double a, b, q;
  const double* a_marker;
} kfbi_bie;

/* y_dev[M] = A x_dev (FP64 in/out; precision selects the grid arithmetic). */
int kfbi_operator(kfbi_ctx* ctx, const kfbi_bie* op, int precision, const double* x_dev,
                  double* y_dev);

typedef struct {
  double tol;        /* true relative residual ||b - A x||_2/||b||_2 to reach (FP64)   */
  int restart;       /* Krylov dimension before restart, 1..64                         */
  int maxit;         /* cap on inner iterations (all cycles)                           */
  int precision;     /* KFBI_FP64: plain GMRES; KFBI_FP32: FP32 operator inside FP64
                        iterative refinement (residuals always with the FP64 operator);
                        KFBI_MIXED: one FP64 GMRES (FP64 Krylov basis, Hessenberg matrix,
                        rotations) whose Arnoldi applies run in FP32 once the residual
                        estimate is at most inner_tol ||b||, the relaxation of inexact
                        Krylov methods (an apply may be less accurate as the residual
                        falls); convergence still on the true FP64 residual, and a cycle
                        that used FP32 applies and ends above tol is followed by cycles
                        with FP64 applies only                                          */
  double inner_tol;  /* KFBI_FP32: relative tolerance of each FP32 inner solve (0: 1e-5);
                        KFBI_MIXED: relative residual below which applies are FP32
                        (0: 1e-5)                                                       */
} kfbi_gmres_opts;

typedef struct {
  int iters;         /* Arnoldi steps in total                                          */
  int outer_iters;   /* restart cycles (FP64) or refinement steps (FP32)                */
  int applies64, applies32;
  double relres;     /* final true FP64 relative residual                               */
  int converged;
} kfbi_gmres_stats;

/* Solve A x = b by restarted GMRES (CGS2 Arnoldi, Givens rotations, device-resident;
 * convergence on the true FP64 residual).  x_dev holds the initial guess on entry and
 * the solution on return.  Synchronises.  KFBI_E_NOCONV if maxit is reached. */
int kfbi_gmres_solve(kfbi_ctx* ctx, const kfbi_bie* op, const double* rhs_dev,
                     double* x_dev, const kfbi_gmres_opts* opts, kfbi_gmres_stats* stats);

/* kfbi_gmres_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve, same
 * arguments, same results, with the Krylov workspace (basis, Hessenberg matrix, rotations,
 * partial sums, work vectors, status words) in one static device array of the library
 * instead of the context's buffers.  Calls no hipMalloc, hipFree or other allocating
 * routine.  Limit: M <= 4096 markers (else KFBI_E_INVALID); the array holds about 2.3 MB on
 * every GPU the library runs on, from its first kfbi_create on that GPU until the process
 * ends.  All calls on one GPU share that array and leave their last contents in it; calls
 * that overlap in time on one GPU (several host threads or streams) race, so they must be
 * serialised by the caller.  The operator applies inside still use the context's apply
 * buffers (allocated by kfbi_create / kfbi_set_interface). */
int kfbi_gmres_solve_static(kfbi_ctx* ctx, const kfbi_bie* op, const double* rhs_dev,
                            double* x_dev, const kfbi_gmres_opts* opts, kfbi_gmres_stats* stats);

/* Measurement hook: while on, every apply brackets its four kernels with HIP events on
 * the context stream (stage 0: density derivatives and marker jump quantities, k_prep;
 * 1: corrected right-hand sides and their row sine transform, k_rowdst; 2: column
 * tridiagonal solves, k_colsolve; 3: inverse transform at the stencil nodes and the
 * corrected interpolation, k_nodes_extract, plus the full grid when requested).  kfbi_profile_read synchronises and
 * returns the summed milliseconds per stage (ms_total[4], host) and the number of
 * recorded applies.  Turning profiling on resets the sums. */
int kfbi_profile(kfbi_ctx* ctx, int on);
int kfbi_profile_read(kfbi_ctx* ctx, double* ms_total, long* napplies);

/* Measurement hook: replays kernel `stage` (0..3, numbered as above) of the last
 * kfbi_apply/kfbi_apply_batch/kfbi_operator call (with the batch size of that call) reps
 * times back to back on the context stream, on the library's own buffers, and returns the average launch duration in microseconds
 * (HIP events around the replays; one untimed launch first).  Stage 0 reads a library
 * workspace as its density and stage 3 writes no caller output, so no caller array is
 * touched.  Synchronises.  KFBI_E_STATE if no apply ran since kfbi_set_interface. */
int kfbi_profile_kernel(kfbi_ctx* ctx, int stage, int reps, double* us_avg);

#ifdef __cplusplus
}
#endif
#endif /* KFBI_H */
