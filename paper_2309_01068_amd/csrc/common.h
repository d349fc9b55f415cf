// Internal declarations of the gfx950 KFBI library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>

#include "../../include/kfbi.h"

namespace kfbi {

constexpr int kWave = 64;

// ------------------------------------------------------------------- error plumbing
void set_error(const char* fmt, ...);

#define KFBI_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::kfbi::set_error("%s failed at %s:%d: %s", #call, __FILE__, __LINE__,        \
                        hipGetErrorString(e_));                                     \
      return KFBI_E_HIP;                                                            \
    }                                                                               \
  } while (0)

#define KFBI_TRY(expr)               \
  do {                               \
    int s_ = (expr);                 \
    if (s_ != KFBI_OK) return s_;    \
  } while (0)

// Device buffer that grows, never shrinks; freed by the context.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Per-crossing record (horizontal: line = j, pos = xi; vertical: line = i, pos = eta).
struct Crossing {
  int line;
  int k;      // marker interval [a_k, a_{k+1}]
  int seg;    // grid segment: node index m with g_m <= pos < g_{m+1}
  int horiz;  // 1 = row crossing, 0 = column crossing
  double t;   // local parameter in [0, 1]
  double pos;
};

// Per-marker extraction data (Sec. 4.3), FP64, structure of arrays: entry q of marker k
// is ext[q * M + k] with
//   q = kExtW + 6r + m   row r of the inverse 6x6 Taylor system (v+, v+_x, v+_y)
//   q = kExtE + 5r + s   jump-correction part: maps the marker quantities (Phi, Phi_a,
//                        Phi_aa, Psi, Psi_a) to the contribution of chi(q_m) C(q_m)
//   q = kExtD + 5r + s   maps the same quantities to ([v], [v_x], [v_y]) at the marker
//   q = kExtN, kExtN+1   outward unit normal;  q = kExtQ: s_a 2 pi / M (trapezoid weight)
constexpr int kExtW = 0, kExtE = 18, kExtD = 33, kExtN = 48, kExtQ = 50, kExtCount = 51;
// Per-arm coefficients in marker-interval order (for the correction kernel), SoA:
// armc[q * cap + a], q = 0..5 Lagrange weights l_m, q = 6..10 coefficients of
// (Phi, Phi_a, Phi_aa, Psi, Psi_a) in -+T/h^2.
constexpr int kArmCoefCount = 11;
constexpr int kArmsPerPart = 16;  // arms of one row handled by one block of the row transform

// Per-arm data (Sec. 4.2.1): correction value r = sum_m l_m sum_q coef_q Q_q(k-2+m).
struct ArmCoef {
  double l[6];
  double coef[5];
  int k;
  int pad;
};

// Byte offset of the geometry status in the context's mapped host status block.
constexpr size_t kGeoStatusOffset = 2048;

// Status words written by the geometry kernels.
struct GeoStatus {
  int err;          // 0 or an error code (1: two crossings in a segment, 2: label mismatch,
                    // 3: margin, 4: capacity, 5: crossing outside grid)
  int n_cross_h, n_cross_v;
  int n_arms;
  int n_nodes;
  int n_rows;
  int row_lo, row_hi;
  int n_parts;
  int arm_lo, arm_hi;  // first and last grid rows holding arms (arm_lo > arm_hi: none)
  int cr_lo, cr_hi;    // rows between which the sampled curve lies (row lines it may cut)
  int cc_lo, cc_hi;    // the same for the columns
};

}  // namespace kfbi

struct kfbi_ctx {
  // grid
  double x0, y0, side, h;
  int N;
  double c2;
  int box_bc;
  int max_markers;
  int max_batch = 1;  // densities per kfbi_apply_batch call the workspaces hold
  hipStream_t stream;
  int device;

  // interface sizes (host copies, valid after set_interface)
  int M = 0;
  int have_interface = 0;
  kfbi::GeoStatus st{};
  // rows whose node maps and labels the last geometry set-up may have written (all rows
  // until the first one: the maps start uninitialised)
  int gb_lo = 0, gb_hi = 1 << 30;
  int d_M = 0;  // M for which the differentiation vectors are built

  // geometry buffers
  kfbi::DBuf X, geo, dvec, cnt, cross, hid, vid, vraw, lab, armcnt, rowsum, armrow, armpk, armcoef,
      intptr, need, nodeidx, nodei, rowptr, rows, mknode, ext, gstat, armc, armk, armsc,
      chpos,
      colc, lanef, bandc, cnode, ccount, mkloc, tmat, pdesc, rowpart, ckoff, cklist, ckcoef, ckmk,
      mqz;
  int arm_cap = 0;
  // the band of rows (first row, rows, rows per lane) that bandc holds the column-solve
  // constants of (bc_nr = 0: none yet)
  int bc_lo = 0, bc_nr = 0, bc_E = 0;
  // per-apply buffers
  kfbi::DBuf mq, armr, qpart, ring, sinT, sinT32, gband, nodeval, tmpM;
  // gmres buffers
  kfbi::DBuf gV, gH, gsc, gpart, gcnt, gw, gx, gr, gd;
  static constexpr int kGmresRing = 4;
  hipEvent_t gev[kGmresRing] = {};
  // status words the kernels write straight into coherent pinned host memory (4 KB):
  // the GMRES slots from offset 0 (under 1 KB), the geometry status at kGeoStatusOffset
  void* hstat = nullptr;
  void* dstat = nullptr;  // its device address

  // stage profiling with HIP events (kfbi_profile)
  int prof_on = 0;
  static constexpr int kProfPool = 320;  // 64 applies x 5 events
  hipEvent_t prof_ev[kProfPool] = {};
  int prof_used = 0;
  double prof_ms[4] = {0, 0, 0, 0};
  long prof_count = 0;

  // kernel replay (kfbi_profile_kernel): layer and precision of the last apply, -1 = none
  int last_layer = -1;
  int last_precision = 0;
  int last_batch = 1;

  // apply launch geometry (set by set_interface)
  int mk_chunk = 8;   // markers per K1 block
  int n_mk_blocks = 0;
  int n_ring_blocks = 0;
};

namespace kfbi {
// stage entry points (implemented in the .hip files)
int geometry_setup(kfbi_ctx* c, int M, const double* xy);
// Zero-normal-derivative box, full fields (FP64): Ghat arrays of neu_field_size(N) doubles.
inline size_t neu_field_size(int N) { return static_cast<size_t>(N + 4) * (N + 1); }
// rows jlo..jhi of the solution of the dense right-hand side ca Fa + cb Fb (column-group
// layout of those rows: element (j, p) at ((p / 4) nb + j - jlo) 4 + p % 4, nb = jhi-jlo+1),
// and the values at the markers from such rows (they must hold every node row)
int neu_dense_solve(kfbi_ctx* c, const double* Fa, const double* Fb, double ca, double cb,
                    double* Gout, int jlo, int jhi);
int neu_interp(kfbi_ctx* c, const double* G, int jlo, int jhi, double* vout);
int neu_apply_full(kfbi_ctx* c, int layer, const double* dens, const double* Fa,
                   const double* Fb, double ca, double cb, double* Gout);
int neu_to_grid(kfbi_ctx* c, const double* Gfull, double* grid);
int neu_from_grid(kfbi_ctx* c, const double* grid, double* Gfull);

// Dynamic LDS: every kernel launched with more than the default is allowed the whole LDS
// of a workgroup beyond its static part, once per device (kernel_attributes, called by
// kfbi_create under a lock); dyn_lds_capacity is that allowance.
size_t dyn_lds_capacity(const void* kernel);
int allow_full_dyn_lds(const void* kernel);
int kernel_attributes();
int apply_kernel_attrs();
int gmres_kernel_attrs();
int thetal_kernel_attrs();
// Dynamic LDS the FP64 column solve of this grid and box may take (bytes).
size_t colsolve_lds_capacity(const kfbi_ctx* c);
// GMRES workspace for max_markers and the largest restart (kfbi_create).
int gmres_alloc(kfbi_ctx* c);
// y = A x for GMRES; the flag asks for the operator in FP32 (iterative refinement and
// mixed modes).
using GmresOp = std::function<int(const double* x, double* y, bool fp32)>;
// kfbi_gmres_solve whose FP64 applies also write the outputs `side`; *side_at_x tells
// whether they belong to the returned solution.
int gmres_solve_side(kfbi_ctx* c, const kfbi_bie* op, const double* b, double* x,
                     const kfbi_gmres_opts* o, kfbi_gmres_stats* stats, const kfbi_out* side,
                     bool* side_at_x);
int gmres_solve_op(kfbi_ctx* c, int n, const GmresOp& op, const double* b, double* x,
                   const kfbi_gmres_opts* o, kfbi_gmres_stats* stats);
// Device address of the static GMRES workspace on the current device (once per device).
int static_scratch_setup();

int apply_impl(kfbi_ctx* c, int layer, int precision, const double* dens, const double* ring_user,
               const kfbi_out* out, const kfbi_bie* op, const double* x_for_op, double* y_op,
               int batch = 1);
int ensure_apply_buffers(kfbi_ctx* c);
int prof_flush(kfbi_ctx* c);
int replay_stage(kfbi_ctx* c, int stage, int reps, double* us_avg);
int colconst_setup(kfbi_ctx* c);
}  // namespace kfbi
