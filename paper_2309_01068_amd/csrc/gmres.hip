// Matrix-free restarted GMRES on gfx950 (Sec. 4 opening: the discretised boundary
// integral equations are solved by GMRES; each iteration applies the operator once).
//
// Device-resident FP64 Arnoldi with classical Gram-Schmidt applied twice (CGS2), inner
// products as fixed-order block partials reduced by the last block to finish (no
// floating-point atomics, so results are bitwise reproducible), Givens rotations in
// that last block, convergence checked on the host from a 64-byte status word.  The
// answer is accepted only on the true residual ||b - A x||_2 <= tol ||b||_2 computed
// with the FP64 operator.  KFBI_FP32 selects iterative refinement: FP64 residual, inner
// GMRES with the FP32 operator, x += d.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "device_util.h"

namespace kfbi {

constexpr int kMaxRestart = 64;
constexpr int kRedBlock = 256;
constexpr int kRing = kfbi_ctx::kGmresRing;  // Arnoldi status slots in flight

struct GmresStatus {
  double resid;   // |g_{j+1}| (Givens estimate) or a reduced norm
  double hnext;   // h_{j+1,j}
  int breakdown;
  int pad[11];
};

// Status of an Arnoldi step for the host: written straight into mapped host memory
// (coherent pinned allocation) and pushed out at system scope, so that the host reads it
// once the step's event has completed, with no copy in the stream.
__device__ __forceinline__ void post_status(GmresStatus* hout, double resid, double hn) {
  hout->resid = resid;
  hout->hnext = hn;
  hout->breakdown = (hn == 0.0);
  __threadfence_system();
}

// Column j of the Hessenberg matrix, h_i = h1_i + h2_i (i <= j) and h_{j+1} = hn, rotated
// by the previous Givens rotations (cs_i, sn_i, i < j), the new rotation j, the update of
// g (gj = g_j on entry), and the status.  One thread; h1, h2, csh, snh are in LDS, so the
// sequential loop over i waits on no memory round trip (H, cs, sn, g are only written).
__device__ void hess_column(int j, const double* h1, const double* h2, double hn,
                            const double* csh, const double* snh, double gj, double* H,
                            double* cs, double* sn, double* g, GmresStatus* st,
                            GmresStatus* hout) {
  double* col = H + static_cast<size_t>(j) * (kMaxRestart + 1);
  double a = h1[0] + h2[0];  // entry i of the column after rotations 0..i-1
  for (int i = 0; i < j; ++i) {
    const double b = h1[i + 1] + h2[i + 1];
    const double c = csh[i], sv = snh[i];
    col[i] = c * a + sv * b;
    a = -sv * a + c * b;
  }
  const double den = hypot(a, hn);
  const double c = a / den, sv = hn / den;
  cs[j] = c;
  sn[j] = sv;
  col[j] = den;
  col[j + 1] = 0.0;
  const double gn = -sv * gj;
  g[j + 1] = gn;
  g[j] = c * gj;
  st->resid = fabs(gn);
  st->hnext = hn;
  st->breakdown = (hn == 0.0);
  post_status(hout, fabs(gn), hn);
}

// Partial inner products <V_i, w> (i < nv) and optionally ||w||^2, after an optional
// update w -= sum_i hprev_i V_i.  The last block to finish reduces the partials in block
// order and writes out[0..nv) (and out[nv] = ||w||^2).
__global__ void __launch_bounds__(kRedBlock)
    k_cgs(int M, int ldv, const double* __restrict__ V, int nv, double* __restrict__ w,
          const double* __restrict__ hprev, int want_norm, double* __restrict__ part,
          unsigned int* __restrict__ counter, double* __restrict__ out) {
  __shared__ double red[kMaxRestart + 2][4];
  __shared__ int is_last;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double wk = 0.0;
  if (k < M) {
    wk = w[k];
    if (hprev) {
      for (int i = 0; i < nv; ++i) wk -= hprev[i] * V[static_cast<size_t>(i) * ldv + k];
      w[k] = wk;
    }
  }
  const int nout = nv + (want_norm ? 1 : 0);
  for (int i = 0; i < nout; ++i) {
    double p = 0.0;
    if (k < M) p = (i < nv) ? V[static_cast<size_t>(i) * ldv + k] * wk : wk * wk;
    p = wave_sum(p);
    if (lane == 0) red[i][wv] = p;
  }
  __syncthreads();
  const int nb = gridDim.x;
  for (int i = threadIdx.x; i < nout; i += blockDim.x)
    part[static_cast<size_t>(blockIdx.x) * nout + i] = ((red[i][0] + red[i][1]) + red[i][2]) + red[i][3];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(counter, 1u);
    is_last = (prev == static_cast<unsigned int>(nb - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  for (int i = threadIdx.x; i < nout; i += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += __builtin_nontemporal_load(&part[static_cast<size_t>(b) * nout + i]);
    out[i] = s;
  }
  if (threadIdx.x == 0) *counter = 0u;
}

// w -= sum_i h_i V_i, then ||w||^2 partials; the last block finishes column j of the
// Hessenberg matrix (h = h1 + h2, h_{j+1,j} = ||w||), applies the previous Givens
// rotations, forms the new one and updates the residual vector g.
__global__ void __launch_bounds__(kRedBlock)
    k_finish(int M, int ldv, const double* __restrict__ V, int j, double* __restrict__ w,
             const double* __restrict__ h1, const double* __restrict__ h2,
             double* __restrict__ part, unsigned int* __restrict__ counter,
             double* __restrict__ H /* (kMaxRestart+1) x kMaxRestart, column-major */,
             double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
             GmresStatus* __restrict__ st, GmresStatus* __restrict__ hout) {
  __shared__ double red[4];
  __shared__ int is_last;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double wk = 0.0;
  if (k < M) {
    wk = w[k];
    for (int i = 0; i <= j; ++i) wk -= h2[i] * V[static_cast<size_t>(i) * ldv + k];
    w[k] = wk;
  }
  double p = wave_sum(wk * wk);
  if (lane == 0) red[wv] = p;
  __syncthreads();
  const int nb = gridDim.x;
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(counter, 1u);
    is_last = (prev == static_cast<unsigned int>(nb - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __shared__ double hs1[kMaxRestart + 1], hs2[kMaxRestart + 1], csh[kMaxRestart], snh[kMaxRestart];
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    hs1[i] = h1[i];
    hs2[i] = h2[i];
    if (i < j) {
      csh[i] = cs[i];
      snh[i] = sn[i];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  __threadfence();
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += __builtin_nontemporal_load(&part[b]);
  hess_column(j, hs1, hs2, sqrt(s), csh, snh, g[j], H, cs, sn, g, st, hout);
  *counter = 0u;
}

// One Arnoldi step in a single workgroup (used while M (j+1) is small): CGS2 against
// V_0..V_j, h_{j+1,j} = ||w||, the Hessenberg column with the previous Givens rotations,
// the new rotation, g, the status word, and V_{j+1} = w / h_{j+1,j}.  All reductions are
// fixed-order within the workgroup.  When V_0..V_j fit (stage != 0) they are copied to LDS
// once, with all loads in flight together, and both passes read them from there.
constexpr int kArnThreads = 1024;
constexpr int kArnPer = 4;  // elements per thread: M <= 4096
constexpr size_t kArnStageBytes = 112 * 1024;  // LDS for the staged basis vectors (+40 KB static)
__global__ void __launch_bounds__(kArnThreads)
    k_arnoldi(int M, int ldv, double* __restrict__ V, int j, const double* __restrict__ w,
              double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
              double* __restrict__ g, GmresStatus* __restrict__ st,
              GmresStatus* __restrict__ hout, int stage) {
  __shared__ double red[kMaxRestart + 1][kArnThreads / 64];
  __shared__ double hv[2][kMaxRestart + 1];
  __shared__ double wsh[kArnThreads * kArnPer];
  __shared__ double csh[kMaxRestart], snh[kMaxRestart];
  extern __shared__ double vsh[];  // (j+1) x M when staged
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = kArnThreads / 64;
  // the previous rotations and g_j, loaded now for the column update at the end
  if (tid < j) {
    csh[tid] = cs[tid];
    snh[tid] = sn[tid];
  }
  const double gj = (tid == 0) ? g[j] : 0.0;
  double wk[kArnPer];
#pragma unroll
  for (int u = 0; u < kArnPer; ++u) {
    const int k = tid + u * kArnThreads;
    wk[u] = (k < M) ? w[k] : 0.0;
  }
  if (stage) {
    // V_0..V_j copied to LDS as one flat array of (j + 1) M values with sixteen loads in
    // flight per thread: the vectors come from earlier launches, mostly not from this
    // XCD's L2, so the copy is bound by memory latency
    const int tot = (j + 1) * M;
    constexpr int U = 16;
    for (int e0 = tid; e0 < tot; e0 += kArnThreads * U) {
      double t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kArnThreads;
        if (e < tot) {
          const int i = e / M, k = e - i * M;
          t[u] = V[static_cast<size_t>(i) * ldv + k];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kArnThreads;
        if (e < tot) vsh[e] = t[u];
      }
    }
  }
  for (int pass = 0; pass < 2; ++pass) {
    // stage w, then wavefront q takes the inner products <V_i, w> for i = q, q + 16, ...
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kArnPer; ++u) {
      const int k = tid + u * kArnThreads;
      if (k < M) wsh[k] = wk[u];
    }
    __syncthreads();
    for (int i = wv; i <= j; i += NW) {
      const double* vi = stage ? vsh + static_cast<size_t>(i) * M : V + static_cast<size_t>(i) * ldv;
      double p = 0.0;
      for (int k = lane; k < M; k += 64) p += vi[k] * wsh[k];
      p = wave_sum(p);
      if (lane == 0) hv[pass][i] = p;
    }
    __syncthreads();
    // w -= sum_i h_i V_i
    for (int i = 0; i <= j; ++i) {
      const double hi = hv[pass][i];
      const double* vi = stage ? vsh + static_cast<size_t>(i) * M : V + static_cast<size_t>(i) * ldv;
#pragma unroll
      for (int u = 0; u < kArnPer; ++u) {
        const int k = tid + u * kArnThreads;
        if (k < M) wk[u] -= hi * vi[k];
      }
    }
  }
  double p = 0.0;
#pragma unroll
  for (int u = 0; u < kArnPer; ++u) p += wk[u] * wk[u];
  p = wave_sum(p);
  if (lane == 0) red[0][wv] = p;
  __syncthreads();
  // every thread forms h_{j+1,j} from the same partials in the same order and stores its
  // part of V_{j+1} at once; thread 0 meanwhile finishes the Hessenberg column
  double s = 0.0;
  for (int q = 0; q < NW; ++q) s += red[0][q];
  const double hn = sqrt(s);
  double* vn = V + static_cast<size_t>(j + 1) * ldv;
#pragma unroll
  for (int u = 0; u < kArnPer; ++u) {
    const int k = tid + u * kArnThreads;
    if (k < M) vn[k] = (hn != 0.0) ? wk[u] / hn : 0.0;
  }
  if (tid == 0) hess_column(j, hv[0], hv[1], hn, csh, snh, gj, H, cs, sn, g, st, hout);
}

__global__ void k_scale(int M, const double* __restrict__ w, const double* __restrict__ hn,
                        double* __restrict__ v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < M) v[k] = (*hn != 0.0) ? w[k] / *hn : 0.0;
}

// r = b - y, partial ||r||^2; last block writes status->resid = ||r||.
__global__ void __launch_bounds__(kRedBlock)
    k_residual(int M, const double* __restrict__ b, const double* __restrict__ y,
               double* __restrict__ r, double* __restrict__ part, unsigned int* __restrict__ counter,
               GmresStatus* __restrict__ st, GmresStatus* __restrict__ hout) {
  __shared__ double red[4];
  __shared__ int is_last;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double rk = 0.0;
  if (k < M) {
    rk = b[k] - (y ? y[k] : 0.0);
    if (r) r[k] = rk;
  }
  double p = wave_sum(rk * rk);
  if (lane == 0) red[wv] = p;
  __syncthreads();
  const int nb = gridDim.x;
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(counter, 1u);
    is_last = (prev == static_cast<unsigned int>(nb - 1));
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __threadfence();
  double s = 0.0;
  for (int bb = 0; bb < nb; ++bb) s += __builtin_nontemporal_load(&part[bb]);
  st->resid = sqrt(s);
  if (hout) post_status(hout, sqrt(s), 1.0);
  *counter = 0u;
}

// Start a cycle: V_0 = r / beta, g = (beta, 0, ...).
__global__ void k_start(int M, const double* __restrict__ r, const GmresStatus* __restrict__ st,
                        double* __restrict__ v0, double* __restrict__ g) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = st->resid;
  if (k < M) v0[k] = r[k] / beta;
  if (k <= kMaxRestart) g[k] = (k == 0) ? beta : 0.0;
}

// Back substitution H(0:m,0:m) y = g(0:m) and x += V y.  The triangle and g are first
// loaded into LDS by the whole block (independent loads), so the sequential substitution
// of thread 0 reads only LDS.
__global__ void __launch_bounds__(256)
    k_update_x(int M, int m, int ldv, const double* __restrict__ V,
               const double* __restrict__ H, const double* __restrict__ g,
               double* __restrict__ x) {
  __shared__ double y[kMaxRestart];
  __shared__ double hs[kMaxRestart * kMaxRestart];  // column q, row i at q m + i
  const int ld = kMaxRestart + 1;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int q = e / m, i = e - q * m;
    hs[e] = (i <= q) ? H[static_cast<size_t>(q) * ld + i] : 0.0;
  }
  if (static_cast<int>(threadIdx.x) < m) y[threadIdx.x] = g[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = m - 1; i >= 0; --i) {
      double s = y[i];
      for (int q = i + 1; q < m; ++q) s -= hs[q * m + i] * y[q];
      y[i] = s / hs[i * m + i];
    }
  }
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  double s = x[k];
  for (int i = 0; i < m; ++i) s += V[static_cast<size_t>(i) * ldv + k] * y[i];
  x[k] = s;
}

__global__ void k_axpy(int M, double a, const double* __restrict__ d, double* __restrict__ x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < M) x[k] += a * d[k];
}

struct GmresWork {
  double* V;
  int ldv;
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* h1;
  double* h2;
  double* w;
  double* part;
  unsigned int* counter;
  GmresStatus* st;   // status of the last reduction (residual norms)
  GmresStatus* ring;   // per-iteration Arnoldi status, slot j % kRing (device)
  GmresStatus* hring;  // status ring in coherent pinned host memory (host view), then the
                       // residual slots kSlotRes, kSlotNb
  GmresStatus* dring;  // the same memory as the kernels address it
  hipEvent_t* ev;      // one event per ring slot, recorded after its copy
  double* r;
  double* d;
  double* y;
  double* dcorr;  // correction of one refinement step (FP32 mode)
};

int gmres_kernel_attrs() { return allow_full_dyn_lds(reinterpret_cast<const void*>(k_arnoldi)); }

// The workspace for M <= max_markers and any restart <= kMaxRestart, allocated once by
// kfbi_create: the Krylov basis (ldv x (kMaxRestart + 1)), the Hessenberg matrix, the
// rotations, block partials, the status slots, four work vectors and the ring events.
int gmres_alloc(kfbi_ctx* c) {
  const int Mx = c->max_markers;
  const int ldv = ((Mx + 63) / 64) * 64;
  const int nblk = (Mx + kRedBlock - 1) / kRedBlock;
  KFBI_TRY(c->gV.ensure(sizeof(double) * static_cast<size_t>(ldv) * (kMaxRestart + 1)));
  KFBI_TRY(c->gH.ensure(sizeof(double) * (kMaxRestart + 1) * (kMaxRestart + 1)));
  KFBI_TRY(c->gsc.ensure(sizeof(double) * 5 * (kMaxRestart + 2)));
  KFBI_TRY(c->gpart.ensure(sizeof(double) * static_cast<size_t>(nblk) * (kMaxRestart + 2)));
  KFBI_TRY(c->gcnt.ensure(sizeof(GmresStatus) * (1 + kRing) + 64));
  KFBI_TRY(c->gw.ensure(sizeof(double) * static_cast<size_t>(ldv) * 4));
  for (int q = 0; q < kRing; ++q)
    if (!c->gev[q]) KFBI_HIP(hipEventCreateWithFlags(&c->gev[q], hipEventDisableTiming));
  return KFBI_OK;
}

// Pointers into the workspace for vectors of length n <= max_markers.
static void bind_work(kfbi_ctx* c, GmresWork* gw, int n) {
  const int ldv = ((n + 63) / 64) * 64;
  gw->V = c->gV.as<double>();
  gw->ldv = ldv;
  gw->H = c->gH.as<double>();
  double* sc = c->gsc.as<double>();
  gw->cs = sc;
  gw->sn = sc + (kMaxRestart + 2);
  gw->g = sc + 2 * (kMaxRestart + 2);
  gw->h1 = sc + 3 * (kMaxRestart + 2);
  gw->h2 = sc + 4 * (kMaxRestart + 2);
  gw->part = c->gpart.as<double>();
  gw->st = c->gcnt.as<GmresStatus>();
  gw->ring = gw->st + 1;
  gw->counter = reinterpret_cast<unsigned int*>(gw->st + 1 + kRing);
  gw->hring = reinterpret_cast<GmresStatus*>(c->hstat);
  gw->dring = reinterpret_cast<GmresStatus*>(c->dstat);
  gw->ev = c->gev;
  double* wb = c->gw.as<double>();
  gw->w = wb;
  gw->r = wb + ldv;
  gw->d = wb + 2 * ldv;
  gw->y = wb + 3 * ldv;
  gw->dcorr = c->tmpM.as<double>();
}

// ------------------------------------------------------------ workspace without allocation
// The variant kfbi_gmres_solve_static keeps its Krylov workspace in this file-scope device
// array instead of the context's buffers.  Each GPU holds its own copy until the process
// ends; host code addresses it only through the pointer hipGetSymbolAddress returns on
// that device (static_scratch_setup, once per device from kfbi_create).
constexpr int kStaticMaxM = 4096;
constexpr int kStaticLdv = kStaticMaxM;  // a multiple of 64
constexpr int kStaticNblk = (kStaticMaxM + kRedBlock - 1) / kRedBlock;
constexpr size_t kStaticDoubles =
    static_cast<size_t>(kStaticLdv) * (kMaxRestart + 1)     // V
    + (kMaxRestart + 1) * (kMaxRestart + 1)                  // H
    + 5 * (kMaxRestart + 2)                                  // cs, sn, g, h1, h2
    + static_cast<size_t>(kStaticNblk) * (kMaxRestart + 2)   // block partials
    + 5 * static_cast<size_t>(kStaticLdv)                    // w, r, d, y, dcorr
    + (1 + kRing) * (sizeof(GmresStatus) / sizeof(double)) + 8;  // status slots, counter
static __device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

int static_scratch_setup() {
  int dev = 0;
  KFBI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the static workspace supports", dev, kMaxDevices);
    return KFBI_E_INVALID;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return KFBI_OK;
  void* p = nullptr;
  KFBI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch[dev] = static_cast<double*>(p);
  return KFBI_OK;
}

// Pointers into the static workspace of the current device (M <= kStaticMaxM).
static int bind_static(kfbi_ctx* c, GmresWork* gw) {
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) base = g_scratch[c->device];
  }
  if (!base) {
    set_error("static GMRES workspace not set up on device %d", c->device);
    return KFBI_E_STATE;
  }
  const int M = c->M;
  const int ldv = ((M + 63) / 64) * 64;
  double* q = base;
  gw->V = q;
  gw->ldv = ldv;
  q += static_cast<size_t>(kStaticLdv) * (kMaxRestart + 1);
  gw->H = q;
  q += (kMaxRestart + 1) * (kMaxRestart + 1);
  gw->cs = q;
  gw->sn = q + (kMaxRestart + 2);
  gw->g = q + 2 * (kMaxRestart + 2);
  gw->h1 = q + 3 * (kMaxRestart + 2);
  gw->h2 = q + 4 * (kMaxRestart + 2);
  q += 5 * (kMaxRestart + 2);
  gw->part = q;
  q += static_cast<size_t>(kStaticNblk) * (kMaxRestart + 2);
  gw->w = q;
  gw->r = q + kStaticLdv;
  gw->d = q + 2 * kStaticLdv;
  gw->y = q + 3 * kStaticLdv;
  gw->dcorr = q + 4 * kStaticLdv;
  q += 5 * static_cast<size_t>(kStaticLdv);
  gw->st = reinterpret_cast<GmresStatus*>(q);
  gw->ring = gw->st + 1;
  gw->counter = reinterpret_cast<unsigned int*>(gw->st + 1 + kRing);
  gw->hring = reinterpret_cast<GmresStatus*>(c->hstat);
  gw->dring = reinterpret_cast<GmresStatus*>(c->dstat);
  gw->ev = c->gev;
  return KFBI_OK;
}

// Host status slots after the Arnoldi ring: the last residual norm and ||b||.
constexpr int kSlotRes = kRing, kSlotNb = kRing + 1;

// ||b - A x|| with the operator (in FP32 when fp32); leaves r in gw->r and the norm in the
// device status and host slot kSlotRes, and synchronises (which also makes every host
// slot written before it readable).
static int true_residual(kfbi_ctx* c, int M, const GmresOp& op, bool fp32, const double* b,
                         const double* x, GmresWork* gw, double* out, int* applies,
                         bool sync = true) {
  const int nblk = (M + kRedBlock - 1) / kRedBlock;
  KFBI_TRY(op(x, gw->y, fp32));
  ++*applies;
  hipLaunchKernelGGL(k_residual, dim3(nblk), dim3(kRedBlock), 0, c->stream, M, b, gw->y, gw->r,
                     gw->part, gw->counter, gw->st, gw->dring + kSlotRes);
  KFBI_HIP(hipGetLastError());
  if (!sync) return KFBI_OK;  // the caller reads the host slot after a later event
  KFBI_HIP(hipStreamSynchronize(c->stream));
  *out = gw->hring[kSlotRes].resid;
  return KFBI_OK;
}

// Restarted GMRES for A x = b with the operator at `precision`; stops when the true
// residual (same precision) is <= tol * nb or after maxit Arnoldi steps.
// With r_ready the residual of the incoming x is already in gw->r and the device status,
// with norm rn0, and the first cycle starts from it.  With pending as well, rn0 and the
// norm nb of the right-hand side are not known on the host yet: the first cycle starts at
// once and reads both from their host slots when it examines its first step (which was
// queued behind them); a right-hand side of zero then ends the solve (*zero_rhs) and an
// initial guess that already meets the tolerance ends the cycle with no update.
// Mixed mode (mixed_thresh > 0, precision FP64): the applies of the Arnoldi steps run in
// FP32 once the last residual estimate the host has read is at most mixed_thresh * nb,
// the Krylov basis, the Hessenberg matrix, the rotations and every true residual staying
// FP64 (relaxed inexact Krylov: the perturbation an apply may carry grows as the
// residual falls).  A cycle that used FP32 applies and ends above tol is followed by
// cycles with FP64 applies only; applies32 counts the FP32 applies.
static int gmres_core(kfbi_ctx* c, int M, const GmresOp& op, int precision, const double* b,
                      double* x, double nb, double tol, int restart, int maxit, GmresWork* gw,
                      int* iters, int* cycles, int* applies, double* relres, bool r_ready,
                      double rn0, double mixed_thresh = 0.0, int* applies32 = nullptr,
                      bool pending = false, double* nb_out = nullptr,
                      bool* zero_rhs = nullptr) {
  const int nblk = (M + kRedBlock - 1) / kRedBlock;
  const int mb = (M + 255) / 256;
  hipStream_t s = c->stream;
  double rn = 0.0;
  bool allow32 = mixed_thresh > 0.0;
  bool used32 = false;  // the cycle just finished ran FP32 applies
  for (;;) {
    if (used32) allow32 = false;  // reached here: that cycle did not converge on its own
    used32 = false;
    if (r_ready) {
      rn = rn0;
      r_ready = false;
    } else {
      KFBI_TRY(true_residual(c, M, op, precision == KFBI_FP32, b, x, gw, &rn, applies));
    }
    if (!pending) {
      if (!std::isfinite(rn)) {
        set_error("non-finite residual in GMRES");
        return KFBI_E_NONFINITE;
      }
      *relres = rn / nb;
      if (rn <= tol * nb) return KFBI_OK;
    }
    if (*iters >= maxit) return KFBI_E_NOCONV;
    ++*cycles;
    hipLaunchKernelGGL(k_start, dim3(mb), dim3(256), 0, s, M, gw->r, gw->st, gw->V, gw->g);
    // Iteration j is enqueued before the status of iteration j-1 is examined, so the GPU
    // always has work queued while the host waits; when j-1 turns out to be the last one,
    // iteration j was computed in vain (its Hessenberg column and g entries beyond j-1 are
    // never used).  (A lag of two iterations was measured slower: the host keeps up, and
    // the second wasted iteration costs more than it hides.)
    const bool one_block = (M <= kArnThreads * kArnPer) &&
                           (static_cast<long long>(M) * restart <= (1 << 17));
    int m = 0;
    int launched = 0, examined = 0;
    const int base = *iters;  // iterations of earlier cycles (< maxit here)
    bool stop = false;
    constexpr int kLag = 1;  // < kRing
    // residual estimates of the last two examined steps (unknown while pending: no
    // prediction and no FP32 apply before the first step is examined)
    double r1 = pending ? INFINITY : rn, r2 = -1.0;
    bool zero = false;
    // reads the status of step q (the next one not yet examined) and decides whether the
    // cycle stops there
    auto examine = [&](int q) -> int {
      KFBI_HIP(hipEventSynchronize(gw->ev[q % kRing]));
      if (pending) {  // ||b|| and the initial residual, posted before this step was queued
        pending = false;
        nb = gw->hring[kSlotNb].resid;
        const double r0 = gw->hring[kSlotRes].resid;
        if (nb_out) *nb_out = nb;
        if (!std::isfinite(r0) || !std::isfinite(nb)) {
          KFBI_HIP(hipStreamSynchronize(s));
          set_error("non-finite residual in GMRES");
          return KFBI_E_NONFINITE;
        }
        if (nb == 0.0 || r0 <= tol * nb) {  // nothing to do: no step counts, no update
          zero = (nb == 0.0);
          *relres = zero ? 0.0 : r0 / nb;
          stop = true;
          m = 0;
          return KFBI_OK;
        }
        *relres = r0 / nb;
        r1 = r0;
      }
      const GmresStatus& hs = gw->hring[q % kRing];
      ++*iters;
      ++examined;
      m = q + 1;
      if (!std::isfinite(hs.resid)) {
        KFBI_HIP(hipStreamSynchronize(s));
        set_error("non-finite Arnoldi residual");
        return KFBI_E_NONFINITE;
      }
      r2 = r1;
      r1 = hs.resid;
      if (hs.resid <= tol * nb || hs.breakdown || *iters >= maxit || m == restart) stop = true;
      return KFBI_OK;
    };
    for (int j = 0; !stop; ++j) {
      // When the step in flight (j - 1) is predicted to converge (its residual extrapolated
      // from the last two ratios of the estimate), its status is read before step j is
      // launched: a correct prediction then costs one host round trip instead of a step
      // computed in vain, a wrong one costs the round trip.  The step at which the cycle
      // stops is the same either way.
      if (j >= 1 && examined == j - 1 && j - 1 < launched && r2 > 0.0 &&
          r1 * (r1 / r2) <= tol * nb) {
        KFBI_TRY(examine(j - 1));
        if (stop) break;
      }
      if (j < restart && base + launched < maxit) {
        double* vj = gw->V + static_cast<size_t>(j) * gw->ldv;
        double* vn = gw->V + static_cast<size_t>(j + 1) * gw->ldv;
        const bool as32 = allow32 && r1 <= mixed_thresh * nb;
        KFBI_TRY(op(vj, gw->w, as32 || precision == KFBI_FP32));
        if (as32) {
          used32 = true;
          if (applies32) ++*applies32;
        } else {
          ++*applies;
        }
        GmresStatus* sj = gw->ring + (j % kRing);
        GmresStatus* hj = gw->dring + (j % kRing);  // device view of the host ring slot
        if (one_block) {
          const size_t vbytes = sizeof(double) * static_cast<size_t>(M) * (j + 1);
          const int stage = vbytes <= kArnStageBytes ? 1 : 0;
          hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(kArnThreads), stage ? vbytes : 0, s, M,
                             gw->ldv, gw->V, j, gw->w, gw->H, gw->cs, gw->sn, gw->g, sj, hj,
                             stage);
        } else {
          hipLaunchKernelGGL(k_cgs, dim3(nblk), dim3(kRedBlock), 0, s, M, gw->ldv, gw->V, j + 1,
                             gw->w, nullptr, 0, gw->part, gw->counter, gw->h1);
          hipLaunchKernelGGL(k_cgs, dim3(nblk), dim3(kRedBlock), 0, s, M, gw->ldv, gw->V, j + 1,
                             gw->w, gw->h1, 0, gw->part, gw->counter, gw->h2);
          hipLaunchKernelGGL(k_finish, dim3(nblk), dim3(kRedBlock), 0, s, M, gw->ldv, gw->V, j,
                             gw->w, gw->h1, gw->h2, gw->part, gw->counter, gw->H, gw->cs, gw->sn,
                             gw->g, sj, hj);
          hipLaunchKernelGGL(k_scale, dim3(mb), dim3(256), 0, s, M, gw->w, &sj->hnext, vn);
        }
        KFBI_HIP(hipGetLastError());
        KFBI_HIP(hipEventRecord(gw->ev[j % kRing], s));
        ++launched;
      }
      // examine step j - kLag (unless the prediction above already did)
      const int q = j - kLag;
      if (q < 0) continue;
      if (q >= launched) break;
      if (q >= examined) KFBI_TRY(examine(q));
    }
    if (zero) {
      if (zero_rhs) *zero_rhs = true;
      return KFBI_OK;
    }
    hipLaunchKernelGGL(k_update_x, dim3(mb), dim3(256), 0, s, M, m, gw->ldv, gw->V, gw->H, gw->g, x);
    KFBI_HIP(hipGetLastError());
  }
}

}  // namespace kfbi

using namespace kfbi;

namespace kfbi {
static int gmres_run(kfbi_ctx* c, int M, const GmresOp& op, const double* b, double* x,
                     const kfbi_gmres_opts* o, kfbi_gmres_stats* stats, GmresWork* gwp,
                     bool* last_at_x = nullptr);

static int gmres_solve_impl(kfbi_ctx* c, const kfbi_bie* op, const double* b, double* x,
                            const kfbi_gmres_opts* o, kfbi_gmres_stats* stats, bool use_static,
                            const kfbi_out* side = nullptr, bool* side_at_x = nullptr) {
  if (!c || !op || !b || !x || !o) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  if (!c->have_interface) {
    set_error("no interface installed");
    return KFBI_E_STATE;
  }
  if (c->box_bc == KFBI_BOX_USER) {
    set_error("GMRES needs box data defined by the density (ZERO, FREESPACE or NEUMANN)");
    return KFBI_E_INVALID;
  }
  if (o->restart < 1 || o->restart > kMaxRestart || o->maxit < 1 || !(o->tol > 0.0) ||
      (o->precision != KFBI_FP64 && o->precision != KFBI_FP32 && o->precision != KFBI_MIXED) ||
      (op->layer != KFBI_SINGLE && op->layer != KFBI_DOUBLE) || op->side < KFBI_PLUS ||
      op->side > KFBI_AVG) {
    set_error("invalid GMRES options or operator");
    return KFBI_E_INVALID;
  }
  GmresWork gw;
  if (use_static) {
    if (c->M > kStaticMaxM) {
      set_error("the static GMRES workspace holds at most %d markers (M = %d)", kStaticMaxM, c->M);
      return KFBI_E_INVALID;
    }
    KFBI_TRY(bind_static(c, &gw));
  } else {
    bind_work(c, &gw, c->M);
  }
  // the boundary operator a x + b trace(layer[x]) + q int x ds of the installed interface;
  // FP64 applies also write the side outputs (traces, normal derivatives) when asked
  const GmresOp op_fn = [c, op, side](const double* xin, double* yout, bool fp32) {
    return apply_impl(c, op->layer, fp32 ? KFBI_FP32 : KFBI_FP64, xin, nullptr,
                      fp32 ? nullptr : side, op, xin, yout);
  };
  return gmres_run(c, c->M, op_fn, b, x, o, stats, &gw, side_at_x);
}

// Restarted GMRES (FP64, FP32 iterative refinement or mixed) for the operator `op` on
// vectors of length M, in the workspace gw, on the stream of c.
// last_at_x (when given) tells whether the last FP64 operator call was at the returned x:
// true after a converged solve (its final true residual), false for a zero right-hand
// side (x set to zero after the residual of the initial guess) or an error.
static int gmres_run(kfbi_ctx* c, int M, const GmresOp& op, const double* b, double* x,
                     const kfbi_gmres_opts* o, kfbi_gmres_stats* stats, GmresWork* gwp,
                     bool* last_at_x) {
  GmresWork& gw = *gwp;
  if (last_at_x) *last_at_x = false;
  const int nblk = (M + kRedBlock - 1) / kRedBlock;
  kfbi_gmres_stats loc{};
  KFBI_HIP(hipMemsetAsync(gw.counter, 0, sizeof(unsigned int), c->stream));
  // ||b|| into its host slot, then the FP64 residual of the initial guess: one host
  // synchronisation for both
  hipLaunchKernelGGL(k_residual, dim3(nblk), dim3(kRedBlock), 0, c->stream, M, b, nullptr, nullptr,
                     gw.part, gw.counter, gw.st, gw.dring + kSlotNb);
  KFBI_HIP(hipGetLastError());
  double rn0 = 0.0;
  int a0 = 0;
  // FP64 and mixed: the first Arnoldi step is queued behind the initial residual without a
  // host synchronisation; the refinement loop needs the residual at once
  const bool lazy = (o->precision == KFBI_FP64 || o->precision == KFBI_MIXED);
  KFBI_TRY(true_residual(c, M, op, false, b, x, &gw, &rn0, &a0, !lazy));
  loc.applies64 = a0;
  double nb = lazy ? NAN : gw.hring[kSlotNb].resid;
  int status = KFBI_OK;
  if (lazy) {
    int applies = 0, applies32 = 0;
    bool zero_rhs = false;
    const double thresh =
        o->precision == KFBI_MIXED ? (o->inner_tol > 0.0 ? o->inner_tol : 1e-5) : 0.0;
    status = gmres_core(c, M, op, KFBI_FP64, b, x, nb, o->tol, o->restart, o->maxit, &gw,
                        &loc.iters, &loc.outer_iters, &applies, &loc.relres, true, rn0, thresh,
                        &applies32, true, &nb, &zero_rhs);
    loc.applies64 += applies;
    loc.applies32 += applies32;
    if (zero_rhs) {
      KFBI_HIP(hipMemsetAsync(x, 0, sizeof(double) * M, c->stream));
      nb = 0.0;
    }
    loc.converged = (status == KFBI_OK);
  } else if (nb == 0.0) {
    KFBI_HIP(hipMemsetAsync(x, 0, sizeof(double) * M, c->stream));
    KFBI_HIP(hipStreamSynchronize(c->stream));
    loc.converged = 1;
  } else {
    // iterative refinement: r = b - A64 x ; A32 d = r ; x += d
    const int mb = (M + 255) / 256;
    double prev = INFINITY;
    bool first = true;
    for (;;) {
      double rn = rn0;
      if (!first) {
        int a64 = 0;
        status = true_residual(c, M, op, false, b, x, &gw, &rn, &a64);
        loc.applies64 += a64;
        if (status != KFBI_OK) break;
      }
      first = false;
      loc.relres = rn / nb;
      if (!std::isfinite(rn)) {
        set_error("non-finite residual in refinement");
        status = KFBI_E_NONFINITE;
        break;
      }
      if (rn <= o->tol * nb) {
        loc.converged = 1;
        break;
      }
      if (loc.iters >= o->maxit || !(rn < prev)) {
        set_error("iterative refinement stalled (relres %.3e)", rn / nb);
        status = KFBI_E_NOCONV;
        break;
      }
      prev = rn;
      ++loc.outer_iters;
      // rhs of the correction equation: keep r in gw.d, solve for the correction in gw.w+?
      double* rr = gw.d;
      KFBI_HIP(hipMemcpyAsync(rr, gw.r, sizeof(double) * M, hipMemcpyDeviceToDevice, c->stream));
      double* dcorr = gw.dcorr;
      KFBI_HIP(hipMemsetAsync(dcorr, 0, sizeof(double) * M, c->stream));
      int it_in = 0, cyc = 0, a32 = 0;
      double rel_in = 0.0;
      const double itol = o->inner_tol > 0.0 ? o->inner_tol : 1e-5;
      // the correction starts from zero, so its first residual is r itself (still in gw.r
      // and the device status)
      const int st_in = gmres_core(c, M, op, KFBI_FP32, rr, dcorr, rn, itol, o->restart,
                                   o->maxit - loc.iters, &gw, &it_in, &cyc, &a32, &rel_in, true,
                                   rn);
      loc.iters += it_in;
      loc.applies32 += a32;
      if (st_in != KFBI_OK && st_in != KFBI_E_NOCONV) {
        status = st_in;
        break;
      }
      hipLaunchKernelGGL(k_axpy, dim3(mb), dim3(256), 0, c->stream, M, 1.0, dcorr, x);
      KFBI_HIP(hipGetLastError());
    }
  }
  KFBI_HIP(hipStreamSynchronize(c->stream));
  if (stats) *stats = loc;
  if (last_at_x) *last_at_x = (status == KFBI_OK && loc.converged && nb != 0.0);
  if (status == KFBI_E_NOCONV)
    set_error("GMRES did not reach tol %.3e in %d iterations (relres %.3e)", o->tol, loc.iters,
              loc.relres);
  return status;
}
}  // namespace kfbi

namespace kfbi {
// kfbi_gmres_solve whose FP64 applies also write the outputs `side` of the layer potential
// of their argument; on return *side_at_x tells whether those outputs belong to the
// returned solution (the last FP64 apply of a converged solve is its final true residual).
int gmres_solve_side(kfbi_ctx* c, const kfbi_bie* op, const double* b, double* x,
                     const kfbi_gmres_opts* o, kfbi_gmres_stats* stats, const kfbi_out* side,
                     bool* side_at_x) {
  return gmres_solve_impl(c, op, b, x, o, stats, false, side, side_at_x);
}

// GMRES with the workspace of c for an operator of the library on vectors of length
// n <= max_markers of c (FP64 only).
int gmres_solve_op(kfbi_ctx* c, int n, const GmresOp& op, const double* b, double* x,
                   const kfbi_gmres_opts* o, kfbi_gmres_stats* stats) {
  if (!b || !x || !o || n < 1 || n > c->max_markers) {
    set_error("invalid GMRES arguments (n = %d)", n);
    return KFBI_E_INVALID;
  }
  if (o->restart < 1 || o->restart > kMaxRestart || o->maxit < 1 || !(o->tol > 0.0) ||
      o->precision != KFBI_FP64) {
    set_error("invalid GMRES options (FP64 only for this operator)");
    return KFBI_E_INVALID;
  }
  GmresWork gw;
  bind_work(c, &gw, n);
  return gmres_run(c, n, op, b, x, o, stats, &gw);
}
}  // namespace kfbi

extern "C" int kfbi_gmres_solve(kfbi_ctx* c, const kfbi_bie* op, const double* b, double* x,
                                const kfbi_gmres_opts* o, kfbi_gmres_stats* stats) {
  return gmres_solve_impl(c, op, b, x, o, stats, false);
}

extern "C" int kfbi_gmres_solve_static(kfbi_ctx* c, const kfbi_bie* op, const double* b,
                                       double* x, const kfbi_gmres_opts* o,
                                       kfbi_gmres_stats* stats) {
  return gmres_solve_impl(c, op, b, x, o, stats, true);
}
