// Modified Stokes double-layer operator on the MAC grid (include/stokes.h).
//
// One apply of D phi (Sec. 3.3, eq. ms-bie; Sec. 4.2.2; App. A.2):
//   k_st_quant    Fourier derivatives of the density at the markers (circulant sums):
//                 Phi_1, Phi_1a, Phi_1aa, Phi_2, Phi_2a, Phi_2aa
//   k_st_jumps    App. A.2 at every interface crossing of the half-spacing grid and at
//                 every marker: 6-point Lagrange interpolation of the marker data, then
//                 the 5x5 and 8x8 systems by Gaussian elimination with partial pivoting
//                 (no traction jump, no forcing: the double layer)
//   k_st_rhs      corrected right-hand sides of eq. (crc-mac-fds), one thread per
//                 equation: every stencil point Q on the other side of the interface adds
//                 a_Q s_Q [w]_Q, the jump extended from the crossing on the segment P-Q by
//                 its Taylor polynomial (second order for velocities, first for pressure)
//   solve         conjugate gradients on the pressure Schur complement
//                 S = G^T (c^2 - Delta_h)^-1 G (G the pressure gradient at the velocity
//                 points), Cahouet-Chabard preconditioner c^2 L^-1 + I; the velocity
//                 solves and L^-1 by orthonormal sine / cosine transforms applied as
//                 dense products on FP64 MFMA (k_st_gemm), divided by the eigenvalues
//   k_st_extract  Sec. 4.3 on each velocity component's grid: six-point stencil, 6x6
//                 Taylor system with the marker jumps -> traces from both sides
// The labels and crossings of the u, v and p points come from the scalar geometry of a
// context on the grid of spacing h/2, whose nodes they are: u (2i, 2j-1), v (2i-1, 2j),
// p (2i-1, 2j-1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/stokes.h"
#include "common.h"
#include "device_util.h"

using namespace kfbi;

// Host-visible record of one CG iteration of the MAC solve (coherent pinned memory).
struct CgPost {
  double rn2, bn2;  // ||r||^2 after the iteration, ||b||^2
  int done, it;     // the residual test has passed; the iteration
  double pad;
};

struct stokes_ctx {
  kfbi_ctx* g2 = nullptr;  // geometry on the half-spacing grid, GMRES workspace
  double x0, y0, side, h, c2;
  int N, Mx;
  hipStream_t stream;
  double tol;
  int maxit;
  int M = 0, nc = 0, have = 0;
  int cg_iters = 0;
  double cg_relres = 0.0;
  DBuf Q, J, ru, rv, rp, u, v, p, S1, S2, C2, S2T, C2T, wk, part, sc, flag;
  CgPost* hpost = nullptr;  // CG records: host view of coherent pinned memory
  CgPost* dpost = nullptr;  // the same memory as the kernels address it
  hipEvent_t ev[4] = {};           // one per record slot
};

namespace {

constexpr int kNJ = 15;  // jump values per point: u, ux, uy, uxx, uyy, uxy, v.., p, px, py
enum { JU = 0, JUX, JUY, JUXX, JUYY, JUXY, JV, JVX, JVY, JVXX, JVYY, JVXY, JP, JPX, JPY };
// device scalars of the CG recurrences
// (SC_RZ, SC_RZ + 1: r . z of even and odd iterations; SC_DONE: the residual test passed)
enum { SC_RZ = 0, SC_DQ = 2, SC_RN, SC_BN, SC_MEAN, SC_DONE, SC_COUNT = 8 };
constexpr int kRedBlocks = 256;

inline int nblk(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

// ----------------------------------------------------------------- transform matrices
// Orthonormal transform matrices (row = mode) and the transposes of S2 and C2 (every
// product then reads its operands along rows):
//   S1[k-1][i-1] = sqrt(2/N) sin(k i pi / N),            k, i = 1..N-1   (DST-I)
//   S2[l-1][j-1] = w_l sin(l (j - 1/2) pi / N),          l, j = 1..N     (DST-II)
//   C2[k][i-1]   = w_k cos(k (i - 1/2) pi / N),          k = 0..N-1      (DCT-II)
// with w = sqrt(2/N), except sqrt(1/N) for l = N (DST-II) and k = 0 (DCT-II).
__global__ void k_st_trmat(int N, double* __restrict__ S1, double* __restrict__ S2,
                           double* __restrict__ C2, double* __restrict__ S2T,
                           double* __restrict__ C2T) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int r = e / N, c = e % N;
  const double w = sqrt(2.0 / N), w1 = sqrt(1.0 / N);
  double sn, cs;
  if (r < N - 1 && c < N - 1) {  // S1 (N-1) x (N-1)
    const long long m = (static_cast<long long>(r + 1) * (c + 1)) % (2 * N);
    sincospi(static_cast<double>(m) / N, &sn, &cs);
    S1[r * (N - 1) + c] = w * sn;
  }
  {  // S2: l = r + 1, j = c + 1: angle l (2j - 1) pi / (2N)
    const long long m = (static_cast<long long>(r + 1) * (2 * c + 1)) % (4 * N);
    sincospi(static_cast<double>(m) / (2 * N), &sn, &cs);
    S2[r * N + c] = S2T[c * N + r] = (r + 1 == N ? w1 : w) * sn;
  }
  {  // C2: k = r, i = c + 1
    const long long m = (static_cast<long long>(r) * (2 * c + 1)) % (4 * N);
    sincospi(static_cast<double>(m) / (2 * N), &sn, &cs);
    C2[r * N + c] = C2T[c * N + r] = (r == 0 ? w1 : w) * cs;
  }
}

// ---------------------------------------------------------------------- dense product
// C (m x n, row-major, ldc) = A (m x k) B (k x n), A row-major with row stride lda, B with
// row stride ldb.  32 x 32 output tiles per block of four wavefronts, each wavefront one
// 16 x 16 quadrant by v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16 x 4 by 4 x 16 step and holds D[4 i + l / 16][l % 16] in element
// i of its accumulator).  k runs in chunks of 32 through LDS; the loads of the next chunk
// are issued before the products of the current one.  A block holds two or four such
// groups of four wavefronts, each on its own share of k with its own chunk buffers, and
// adds their tiles in group order at the end (deterministic): the grids of these
// transforms are small (256 tiles at N = 512), and several wavefronts per SIMD instead of
// one keep the matrix cores busy while the chunk loads are in flight.
//
// One launch computes up to two independent products (blockIdx.z selects the argument
// set: the u and v velocity solves run side by side).  Operand A can be formed on the fly
// as the pressure gradient of a cell array (amode), and the result can be divided by the
// eigenvalues of a transform basis and have a matrix added (epi, D) as it is stored.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kGT = 32;   // output tile
constexpr int kGK = 32;   // k-chunk staged in LDS
constexpr int kLdk = kGK + 2;  // LDS row of a chunk buffer: 16-byte reads of consecutive rows
                               // land in different banks
static_assert(kGK % 8 == 0 && 2 * kGT * kLdk >= kGT * (kGT + 1),
              "a group's chunk buffers hold at least one partial tile");
enum { AM_PLAIN = 0, AM_GRAD_U, AM_GRAD_V };      // A = A, (G p) at u points, at v points
enum { EP_NONE = 0, EP_VEL, EP_CELL };            // C = acc, acc / (lam + c^2), c^2 acc / lam
struct GemmArgs {
  int m, n, k, lda, ldb, ldc;
  const double* A;  // AM_GRAD_*: the N x N cell array p
  const double* B;
  double* C;
  const double* D;  // added to the result when not null (row stride ldc)
  int amode, epi;
};
struct GemmConst {
  int N;
  double ih, ih2, c2;
};

__device__ __forceinline__ double gemm_a(const GemmArgs& g, const GemmConst& gc, int r, int c) {
  if (g.amode == AM_GRAD_U)  // u point (c + 1, r + 1): (p(c + 2, r + 1) - p(c + 1, r + 1)) / h
    return (g.A[r * gc.N + c + 1] - g.A[r * gc.N + c]) * gc.ih;
  if (g.amode == AM_GRAD_V)  // v point (c + 1, r + 1): (p(c + 1, r + 2) - p(c + 1, r + 1)) / h
    return (g.A[(r + 1) * gc.N + c] - g.A[r * gc.N + c]) * gc.ih;
  return g.A[static_cast<size_t>(r) * g.lda + c];
}

// Eigenvalue factor of output (r, c): EP_VEL, both directions sine modes r + 1 and c + 1
// (DST-I or DST-II, the same eigenvalues 4/h^2 sin^2(k pi / 2N)); EP_CELL, cosine modes r
// and c (DCT-II), the (0, 0) mode set to zero.
__device__ __forceinline__ double gemm_epi(int epi, const GemmConst& gc, int r, int c, double v) {
  if (epi == EP_NONE) return v;
  const int l = (epi == EP_CELL) ? r : r + 1, k = (epi == EP_CELL) ? c : c + 1;
  const double sl = sinpi(static_cast<double>(l) / (2 * gc.N));
  const double sk = sinpi(static_cast<double>(k) / (2 * gc.N));
  const double lam = 4.0 * gc.ih2 * (sl * sl + sk * sk);
  if (epi == EP_CELL) return (l == 0 && k == 0) ? 0.0 : v * (gc.c2 / lam);
  return v / (lam + gc.c2);
}

template <int kKS>  // k-slice groups per block
__global__ void __launch_bounds__(256 * kKS)
    k_st_gemm(GemmArgs g0, GemmArgs g1, GemmConst gc) {
  const GemmArgs g = blockIdx.z ? g1 : g0;  // block-uniform
  const int m = g.m, n = g.n, k = g.k;
  const int r0 = blockIdx.y * kGT, c0 = blockIdx.x * kGT;
  if (r0 >= m || c0 >= n) return;  // the other product's grid is larger
  // k-slice group ks of four wavefronts: its own chunk buffers, A as [row][k] and B
  // transposed as [col][k], rows padded to kLdk doubles; after the loop the same LDS
  // holds the groups' partial tiles
  __shared__ __align__(16) double lds[kKS * 2 * kGT * kLdk];
  const int tid = threadIdx.x & 255, ks = threadIdx.x >> 8;
  double (*As)[kLdk] = reinterpret_cast<double (*)[kLdk]>(lds + ks * 2 * kGT * kLdk);
  double (*Bt)[kLdk] = reinterpret_cast<double (*)[kLdk]>(lds + (ks * 2 + 1) * kGT * kLdk);
  const int lane = tid & 63, w = tid >> 6;
  const int wr = 16 * (w >> 1), wc = 16 * (w & 1);
  const int lr = lane & 15, lk = lane >> 4;
  // this group's k range: whole chunks
  const int nch = (k + kGK - 1) / kGK;
  const int per = (nch + kKS - 1) / kKS;
  const int kb = ks * per * kGK, ke = min(k, (ks + 1) * per * kGK);
  // this thread's elements of a chunk: A row e / kGK, k e % kGK; B k e / kGT, column
  // e % kGT (e = tid + 256 q)
  constexpr int QA = kGT * kGK / 256, QB = kGK * kGT / 256;
  double pa[QA], pb[QB];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + 256 * q;
      const int gr = r0 + e / kGK, gk = k0 + e % kGK;
      pa[q] = (gr < m && gk < ke) ? gemm_a(g, gc, gr, gk) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + 256 * q;
      const int gkb = k0 + e / kGT, gcol = c0 + e % kGT;
      pb[q] = (gkb < ke && gcol < n) ? g.B[static_cast<size_t>(gkb) * g.ldb + gcol] : 0.0;
    }
  };
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  load(kb);
  // every group runs the same number of chunks (the last ones may be empty: zeros), so
  // the block-wide barriers match
  for (int c = 0; c < per; ++c) {
    const int k0 = kb + c * kGK;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + 256 * q;
      As[e / kGK][e % kGK] = pa[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + 256 * q;
      Bt[e % kGT][e / kGT] = pb[q];
    }
    __syncthreads();
    if (c + 1 < per) load(k0 + kGK);  // in flight during the products below
    // two products per 16-byte read: lane (lr, lk) takes k = kk + 2 lk in the first and
    // kk + 2 lk + 1 in the second, the same k for A and B (any assignment of the chunk's
    // k to (product, lk) that A and B share gives the same sums)
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 8) {
      const double2 a2 = *reinterpret_cast<const double2*>(&As[wr + lr][kk + 2 * lk]);
      const double2 b2 = *reinterpret_cast<const double2*>(&Bt[wc + lr][kk + 2 * lk]);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.x, b2.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.y, b2.y, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // the groups' tiles added in group order
  double (*red)[kGT][kGT + 1] = reinterpret_cast<double (*)[kGT][kGT + 1]>(lds);
  if (ks > 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[ks - 1][wr + 4 * i + lk][wc + lr] = acc[i];
  }
  __syncthreads();
  if (ks > 0) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = acc[i];
    for (int q = 1; q < kKS; ++q) v += red[q - 1][wr + 4 * i + lk][wc + lr];
    const int gr = r0 + wr + 4 * i + lk, gcol = c0 + wc + lr;
    if (gr < m && gcol < n) {
      const size_t o = static_cast<size_t>(gr) * g.ldc + gcol;
      v = gemm_epi(g.epi, gc, gr, gcol, v);
      if (g.D) v += g.D[o];
      g.C[o] = v;
    }
  }
}

// ------------------------------------------------------------------- pointwise stencils
// Pressure gradient at the interior velocity points: gu[j-1][i-1] = (p(i+1, j) - p(i, j))/h
// (i = 1..N-1, j = 1..N), gv[j-1][i-1] = (p(i, j+1) - p(i, j))/h (i = 1..N, j = 1..N-1),
// p[j-1][i-1]; with add, gu/gv += the given face values first (fu, fv).
__global__ void k_st_grad(int N, double ih, const double* __restrict__ p,
                          const double* __restrict__ fu, const double* __restrict__ fv,
                          double* __restrict__ gu, double* __restrict__ gv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nu = N * (N - 1);
  if (e < nu) {
    const int j = e / (N - 1), i = e % (N - 1);  // u point (i + 1, j + 1)
    const double g = (p[j * N + i + 1] - p[j * N + i]) * ih;
    gu[e] = fu ? fu[e] + g : g;
  } else if (e < 2 * nu) {
    const int f = e - nu;
    const int j = f / N, i = f % N;  // v point (i + 1, j + 1)
    const double g = (p[(j + 1) * N + i] - p[j * N + i]) * ih;
    gv[f] = fv ? fv[f] + g : g;
  }
}

// out[j-1][i-1] = a G^T z + b base = a ((zu(i-1, j) - zu(i, j)) + (zv(i, j-1) - zv(i, j)))/h
// + b base (zero velocity on the box faces).
__global__ void k_st_gradT(int N, double ih, const double* __restrict__ zu,
                           const double* __restrict__ zv, double a, const double* __restrict__ base,
                           double b, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int j = e / N, i = e % N;  // cell (i + 1, j + 1)
  const double uw = (i >= 1) ? zu[j * (N - 1) + i - 1] : 0.0;
  const double ue = (i <= N - 2) ? zu[j * (N - 1) + i] : 0.0;
  const double vs = (j >= 1) ? zv[(j - 1) * N + i] : 0.0;
  const double vn = (j <= N - 2) ? zv[j * N + i] : 0.0;
  const double g = ((uw - ue) + (vs - vn)) * ih;
  out[e] = a * g + (base ? b * base[e] : 0.0);
}

// Reductions in two steps without atomics or fences: a launch of at most kRedBlocks
// blocks (grid-stride) stores one partial sum per block, and a later launch adds them in
// block order (every block of it that needs the total forms it itself, so all of them
// hold the same value whatever order the blocks run in).
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int np,
                                            double* scratch) {
  const double v = (static_cast<int>(threadIdx.x) < np) ? part[threadIdx.x] : 0.0;
  return block_sum<double>(v, scratch);
}

// part[block] = partial sum of a . b (a . a when b is null and sq, of a when b is null and
// not sq)
__global__ void __launch_bounds__(256)
    k_st_dot(int n, const double* __restrict__ a, const double* __restrict__ b, int sq,
             double* __restrict__ part) {
  __shared__ double scratch[16];
  double s = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256)
    s += b ? a[e] * b[e] : (sq ? a[e] * a[e] : a[e]);
  s = block_sum<double>(s, scratch);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// *out = scale * (sum of the np partials)
__global__ void __launch_bounds__(256)
    k_st_dot_fin(int np, const double* __restrict__ part, double* __restrict__ out, double scale) {
  __shared__ double scratch[16];
  const double s = sum_parts(part, np, scratch);
  if (threadIdx.x == 0) *out = s * scale;
}

// x -= sc[slot] (mean removal); y = x otherwise
__global__ void k_st_sub_scalar(int n, const double* __restrict__ sc, int slot,
                                const double* __restrict__ x, double* __restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = x[e] - sc[slot];
}

// CG on the Schur complement, iteration it (rz_it = sc[SC_RZ + it % 2]).  Once the
// residual test has passed (sc[SC_DONE] set) the updates are skipped, so iterations
// launched ahead of the host's convergence check leave the solution unchanged.  The
// partial sums of d . q, r . r and r . z sit at part + {0, 1, 2} kRedBlocks.
//
// q = G^T z (cells, zero velocity on the box faces) and the partials of d . q
__global__ void __launch_bounds__(256)
    k_st_gradT_dot(int N, double ih, const double* __restrict__ zu,
                   const double* __restrict__ zv, const double* __restrict__ d,
                   double* __restrict__ q, double* __restrict__ part) {
  __shared__ double scratch[16];
  double dq = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < N * N; e += gridDim.x * 256) {
    const int j = e / N, i = e % N;  // cell (i + 1, j + 1)
    const double uw = (i >= 1) ? zu[j * (N - 1) + i - 1] : 0.0;
    const double ue = (i <= N - 2) ? zu[j * (N - 1) + i] : 0.0;
    const double vs = (j >= 1) ? zv[(j - 1) * N + i] : 0.0;
    const double vn = (j <= N - 2) ? zv[j * N + i] : 0.0;
    const double g = ((uw - ue) + (vs - vn)) * ih;
    q[e] = g;
    dq += d[e] * g;
  }
  dq = block_sum<double>(dq, scratch);
  if (threadIdx.x == 0) part[blockIdx.x] = dq;
}

// p += alpha d, r -= alpha q (alpha = rz_it / (d . q)) unless done; partials of r . r
__global__ void __launch_bounds__(256)
    k_st_cg_step(int n, int it, int np, const double* __restrict__ sc, double* __restrict__ p,
                 double* __restrict__ r, const double* __restrict__ d,
                 const double* __restrict__ q, double* __restrict__ part) {
  __shared__ double scratch[16];
  const bool done = sc[SC_DONE] != 0.0;
  const double dq = sum_parts(part, np, scratch);
  const double alpha = sc[SC_RZ + (it & 1)] / dq;
  double rr = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    double re = r[e];
    if (!done) {
      p[e] += alpha * d[e];
      re -= alpha * q[e];
      r[e] = re;
    }
    rr += re * re;
  }
  rr = block_sum<double>(rr, scratch);
  if (threadIdx.x == 0) part[kRedBlocks + blockIdx.x] = rr;
}

// The residual test ||r||^2 <= tol2 ||b||^2 (sticky in sc[SC_DONE]), then, unless it has
// passed, d = z + beta d (beta = rz_{it+1} / rz_it); block 0 stores the new flag and
// rz_{it+1} and writes the record for the host.  Every block forms the test from the same
// partials, so all agree, and a block that reads the flag block 0 has already updated
// reaches the same decision (the flag only ever turns on, with this test).
__global__ void __launch_bounds__(256)
    k_st_cg_dir(int n, int it, int np, double tol2, double* __restrict__ sc,
                const double* __restrict__ z, double* __restrict__ d,
                const double* __restrict__ part, CgPost* __restrict__ post) {
  __shared__ double scratch[16];
  const double rn2 = sum_parts(part + kRedBlocks, np, scratch);
  const double rz = sum_parts(part + 2 * kRedBlocks, np, scratch);
  const double bn2 = sc[SC_BN];
  const double rz_old = sc[SC_RZ + (it & 1)];
  const bool done = (sc[SC_DONE] != 0.0) || rn2 <= tol2 * bn2;
  __syncthreads();  // every thread has read the scalars before block 0 replaces them
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[SC_RZ + ((it + 1) & 1)] = rz;
    sc[SC_RN] = rn2;
    sc[SC_DONE] = done ? 1.0 : 0.0;
    post->rn2 = rn2;
    post->bn2 = bn2;
    post->done = done ? 1 : 0;
    post->it = it;
    __threadfence_system();
  }
  if (done) return;
  const double beta = rz / rz_old;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256)
    d[e] = z[e] + beta * d[e];
}

// Start of the CG: done at once for a zero right-hand side.
__global__ void k_st_cg_init(double* __restrict__ sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[SC_DONE] = (sc[SC_BN] > 0.0) ? 0.0 : 1.0;
}

// Full velocity fields from the interior unknowns (sign s): u [N][N+1] with u = 0 on the
// columns i = 0, N; v [N+1][N] with v = 0 on the rows j = 0, N.
__global__ void k_st_fields(int N, double s, const double* __restrict__ zu,
                            const double* __restrict__ zv, double* __restrict__ u,
                            double* __restrict__ v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nu = N * (N + 1);
  if (e < nu) {
    const int j = e / (N + 1), i = e % (N + 1);
    u[e] = (i == 0 || i == N) ? 0.0 : s * zu[j * (N - 1) + i - 1];
  } else if (e < 2 * nu) {
    const int f = e - nu;
    const int j = f / N, i = f % N;
    v[f] = (j == 0 || j == N) ? 0.0 : s * zv[(j - 1) * N + i];
  }
}

// ---------------------------------------------------------------- interface quantities
// Markers outside [lo, hi]^2 (the 3h margin): flag set.
__global__ void k_st_margin(int M, const double* __restrict__ X, double xlo, double xhi,
                            double ylo, double yhi, int* __restrict__ flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double x = X[k], y = X[M + k];
  if (!(x >= xlo && x <= xhi && y >= ylo && y <= yhi)) atomicMax(flag, 1);
}

// Q[c][k], c = 0..5: phi_1, its first and second Fourier derivatives, then phi_2's, with
// f'(a_k) = sum_m d1[(k - m) mod M] f_m and f'' by d2 (differentiation vectors of the
// geometry context).
// Block (g, comp): the derivatives of component comp at markers 8g .. 8g + 7.  The
// density and both circulant coefficient rows are staged in LDS; thread t sums the terms
// m = t, t + 256, ... of all sixteen outputs, and the partial sums are added in a fixed
// order (wavefront shuffles, then the four wavefronts).
constexpr int kQuantOut = 8;
__global__ void __launch_bounds__(256)
    k_st_quant(int M, const double* __restrict__ phi, const double* __restrict__ d1,
               const double* __restrict__ d2, double* __restrict__ Q) {
  extern __shared__ double qs[];  // f, d1, d2: 3M
  __shared__ double red[4][2 * kQuantOut];
  const int comp = blockIdx.y, k0 = blockIdx.x * kQuantOut;
  const double* f = phi + comp * M;
  double* fs = qs;
  double* c1 = qs + M;
  double* c2 = qs + 2 * M;
  for (int m = threadIdx.x; m < M; m += 256) {
    fs[m] = f[m];
    c1[m] = d1[m];
    c2[m] = d2[m];
  }
  __syncthreads();
  double s1[kQuantOut], s2[kQuantOut];
#pragma unroll
  for (int r = 0; r < kQuantOut; ++r) s1[r] = s2[r] = 0.0;
  for (int m = threadIdx.x; m < M; m += 256) {
    const double fm = fs[m];
#pragma unroll
    for (int r = 0; r < kQuantOut; ++r) {
      int q = k0 + r - m;
      q += (q < 0) ? M : 0;
      q -= (q >= M) ? M : 0;
      s1[r] += c1[q] * fm;
      s2[r] += c2[q] * fm;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < kQuantOut; ++r) {
    const double a = wave_sum(s1[r]), b = wave_sum(s2[r]);
    if (lane == 0) {
      red[w][r] = a;
      red[w][kQuantOut + r] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < kQuantOut) {
    const int r = threadIdx.x, k = k0 + r;
    if (k < M) {
      Q[(3 * comp) * M + k] = fs[k];
      Q[(3 * comp + 1) * M + k] = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
      Q[(3 * comp + 2) * M + k] =
          ((red[0][kQuantOut + r] + red[1][kQuantOut + r]) + red[2][kQuantOut + r]) +
          red[3][kQuantOut + r];
    }
  }
}

// Gaussian elimination with partial pivoting of an n x n system in registers (b
// overwritten by the solution).
template <int n>
__device__ __forceinline__ void gauss(double (&A)[n][n], double (&b)[n]) {
#pragma unroll
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r][c]) > best) {
        best = fabs(A[r][c]);
        piv = r;
      }
#pragma unroll
    for (int r = c; r < n; ++r) {  // swap rows c and piv (branch-free over registers)
      if (r == piv && r != c) {
#pragma unroll
        for (int q = 0; q < n; ++q) {
          const double t = A[c][q];
          A[c][q] = A[r][q];
          A[r][q] = t;
        }
        const double t = b[c];
        b[c] = b[r];
        b[r] = t;
      }
    }
    const double inv = 1.0 / A[c][c];
#pragma unroll
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r][c] * inv;
#pragma unroll
      for (int q = c; q < n; ++q) A[r][q] -= f * A[c][q];
      b[r] -= f * b[c];
    }
  }
#pragma unroll
  for (int c = n - 1; c >= 0; --c) {
    double s = b[c];
#pragma unroll
    for (int q = c + 1; q < n; ++q) s -= A[c][q] * b[q];
    b[c] = s / A[c][c];
  }
}

// App. A.2 jumps at point e: crossings e < nc (marker interval k, parameter t), markers
// e = nc + k (t = 0).  J[q][e], q over the kNJ values.
__global__ void k_st_jumps(int M, int nc, const Crossing* __restrict__ cr,
                           const double* __restrict__ geo, const double* __restrict__ Q,
                           double c2, double* __restrict__ J) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int npt = nc + M;
  if (e >= npt) return;
  int k;
  double t;
  if (e < nc) {
    k = cr[e].k;
    t = cr[e].t;
  } else {
    k = e - nc;
    t = 0.0;
  }
  // 6-point Lagrange weights on t_m = m - 2 (markers k-2..k+3)
  double w[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double num = 1.0, den = 1.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (q != m) {
        num *= (t - (q - 2));
        den *= static_cast<double>(m - q);
      }
    w[m] = num / den;
  }
  double g[4] = {0, 0, 0, 0}, d[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    int q = k - 2 + m;
    q += (q < 0) ? M : 0;
    q -= (q >= M) ? M : 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] += w[m] * geo[c * M + q];
#pragma unroll
    for (int c = 0; c < 6; ++c) d[c] += w[m] * Q[c * M + q];
  }
  const double xa = g[0], ya = g[1], xaa = g[2], yaa = g[3];
  const double P1 = d[0], P1a = d[1], P1aa = d[2], P2 = d[3], P2a = d[4], P2aa = d[5];
  // 5x5: ([u_x], [u_y], [v_x], [v_y], [p]); no traction jump
  double A5[5][5] = {{xa, ya, 0, 0, 0},
                     {0, 0, xa, ya, 0},
                     {2 * ya, -xa, -xa, 0, -ya},
                     {0, ya, ya, -2 * xa, xa},
                     {1, 0, 0, 1, 0}};
  double b5[5] = {P1a, P2a, 0.0, 0.0, 0.0};
  gauss<5>(A5, b5);
  const double ux = b5[0], uy = b5[1], vx = b5[2], vy = b5[3], p = b5[4];
  // 8x8: ([u_xx], [u_yy], [u_xy], [v_xx], [v_yy], [v_xy], [p_x], [p_y])
  double A8[8][8] = {
      {xa * xa, ya * ya, 2 * xa * ya, 0, 0, 0, 0, 0},
      {0, 0, 0, xa * xa, ya * ya, 2 * xa * ya, 0, 0},
      {2 * xa * ya, -xa * ya, 2 * ya * ya - xa * xa, -xa * xa, 0, -xa * ya, -xa * ya, -ya * ya},
      {0, ya * ya, xa * ya, xa * ya, -2 * xa * ya, ya * ya - 2 * xa * xa, xa * xa, xa * ya},
      {1, 1, 0, 0, 0, 0, -1, 0},
      {0, 0, 0, 1, 1, 0, 0, -1},
      {1, 0, 0, 0, 0, 1, 0, 0},
      {0, 0, 1, 0, 1, 0, 0, 0}};
  double b8[8] = {P1aa - xaa * ux - yaa * uy,
                  P2aa - xaa * vx - yaa * vy,
                  -2 * yaa * ux + xaa * uy + xaa * vx + yaa * p,
                  -yaa * uy - yaa * vx + 2 * xaa * vy - xaa * p,
                  c2 * P1,
                  c2 * P2,
                  0.0,
                  0.0};
  gauss<8>(A8, b8);
  const double out[kNJ] = {P1, ux, uy, b8[0], b8[1], b8[2], P2, vx, vy, b8[3], b8[4], b8[5],
                           p, b8[6], b8[7]};
#pragma unroll
  for (int q = 0; q < kNJ; ++q) J[static_cast<size_t>(q) * npt + e] = out[q];
}

// Correction a s_Q [w]_Q of the stencil pair P -> Q (nodes of the half-spacing grid, on
// one row or one column, one or two steps apart) for the quantity whose jump values
// start at J index jq (JU, JV or JP; the pressure extension is first order).
__device__ __forceinline__ double pair_corr(int Pi, int Pj, int Qi, int Qj, double a, int jq,
                                            int n1, const int8_t* __restrict__ lab,
                                            const int* __restrict__ hid,
                                            const int* __restrict__ vid,
                                            const Crossing* __restrict__ cr,
                                            const double* __restrict__ J, int npt, double x0,
                                            double y0, double h2, int* __restrict__ err) {
  const int8_t lq = lab[Qj * n1 + Qi];
  if (lab[Pj * n1 + Pi] == lq) return 0.0;
  int c = -1, found = 0;
  const bool horiz = (Pj == Qj);
  const int lo = horiz ? min(Pi, Qi) : min(Pj, Qj), hi = horiz ? max(Pi, Qi) : max(Pj, Qj);
  for (int s = lo; s < hi; ++s) {
    const int id = horiz ? hid[Pj * n1 + s] : vid[s * n1 + Pi];
    if (id >= 0) {
      c = id;
      ++found;
    }
  }
  if (found != 1) {
    atomicMax(err, 1);
    return 0.0;
  }
  const double d = horiz ? (x0 + Qi * h2) - cr[c].pos : (y0 + Qj * h2) - cr[c].pos;
  const double j0 = J[static_cast<size_t>(jq) * npt + c];
  const double j1 = J[static_cast<size_t>(jq + (horiz ? 1 : 2)) * npt + c];
  double wq = j0 + d * j1;
  if (jq != JP) wq += 0.5 * d * d * J[static_cast<size_t>(jq + (horiz ? 3 : 4)) * npt + c];
  return a * (lq ? 1.0 : -1.0) * wq;
}

// Corrected right-hand sides (no forcing): ru [N][N-1] (u points), rv [N-1][N] (v
// points), rp [N][N] (cells); one thread per equation.
__global__ void k_st_rhs(int N, double h, double x0, double y0, const int8_t* __restrict__ lab,
                         const int* __restrict__ hid, const int* __restrict__ vid,
                         const Crossing* __restrict__ cr, const double* __restrict__ J, int npt,
                         double* __restrict__ ru, double* __restrict__ rv,
                         double* __restrict__ rp, int* __restrict__ err) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nu = N * (N - 1);
  const int n1 = 2 * N + 1;
  const double ih2 = 1.0 / (h * h), ih = 1.0 / h, h2 = 0.5 * h;
#define PC(PI, PJ, QI, QJ, A, Q) \
  pair_corr(PI, PJ, QI, QJ, A, Q, n1, lab, hid, vid, cr, J, npt, x0, y0, h2, err)
  if (e < nu) {  // u point (i, j), i = 1..N-1, j = 1..N
    const int j = e / (N - 1) + 1, i = e % (N - 1) + 1;
    const int Pi = 2 * i, Pj = 2 * j - 1;
    double s = PC(Pi, Pj, Pi - 2, Pj, ih2, JU) + PC(Pi, Pj, Pi + 2, Pj, ih2, JU);
    if (j >= 2) s += PC(Pi, Pj, Pi, Pj - 2, ih2, JU);
    if (j <= N - 1) s += PC(Pi, Pj, Pi, Pj + 2, ih2, JU);
    s += PC(Pi, Pj, Pi + 1, Pj, -ih, JP) + PC(Pi, Pj, Pi - 1, Pj, ih, JP);
    ru[e] = s;
  } else if (e < 2 * nu) {  // v point (i, j), i = 1..N, j = 1..N-1
    const int f = e - nu;
    const int j = f / N + 1, i = f % N + 1;
    const int Pi = 2 * i - 1, Pj = 2 * j;
    double s = PC(Pi, Pj, Pi, Pj - 2, ih2, JV) + PC(Pi, Pj, Pi, Pj + 2, ih2, JV);
    if (i >= 2) s += PC(Pi, Pj, Pi - 2, Pj, ih2, JV);
    if (i <= N - 1) s += PC(Pi, Pj, Pi + 2, Pj, ih2, JV);
    s += PC(Pi, Pj, Pi, Pj + 1, -ih, JP) + PC(Pi, Pj, Pi, Pj - 1, ih, JP);
    rv[f] = s;
  } else if (e < 2 * nu + N * N) {  // cell (i, j)
    const int f = e - 2 * nu;
    const int j = f / N + 1, i = f % N + 1;
    const int Pi = 2 * i - 1, Pj = 2 * j - 1;
    rp[f] = PC(Pi, Pj, Pi + 1, Pj, ih, JU) + PC(Pi, Pj, Pi - 1, Pj, -ih, JU) +
            PC(Pi, Pj, Pi, Pj + 1, ih, JV) + PC(Pi, Pj, Pi, Pj - 1, -ih, JV);
  }
#undef PC
}

// Traces at marker k (Sec. 4.3 on each component's grid): plus/minus [2][M].
__global__ void k_st_extract(int M, int N, double h, double x0, double y0,
                             const double* __restrict__ X, const int8_t* __restrict__ lab,
                             const double* __restrict__ J, int nc, const double* __restrict__ u,
                             const double* __restrict__ v, double* __restrict__ plus,
                             double* __restrict__ minus) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * M) return;
  const int comp = e / M, k = e % M;
  const int npt = nc + M, pe = nc + k;
  const int n1 = 2 * N + 1;
  const double px = X[k], py = X[M + k];
  const double ox = comp == 0 ? x0 : x0 - 0.5 * h;
  const double oy = comp == 0 ? y0 - 0.5 * h : y0;
  const int jb = comp == 0 ? JU : JV;
  const double jv = J[static_cast<size_t>(jb) * npt + pe];
  const double jx = J[static_cast<size_t>(jb + 1) * npt + pe];
  const double jy = J[static_cast<size_t>(jb + 2) * npt + pe];
  const double jxx = J[static_cast<size_t>(jb + 3) * npt + pe];
  const double jyy = J[static_cast<size_t>(jb + 4) * npt + pe];
  const double jxy = J[static_cast<size_t>(jb + 5) * npt + pe];
  const int i0 = static_cast<int>(floor((px - ox) / h + 0.5));
  const int j0 = static_cast<int>(floor((py - oy) / h + 0.5));
  const int d1 = (px > ox + i0 * h) ? 1 : -1;
  const int d2 = (py > oy + j0 * h) ? 1 : -1;
  const int si[6] = {0, 1, 0, 0, -1, d1}, sj[6] = {0, 0, 1, -1, 0, d2};
  double A[6][6], b[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int I = i0 + si[m], Jj = j0 + sj[m];
    const double dx = (ox + I * h - px) / h, dy = (oy + Jj * h - py) / h;
    A[m][0] = 1.0;
    A[m][1] = dx;
    A[m][2] = dy;
    A[m][3] = 0.5 * dx * dx;
    A[m][4] = dx * dy;
    A[m][5] = 0.5 * dy * dy;
    double val;
    int8_t in;
    if (comp == 0) {
      val = u[(Jj - 1) * (N + 1) + I];
      in = lab[(2 * Jj - 1) * n1 + 2 * I];
    } else {
      val = v[Jj * N + I - 1];
      in = lab[(2 * Jj) * n1 + 2 * I - 1];
    }
    const double Dx = dx * h, Dy = dy * h;
    const double C = jv + Dx * jx + Dy * jy + 0.5 * (Dx * Dx * jxx + 2.0 * Dx * Dy * jxy + Dy * Dy * jyy);
    b[m] = in ? val : val + C;
  }
  gauss<6>(A, b);
  if (plus) plus[comp * M + k] = b[0];
  if (minus) minus[comp * M + k] = b[0] - jv;
}

// ------------------------------------------------------------------------- host side
struct Work {
  double *zu, *zv, *gu, *gv, *t1, *t1v, *pv, *r, *z, *d, *q, *b;
};

Work bind(stokes_ctx* st) {
  const size_t NN = static_cast<size_t>(st->N) * st->N;
  double* w = st->wk.as<double>();
  Work k;
  double** f[] = {&k.zu, &k.zv, &k.gu, &k.gv, &k.t1, &k.t1v, &k.pv, &k.r, &k.z, &k.d, &k.q, &k.b};
  for (size_t i = 0; i < sizeof(f) / sizeof(f[0]); ++i) *f[i] = w + i * NN;
  return k;
}
constexpr int kWorkFields = 12;
constexpr int kPostRing = 4;  // CG records in flight (at most two iterations are unexamined)
static_assert(sizeof(stokes_ctx::ev) / sizeof(hipEvent_t) == kPostRing, "one event per record");

GemmArgs ga(int m, int n, int k, const double* A, int lda, const double* B, int ldb, double* C,
            int ldc, int epi = EP_NONE, int amode = AM_PLAIN, const double* D = nullptr) {
  GemmArgs g;
  g.m = m;
  g.n = n;
  g.k = k;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.A = A;
  g.B = B;
  g.C = C;
  g.D = D;
  g.amode = amode;
  g.epi = epi;
  return g;
}

GemmConst gconst(const stokes_ctx* st) {
  return GemmConst{st->N, 1.0 / st->h, 1.0 / (st->h * st->h), st->c2};
}

// One product, or two independent ones in the same launch.
void gemm(stokes_ctx* st, const GemmArgs& a, const GemmArgs* b = nullptr) {
  int gx = nblk(a.n, kGT), gy = nblk(a.m, kGT);
  if (b) {
    gx = std::max(gx, nblk(b->n, kGT));
    gy = std::max(gy, nblk(b->m, kGT));
  }
  // a single product: four k-groups per block (one block per CU, four wavefronts per
  // SIMD); a pair: two k-groups, so two blocks share a CU and the twice larger grid runs
  // in one round
  if (b)
    hipLaunchKernelGGL(k_st_gemm<2>, dim3(gx, gy, 2), dim3(512), 0, st->stream, a, *b,
                       gconst(st));
  else
    hipLaunchKernelGGL(k_st_gemm<4>, dim3(gx, gy, 1), dim3(1024), 0, st->stream, a, a,
                       gconst(st));
}

// z = (c^2 - Delta_h)^-1 f for both velocity components at once: the u unknowns ([N][N-1]:
// rows DST-II, columns DST-I) and the v unknowns ([N-1][N]: rows DST-I, columns DST-II);
// forward transforms, division by the eigenvalues (with the second product), inverse.
// With grad, f is the pressure gradient of the cell array fu (fv unused).
void vel_solve(stokes_ctx* st, const double* fu, const double* fv, bool grad, double* zu,
               double* zv, double* t1u, double* t1v) {
  const int N = st->N, n = N - 1;
  const double* S1 = st->S1.as<double>();
  const double* S2 = st->S2.as<double>();
  const double* S2T = st->S2T.as<double>();
  GemmArgs u, v;
  u = ga(N, n, n, fu, n, S1, n, t1u, n, EP_NONE, grad ? AM_GRAD_U : AM_PLAIN);  // F S1^T
  v = ga(n, N, N, grad ? fu : fv, N, S2T, N, t1v, N, EP_NONE, grad ? AM_GRAD_V : AM_PLAIN);
  gemm(st, u, &v);
  u = ga(N, n, N, S2, N, t1u, n, zu, n, EP_VEL);  // S2 t1 / lambda
  v = ga(n, N, n, S1, n, t1v, N, zv, N, EP_VEL);  // S1 t1 / lambda
  gemm(st, u, &v);
  u = ga(N, n, N, S2T, N, zu, n, t1u, n);         // S2^T z
  v = ga(n, N, n, S1, n, zv, N, t1v, N);          // S1^T z (S1 symmetric)
  gemm(st, u, &v);
  u = ga(N, n, n, t1u, n, S1, n, zu, n);          // t1 S1
  v = ga(n, N, N, t1v, N, S2, N, zv, N);          // t1 S2
  gemm(st, u, &v);
}

// z = r + c^2 L^-1 r (cells; L the zero-flux cell Laplacian, mean-free part); c^2 > 0
void precond(stokes_ctx* st, const double* r, double* z, double* t1) {
  const int N = st->N;
  const double* C2 = st->C2.as<double>();
  const double* C2T = st->C2T.as<double>();
  gemm(st, ga(N, N, N, r, N, C2T, N, t1, N));                      // R C2^T
  gemm(st, ga(N, N, N, C2, N, t1, N, z, N, EP_CELL));              // c^2 C2 t1 / lambda
  gemm(st, ga(N, N, N, C2T, N, z, N, t1, N));                      // C2^T z
  gemm(st, ga(N, N, N, t1, N, C2, N, z, N, EP_NONE, AM_PLAIN, r)); // t1 C2 + r
}

int red_blocks(int n) { return std::min(kRedBlocks, nblk(n, 256)); }

// sc[slot] = scale * (a . b), or scale * sum(a) when b is null and sq is 0
void dot(stokes_ctx* st, int n, const double* a, const double* b, int slot, double scale = 1.0,
         int sq = 1) {
  const int nb = red_blocks(n);
  double* part = st->part.as<double>();
  hipLaunchKernelGGL(k_st_dot, dim3(nb), dim3(256), 0, st->stream, n, a, b, sq, part);
  hipLaunchKernelGGL(k_st_dot_fin, dim3(1), dim3(256), 0, st->stream, nb, part,
                     st->sc.as<double>() + slot, scale);
}

// The MAC system with right-hand sides ru, rv, rp (zero box data): CG on
// S p = (rp - mean rp) - G^T (c^2 - Delta)^-1 F, then u = -(c^2 - Delta)^-1 (F + G p).
// The host checks convergence one iteration behind the GPU: iteration it + 1 is queued
// before the record of iteration it is read, and runs without effect when it was the last.
int mac_solve(stokes_ctx* st) {
  const int N = st->N;
  const int NN = N * N, nu = N * (N - 1);
  hipStream_t s = st->stream;
  Work w = bind(st);
  const double ih = 1.0 / st->h;
  double* sc = st->sc.as<double>();
  double* part = st->part.as<double>();
  const double* ru = st->ru.as<double>();
  const double* rv = st->rv.as<double>();
  const double* rp = st->rp.as<double>();
  const bool pre = st->c2 > 0.0;  // with c^2 = 0 the preconditioner is the identity
  double* z = pre ? w.z : w.r;
  // b = (rp - mean) - G^T (c^2 - Delta)^-1 F
  vel_solve(st, ru, rv, false, w.zu, w.zv, w.t1, w.t1v);
  dot(st, NN, rp, nullptr, SC_MEAN, 1.0 / NN, 0);  // mean of the continuity right-hand side
  hipLaunchKernelGGL(k_st_sub_scalar, dim3(nblk(NN, 256)), dim3(256), 0, s, NN, sc, SC_MEAN, rp,
                     w.t1);
  hipLaunchKernelGGL(k_st_gradT, dim3(nblk(NN, 256)), dim3(256), 0, s, N, ih, w.zu, w.zv, -1.0,
                     w.t1, 1.0, w.b);
  // CG from p = 0: r = b, z = M^-1 r, d = z
  KFBI_HIP(hipMemsetAsync(w.pv, 0, sizeof(double) * NN, s));
  KFBI_HIP(hipMemcpyAsync(w.r, w.b, sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  dot(st, NN, w.b, nullptr, SC_BN);
  hipLaunchKernelGGL(k_st_cg_init, dim3(1), dim3(64), 0, s, sc);
  if (pre) precond(st, w.r, w.z, w.t1);
  KFBI_HIP(hipMemcpyAsync(w.d, z, sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  dot(st, NN, w.r, z, SC_RZ);
  const double tol2 = st->tol * st->tol;
  const int G = red_blocks(NN);  // blocks of the reduction launches, partials per sum
  int launched = 0, examined = 0, it = 0;
  bool done = false;
  double rel = 0.0;
  while (!done && examined < st->maxit) {
    if (launched < st->maxit) {
      const int k = launched;
      // q = S d = G^T (c^2 - Delta)^-1 G d, and d . q
      vel_solve(st, w.d, nullptr, true, w.zu, w.zv, w.t1, w.t1v);
      hipLaunchKernelGGL(k_st_gradT_dot, dim3(G), dim3(256), 0, s, N, ih, w.zu, w.zv, w.d, w.q,
                         part);
      hipLaunchKernelGGL(k_st_cg_step, dim3(G), dim3(256), 0, s, NN, k, G, sc, w.pv, w.r, w.d,
                         w.q, part);
      if (pre) precond(st, w.r, w.z, w.t1);
      hipLaunchKernelGGL(k_st_dot, dim3(G), dim3(256), 0, s, NN, w.r, z, 1, part + 2 * kRedBlocks);
      hipLaunchKernelGGL(k_st_cg_dir, dim3(G), dim3(256), 0, s, NN, k, G, tol2, sc, z, w.d, part,
                         st->dpost + (k % kPostRing));
      KFBI_HIP(hipGetLastError());
      KFBI_HIP(hipEventRecord(st->ev[k % kPostRing], s));
      ++launched;
    }
    // examine every launched iteration but the newest (all of them once no more launch)
    const int upto = (launched < st->maxit) ? launched - 1 : launched;
    while (!done && examined < upto) {
      KFBI_HIP(hipEventSynchronize(st->ev[examined % kPostRing]));
      const CgPost& rec = st->hpost[examined % kPostRing];
      ++examined;
      it = examined;
      rel = rec.bn2 > 0.0 ? sqrt(rec.rn2 / rec.bn2) : 0.0;
      if (rec.bn2 == 0.0) it = 0;
      if (!std::isfinite(rel)) {
        KFBI_HIP(hipStreamSynchronize(s));
        set_error("stokes: non-finite CG residual");
        return KFBI_E_NONFINITE;
      }
      done = rec.done != 0;
    }
  }
  st->cg_iters = it;
  st->cg_relres = rel;
  if (!done) {
    KFBI_HIP(hipStreamSynchronize(s));
    set_error("stokes: CG did not reach %.3e in %d iterations (relres %.3e)", st->tol, it, rel);
    return KFBI_E_NOCONV;
  }
  // velocities u = -(c^2 - Delta)^-1 (F + G p); pressure p
  hipLaunchKernelGGL(k_st_grad, dim3(nblk(2 * nu, 256)), dim3(256), 0, s, N, ih, w.pv, ru, rv,
                     w.gu, w.gv);
  vel_solve(st, w.gu, w.gv, false, w.zu, w.zv, w.t1, w.t1v);
  hipLaunchKernelGGL(k_st_fields, dim3(nblk(2 * N * (N + 1), 256)), dim3(256), 0, s, N, -1.0, w.zu,
                     w.zv, st->u.as<double>(), st->v.as<double>());
  KFBI_HIP(hipMemcpyAsync(st->p.as<double>(), w.pv, sizeof(double) * NN, hipMemcpyDeviceToDevice,
                          s));
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int apply_impl(stokes_ctx* st, const double* phi, double* plus, double* minus) {
  if (!st->have) {
    set_error("stokes: no interface installed");
    return KFBI_E_STATE;
  }
  if (!phi) {
    set_error("null density");
    return KFBI_E_INVALID;
  }
  kfbi_ctx* g = st->g2;
  const int M = st->M, N = st->N, nc = st->nc, npt = nc + M;
  hipStream_t s = st->stream;
  const double* d1 = g->dvec.as<double>();
  const double* d2 = d1 + M;
  hipLaunchKernelGGL(k_st_quant, dim3(nblk(M, kQuantOut), 2), dim3(256), sizeof(double) * 3 * M,
                     s, M, phi, d1, d2, st->Q.as<double>());
  hipLaunchKernelGGL(k_st_jumps, dim3(nblk(npt, 64)), dim3(64), 0, s, M, nc, g->cross.as<Crossing>(),
                     g->geo.as<double>(), st->Q.as<double>(), st->c2, st->J.as<double>());
  KFBI_HIP(hipMemsetAsync(st->flag.p, 0, sizeof(int), s));
  const int neq = 2 * N * (N - 1) + N * N;
  hipLaunchKernelGGL(k_st_rhs, dim3(nblk(neq, 256)), dim3(256), 0, s, N, st->h, st->x0, st->y0,
                     g->lab.as<int8_t>(), g->hid.as<int>(), g->vid.as<int>(),
                     g->cross.as<Crossing>(), st->J.as<double>(), npt, st->ru.as<double>(),
                     st->rv.as<double>(), st->rp.as<double>(), st->flag.as<int>());
  KFBI_HIP(hipGetLastError());
  KFBI_TRY(mac_solve(st));
  int flag = 0;
  KFBI_HIP(hipMemcpyAsync(&flag, st->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  hipLaunchKernelGGL(k_st_extract, dim3(nblk(2 * M, 64)), dim3(64), 0, s, M, N, st->h, st->x0,
                     st->y0, g->X.as<double>(), g->lab.as<int8_t>(), st->J.as<double>(), nc,
                     st->u.as<double>(), st->v.as<double>(), plus, minus);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(s));
  if (flag) {
    set_error("stokes: a MAC stencil pair and the interface crossings disagree");
    return KFBI_E_GEOMETRY;
  }
  return KFBI_OK;
}

}  // namespace

extern "C" {

int stokes_create(const stokes_params* p, stokes_ctx** out) {
  if (!p || !out) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *out = nullptr;
  const int N = p->N;
  if (N < 32 || N > 1024 || (N & (N - 1)) || !(p->side > 0.0) || !(p->c2 >= 0.0) ||
      p->max_markers < 16 || p->max_markers > 2048 || !(p->solve_tol > 0.0) ||
      p->solve_maxit < 1) {
    set_error("stokes: N a power of two in [32, 1024], side > 0, c2 >= 0, max_markers in "
              "[16, 2048], solve_tol > 0, solve_maxit >= 1");
    return KFBI_E_INVALID;
  }
  stokes_ctx* st = new stokes_ctx();
  st->x0 = p->x0;
  st->y0 = p->y0;
  st->side = p->side;
  st->N = N;
  st->h = p->side / N;
  st->c2 = p->c2;
  st->Mx = p->max_markers;
  st->stream = static_cast<hipStream_t>(p->stream);
  st->tol = p->solve_tol;
  st->maxit = p->solve_maxit;
  auto fail = [&](int code) {
    stokes_destroy(st);
    return code;
  };
  // the half-spacing grid (labels, crossings, marker geometry) and a GMRES workspace for
  // vectors of 2 max_markers
  kfbi_grid g{p->x0, p->y0, p->side, 2 * N, 0.0, KFBI_BOX_ZERO, 2 * p->max_markers, p->stream, 1};
  int rc = kfbi_create(&g, &st->g2);
  if (rc != KFBI_OK) return fail(rc);
  const size_t NN = static_cast<size_t>(N) * N;
  if ((rc = st->ru.ensure(sizeof(double) * NN)) || (rc = st->rv.ensure(sizeof(double) * NN)) ||
      (rc = st->rp.ensure(sizeof(double) * NN)) ||
      (rc = st->u.ensure(sizeof(double) * N * (N + 1))) ||
      (rc = st->v.ensure(sizeof(double) * N * (N + 1))) ||
      (rc = st->p.ensure(sizeof(double) * NN)) || (rc = st->S1.ensure(sizeof(double) * NN)) ||
      (rc = st->S2.ensure(sizeof(double) * NN)) || (rc = st->C2.ensure(sizeof(double) * NN)) ||
      (rc = st->S2T.ensure(sizeof(double) * NN)) || (rc = st->C2T.ensure(sizeof(double) * NN)) ||
      (rc = st->wk.ensure(sizeof(double) * NN * kWorkFields)) ||
      (rc = st->part.ensure(sizeof(double) * 3 * kRedBlocks)) ||
      (rc = st->sc.ensure(sizeof(double) * SC_COUNT)) ||
      (rc = st->flag.ensure(sizeof(int))) ||
      (rc = st->Q.ensure(sizeof(double) * 6 * p->max_markers)))
    return fail(rc);
  void* hp = nullptr;
  if (hipHostMalloc(&hp, sizeof(CgPost) * kPostRing, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    set_error("stokes: pinned host memory for the CG records");
    return fail(KFBI_E_HIP);
  }
  st->hpost = static_cast<CgPost*>(hp);
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) {
    set_error("stokes: device view of the CG records");
    return fail(KFBI_E_HIP);
  }
  st->dpost = static_cast<CgPost*>(dp);
  for (int q = 0; q < kPostRing; ++q)
    if (hipEventCreateWithFlags(&st->ev[q], hipEventDisableTiming) != hipSuccess) {
      set_error("stokes: CG events");
      return fail(KFBI_E_HIP);
    }
  hipLaunchKernelGGL(k_st_trmat, dim3(nblk(NN, 256)), dim3(256), 0, st->stream, N,
                     st->S1.as<double>(), st->S2.as<double>(), st->C2.as<double>(),
                     st->S2T.as<double>(), st->C2T.as<double>());
  if (hipStreamSynchronize(st->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
    set_error("stokes: set-up kernels failed");
    return fail(KFBI_E_HIP);
  }
  *out = st;
  return KFBI_OK;
}

int stokes_destroy(stokes_ctx* st) {
  if (!st) return KFBI_OK;
  if (st->g2) (void)hipStreamSynchronize(st->stream);
  for (DBuf* b : {&st->Q, &st->J, &st->ru, &st->rv, &st->rp, &st->u, &st->v, &st->p, &st->S1,
                  &st->S2, &st->C2, &st->S2T, &st->C2T, &st->wk, &st->part, &st->sc, &st->flag})
    b->release();
  for (hipEvent_t& e : st->ev)
    if (e) (void)hipEventDestroy(e);
  if (st->hpost) (void)hipHostFree(st->hpost);
  if (st->g2) kfbi_destroy(st->g2);
  delete st;
  return KFBI_OK;
}

int stokes_set_interface(stokes_ctx* st, int M, const double* xy) {
  if (!st || !xy || M < 16 || M > st->Mx || (M & 1)) {
    set_error("stokes: M must be even and in [16, max_markers] with a non-null xy (M=%d)", M);
    return KFBI_E_INVALID;
  }
  st->have = 0;
  KFBI_TRY(kfbi_set_interface(st->g2, M, xy));
  kfbi_ctx* g = st->g2;
  const double m = 3.0 * st->h;
  KFBI_HIP(hipMemsetAsync(st->flag.p, 0, sizeof(int), st->stream));
  hipLaunchKernelGGL(k_st_margin, dim3(nblk(M, 256)), dim3(256), 0, st->stream, M,
                     g->X.as<double>(), st->x0 + m, st->x0 + st->side - m, st->y0 + m,
                     st->y0 + st->side - m, st->flag.as<int>());
  int flag = 0;
  KFBI_HIP(hipMemcpyAsync(&flag, st->flag.p, sizeof(int), hipMemcpyDeviceToHost, st->stream));
  KFBI_HIP(hipStreamSynchronize(st->stream));
  if (flag) {
    set_error("stokes: interface marker closer than 3h to the box boundary");
    return KFBI_E_GEOMETRY;
  }
  st->M = M;
  st->nc = g->st.n_cross_h + g->st.n_cross_v;
  KFBI_TRY(st->J.ensure(sizeof(double) * kNJ * static_cast<size_t>(st->nc + M)));
  st->have = 1;
  return KFBI_OK;
}

int stokes_apply(stokes_ctx* st, const double* phi, double* plus, double* minus) {
  if (!st) {
    set_error("null context");
    return KFBI_E_INVALID;
  }
  return apply_impl(st, phi, plus, minus);
}

int stokes_fields(stokes_ctx* st, double* u, double* v, double* p) {
  if (!st) {
    set_error("null context");
    return KFBI_E_INVALID;
  }
  const size_t N = st->N;
  if (u) KFBI_HIP(hipMemcpyAsync(u, st->u.p, sizeof(double) * N * (N + 1), hipMemcpyDeviceToDevice, st->stream));
  if (v) KFBI_HIP(hipMemcpyAsync(v, st->v.p, sizeof(double) * N * (N + 1), hipMemcpyDeviceToDevice, st->stream));
  if (p) KFBI_HIP(hipMemcpyAsync(p, st->p.p, sizeof(double) * N * N, hipMemcpyDeviceToDevice, st->stream));
  KFBI_HIP(hipStreamSynchronize(st->stream));
  return KFBI_OK;
}

int stokes_operator(stokes_ctx* st, const double* x, double* y) {
  if (!st || !y) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  return apply_impl(st, x, nullptr, y);
}

int stokes_gmres_solve(stokes_ctx* st, const double* rhs, double* x, const kfbi_gmres_opts* o,
                       kfbi_gmres_stats* stats) {
  if (!st) {
    set_error("null context");
    return KFBI_E_INVALID;
  }
  if (!st->have) {
    set_error("stokes: no interface installed");
    return KFBI_E_STATE;
  }
  const GmresOp op = [st](const double* xin, double* yout, bool) {
    return apply_impl(st, xin, nullptr, yout);
  };
  return gmres_solve_op(st->g2, 2 * st->M, op, rhs, x, o, stats);
}

int stokes_get_info(const stokes_ctx* st, stokes_info* info) {
  if (!st || !info) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  info->M = st->M;
  info->n_crossings = st->nc;
  info->cg_iters = st->cg_iters;
  info->cg_relres = st->cg_relres;
  return KFBI_OK;
}

}  // extern "C"
