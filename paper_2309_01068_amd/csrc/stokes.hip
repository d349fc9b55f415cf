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

#include <cmath>
#include <cstring>

#include "../../include/stokes.h"
#include "common.h"
#include "device_util.h"

using namespace kfbi;

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
};

namespace {

constexpr int kNJ = 15;  // jump values per point: u, ux, uy, uxx, uyy, uxy, v.., p, px, py
enum { JU = 0, JUX, JUY, JUXX, JUYY, JUXY, JV, JVX, JVY, JVXX, JVYY, JVXY, JP, JPX, JPY };
// device scalars of the CG recurrences
enum { SC_RZ = 0, SC_RZN, SC_DQ, SC_RN, SC_BN, SC_MEAN, SC_COUNT = 8 };
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
// are issued before the products of the current one (every k-chunk would otherwise wait
// for its own loads: the grids of these transforms are small).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kGT = 32;  // output tile and k-chunk
__global__ void __launch_bounds__(256)
    k_st_gemm(int m, int n, int k, const double* __restrict__ A, int lda,
              const double* __restrict__ B, int ldb, double* __restrict__ C, int ldc) {
  __shared__ double As[kGT][kGT + 1];  // [row][k]
  __shared__ double Bs[kGT][kGT + 1];  // [k][col]
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r0 = blockIdx.y * kGT, c0 = blockIdx.x * kGT;
  const int wr = 16 * (w >> 1), wc = 16 * (w & 1);
  const int lr = lane & 15, lk = lane >> 4;
  // this thread's four elements of each tile: row tid / 8 + 0..3 * 8 ... (e = tid + 256 q)
  double pa[4], pb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 5, cc = e & 31;
      const int gr = r0 + rr, gk = k0 + cc;
      pa[q] = (gr < m && gk < k) ? A[static_cast<size_t>(gr) * lda + gk] : 0.0;
      const int gkb = k0 + rr, gc = c0 + cc;
      pb[q] = (gkb < k && gc < n) ? B[static_cast<size_t>(gkb) * ldb + gc] : 0.0;
    }
  };
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int k0 = 0; k0 < k; k0 += kGT) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      As[e >> 5][e & 31] = pa[q];
      Bs[e >> 5][e & 31] = pb[q];
    }
    __syncthreads();
    if (k0 + kGT < k) load(k0 + kGT);  // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < kGT; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[wr + lr][kk + lk], Bs[kk + lk][wc + lr], acc,
                                                 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gr = r0 + wr + 4 * i + lk, gc = c0 + wc + lr;
    if (gr < m && gc < n) C[static_cast<size_t>(gr) * ldc + gc] = acc[i];
  }
}

// X[r][c] /= lambda: mode 0 (u: rows DST-II l = r + 1, columns DST-I k = c + 1), mode 1
// (v: rows DST-I, columns DST-II), both with lambda = (4/h^2)(sin^2(k pi/2N) +
// sin^2(l pi/2N)) + c^2; mode 2 (cells, DCT-II k = c, l = r): X *= c^2 / ((4/h^2)(...)),
// the (0, 0) mode set to zero.
__global__ void k_st_scale(int rows, int cols, int N, double ih2, double c2, int mode,
                           double* __restrict__ X) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int r = e / cols, c = e % cols;
  const int l = (mode == 2) ? r : r + 1, k = (mode == 2) ? c : c + 1;
  const double sl = sinpi(static_cast<double>(l) / (2 * N));
  const double sk = sinpi(static_cast<double>(k) / (2 * N));
  const double lam = 4.0 * ih2 * (sl * sl + sk * sk);
  if (mode == 2)
    X[e] = (l == 0 && k == 0) ? 0.0 : X[e] * (c2 / lam);
  else
    X[e] = X[e] / (lam + c2);
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

// Block partial sums of a . b (a . a when b is null and sq, the sum of a when b is null and
// not sq), then the ordered total.
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

__global__ void __launch_bounds__(256)
    k_st_dot_fin(int nb, const double* __restrict__ part, double* __restrict__ out, double scale) {
  __shared__ double scratch[16];
  double s = 0.0;
  for (int e = threadIdx.x; e < nb; e += 256) s += part[e];
  s = block_sum<double>(s, scratch);
  if (threadIdx.x == 0) *out = s * scale;
}

// x -= sc[slot] (mean removal); y = x otherwise
__global__ void k_st_sub_scalar(int n, const double* __restrict__ sc, int slot,
                                const double* __restrict__ x, double* __restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = x[e] - sc[slot];
}

// p += alpha d, r -= alpha q with alpha = sc[RZ] / sc[DQ]
__global__ void k_st_cg_step(int n, const double* __restrict__ sc, double* __restrict__ p,
                             double* __restrict__ r, const double* __restrict__ d,
                             const double* __restrict__ q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double alpha = sc[SC_RZ] / sc[SC_DQ];
  p[e] += alpha * d[e];
  r[e] -= alpha * q[e];
}

// d = z + beta d with beta = sc[RZN] / sc[RZ]
__global__ void k_st_cg_dir(int n, const double* __restrict__ sc, const double* __restrict__ z,
                            double* __restrict__ d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  d[e] = z[e] + (sc[SC_RZN] / sc[SC_RZ]) * d[e];
}

__global__ void k_st_shift(double* __restrict__ sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[SC_RZ] = sc[SC_RZN];
}

// y = a x + b y (y is not read when b = 0)
__global__ void k_st_axpby(int n, double a, const double* __restrict__ x, double b,
                           double* __restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = a * x[e] + (b != 0.0 ? b * y[e] : 0.0);
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
__global__ void k_st_quant(int M, const double* __restrict__ phi, const double* __restrict__ d1,
                           const double* __restrict__ d2, double* __restrict__ Q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * M) return;
  const int comp = e / M, k = e % M;
  const double* f = phi + comp * M;
  double s1 = 0.0, s2 = 0.0;
  for (int m = 0; m < M; ++m) {
    int q = k - m;
    q += (q < 0) ? M : 0;
    s1 += d1[q] * f[m];
    s2 += d2[q] * f[m];
  }
  Q[(3 * comp) * M + k] = f[k];
  Q[(3 * comp + 1) * M + k] = s1;
  Q[(3 * comp + 2) * M + k] = s2;
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
  double *zu, *zv, *gu, *gv, *t1, *pv, *r, *z, *d, *q, *b;
};

Work bind(stokes_ctx* st) {
  const size_t NN = static_cast<size_t>(st->N) * st->N;
  double* w = st->wk.as<double>();
  Work k;
  k.zu = w;
  k.zv = w + NN;
  k.gu = w + 2 * NN;
  k.gv = w + 3 * NN;
  k.t1 = w + 4 * NN;
  k.pv = w + 5 * NN;
  k.r = w + 6 * NN;
  k.z = w + 7 * NN;
  k.d = w + 8 * NN;
  k.q = w + 9 * NN;
  k.b = w + 10 * NN;
  return k;
}
constexpr int kWorkFields = 11;

// C = A B, row-major operands: A (m x k, row stride lda), B (k x n, row stride ldb)
void gemm(hipStream_t s, int m, int n, int k, const double* A, int lda, const double* B, int ldb,
          double* C, int ldc) {
  hipLaunchKernelGGL(k_st_gemm, dim3(nblk(n, kGT), nblk(m, kGT)), dim3(256), 0, s, m, n, k, A, lda,
                     B, ldb, C, ldc);
}

// z = (c^2 - Delta_h)^-1 f for the u unknowns ([N][N-1]; comp 0) or the v unknowns
// ([N-1][N]; comp 1): forward transforms, division by the eigenvalues, inverse.
void vel_solve(stokes_ctx* st, int comp, const double* f, double* z, double* t1) {
  const int N = st->N, n = N - 1;
  hipStream_t s = st->stream;
  const double* S1 = st->S1.as<double>();
  const double* S2 = st->S2.as<double>();
  const double* S2T = st->S2T.as<double>();
  const double ih2 = 1.0 / (st->h * st->h);
  if (comp == 0) {  // rows: DST-II (N), columns: DST-I (N-1)
    gemm(s, N, n, n, f, n, S1, n, t1, n);        // t1 = F S1^T (S1 symmetric)
    gemm(s, N, n, N, S2, N, t1, n, z, n);        // z = S2 t1
    hipLaunchKernelGGL(k_st_scale, dim3(nblk(N * n, 256)), dim3(256), 0, s, N, n, N, ih2, st->c2,
                       0, z);
    gemm(s, N, n, N, S2T, N, z, n, t1, n);       // t1 = S2^T z
    gemm(s, N, n, n, t1, n, S1, n, z, n);        // z = t1 S1
  } else {  // rows: DST-I (N-1), columns: DST-II (N)
    gemm(s, n, N, N, f, N, S2T, N, t1, N);       // t1 = F S2^T
    gemm(s, n, N, n, S1, n, t1, N, z, N);        // z = S1 t1
    hipLaunchKernelGGL(k_st_scale, dim3(nblk(N * n, 256)), dim3(256), 0, s, n, N, N, ih2, st->c2,
                       1, z);
    gemm(s, n, N, n, S1, n, z, N, t1, N);        // t1 = S1^T z (S1 symmetric)
    gemm(s, n, N, N, t1, N, S2, N, z, N);        // z = t1 S2
  }
}

// z = r + c^2 L^-1 r (cells; L the zero-flux cell Laplacian, mean-free part)
void precond(stokes_ctx* st, const double* r, double* z, double* t1) {
  const int N = st->N;
  const size_t NN = static_cast<size_t>(N) * N;
  hipStream_t s = st->stream;
  if (st->c2 == 0.0) {
    hipLaunchKernelGGL(k_st_axpby, dim3(nblk(NN, 256)), dim3(256), 0, s, static_cast<int>(NN),
                       1.0, r, 0.0, z);
    return;
  }
  const double* C2 = st->C2.as<double>();
  const double* C2T = st->C2T.as<double>();
  gemm(s, N, N, N, r, N, C2T, N, t1, N);         // t1 = R C2^T
  gemm(s, N, N, N, C2, N, t1, N, z, N);          // z = C2 t1
  hipLaunchKernelGGL(k_st_scale, dim3(nblk(NN, 256)), dim3(256), 0, s, N, N, N,
                     1.0 / (st->h * st->h), st->c2, 2, z);
  gemm(s, N, N, N, C2T, N, z, N, t1, N);         // t1 = C2^T z
  gemm(s, N, N, N, t1, N, C2, N, z, N);          // z = t1 C2
  hipLaunchKernelGGL(k_st_axpby, dim3(nblk(NN, 256)), dim3(256), 0, s, static_cast<int>(NN), 1.0,
                     r, 1.0, z);
}

// sc[slot] = scale * (a . b), or scale * sum(a) when b is null and sq is 0
void dot(stokes_ctx* st, int n, const double* a, const double* b, int slot, double scale = 1.0,
         int sq = 1) {
  hipStream_t s = st->stream;
  const int nb = std::min(kRedBlocks, nblk(n, 256));
  hipLaunchKernelGGL(k_st_dot, dim3(nb), dim3(256), 0, s, n, a, b, sq, st->part.as<double>());
  hipLaunchKernelGGL(k_st_dot_fin, dim3(1), dim3(256), 0, s, nb, st->part.as<double>(),
                     st->sc.as<double>() + slot, scale);
}

int read_scalar(stokes_ctx* st, int slot, double* out) {
  KFBI_HIP(hipMemcpyAsync(out, st->sc.as<double>() + slot, sizeof(double), hipMemcpyDeviceToHost,
                          st->stream));
  KFBI_HIP(hipStreamSynchronize(st->stream));
  return KFBI_OK;
}

// The MAC system with right-hand sides ru, rv, rp (zero box data): CG on
// S p = (rp - mean rp) - G^T (c^2 - Delta)^-1 F, then u = -(c^2 - Delta)^-1 (F + G p).
int mac_solve(stokes_ctx* st) {
  const int N = st->N;
  const int NN = N * N, nu = N * (N - 1);
  hipStream_t s = st->stream;
  Work w = bind(st);
  const double ih = 1.0 / st->h;
  double* sc = st->sc.as<double>();
  const double* ru = st->ru.as<double>();
  const double* rv = st->rv.as<double>();
  const double* rp = st->rp.as<double>();
  // b = (rp - mean) - G^T (c^2 - Delta)^-1 F
  vel_solve(st, 0, ru, w.zu, w.t1);
  vel_solve(st, 1, rv, w.zv, w.t1);
  dot(st, NN, rp, nullptr, SC_MEAN, 1.0 / NN, 0);  // mean of the continuity right-hand side
  hipLaunchKernelGGL(k_st_sub_scalar, dim3(nblk(NN, 256)), dim3(256), 0, s, NN, sc, SC_MEAN, rp,
                     w.t1);
  hipLaunchKernelGGL(k_st_gradT, dim3(nblk(NN, 256)), dim3(256), 0, s, N, ih, w.zu, w.zv, -1.0,
                     w.t1, 1.0, w.b);
  // CG from p = 0
  KFBI_HIP(hipMemsetAsync(w.pv, 0, sizeof(double) * NN, s));
  KFBI_HIP(hipMemcpyAsync(w.r, w.b, sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  dot(st, NN, w.b, nullptr, SC_BN);
  precond(st, w.r, w.z, w.t1);
  KFBI_HIP(hipMemcpyAsync(w.d, w.z, sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  dot(st, NN, w.r, w.z, SC_RZ);
  double bn2 = 0.0;
  KFBI_TRY(read_scalar(st, SC_BN, &bn2));
  const double bn = sqrt(bn2);
  int it = 0;
  double rel = 0.0;
  if (bn > 0.0) {
    for (; it < st->maxit;) {
      // q = S d = G^T (c^2 - Delta)^-1 G d
      hipLaunchKernelGGL(k_st_grad, dim3(nblk(2 * nu, 256)), dim3(256), 0, s, N, ih, w.d, nullptr,
                         nullptr, w.gu, w.gv);
      vel_solve(st, 0, w.gu, w.zu, w.t1);
      vel_solve(st, 1, w.gv, w.zv, w.t1);
      hipLaunchKernelGGL(k_st_gradT, dim3(nblk(NN, 256)), dim3(256), 0, s, N, ih, w.zu, w.zv, 1.0,
                         nullptr, 0.0, w.q);
      dot(st, NN, w.d, w.q, SC_DQ);
      hipLaunchKernelGGL(k_st_cg_step, dim3(nblk(NN, 256)), dim3(256), 0, s, NN, sc, w.pv, w.r,
                         w.d, w.q);
      ++it;
      dot(st, NN, w.r, nullptr, SC_RN);
      double rn2 = 0.0;
      KFBI_TRY(read_scalar(st, SC_RN, &rn2));
      rel = sqrt(rn2) / bn;
      if (!std::isfinite(rel)) {
        set_error("stokes: non-finite CG residual");
        return KFBI_E_NONFINITE;
      }
      if (rel <= st->tol) break;
      precond(st, w.r, w.z, w.t1);
      dot(st, NN, w.r, w.z, SC_RZN);
      hipLaunchKernelGGL(k_st_cg_dir, dim3(nblk(NN, 256)), dim3(256), 0, s, NN, sc, w.z, w.d);
      hipLaunchKernelGGL(k_st_shift, dim3(1), dim3(1), 0, s, sc);
    }
  }
  st->cg_iters = it;
  st->cg_relres = rel;
  if (bn > 0.0 && rel > st->tol) {
    set_error("stokes: CG did not reach %.3e in %d iterations (relres %.3e)", st->tol, it, rel);
    return KFBI_E_NOCONV;
  }
  // velocities u = -(c^2 - Delta)^-1 (F + G p); pressure p
  hipLaunchKernelGGL(k_st_grad, dim3(nblk(2 * nu, 256)), dim3(256), 0, s, N, ih, w.pv, ru, rv,
                     w.gu, w.gv);
  vel_solve(st, 0, w.gu, w.zu, w.t1);
  vel_solve(st, 1, w.gv, w.zv, w.t1);
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
  hipLaunchKernelGGL(k_st_quant, dim3(nblk(2 * M, 128)), dim3(128), 0, s, M, phi, d1, d2,
                     st->Q.as<double>());
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
      (rc = st->part.ensure(sizeof(double) * kRedBlocks)) ||
      (rc = st->sc.ensure(sizeof(double) * SC_COUNT)) ||
      (rc = st->flag.ensure(sizeof(int))) ||
      (rc = st->Q.ensure(sizeof(double) * 6 * p->max_markers)))
    return fail(rc);
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
