// One KFBI operator apply on gfx950 (Sec. 4): four kernels per apply.
//
//  K1 k_prep     density -> Fourier derivatives at markers (circulant form, FP64), jump
//                corrections of every irregular arm (Sec. 4.2.1 eq. modified-fdm with the
//                App. A.1 jumps, coefficients precomputed per interface), trapezoid weight
//                partial sums, and free-space box data (Sec. 4.1) when requested.
//  K2 k_colsolve fast solve of (Delta_h - c^2) v = RHS.  The RHS is non-zero only at
//                irregular nodes and next to the box, so the sine transform along x is
//                formed directly from the arm list; along y each sine mode p leaves the
//                constant tridiagonal system
//                    G_{j+1} - (2 + delta_p) G_j + G_{j-1} = h^2 Rhat_{p,j},  G_0 = G_N = 0,
//                    delta_p = 4 sin^2(p pi / 2N) + h^2 c^2,
//                solved per wavefront by two first-order recurrences with root
//                rho_p (rho + 1/rho = 2 + delta_p) and a rank-one boundary correction.
//                One wavefront per mode, four modes per block; output rows of G.
//  K3 k_nodes    inverse sine transform along x evaluated only at the interpolation
//                nodes: v_ij = (2/N) sum_p G_{j,p} sin(p i pi / N).
//  K4 k_extract  Sec. 4.3 corrected interpolation with precomputed weights -> v+-,
//                n.grad v+-, and the boundary operator a x + b trace + q int x ds.
// The full-grid variant writes every row in K2 and evaluates the whole grid with a
// tiled product against the sine matrix.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "device_util.h"

namespace kfbi {

constexpr int kColsPerBlock = 4;

// ---------------------------------------------------------------------------------- K1
// Marker-chunk blocks: blocks [0, nmk).  Ring blocks (free-space box): [nmk, nmk+nring).
template <class T>
__global__ void __launch_bounds__(256)
    k_prep(int M, int C, int nmk, int layer, const double* __restrict__ dens,
           const double* __restrict__ d1, const double* __restrict__ d2,
           const ArmCoef* __restrict__ armc, const int* __restrict__ armint,
           const int* __restrict__ intoff, T* __restrict__ armr, double* __restrict__ mq,
           double* __restrict__ qpart, const MarkerExt* __restrict__ ext,
           // free-space box data
           int nring, int N, double x0, double y0, double h, const double* __restrict__ X,
           const double* __restrict__ geo, T* __restrict__ ring) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  if (static_cast<int>(blockIdx.x) >= nmk) {
    // ----- box data: one wavefront per box node, lanes split the markers
    const int rb = blockIdx.x - nmk;
    const int lane = tid & 63, w = tid >> 6;
    const int n1 = N + 1;
    const int total = 4 * n1;
    const double* xs = X;
    const double* ys = X + M;
    const double* xa = geo;
    const double* ya = geo + M;
    const double* sa = geo + 4 * M;
    for (int q = 0; q < 4; ++q) {
      const int node = rb * 16 + w * 4 + q;
      if (node >= total) break;
      const int side = node / n1, r = node % n1;
      double zx, zy;
      if (side == 0) {
        zx = x0 + r * h;
        zy = y0;
      } else if (side == 1) {
        zx = x0 + r * h;
        zy = y0 + N * h;
      } else if (side == 2) {
        zx = x0;
        zy = y0 + r * h;
      } else {
        zx = x0 + N * h;
        zy = y0 + r * h;
      }
      double acc = 0.0;
      for (int k = lane; k < M; k += 64) {
        const double dx = xs[k] - zx, dy = ys[k] - zy;
        const double r2 = dx * dx + dy * dy;
        if (layer == KFBI_DOUBLE)
          acc += dens[k] * (dx * ya[k] - dy * xa[k]) / r2;
        else
          acc += dens[k] * sa[k] * 0.5 * log(r2);
      }
      acc = wave_sum(acc);
      if (lane == 0) ring[node] = static_cast<T>(acc / M);
    }
    return;
  }
  // ----- marker chunk
  const int b = blockIdx.x;
  const int k0 = b * C;
  const int k1 = min(M, k0 + C);
  const int H = k1 - k0 + 5;  // markers k0-2 .. k1+2
  const int nd = (layer == KFBI_DOUBLE) ? 2 : 1;
  const int nout = H * nd;
  double* ph = lds;             // M
  double* part = lds + M;       // 8 * nout
  double* Qh = part + 8 * nout; // 5 * H
  for (int m = tid; m < M; m += 256) ph[m] = dens[m];
  __syncthreads();
  // circulant dot products: output o = (hm, deriv), 8 slices of m
  {
    const int slices = 8;
    const int per = (M + slices - 1) / slices;
    for (int task = tid; task < nout * slices; task += 256) {
      const int o = task % nout, sl = task / nout;
      const int hm = o % H, dv = o / H;
      int k = k0 - 2 + hm;
      k = (k < 0) ? k + M : (k >= M ? k - M : k);
      const double* dd = (dv == 0) ? d1 : d2;
      const int mb = sl * per, me = min(M, mb + per);
      double acc = 0.0;
      for (int m = mb; m < me; ++m) {
        int q = k - m;
        q += (q < 0) ? M : 0;
        acc += dd[q] * ph[m];
      }
      part[sl * nout + o] = acc;
    }
  }
  __syncthreads();
  for (int hm = tid; hm < H; hm += 256) {
    int k = k0 - 2 + hm;
    k = (k < 0) ? k + M : (k >= M ? k - M : k);
    double v1 = 0.0, v2 = 0.0;
    for (int sl = 0; sl < 8; ++sl) {
      v1 += part[sl * nout + hm];
      if (nd == 2) v2 += part[sl * nout + H + hm];
    }
    double Q[5];
    if (layer == KFBI_DOUBLE) {
      Q[0] = ph[k];
      Q[1] = v1;
      Q[2] = v2;
      Q[3] = 0.0;
      Q[4] = 0.0;
    } else {  // Psi = -psi
      Q[0] = 0.0;
      Q[1] = 0.0;
      Q[2] = 0.0;
      Q[3] = -ph[k];
      Q[4] = -v1;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) Qh[q * H + hm] = Q[q];
    if (hm >= 2 && hm < H - 3) {
#pragma unroll
      for (int q = 0; q < 5; ++q) mq[q * M + k] = Q[q];
    }
  }
  __syncthreads();
  // arm corrections for crossings in intervals k0 .. k1-1
  const int a0 = intoff[k0], a1 = intoff[k1];
  for (int t = a0 + tid; t < a1; t += 256) {
    const int a = armint[t];
    const ArmCoef ac = armc[a];
    const int base = ac.k - k0;  // Lagrange node m -> halo index base + m
    double r = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 5; ++q) s += ac.coef[q] * Qh[q * H + base + m];
      r += ac.l[m] * s;
    }
    armr[a] = static_cast<T>(r);
  }
  // trapezoid partial sum of the density
  double qs = 0.0;
  for (int k = k0 + tid; k < k1; k += 256) qs += ph[k] * ext[k].wq;
  qs = block_sum<double>(qs, part);
  if (tid == 0) qpart[b] = qs;
}

// ---------------------------------------------------------------------------------- K2
template <int E>
__device__ __forceinline__ int slot(int j) {  // row j (1-based) -> LDS slot, padded
  const int e = j - 1;
  return (e / E) * (E + 1) + (e % E);
}

template <class T, int E>
__global__ void __launch_bounds__(256)
    k_colsolve(int N, double h, double c2, const int* __restrict__ rowoff,
               const int* __restrict__ armi, const T* __restrict__ armr,
               const T* __restrict__ sinT, const T* __restrict__ ring, int jlo, int jhi,
               int ldG, T* __restrict__ G, int nblk_x) {
  __shared__ T col[kColsPerBlock][64 * (E + 1)];
  const int n = N - 1;
  const int mask = 2 * N - 1;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // XCD-aware order: blocks resident on one XCD (ids congruent mod 8) take adjacent
  // column groups, so partial cache lines of the row-major output meet in one L2.
  const int bid = blockIdx.x;
  const int per_xcd = (nblk_x + 7) / 8;
  const int grp = (bid % 8) * per_xcd + bid / 8;
  if (grp * kColsPerBlock + 1 > n) return;  // whole block beyond the last mode
  const int p0 = 1 + grp * kColsPerBlock;
  int pc[kColsPerBlock];
#pragma unroll
  for (int c = 0; c < kColsPerBlock; ++c) pc[c] = p0 + c;
  const T ih2 = static_cast<T>(1.0 / (h * h));
  // phase 1: sine transform along x of the sparse right-hand side, row by row
  for (int idx = tid; idx < kColsPerBlock * 64 * (E + 1); idx += 256) (&col[0][0])[idx] = T(0);
  __syncthreads();
  for (int j = 1 + tid; j <= n; j += 256) {
    T acc[kColsPerBlock];
#pragma unroll
    for (int c = 0; c < kColsPerBlock; ++c) acc[c] = T(0);
    const int ae = rowoff[j + 1];
    for (int a = rowoff[j]; a < ae; ++a) {
      const int i = armi[a];
      const T r = armr[a];
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) acc[c] += r * sinT[(pc[c] * i) & mask];
    }
    if (ring) {  // left (i=0) and right (i=N) box nodes next to (1, j) and (N-1, j)
      const int n1 = N + 1;
      const T gl = ring[2 * n1 + j], gr = ring[3 * n1 + j];
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c)
        acc[c] -= ih2 * (gl * sinT[pc[c] & mask] + gr * sinT[(pc[c] * n) & mask]);
    }
#pragma unroll
    for (int c = 0; c < kColsPerBlock; ++c) col[c][slot<E>(j)] = acc[c];
  }
  __syncthreads();
  if (ring) {  // bottom (j=0) and top (j=N) box rows: a full sine sum each
    const int p = pc[w];
    T sb = T(0), st = T(0);
    for (int i = 1 + lane; i <= n; i += 64) {
      const T s = sinT[(p * i) & mask];
      sb += ring[i] * s;
      st += ring[(N + 1) + i] * s;
    }
    sb = wave_sum(sb);
    st = wave_sum(st);
    if (lane == 0) {
      col[w][slot<E>(1)] -= ih2 * sb;
      col[w][slot<E>(n)] -= ih2 * st;
    }
  }
  __syncthreads();
  // phase 2: tridiagonal solve along y for mode p = pc[w], one wavefront
  const int p = pc[w];
  if (p <= n) {
    const double sp = sinpi(0.5 * p / N);
    const double delta = 4.0 * sp * sp + h * h * c2;
    const double sq = sqrt(delta * (4.0 + delta));
    const double rho = 2.0 / (2.0 + delta + sq);
    const double eps = (delta + sq) / (2.0 + delta + sq);  // 1 - rho without cancellation
    const T rhoT = static_cast<T>(rho), epsT = static_cast<T>(eps);
    const T h2 = static_cast<T>(h * h);
    // powers rho^e, e = 0..E
    double pw[E + 1];
    pw[0] = 1.0;
#pragma unroll
    for (int e = 1; e <= E; ++e) pw[e] = pw[e - 1] * rho;
    T y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = h2 * col[w][lane * (E + 1) + e];
    // backward recurrence y_j = b_j + rho y_{j+1}
#pragma unroll
    for (int e = E - 2; e >= 0; --e) y[e] = (y[e] - epsT * y[e + 1]) + y[e + 1];
    {
      T v = y[0];
      double fe = pw[E];
#pragma unroll
      for (int s = 1; s < 64; s <<= 1) {
        const T o = __shfl_down(v, s, 64);
        if (lane + s < 64) v += static_cast<T>(fe) * o;
        fe *= fe;
      }
      T carry = __shfl_down(v, 1, 64);
      if (lane == 63) carry = T(0);
#pragma unroll
      for (int e = 0; e < E; ++e) y[e] += static_cast<T>(pw[E - e]) * carry;
    }
    // forward recurrence z_j = y_j + rho z_{j-1}
#pragma unroll
    for (int e = 1; e < E; ++e) y[e] = (y[e] - epsT * y[e - 1]) + y[e - 1];
    {
      T v = y[E - 1];
      double fe = pw[E];
#pragma unroll
      for (int s = 1; s < 64; s <<= 1) {
        const T o = __shfl_up(v, s, 64);
        if (lane >= s) v += static_cast<T>(fe) * o;
        fe *= fe;
      }
      T carry = __shfl_up(v, 1, 64);
      if (lane == 0) carry = T(0);
#pragma unroll
      for (int e = 0; e < E; ++e) y[e] += static_cast<T>(pw[e + 1]) * carry;
    }
    // z_n and the rank-one boundary correction
    const int ln = (n - 1) / E, en = (n - 1) % E;
    T sel = T(0);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e == en) sel = y[e];
    const T zn = __shfl(sel, ln, 64);
    const double lr = log1p(-eps);
    const double den = -expm1((2.0 * n + 2.0) * lr);
    const int j0 = lane * E + 1;
    // rho^{n - j + 3} for j = j0 + E - 1, then multiply up
    const double abase = exp(static_cast<double>(n - (j0 + E - 1) + 3) * lr);
    const double r2j0 = exp(2.0 * j0 * lr);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double a = abase * pw[E - 1 - e];
      const double om = 1.0 - r2j0 * pw[e] * pw[e];
      const double f = a * om / den;
      y[e] = -rhoT * y[e] + static_cast<T>(f) * zn;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) col[w][lane * (E + 1) + e] = y[e];
  }
  __syncthreads();
  // phase 3: rows jlo..jhi of G (row-major, ldG; column p stored at p - 1)
  const int nb = jhi - jlo + 1;
  for (int r = tid; r < nb; r += 256) {
    const int j = jlo + r;
    const int sj = slot<E>(j);
    T* dst = G + static_cast<size_t>(r) * ldG + (p0 - 1);
#pragma unroll
    for (int c = 0; c < kColsPerBlock; ++c)
      if (p0 + c <= n) dst[c] = col[c][sj];
  }
}

// ---------------------------------------------------------------------------------- K3
template <class T, int E>
__global__ void __launch_bounds__(256)
    k_nodes(int N, const int* __restrict__ rows, const int* __restrict__ rowptr,
            const int* __restrict__ nodei, const T* __restrict__ sinT, int jlo, int ldG,
            const T* __restrict__ G, T* __restrict__ nodeval) {
  const int n = N - 1;
  const int mask = 2 * N - 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = blockIdx.x;
  const int j = rows[r];
  const int nb = rowptr[r], ne = rowptr[r + 1];
  const T* g = G + static_cast<size_t>(j - jlo) * ldG;
  T gv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = 1 + lane + 64 * e;
    gv[e] = (p <= n) ? g[p - 1] : T(0);
  }
  const T scale = static_cast<T>(2.0 / N);
  for (int idx = nb + w; idx < ne; idx += 4) {
    const int i = nodei[idx];
    T s = T(0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = 1 + lane + 64 * e;
      s += gv[e] * sinT[(p * i) & mask];
    }
    s = wave_sum(s);
    if (lane == 0) nodeval[idx] = scale * s;
  }
}

// ---------------------------------------------------------------------------------- K4
template <class T>
__global__ void __launch_bounds__(256)
    k_extract(int M, const int* __restrict__ stn, const T* __restrict__ nodeval,
              const double* __restrict__ mq, const MarkerExt* __restrict__ ext,
              const double* __restrict__ qpart, int nq, double* __restrict__ vp_out,
              double* __restrict__ vm_out, double* __restrict__ dnp_out,
              double* __restrict__ dnm_out, int side, double oa, double ob, double oq,
              const double* __restrict__ xop, double* __restrict__ yop) {
  __shared__ double scratch[16];
  double qs = 0.0;
  if (yop && oq != 0.0) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nq; i += blockDim.x) s += qpart[i];
    qs = block_sum<double>(s, scratch);
  }
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const MarkerExt& me = ext[k];
  double v[6], Q[5];
#pragma unroll
  for (int m = 0; m < 6; ++m) v[m] = static_cast<double>(nodeval[stn[6 * k + m]]);
#pragma unroll
  for (int q = 0; q < 5; ++q) Q[q] = mq[q * M + k];
  double out[3], jm[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double s = 0.0, t = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) s += me.W[6 * r + m] * v[m];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      s += me.E[5 * r + q] * Q[q];
      t += me.D[5 * r + q] * Q[q];
    }
    out[r] = s;
    jm[r] = t;
  }
  const double vp = out[0], vm = out[0] - jm[0];
  const double dnp = me.nx * out[1] + me.ny * out[2];
  const double dnm = me.nx * (out[1] - jm[1]) + me.ny * (out[2] - jm[2]);
  if (vp_out) vp_out[k] = vp;
  if (vm_out) vm_out[k] = vm;
  if (dnp_out) dnp_out[k] = dnp;
  if (dnm_out) dnm_out[k] = dnm;
  if (yop) {
    const double tr = (side == KFBI_PLUS) ? vp : (side == KFBI_MINUS ? vm : 0.5 * (vp + vm));
    yop[k] = oa * xop[k] + ob * tr + oq * qs;
  }
}

// -------------------------------------------------------------------- full-grid evaluation
// grid[j][i] = (2/N) sum_p G[j-1][p-1] sin(p i pi / N), 64x64 output tiles, 4x4 per thread.
template <class T>
__global__ void __launch_bounds__(256)
    k_fullgrid(int N, const T* __restrict__ G, int ldG, const T* __restrict__ sinT,
               double* __restrict__ grid) {
  __shared__ T As[16][65];
  __shared__ T Bs[16][65];
  const int n = N - 1;
  const int mask = 2 * N - 1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;  // 0-based interior indices
  T acc[4][4] = {};
  for (int k0 = 0; k0 < n; k0 += 16) {
    for (int t = threadIdx.x; t < 16 * 64; t += 256) {
      const int kk = t & 15, rr = t >> 4;
      const int jr = j0 + rr, kp = k0 + kk;
      As[kk][rr] = (jr < n && kp < n) ? G[static_cast<size_t>(jr) * ldG + kp] : T(0);
      const int ic = i0 + rr;
      Bs[kk][rr] = (ic < n && kp < n) ? sinT[((kp + 1) * (ic + 1)) & mask] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty * 4 + q];
        bv[q] = Bs[kk][tx * 4 + q];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] += a[r] * bv[q];
    }
    __syncthreads();
  }
  const double sc = 2.0 / N;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jr = j0 + ty * 4 + r, ic = i0 + tx * 4 + q;
      if (jr < n && ic < n)
        grid[static_cast<size_t>(jr + 1) * (N + 1) + (ic + 1)] = sc * static_cast<double>(acc[r][q]);
    }
}

template <class T>
__global__ void k_grid_ring(int N, const T* __restrict__ ring, double* __restrict__ grid) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = N + 1;
  if (t >= n1) return;
  const double b = ring ? static_cast<double>(ring[t]) : 0.0;
  const double tp = ring ? static_cast<double>(ring[n1 + t]) : 0.0;
  const double l = ring ? static_cast<double>(ring[2 * n1 + t]) : 0.0;
  const double r = ring ? static_cast<double>(ring[3 * n1 + t]) : 0.0;
  if (t > 0 && t < N) {  // corners come from the left/right columns
    grid[t] = b;
    grid[static_cast<size_t>(N) * n1 + t] = tp;
  }
  grid[static_cast<size_t>(t) * n1] = l;
  grid[static_cast<size_t>(t) * n1 + N] = r;
}

template <class T>
__global__ void k_ring_cast(int n, const double* __restrict__ src, T* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = static_cast<T>(src[t]);
}

static inline int nblk(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

template <class T, int E>
static void launch_solve(kfbi_ctx* c, const T* armr, const T* sinT, const T* ring, int jlo,
                         int jhi, T* G, bool full, double* grid, T* nodeval, hipEvent_t ev2) {
  const int N = c->N, n = N - 1;
  const int ngrp = nblk(n, kColsPerBlock);
  const int nb = ((ngrp + 7) / 8) * 8;
  hipLaunchKernelGGL((k_colsolve<T, E>), dim3(nb), dim3(256), 0, c->stream, N, c->h, c->c2,
                     c->armrow.as<int>(), c->armi.as<int>(), armr, sinT, ring, jlo, jhi, N, G,
                     nb);
  if (ev2) hipEventRecord(ev2, c->stream);
  if (c->st.n_rows > 0)
    hipLaunchKernelGGL((k_nodes<T, E>), dim3(c->st.n_rows), dim3(256), 0, c->stream, N,
                       c->rows.as<int>(), c->rowptr.as<int>(), c->nodei.as<int>(), sinT, jlo, N,
                       G, nodeval);
  if (full) {
    hipLaunchKernelGGL((k_fullgrid<T>), dim3(nblk(n, 64), nblk(n, 64)), dim3(256), 0, c->stream,
                       N, G, N, sinT, grid);
    hipLaunchKernelGGL((k_grid_ring<T>), dim3(nblk(N + 1, 256)), dim3(256), 0, c->stream, N, ring,
                       grid);
  }
}

template <class T>
static int apply_t(kfbi_ctx* c, int layer, const double* dens, const double* ring_user,
                   const kfbi_out* out, const kfbi_bie* op, const double* xop, double* yop) {
  const int M = c->M, N = c->N;
  hipStream_t s = c->stream;
  const bool full = out && out->grid;
  T* armr = reinterpret_cast<T*>(c->armr.p);
  T* ring = nullptr;
  const T* sinT = reinterpret_cast<const T*>(sizeof(T) == 8 ? c->sinT.p : c->sinT32.p);
  T* G = reinterpret_cast<T*>(c->gband.p);
  T* nodeval = reinterpret_cast<T*>(c->nodeval.p);
  int nring = 0;
  if (c->box_bc == KFBI_BOX_FREESPACE) {
    ring = reinterpret_cast<T*>(c->ring.p);
    nring = nblk(4 * (N + 1), 16);
  } else if (c->box_bc == KFBI_BOX_USER) {
    ring = reinterpret_cast<T*>(c->ring.p);
    hipLaunchKernelGGL((k_ring_cast<T>), dim3(nblk(4 * (N + 1), 256)), dim3(256), 0, s,
                       4 * (N + 1), ring_user, ring);
  }
  hipEvent_t* ev = nullptr;
  if (c->prof_on) {
    if (c->prof_used + 5 > kfbi_ctx::kProfPool) KFBI_TRY(prof_flush(c));
    ev = c->prof_ev + c->prof_used;
    c->prof_used += 5;
    hipEventRecord(ev[0], s);
  }
  const int C = c->mk_chunk, nmk = c->n_mk_blocks;
  const int H = C + 5;
  const size_t lds = sizeof(double) * (M + 8 * 2 * H + 5 * H);
  hipLaunchKernelGGL((k_prep<T>), dim3(nmk + nring), dim3(256), lds, s, M, C, nmk, layer, dens,
                     c->dvec.as<double>(), c->dvec.as<double>() + M, c->armcoef.as<ArmCoef>(),
                     c->armint.as<int>(), c->intptr.as<int>(), armr, c->mq.as<double>(),
                     c->qpart.as<double>(), c->ext.as<MarkerExt>(), nring, N, c->x0, c->y0, c->h,
                     c->X.as<double>(), c->geo.as<double>(), ring);
  if (ev) hipEventRecord(ev[1], s);
  const int jlo = full ? 1 : c->st.row_lo;
  const int jhi = full ? N - 1 : c->st.row_hi;
  double* grid = full ? out->grid : nullptr;
  const int E = (N - 1 + 63) / 64;
  switch (E <= 1 ? 1 : E <= 2 ? 2 : E <= 4 ? 4 : E <= 8 ? 8 : E <= 16 ? 16 : E <= 32 ? 32 : 64) {
    case 1: launch_solve<T, 1>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
    case 2: launch_solve<T, 2>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
    case 4: launch_solve<T, 4>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
    case 8: launch_solve<T, 8>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
    case 16: launch_solve<T, 16>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
    case 32: launch_solve<T, 32>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
    default: launch_solve<T, 64>(c, armr, sinT, ring, jlo, jhi, G, full, grid, nodeval, ev ? ev[2] : nullptr); break;
  }
  if (ev) hipEventRecord(ev[3], s);
  const int side = op ? op->side : 0;
  const double oa = op ? op->a : 0.0, ob = op ? op->b : 0.0, oq = op ? op->q : 0.0;
  hipLaunchKernelGGL((k_extract<T>), dim3(nblk(M, 256)), dim3(256), 0, s, M, c->mknode.as<int>(),
                     nodeval, c->mq.as<double>(), c->ext.as<MarkerExt>(), c->qpart.as<double>(),
                     nmk, out ? out->v_plus : nullptr, out ? out->v_minus : nullptr,
                     out ? out->dn_plus : nullptr, out ? out->dn_minus : nullptr, side, oa, ob, oq,
                     xop, yop);
  if (ev) hipEventRecord(ev[4], s);
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

// Accumulate the elapsed times of the recorded applies (synchronises the stream).
int prof_flush(kfbi_ctx* c) {
  KFBI_HIP(hipStreamSynchronize(c->stream));
  for (int b = 0; b + 5 <= c->prof_used; b += 5) {
    for (int q = 0; q < 4; ++q) {
      float ms = 0.f;
      KFBI_HIP(hipEventElapsedTime(&ms, c->prof_ev[b + q], c->prof_ev[b + q + 1]));
      c->prof_ms[q] += ms;
    }
    ++c->prof_count;
  }
  c->prof_used = 0;
  return KFBI_OK;
}

int apply_impl(kfbi_ctx* c, int layer, int precision, const double* dens, const double* ring_user,
               const kfbi_out* out, const kfbi_bie* op, const double* xop, double* yop) {
  if (precision == KFBI_FP32) return apply_t<float>(c, layer, dens, ring_user, out, op, xop, yop);
  return apply_t<double>(c, layer, dens, ring_user, out, op, xop, yop);
}

}  // namespace kfbi
