// One KFBI operator apply on gfx950 (Sec. 4): four kernels per apply.
//
//  K1 k_prep     per chunk of markers: Fourier derivatives at the markers in circulant
//                form (Phi_a, Phi_aa or Psi_a; FP64), the marker jump quantities, the
//                jump corrections r_a of the irregular arms whose interval starts in the
//                chunk (Sec. 4.2.1 eq. modified-fdm with App. A.1 jumps; 6-point
//                interpolation of the marker quantities, coefficients precomputed per
//                interface), trapezoid-weight partial sums, and the free-space box data of
//                Sec. 4.1 when requested.
//  K2 k_rowdst   per row part: the sine transform along x of the row's sparse right-hand
//                side, T[j][p] = sum_{arms in row j} r_a sin(p i_a pi / N).
//  K3 k_colsolve per sine mode p along y, the constant tridiagonal system
//                    G_{j+1} - (2 + delta_p) G_j + G_{j-1} = h^2 T[j][p] (+ box terms),
//                    delta_p = 4 sin^2(p pi / 2N) + h^2 c^2,  G_0 = G_N = 0,
//                solved per wavefront by two first-order recurrences (root rho_p of
//                rho + 1/rho = 2 + delta_p) and a rank-one boundary correction; four modes
//                per block, output rows row_lo..row_hi of G.  When the arm rows carry the
//                whole right-hand side (zero box), k_colsolve_band solves only the band of
//                rows between the first and last arm or node row, with the exact
//                condition of the empty rows beyond it at each end.
//  K4 k_nodes_extract  per chunk of markers: inverse transform along x at the chunk's
//                interpolation nodes, v_ij = (2/N) sum_p G[j][p] sin(p i pi / N), then the
//                Sec. 4.3 corrected interpolation with precomputed weights -> v+-,
//                n.grad v+-, and the boundary operator a x + b trace + q int x ds.
// Together K2-K4 are the exact solution of the corrected five-point system (the 2-D
// sine transform with the y-direction replaced by its tridiagonal equivalent).  The
// full-grid variant writes every row in K3 and evaluates the whole grid with a tiled
// product against the sine matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.h"
#include "device_util.h"

namespace kfbi {

constexpr int kColsPerBlock = 4;
constexpr int kReg = 8;       // circulant outputs per thread in K1
constexpr int kNodeBatch = 8; // nodes reduced together in K4
// K4 for chunks of one marker (M < 512, at most six nodes) splits the mode slots of every
// node among its eight wavefronts once each lane holds at least this many slots
constexpr int kModeSplitMinE = 9;
constexpr int kMaxChunk = 16;  // markers per K1/K4 chunk: M / 256 for M <= 4096
constexpr int kRingNodes = 8;  // free-space box nodes per K1 block
constexpr int kWinMax = 24;     // derivative window per K1 chunk: at most 16 + 5 markers
// K4 block size for a single density: eight wavefronts share a chunk's nodes (fewer rows,
// the long-latency loads of the node loop, per wavefront).  The FP64 row of E > 32 mode
// slots per lane fits the registers of eight only when the chunk's extraction weights are
// staged in LDS instead of being held in registers through the node loop
// (node_stage_ext).  A batch launches four-wavefront blocks: with many blocks per CU they
// overlap better.
template <class T, int E>
__host__ __device__ constexpr bool node_stage_ext() {
  return sizeof(T) == 8 && E > 32;
}
template <class T, int E>
__host__ __device__ constexpr int node_threads() {
  return 512;
}
static_assert(kMaxChunk * 256 >= 4096, "chunks of M / 256 markers for M up to 4096");

// Two-level sine table in LDS: sin/cos(pi m / N) for m = 64 q + r from
// hs/hc[q] = sin/cos(pi 64 q / N) and ls/lc[r] = sin/cos(pi r / N) by angle addition.
template <class T>
struct SinTab2 {
  T* hs;
  T* hc;
  T* ls;
  T* lc;
  __device__ void stage(T* base, int N, const T* __restrict__ sinT) {
    const int nh = (2 * N) / 64 > 0 ? (2 * N) / 64 : 1;
    hs = base;
    hc = base + nh;
    ls = base + 2 * nh;
    lc = base + 2 * nh + 64;
    const int mask = 2 * N - 1, quarter = N / 2;
    const int t = threadIdx.x;
    if (t < nh) {
      hs[t] = sinT[(64 * t) & mask];
      hc[t] = sinT[(64 * t + quarter) & mask];
    }
    if (t < 64) {
      ls[t] = sinT[t & mask];
      lc[t] = sinT[(t + quarter) & mask];
    }
  }
  __device__ __forceinline__ void get(int m, T& s, T& c) const {
    const int q = m >> 6, r = m & 63;
    const T sa = hs[q], ca = hc[q], sb = ls[r], cb = lc[r];
    s = sa * cb + ca * sb;
    c = ca * cb - sa * sb;
  }
};
template <class T>
__host__ __device__ constexpr int sintab2_size(int N) {
  return 2 * ((2 * N) / 64 > 0 ? (2 * N) / 64 : 1) + 128;
}

// Padded LDS position of entry m of a marker array in K1.
__host__ __device__ __forceinline__ int lpad(int m) { return m + (m >> 5); }

// Column-group-major layouts: the four modes p = 4g+1..4g+4 of a row are adjacent and
// the rows of one group are contiguous.
__device__ __forceinline__ size_t grp_index(int p, int r, int nrows) {
  return (static_cast<size_t>((p - 1) >> 2) * nrows + r) * 4 + ((p - 1) & 3);
}
// Band layout of a solve output, element (mode slot q, row r): r ldr + q, row-major, when
// ldr > 0 (the band of rows that the node kernel reads: a lane-consecutive run of modes is
// then one contiguous piece of a row), else grp_index(q + 1, r, nrows), the column-group
// layout (full fields).  q = p - 1 for the sine modes p = 1..n, q = p for the cosine modes.

// LDS doubles after ph in a K1 marker block: d1 (and d2) during the circulant sums, then
// the 256 x kReg partial sums.
__host__ __device__ __forceinline__ int kprep_region(int M, int nd) {
  const int r = nd * (lpad(M - 1) + 1);
  return r > 256 * kReg ? r : 256 * kReg;
}

// Free-space box data of one K1 ring block in arithmetic R: thread (node nd, slice sl) sums
// the trapezoid terms of one slice of the markers, staged in LDS ((x, y, phi y_a, phi x_a)
// for the double layer, (x, y, psi s_a / 2) for the single layer) kRingChunk markers at a
// time, every thread's loads of a chunk in flight together; the slices are then added in
// order.  Writes ring (FP64, when R is double) and ringT (FP32 copy, when given).
constexpr int kRingChunk = 2048;
template <class R>
__device__ __forceinline__ void ring_sums(double* lds, int tid, int sl, int nd, int S, bool live,
                                          int node, int M, int layer,
                                          const double* __restrict__ X,
                                          const double* __restrict__ geo,
                                          const double* __restrict__ dens, R zx, R zy,
                                          double* __restrict__ ring, float* __restrict__ ringT) {
  const int CH = M < kRingChunk ? M : kRingChunk;
  R* cx = reinterpret_cast<R*>(lds);
  R* cy = cx + CH;
  R* ca = cy + CH;
  R* cb = ca + CH;
  R acc = R(0);
  constexpr int U = kRingChunk / 256;
  for (int c0 = 0; c0 < M; c0 += CH) {
    const int nk = min(CH, M - c0);
    if (c0 > 0) __syncthreads();
    {
      R vx[U], vy[U], va[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // loads first, all in flight
        const int e = tid + 256 * u;
        const int k = c0 + e;
        vx[u] = vy[u] = va[u] = vb[u] = R(0);
        if (e < nk) {
          vx[u] = static_cast<R>(X[k]);
          vy[u] = static_cast<R>(X[M + k]);
          if (layer == KFBI_DOUBLE) {
            const double f = dens[k];
            va[u] = static_cast<R>(f * geo[M + k]);
            vb[u] = static_cast<R>(f * geo[k]);
          } else {
            va[u] = static_cast<R>(0.5 * dens[k] * geo[4 * M + k]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = tid + 256 * u;
        if (e < nk) {
          cx[e] = vx[u];
          cy[e] = vy[u];
          ca[e] = va[u];
          cb[e] = vb[u];
        }
      }
    }
    __syncthreads();
    // slice sl takes markers sl, sl + S, sl + 2S, ...: the slices of a wavefront read
    // consecutive LDS entries (no bank conflicts)
    if (layer == KFBI_DOUBLE) {
#pragma unroll 4
      for (int q = sl; q < nk; q += S) {
        const R dx = cx[q] - zx, dy = cy[q] - zy;
        // 1 / |d|^2 from the hardware reciprocal and Newton steps (|d| >= 3h, far from the
        // under- and overflow range): two in FP64, one in FP32
        const R d2 = dx * dx + dy * dy;
        R rc;
        if constexpr (sizeof(R) == 8) {
          rc = __builtin_amdgcn_rcp(d2);
          rc = fma(fma(-d2, rc, 1.0), rc, rc);
          rc = fma(fma(-d2, rc, 1.0), rc, rc);
        } else {
          rc = __builtin_amdgcn_rcpf(d2);
          rc = fmaf(fmaf(-d2, rc, 1.0f), rc, rc);
        }
        acc += (dx * ca[q] - dy * cb[q]) * rc;
      }
    } else {
#pragma unroll 4
      for (int q = sl; q < nk; q += S) {
        const R dx = cx[q] - zx, dy = cy[q] - zy;
        acc += ca[q] * log(dx * dx + dy * dy);
      }
    }
  }
  __syncthreads();
  R* part = reinterpret_cast<R*>(lds);  // S x kRingNodes
  part[sl * kRingNodes + nd] = acc;
  __syncthreads();
  if (tid < kRingNodes && live) {
    R v = R(0);
    for (int q = 0; q < S; ++q) v += part[q * kRingNodes + tid];
    v /= static_cast<R>(M);
    if constexpr (sizeof(R) == 8) ring[node] = v;
    if (ringT) ringT[node] = static_cast<float>(v);
  }
}

// ---------------------------------------------------------------------------------- K1
// Marker-chunk blocks [0, nmk): derivatives at markers k0..k1-1 with phi, d1, d2 staged
// in LDS; every thread accumulates kReg consecutive outputs over a slice of m with a
// sliding window on d.  Ring blocks [nmk, nmk+nring): free-space box data.
__global__ void __launch_bounds__(256)
    k_prep(int M, int C, int nmk, int layer, const double* __restrict__ dens,
           const double* __restrict__ d1, const double* __restrict__ d2,
           double* __restrict__ mq, double* __restrict__ qpart, const double* __restrict__ wq,
           int N, double x0, double y0, double h, const double* __restrict__ X,
           const double* __restrict__ geo, double* __restrict__ ring, float* __restrict__ ringT,
           const int* __restrict__ ckoff, const int* __restrict__ cklist,
           const double* __restrict__ ckc, const int* __restrict__ ckk, int cap,
           double* __restrict__ rarm, int ring32) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  {  // density blockIdx.y of a batch: its own slices of every per-density array
    const int bd = blockIdx.y;
    dens += static_cast<size_t>(bd) * M;
    mq += static_cast<size_t>(bd) * 5 * M;
    qpart += static_cast<size_t>(bd) * nmk;
    rarm += static_cast<size_t>(bd) * cap;
    ring += static_cast<size_t>(bd) * 8 * (N + 1);
    if (ringT) ringT += static_cast<size_t>(bd) * 16 * (N + 1);
  }
  if (static_cast<int>(blockIdx.x) >= nmk) {
    // ----- box data: kRingNodes box nodes per block; thread (node, slice) sums the
    // trapezoid terms of one slice of the markers, slices are then added in order
    const int rb = blockIdx.x - nmk;
    const int nd = tid % kRingNodes, sl = tid / kRingNodes;
    constexpr int S = 256 / kRingNodes;
    const int n1 = N + 1;
    const int node = rb * kRingNodes + nd;
    const bool live = node < 4 * n1;
    double zx = 0.0, zy = 0.0;
    if (live) {
      const int side = node / n1, r = node % n1;
      zx = (side == 2) ? x0 : (side == 3 ? x0 + N * h : x0 + r * h);
      zy = (side == 0) ? y0 : (side == 1 ? y0 + N * h : y0 + r * h);
    }
    if (ring32) {  // an FP32 apply: the box data in FP32 (its only consumer is FP32)
      ring_sums<float>(lds, tid, sl, nd, S, live, node, M, layer, X, geo, dens,
                       static_cast<float>(zx), static_cast<float>(zy), ring, ringT);
    } else {
      ring_sums<double>(lds, tid, sl, nd, S, live, node, M, layer, X, geo, dens, zx, zy, ring,
                        ringT);
    }
    return;
  }
  // ----- marker chunk [k0, k1): derivatives on the window k0-2 .. k1+2 (the markers the
  // 6-point interpolation of this chunk's arms reads), marker quantities of the chunk,
  // and the arm corrections r_a of the arms whose interval starts in the chunk
  const int b = blockIdx.x;
  const int k0 = b * C;
  const int k1 = min(M, k0 + C);
  const int H = k1 - k0;
  const int HW = H + 5;
  const int w0 = k0 - 2;
  const int nd = (layer == KFBI_DOUBLE) ? 2 : 1;
  const int ngr = (HW + kReg - 1) / kReg;
  const int ng = ngr * nd;
  int ngp = 1;  // groups rounded up to a power of two (at most 16)
  while (ngp < ng) ngp <<= 1;
  const int S = 256 / ngp;  // slices of m
  // ph, dl1, dl2 hold M values each at padded positions lpad(m) = m + m / 32: the slices
  // of m summed by the lanes of a wavefront start 32 apart, and the padding puts their
  // reads in different LDS banks
  const int Mp = lpad(M - 1) + 1;
  double* ph = lds;              // Mp
  double* dl1 = ph + Mp;         // Mp
  double* dl2 = dl1 + Mp;        // Mp (double layer only)
  double* red = dl1;             // after the sums: the 256 x kReg partial sums
  double* part = dl1 + kprep_region(M, nd);  // 16 x kReg window sums (and block_sum)
  double* qw = part + 16 * kReg;  // 5 x kWinMax
  // this chunk's arm records, in list order (issued first: the record loads below depend
  // on them and then overlap the circulant sums); ckk holds the window offset k_a - k0
  // of marker k_a - 2
  const int a0 = ckoff[b], a1 = ckoff[b + 1];
  const double wmine = (wq && k0 + tid < k1) ? wq[k0 + tid] : 0.0;
  for (int m0 = tid; m0 < M; m0 += 256 * 8) {
    double a[8], bb[8], cc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = m0 + 256 * u;
      if (m < M) {
        a[u] = dens[m];
        bb[u] = d1[m];
        cc[u] = (nd == 2) ? d2[m] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = m0 + 256 * u;
      if (m < M) {
        ph[lpad(m)] = a[u];
        dl1[lpad(m)] = bb[u];
        if (nd == 2) dl2[lpad(m)] = cc[u];
      }
    }
  }
  // first arm of this thread: slot, window offset of marker k_a - 2, coefficients
  const int e0 = a0 + tid;
  const bool arm0 = e0 < a1;
  unsigned slot0 = 0, t00 = 0;  // unsigned: nothing needs the values before the barrier
  double cf[kArmCoefCount];
  if (arm0) {
    slot0 = static_cast<unsigned>(cklist[e0]);
    t00 = static_cast<unsigned>(ckk[e0]);
#pragma unroll
    for (int qq = 0; qq < kArmCoefCount; ++qq) cf[qq] = ckc[qq * cap + e0];
  }
  __syncthreads();
  // thread = (slice sl, group g): g = tid mod ngp, so the slices of one group sit in
  // lanes ngp apart and are summed by shuffles, then over the four wavefronts
  const int g = tid & (ngp - 1), sl = tid / ngp;
  double acc[kReg];
#pragma unroll
  for (int r = 0; r < kReg; ++r) acc[r] = 0.0;
  if (g < ng) {
    const int dv = g / ngr, gr = g % ngr;
    const double* dd = dv == 0 ? dl1 : dl2;
    const int per = (M + S - 1) / S;
    const int mb = sl * per, me = min(M, mb + per);
    // outputs k_r = w0 + gr*kReg + r ; window w[r] = d[(k_r - m) mod M]
    int kb = (w0 + gr * kReg - mb) % M;
    kb += (kb < 0) ? M : 0;
    double w[kReg];
#pragma unroll
    for (int r = 0; r < kReg; ++r) {
      int q = kb + r;
      q -= (q >= M) ? M : 0;
      w[r] = dd[lpad(q)];
    }
    int q = kb;  // index of w[0]
    int m = mb;
    double acc2[kReg];  // odd steps: two independent FMA chains per output
#pragma unroll
    for (int r = 0; r < kReg; ++r) acc2[r] = 0.0;
    for (; m + 8 <= me; m += 8) {
      double f[8], nw[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        f[u] = ph[lpad(m + u)];
        int qq = q - 1 - u;
        qq += (qq < 0) ? M : 0;
        nw[u] = dd[lpad(qq)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
#pragma unroll
        for (int r = 0; r < kReg; ++r) {
          if (u & 1) acc2[r] += w[r] * f[u];
          else acc[r] += w[r] * f[u];
        }
#pragma unroll
        for (int r = kReg - 1; r > 0; --r) w[r] = w[r - 1];
        w[0] = nw[u];
      }
      q -= 8;
      q += (q < 0) ? M : 0;
    }
#pragma unroll
    for (int r = 0; r < kReg; ++r) acc[r] += acc2[r];
    for (; m < me; ++m) {
      const double f = ph[lpad(m)];
#pragma unroll
      for (int r = 0; r < kReg; ++r) acc[r] += w[r] * f;
#pragma unroll
      for (int r = kReg - 1; r > 0; --r) w[r] = w[r - 1];
      q = (q == 0) ? M - 1 : q - 1;
      w[0] = dd[lpad(q)];
    }
  }
  // slices summed through LDS: the partial sums replace d1, d2; output (g, r) is then
  // summed by T2 = 32 / ngp threads, eight slices each, and a shuffle tree over them
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kReg; ++r) red[tid * kReg + r] = acc[r];
  __syncthreads();
  {
    const int T2 = 32 / ngp;  // threads per output (ngp * kReg outputs, 256 threads)
    const int o = tid / T2, p = tid % T2;
    const int go = o / kReg, ro = o % kReg;
    double sacc = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) sacc += red[((p + u * T2) * ngp + go) * kReg + ro];
    for (int off = 1; off < T2; off <<= 1) sacc += __shfl_xor(sacc, off, 64);
    if (p == 0) part[o] = sacc;
  }
  __syncthreads();
  // window quantities Q = (Phi, Phi_a, Phi_aa, Psi, Psi_a) at markers w0 + t
  double v1 = 0.0, v2 = 0.0, vph = 0.0;
  if (tid < HW) {
    const int gr = tid / kReg, r = tid % kReg;
    v1 = part[gr * kReg + r];
    if (nd == 2) v2 = part[(ngr + gr) * kReg + r];
    int km = w0 + tid;
    km += (km < 0) ? M : 0;
    km -= (km >= M) ? M : 0;
    vph = ph[lpad(km)];
    const bool dl = (layer == KFBI_DOUBLE);
    qw[0 * kWinMax + tid] = dl ? vph : 0.0;
    qw[1 * kWinMax + tid] = dl ? v1 : 0.0;
    qw[2 * kWinMax + tid] = dl ? v2 : 0.0;
    qw[3 * kWinMax + tid] = dl ? 0.0 : -vph;  // Psi = -psi for the single layer
    qw[4 * kWinMax + tid] = dl ? 0.0 : -v1;
  }
  // trapezoid partial sum of the density (only for an operator with a q term: wq given)
  double qs = (wq && k0 + tid < k1) ? ph[lpad(k0 + tid)] * wmine : 0.0;
  if (wq)
    for (int k = k0 + 256 + tid; k < k1; k += 256) qs += ph[lpad(k)] * wq[k];
  __syncthreads();
  // arm corrections r_a = sum_m l_m sum_q coef_q Q_q(k_a - 2 + m) (Sec. 4.2.1 with the
  // App. A.1 jumps; coefficients per arm from the interface setup)
  if (arm0) {
    double r = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double sm = 0.0;
#pragma unroll
      for (int qq = 0; qq < 5; ++qq) sm += cf[6 + qq] * qw[qq * kWinMax + t00 + m];
      r += cf[m] * sm;
    }
    rarm[slot0] = r;
  }
  for (int e = e0 + 256; e < a1; e += 256) {  // chunks with more than 256 arms
    const int t0 = ckk[e];
    double r = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double sm = 0.0;
#pragma unroll
      for (int qq = 0; qq < 5; ++qq) sm += ckc[(6 + qq) * cap + e] * qw[qq * kWinMax + t0 + m];
      r += ckc[m * cap + e] * sm;
    }
    rarm[cklist[e]] = r;
  }
  if (wq) qs = block_sum<double>(qs, part);  // block-uniform condition
  // global stores last (no barrier waits on them)
  if (tid >= 2 && tid < 2 + H) {
    const int k = w0 + tid;
#pragma unroll
    for (int qq = 0; qq < 5; ++qq) mq[qq * M + k] = qw[qq * kWinMax + tid];
  }
  if (wq && tid == 0) qpart[b] = qs;
}

// ---------------------------------------------------------------------------------- K2
// One block per row part (a row's arms in groups of at most kArmsPerPart, corrections r_a
// from K1 in part-slot order); every thread evaluates the partial transform
// T_part[p] = sum_a r_a sin(p i_a pi / N) for PT consecutive modes p, starting from the
// two-level table and advancing by the three-term sine recurrence in steps of i_a pi / N.
// Parts of one row are summed in
// part order by the solve kernel.
// COSB (zero-normal-derivative box): the cosine transform T[j][p] = sum_a r_a cos(p i_a pi/N)
// over the modes p = 0..N instead (mode index p, not p - 1, in the column-group layout).
template <class T, int PT, bool COSB>
__global__ void __launch_bounds__(256)
    k_rowdst(int N, int P, const int4* __restrict__ pdesc, const double* __restrict__ rslot,
             const int* __restrict__ iR, const double* __restrict__ sc,
             const T* __restrict__ sinT, T* __restrict__ Tg, size_t tstride) {
  __shared__ T tab[sintab2_size<T>(4096)];
  __shared__ T rr[kArmsPerPart], ssb[kArmsPerPart], scb[kArmsPerPart];
  __shared__ int ii[kArmsPerPart];
  const int n = N - 1;
  const int mask = 2 * N - 1;
  const int tid = threadIdx.x;
  // XCD-aware order: blocks resident on one XCD (ids congruent mod 8) take consecutive
  // parts, so the four parts that share each 128-byte line of the output meet in one L2
  const int per_xcd = static_cast<int>(gridDim.x) / 8;
  const int q = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (q >= P) return;
  const int cap = kArmsPerPart * P;
  rslot += static_cast<size_t>(blockIdx.y) * cap;
  Tg += static_cast<size_t>(blockIdx.y) * tstride;
  const int4 d = pdesc[q];
  SinTab2<T> st2;
  st2.stage(tab, N, sinT);
  if (tid < kArmsPerPart) {  // slot tid of the part (empty slots have r = 0, i = 0)
    const int a = q * kArmsPerPart + tid;
    rr[tid] = static_cast<T>(rslot[a]);
    ii[tid] = iR[a];
    ssb[tid] = static_cast<T>(sc[a]);        // sin(i pi / N), the recurrence step
    scb[tid] = static_cast<T>(sc[cap + a]);  // cos(i pi / N)
  }
  const int na = d.z - d.y;
  __syncthreads();
  const int p0 = (COSB ? 0 : 1) + tid * PT;
  const int pmax = COSB ? N : n;  // last mode
  T acc[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) acc[k] = T(0);
  for (int t = 0; t < na; ++t) {
    const int i = ii[t];
    const T r = rr[t];
    T s, c;
    st2.get((p0 * i) & mask, s, c);
    const T sb = ssb[t], cb = scb[t];
    // sin((p + 1) x) = 2 cos(x) sin(p x) - sin((p - 1) x), started from sin(p0 x) and
    // sin((p0 - 1) x); over PT steps the rounding grows by at most a factor PT.  The
    // cosine obeys the same recurrence.
    const T c2 = cb + cb;
    T sm;
    if constexpr (COSB) {
      sm = c * cb + s * sb;  // cos((p0 - 1) x)
      s = c;
    } else {
      sm = s * cb - c * sb;
    }
    acc[0] += r * s;
#pragma unroll
    for (int k = 1; k < PT; ++k) {
      const T sn = c2 * s - sm;
      sm = s;
      s = sn;
      acc[k] += r * s;
    }
  }
  if constexpr (PT % 4 == 0 && !COSB) {
    // whole groups of four modes: one 32-byte (FP64) or 16-byte (FP32) piece each; modes
    // beyond n land in the padding of the last group
#pragma unroll
    for (int k = 0; k < PT; k += 4) {
      T* dst = Tg + grp_index(p0 + k, q, P);
      if constexpr (sizeof(T) == 8) {
        reinterpret_cast<double2*>(dst)[0] = make_double2(acc[k], acc[k + 1]);
        reinterpret_cast<double2*>(dst)[1] = make_double2(acc[k + 2], acc[k + 3]);
      } else {
        reinterpret_cast<float4*>(dst)[0] = make_float4(acc[k], acc[k + 1], acc[k + 2], acc[k + 3]);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < PT; ++k)
      if (p0 + k <= pmax) Tg[grp_index(p0 + k + (COSB ? 1 : 0), q, P)] = acc[k];
  }
}

// ---------------------------------------------------------------------------------- K3
template <int E>
__device__ __forceinline__ int slot(int j) {  // row j (1-based) -> LDS slot, padded
  const int e = j - 1;
  return (e / E) * (E + 1) + (e % E);
}

template <class T, int E>
__global__ void __launch_bounds__(256)
    k_colsolve(int N, double h, int P, const T* __restrict__ Tg, const int* __restrict__ rowpart,
               const T* __restrict__ sinTg, const T* __restrict__ ring,
               const double* __restrict__ colc, const double* __restrict__ lanef, int jlo,
               int jhi, T* __restrict__ Gg, int nblk_x, size_t tstride, size_t rstride,
               size_t gstride, int ldr) {
  // dynamic LDS: the group's P part rows (4 modes each), then over the same bytes the
  // four modes' columns (each lane's E rows padded to E + 1)
  extern __shared__ double dynp[];
  T* tp = reinterpret_cast<T*>(dynp);
  T (*col)[64 * (E + 1)] = reinterpret_cast<T (*)[64 * (E + 1)]>(dynp);
  const int n = N - 1;
  const int mask = 2 * N - 1;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // XCD-aware order: blocks resident on one XCD (ids congruent mod 8) take adjacent
  // column groups.
  const int bid = blockIdx.x;
  const int per_xcd = (nblk_x + 7) / 8;
  const int grp = (bid % 8) * per_xcd + bid / 8;
  if (grp * kColsPerBlock + 1 > n) return;  // whole block beyond the last mode
  Tg += static_cast<size_t>(blockIdx.y) * tstride;
  if (ring) ring += static_cast<size_t>(blockIdx.y) * rstride;
  Gg += static_cast<size_t>(blockIdx.y) * gstride;
  const int p0 = 1 + grp * kColsPerBlock;
  const int p = p0 + w;
  const bool live = (p <= n);
  double rho = 0.0, eps = 0.0, inv_den = 0.0, abase = 0.0, r2j0 = 0.0;
  if (live) {
    rho = colc[3 * (p - 1)];
    eps = colc[3 * (p - 1) + 1];
    inv_den = colc[3 * (p - 1) + 2];
    abase = lanef[(static_cast<size_t>(p - 1) * 64 + lane) * 2];
    r2j0 = lanef[(static_cast<size_t>(p - 1) * 64 + lane) * 2 + 1];
  }
  constexpr int R = (64 * E + 255) / 256;  // rows per thread in the row sums
  int rq0[R], rq1[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int j = 1 + tid + 256 * u;
    rq0[u] = (j <= n) ? rowpart[j] : 0;
    rq1[u] = (j <= n) ? rowpart[j + 1] : 0;
  }
  // box data (issued with the slab loads below, consumed after the row sums): the left
  // (i=0) and right (i=N) box nodes next to (1, j) and (N-1, j) of this thread's rows, and
  // this wavefront's sine sums of the bottom (j=0) and top (j=N) box rows
  const int n1 = N + 1;
  T gl[R], gr[R], s1[kColsPerBlock], sn[kColsPerBlock];
  T sb = T(0), st = T(0);
  if (ring) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = 1 + tid + 256 * u;
      gl[u] = (j <= n) ? ring[2 * n1 + j] : T(0);
      gr[u] = (j <= n) ? ring[3 * n1 + j] : T(0);
    }
#pragma unroll
    for (int c = 0; c < kColsPerBlock; ++c) {
      s1[c] = sinTg[(p0 + c) & mask];
      sn[c] = sinTg[((p0 + c) * n) & mask];
    }
    // sin(p i pi / N) at i = 1 + lane + 64 u by the three-term recurrence in steps of
    // 64 p pi / N from two table values per lane (rounding grows at most E-fold)
    const int quarter = N / 2;
    const int m0 = (p * (1 + lane)) & mask, m64 = (64 * p) & mask;
    T a = sinTg[m0], c = sinTg[(m0 + quarter) & mask];
    const T sb64 = sinTg[m64], cb64 = sinTg[(m64 + quarter) & mask];
    const T c2 = cb64 + cb64;
    T am = a * cb64 - c * sb64;  // sin(p (1 + lane - 64) pi / N)
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int i = 1 + lane + 64 * u;
      const bool in = (i <= n);
      sb += (in ? ring[i] : T(0)) * a;
      st += (in ? ring[n1 + i] : T(0)) * a;
      const T an = c2 * a - am;
      am = a;
      a = an;
    }
  }
  // the group's part rows are contiguous: P x 4 values
  {
    const T* src = Tg + static_cast<size_t>(grp) * P * 4;
    constexpr int U = 16;
    for (int e0 = tid; e0 < 4 * P; e0 += 256 * U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 256 * u;
        v[u] = (e < 4 * P) ? src[e] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 256 * u;
        if (e < 4 * P) tp[e] = v[u];
      }
    }
  }
  __syncthreads();
  // rows: sum of their parts in part order (rows without arms are zero), then the left
  // and right box terms
  const T ih2 = static_cast<T>(1.0 / (h * h));
  {
    T a4[R][kColsPerBlock];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = 1 + tid + 256 * u;
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) a4[u][c] = T(0);
      if (j <= n) {
        for (int qq = rq0[u]; qq < rq1[u]; ++qq)
#pragma unroll
          for (int c = 0; c < kColsPerBlock; ++c) a4[u][c] += tp[4 * qq + c];
        if (ring)
#pragma unroll
          for (int c = 0; c < kColsPerBlock; ++c)
            a4[u][c] -= ih2 * (gl[u] * s1[c] + gr[u] * sn[c]);
      }
    }
    __syncthreads();  // the part rows are read: their bytes become the columns
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = 1 + tid + 256 * u;
      if (j > 64 * E) continue;
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) col[c][slot<E>(j)] = a4[u][c];
    }
  }
  __syncthreads();
  if (ring) {  // bottom and top box rows: rows 1 and n of this wavefront's mode
    sb = wave_sum(sb);
    st = wave_sum(st);
    if (lane == 0) {
      col[w][slot<E>(1)] -= ih2 * sb;
      col[w][slot<E>(n)] -= ih2 * st;
    }
    __syncthreads();
  }
  // tridiagonal solve along y for mode p, one wavefront; recurrences in eps = 1 - rho
  // form so FP32 keeps 1 - rho to full precision
  if (live) {
    const T rhoT = static_cast<T>(rho), epsT = static_cast<T>(eps);
    const T h2 = static_cast<T>(h * h);
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
    // G_j = -rho z_j + z_n rho^{n-j+3} (1 - rho^{2j}) / (1 - rho^{2n+2})
    const int ln = (n - 1) / E, en = (n - 1) % E;
    T sel = T(0);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e == en) sel = y[e];
    const T zn = __shfl(sel, ln, 64);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double a = abase * pw[E - 1 - e];
      const double om = 1.0 - r2j0 * pw[e] * pw[e];
      y[e] = -rhoT * y[e] + static_cast<T>(a * om * inv_den) * zn;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) col[w][lane * (E + 1) + e] = y[e];
  }
  __syncthreads();
  // rows jlo..jhi of G (band layout: this group's four slots of row r start at
  // base + r rs)
  const int nb = jhi - jlo + 1;
  const size_t base = ldr > 0 ? 4 * static_cast<size_t>(grp) : 4 * static_cast<size_t>(grp) * nb;
  const size_t rs = ldr > 0 ? static_cast<size_t>(ldr) : 4;
  for (int e = tid; e < 4 * nb; e += 256) {
    const int r = e >> 2, c = e & 3;
    Gg[base + r * rs + c] = (p0 + c <= n) ? col[c][slot<E>(jlo + r)] : T(0);
  }
}

// Per-mode constants of the column solve (depend on N, h, c^2 only):
//   colc[3(p-1) + {0,1,2}] = rho_p, 1 - rho_p, 1 / (1 - rho_p^{2n+2})
//   lanef[((p-1) 64 + l) 2 + {0,1}] = rho^{n - (j0+E-1) + 3}, rho^{2 j0}, j0 = l E + 1
__global__ void k_colconst(int N, double hc2, int E, double* __restrict__ colc,
                           double* __restrict__ lanef) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = N - 1;
  if (t >= n * 64) return;
  const int p = 1 + t / 64, l = t % 64;
  const double sp = sinpi(0.5 * p / N);
  const double delta = 4.0 * sp * sp + hc2;
  const double sq = sqrt(delta * (4.0 + delta));
  const double rho = 2.0 / (2.0 + delta + sq);
  const double eps = (delta + sq) / (2.0 + delta + sq);
  const double lr = log1p(-eps);
  if (l == 0) {
    colc[3 * (p - 1)] = rho;
    colc[3 * (p - 1) + 1] = eps;
    colc[3 * (p - 1) + 2] = 1.0 / (-expm1((2.0 * n + 2.0) * lr));
  }
  const int j0 = l * E + 1;
  lanef[static_cast<size_t>(t) * 2] = exp(static_cast<double>(n - (j0 + E - 1) + 3) * lr);
  lanef[static_cast<size_t>(t) * 2 + 1] = exp(2.0 * j0 * lr);
}

// ------------------------------------------------------ K3 for the zero-normal-derivative box
// Rows j = 0..N with mirrored ghosts: per cosine mode p = 0..N the system
//     G_{j+1} - (2 + delta_p) G_j + G_{j-1} = b_j,  j = 0..N,  G_{-1} = G_1, G_{N+1} = G_{N-1},
// b_j = h^2 (T[j][p] + ca Fa[j][p] + cb Fb[j][p]) (arm parts of the interior rows plus
// optional dense right-hand sides in the column-group layout).  The two first-order
// recurrences give a particular solution P_j = -rho z_j of the interior equations, valid
// for all j with P_{-1} = 0 and P_{N+1} = rho P_N; the mirror conditions then fix the
// homogeneous part:  G_j = P_j + A rho^j + B rho^{N-j} with
//     A = (D0 + rho^N D1) / (d (1 - rho^{2N})),  B = (D1 + rho^N D0) / (d (1 - rho^{2N})),
//     D0 = P_1,  D1 = P_{N-1} - rho P_N,  d = 1/rho - rho.
// Lane l of the wavefront holds rows l E .. l E + E - 1.
template <int E>
__device__ __forceinline__ int slot0(int r) {  // row r (0-based) -> LDS slot, padded
  return (r / E) * (E + 1) + (r % E);
}

template <class T, int E>
__global__ void __launch_bounds__(256)
    k_colsolve_neu(int N, double h, int P, const T* __restrict__ Tg,
                   const int* __restrict__ rowpart, const T* __restrict__ Fa,
                   const T* __restrict__ Fb, double ca, double cb,
                   const double* __restrict__ colc, const double* __restrict__ lanef, int jlo,
                   int jhi, T* __restrict__ Gg, int nblk_x, size_t tstride, size_t gstride,
                   int ldr) {
  // dynamic LDS: the group's P part rows (4 modes each), then over the same bytes the
  // four modes' columns (each lane's E rows padded to E + 1)
  extern __shared__ double dynp[];
  T* tp = reinterpret_cast<T*>(dynp);
  T (*col)[64 * (E + 1)] = reinterpret_cast<T (*)[64 * (E + 1)]>(dynp);
  const int nm = N + 1;  // modes and rows
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int bid = blockIdx.x;
  const int per_xcd = (nblk_x + 7) / 8;
  const int grp = (bid % 8) * per_xcd + bid / 8;
  if (grp * kColsPerBlock > N) return;  // whole block beyond the last mode
  Tg += static_cast<size_t>(blockIdx.y) * tstride;
  Gg += static_cast<size_t>(blockIdx.y) * gstride;
  const int m0 = grp * kColsPerBlock;
  const int m = m0 + w;
  const bool live = (m <= N);
  double rho = 0.0, eps = 0.0, inv_den = 0.0, rN = 0.0, lr0 = 0.0, lr1 = 0.0;
  if (live) {
    rho = colc[4 * m];
    eps = colc[4 * m + 1];
    inv_den = colc[4 * m + 2];
    rN = colc[4 * m + 3];
    lr0 = lanef[(static_cast<size_t>(m) * 64 + lane) * 2];
    lr1 = lanef[(static_cast<size_t>(m) * 64 + lane) * 2 + 1];
  }
  constexpr int R = (64 * E + 255) / 256;  // rows per thread in the row sums
  int rq0[R], rq1[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = tid + 256 * u;
    const bool in = (P > 0) && r >= 1 && r <= N - 1;  // arms sit on interior rows only
    rq0[u] = in ? rowpart[r] : 0;
    rq1[u] = in ? rowpart[r + 1] : 0;
  }
  if (P > 0) {
    const T* src = Tg + static_cast<size_t>(grp) * P * 4;
    constexpr int U = 16;
    for (int e0 = tid; e0 < 4 * P; e0 += 256 * U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 256 * u;
        v[u] = (e < 4 * P) ? src[e] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 256 * u;
        if (e < 4 * P) tp[e] = v[u];
      }
    }
  }
  __syncthreads();
  {
    const T tca = static_cast<T>(ca), tcb = static_cast<T>(cb);
    T a4[R][kColsPerBlock];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int r = tid + 256 * u;
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) a4[u][c] = T(0);
      if (r >= 64 * E) continue;
      for (int qq = rq0[u]; qq < rq1[u]; ++qq)
#pragma unroll
        for (int c = 0; c < kColsPerBlock; ++c) a4[u][c] += tp[4 * qq + c];
      if (Fa && r <= N) {
        const size_t o = (static_cast<size_t>(grp) * nm + r) * 4;
#pragma unroll
        for (int c = 0; c < kColsPerBlock; ++c) {
          T f = tca * Fa[o + c];
          if (Fb) f += tcb * Fb[o + c];
          a4[u][c] += f;
        }
      }
    }
    __syncthreads();  // the part rows are read: their bytes become the columns
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int r = tid + 256 * u;
      if (r >= 64 * E) continue;
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) col[c][slot0<E>(r)] = a4[u][c];
    }
  }
  __syncthreads();
  if (live) {
    const T rhoT = static_cast<T>(rho), epsT = static_cast<T>(eps);
    const T h2 = static_cast<T>(h * h);
    double pw[E + 1];
    pw[0] = 1.0;
#pragma unroll
    for (int e = 1; e <= E; ++e) pw[e] = pw[e - 1] * rho;
    T y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = h2 * col[w][lane * (E + 1) + e];
    // backward recurrence y_j = b_j + rho y_{j+1} (rows beyond N carry zeros)
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
    // P_j = -rho z_j; boundary differences from rows 1, N-1, N
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = -rhoT * y[e];
    T s1 = T(0), sa = T(0), sb = T(0);
    const int la = (N - 1) / E, ea = (N - 1) % E, lb = N / E, eb = N % E;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e == 1) s1 = y[e];
      if (e == ea) sa = y[e];
      if (e == eb) sb = y[e];
    }
    const double P1 = static_cast<double>(__shfl(s1, 0, 64));
    const double PNm = static_cast<double>(__shfl(sa, la, 64));
    const double PN = static_cast<double>(__shfl(sb, lb, 64));
    const double D0 = P1, D1 = PNm - rho * PN;
    const double A = (D0 + rN * D1) * inv_den, B = (D1 + rN * D0) * inv_den;
    // rows j = lane E + e: rho^j = lr0 rho^e, rho^{N-j} = lr1 rho^{E-1-e}
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = lane * E + e;
      if (j <= N) y[e] += static_cast<T>(A * lr0 * pw[e] + B * lr1 * pw[E - 1 - e]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) col[w][lane * (E + 1) + e] = y[e];
  }
  __syncthreads();
  // rows jlo..jhi (band layout: this group's four slots of row r start at
  // base + r rs)
  const int nb = jhi - jlo + 1;
  const size_t base = ldr > 0 ? 4 * static_cast<size_t>(grp) : 4 * static_cast<size_t>(grp) * nb;
  const size_t rs = ldr > 0 ? static_cast<size_t>(ldr) : 4;
  for (int e = tid; e < 4 * nb; e += 256) {
    const int r = e >> 2, c = e & 3;
    Gg[base + r * rs + c] = (m0 + c <= N) ? col[c][slot0<E>(jlo + r)] : T(0);
  }
}

// Per-mode constants of the mirrored-ghost column solve (p = 0..N):
//   colc[4p + {0,1,2,3}] = rho, 1 - rho, 1 / (d (1 - rho^{2N})), rho^N,  d = 1/rho - rho
//   lanef[(p 64 + l) 2 + {0,1}] = rho^{j0}, rho^{N - (j0 + E - 1)},  j0 = l E
__global__ void k_colconst_neu(int N, double hc2, int E, double* __restrict__ colc,
                               double* __restrict__ lanef) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (N + 1) * 64) return;
  const int p = t / 64, l = t % 64;
  const double sp = sinpi(0.5 * p / N);
  const double delta = 4.0 * sp * sp + hc2;
  const double sq = sqrt(delta * (4.0 + delta));
  const double rho = 2.0 / (2.0 + delta + sq);
  const double eps = (delta + sq) / (2.0 + delta + sq);
  const double lr = log1p(-eps);
  if (l == 0) {
    const double d = 1.0 / rho - rho;
    colc[4 * p] = rho;
    colc[4 * p + 1] = eps;
    colc[4 * p + 2] = 1.0 / (d * (-expm1(2.0 * N * lr)));
    colc[4 * p + 3] = exp(N * lr);
  }
  const int j0 = l * E;
  lanef[static_cast<size_t>(t) * 2] = exp(static_cast<double>(j0) * lr);
  lanef[static_cast<size_t>(t) * 2 + 1] = exp(static_cast<double>(N - (j0 + E - 1)) * lr);
}

// ------------------------------------------------- K3 on the band of rows that carry data
// When the only right-hand sides are the arm rows (zero box, or the zero-normal-derivative
// box inside the boundary operator), rows below lo and above hi = lo + nr - 1 carry none,
// and the solve is needed only on rows lo..hi (lo <= every arm row and node row <= hi).
// Outside that band the solution is the homogeneous one that meets the box condition, so
// the rows next to the band obey G_{lo-1} = kL G_lo and G_{hi+1} = kR G_hi with
//     zero box:    kL = rho (1 - rho^(2 lo - 2)) / (1 - rho^(2 lo))
//     mirror box:  kL = rho (1 + rho^(2 lo - 2)) / (1 + rho^(2 lo))
// (kR likewise with N - hi in place of lo); the mirror box keeps G_{-1} = G_1 when lo = 0
// and G_{N+1} = G_{N-1} when hi = N.  With the particular solution P of the two recurrences
// on the band (local rows i = 0..nr-1, P_{-1} = 0, P_nr = rho P_{nr-1}) the band solution is
// G_i = P_i + A rho^i + B rho^(nr-1-i), and the two conditions reduce to
//     A - cL B = RL,  B - cR A = RR,  cL cR = rho^(2N),
// zero box:   cL = -rho^(nr-1+2lo),  RL = rho (1 - rho^(2lo-2)) P_0 / d,
//             cR = -rho^(nr-1+2hb),  RR = -rho^(2hb) P_{nr-1}          (hb = N - hi)
// mirror box: cL = rho^(nr-1+2lo),   RL = rho (1 + rho^(2lo-2)) P_0 / d  (P_1 / d if lo = 0),
//             cR = rho^(nr-1+2hb),   RR = rho^(2hb) P_{nr-1}  ((P_{nr-2} - rho P_{nr-1}) / d
//                                                             if hb = 0),
// d = 1/rho - rho.  The result equals the full solve up to rounding; E rows per lane cover
// the band instead of the whole column.
// Per-mode constants of the band column solve for the band lo .. lo + nr - 1 with E rows
// per lane (formed once per band instead of in every solve): bc[kBandModeConsts q + {0..5}]
// = cL, cR, gL, gR, 1 / (1 - rho^(2N)), 1 / (1/rho - rho) of mode slot q, then per (q, lane)
// rho^(lane E) and rho^(nr - lane E - E) (zero for lanes wholly past the band).
constexpr int kBandModeConsts = 8;
template <bool NEU>
__global__ void k_band_const(int N, int lo, int nr, int E, const double* __restrict__ colc,
                             double* __restrict__ bc) {
  const int nmodes = NEU ? N + 1 : N - 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nmodes * 64) return;
  const int q = t / 64, lane = t % 64;
  const double rho = colc[(NEU ? 4 : 3) * q];
  const double eps = colc[(NEU ? 4 : 3) * q + 1];
  double id = colc[(NEU ? 4 : 3) * q + 2];  // 1 / (1 - rho^(2N)), divided by d for the mirror box
  const int hb = N - (lo + nr - 1);
  const double lr = log1p(-eps);
  const int k1 = nr - lane * E - E;
  double* lf = bc + static_cast<size_t>(kBandModeConsts) * nmodes;
  lf[static_cast<size_t>(t) * 2] = (lane * E < nr) ? exp(static_cast<double>(lane * E) * lr) : 0.0;
  lf[static_cast<size_t>(t) * 2 + 1] = (k1 > -E) ? exp(static_cast<double>(k1) * lr) : 0.0;
  if (lane != 0) return;
  const double invd = rho / (eps * (2.0 - eps));  // 1 / (1/rho - rho)
  const double gL = NEU ? ((lo == 0) ? invd
                                     : rho * (1.0 + exp(static_cast<double>(2 * lo - 2) * lr)) * invd)
                        : rho * (-expm1(static_cast<double>(2 * lo - 2) * lr)) * invd;
  if (NEU) id *= eps * (2.0 - eps) / rho;
  double* m = bc + static_cast<size_t>(kBandModeConsts) * q;
  m[0] = exp(static_cast<double>(nr - 1 + 2 * lo) * lr);
  m[1] = exp(static_cast<double>(nr - 1 + 2 * hb) * lr);
  m[2] = gL;
  m[3] = (NEU ? 1.0 : -1.0) * exp(static_cast<double>(2 * hb) * lr);
  m[4] = id;
  m[5] = invd;
}

template <class T, int E, bool NEU>
__global__ void __launch_bounds__(256)
    k_colsolve_band(int N, double h, int P, const T* __restrict__ Tg,
                    const int* __restrict__ rowpart, const double* __restrict__ colc,
                    const double* __restrict__ bc, int lo, int nr, int jlo, int jhi,
                    T* __restrict__ Gg, int nblk_x, size_t tstride, size_t gstride, int ldr) {
  extern __shared__ double dynp[];
  T* tp = reinterpret_cast<T*>(dynp);
  T (*col)[64 * (E + 1)] = reinterpret_cast<T (*)[64 * (E + 1)]>(dynp);
  const int nmodes = NEU ? N + 1 : N - 1;  // mirror box: cosine modes 0..N; zero box: 1..N-1
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int bid = blockIdx.x;
  const int per_xcd = (nblk_x + 7) / 8;
  const int grp = (bid % 8) * per_xcd + bid / 8;
  if (grp * kColsPerBlock >= nmodes) return;  // whole block beyond the last mode
  Tg += static_cast<size_t>(blockIdx.y) * tstride;
  Gg += static_cast<size_t>(blockIdx.y) * gstride;
  const int q = grp * kColsPerBlock + w;  // this wavefront's mode slot
  const bool live = q < nmodes;
  const int hb = N - (lo + nr - 1);
  // the band conditions' constants (k_band_const): RL = gL P_0 (P_1 / d for the mirror box
  // at lo = 0), RR = gR P_{nr-1} (mirror box at hi = N: (P_{nr-2} - rho P_{nr-1}) / d), and
  // this lane's rho^(lane E) and rho^(nr - 1 - (lane E + E - 1))
  double rho = 0.0, eps = 0.0, id = 0.0, invd = 0.0, cL = 0.0, cR = 0.0, gL = 0.0, gR = 0.0;
  double f0 = 0.0, f1 = 0.0;
  if (live) {
    rho = colc[(NEU ? 4 : 3) * q];
    eps = colc[(NEU ? 4 : 3) * q + 1];
    cL = bc[kBandModeConsts * q];
    cR = bc[kBandModeConsts * q + 1];
    gL = bc[kBandModeConsts * q + 2];
    gR = bc[kBandModeConsts * q + 3];
    id = bc[kBandModeConsts * q + 4];
    invd = bc[kBandModeConsts * q + 5];
    const double* lf = bc + static_cast<size_t>(kBandModeConsts) * nmodes;
    f0 = lf[(static_cast<size_t>(q) * 64 + lane) * 2];
    f1 = lf[(static_cast<size_t>(q) * 64 + lane) * 2 + 1];
  }
  constexpr int R = (64 * E + 255) / 256;  // band rows per thread in the row sums
  int rq0[R], rq1[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = tid + 256 * u;
    const int r = lo + i;
    const bool in = (P > 0) && i < nr && r >= 1 && r <= N - 1;  // arms: interior rows only
    rq0[u] = in ? rowpart[r] : 0;
    rq1[u] = in ? rowpart[r + 1] : 0;
  }
  if (P > 0) {
    const T* src = Tg + static_cast<size_t>(grp) * P * 4;
    constexpr int U = 16;
    for (int e0 = tid; e0 < 4 * P; e0 += 256 * U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 256 * u;
        v[u] = (e < 4 * P) ? src[e] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 256 * u;
        if (e < 4 * P) tp[e] = v[u];
      }
    }
  }
  __syncthreads();
  {
    T a4[R][kColsPerBlock];
#pragma unroll
    for (int u = 0; u < R; ++u) {
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) a4[u][c] = T(0);
      for (int qq = rq0[u]; qq < rq1[u]; ++qq)
#pragma unroll
        for (int c = 0; c < kColsPerBlock; ++c) a4[u][c] += tp[4 * qq + c];
    }
    __syncthreads();  // the part rows are read: their bytes become the columns
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = tid + 256 * u;
      if (i >= 64 * E) continue;
#pragma unroll
      for (int c = 0; c < kColsPerBlock; ++c) col[c][slot0<E>(i)] = a4[u][c];
    }
  }
  __syncthreads();
  if (live) {
    const T rhoT = static_cast<T>(rho), epsT = static_cast<T>(eps);
    const T h2 = static_cast<T>(h * h);
    double pw[E + 1];
    pw[0] = 1.0;
#pragma unroll
    for (int e = 1; e <= E; ++e) pw[e] = pw[e - 1] * rho;
    T y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = h2 * col[w][lane * (E + 1) + e];
    // backward recurrence y_i = b_i + rho y_{i+1} (rows past the band are zero)
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
    // forward recurrence z_i = y_i + rho z_{i-1}
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
    // P_i = -rho z_i; P_0, P_1, P_{nr-2}, P_{nr-1} for the band conditions
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = -rhoT * y[e];
    const int ib = nr - 2, ic = nr - 1;
    T s0 = T(0), s1 = T(0), sb = T(0), sc = T(0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e == 0) s0 = y[e];
      if (e == 1 % E) s1 = y[e];
      if (e == ib % E) sb = y[e];
      if (e == ic % E) sc = y[e];
    }
    const double P0 = static_cast<double>(__shfl(s0, 0, 64));
    const double P1 = static_cast<double>(__shfl(s1, 1 / E, 64));
    const double Pb = static_cast<double>(__shfl(sb, ib / E, 64));
    const double Pc = static_cast<double>(__shfl(sc, ic / E, 64));
    const double RL = gL * ((NEU && lo == 0) ? P1 : P0);
    const double RR = (NEU && hb == 0) ? (Pb - rho * Pc) * invd : gR * Pc;
    const double A = (NEU ? RL + cL * RR : RL - cL * RR) * id;
    const double B = (NEU ? RR + cR * RL : RR - cR * RL) * id;
#pragma unroll
    for (int e = 0; e < E; ++e)
      y[e] += static_cast<T>(A * (f0 * pw[e]) + B * (f1 * pw[E - 1 - e]));
#pragma unroll
    for (int e = 0; e < E; ++e) col[w][lane * (E + 1) + e] = y[e];
  }
  __syncthreads();
  // rows jlo..jhi (band layout: this group's four slots of row r start at base + r rs)
  const int nb = jhi - jlo + 1;
  const size_t base = ldr > 0 ? 4 * static_cast<size_t>(grp) : 4 * static_cast<size_t>(grp) * nb;
  const size_t rs = ldr > 0 ? static_cast<size_t>(ldr) : 4;
  const int q0 = grp * kColsPerBlock;
  for (int e = tid; e < 4 * nb; e += 256) {
    const int r = e >> 2, c = e & 3;
    Gg[base + r * rs + c] = (q0 + c < nmodes) ? col[c][slot0<E>(jlo + r - lo)] : T(0);
  }
}

// ---------------------------------------------------------------------------------- K4
// One block per chunk of MC markers.  Its distinct stencil nodes (sorted by row) are
// split over the wavefronts; lane l of a wavefront keeps G[j][p] for
// p = 1 + l + 64 e and advances sin(p i pi / N) over e by the three-term sine recurrence
// with step 64 i pi / N.  Eight nodes are reduced together by recursive halving.  Then
// MC threads apply the Sec. 4.3 corrected interpolation.
// COSB (zero-normal-derivative box): v_ij = (2/N) sum_{p=0}^{N} w_p G[j][p] cos(p i pi / N)
// with w_0 = w_N = 1/2; lane l keeps the modes p = l + 64 e.
// Recursive-halving reduction of eight per-lane values over the 64 lanes of a wavefront:
// lane l ends with the sum of value (l >> 3) & 7.
template <class T>
__device__ __forceinline__ T batch_reduce8(const T (&part)[kNodeBatch], int lane) {
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  T h4[4], h2[2], h1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T keep = b5 ? part[q + 4] : part[q];
    const T send = b5 ? part[q] : part[q + 4];
    h4[q] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const T keep = b4 ? h4[q + 2] : h4[q];
    const T send = b4 ? h4[q] : h4[q + 2];
    h2[q] = keep + __shfl_xor(send, 16, 64);
  }
  {
    const T keep = b3 ? h2[1] : h2[0];
    const T send = b3 ? h2[0] : h2[1];
    h1 = keep + __shfl_xor(send, 8, 64);
  }
  h1 += __shfl_xor(h1, 4, 64);
  h1 += __shfl_xor(h1, 2, 64);
  h1 += __shfl_xor(h1, 1, 64);
  return h1;
}

template <class T, int E, bool COSB, int NT, bool MS = false>
__global__ void __launch_bounds__(NT)
    k_nodes_extract(int N, int M, int MC, int nch, const int* __restrict__ cnode,
                    const int* __restrict__ ccount, const int* __restrict__ chpos,
                    const int* __restrict__ mkloc,
                    const T* __restrict__ sinT, int jlo, int nbr, const T* __restrict__ G,
                    const double* __restrict__ mq, const double* __restrict__ ext,
                    const double* __restrict__ qpart, int nq, double* __restrict__ vp_out,
                    double* __restrict__ vm_out, double* __restrict__ dnp_out,
                    double* __restrict__ dnm_out, int side, double oa, double ob, double oq,
                    const double* __restrict__ xop, double* __restrict__ yop, size_t gstride,
                    const double* __restrict__ amk, int ldr) {
  extern __shared__ double nval[];  // 6 * MC node values
  {  // density blockIdx.y of a batch
    const size_t bd = blockIdx.y;
    G += bd * gstride;
    mq += bd * 5 * M;
    qpart += bd * nq;
    if (vp_out) vp_out += bd * M;
    if (vm_out) vm_out += bd * M;
    if (dnp_out) dnp_out += bd * M;
    if (dnm_out) dnm_out += bd * M;
  }
  __shared__ double red[16];
  __shared__ T tab[sintab2_size<T>(4096)];
  const int n = N - 1;
  const int mask = 2 * N - 1;
  const int quarter = N / 2;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // XCD-aware order: blocks resident on one XCD (ids congruent mod 8) take consecutive
  // positions of the chunk list, which the interface setup orders by grid row,
  // so an XCD's chunks share grid rows and those rows are fetched into its L2 once
  const int per_xcd = gridDim.x / 8;  // the grid is 8 per_xcd blocks
  const int bx = blockIdx.x;
  const int pos = (bx % 8) * per_xcd + bx / 8;
  if (pos >= nch) return;
  const int ch = chpos[pos];  // the marker chunk at this position
  const int nn = ccount[pos];
  const int* keys = cnode + static_cast<size_t>(pos) * 6 * MC;
  // the chunk's node keys (at most 6 MC <= 128), two per lane, loaded with the table
  const int key_lo = (lane < 6 * MC) ? keys[lane] : -1;
  const int key_hi = (64 + lane < 6 * MC) ? keys[64 + lane] : -1;
  SinTab2<T> st2;
  st2.stage(tab, N, sinT);
  __syncthreads();
  // prefetch the extraction data of this thread's marker (used after the node phase): in
  // the registers of thread m < MC, except the weights of the FP64 rows of more than 32
  // mode slots per lane, which the block stages in LDS (their registers would otherwise
  // keep the kernel at four wavefronts)
  constexpr bool kStageX = node_stage_ext<T, E>();
  const int kx = ch * MC + tid;
  const bool xmk = (tid < MC && kx < M);
  int loc[6];
  double Q[5], xw[kExtCount - 1];
  __shared__ double xs[kStageX ? (kExtCount - 1) * kMaxChunk : 1];
  if (xmk) {
#pragma unroll
    for (int m = 0; m < 6; ++m) loc[m] = mkloc[6 * kx + m];
#pragma unroll
    for (int q = 0; q < 5; ++q) Q[q] = mq[q * M + kx];
    if constexpr (!kStageX) {
#pragma unroll
      for (int q = 0; q < kExtCount - 1; ++q) xw[q] = ext[q * M + kx];
    }
  }
  if constexpr (kStageX) {
    for (int e = tid; e < (kExtCount - 1) * MC; e += NT) {
      const int q = e / MC, m = e - q * MC, km = ch * MC + m;
      if (km < M) xs[q * MC + m] = ext[q * M + km];
    }
  }
  double qs = 0.0;
  if (yop && oq != 0.0) {
    double s = 0.0;
    for (int i = tid; i < nq; i += NT) s += qpart[i];
    qs = block_sum<double>(s, red);
  }
  // distance between groups of four mode slots: 4 in a row-major band, 4 nbr in the
  // column-group layout
  const size_t g_grp = ldr > 0 ? 4 : 4 * static_cast<size_t>(nbr);
  const size_t g_lane = static_cast<size_t>(lane >> 2) * g_grp + (lane & 3);
  const size_t g_step = 16 * g_grp;
  constexpr int NWV = NT / 64;
  if constexpr (MS) {
    // chunks of one marker (at most six nodes): wavefront w takes the mode slots
    // e = w EW .. w EW + EW - 1 of every node, so the block reads each distinct node row
    // once (each wavefront its slice) instead of once per node; a node's NWV partial sums
    // are then added in wavefront order
    constexpr int EW = (E + NWV - 1) / NWV;
    __shared__ T wsum[NWV][kNodeBatch];
    const int e0 = w * EW;
    int curj = -1;
    T gv[EW];
#pragma unroll
    for (int e = 0; e < EW; ++e) gv[e] = T(0);
    T part[kNodeBatch];
#pragma unroll
    for (int u = 0; u < kNodeBatch; ++u) {
      const int kq = __shfl(key_lo, u, 64);
      const int key = (u < nn) ? kq : -1;
      const int i = key & 0xffff, j = key >> 16;
      if (key >= 0 && j != curj) {  // wave-uniform branch
        const T* Gr = G + (ldr > 0 ? static_cast<size_t>(j - jlo) * ldr
                                   : 4 * static_cast<size_t>(j - jlo)) + g_lane;
#pragma unroll
        for (int e = 0; e < EW; ++e) {
          const int ee = e0 + e;
          if constexpr (COSB) {
            const int pp = lane + 64 * ee;
            const T wgt = (pp == 0 || pp == N) ? T(0.5) : T(1);
            gv[e] = (ee < E && pp <= N) ? wgt * Gr[static_cast<size_t>(ee) * g_step] : T(0);
          } else {
            const int pp = 1 + lane + 64 * ee;
            gv[e] = (ee < E && pp <= n) ? Gr[static_cast<size_t>(ee) * g_step] : T(0);
          }
        }
        curj = j;
      }
      T sacc = T(0);
      if (key >= 0 && e0 < E) {
        T a, c, sb, cb;
        st2.get((((COSB ? 0 : 1) + lane + 64 * e0) * i) & mask, a, c);
        st2.get((64 * i) & mask, sb, cb);
        const T c2 = cb + cb;
        T am;
        if constexpr (COSB) {
          am = c * cb + a * sb;
          a = c;
        } else {
          am = a * cb - c * sb;
        }
        sacc += gv[0] * a;
#pragma unroll
        for (int e = 1; e < EW; ++e) {
          const T an = c2 * a - am;
          am = a;
          a = an;
          sacc += gv[e] * a;
        }
      }
      part[u] = sacc;
    }
    const T h1 = batch_reduce8<T>(part, lane);
    if ((lane & 7) == 0) wsum[w][(lane >> 3) & 7] = h1;
    __syncthreads();
    if (tid < nn) {
      double sum = 0.0;
#pragma unroll
      for (int ww = 0; ww < NWV; ++ww) sum += static_cast<double>(wsum[ww][tid]);
      nval[tid] = sum * (2.0 / N);
    }
  } else {
    // this wavefront's nodes (contiguous in the sorted list, so rows repeat)
    const int per = (nn + NWV - 1) / NWV;
    const int qb = w * per, qe = min(nn, qb + per);
    int curj = -1;
    T gv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) gv[e] = T(0);
    for (int q0 = qb; q0 < qe; q0 += kNodeBatch) {
      T part[kNodeBatch];
#pragma unroll
      for (int u = 0; u < kNodeBatch; ++u) {
        const int q = q0 + u;
        const int kq = __shfl(q < 64 ? key_lo : key_hi, q & 63, 64);
        const int key = (q < qe) ? kq : -1;
        const int i = key & 0xffff, j = key >> 16;
        if (key >= 0 && j != curj) {  // wave-uniform branch
          // mode slot lane + 64 e of row j: one base per lane, a fixed step per e
          // (band layout with q >> 2 = (lane >> 2) + 16 e and q & 3 = lane & 3)
          const T* Gr = G + (ldr > 0 ? static_cast<size_t>(j - jlo) * ldr
                                     : 4 * static_cast<size_t>(j - jlo)) + g_lane;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if constexpr (COSB) {
              const int pp = lane + 64 * e;
              const T wgt = (pp == 0 || pp == N) ? T(0.5) : T(1);
              gv[e] = (pp <= N) ? wgt * Gr[e * g_step] : T(0);
            } else {
              const int pp = 1 + lane + 64 * e;
              gv[e] = (pp <= n) ? Gr[e * g_step] : T(0);
            }
          }
          curj = j;
        }
        T sacc = T(0);
        if (key >= 0) {
          T a, c, sb, cb;
          st2.get((((COSB ? 0 : 1) + lane) * i) & mask, a, c);
          st2.get((64 * i) & mask, sb, cb);
          // three-term recurrence in steps of 64 i pi / N (rounding grows at most E-fold)
          const T c2 = cb + cb;
          T am;
          if constexpr (COSB) {
            am = c * cb + a * sb;  // cos((p - 64) x)
            a = c;
          } else {
            am = a * cb - c * sb;
          }
          sacc += gv[0] * a;
#pragma unroll
          for (int e = 1; e < E; ++e) {
            const T an = c2 * a - am;
            am = a;
            a = an;
            sacc += gv[e] * a;
          }
        }
        part[u] = sacc;
      }
      const T h1 = batch_reduce8<T>(part, lane);
      const int u = (lane >> 3) & 7;
      if ((lane & 7) == 0 && q0 + u < qe) nval[q0 + u] = static_cast<double>(h1) * (2.0 / N);
    }
  }
  __syncthreads();
  if (!xmk) return;
  const int k = kx;
  if constexpr (kStageX) {
#pragma unroll
    for (int q = 0; q < kExtCount - 1; ++q) xw[q] = xs[q * MC + tid];
  }
  double v[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) v[m] = nval[loc[m]];
  double out[3], jm[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double s = 0.0, t = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) s += xw[kExtW + 6 * r + m] * v[m];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      s += xw[kExtE + 5 * r + q] * Q[q];
      t += xw[kExtD + 5 * r + q] * Q[q];
    }
    out[r] = s;
    jm[r] = t;
  }
  const double nx = xw[kExtN], ny = xw[kExtN + 1];
  const double vp = out[0], vm = out[0] - jm[0];
  const double dnp = nx * out[1] + ny * out[2];
  const double dnm = nx * (out[1] - jm[1]) + ny * (out[2] - jm[2]);
  if (vp_out) vp_out[k] = vp;
  if (vm_out) vm_out[k] = vm;
  if (dnp_out) dnp_out[k] = dnp;
  if (dnm_out) dnm_out[k] = dnm;
  if (yop) {
    const double tr = (side == KFBI_PLUS) ? vp : (side == KFBI_MINUS ? vm : 0.5 * (vp + vm));
    yop[k] = (amk ? amk[k] : oa) * xop[k] + ob * tr + oq * qs;
  }
}

// -------------------------------------------------------------------- full-grid evaluation
// grid[j][i] = (2/N) sum_p G[j-1][p-1] sin(p i pi / N) on the interior, 64x64 output tiles,
// 4x4 per thread.  COSB: grid[j][i] = (2/N) sum_{p=0}^{N} w_p G[j][p] cos(p i pi / N) on all
// nodes (w_0 = w_N = 1/2).
template <class T, bool COSB>
__global__ void __launch_bounds__(256)
    k_fullgrid(int N, const T* __restrict__ G, int ldG, const T* __restrict__ sinT,
               double* __restrict__ grid) {
  __shared__ T As[16][65];
  __shared__ T Bs[16][65];
  const int n = COSB ? N + 1 : N - 1;  // modes and output rows/columns
  const int off = COSB ? 0 : 1;       // index of the first row/column/mode
  const int mask = 2 * N - 1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  T acc[4][4] = {};
  for (int k0 = 0; k0 < n; k0 += 16) {
    for (int t = threadIdx.x; t < 16 * 64; t += 256) {
      const int kk = t & 15, rr = t >> 4;
      const int jr = j0 + rr, kp = k0 + kk;
      T a = (jr < n && kp < n) ? G[grp_index(kp + 1, jr, ldG)] : T(0);
      if (COSB && (kp == 0 || kp == N)) a *= T(0.5);
      As[kk][rr] = a;
      const int ic = i0 + rr;
      const int arg = (kp + off) * (ic + off) + (COSB ? N / 2 : 0);  // cos x = sin(x + pi/2)
      Bs[kk][rr] = (ic < n && kp < n) ? sinT[arg & mask] : T(0);
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
        grid[static_cast<size_t>(jr + off) * (N + 1) + (ic + off)] =
            sc * static_cast<double>(acc[r][q]);
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

static inline int nblk(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

// Dynamic LDS elements of a column-solve block: the P part rows of its group (4 modes
// each), later overwritten by its four columns of 64 (E + 1) rows.
static inline size_t colsolve_lds_elems(int P, int E) {
  const size_t parts = 4 * static_cast<size_t>(P > 0 ? P : 1);
  const size_t cols = static_cast<size_t>(kColsPerBlock) * 64 * (E + 1);
  return parts > cols ? parts : cols;
}

template <class K>
static const void* kptr(K kernel) {
  return reinterpret_cast<const void*>(kernel);
}

// Rows per lane of the band column solve: E >= ceil(nr / 64) from a short list.
static int band_rows_per_lane(int nr) {
  const int e = (nr + 63) / 64;
  return e <= 2 ? 2 : e <= 4 ? 4 : e <= 8 ? 8 : e <= 12 ? 12 : e <= 16 ? 16 : e <= 24 ? 24 : 33;
}
template <class F>
static void band_dispatch(int nr, F&& f) {
  const int e = (nr + 63) / 64;
  if (e <= 2) f(std::integral_constant<int, 2>{});
  else if (e <= 4) f(std::integral_constant<int, 4>{});
  else if (e <= 8) f(std::integral_constant<int, 8>{});
  else if (e <= 12) f(std::integral_constant<int, 12>{});
  else if (e <= 16) f(std::integral_constant<int, 16>{});
  else if (e <= 24) f(std::integral_constant<int, 24>{});
  else f(std::integral_constant<int, 33>{});
}

// The band of rows lo .. lo + nr - 1 that holds every arm row and every node row (at least
// two rows, inside the rows of the box condition); false when the interface has neither, or
// when the band needs as many rows per lane as the whole column.
static bool solve_band(const kfbi_ctx* c, bool neu, int* lo, int* nr) {
  const int N = c->N;
  const GeoStatus& g = c->st;
  if (g.row_lo > g.row_hi) return false;
  int a = g.row_lo, b = g.row_hi;
  if (g.arm_lo <= g.arm_hi) {
    a = std::min(a, g.arm_lo);
    b = std::max(b, g.arm_hi);
  }
  const int rmin = neu ? 0 : 1, rmax = neu ? N : N - 1;
  if (g.row_lo < rmin || g.row_hi > rmax) return false;  // output rows must lie in the band
  a = std::max(a, rmin);
  b = std::min(b, rmax);
  if (b - a + 1 < 2) {
    if (b < rmax) b = a + 1;
    else a = b - 1;
  }
  if (a < rmin || b > rmax || a > b) return false;
  // nothing to gain unless the band needs fewer rows per lane than the whole column
  const int rows = rmax - rmin + 1, ef = (rows + 63) / 64;
  const int efull = neu ? (ef <= 2 ? 2 : ef <= 3 ? 3 : ef <= 5 ? 5 : ef <= 9 ? 9 : ef <= 17 ? 17 : 33)
                        : (ef <= 1 ? 1 : ef <= 2 ? 2 : ef <= 4 ? 4 : ef <= 8 ? 8 : ef <= 16 ? 16 : 32);
  if (band_rows_per_lane(b - a + 1) >= efull) return false;
  *lo = a;
  *nr = b - a + 1;
  return true;
}

// The band solve's constants for (lo, nr, E), formed when the band differs from the one
// bandc holds (once per interface, not per apply).
template <bool NEU>
static void band_constants(kfbi_ctx* c, int lo, int nr, int E) {
  if (c->bc_nr == nr && c->bc_lo == lo && c->bc_E == E) return;
  const int nmodes = NEU ? c->N + 1 : c->N - 1;
  hipLaunchKernelGGL((k_band_const<NEU>), dim3(nblk(64LL * nmodes, 256)), dim3(256), 0, c->stream,
                     c->N, lo, nr, E, c->colc.as<double>(), c->bandc.as<double>());
  c->bc_lo = lo;
  c->bc_nr = nr;
  c->bc_E = E;
}

template <class T, int E>
static void launch_grid_stages(kfbi_ctx* c, int B, const T* sinT, const T* ring, size_t rstride,
                               int jlo, int jhi, T* Tg, T* G, bool full, double* grid,
                               hipEvent_t* ev, const kfbi_out* out, const kfbi_bie* op,
                               const double* xop, double* yop, int stages) {
  const int N = c->N, n = N - 1, M = c->M;
  const int P = c->st.n_parts;
  hipStream_t s = c->stream;
  constexpr int PT = (64 * E + 255) / 256;
  const size_t tstride = 4 * static_cast<size_t>((n + 3) / 4) * (P + 1);
  const size_t gstride = static_cast<size_t>(n) * N;
  // band rows row-major (row stride: the modes rounded up to whole groups of four, so a
  // band fits where the column-group one did); the full grid keeps the column groups
  const int ldr = full ? 0 : 4 * ((n + 3) / 4);
  if (P > 0 && (stages & 2))
    hipLaunchKernelGGL((k_rowdst<T, PT, false>), dim3(8 * nblk(P, 8), B), dim3(256), 0, s, N, P, c->pdesc.as<int4>(),
                       c->armr.as<double>(), c->armk.as<int>() + c->arm_cap,
                       c->armsc.as<double>(), sinT, Tg, tstride);
  if (ev) hipEventRecord(ev[2], s);
  const int ngrp = nblk(n, kColsPerBlock);
  const int nb = ((ngrp + 7) / 8) * 8;
  int blo = 0, bnr = 0;
  if ((stages & 4) && !full && !ring && solve_band(c, false, &blo, &bnr)) {
    // zero box: the right-hand side lives on the arm rows only
    band_dispatch(bnr, [&](auto EC) {
      constexpr int EB = decltype(EC)::value;
      band_constants<false>(c, blo, bnr, EB);
      hipLaunchKernelGGL((k_colsolve_band<T, EB, false>), dim3(nb, B), dim3(256),
                         sizeof(T) * colsolve_lds_elems(P, EB), s, N, c->h, P, Tg,
                         c->rowpart.as<int>(), c->colc.as<double>(), c->bandc.as<double>(), blo,
                         bnr, jlo, jhi, G, nb, tstride, gstride, ldr);
    });
  } else if (stages & 4) {
    const size_t lds_dyn = sizeof(T) * colsolve_lds_elems(P, E);
    hipLaunchKernelGGL((k_colsolve<T, E>), dim3(nb, B), dim3(256), lds_dyn, s, N, c->h, P, Tg,
                       c->rowpart.as<int>(), sinT, ring, c->colc.as<double>(),
                       c->lanef.as<double>(), jlo, jhi, G, nb, tstride, rstride, gstride, ldr);
  }
  if (ev) hipEventRecord(ev[3], s);
  const int nbr = jhi - jlo + 1;
  if (full) {  // single density only
    hipLaunchKernelGGL((k_fullgrid<T, false>), dim3(nblk(n, 64), nblk(n, 64)), dim3(256), 0, s, N,
                       G, nbr, sinT, grid);
    hipLaunchKernelGGL((k_grid_ring<T>), dim3(nblk(N + 1, 256)), dim3(256), 0, s, N, ring, grid);
  }
  const int MC = c->mk_chunk;
  const int nch = nblk(M, MC);
  const int side = op ? op->side : 0;
  const double oa = op ? op->a : 0.0, ob = op ? op->b : 0.0, oq = op ? op->q : 0.0;
  if (stages & 8) {
    constexpr int NT1 = node_threads<T, E>();
    auto kn = (B == 1) ? k_nodes_extract<T, E, false, NT1> : k_nodes_extract<T, E, false, 256>;
    if constexpr (E >= kModeSplitMinE)
      if (B == 1 && MC == 1) kn = k_nodes_extract<T, E, false, 512, true>;
    hipLaunchKernelGGL(kn, dim3(8 * nblk(nch, 8), B), dim3(B == 1 ? NT1 : 256),
                       sizeof(double) * 6 * MC, s, N, M, MC, nch, c->cnode.as<int>(),
                       c->ccount.as<int>(), c->chpos.as<int>(), c->mkloc.as<int>(), sinT, jlo, nbr, G,
                       c->mq.as<double>(), c->ext.as<double>(), c->qpart.as<double>(),
                       c->n_mk_blocks, out ? out->v_plus : nullptr,
                       out ? out->v_minus : nullptr, out ? out->dn_plus : nullptr,
                       out ? out->dn_minus : nullptr, side, oa, ob, oq, xop, yop, gstride,
                       op ? op->a_marker : nullptr, ldr);
  }
}

// Grid stages of the zero-normal-derivative box: cosine row transform of the arm parts
// (when `parts`), the mirrored-ghost column solve with optional dense right-hand sides
// ca Fa + cb Fb (column-group layout, all N+1 rows), rows jlo..jhi of G, then the node
// evaluation and extraction with the marker quantities mqv.
struct NeuRhs {
  const void* Fa = nullptr;
  const void* Fb = nullptr;
  double ca = 0.0, cb = 0.0;
  bool parts = true;
};

template <class T, int E>
static void launch_grid_stages_neu(kfbi_ctx* c, int B, const T* sinT, int jlo, int jhi, T* Tg,
                                   T* G, bool full, double* grid, hipEvent_t* ev,
                                   const kfbi_out* out, const kfbi_bie* op, const double* xop,
                                   double* yop, int stages, const NeuRhs& rr,
                                   const double* mqv, int ldr) {
  const int N = c->N, M = c->M, nm = N + 1;
  const int P = rr.parts ? c->st.n_parts : 0;
  hipStream_t s = c->stream;
  constexpr int PT = (64 * E + 255) / 256;
  const int ngm = nblk(nm, 4);
  const size_t tstride = 4 * static_cast<size_t>(ngm) * (c->st.n_parts + 1);
  const size_t gstride = 4 * static_cast<size_t>(ngm) * nm;
  if (P > 0 && (stages & 2))
    hipLaunchKernelGGL((k_rowdst<T, PT, true>), dim3(8 * nblk(P, 8), B), dim3(256), 0, s, N, P,
                       c->pdesc.as<int4>(), c->armr.as<double>(),
                       c->armk.as<int>() + c->arm_cap, c->armsc.as<double>(), sinT, Tg,
                       tstride);
  if (ev) hipEventRecord(ev[2], s);
  const int nb = ((ngm + 7) / 8) * 8;
  int blo = 0, bnr = 0;
  if ((stages & 4) && !full && !rr.Fa && solve_band(c, true, &blo, &bnr)) {
    // no dense right-hand side: the arm rows carry all of it
    band_dispatch(bnr, [&](auto EC) {
      constexpr int EB = decltype(EC)::value;
      band_constants<true>(c, blo, bnr, EB);
      hipLaunchKernelGGL((k_colsolve_band<T, EB, true>), dim3(nb, B), dim3(256),
                         sizeof(T) * colsolve_lds_elems(P, EB), s, N, c->h, P, Tg,
                         c->rowpart.as<int>(), c->colc.as<double>(), c->bandc.as<double>(), blo,
                         bnr, jlo, jhi, G, nb, tstride, gstride, ldr);
    });
  } else if (stages & 4) {
    const size_t lds_dyn = sizeof(T) * colsolve_lds_elems(P, E);
    hipLaunchKernelGGL((k_colsolve_neu<T, E>), dim3(nb, B), dim3(256), lds_dyn, s, N, c->h, P,
                       Tg, c->rowpart.as<int>(), static_cast<const T*>(rr.Fa),
                       static_cast<const T*>(rr.Fb), rr.ca, rr.cb, c->colc.as<double>(),
                       c->lanef.as<double>(), jlo, jhi, G, nb, tstride, gstride, ldr);
  }
  if (ev) hipEventRecord(ev[3], s);
  const int nbr = jhi - jlo + 1;
  if (full)  // single density, all rows
    hipLaunchKernelGGL((k_fullgrid<T, true>), dim3(nblk(nm, 64), nblk(nm, 64)), dim3(256), 0, s,
                       N, G, nbr, sinT, grid);
  const int MC = c->mk_chunk;
  const int nch = nblk(M, MC);
  const int side = op ? op->side : 0;
  const double oa = op ? op->a : 0.0, ob = op ? op->b : 0.0, oq = op ? op->q : 0.0;
  if (stages & 8) {
    constexpr int NT1 = node_threads<T, E>();
    auto kn = (B == 1) ? k_nodes_extract<T, E, true, NT1> : k_nodes_extract<T, E, true, 256>;
    if constexpr (E >= kModeSplitMinE)
      if (B == 1 && MC == 1) kn = k_nodes_extract<T, E, true, 512, true>;
    hipLaunchKernelGGL(kn, dim3(8 * nblk(nch, 8), B), dim3(B == 1 ? NT1 : 256),
                       sizeof(double) * 6 * MC, s, N, M, MC, nch, c->cnode.as<int>(),
                       c->ccount.as<int>(), c->chpos.as<int>(), c->mkloc.as<int>(), sinT, jlo, nbr, G, mqv,
                       c->ext.as<double>(), c->qpart.as<double>(), c->n_mk_blocks,
                       out ? out->v_plus : nullptr, out ? out->v_minus : nullptr,
                       out ? out->dn_plus : nullptr, out ? out->dn_minus : nullptr, side, oa, ob,
                       oq, xop, yop, gstride, op ? op->a_marker : nullptr, ldr);
  }
}

// Dispatch on E = ceil((N+1)/64) for N = 64 .. 2048.
template <class T, class F>
static void neu_dispatch(int N, F&& f) {
  switch ((N + 1 + 63) / 64) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 17: f(std::integral_constant<int, 17>{}); break;
    default: f(std::integral_constant<int, 33>{}); break;
  }
}

// FP32 copies of user box values for a batch: src [B][4(N+1)] -> dst with stride dstride.
__global__ void k_ring_cast_b(int n4, int B, const double* __restrict__ src, float* __restrict__ dst,
                              size_t dstride) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n4 * B) return;
  const int b = t / n4, r = t % n4;
  dst[b * dstride + r] = static_cast<float>(src[t]);
}

// Launches the selected kernels (bit s = stage s) of one apply of B densities (B = 1 for
// the single apply and the operator).
template <class T>
static int apply_t(kfbi_ctx* c, int B, int layer, const double* dens, const double* ring_user,
                   const kfbi_out* out, const kfbi_bie* op, const double* xop, double* yop,
                   int stages = 15) {
  const int M = c->M, N = c->N;
  hipStream_t s = c->stream;
  const bool full = out && out->grid;
  const T* sinT = reinterpret_cast<const T*>(sizeof(T) == 8 ? c->sinT.p : c->sinT32.p);
  T* Tg = reinterpret_cast<T*>(c->tmat.p);
  T* G = reinterpret_cast<T*>(c->gband.p);
  double* ring64 = c->ring.as<double>();
  T* ringT = nullptr;  // box data in the working precision
  size_t rstride = 0;  // its stride between densities, in T elements
  int nring = 0;
  hipEvent_t* ev = nullptr;
  if (c->prof_on && stages == 15) {
    if (c->prof_used + 5 > kfbi_ctx::kProfPool) KFBI_TRY(prof_flush(c));
    ev = c->prof_ev + c->prof_used;
    c->prof_used += 5;
    hipEventRecord(ev[0], s);
  }
  if (c->box_bc == KFBI_BOX_FREESPACE) nring = nblk(4 * (N + 1), kRingNodes);
  // box data per density: 8(N+1) doubles, the FP64 values then (FP32 applies) a float copy
  float* ring32 = reinterpret_cast<float*>(ring64 + 4 * (N + 1));
  const int C = c->mk_chunk, nmk = c->n_mk_blocks;
  const int nd = (layer == KFBI_DOUBLE) ? 2 : 1;
  // marker blocks: the density, d1 (and d2) or the partial sums, the window sums (also the
  // block_sum scratch) and the window quantities; ring blocks: four chunks of 256 markers
  const size_t lds_mk = static_cast<size_t>((lpad(M - 1) + 1) + kprep_region(M, nd) +
                                            16 * kReg + 5 * kWinMax);
  // ring blocks: four arrays of min(M, kRingChunk) markers
  const size_t lds_ring = nring > 0 ? 4 * static_cast<size_t>(M < kRingChunk ? M : kRingChunk) : 0;
  const size_t lds = sizeof(double) * (lds_mk > lds_ring ? lds_mk : lds_ring);
  if (stages & 1)
    hipLaunchKernelGGL(k_prep, dim3(nmk + nring, B), dim3(256), lds, s, M, C, nmk, layer, dens,
                       c->dvec.as<double>(), c->dvec.as<double>() + M, c->mq.as<double>(),
                       c->qpart.as<double>(),
                       (op && op->q != 0.0) ? c->ext.as<double>() + kExtQ * M : nullptr, N,
                       c->x0, c->y0,
                       c->h, c->X.as<double>(), c->geo.as<double>(), ring64,
                       sizeof(T) == 4 ? ring32 : nullptr, c->ckoff.as<int>(),
                       c->cklist.as<int>(), c->ckcoef.as<double>(), c->ckmk.as<int>(),
                       c->arm_cap, c->armr.as<double>(), sizeof(T) == 4 ? 1 : 0);
  if (c->box_bc == KFBI_BOX_FREESPACE) {
    ringT = sizeof(T) == 8 ? reinterpret_cast<T*>(ring64) : reinterpret_cast<T*>(ring32);
    rstride = sizeof(T) == 8 ? 8 * static_cast<size_t>(N + 1) : 16 * static_cast<size_t>(N + 1);
  } else if (c->box_bc == KFBI_BOX_USER) {
    if (sizeof(T) == 8) {
      ringT = const_cast<T*>(reinterpret_cast<const T*>(ring_user));
      rstride = 4 * static_cast<size_t>(N + 1);
    } else {
      ringT = reinterpret_cast<T*>(ring32);
      rstride = 16 * static_cast<size_t>(N + 1);
      if ((stages & 1) && ring_user)
        hipLaunchKernelGGL(k_ring_cast_b, dim3(nblk(4LL * (N + 1) * B, 256)), dim3(256), 0, s,
                           4 * (N + 1), B, ring_user, ring32, rstride);
    }
  }
  if (ev) hipEventRecord(ev[1], s);
  double* grid = full ? out->grid : nullptr;
  if (c->box_bc == KFBI_BOX_NEUMANN) {
    const int jlo = full ? 0 : c->st.row_lo;
    const int jhi = full ? N : c->st.row_hi;
    const NeuRhs rr;
    neu_dispatch<T>(N, [&](auto EC) {
      // band rows row-major (stride: the N + 1 modes rounded up to whole groups of four);
      // the full grid keeps the column groups
      launch_grid_stages_neu<T, decltype(EC)::value>(
          c, B, sinT, jlo, jhi, Tg, G, full, grid, ev, out, op, xop, yop, stages, rr,
          c->mq.as<double>(), full ? 0 : 4 * ((N + 4) / 4));
    });
    if (ev) hipEventRecord(ev[4], s);
    KFBI_HIP(hipGetLastError());
    c->last_layer = layer;
    c->last_precision = sizeof(T) == 8 ? KFBI_FP64 : KFBI_FP32;
    c->last_batch = B;
    return KFBI_OK;
  }
  const int jlo = full ? 1 : c->st.row_lo;
  const int jhi = full ? N - 1 : c->st.row_hi;
  const int E = (N - 1 + 63) / 64;
  switch (E <= 1 ? 1 : E <= 2 ? 2 : E <= 4 ? 4 : E <= 8 ? 8 : E <= 16 ? 16 : 32) {
#define KFBI_CASE(EE)                                                                         \
  case EE:                                                                                    \
    launch_grid_stages<T, EE>(c, B, sinT, ringT, rstride, jlo, jhi, Tg, G, full, grid, ev, out, \
                              op, xop, yop, stages);                                          \
    break;
    KFBI_CASE(1)
    KFBI_CASE(2)
    KFBI_CASE(4)
    KFBI_CASE(8)
    KFBI_CASE(16)
    default:
      launch_grid_stages<T, 32>(c, B, sinT, ringT, rstride, jlo, jhi, Tg, G, full, grid, ev, out,
                                op, xop, yop, stages);
      break;
#undef KFBI_CASE
  }
  if (ev) hipEventRecord(ev[4], s);
  KFBI_HIP(hipGetLastError());
  c->last_layer = layer;
  c->last_precision = sizeof(T) == 8 ? KFBI_FP64 : KFBI_FP32;
  c->last_batch = B;
  return KFBI_OK;
}

// ------------------------------------------------- zero-normal-derivative box: full fields
// Forward cosine transform of grid rows into the column-group layout,
//   Ghat[j][p] = sum_{i=0}^{N} w_i grid[j][i] cos(p i pi / N),  w_0 = w_N = 1/2,
// as a tiled product with the cosine matrix (64x64 output tiles, 4x4 per thread).
__global__ void __launch_bounds__(256)
    k_rows_dct(int N, const double* __restrict__ grid, const double* __restrict__ sinT,
               double* __restrict__ G) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int nm = N + 1;
  const int mask = 2 * N - 1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int p0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < nm; k0 += 16) {
    for (int t = threadIdx.x; t < 16 * 64; t += 256) {
      const int kk = t & 15, rr = t >> 4;
      const int jr = j0 + rr, i = k0 + kk;
      double a = (jr < nm && i < nm) ? grid[static_cast<size_t>(jr) * nm + i] : 0.0;
      if (i == 0 || i == N) a *= 0.5;
      As[kk][rr] = a;
      const int pc = p0 + rr;
      Bs[kk][rr] = (pc < nm && i < nm) ? sinT[(i * pc + N / 2) & mask] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], bv[4];
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
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jr = j0 + ty * 4 + r, pc = p0 + tx * 4 + q;
      if (jr < nm && pc < nm) G[grp_index(pc + 1, jr, nm)] = acc[r][q];
    }
}

// Full-field operations of the zero-normal-derivative box (FP64, one density).  A field
// "Ghat" holds, for every row j = 0..N, the cosine coefficients along x in the column-group
// layout: element (j, p) at ((p / 4) (N + 1) + j) 4 + p % 4.
int neu_dense_solve(kfbi_ctx* c, const double* Fa, const double* Fb, double ca, double cb,
                    double* Gout, int jlo, int jhi) {
  const int N = c->N;
  NeuRhs rr;
  rr.Fa = Fa;
  rr.Fb = Fb;
  rr.ca = ca;
  rr.cb = cb;
  rr.parts = false;
  const double* sinT = c->sinT.as<double>();
  neu_dispatch<double>(N, [&](auto EC) {
    launch_grid_stages_neu<double, decltype(EC)::value>(
        c, 1, sinT, jlo, jhi, c->tmat.as<double>(), Gout, false, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, 4, rr, c->mq.as<double>(), 0);
  });
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int neu_interp(kfbi_ctx* c, const double* G, int jlo, int jhi, double* vout) {
  const int N = c->N;
  const NeuRhs rr;
  const double* sinT = c->sinT.as<double>();
  kfbi_out o{vout, nullptr, nullptr, nullptr, nullptr};
  neu_dispatch<double>(N, [&](auto EC) {
    launch_grid_stages_neu<double, decltype(EC)::value>(
        c, 1, sinT, jlo, jhi, c->tmat.as<double>(), const_cast<double*>(G), false, nullptr,
        nullptr, &o, nullptr, nullptr, nullptr, 8, rr, c->mqz.as<double>(), 0);
  });
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int neu_apply_full(kfbi_ctx* c, int layer, const double* dens, const double* Fa,
                   const double* Fb, double ca, double cb, double* Gout) {
  const int N = c->N;
  KFBI_TRY(apply_t<double>(c, 1, layer, dens, nullptr, nullptr, nullptr, nullptr, nullptr, 1));
  NeuRhs rr;
  rr.Fa = Fa;
  rr.Fb = Fb;
  rr.ca = ca;
  rr.cb = cb;
  const double* sinT = c->sinT.as<double>();
  neu_dispatch<double>(N, [&](auto EC) {
    launch_grid_stages_neu<double, decltype(EC)::value>(
        c, 1, sinT, 0, N, c->tmat.as<double>(), Gout, false, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, 2 | 4, rr, c->mq.as<double>(), 0);
  });
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int neu_to_grid(kfbi_ctx* c, const double* Gfull, double* grid) {
  const int N = c->N, nm = N + 1;
  hipLaunchKernelGGL((k_fullgrid<double, true>), dim3(nblk(nm, 64), nblk(nm, 64)), dim3(256), 0,
                     c->stream, N, Gfull, nm, c->sinT.as<double>(), grid);
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int neu_from_grid(kfbi_ctx* c, const double* grid, double* Gfull) {
  const int N = c->N, nm = N + 1;
  // padding modes of the last group stay zero
  KFBI_HIP(hipMemsetAsync(Gfull, 0, sizeof(double) * neu_field_size(N), c->stream));
  hipLaunchKernelGGL(k_rows_dct, dim3(nblk(nm, 64), nblk(nm, 64)), dim3(256), 0, c->stream, N,
                     grid, c->sinT.as<double>(), Gfull);
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

int colconst_setup(kfbi_ctx* c) {
  const int N = c->N, n = N - 1;
  if (c->box_bc == KFBI_BOX_NEUMANN) {
    const int nm = N + 1, E = (nm + 63) / 64;
    KFBI_TRY(c->colc.ensure(sizeof(double) * 4 * nm));
    KFBI_TRY(c->lanef.ensure(sizeof(double) * 2 * 64 * nm));
    KFBI_TRY(c->bandc.ensure(sizeof(double) * (kBandModeConsts + 2 * 64) * nm));
    c->bc_nr = 0;
    hipLaunchKernelGGL(k_colconst_neu, dim3(nblk(64 * nm, 256)), dim3(256), 0, c->stream, N,
                       c->h * c->h * c->c2, E, c->colc.as<double>(), c->lanef.as<double>());
    KFBI_HIP(hipGetLastError());
    return KFBI_OK;
  }
  const int E0 = (n + 63) / 64;
  const int E = E0 <= 1 ? 1 : E0 <= 2 ? 2 : E0 <= 4 ? 4 : E0 <= 8 ? 8 : E0 <= 16 ? 16 : 32;
  KFBI_TRY(c->colc.ensure(sizeof(double) * 3 * n));
  KFBI_TRY(c->lanef.ensure(sizeof(double) * 2 * 64 * n));
  KFBI_TRY(c->bandc.ensure(sizeof(double) * (kBandModeConsts + 2 * 64) * n));
  c->bc_nr = 0;
  hipLaunchKernelGGL(k_colconst, dim3(nblk(64 * n, 256)), dim3(256), 0, c->stream, N,
                     c->h * c->h * c->c2, E, c->colc.as<double>(), c->lanef.as<double>());
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

// Back-to-back replay of one kernel of the last apply on its own buffers (the outputs of
// the last stage are not written; the first stage reads a workspace as its density).
int replay_stage(kfbi_ctx* c, int stage, int reps, double* us_avg) {
  if (c->last_layer < 0) {
    set_error("kfbi_profile_kernel: no apply since the interface was installed");
    return KFBI_E_STATE;
  }
  if (stage < 0 || stage > 3 || reps < 1) {
    set_error("kfbi_profile_kernel: stage must be 0..3 and reps >= 1");
    return KFBI_E_INVALID;
  }
  hipEvent_t e0, e1;
  KFBI_HIP(hipEventCreate(&e0));
  KFBI_HIP(hipEventCreate(&e1));
  const double* dens = c->tmpM.as<double>();  // max(4, max_batch) * max_markers doubles
  const int layer = c->last_layer, B = c->last_batch, mask = 1 << stage;
  // one untimed launch, then the timed ones
  int st = KFBI_OK;
  for (int r = 0; r <= reps && st == KFBI_OK; ++r) {
    if (r == 1) hipEventRecord(e0, c->stream);
    st = (c->last_precision == KFBI_FP32)
             ? apply_t<float>(c, B, layer, dens, nullptr, nullptr, nullptr, nullptr, nullptr, mask)
             : apply_t<double>(c, B, layer, dens, nullptr, nullptr, nullptr, nullptr, nullptr, mask);
  }
  hipEventRecord(e1, c->stream);
  float ms = 0.f;
  hipError_t e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != KFBI_OK) return st;
  if (e != hipSuccess) {
    set_error("kfbi_profile_kernel: %s", hipGetErrorString(e));
    return KFBI_E_HIP;
  }
  *us_avg = 1e3 * static_cast<double>(ms) / reps;
  return KFBI_OK;
}

// Every instantiation that takes dynamic LDS may use all of a workgroup's LDS beyond its
// static part (set once per device from kfbi_create).
template <class T>
static int colsolve_attrs() {
  const void* ks[] = {kptr(k_colsolve<T, 1>),      kptr(k_colsolve<T, 2>),
                      kptr(k_colsolve<T, 4>),      kptr(k_colsolve<T, 8>),
                      kptr(k_colsolve<T, 16>),     kptr(k_colsolve<T, 32>),
                      kptr(k_colsolve_neu<T, 2>),  kptr(k_colsolve_neu<T, 3>),
                      kptr(k_colsolve_neu<T, 5>),  kptr(k_colsolve_neu<T, 9>),
                      kptr(k_colsolve_neu<T, 17>), kptr(k_colsolve_neu<T, 33>),
                      kptr(k_colsolve_band<T, 2, false>),  kptr(k_colsolve_band<T, 4, false>),
                      kptr(k_colsolve_band<T, 8, false>),  kptr(k_colsolve_band<T, 12, false>),
                      kptr(k_colsolve_band<T, 16, false>), kptr(k_colsolve_band<T, 24, false>),
                      kptr(k_colsolve_band<T, 33, false>), kptr(k_colsolve_band<T, 2, true>),
                      kptr(k_colsolve_band<T, 4, true>),   kptr(k_colsolve_band<T, 8, true>),
                      kptr(k_colsolve_band<T, 12, true>),  kptr(k_colsolve_band<T, 16, true>),
                      kptr(k_colsolve_band<T, 24, true>),  kptr(k_colsolve_band<T, 33, true>)};
  for (const void* k : ks) KFBI_TRY(allow_full_dyn_lds(k));
  return KFBI_OK;
}

int apply_kernel_attrs() {
  KFBI_TRY(allow_full_dyn_lds(kptr(k_prep)));
  KFBI_TRY(colsolve_attrs<double>());
  return colsolve_attrs<float>();
}

size_t colsolve_lds_capacity(const kfbi_ctx* c) {
  const int N = c->N;
  if (c->box_bc == KFBI_BOX_NEUMANN) {
    size_t cap = 0;
    neu_dispatch<double>(N, [&](auto EC) {
      cap = dyn_lds_capacity(kptr(k_colsolve_neu<double, decltype(EC)::value>));
    });
    return cap;
  }
  const int E = (N - 1 + 63) / 64;
  switch (E <= 1 ? 1 : E <= 2 ? 2 : E <= 4 ? 4 : E <= 8 ? 8 : E <= 16 ? 16 : 32) {
    case 1: return dyn_lds_capacity(kptr(k_colsolve<double, 1>));
    case 2: return dyn_lds_capacity(kptr(k_colsolve<double, 2>));
    case 4: return dyn_lds_capacity(kptr(k_colsolve<double, 4>));
    case 8: return dyn_lds_capacity(kptr(k_colsolve<double, 8>));
    case 16: return dyn_lds_capacity(kptr(k_colsolve<double, 16>));
    default: return dyn_lds_capacity(kptr(k_colsolve<double, 32>));
  }
}

int apply_impl(kfbi_ctx* c, int layer, int precision, const double* dens, const double* ring_user,
               const kfbi_out* out, const kfbi_bie* op, const double* xop, double* yop, int B) {
  if (precision == KFBI_FP32)
    return apply_t<float>(c, B, layer, dens, ring_user, out, op, xop, yop);
  return apply_t<double>(c, B, layer, dens, ring_user, out, op, xop, yop);
}

}  // namespace kfbi
