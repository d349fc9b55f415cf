// Per-interface geometry on gfx950 (run once per time step by kfbi_set_interface).
//
// Sec. 4.2: grid, irregular nodes and the grid-line / interface intersection points;
// Sec. 4.3: interpolation stencil {(0,0),(1,0),(0,1),(0,-1),(-1,0),(d1,d2)} around the
// closest node; App. A.1: jump values from the interface data; Sec. 5.3 (remark):
// derivatives of periodic interface quantities in Fourier space.
//
// Readings fixed here (the paper leaves them open): interface quantities between markers
// come from the 6-point Lagrange polynomial through markers k-2..k+3; crossings are
// searched on that polynomial sampled at t = s/8 of each marker interval (sign rule
// (v >= g) per sub-interval) and located by safeguarded Newton; a grid segment cut twice
// is treated as not cut, three times is an error; node (i, j) is inside iff an odd number
// of kept row-j crossings lie strictly left of x_i; closest node = floor(t + 1/2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "device_util.h"

namespace kfbi {

// --------------------------------------------------------------- differentiation vectors
// Circulant form of Fourier differentiation on M equispaced samples (Nyquist mode dropped):
//   f'(a_l)  = sum_m d1[(l - m) mod M] f_m,  d1[q] = -(2/M) sum_{k=1}^{M/2-1} k   sin(k a_q)
//   f''(a_l) = sum_m d2[(l - m) mod M] f_m,  d2[q] = -(2/M) sum_{k=1}^{M/2-1} k^2 cos(k a_q)
__global__ void k_diffvec(int M, double* __restrict__ d1, double* __restrict__ d2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M) return;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 1; k < M / 2; ++k) {
    const long long r = (static_cast<long long>(k) * q) % M;
    double sn, cs;
    sincospi(2.0 * static_cast<double>(r) / M, &sn, &cs);
    s1 += k * sn;
    s2 += static_cast<double>(k) * k * cs;
  }
  d1[q] = -2.0 * s1 / M;
  d2[q] = -2.0 * s2 / M;
}

// Marker geometry: x_a, y_a, x_aa, y_aa, s_a, s_aa (App. A: n = (y_a, -x_a)/s_a) and the
// 3h margin test against the box.  One block per marker: the four circulant sums are split
// over the threads and reduced in a fixed order.
__global__ void __launch_bounds__(256)
    k_marker_geo(int M, const double* __restrict__ X, const double* __restrict__ d1,
                 const double* __restrict__ d2, double* __restrict__ geo, double lox,
                 double hix, double loy, double hiy, const int* __restrict__ rng,
                 GeoStatus* st) {
  __shared__ double red[4][4];
  const int k = blockIdx.x;
  if (threadIdx.x == 0 && k < (M + 255) / 256) {  // ranges of the k_count_cross blocks
    atomicMin(&st->cr_lo, rng[4 * k]);
    atomicMax(&st->cr_hi, rng[4 * k + 1]);
    atomicMin(&st->cc_lo, rng[4 * k + 2]);
    atomicMax(&st->cc_hi, rng[4 * k + 3]);
  }
  const double* x = X;
  const double* y = X + M;
  double xa = 0, ya = 0, xaa = 0, yaa = 0;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    int q = k - m;
    q += (q < 0) ? M : 0;
    const double a1 = d1[q], a2 = d2[q], xm = x[m], ym = y[m];
    xa += a1 * xm;
    ya += a1 * ym;
    xaa += a2 * xm;
    yaa += a2 * ym;
  }
  xa = wave_sum(xa);
  ya = wave_sum(ya);
  xaa = wave_sum(xaa);
  yaa = wave_sum(yaa);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = xa;
    red[1][w] = ya;
    red[2][w] = xaa;
    red[3][w] = yaa;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  xa = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  ya = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  xaa = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
  yaa = ((red[3][0] + red[3][1]) + red[3][2]) + red[3][3];
  const double sa = sqrt(xa * xa + ya * ya);
  geo[k] = xa;
  geo[M + k] = ya;
  geo[2 * M + k] = xaa;
  geo[3 * M + k] = yaa;
  geo[4 * M + k] = sa;
  geo[5 * M + k] = (xa * xaa + ya * yaa) / sa;
  if (!(x[k] >= lox && x[k] <= hix && y[k] >= loy && y[k] <= hiy)) atomicMax(&st->err, 3);
}

// Crossing search on the 6-point Lagrange interpolant of one marker interval sampled at
// t = s / kSub, s = 0..kSub (the marker values themselves at t = 0 and 1): sub-interval s
// crosses the line g iff (v(t_s) >= g) != (v(t_{s+1}) >= g).  A curve nearly tangent to a
// line between two markers thereby shows both of its crossings.
constexpr int kSub = 8;

__device__ inline void sub_values(const double* cv, double* vals) {
  vals[0] = cv[2];
  vals[kSub] = cv[3];
#pragma unroll
  for (int s = 1; s < kSub; ++s) {
    double w[6];
    lagrange6(static_cast<double>(s) / kSub, w, nullptr);
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) v += cv[m] * w[m];
    vals[s] = v;
  }
}

// Lines g_j = lo + j h, j = 1..N-1, that the sampled values can cross.
__device__ inline void line_range(const double* vals, double lo, double h, int N, int* jb,
                                  int* je) {
  double vmin = vals[0], vmax = vals[0];
#pragma unroll
  for (int s = 1; s <= kSub; ++s) {
    vmin = fmin(vmin, vals[s]);
    vmax = fmax(vmax, vals[s]);
  }
  int a = static_cast<int>(floor((vmin - lo) / h)) - 1;
  int b = static_cast<int>(floor((vmax - lo) / h)) + 1;
  *jb = a < 1 ? 1 : a;
  *je = b > N - 1 ? N - 1 : b;
}

__device__ inline void stencil_values(const double* v, int k, int M, double* cv) {
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    int q = k - 2 + m;
    q = (q < 0) ? q + M : (q >= M ? q - M : q);
    cv[m] = v[q];
  }
}

// Also copies the markers xy into the context (X) and resets the status words (thread 0),
// so that no copy precedes it.
// rng[4 b + {0, 1, 2, 3}]: over the intervals of block b, the first and last row lines and
// the first and last column lines that their samples may cut (reduced in the block, so
// that few atomics fold them into the status afterwards).
__global__ void __launch_bounds__(256)
    k_count_cross(int M, const double* __restrict__ xy, double* __restrict__ Xc, double x0,
                  double y0, double h, int N, int* __restrict__ cnt, int* __restrict__ rng,
                  GeoStatus* __restrict__ st) {
  __shared__ int wr[4][4];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k < M;
  int lo_hi[4] = {1 << 30, -1, 1 << 30, -1};  // row lo, row hi, column lo, column hi
  if (live) {
    const double* X = xy;
    Xc[k] = xy[k];
    Xc[M + k] = xy[M + k];
    if (k == 0) {
      GeoStatus init{};
      init.row_lo = 1 << 30;
      init.row_hi = -1;
      init.arm_lo = 1 << 30;
      init.arm_hi = -1;
      init.cr_lo = init.cc_lo = 1 << 30;
      init.cr_hi = init.cc_hi = -1;
      *st = init;
    }
    for (int ax = 0; ax < 2; ++ax) {
      // ax = 0: rows y = y_j (compare y); ax = 1: columns x = x_i (compare x)
      const double* v = (ax == 0) ? X + M : X;
      const double lo = (ax == 0) ? y0 : x0;
      double cv[6], vals[kSub + 1];
      stencil_values(v, k, M, cv);
      sub_values(cv, vals);
      int jb, je, c = 0;
      line_range(vals, lo, h, N, &jb, &je);
      lo_hi[2 * ax] = jb;
      lo_hi[2 * ax + 1] = je;
      for (int j = jb; j <= je; ++j) {
        const double g = lo + j * h;
#pragma unroll
        for (int s = 0; s < kSub; ++s) c += ((vals[s] >= g) != (vals[s + 1] >= g)) ? 1 : 0;
      }
      cnt[ax * M + k] = c;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int v = lo_hi[q];
    for (int off = 32; off > 0; off >>= 1) {
      const int o = __shfl_xor(v, off, 64);
      v = (q & 1) ? max(v, o) : min(v, o);
    }
    if (lane == 0) wr[q][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int q = threadIdx.x;
    int v = wr[q][0];
    for (int u = 1; u < static_cast<int>(blockDim.x) / 64; ++u)
      v = (q & 1) ? max(v, wr[q][u]) : min(v, wr[q][u]);
    rng[4 * blockIdx.x + q] = v;
  }
}

// Single-block exclusive scans in place of nseg consecutive segments of n ints; the total
// of segment g to total[g] (when total is not null).  With hpost, total points into *st
// and thread 0 then writes the whole status, with the new totals, to hpost (mapped host
// memory) at system scope.
__global__ void k_scan_inplace(int n, int nseg, int* __restrict__ a, int* total,
                               const GeoStatus* st, GeoStatus* __restrict__ hpost) {
  __shared__ int scratch[17];
  const int T = blockDim.x;
  const int per = (n + T - 1) / T;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  int tots[2] = {0, 0};
  for (int g = 0; g < nseg; ++g) {
    int* ag = a + static_cast<size_t>(g) * n;
    int s = 0;
    for (int i = b; i < e; ++i) s += ag[i];
    int tot;
    int off = block_excl_scan(s, scratch, &tot);
    for (int i = b; i < e; ++i) {
      const int v = ag[i];
      ag[i] = off;
      off += v;
    }
    if (threadIdx.x == 0 && total) total[g] = tot;
    if (g < 2) tots[g] = tot;
    __syncthreads();  // scratch is reused by the next segment
  }
  if (threadIdx.x == 0 && hpost) {
    GeoStatus v = *st;
    int* vf = reinterpret_cast<int*>(&v);
    const int f0 = static_cast<int>(total - reinterpret_cast<const int*>(st));
    for (int g = 0; g < nseg && g < 2; ++g) vf[f0 + g] = tots[g];
    *hpost = v;
    __threadfence_system();
  }
}

// Safeguarded Newton for P(t) = g on [ta, tb], P the Lagrange polynomial with nodal values
// c; a = P(ta) - g and b = P(tb) - g differ in sign under sign(v) = (v >= 0).
__device__ inline double newton_root(const double* c, double g, double a, double b, double ta,
                                     double tb) {
  double lo = ta, hi = tb;
  double t = ta + (tb - ta) * (a / (a - b));
  const bool sa = (a >= 0.0);
  for (int it = 0; it < 60; ++it) {
    double w[6], dw[6];
    lagrange6(t, w, dw);
    double f = -g, fp = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      f += w[m] * c[m];
      fp += dw[m] * c[m];
    }
    const bool same = ((f >= 0.0) == sa);
    if (same)
      lo = t;
    else
      hi = t;
    double tn = t - f / fp;
    if (!isfinite(tn) || tn <= lo || tn >= hi) tn = 0.5 * (lo + hi);
    if (f == 0.0) tn = t;
    const double step = fabs(tn - t);
    t = tn;
    if (step <= 1e-12) break;
  }
  return t;
}

// Crossing records in marker order: (line, marker interval, sub-interval in t) per
// crossing; the root itself is found by k_cross_newton, one thread per crossing.
__global__ void __launch_bounds__(64) k_fill_cross(int M, const double* __restrict__ X, double x0,
                                                   double y0, double h, int N,
                                                   const int* __restrict__ off, int nh,
                                                   Crossing* __restrict__ cr, int cap,
                                                   GeoStatus* st) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  for (int ax = 0; ax < 2; ++ax) {
    const double* v = (ax == 0) ? X + M : X;
    const double lo = (ax == 0) ? y0 : x0;
    double cv[6], vals[kSub + 1];
    stencil_values(v, k, M, cv);
    sub_values(cv, vals);
    int jb, je;
    line_range(vals, lo, h, N, &jb, &je);
    int slot = off[ax * M + k] + (ax == 0 ? 0 : nh);
    for (int j = jb; j <= je; ++j) {
      const double g = lo + j * h;
      for (int sb = 0; sb < kSub; ++sb) {
        if ((vals[sb] >= g) == (vals[sb + 1] >= g)) continue;
        if (slot < cap) {
          Crossing c;
          c.line = j;
          c.k = k;
          c.seg = sb;  // sub-interval until k_cross_newton
          c.horiz = (ax == 0);
          c.t = 0.0;
          c.pos = 0.0;
          cr[slot] = c;
        } else {
          atomicMax(&st->err, 4);
        }
        ++slot;
      }
    }
  }
}

// Root of the crossing in its sub-interval (safeguarded Newton), the other coordinate and
// the grid segment lo + seg h <= pos < lo + (seg + 1) h.
__global__ void __launch_bounds__(64) k_cross_newton(int nc, int M, const double* __restrict__ X,
                                                     double x0, double y0, double h,
                                                     Crossing* __restrict__ cr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  Crossing x = cr[c];
  const int ax = x.horiz ? 0 : 1;
  const double* v = (ax == 0) ? X + M : X;
  const double* o = (ax == 0) ? X : X + M;
  const double lo = (ax == 0) ? y0 : x0;
  const double olo = (ax == 0) ? x0 : y0;
  double cv[6], co[6], vals[kSub + 1];
  stencil_values(v, x.k, M, cv);
  stencil_values(o, x.k, M, co);
  sub_values(cv, vals);
  const int sb = x.seg;
  const double g = lo + x.line * h;
  const double t = newton_root(cv, g, vals[sb] - g, vals[sb + 1] - g,
                               static_cast<double>(sb) / kSub, static_cast<double>(sb + 1) / kSub);
  double w[6];
  lagrange6(t, w, nullptr);
  double pos = 0.0;
#pragma unroll
  for (int m = 0; m < 6; ++m) pos += w[m] * co[m];
  int seg = static_cast<int>(floor((pos - olo) / h));
  for (int r = 0; r < 2; ++r) {
    if (olo + (seg + 1) * h <= pos) seg += 1;
    if (olo + seg * h > pos) seg -= 1;
  }
  x.t = t;
  x.pos = pos;
  x.seg = seg;
  cr[c] = x;
}

// Segment marking with pairs dropped: the first crossing of a segment stores its id, a
// second one turns the entry into -2 (segment cut twice: treated as not cut), a third is
// a geometry error (1).
__device__ inline void mark_segment(int* slot, int c, GeoStatus* st) {
  const int prev = atomicCAS(slot, -1, c);
  if (prev == -1) return;
  const int old = atomicExch(slot, -2);
  if (old < 0) atomicMax(&st->err, 1);
}

// Mark row segments: hid[j*(N+1)+i] = crossing on row segment (i, i+1) of row j.
__global__ void k_mark_h(int nh, const Crossing* __restrict__ cr, int N, int* __restrict__ hid,
                         GeoStatus* st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nh) return;
  const Crossing x = cr[c];
  if (x.seg < 0 || x.seg > N - 1) {
    atomicMax(&st->err, 5);
    return;
  }
  mark_segment(&hid[x.line * (N + 1) + x.seg], c, st);
}

// Raw column segments of the column crossings (pairs marked -2 as for rows).
__global__ void k_pair_v(int nh, int nv, const Crossing* __restrict__ cr, int N,
                         int* __restrict__ vraw, GeoStatus* st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nv) return;
  const Crossing x = cr[nh + c];
  if (x.seg < 0 || x.seg > N - 1) {
    atomicMax(&st->err, 5);
    return;
  }
  mark_segment(&vraw[x.seg * (N + 1) + x.line], nh + c, st);
}

// Mark column segments after the labels exist: vid[j*(N+1)+i] = crossing on column i
// between rows j and j+1.  A crossing within 1e-9 h of a segment end moves to the
// neighbouring segment when only that one changes label (interface through a node up
// to rounding); a crossing with no label change nearby is a geometry error.
__global__ void k_mark_v(int nh, int nv, const Crossing* __restrict__ cr, int N, double y0,
                         double h, const int8_t* __restrict__ lab, const int* __restrict__ vraw,
                         int* __restrict__ vid, GeoStatus* st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nv) return;
  const Crossing x = cr[nh + c];
  const int i = x.line, s = x.seg, n1 = N + 1;
  if (s < 0 || s > N - 1) {
    atomicMax(&st->err, 5);
    return;
  }
  const double tol = 1e-9 * h;
  auto flips = [&](int t) { return t >= 0 && t <= N - 1 && lab[t * n1 + i] != lab[(t + 1) * n1 + i]; };
  if (vraw[s * n1 + i] == -2) {  // one of a pair: the segment must not change label
    if (flips(s)) atomicMax(&st->err, 2);
    return;
  }
  int seg;
  if (flips(s))
    seg = s;
  else if (x.pos - (y0 + s * h) <= tol && flips(s - 1))
    seg = s - 1;
  else if ((y0 + (s + 1) * h) - x.pos <= tol && flips(s + 1))
    seg = s + 1;
  else {
    atomicMax(&st->err, 2);
    return;
  }
  const int old = atomicExch(&vid[seg * n1 + i], nh + c);
  if (old != -1) atomicMax(&st->err, 1);
}

// Labels per row: node (i, j) is in Omega+ iff #{row-j crossings with seg < i} is odd
// (seg < i  <=>  xi < x_i).  One block per row.
// hid, vid, vraw = -1 and need = 0 on the nn nodes; rowoff[0..nr) = 0.
// Node maps cleared over node indices [4 t0, 4 t1) (whole rows, rounded out to groups of
// four: the extra nodes lie in rows that are clear already), rowoff[0..nr) and
// rowcnt[0..nc) zeroed.
__global__ void k_geo_clear(int nn, int t0, int t1, int nr, int nc, int* __restrict__ hid,
                            int* __restrict__ vid, int* __restrict__ vraw,
                            int* __restrict__ need, int* __restrict__ rowoff,
                            int* __restrict__ rowcnt) {
  const int tt = blockIdx.x * blockDim.x + threadIdx.x;
  if (tt < nr) rowoff[tt] = 0;
  if (tt < nc) rowcnt[tt] = 0;
  const int t = t0 + tt;
  if (t >= t1) return;
  const int i = 4 * t;
  if (i + 3 < nn) {
    const int4 m1 = make_int4(-1, -1, -1, -1), z = make_int4(0, 0, 0, 0);
    reinterpret_cast<int4*>(hid)[t] = m1;
    reinterpret_cast<int4*>(vid)[t] = m1;
    reinterpret_cast<int4*>(vraw)[t] = m1;
    reinterpret_cast<int4*>(need)[t] = z;
  } else {
    for (int k = i; k < nn; ++k) {
      hid[k] = vid[k] = vraw[k] = -1;
      need[k] = 0;
    }
  }
}

// Labels of row j: node i is inside iff the row's crossings on the segments left of it are
// odd in number.  Each wavefront takes consecutive chunks of 64 nodes: one coalesced load
// per lane and chunk, the chunk's crossings as a ballot mask, the parity before a lane by
// a popcount of the mask's lower bits, the parity carried in from the wavefronts to the
// left through LDS.  One block of 256 threads per row, N + 1 <= 64 * 4 * kLabelChunks.
constexpr int kLabelChunks = 9;
static_assert(64 * 4 * kLabelChunks >= 2049, "rows of up to 2049 nodes (N <= 2048)");
__global__ void __launch_bounds__(256) k_label(int N, int j0, const int* __restrict__ hid,
                                               int8_t* __restrict__ lab) {
  __shared__ int wpar[4];
  const int j = j0 + blockIdx.x;
  const int n1 = N + 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nch = (n1 + 63) >> 6;
  const int per = (nch + 3) >> 2;
  const int c0 = w * per, c1 = min(nch, c0 + per);
  unsigned long long mask[kLabelChunks];
  int par = 0;
#pragma unroll
  for (int u = 0; u < kLabelChunks; ++u) {
    const int i = (c0 + u) * 64 + lane;
    const bool x = (c0 + u < c1) && i < n1 && hid[j * n1 + i] >= 0;
    mask[u] = __ballot(x);
    par ^= __popcll(mask[u]) & 1;
  }
  if (lane == 0) wpar[w] = par;
  __syncthreads();
  int carry = 0;
  for (int q = 0; q < w; ++q) carry ^= wpar[q];
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int u = 0; u < kLabelChunks; ++u) {
    const int i = (c0 + u) * 64 + lane;
    if (c0 + u < c1 && i < n1)
      lab[j * n1 + i] = static_cast<int8_t>(carry ^ (__popcll(mask[u] & below) & 1));
    carry ^= __popcll(mask[u]) & 1;
  }
}

// Irregular arms P -> Q (Sec. 4.2.1) of interior node P: neighbour Q with another label.
// Order within a node: east, west, north, south.
__device__ inline int node_arms(int i, int j, int N, const int8_t* lab, const int* hid,
                                const int* vid, int* cid, int* qi, int* qj, GeoStatus* st) {
  const int n1 = N + 1;
  const int8_t lp = lab[j * n1 + i];
  int na = 0;
  const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
  for (int d = 0; d < 4; ++d) {
    const int ii = i + di[d], jj = j + dj[d];
    if (lab[jj * n1 + ii] == lp) continue;
    int c;
    if (d == 0)
      c = hid[j * n1 + i];
    else if (d == 1)
      c = hid[j * n1 + i - 1];
    else if (d == 2)
      c = vid[j * n1 + i];
    else
      c = vid[(j - 1) * n1 + i];
    if (c < 0) {
      atomicMax(&st->err, 2);
      continue;
    }
    if (cid) {
      cid[na] = c;
      qi[na] = ii;
      qj[na] = jj;
    }
    ++na;
  }
  return na;
}

// Arms of the interior nodes i0..i1 of row j0 + blockIdx.x (the nodes outside have no
// label change around them).
__global__ void k_arm_rowcount(int N, int j0, int i0, int i1, const int8_t* __restrict__ lab,
                               const int* __restrict__ hid, const int* __restrict__ vid,
                               int* __restrict__ rowcnt, GeoStatus* st) {
  __shared__ double scratch[16];
  const int j = j0 + blockIdx.x;  // interior rows j0.. (1 <= j0, last <= N - 1)
  int s = 0;
  for (int i = i0 + threadIdx.x; i <= i1; i += blockDim.x)
    s += node_arms(i, j, N, lab, hid, vid, nullptr, nullptr, nullptr, st);
  const double tot = block_sum<double>(static_cast<double>(s), scratch);
  if (threadIdx.x == 0) rowcnt[j] = static_cast<int>(tot);
}

// Write arms of row j in (i, direction) order with the data of their correction
// coefficients (formed by k_arm_coef).
// For arm P -> Q cut at the crossing with signed offset d = coord(Q) - crossing coord:
//   T = [u] + d [u_s] + d^2/2 [u_ss],  RHS_P += -T/h^2 (P inside) or +T/h^2 (P outside),
// T linear in (Phi, Phi_a, Phi_aa, Psi, Psi_a) at the crossing (App. A.1), each of which
// is the 6-point Lagrange combination of marker values.
__global__ void k_arm_fill(int N, int j0, int i0, int i1, double x0, double y0, double h, int M,
                           const int8_t* __restrict__ lab, const int* __restrict__ hid,
                           const int* __restrict__ vid, const int* __restrict__ rowoff,
                           const Crossing* __restrict__ cr, const double* __restrict__ geo,
                           int* __restrict__ armpk, ArmCoef* __restrict__ armc, GeoStatus* st) {
  __shared__ int scratch[17];
  const int j = j0 + blockIdx.x;
  // a row without arms has nothing to fill (k_arm_rowcount has checked it already); the
  // condition is the same for the whole block
  if (rowoff[j] == rowoff[j + 1]) return;
  const int n = i1 - i0 + 1;  // the row's nodes i0..i1, as in k_arm_rowcount
  const int T = blockDim.x;
  const int per = (n + T - 1) / T;
  const int b = i0 + threadIdx.x * per, e = min(i1 + 1, b + per);  // i in [b, e)
  int cnt = 0;
  for (int i = b; i < e; ++i) cnt += node_arms(i, j, N, lab, hid, vid, nullptr, nullptr, nullptr, st);
  int slot = rowoff[j] + block_excl_scan(cnt, scratch, nullptr);
  const double* xa = geo;
  const double* ya = geo + M;
  const double* xaa = geo + 2 * M;
  const double* yaa = geo + 3 * M;
  const double ih2 = 1.0 / (h * h);
  for (int i = b; i < e; ++i) {
    int cid[4], qi[4], qj[4];
    const int na = node_arms(i, j, N, lab, hid, vid, cid, qi, qj, st);
    const double sgn = lab[j * (N + 1) + i] ? -ih2 : ih2;
    for (int a = 0; a < na; ++a) {
      const Crossing x = cr[cid[a]];
      double w[6];
      lagrange6(x.t, w, nullptr);
      double g[4] = {0, 0, 0, 0};
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        int q = x.k - 2 + m;
        q = (q < 0) ? q + M : (q >= M ? q - M : q);
        g[0] += w[m] * xa[q];
        g[1] += w[m] * ya[q];
        g[2] += w[m] * xaa[q];
        g[3] += w[m] * yaa[q];
      }
      const bool hz = x.horiz;
      const double d = hz ? (x0 + qi[a] * h) - x.pos : (y0 + qj[a] * h) - x.pos;
      // the correction coefficients are formed by k_arm_coef, one thread per arm: here the
      // record holds the crossing's tangent and its derivative, d, and the side and
      // direction flags
      ArmCoef ac;
#pragma unroll
      for (int m = 0; m < 6; ++m) ac.l[m] = w[m];
#pragma unroll
      for (int q = 0; q < 4; ++q) ac.coef[q] = g[q];
      ac.coef[4] = d;
      ac.k = x.k;
      ac.pad = (hz ? 1 : 0) | (sgn < 0.0 ? 2 : 0);
      armpk[slot] = i | (j << 16);
      armc[slot] = ac;
      ++slot;
    }
  }
}

// The five correction coefficients of arm a (Sec. 4.2.1 eq. modified-fdm with the App. A.1
// jumps): the jump T = [u] + d [u_s] + d^2/2 [u_ss] along the arm for each unit vector of
// (Phi, Phi_a, Phi_aa, Psi, Psi_a), with the sign of P's side and 1/h^2; the record's
// geometry fields (written by k_arm_fill) are replaced by the coefficients.  One thread
// per arm, so an arm-rich node no longer holds up its row's block.
__global__ void k_arm_coef(int cap, const int* __restrict__ narms, double h, double c2,
                           ArmCoef* __restrict__ armc) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= cap || a >= *narms) return;
  ArmCoef ac = armc[a];
  const double g0 = ac.coef[0], g1 = ac.coef[1], g2 = ac.coef[2], g3 = ac.coef[3];
  const double d = ac.coef[4];
  const bool hz = ac.pad & 1;
  const double ih2 = 1.0 / (h * h);
  const double sgn = (ac.pad & 2) ? -ih2 : ih2;
  for (int qv = 0; qv < 5; ++qv) {
    double u[5] = {0, 0, 0, 0, 0};
    u[qv] = 1.0;
    double J[6];
    jumps_closed(g0, g1, g2, g3, u[0], u[1], u[2], u[3], u[4], c2, J);
    const double Tv = hz ? J[0] + d * J[1] + 0.5 * d * d * J[3]
                         : J[0] + d * J[2] + 0.5 * d * d * J[4];
    ac.coef[qv] = sgn * Tv;
  }
  ac.pad = 0;
  armc[a] = ac;
}

// Row-ordered arm coefficients as structure of arrays (coefR[q * cap + a], kR[a]).
// Arm coefficients in part-slot order for the row transform kernel: slot t of part q
// is arm pdesc[q].a0 + t, or an empty slot (zero coefficients) past the part's end.
// Structure of arrays: coefR[c * cap + 16 q + t] (c = 0..10), kR[16 q + t] (first
// stencil marker), iR = kR + cap (grid column of the arm's node), cap = 16 P.
// The same launch zeroes the per-apply corrections r of every slot (nbatch copies) and
// writes sc[s], sc[cap + s] = sin, cos (i pi / N) of the slot's column i (the step of the
// row transform's recurrence; 0 and 1 for an empty slot), from the sine table
// sinT[t] = sin(t pi / N), t < 2N.
__global__ void k_part_soa(int P, int cap, const int4* __restrict__ pdesc,
                           const ArmCoef* __restrict__ armc, const int* __restrict__ armpk,
                           double* __restrict__ coefR, int* __restrict__ kR,
                           double* __restrict__ armr, int nbatch, int N,
                           const double* __restrict__ sinT, double* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= cap) return;
  for (int b = 0; b < nbatch; ++b) armr[static_cast<size_t>(b) * cap + s] = 0.0;
  sc[s] = 0.0;
  sc[cap + s] = 1.0;
  if (P == 0) return;
  const int q = s / kArmsPerPart, t = s % kArmsPerPart;
  const int4 d = pdesc[q];
  const int a = d.y + t;
  if (a < d.z) {
    const ArmCoef ac = armc[a];
#pragma unroll
    for (int m = 0; m < 6; ++m) coefR[m * cap + s] = ac.l[m];
#pragma unroll
    for (int c = 0; c < 5; ++c) coefR[(6 + c) * cap + s] = ac.coef[c];
    kR[s] = ac.k;
    const int i = armpk[a] & 0xffff;
    kR[cap + s] = i;
    const int mask = 2 * N - 1;
    sc[s] = sinT[i & mask];
    sc[cap + s] = sinT[(i + N / 2) & mask];
  } else {
#pragma unroll
    for (int c = 0; c < kArmCoefCount; ++c) coefR[c * cap + s] = 0.0;
    kR[s] = 0;
    kR[cap + s] = 0;
  }
}

// Arm slots grouped by the marker chunk of their interval (the chunks of the derivative
// kernel, which forms their corrections), in one block: counts per chunk (LDS atomics),
// their exclusive scan into off[0..nmk] (off[nmk] = total), then every slot appended to
// its chunk's range through an LDS cursor (order within a chunk is free).  Empty slots
// (column 0) are skipped.
__global__ void __launch_bounds__(1024)
    k_chunk_arms(int cap, int MC, int nmk, const int* __restrict__ kR, int* __restrict__ off,
                 int* __restrict__ list) {
  extern __shared__ int cur[];  // nmk + 1 counters, then cursors
  __shared__ int scratch[17];
  const int T = blockDim.x;
  for (int i = threadIdx.x; i <= nmk; i += T) cur[i] = 0;
  __syncthreads();
  for (int a = threadIdx.x; a < cap; a += T)
    if (kR[cap + a] != 0) atomicAdd(&cur[kR[a] / MC], 1);
  __syncthreads();
  const int n = nmk + 1;
  const int per = (n + T - 1) / T;
  const int b = threadIdx.x * per, e = min(n, b + per);
  int sum = 0;
  for (int i = b; i < e; ++i) sum += cur[i];
  int o = block_excl_scan(sum, scratch, nullptr);
  for (int i = b; i < e; ++i) {
    const int v = cur[i];
    off[i] = o;
    cur[i] = o;
    o += v;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < cap; a += T)
    if (kR[cap + a] != 0) list[atomicAdd(&cur[kR[a] / MC], 1)] = a;
}

// The chunk lists' arm data in list order (coefficients [kArmCoefCount][cap], and the
// offset k_a - k0 of the arm's interval in its chunk, which is the window position of
// marker k_a - 2), so that the derivative kernel reads a chunk's arms with contiguous loads.
__global__ void k_chunk_arm_pack(int cap, int MC, const int* __restrict__ total,
                                 const int* __restrict__ list, const double* __restrict__ coefR,
                                 const int* __restrict__ kR, double* __restrict__ cc,
                                 int* __restrict__ ck) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cap || e >= *total) return;
  const int s = list[e];
#pragma unroll
  for (int q = 0; q < kArmCoefCount; ++q) cc[q * cap + e] = coefR[q * cap + s];
  ck[e] = kR[s] % MC;
}

// Part descriptors (row, first arm, end arm) in row order, from the part offsets of
// k_rows_scan.
__global__ void k_part_fill(int N, const int* __restrict__ rowoff,
                            const int* __restrict__ rowpart, int4* __restrict__ pdesc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 1 || j > N - 1) return;
  const int a0 = rowoff[j], a1 = rowoff[j + 1];
  int q = rowpart[j];
  for (int a = a0; a < a1; a += kArmsPerPart, ++q) pdesc[q] = make_int4(j, a, min(a1, a + kArmsPerPart), 0);
}

// Distinct interpolation nodes of each chunk of MC consecutive markers, sorted by (row,
// column), and each marker's six stencil slots as indices into its chunk's list.
//
// The chunk list is stored in the order of the grid row of the first stencil node of each
// chunk's first marker (ties by chunk index): chunk ch goes to position pos, whose node keys and count
// are cnode[pos * 6 MC ...] and ccount[pos], and chpos[pos] = ch.  The node kernel hands
// consecutive positions to one XCD, so the chunks of an XCD share grid rows.  Any order
// gives the same results; this one only saves L2 misses.
__global__ void k_chunk_nodes(int M, int MC, const int* __restrict__ mkkey,
                              int* __restrict__ cnode, int* __restrict__ ccount,
                              int* __restrict__ chpos, int* __restrict__ mkloc) {
  extern __shared__ int keys[];  // 2 * 6 * MC: keys, first-occurrence flags
  __shared__ int rank;
  int* first = keys + 6 * MC;
  const int ch = blockIdx.x, nch = gridDim.x;
  const int k0 = ch * MC, k1 = min(M, k0 + MC);
  const int ns = 6 * (k1 - k0);
  if (threadIdx.x == 0) rank = 0;
  for (int t = threadIdx.x; t < ns; t += blockDim.x) keys[t] = mkkey[6 * k0 + t];
  __syncthreads();
  {  // position of this chunk: chunks with a lower first row, or the same row and index
    const int v = keys[0] >> 16;
    int r = 0;
    for (int o = threadIdx.x; o < nch; o += blockDim.x) {
      const int u = mkkey[6 * o * MC] >> 16;
      r += (u < v || (u == v && o < ch)) ? 1 : 0;
    }
    if (r) atomicAdd(&rank, r);
  }
  // rank-based sort with duplicates removed: a key's slot is the number of distinct keys
  // below it (ns <= 96, one thread per stencil slot)
  for (int t = threadIdx.x; t < ns; t += blockDim.x) {
    const int v = keys[t];
    int f = 1;
    for (int a = 0; a < t; ++a) f &= (keys[a] != v);
    first[t] = f;
  }
  __syncthreads();
  int nu = 0;
  for (int a = 0; a < ns; ++a) nu += first[a];
  for (int t = threadIdx.x; t < ns; t += blockDim.x) {
    const int v = keys[t];
    int r = 0;
    for (int a = 0; a < ns; ++a) r += (first[a] && keys[a] < v) ? 1 : 0;
    mkloc[6 * k0 + t] = r;
    if (first[t]) cnode[rank * 6 * MC + r] = v;
  }
  if (threadIdx.x == 0) {
    ccount[rank] = nu;
    chpos[rank] = ch;
  }
}

// Gauss-Jordan inverse of a 6x6 matrix with partial pivoting.  Every loop is unrolled and
// the row exchange is done with selects, so both matrices stay in registers.
__device__ inline void inv6(double A[6][6], double R[6][6]) {
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) R[r][c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    int p = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < 6; ++r)
      if (fabs(A[r][c]) > best) {
        best = fabs(A[r][c]);
        p = r;
      }
#pragma unroll
    for (int r = c + 1; r < 6; ++r) {
      const bool sw = (r == p);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double ac = A[c][q], ar = A[r][q], rc = R[c][q], rr = R[r][q];
        A[c][q] = sw ? ar : ac;
        A[r][q] = sw ? ac : ar;
        R[c][q] = sw ? rr : rc;
        R[r][q] = sw ? rc : rr;
      }
    }
    const double piv = 1.0 / A[c][c];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      A[c][q] *= piv;
      R[c][q] *= piv;
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const double f = A[r][c];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        A[r][q] -= f * A[c][q];
        R[r][q] -= f * R[c][q];
      }
    }
  }
}

// Sec. 4.3 extraction weights for every marker; marks the needed stencil nodes.
__global__ void __launch_bounds__(64) k_marker_ext(int M, const double* __restrict__ X, const double* __restrict__ geo,
                             double x0, double y0, double h, int N, double c2,
                             const int8_t* __restrict__ lab, double* __restrict__ ext,
                             int* __restrict__ need, int* __restrict__ stn) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double px = X[k], py = X[M + k];
  const int i0 = static_cast<int>(floor((px - x0) / h + 0.5));
  const int j0 = static_cast<int>(floor((py - y0) / h + 0.5));
  const int d1 = (px > x0 + i0 * h) ? 1 : -1;
  const int d2 = (py > y0 + j0 * h) ? 1 : -1;
  const int ri[6] = {0, 1, 0, 0, -1, d1}, rj[6] = {0, 0, 1, -1, 0, d2};
  double A[6][6], Rv[6][6], At[6][6];
  double chi[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int I = i0 + ri[m], J = j0 + rj[m];
    const double dx = (x0 + I * h - px) / h, dy = (y0 + J * h - py) / h;
    A[m][0] = 1.0;
    A[m][1] = dx;
    A[m][2] = dy;
    A[m][3] = 0.5 * dx * dx;
    A[m][4] = dx * dy;
    A[m][5] = 0.5 * dy * dy;
    const double Dx = dx * h, Dy = dy * h;
    At[m][0] = 1.0;
    At[m][1] = Dx;
    At[m][2] = Dy;
    At[m][3] = 0.5 * Dx * Dx;
    At[m][4] = Dx * Dy;
    At[m][5] = 0.5 * Dy * Dy;
    chi[m] = lab[J * (N + 1) + I] ? 0.0 : 1.0;  // correction added for nodes in Omega-
    need[J * (N + 1) + I] = 1;
    stn[6 * k + m] = (J << 16) | I;
  }
  inv6(A, Rv);
  double Wr[18];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    Wr[m] = Rv[0][m];
    Wr[6 + m] = Rv[1][m] / h;
    Wr[12 + m] = Rv[2][m] / h;
  }
  for (int q = 0; q < 18; ++q) ext[(kExtW + q) * M + k] = Wr[q];
  // jumps at the marker as linear maps of (Phi, Phi_a, Phi_aa, Psi, Psi_a)
  const double xa = geo[k], ya = geo[M + k], xaa = geo[2 * M + k], yaa = geo[3 * M + k];
  double Cj[6][5];  // rows in Taylor order ([v],[v_x],[v_y],[v_xx],[v_xy],[v_yy])
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    double u[5] = {0, 0, 0, 0, 0};
    u[q] = 1.0;
    double J[6];
    jumps_closed(xa, ya, xaa, yaa, u[0], u[1], u[2], u[3], u[4], c2, J);
    Cj[0][q] = J[0];
    Cj[1][q] = J[1];
    Cj[2][q] = J[2];
    Cj[3][q] = J[3];
    Cj[4][q] = J[5];
    Cj[5][q] = J[4];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double e = 0.0;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        double cm = 0.0;
#pragma unroll
        for (int s = 0; s < 6; ++s) cm += At[m][s] * Cj[s][q];
        e += chi[m] * (Wr[6 * r + m] * cm);
      }
      ext[(kExtE + 5 * r + q) * M + k] = e;
      ext[(kExtD + 5 * r + q) * M + k] = Cj[r][q];
    }
  const double sa = geo[4 * M + k];
  ext[kExtN * M + k] = ya / sa;
  ext[(kExtN + 1) * M + k] = -xa / sa;
  ext[kExtQ * M + k] = sa * (2.0 * M_PI / M);
}

// Node numbering: per row count of needed nodes, then scan over rows (single block):
// node offsets, compact list of needed rows, band [row_lo, row_hi].
__global__ void k_need_rowcount(int N, int j0, int i0, int i1, const int* __restrict__ need,
                                int* __restrict__ rowcnt) {
  __shared__ double scratch[16];
  const int j = j0 + blockIdx.x;
  int s = 0;
  for (int i = i0 + threadIdx.x; i <= i1; i += blockDim.x) s += need[j * (N + 1) + i];
  const double t = block_sum<double>(static_cast<double>(s), scratch);
  if (threadIdx.x == 0) rowcnt[j] = static_cast<int>(t);
}

__global__ void __launch_bounds__(1024)
    k_rows_scan(int N, const int* __restrict__ rowcnt, int* __restrict__ nodeoff,
                int* __restrict__ rows, int* __restrict__ rowptr,
                const int* __restrict__ rowoff, int* __restrict__ rowpart, GeoStatus* st,
                GeoStatus* __restrict__ hpost) {
  // single block: exclusive scans of the node counts and of (count > 0), the band of node
  // rows, the first and last rows holding arms, and the row parts of the row transform
  // (ceil(arms / kArmsPerPart) per interior row); thread 0 then posts the whole status to
  // mapped host memory at system scope
  __shared__ int scratch[17];
  __shared__ int band[4][32];  // per wavefront: node rows lo, hi, arm rows lo, hi
  const int n1 = N + 1;
  const int T = blockDim.x;
  const int per = (n1 + T - 1) / T;
  const int b = threadIdx.x * per, e = min(n1, b + per);
  int s = 0, f = 0, pc = 0;
  for (int j = b; j < e; ++j) {
    s += rowcnt[j];
    f += rowcnt[j] > 0;
    if (j >= 1 && j <= N - 1) pc += (rowoff[j + 1] - rowoff[j] + kArmsPerPart - 1) / kArmsPerPart;
  }
  int tot_nodes, tot_rows, tot_parts;
  int off = block_excl_scan(s, scratch, &tot_nodes);
  int roff = block_excl_scan(f, scratch, &tot_rows);
  int poff = block_excl_scan(pc, scratch, &tot_parts);
  int lo = 1 << 30, hi = -1, alo = 1 << 30, ahi = -1;
  for (int j = b; j < e; ++j) {
    nodeoff[j] = off;
    if (j >= 1 && j <= N - 1 && rowoff[j + 1] > rowoff[j]) {
      alo = min(alo, j);
      ahi = max(ahi, j);
    }
    if (rowcnt[j] > 0) {
      rows[roff] = j;
      rowptr[roff] = off;
      ++roff;
      lo = min(lo, j);
      hi = max(hi, j);
    }
    off += rowcnt[j];
    rowpart[j] = poff;
    if (j >= 1 && j <= N - 1) poff += (rowoff[j + 1] - rowoff[j] + kArmsPerPart - 1) / kArmsPerPart;
  }
  // the bands by shuffles within each wavefront, then over the wavefronts (atomics on
  // one LDS word from every thread serialise)
  int bv[4] = {lo, hi, alo, ahi};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (int o = 32; o > 0; o >>= 1) {
      const int x = __shfl_xor(bv[q], o, 64);
      bv[q] = (q & 1) ? max(bv[q], x) : min(bv[q], x);
    }
    if (lane == 0) band[q][wv] = bv[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int r[4] = {band[0][0], band[1][0], band[2][0], band[3][0]};
    for (int u = 1; u < T / 64; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] = (q & 1) ? max(r[q], band[q][u]) : min(r[q], band[q][u]);
    rowptr[tot_rows] = tot_nodes;
    GeoStatus v = *st;
    v.n_nodes = tot_nodes;
    v.n_rows = tot_rows;
    v.n_parts = tot_parts;
    v.row_lo = r[0];
    v.row_hi = r[1];
    v.arm_lo = r[2];
    v.arm_hi = r[3];
    *st = v;
    *hpost = v;
    __threadfence_system();
  }
}

static inline int nblk(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

// Rows beyond the curve's sampled rows that a set-up may touch: vertical crossings and arms
// one row out, stencil nodes two rows out of their marker; the rest is slack.
constexpr int kGeoBandMargin = 6;

int geometry_setup(kfbi_ctx* c, int M, const double* xy) {
  const int N = c->N;
  const int n1 = N + 1;
  const double h = c->h;
  hipStream_t s = c->stream;
  GeoStatus* st = c->gstat.as<GeoStatus>();

  KFBI_TRY(c->X.ensure(sizeof(double) * 2 * M));
  KFBI_TRY(c->geo.ensure(sizeof(double) * 6 * M));
  KFBI_TRY(c->dvec.ensure(sizeof(double) * 2 * M));
  KFBI_TRY(c->cnt.ensure(sizeof(int) * (2 * M + 2)));
  KFBI_TRY(c->intptr.ensure(sizeof(int) * (4 * ((M + 255) / 256) + 2)));
  KFBI_TRY(c->ext.ensure(sizeof(double) * kExtCount * M));
  KFBI_TRY(c->mknode.ensure(sizeof(int) * 6 * M));

  double* d1 = c->dvec.as<double>();
  double* d2 = d1 + M;
  if (c->d_M != M) {
    hipLaunchKernelGGL(k_diffvec, dim3(nblk(M, 256)), dim3(256), 0, s, M, d1, d2);
    c->d_M = M;
  }
  // crossing counts per marker interval (this launch also copies the markers into X and
  // resets the status), the marker geometry with the margin test, and the two scans,
  // which post the status to mapped host memory for the host to size the crossing list
  int* cnt = c->cnt.as<int>();
  int* rng = c->intptr.as<int>();
  hipLaunchKernelGGL(k_count_cross, dim3(nblk(M, 256)), dim3(256), 0, s, M, xy,
                     c->X.as<double>(), c->x0, c->y0, h, N, cnt, rng, st);
  const double mg = 3.0 * h;
  hipLaunchKernelGGL(k_marker_geo, dim3(M), dim3(256), 0, s, M, c->X.as<double>(), d1,
                     d2, c->geo.as<double>(), c->x0 + mg, c->x0 + c->side - mg, c->y0 + mg,
                     c->y0 + c->side - mg, rng, st);
  GeoStatus* hs = reinterpret_cast<GeoStatus*>(static_cast<char*>(c->hstat) + kGeoStatusOffset);
  GeoStatus* hs_dev =
      reinterpret_cast<GeoStatus*>(static_cast<char*>(c->dstat) + kGeoStatusOffset);
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, M, 2, cnt, &st->n_cross_h, st,
                     hs_dev);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(s));
  if (hs->err == 3) {
    set_error("interface marker closer than 3h to the box boundary");
    return KFBI_E_GEOMETRY;
  }
  const int nh = hs->n_cross_h, nv = hs->n_cross_v, nc = nh + nv;
  KFBI_TRY(c->cross.ensure(sizeof(Crossing) * (nc + 1)));
  const int narm_cap = 2 * nc + 1;
  KFBI_TRY(c->armpk.ensure(sizeof(int) * narm_cap));
  KFBI_TRY(c->armcoef.ensure(sizeof(ArmCoef) * narm_cap));
  KFBI_TRY(c->armr.ensure(sizeof(double) * narm_cap));


  Crossing* cr = c->cross.as<Crossing>();
  hipLaunchKernelGGL(k_fill_cross, dim3(nblk(M, 64)), dim3(64), 0, s, M, c->X.as<double>(), c->x0,
                     c->y0, h, N, cnt, nh, cr, nc, st);
  if (nc > 0)
    hipLaunchKernelGGL(k_cross_newton, dim3(nblk(nc, 64)), dim3(64), 0, s, nc, M,
                       c->X.as<double>(), c->x0, c->y0, h, cr);
  int* hid = c->hid.as<int>();
  int* vid = c->vid.as<int>();
  int* vraw = c->vraw.as<int>();
  int* need = c->need.as<int>();
  int* rowoff = c->armrow.as<int>();  // N+2 entries
  int* rowcnt = c->rowsum.as<int>();
  // The rows that can hold crossings, labels, arms or stencil nodes: the rows of the
  // curve's samples and kGeoBandMargin more on each side.  The node maps and labels of the
  // rows that the previous interface used (c->gb_lo..c->gb_hi) are cleared as well; every
  // row outside both keeps cleared maps and zero labels from before.
  const int glo = std::max(0, hs->cr_lo - kGeoBandMargin);
  const int ghi = std::min(N, hs->cr_hi + kGeoBandMargin);
  const int clo = std::max(0, hs->cc_lo - kGeoBandMargin);  // columns likewise (the node
  const int chi = std::min(N, hs->cc_hi + kGeoBandMargin);  // sweeps inside the rows)
  const int ulo = std::min(glo, c->gb_lo), uhi = std::min(N, std::max(ghi, c->gb_hi));
  c->gb_lo = ulo;  // until this interface is in place: the union may hold old entries
  c->gb_hi = uhi;
  {  // the per-node maps of those rows, the arm and node row counts
    const int nn = n1 * n1;
    const int t0 = (ulo * n1) / 4, t1 = std::min((nn + 3) / 4, ((uhi + 1) * n1 + 3) / 4);
    const int nt = std::max(t1 - t0, N + 2);
    hipLaunchKernelGGL(k_geo_clear, dim3(nblk(nt, 256)), dim3(256), 0, s, nn, t0, t1, N + 2,
                       n1, hid, vid, vraw, need, rowoff, rowcnt);
  }
  if (nh > 0)
    hipLaunchKernelGGL(k_mark_h, dim3(nblk(nh, 256)), dim3(256), 0, s, nh, cr, N, hid, st);
  int8_t* lab = c->lab.as<int8_t>();
  hipLaunchKernelGGL(k_label, dim3(uhi - ulo + 1), dim3(256), 0, s, N, ulo, hid, lab);
  if (nv > 0) {
    hipLaunchKernelGGL(k_pair_v, dim3(nblk(nv, 256)), dim3(256), 0, s, nh, nv, cr, N, vraw, st);
    hipLaunchKernelGGL(k_mark_v, dim3(nblk(nv, 256)), dim3(256), 0, s, nh, nv, cr, N, c->y0, h,
                       lab, vraw, vid, st);
  }
  // arms
  const int alo = std::max(1, glo), ahi = std::min(N - 1, ghi);  // interior rows of the band
  const int ilo = std::max(1, clo), ihi = std::min(N - 1, chi);  // interior columns
  hipLaunchKernelGGL(k_arm_rowcount, dim3(ahi - alo + 1), dim3(256), 0, s, N, alo, ilo, ihi, lab,
                     hid, vid, rowoff, st);
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, N + 1, 1, rowoff, &st->n_arms,
                     nullptr, nullptr);
  hipLaunchKernelGGL(k_arm_fill, dim3(ahi - alo + 1), dim3(1024), 0, s, N, alo, ilo, ihi, c->x0,
                     c->y0, h, M, lab,
                     hid, vid, rowoff, cr, c->geo.as<double>(), c->armpk.as<int>(),
                     c->armcoef.as<ArmCoef>(), st);
  hipLaunchKernelGGL(k_arm_coef, dim3(nblk(narm_cap, 256)), dim3(256), 0, s, narm_cap,
                     &st->n_arms, h, c->c2, c->armcoef.as<ArmCoef>());
  // markers / nodes
  hipLaunchKernelGGL(k_marker_ext, dim3(nblk(M, 64)), dim3(64), 0, s, M, c->X.as<double>(),
                     c->geo.as<double>(), c->x0, c->y0, h, N, c->c2, lab, c->ext.as<double>(),
                     need, c->mknode.as<int>());
  hipLaunchKernelGGL(k_need_rowcount, dim3(ghi - glo + 1), dim3(256), 0, s, N, glo, clo, chi, need,
                     rowcnt);
  // per-chunk node lists for the node-transform + extraction kernel
  const int MC = c->mk_chunk;
  const int nch = (M + MC - 1) / MC;
  KFBI_TRY(c->cnode.ensure(sizeof(int) * nch * 6 * MC));
  KFBI_TRY(c->ccount.ensure(sizeof(int) * nch));
  KFBI_TRY(c->chpos.ensure(sizeof(int) * nch));
  KFBI_TRY(c->mkloc.ensure(sizeof(int) * 6 * M));
  hipLaunchKernelGGL(k_chunk_nodes, dim3(nch), dim3(128), sizeof(int) * 12 * MC, s, M, MC,
                     c->mknode.as<int>(), c->cnode.as<int>(), c->ccount.as<int>(),
                     c->chpos.as<int>(), c->mkloc.as<int>());
  // node offsets, needed rows, band and row parts; posts the status for the host
  int* nodeoff = rowcnt + n1 + 1;
  int* rowpart = c->rowpart.as<int>();
  hipLaunchKernelGGL(k_rows_scan, dim3(1), dim3(1024), 0, s, N, rowcnt, nodeoff, c->rows.as<int>(),
                     c->rowptr.as<int>(), rowoff, rowpart, st, hs_dev);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(s));
  if (hs->err != 0) {
    static const char* msg[] = {"", "a grid segment is cut twice by the interface",
                                "grid labels and interface crossings disagree",
                                "interface marker closer than 3h to the box boundary",
                                "crossing buffer overflow", "crossing outside the grid"};
    set_error("geometry error: %s", msg[hs->err < 6 ? hs->err : 0]);
    return KFBI_E_GEOMETRY;
  }
  // row parts for the row transform kernel
  {
    const int P = hs->n_parts;
    KFBI_TRY(c->pdesc.ensure(sizeof(int4) * (P + 1)));
    const int ng = (N + 1 + 3) / 4;  // mode groups (cosine layout; the sine one needs fewer)
    KFBI_TRY(c->tmat.ensure(sizeof(double) * 4 * static_cast<size_t>(ng) * (P + 1) *
                            c->max_batch));
    hipLaunchKernelGGL(k_part_fill, dim3(nblk(N + 1, 256)), dim3(256), 0, s, N, rowoff, rowpart,
                       c->pdesc.as<int4>());
    // part-slot arm coefficients for the row transform kernel; the same launch zeroes the
    // per-apply corrections r (one copy per density of a batch; empty slots stay zero)
    const int cap = kArmsPerPart * (P > 0 ? P : 1);
    KFBI_TRY(c->armc.ensure(sizeof(double) * kArmCoefCount * cap));
    KFBI_TRY(c->armk.ensure(sizeof(int) * 2 * cap));
    KFBI_TRY(c->armsc.ensure(sizeof(double) * 2 * cap));
    KFBI_TRY(c->armr.ensure(sizeof(double) * cap * c->max_batch));
    c->arm_cap = cap;
    const int nmk = c->n_mk_blocks;
    KFBI_TRY(c->ckoff.ensure(sizeof(int) * (nmk + 1)));
    KFBI_TRY(c->cklist.ensure(sizeof(int) * cap));
    int* ckoff = c->ckoff.as<int>();
    hipLaunchKernelGGL(k_part_soa, dim3(nblk(cap, 256)), dim3(256), 0, s, P, cap,
                       c->pdesc.as<int4>(), c->armcoef.as<ArmCoef>(), c->armpk.as<int>(),
                       c->armc.as<double>(), c->armk.as<int>(), c->armr.as<double>(),
                       c->max_batch, N, c->sinT.as<double>(), c->armsc.as<double>());
    // chunk offsets (ckoff[nmk] = number of arms) and the slots of each chunk
    hipLaunchKernelGGL(k_chunk_arms, dim3(1), dim3(1024), sizeof(int) * (nmk + 1), s,
                       P > 0 ? cap : 0, c->mk_chunk, nmk, c->armk.as<int>(), ckoff,
                       c->cklist.as<int>());
    KFBI_TRY(c->ckcoef.ensure(sizeof(double) * kArmCoefCount * cap));
    KFBI_TRY(c->ckmk.ensure(sizeof(int) * cap));
    if (P > 0)
      hipLaunchKernelGGL(k_chunk_arm_pack, dim3(nblk(cap, 256)), dim3(256), 0, s, cap,
                         c->mk_chunk, ckoff + nmk, c->cklist.as<int>(), c->armc.as<double>(),
                         c->armk.as<int>(), c->ckcoef.as<double>(), c->ckmk.as<int>());
  }
  KFBI_HIP(hipGetLastError());
  c->st = *hs;
  c->M = M;
  c->gb_lo = glo;  // every entry this interface wrote lies in rows glo..ghi
  c->gb_hi = ghi;
  return KFBI_OK;
}

}  // namespace kfbi
