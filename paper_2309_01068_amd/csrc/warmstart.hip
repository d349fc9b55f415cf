// Learned initial guess for the theta-L pressure solve: a circular 1-D convolutional
// network (widths 5 -> 64 -> 64 -> 64 -> 1, 5 taps, SiLU) with hand-written bfloat16
// kernels that accumulate in FP32.  The two 64 -> 64 layers run on MFMA matrix cores
// (v_mfma_f32_16x16x16_bf16: per wavefront a 16 x 16 output tile, K = 16 per instruction),
// forward, backward-data and backward-weights; the 5 -> 64 and 64 -> 1 layers, the loss,
// Adam and the feature/assembly steps are plain vector kernels.
//
// Activation layout: channels last, [sample][marker][channel], bfloat16 (pre-activations
// Z in FP32 for the SiLU derivative).  Weights [out][tap][in] (and a transposed bfloat16
// copy [in][tap][out] of the 64 -> 64 layers for the data gradient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/warmstart.h"
#include "common.h"
#include "device_util.h"
#include "thetal_internal.h"

namespace kfbi {
namespace {

constexpr int kCin = 5, kW = 64, kTaps = 5, kPad = 2;
constexpr int kOW1 = 0, kOB1 = kOW1 + kW * kTaps * kCin;  // 1600
constexpr int kOW2 = kOB1 + kW, kOB2 = kOW2 + kW * kTaps * kW;
constexpr int kOW3 = kOB2 + kW, kOB3 = kOW3 + kW * kTaps * kW;
constexpr int kOW4 = kOB3 + kW, kOB4 = kOW4 + kTaps * kW;
constexpr int kNP = kOB4 + 1;  // 43073
constexpr int kMidLen = kW * kTaps * kW + kW;  // one 64 -> 64 layer: weights then biases
constexpr int kChunk = 128;  // positions per block in the weight-gradient kernels
// bfloat16 weight copies (element offsets, multiples of 4)
constexpr int kBW1 = 0, kBW2 = kBW1 + kW * kTaps * kCin, kBW2T = kBW2 + kW * kTaps * kW,
              kBW3 = kBW2T + kW * kTaps * kW, kBW3T = kBW3 + kW * kTaps * kW,
              kBW4 = kBW3T + kW * kTaps * kW, kBWCount = kBW4 + kTaps * kW;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf;

__device__ __forceinline__ bf f2bf(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<bf>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<bf>(u >> 16);
}
__device__ __forceinline__ float bf2f(bf h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float sg = 1.0f / (1.0f + expf(-z));
  return sg * (1.0f + z * (1.0f - sg));
}

// ------------------------------------------------------------------ features / assembly
// feat[k][0..4] = eta, L / L_ref, theta_a, phi1 / s1, (phi1 - phi2) / s2 with
// s1 = RMS(phi1), s2 = RMS(phi1 - phi2); s_out = (s2, s1).  One workgroup.
__global__ void __launch_bounds__(1024)
    k_ws_feat(int M, const double* __restrict__ eta, const double* __restrict__ tha,
              const double* __restrict__ phi1, const double* __restrict__ phi2,
              const double* __restrict__ scal, double L_ref, bf* __restrict__ feat,
              double* __restrict__ s_out) {
  __shared__ double red[32];
  double s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    const double d = phi1[k] - phi2[k];
    s1 += phi1[k] * phi1[k];
    s2 += d * d;
  }
  s1 = sqrt(block_sum<double>(s1, red) / M);
  s2 = sqrt(block_sum<double>(s2, red) / M);
  const double i1 = s1 > 0.0 ? 1.0 / s1 : 0.0, i2 = s2 > 0.0 ? 1.0 / s2 : 0.0;
  const double lf = scal[S_L] / L_ref;
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    bf* f = feat + 5 * k;
    f[0] = f2bf(static_cast<float>(eta[k]));
    f[1] = f2bf(static_cast<float>(lf));
    f[2] = f2bf(static_cast<float>(tha[k]));
    f[3] = f2bf(static_cast<float>(phi1[k] * i1));
    f[4] = f2bf(static_cast<float>((phi1[k] - phi2[k]) * i2));
  }
  if (threadIdx.x == 0) {
    s_out[0] = s2;
    s_out[1] = s1;
  }
}

// x0 = 2 phi1 - phi2 + s2 sigma y, or phi1 when s2 = 0 or any value is not finite; one
// workgroup.
__global__ void __launch_bounds__(1024)
    k_ws_assemble(int M, const double* __restrict__ phi1, const double* __restrict__ phi2,
                  const double* __restrict__ s_in, double sigma, const float* __restrict__ y,
                  double* __restrict__ x0) {
  const double s = s_in[0] * sigma;
  int bad = !(s_in[0] > 0.0);
  for (int k = threadIdx.x; k < M; k += blockDim.x) bad |= !isfinite(y[k]);
  bad = __syncthreads_or(bad);
  for (int k = threadIdx.x; k < M; k += blockDim.x)
    x0[k] = bad ? phi1[k] : 2.0 * phi1[k] - phi2[k] + s * static_cast<double>(y[k]);
}

// target (phi_n - 2 phi1 + phi2) / s2 (before the fixed target scale)
__global__ void k_ws_target(int M, const double* __restrict__ phin, const double* __restrict__ phi1,
                            const double* __restrict__ phi2, const double* __restrict__ s_in,
                            float* __restrict__ tgt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double s = s_in[0];
  tgt[k] = static_cast<float>((phin[k] - 2.0 * phi1[k] + phi2[k]) / s);
}

__global__ void k_ws_cast_feat(int n, const float* __restrict__ src, bf* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// Batch gather: sample idx[i] (or first + i when idx is null) of the set -> slot i, the
// target divided by the target scale.
__global__ void k_ws_gather(int B, int M, const int* __restrict__ idx, int first, float inv_sigma,
                            const bf* __restrict__ dfeat, const float* __restrict__ dtarg,
                            bf* __restrict__ X, float* __restrict__ T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * M) return;
  const int i = t / M, k = t % M;
  const size_t src = static_cast<size_t>(idx ? idx[i] : first + i) * M + k;
#pragma unroll
  for (int c = 0; c < kCin; ++c) X[static_cast<size_t>(t) * kCin + c] = dfeat[src * kCin + c];
  T[t] = dtarg[src] * inv_sigma;
}

// sum of squares of n floats -> acc[0] (one workgroup)
__global__ void k_ws_sumsq(long long n, const float* __restrict__ a, double* __restrict__ acc) {
  __shared__ double red[32];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) s += static_cast<double>(a[i]) * a[i];
  s = block_sum<double>(s, red);
  if (threadIdx.x == 0) acc[0] = s;
}

// ------------------------------------------------------------------------ layer 1 (5->64)
__global__ void k_l1_fwd(int B, int M, const bf* __restrict__ X, const bf* __restrict__ W,
                         const float* __restrict__ bias, float* __restrict__ Z,
                         bf* __restrict__ A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * M * kW) return;
  const int o = t & (kW - 1);
  const int bp = t >> 6;  // b * M + p
  const int b = bp / M, p = bp % M;
  float z = bias[o];
#pragma unroll
  for (int tp = 0; tp < kTaps; ++tp) {
    const int pp = (p + tp - kPad + M) & (M - 1);
    const bf* x = X + (static_cast<size_t>(b) * M + pp) * kCin;
#pragma unroll
    for (int c = 0; c < kCin; ++c) z += bf2f(W[(o * kTaps + tp) * kCin + c]) * bf2f(x[c]);
  }
  Z[t] = z;
  A[t] = f2bf(silu(z));
}

// ------------------------------------------------------------------ layers 2, 3 (64->64)
// MODE 0 (forward):  Z[b][p][o] = bias[o] + sum_t sum_c W[o][t][c] In[b][p+t-2][c],
//                    A = bf16(SiLU(Z)).
// MODE 1 (data gradient): G[b][p][c] = sum_t sum_o WT[c][t][o] dZ[b][p-t+2][o], then
//                    dZprev = bf16(G * SiLU'(Zprev)).
// One block = 16 positions of one sample; wavefront w = output channels 16w..16w+15.
template <int MODE>
__global__ void __launch_bounds__(256)
    k_mid(int M, const bf* __restrict__ W, const float* __restrict__ bias,
          const bf* __restrict__ In, const float* __restrict__ Zp, float* __restrict__ Zout,
          bf* __restrict__ Aout) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = l & 15, g = l >> 4;
  const int b = blockIdx.y, p0 = blockIdx.x * 16;
  const int p = p0 + n;
  const bf* inb = In + static_cast<size_t>(b) * M * kW;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int kk = 0; kk < 4 * kTaps; ++kk) {
    const int tp = kk >> 2, c0 = (kk & 3) * 16 + 4 * g;
    const s4 a = *reinterpret_cast<const s4*>(W + ((16 * w + n) * kTaps + tp) * kW + c0);
    const int pp = (MODE == 0 ? p + tp - kPad : p - tp + kPad + M) & (M - 1);
    const s4 bv = *reinterpret_cast<const s4*>(inb + static_cast<size_t>(pp) * kW + c0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc, 0, 0, 0);
  }
  const int o = 16 * w + 4 * g;  // rows 4g..4g+3 of this wavefront's tile
  const size_t base = (static_cast<size_t>(b) * M + p) * kW + o;
  if (MODE == 0) {
    f4 z;
    bf a4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      z[v] = acc[v] + bias[o + v];
      a4[v] = f2bf(silu(z[v]));
    }
    *reinterpret_cast<f4*>(Zout + base) = z;
    *reinterpret_cast<uint2*>(Aout + base) =
        make_uint2(a4[0] | (static_cast<uint32_t>(a4[1]) << 16),
                   a4[2] | (static_cast<uint32_t>(a4[3]) << 16));
  } else {
    const f4 zp = *reinterpret_cast<const f4*>(Zp + base);
    bf a4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) a4[v] = f2bf(acc[v] * dsilu(zp[v]));
    *reinterpret_cast<uint2*>(Aout + base) =
        make_uint2(a4[0] | (static_cast<uint32_t>(a4[1]) << 16),
                   a4[2] | (static_cast<uint32_t>(a4[3]) << 16));
  }
}

// Weight gradient of a 64 -> 64 layer over one chunk of 256 positions of one sample:
// part[o][t][c] = sum_q dZ[q][o] In[q+t-2][c], part[20480 + o] = sum_q dZ[q][o].
// MFMA with A = dZ^T (rows o, K = positions), B = shifted input (K = positions,
// columns (t, c)); both chunks staged in LDS.
__global__ void __launch_bounds__(256)
    k_mid_wgrad(int M, const bf* __restrict__ dZ, const bf* __restrict__ In,
                float* __restrict__ part) {
  __shared__ bf sdz[kChunk * kW];               // [q][o]
  __shared__ bf sin_[(kChunk + 2 * kPad) * kW];  // [q + 2][c], q = -2 .. 257
  const int nchunk = M / kChunk;
  const int b = blockIdx.x / nchunk, q0 = (blockIdx.x % nchunk) * kChunk;
  const bf* dzb = dZ + (static_cast<size_t>(b) * M + q0) * kW;
  const bf* inb = In + static_cast<size_t>(b) * M * kW;
  for (int e = threadIdx.x; e < kChunk * kW / 4; e += 256)
    reinterpret_cast<uint2*>(sdz)[e] = reinterpret_cast<const uint2*>(dzb)[e];
  for (int e = threadIdx.x; e < (kChunk + 2 * kPad) * kW / 4; e += 256) {
    const int r = e / (kW / 4), c4 = e % (kW / 4);
    const int q = (q0 + r - kPad + M) & (M - 1);
    reinterpret_cast<uint2*>(sin_)[e] =
        reinterpret_cast<const uint2*>(inb + static_cast<size_t>(q) * kW)[c4];
  }
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = l & 15, g = l >> 4;
  f4 acc[4 * kTaps];
#pragma unroll
  for (int j = 0; j < 4 * kTaps; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;
  for (int s = 0; s < kChunk / 16; ++s) {
    const int qa = 16 * s + 4 * g;  // K rows of this lane: positions qa .. qa+3
    s4 a;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bf h = sdz[(qa + v) * kW + 16 * w + n];
      a[v] = static_cast<short>(h);
      db += bf2f(h);
    }
#pragma unroll
    for (int j = 0; j < 4 * kTaps; ++j) {
      const int tp = j >> 2, c = 16 * (j & 3) + n;
      s4 bv;
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = static_cast<short>(sin_[(qa + v + tp) * kW + c]);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[j], 0, 0, 0);
    }
  }
  float* out = part + static_cast<size_t>(blockIdx.x) * kMidLen;
#pragma unroll
  for (int j = 0; j < 4 * kTaps; ++j) {
    const int tp = j >> 2, c = 16 * (j & 3) + n;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[((16 * w + 4 * g + v) * kTaps + tp) * kW + c] = acc[j][v];
  }
  db += __shfl_xor(db, 16, 64);
  db += __shfl_xor(db, 32, 64);
  if (g == 0) out[kW * kTaps * kW + 16 * w + n] = db;
}

// ----------------------------------------------------------------------- layer 4 (64->1)
__global__ void k_l4_fwd(int B, int M, const bf* __restrict__ A, const bf* __restrict__ W,
                         const float* __restrict__ bias, float* __restrict__ Y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * M) return;
  const int b = t / M, p = t % M;
  float y = bias[0];
#pragma unroll
  for (int tp = 0; tp < kTaps; ++tp) {
    const int pp = (p + tp - kPad + M) & (M - 1);
    const uint2* a = reinterpret_cast<const uint2*>(A + (static_cast<size_t>(b) * M + pp) * kW);
    const uint2* ww = reinterpret_cast<const uint2*>(W + tp * kW);
#pragma unroll 4
    for (int c4 = 0; c4 < kW / 4; ++c4) {
      const uint2 av = a[c4], wv = ww[c4];
      y += bf2f(av.x & 0xffff) * bf2f(wv.x & 0xffff) + bf2f(av.x >> 16) * bf2f(wv.x >> 16) +
           bf2f(av.y & 0xffff) * bf2f(wv.y & 0xffff) + bf2f(av.y >> 16) * bf2f(wv.y >> 16);
    }
  }
  Y[t] = y;
}

// dY = 2 (Y - T) / n_total, per-block sums of (Y - T)^2
__global__ void k_ws_loss(int n, float scale, const float* __restrict__ Y,
                          const float* __restrict__ T, float* __restrict__ dY,
                          float* __restrict__ lossp) {
  __shared__ float red[32];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float d = 0.f;
  if (t < n) {
    d = Y[t] - T[t];
    dY[t] = scale * d;
  }
  const float s = block_sum<float>(d * d, red);
  if (threadIdx.x == 0) lossp[blockIdx.x] = s;
}

// acc[0] += (sum of the block sums) / n_total, in block order; acc[1] = this batch's loss
__global__ void k_ws_loss_sum(int nb, double inv_n, const float* __restrict__ lossp,
                              double* __restrict__ acc) {
  __shared__ double red[32];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += lossp[i];
  s = block_sum<double>(s, red);
  if (threadIdx.x == 0) {
    acc[0] += s * inv_n;
    acc[1] = s * inv_n;
  }
}

// data gradient of layer 4 times SiLU'(Z3): dZ3[b][p][c] = bf16(SiLU'(Z3) sum_t W4[t][c] dY[p-t+2])
__global__ void k_l4_dgrad(int B, int M, const float* __restrict__ dY, const bf* __restrict__ W,
                           const float* __restrict__ Z3, bf* __restrict__ dZ3) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * M * kW) return;
  const int c = t & (kW - 1);
  const int bp = t >> 6;
  const int b = bp / M, p = bp % M;
  float g = 0.f;
#pragma unroll
  for (int tp = 0; tp < kTaps; ++tp)
    g += bf2f(W[tp * kW + c]) * dY[static_cast<size_t>(b) * M + ((p - tp + kPad + M) & (M - 1))];
  dZ3[t] = f2bf(g * dsilu(Z3[t]));
}

// weight gradient of layer 4 over one chunk: part[t*64 + c] = sum_q dY[q] A3[q+t-2][c],
// part[320] = sum_q dY[q]
__global__ void __launch_bounds__(256)
    k_l4_wgrad(int M, const float* __restrict__ dY, const bf* __restrict__ A,
               float* __restrict__ part) {
  __shared__ float sy[kChunk];
  const int nchunk = M / kChunk;
  const int b = blockIdx.x / nchunk, q0 = (blockIdx.x % nchunk) * kChunk;
  if (threadIdx.x < kChunk) sy[threadIdx.x] = dY[static_cast<size_t>(b) * M + q0 + threadIdx.x];
  __syncthreads();
  float* out = part + static_cast<size_t>(blockIdx.x) * (kTaps * kW + 1);
  for (int o = threadIdx.x; o <= kTaps * kW; o += 256) {
    float s = 0.f;
    if (o == kTaps * kW) {
      for (int q = 0; q < kChunk; ++q) s += sy[q];
    } else {
      const int tp = o / kW, c = o % kW;
      const bf* ab = A + static_cast<size_t>(b) * M * kW + c;
      for (int q = 0; q < kChunk; ++q)
        s += sy[q] * bf2f(ab[static_cast<size_t>((q0 + q + tp - kPad + M) & (M - 1)) * kW]);
    }
    out[o] = s;
  }
}

// weight gradient of layer 1 over one chunk: part[(o*5 + t)*5 + c] = sum_q dZ1[q][o] X[q+t-2][c],
// part[1600 + o] = sum_q dZ1[q][o]
__global__ void __launch_bounds__(256)
    k_l1_wgrad(int M, const bf* __restrict__ dZ, const bf* __restrict__ X,
               float* __restrict__ part) {
  __shared__ float sdz[kChunk][kW + 1];
  __shared__ float sx[kChunk + 2 * kPad][kCin];
  const int nchunk = M / kChunk;
  const int b = blockIdx.x / nchunk, q0 = (blockIdx.x % nchunk) * kChunk;
  for (int e = threadIdx.x; e < kChunk * kW; e += 256)
    sdz[e / kW][e % kW] = bf2f(dZ[(static_cast<size_t>(b) * M + q0) * kW + e]);
  for (int e = threadIdx.x; e < (kChunk + 2 * kPad) * kCin; e += 256) {
    const int r = e / kCin, c = e % kCin;
    const int q = (q0 + r - kPad + M) & (M - 1);
    sx[r][c] = bf2f(X[(static_cast<size_t>(b) * M + q) * kCin + c]);
  }
  __syncthreads();
  constexpr int nw = kW * kTaps * kCin;
  float* out = part + static_cast<size_t>(blockIdx.x) * (nw + kW);
  for (int e = threadIdx.x; e < nw + kW; e += 256) {
    float s = 0.f;
    if (e < nw) {
      const int o = e / (kTaps * kCin), tp = (e / kCin) % kTaps, c = e % kCin;
      for (int q = 0; q < kChunk; ++q) s += sdz[q][o] * sx[q + tp][c];
    } else {
      const int o = e - nw;
      for (int q = 0; q < kChunk; ++q) s += sdz[q][o];
    }
    out[e] = s;
  }
}

// grad[i] = sum over blocks of part[blk][i], in block order
__global__ void k_ws_reduce(int nblk, int len, const float* __restrict__ part,
                            float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += part[static_cast<size_t>(k) * len + i];
  grad[i] = s;
}

__global__ void k_ws_adam(int n, float lr, float b1, float b2, float eps, float bc1, float bc2,
                          float* __restrict__ th, const float* __restrict__ g,
                          float* __restrict__ m, float* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// bfloat16 working copies of the weights (and the transposed 64 -> 64 weights)
__global__ void k_ws_cast_w(const float* __restrict__ th, bf* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int n1 = kW * kTaps * kCin, n2 = kW * kTaps * kW, n4 = kTaps * kW;
  if (i < n1) wb[kBW1 + i] = f2bf(th[kOW1 + i]);
  if (i < n2) {
    const int o = i / (kTaps * kW), tp = (i / kW) % kTaps, c = i % kW;
    const int it = (c * kTaps + tp) * kW + o;
    const bf w2 = f2bf(th[kOW2 + i]), w3 = f2bf(th[kOW3 + i]);
    wb[kBW2 + i] = w2;
    wb[kBW3 + i] = w3;
    wb[kBW2T + it] = w2;
    wb[kBW3T + it] = w3;
  }
  if (i < n4) wb[kBW4 + i] = f2bf(th[kOW4 + i]);
}

// host-side counter-based generator (splitmix64) for initialisation and shuffling
uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
double unit(uint64_t seed, uint64_t i) {
  return static_cast<double>(splitmix64(seed * 0x100000001b3ull + i) >> 11) * 0x1.0p-53;
}

int nb(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

}  // namespace
}  // namespace kfbi

using namespace kfbi;

struct kfbi_ws {
  kfbi_ws_cfg cfg{};
  hipStream_t s = nullptr;
  int M = 0, Bmax = 0, cap = 0;
  int nsamp = 0;
  long adam_t = 0;
  int pending = 0, pending_n = -1;
  double sigma = 0.0;  // target scale (0 until set by the config or the first training)
  DBuf theta, m1, m2, grad, wb, X, T, Z1, Z2, Z3, A1, A2, A3, Y, dY, dZa, dZb, part, lossp,
      lacc, dfeat, dtarg, perm, pfeat, ps, pphi2;
  int* hperm = nullptr;
  double* hacc = nullptr;
};

namespace {

int ws_check(const kfbi_ws* ws) {
  if (!ws) {
    set_error("null warm-start object");
    return KFBI_E_INVALID;
  }
  return KFBI_OK;
}

void ws_free(kfbi_ws* ws) {
  for (DBuf* b : {&ws->theta, &ws->m1, &ws->m2, &ws->grad, &ws->wb, &ws->X, &ws->T, &ws->Z1,
                  &ws->Z2, &ws->Z3, &ws->A1, &ws->A2, &ws->A3, &ws->Y, &ws->dY, &ws->dZa,
                  &ws->dZb, &ws->part, &ws->lossp, &ws->lacc, &ws->dfeat, &ws->dtarg, &ws->perm,
                  &ws->pfeat, &ws->ps, &ws->pphi2})
    b->release();
  if (ws->hperm) (void)hipHostFree(ws->hperm);
  if (ws->hacc) (void)hipHostFree(ws->hacc);
  ws->hperm = nullptr;
  ws->hacc = nullptr;
}

const float* P(const kfbi_ws* ws, int off) { return ws->theta.as<float>() + off; }
const bf* WB(const kfbi_ws* ws, int off) { return ws->wb.as<bf>() + off; }

// forward pass of the B samples in X -> Y
void ws_forward(kfbi_ws* ws, int B) {
  const int M = ws->M;
  hipStream_t s = ws->s;
  hipLaunchKernelGGL(k_l1_fwd, dim3(nb(static_cast<long long>(B) * M * kW, 256)), dim3(256), 0, s,
                     B, M, ws->X.as<bf>(), WB(ws, kBW1), P(ws, kOB1), ws->Z1.as<float>(),
                     ws->A1.as<bf>());
  hipLaunchKernelGGL(k_mid<0>, dim3(M / 16, B), dim3(256), 0, s, M, WB(ws, kBW2), P(ws, kOB2),
                     ws->A1.as<bf>(), nullptr, ws->Z2.as<float>(), ws->A2.as<bf>());
  hipLaunchKernelGGL(k_mid<0>, dim3(M / 16, B), dim3(256), 0, s, M, WB(ws, kBW3), P(ws, kOB3),
                     ws->A2.as<bf>(), nullptr, ws->Z3.as<float>(), ws->A3.as<bf>());
  hipLaunchKernelGGL(k_l4_fwd, dim3(nb(static_cast<long long>(B) * M, 256)), dim3(256), 0, s, B,
                     M, ws->A3.as<bf>(), WB(ws, kBW4), P(ws, kOB4), ws->Y.as<float>());
}

// loss (accumulated into lacc[0], batch value in lacc[1]) and dY
void ws_loss(kfbi_ws* ws, int B) {
  const int n = B * ws->M;
  const int nbk = nb(n, 256);
  hipLaunchKernelGGL(k_ws_loss, dim3(nbk), dim3(256), 0, ws->s, n, 2.0f / n, ws->Y.as<float>(),
                     ws->T.as<float>(), ws->dY.as<float>(), ws->lossp.as<float>());
  hipLaunchKernelGGL(k_ws_loss_sum, dim3(1), dim3(256), 0, ws->s, nbk, 1.0 / n,
                     ws->lossp.as<float>(), ws->lacc.as<double>());
}

// backward pass (after ws_forward and ws_loss) -> grad
void ws_backward(kfbi_ws* ws, int B) {
  const int M = ws->M;
  hipStream_t s = ws->s;
  const int nblk = B * (M / kChunk);
  float* g = ws->grad.as<float>();
  float* part = ws->part.as<float>();
  // layer 4
  hipLaunchKernelGGL(k_l4_wgrad, dim3(nblk), dim3(256), 0, s, M, ws->dY.as<float>(),
                     ws->A3.as<bf>(), part);
  hipLaunchKernelGGL(k_ws_reduce, dim3(nb(kTaps * kW + 1, 256)), dim3(256), 0, s, nblk,
                     kTaps * kW + 1, part, g + kOW4);
  hipLaunchKernelGGL(k_l4_dgrad, dim3(nb(static_cast<long long>(B) * M * kW, 256)), dim3(256), 0,
                     s, B, M, ws->dY.as<float>(), WB(ws, kBW4), ws->Z3.as<float>(),
                     ws->dZa.as<bf>());
  // layer 3: weights from (dZ3, A2); data gradient -> dZ2
  hipLaunchKernelGGL(k_mid_wgrad, dim3(nblk), dim3(256), 0, s, M, ws->dZa.as<bf>(),
                     ws->A2.as<bf>(), part);
  hipLaunchKernelGGL(k_ws_reduce, dim3(nb(kMidLen, 256)), dim3(256), 0, s, nblk, kMidLen, part,
                     g + kOW3);
  hipLaunchKernelGGL(k_mid<1>, dim3(M / 16, B), dim3(256), 0, s, M, WB(ws, kBW3T), nullptr,
                     ws->dZa.as<bf>(), ws->Z2.as<float>(), nullptr, ws->dZb.as<bf>());
  // layer 2: weights from (dZ2, A1); data gradient -> dZ1
  hipLaunchKernelGGL(k_mid_wgrad, dim3(nblk), dim3(256), 0, s, M, ws->dZb.as<bf>(),
                     ws->A1.as<bf>(), part);
  hipLaunchKernelGGL(k_ws_reduce, dim3(nb(kMidLen, 256)), dim3(256), 0, s, nblk, kMidLen, part,
                     g + kOW2);
  hipLaunchKernelGGL(k_mid<1>, dim3(M / 16, B), dim3(256), 0, s, M, WB(ws, kBW2T), nullptr,
                     ws->dZb.as<bf>(), ws->Z1.as<float>(), nullptr, ws->dZa.as<bf>());
  // layer 1 weights from (dZ1, X)
  hipLaunchKernelGGL(k_l1_wgrad, dim3(nblk), dim3(256), 0, s, M, ws->dZa.as<bf>(),
                     ws->X.as<bf>(), part);
  hipLaunchKernelGGL(k_ws_reduce, dim3(nb(kW * kTaps * kCin + kW, 256)), dim3(256), 0, s, nblk,
                     kW * kTaps * kCin + kW, part, g + kOW1);
}

void ws_adam(kfbi_ws* ws) {
  ws->adam_t += 1;
  const float b1 = ws->cfg.beta1, b2 = ws->cfg.beta2;
  const float bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), ws->adam_t));
  const float bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), ws->adam_t));
  hipLaunchKernelGGL(k_ws_adam, dim3(nb(kNP, 256)), dim3(256), 0, ws->s, kNP, ws->cfg.lr, b1, b2,
                     ws->cfg.eps, bc1, bc2, ws->theta.as<float>(), ws->grad.as<float>(),
                     ws->m1.as<float>(), ws->m2.as<float>());
  hipLaunchKernelGGL(k_ws_cast_w, dim3(nb(kW * kTaps * kW, 256)), dim3(256), 0, ws->s,
                     ws->theta.as<float>(), ws->wb.as<bf>());
}

int ws_upload(kfbi_ws* ws, const float* host) {
  KFBI_HIP(hipMemcpyAsync(ws->theta.p, host, sizeof(float) * kNP, hipMemcpyHostToDevice, ws->s));
  KFBI_HIP(hipMemsetAsync(ws->m1.p, 0, sizeof(float) * kNP, ws->s));
  KFBI_HIP(hipMemsetAsync(ws->m2.p, 0, sizeof(float) * kNP, ws->s));
  hipLaunchKernelGGL(k_ws_cast_w, dim3(nb(kW * kTaps * kW, 256)), dim3(256), 0, ws->s,
                     ws->theta.as<float>(), ws->wb.as<bf>());
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(ws->s));
  ws->adam_t = 0;
  return KFBI_OK;
}

}  // namespace

extern "C" {

int kfbi_ws_create(const kfbi_ws_cfg* cfg, kfbi_ws** out) {
  if (!cfg || !out) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *out = nullptr;
  const int M = cfg->M;
  if (M < kChunk || M > kTLMaxM || (M & (M - 1)) || cfg->max_batch < 1 || cfg->capacity < 1 ||
      !(cfg->L_ref > 0.0) || !(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
      !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f) ||
      !(cfg->target_scale >= 0.0)) {
    set_error("kfbi_ws_create: M a power of two in [%d, %d], max_batch >= 1, capacity >= 1, "
              "L_ref > 0, lr > 0, 0 <= beta < 1, eps > 0, target_scale >= 0", kChunk, kTLMaxM);
    return KFBI_E_INVALID;
  }
  kfbi_ws* ws = new (std::nothrow) kfbi_ws();
  if (!ws) {
    set_error("out of host memory");
    return KFBI_E_NOMEM;
  }
  ws->cfg = *cfg;
  ws->s = static_cast<hipStream_t>(cfg->stream);
  ws->M = M;
  ws->Bmax = cfg->max_batch;
  ws->cap = cfg->capacity;
  ws->sigma = cfg->target_scale;
  const size_t BM = static_cast<size_t>(ws->Bmax) * M;
  const size_t nblk = static_cast<size_t>(ws->Bmax) * (M / kChunk);
  int st = KFBI_OK;
  if ((st = ws->theta.ensure(sizeof(float) * kNP)) || (st = ws->m1.ensure(sizeof(float) * kNP)) ||
      (st = ws->m2.ensure(sizeof(float) * kNP)) || (st = ws->grad.ensure(sizeof(float) * kNP)) ||
      (st = ws->wb.ensure(sizeof(bf) * kBWCount)) || (st = ws->X.ensure(sizeof(bf) * BM * kCin)) ||
      (st = ws->T.ensure(sizeof(float) * BM)) || (st = ws->Z1.ensure(sizeof(float) * BM * kW)) ||
      (st = ws->Z2.ensure(sizeof(float) * BM * kW)) || (st = ws->Z3.ensure(sizeof(float) * BM * kW)) ||
      (st = ws->A1.ensure(sizeof(bf) * BM * kW)) || (st = ws->A2.ensure(sizeof(bf) * BM * kW)) ||
      (st = ws->A3.ensure(sizeof(bf) * BM * kW)) || (st = ws->Y.ensure(sizeof(float) * BM)) ||
      (st = ws->dY.ensure(sizeof(float) * BM)) || (st = ws->dZa.ensure(sizeof(bf) * BM * kW)) ||
      (st = ws->dZb.ensure(sizeof(bf) * BM * kW)) ||
      (st = ws->part.ensure(sizeof(float) * nblk * kMidLen)) ||
      (st = ws->lossp.ensure(sizeof(float) * (BM / 256 + 1))) ||
      (st = ws->lacc.ensure(sizeof(double) * 2)) ||
      (st = ws->dfeat.ensure(sizeof(bf) * static_cast<size_t>(ws->cap) * M * kCin)) ||
      (st = ws->dtarg.ensure(sizeof(float) * static_cast<size_t>(ws->cap) * M)) ||
      (st = ws->perm.ensure(sizeof(int) * ws->cap)) ||
      (st = ws->pfeat.ensure(sizeof(bf) * M * kCin)) || (st = ws->ps.ensure(2 * sizeof(double))) ||
      (st = ws->pphi2.ensure(sizeof(double) * M))) {
    ws_free(ws);
    delete ws;
    return st;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&ws->hperm), sizeof(int) * ws->cap,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ws->hacc), sizeof(double) * 2,
                    hipHostMallocDefault) != hipSuccess) {
    ws_free(ws);
    delete ws;
    set_error("hipHostMalloc failed");
    return KFBI_E_NOMEM;
  }
  // seeded initialisation: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for layers 1-3, zero for the
  // output layer (the initial guess starts as the linear extrapolation)
  std::vector<float> h(kNP, 0.f);
  const int lay[3][3] = {{kOW1, kOB1, kCin * kTaps}, {kOW2, kOB2, kW * kTaps}, {kOW3, kOB3, kW * kTaps}};
  for (const auto& L : lay) {
    const double bound = 1.0 / std::sqrt(static_cast<double>(L[2]));
    for (int i = L[0]; i < L[1] + kW; ++i)
      h[i] = static_cast<float>((2.0 * unit(cfg->seed, i) - 1.0) * bound);
  }
  st = ws_upload(ws, h.data());
  if (st != KFBI_OK) {
    ws_free(ws);
    delete ws;
    return st;
  }
  *out = ws;
  return KFBI_OK;
}

int kfbi_ws_destroy(kfbi_ws* ws) {
  if (!ws) return KFBI_OK;
  (void)hipStreamSynchronize(ws->s);
  ws_free(ws);
  delete ws;
  return KFBI_OK;
}

int kfbi_ws_n_params(const kfbi_ws* ws, int* n) {
  KFBI_TRY(ws_check(ws));
  if (!n) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *n = kNP;
  return KFBI_OK;
}

int kfbi_ws_get_weights(const kfbi_ws* ws, float* host) {
  KFBI_TRY(ws_check(ws));
  if (!host) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  KFBI_HIP(hipMemcpyAsync(host, ws->theta.p, sizeof(float) * kNP, hipMemcpyDeviceToHost, ws->s));
  KFBI_HIP(hipStreamSynchronize(ws->s));
  return KFBI_OK;
}

int kfbi_ws_set_weights(kfbi_ws* ws, const float* host) {
  KFBI_TRY(ws_check(ws));
  if (!host) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  return ws_upload(ws, host);
}

int kfbi_ws_predict(kfbi_ws* ws, thetaL* th, double* x0) {
  KFBI_TRY(ws_check(ws));
  if (!th || !th->ready || th->M != ws->M) {
    set_error("kfbi_ws_predict: need an initialised thetaL object with the same M");
    return th && !th->ready ? KFBI_E_STATE : KFBI_E_INVALID;
  }
  const int M = ws->M;
  hipStream_t s = ws->s;
  ws->pending = 0;
  if (th->n < 2) {  // no two previous solves yet: the previous density
    if (x0) KFBI_HIP(hipMemcpyAsync(x0, th->phi.p, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
    return KFBI_OK;
  }
  KFBI_TRY(thetal_refresh(th));
  hipLaunchKernelGGL(k_ws_feat, dim3(1), dim3(1024), 0, s, M, th->eta.as<double>(),
                     th->aux.as<double>() + A_THA * M, th->phi.as<double>(), th->phi2.as<double>(),
                     th->scal.as<double>(), ws->cfg.L_ref, ws->pfeat.as<bf>(), ws->ps.as<double>());
  KFBI_HIP(hipMemcpyAsync(ws->pphi2.p, th->phi2.p, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  if (x0) {
    KFBI_HIP(hipMemcpyAsync(ws->X.p, ws->pfeat.p, sizeof(bf) * M * kCin, hipMemcpyDeviceToDevice, s));
    ws_forward(ws, 1);
    hipLaunchKernelGGL(k_ws_assemble, dim3(1), dim3(1024), 0, s, M, th->phi.as<double>(),
                       th->phi2.as<double>(), ws->ps.as<double>(), ws->sigma, ws->Y.as<float>(),
                       x0);
  }
  KFBI_HIP(hipGetLastError());
  ws->pending = 1;
  ws->pending_n = th->n;
  return KFBI_OK;
}

int kfbi_ws_record(kfbi_ws* ws, thetaL* th, int* stored) {
  KFBI_TRY(ws_check(ws));
  if (!th || th->M != ws->M) {
    set_error("kfbi_ws_record: thetaL object with a different M");
    return KFBI_E_INVALID;
  }
  if (stored) *stored = 0;
  if (!ws->pending || th->n != ws->pending_n + 1 || ws->nsamp >= ws->cap) {
    ws->pending = 0;
    return KFBI_OK;
  }
  const int M = ws->M;
  hipStream_t s = ws->s;
  // after the step: th->phi = phi_n, th->phi2 = phi1 of the pending state
  hipLaunchKernelGGL(k_ws_target, dim3(nb(M, 256)), dim3(256), 0, s, M, th->phi.as<double>(),
                     th->phi2.as<double>(), ws->pphi2.as<double>(), ws->ps.as<double>(),
                     ws->dtarg.as<float>() + static_cast<size_t>(ws->nsamp) * M);
  KFBI_HIP(hipMemcpyAsync(ws->dfeat.as<bf>() + static_cast<size_t>(ws->nsamp) * M * kCin,
                          ws->pfeat.p, sizeof(bf) * M * kCin, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipGetLastError());
  ws->nsamp += 1;
  ws->pending = 0;
  if (stored) *stored = 1;
  return KFBI_OK;
}

int kfbi_ws_n_samples(const kfbi_ws* ws, int* n) {
  KFBI_TRY(ws_check(ws));
  if (!n) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *n = ws->nsamp;
  return KFBI_OK;
}

int kfbi_ws_clear(kfbi_ws* ws) {
  KFBI_TRY(ws_check(ws));
  ws->nsamp = 0;
  ws->pending = 0;
  return KFBI_OK;
}

int kfbi_ws_train(kfbi_ws* ws, int n_train, int epochs, int batch, float* loss_host) {
  KFBI_TRY(ws_check(ws));
  if (n_train < 1 || n_train > ws->nsamp || epochs < 0 || batch < 1 || batch > ws->Bmax ||
      batch > n_train) {
    set_error("kfbi_ws_train: need 1 <= batch <= min(max_batch, n_train), n_train <= samples");
    return KFBI_E_INVALID;
  }
  hipStream_t s = ws->s;
  const int nbatch = n_train / batch;
  if (ws->sigma == 0.0) {  // target scale: RMS of the stored targets of the training set
    const long long n = static_cast<long long>(n_train) * ws->M;
    hipLaunchKernelGGL(k_ws_sumsq, dim3(1), dim3(1024), 0, s, n, ws->dtarg.as<float>(),
                       ws->lacc.as<double>());
    KFBI_HIP(hipMemcpyAsync(ws->hacc, ws->lacc.p, sizeof(double), hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    const double rms = std::sqrt(ws->hacc[0] / static_cast<double>(n));
    if (!(rms > 0.0) || !std::isfinite(rms)) {
      set_error("kfbi_ws_train: the stored targets have no finite positive scale");
      return KFBI_E_NONFINITE;
    }
    ws->sigma = rms;
  }
  const float inv_sigma = static_cast<float>(1.0 / ws->sigma);
  for (int e = 0; e < epochs; ++e) {
    // seeded Fisher-Yates shuffle of [0, n_train)
    for (int i = 0; i < n_train; ++i) ws->hperm[i] = i;
    const uint64_t es = splitmix64(ws->cfg.seed ^ (0xabcdef12345ull + static_cast<uint64_t>(ws->adam_t)));
    for (int i = n_train - 1; i > 0; --i) {
      const int j = static_cast<int>(splitmix64(es + static_cast<uint64_t>(i)) % static_cast<uint64_t>(i + 1));
      const int t = ws->hperm[i];
      ws->hperm[i] = ws->hperm[j];
      ws->hperm[j] = t;
    }
    KFBI_HIP(hipMemcpyAsync(ws->perm.p, ws->hperm, sizeof(int) * n_train, hipMemcpyHostToDevice, s));
    KFBI_HIP(hipMemsetAsync(ws->lacc.p, 0, sizeof(double) * 2, s));
    for (int bi = 0; bi < nbatch; ++bi) {
      hipLaunchKernelGGL(k_ws_gather, dim3(nb(static_cast<long long>(batch) * ws->M, 256)),
                         dim3(256), 0, s, batch, ws->M, ws->perm.as<int>() + bi * batch, 0,
                         inv_sigma, ws->dfeat.as<bf>(), ws->dtarg.as<float>(), ws->X.as<bf>(),
                         ws->T.as<float>());
      ws_forward(ws, batch);
      ws_loss(ws, batch);
      ws_backward(ws, batch);
      ws_adam(ws);
    }
    KFBI_HIP(hipGetLastError());
    KFBI_HIP(hipMemcpyAsync(ws->hacc, ws->lacc.p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    if (loss_host) loss_host[e] = static_cast<float>(ws->hacc[0] / nbatch);
  }
  return KFBI_OK;
}

int kfbi_ws_eval(kfbi_ws* ws, int first, int count, float* loss_host) {
  KFBI_TRY(ws_check(ws));
  if (!loss_host || first < 0 || count < 1 || first + count > ws->nsamp) {
    set_error("kfbi_ws_eval: sample range outside the stored set");
    return KFBI_E_INVALID;
  }
  if (!(ws->sigma > 0.0)) {
    set_error("kfbi_ws_eval: no target scale yet (train first or set target_scale)");
    return KFBI_E_STATE;
  }
  hipStream_t s = ws->s;
  const float inv_sigma = static_cast<float>(1.0 / ws->sigma);
  KFBI_HIP(hipMemsetAsync(ws->lacc.p, 0, sizeof(double) * 2, s));
  double weighted = 0.0;
  for (int i = first; i < first + count; i += ws->Bmax) {
    const int B = std::min(ws->Bmax, first + count - i);
    hipLaunchKernelGGL(k_ws_gather, dim3(nb(static_cast<long long>(B) * ws->M, 256)), dim3(256),
                       0, s, B, ws->M, nullptr, i, inv_sigma, ws->dfeat.as<bf>(), ws->dtarg.as<float>(),
                       ws->X.as<bf>(), ws->T.as<float>());
    ws_forward(ws, B);
    ws_loss(ws, B);
    KFBI_HIP(hipMemcpyAsync(ws->hacc, ws->lacc.p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    weighted += ws->hacc[1] * B;
  }
  KFBI_HIP(hipGetLastError());
  *loss_host = static_cast<float>(weighted / count);
  return KFBI_OK;
}

int kfbi_ws_forward(kfbi_ws* ws, int B, const float* feat, float* out) {
  KFBI_TRY(ws_check(ws));
  if (!feat || !out || B < 1 || B > ws->Bmax) {
    set_error("kfbi_ws_forward: null array or B outside [1, max_batch]");
    return KFBI_E_INVALID;
  }
  const long long n = static_cast<long long>(B) * ws->M;
  hipLaunchKernelGGL(k_ws_cast_feat, dim3(nb(n * kCin, 256)), dim3(256), 0, ws->s,
                     static_cast<int>(n * kCin), feat, ws->X.as<bf>());
  ws_forward(ws, B);
  KFBI_HIP(hipMemcpyAsync(out, ws->Y.p, sizeof(float) * n, hipMemcpyDeviceToDevice, ws->s));
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int kfbi_ws_backward(kfbi_ws* ws, int B, const float* feat, const float* target, float* grad,
                     float* loss_host) {
  KFBI_TRY(ws_check(ws));
  if (!feat || !target || !grad || !loss_host || B < 1 || B > ws->Bmax) {
    set_error("kfbi_ws_backward: null array or B outside [1, max_batch]");
    return KFBI_E_INVALID;
  }
  hipStream_t s = ws->s;
  const long long n = static_cast<long long>(B) * ws->M;
  hipLaunchKernelGGL(k_ws_cast_feat, dim3(nb(n * kCin, 256)), dim3(256), 0, s,
                     static_cast<int>(n * kCin), feat, ws->X.as<bf>());
  KFBI_HIP(hipMemcpyAsync(ws->T.p, target, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemsetAsync(ws->lacc.p, 0, sizeof(double) * 2, s));
  ws_forward(ws, B);
  ws_loss(ws, B);
  ws_backward(ws, B);
  KFBI_HIP(hipMemcpyAsync(grad, ws->grad.p, sizeof(float) * kNP, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(ws->hacc, ws->lacc.p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(s));
  *loss_host = static_cast<float>(ws->hacc[1]);
  return KFBI_OK;
}

}  // extern "C"

extern "C" int kfbi_ws_target_scale(const kfbi_ws* ws, double* sigma) {
  KFBI_TRY(ws_check(ws));
  if (!sigma) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *sigma = ws->sigma;
  return KFBI_OK;
}
