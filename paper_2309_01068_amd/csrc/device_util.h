// Small device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace kfbi {

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of one value per thread (blockDim.x a multiple of 64, <= 1024).
template <class T>
__device__ T block_sum(T v, T* scratch /* >= 16 entries in LDS */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  T r = 0;
  if (threadIdx.x < 64) {
    r = threadIdx.x < nw ? scratch[threadIdx.x] : T(0);
    r = wave_sum(r);
  }
  __syncthreads();
  if (threadIdx.x == 0) scratch[0] = r;
  __syncthreads();
  r = scratch[0];
  __syncthreads();
  return r;
}

// Block-wide exclusive prefix sum of ints (blockDim.x a multiple of 64, <= 1024).
__device__ inline int block_excl_scan(int v, int* scratch /* >= 17 ints */, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) scratch[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) {
      int t = scratch[i];
      scratch[i] = acc;
      acc += t;
    }
    scratch[16] = acc;
  }
  __syncthreads();
  int res = scratch[w] + incl - v;
  if (total) *total = scratch[16];
  __syncthreads();
  return res;
}

// 6-point Lagrange basis on the nodes t_m = m - 2 (markers k-2..k+3) and its derivative.
__device__ inline void lagrange6(double t, double* w, double* dw) {
  const double tm[6] = {-2.0, -1.0, 0.0, 1.0, 2.0, 3.0};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double denom = 1.0, prod = 1.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (q != m) {
        denom *= (tm[m] - tm[q]);
        prod *= (t - tm[q]);
      }
    w[m] = prod / denom;
    if (dw) {
      double d = 0.0;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        if (r == m) continue;
        double pr = 1.0;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (q != m && q != r) pr *= (t - tm[q]);
        d += pr;
      }
      dw[m] = d / denom;
    }
  }
}

// Jumps ([u], [u_x], [u_y], [u_xx], [u_yy], [u_xy]) at an interface point from the
// interface data of App. A.1 (2x2 and 3x3 systems solved in closed form through the
// tangential/normal frame: u_tt = R1/S, u_tn = R2/S, u_nn = R3 - u_tt, S = s_a^2).
__device__ inline void jumps_closed(double a, double b, double xaa, double yaa, double Phi,
                                    double Phia, double Phiaa, double Psi, double Psia, double c2,
                                    double* J) {
  const double S = a * a + b * b;
  const double s = sqrt(S);
  const double saa = (a * xaa + b * yaa) / s;
  const double ux = (a * Phia + b * s * Psi) / S;
  const double uy = (b * Phia - a * s * Psi) / S;
  const double R1 = Phiaa - xaa * ux - yaa * uy;
  const double R2 = saa * Psi + s * Psia - yaa * ux + xaa * uy;
  const double R3 = c2 * Phi;
  const double utt = R1 / S, utn = R2 / S, unn = R3 - utt;
  J[0] = Phi;
  J[1] = ux;
  J[2] = uy;
  J[3] = (a * a * utt + 2.0 * a * b * utn + b * b * unn) / S;
  J[4] = (b * b * utt - 2.0 * a * b * utn + a * a * unn) / S;
  J[5] = (a * b * utt + (b * b - a * a) * utn - a * b * unn) / S;
}

}  // namespace kfbi
