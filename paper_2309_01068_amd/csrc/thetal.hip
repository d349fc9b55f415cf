// theta-L / small-scale-decomposition Hele-Shaw evolution on gfx950 (Sec. 5), driving the
// KFBI pressure solve of eq. bie-HS through the kfbi C ABI.
//
// Per step: k_tl_pre (one workgroup) reconstructs the markers from (eta, L, Xbar) and
// forms the right-hand side -sigma kappa - v; kfbi_set_interface rebuilds the grid
// geometry; GMRES finds the density, its last apply (the true residual at the solution)
// also gives d_n(D phi);
// k_tl_post (one workgroup) forms U, V, the explicit term, and advances eta (integrating
// factor AB2 in Fourier space), L and Xbar (AB2).  All spectral operations are radix-2
// Stockham FFTs of length M held in LDS, FP64.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <new>
#include <utility>

#include "common.h"
#include "device_util.h"
#include "thetal_internal.h"

namespace kfbi {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;


__device__ __forceinline__ int wavenum(int q, int M) {  // signed wavenumber, Nyquist -> 0
  const int h = M >> 1;
  return q < h ? q : (q == h ? 0 : q - M);
}

// Radix-2 Stockham FFT of length M (power of two) on LDS arrays; (xr, xi) holds the input
// and, on return, the output (the pointers are swapped as the passes ping-pong).  The
// inverse is unscaled.  Twiddles tw[k] = exp(-2 pi i k / M), k < M/2, in LDS.
__device__ void fft_lds(double*& xr, double*& xi, double*& yr, double*& yi,
                        const double* __restrict__ twr, const double* __restrict__ twi, int M,
                        bool inverse) {
  const int h = M >> 1;
  for (int ns = 1; ns < M; ns <<= 1) {
    const int stride = M / (2 * ns);
    for (int j = threadIdx.x; j < h; j += blockDim.x) {
      const int k = j & (ns - 1);
      const double ar = xr[j], ai = xi[j], br = xr[j + h], bi = xi[j + h];
      const double wr = twr[k * stride];
      const double wi = inverse ? -twi[k * stride] : twi[k * stride];
      const double tr = br * wr - bi * wi, ti = br * wi + bi * wr;
      const int d = ((j - k) << 1) + k;
      yr[d] = ar + tr;
      yi[d] = ai + ti;
      yr[d + ns] = ar - tr;
      yi[d + ns] = ai - ti;
    }
    __syncthreads();
    double* t = xr;
    xr = yr;
    yr = t;
    t = xi;
    xi = yi;
    yi = t;
  }
}

struct TLShared {
  double *xr, *xi, *yr, *yi, *twr, *twi, *red;
  __device__ void setup(double* lds, int M, const double* __restrict__ tw) {
    xr = lds;
    xi = xr + M;
    yr = xi + M;
    yi = yr + M;
    twr = yi + M;
    twi = twr + M / 2;
    red = twi + M / 2;
    for (int k = threadIdx.x; k < M / 2; k += blockDim.x) {
      twr[k] = tw[2 * k];
      twi[k] = tw[2 * k + 1];
    }
    __syncthreads();
  }
};
inline size_t tl_lds_bytes(int M) { return sizeof(double) * (5 * static_cast<size_t>(M) + 32); }

// Problem of the step: Hele-Shaw (stefan = 0: right-hand side -sigma kappa + J ln|x|, U from
// the pressure) or Stefan (right-hand side -eps_C kappa, eps_V per marker, U = psi); pw = 3
// for the L_2 term lambda (2pi/L)^3 H[theta_aaa], 2 for L_1 = lambda (2pi/L)^2 theta_aa.
struct Aniso {
  double e0, e1, e2, m, p0;
  __device__ double at(double phi) const {
    return e0 * (1.0 + e1 * cos(m * (phi - p0)) + e2 * cos(2.0 * m * (phi - p0)));
  }
};
struct TLMode {
  int stefan;
  int pw;
  Aniso ec, ev;
};

// ---------------------------------------------------------------------------- pre-step
// Reconstruction (Sec. 5.1): theta = alpha + eta, X = Xbar + (L/2pi) A[exp(i theta)] with
// the mean-free antiderivative A; eta_a and H[eta_aaa] (Sec. 5.2.1); curvature
// kappa = (2pi/L) theta_a; right-hand side -sigma kappa + J ln|x| (eq. bie-HS with
// v = -J ln|x|); area (1/2) int (x y_a - y x_a) da.
__global__ void __launch_bounds__(kTLThreads)
    k_tl_pre(int M, double sigma, double J, const double* __restrict__ tw,
             const double* __restrict__ eta, double* __restrict__ scal, double* __restrict__ X,
             double* __restrict__ rhs, double* __restrict__ aux, double* __restrict__ etahat,
             TLMode md, double* __restrict__ amk, const double* __restrict__ guess,
             double* __restrict__ xw) {
  extern __shared__ double lds[];
  TLShared sh;
  sh.setup(lds, M, tw);
  const int tid = threadIdx.x;
  if (xw)  // the GMRES initial guess into the working density
    for (int j = tid; j < M; j += blockDim.x) xw[j] = guess[j];
  const double L = scal[S_L], xbx = scal[S_XBX], xby = scal[S_XBY];
  const double invM = 1.0 / M;
  // exp(i theta)
  for (int j = tid; j < M; j += blockDim.x) {
    double s, c;
    sincos(kTwoPi * j * invM + eta[j], &s, &c);
    sh.xr[j] = c;
    sh.xi[j] = s;
  }
  __syncthreads();
  fft_lds(sh.xr, sh.xi, sh.yr, sh.yi, sh.twr, sh.twi, M, false);
  // keep zhat (k = 0 and Nyquist removed) in registers for the tangent; antiderivative
  constexpr int U = kTLMaxM / kTLThreads;
  double zr[U], zi[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * kTLThreads;
    zr[u] = zi[u] = 0.0;
    if (q < M) {
      const int k = wavenum(q, M);
      const double a = sh.xr[q], b = sh.xi[q];
      if (k != 0) {
        zr[u] = a;
        zi[u] = b;
      }
      sh.yr[q] = (k != 0) ? b / k : 0.0;
      sh.yi[q] = (k != 0) ? -a / k : 0.0;
    }
  }
  __syncthreads();
  fft_lds(sh.yr, sh.yi, sh.xr, sh.xi, sh.twr, sh.twi, M, true);
  const double sc = L / kTwoPi * invM;
  double xs[U], ys[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = tid + u * kTLThreads;
    if (j < M) {
      xs[u] = xbx + sc * sh.yr[j];
      ys[u] = xby + sc * sh.yi[j];
    }
  }
  __syncthreads();
  // tangent X_a + i Y_a = (L/2pi) IFFT(zhat without k = 0, Nyquist)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * kTLThreads;
    if (q < M) {
      sh.xr[q] = zr[u];
      sh.xi[q] = zi[u];
    }
  }
  __syncthreads();
  fft_lds(sh.xr, sh.xi, sh.yr, sh.yi, sh.twr, sh.twi, M, true);
  double ar = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = tid + u * kTLThreads;
    if (j < M) ar += xs[u] * (sc * sh.xi[j]) - ys[u] * (sc * sh.xr[j]);
  }
  ar = block_sum<double>(ar, sh.red);
  // eta_hat, then eta_a + i H[eta_aaa] (multipliers ik and -|k|^3)
  for (int j = tid; j < M; j += blockDim.x) {
    sh.xr[j] = eta[j];
    sh.xi[j] = 0.0;
  }
  __syncthreads();
  fft_lds(sh.xr, sh.xi, sh.yr, sh.yi, sh.twr, sh.twi, M, false);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * kTLThreads;
    if (q < M) {
      const double er = sh.xr[q], ei = sh.xi[q];
      etahat[2 * q] = er;
      etahat[2 * q + 1] = ei;
      const double k = wavenum(q, M);
      // H[eta_aaa] (multiplier -|k|^3) or eta_aa (multiplier -k^2)
      const double k3 = md.pw == 2 ? k * k : fabs(k) * k * k;
      sh.yr[q] = -k * ei + k3 * ei;
      sh.yi[q] = k * er - k3 * er;
    }
  }
  __syncthreads();
  fft_lds(sh.yr, sh.yi, sh.xr, sh.xi, sh.twr, sh.twi, M, true);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = tid + u * kTLThreads;
    if (j < M) {
      const double eta_a = sh.yr[j] * invM, heta = sh.yi[j] * invM;
      const double tha = 1.0 + eta_a;
      const double kappa = kTwoPi / L * tha;
      const double r2 = xs[u] * xs[u] + ys[u] * ys[u];
      double s, c;
      sincos(kTwoPi * j * invM + eta[j], &s, &c);
      X[j] = xs[u];
      X[M + j] = ys[u];
      if (md.stefan) {
        // angle of the outward normal n = (sin theta, -cos theta): theta - pi/2
        const double nphi = kTwoPi * j * invM + eta[j] - 0.5 * M_PI;
        rhs[j] = -md.ec.at(nphi) * kappa;
        amk[j] = md.ev.at(nphi);
      } else {
        rhs[j] = -sigma * kappa + J * 0.5 * log(r2);
      }
      aux[A_THA * M + j] = tha;
      aux[A_HETA * M + j] = heta;
      aux[A_NX * M + j] = s;
      aux[A_NY * M + j] = -c;
      aux[A_R2 * M + j] = r2;
    }
  }
  if (tid == 0) {
    scal[S_AREA] = 0.5 * ar * kTwoPi * invM;
    scal[S_LEN] = L;
  }
}

// --------------------------------------------------------------------------- post-step
// U = J (x.n)/|x|^2 - (d_n+ + d_n-)/2 of D phi; M_dot = int theta_a U da;
// V = -(int_0^a theta_a U - mean part) (eq. L-evo/the-evo); Qbar = mean(U n + V s);
// explicit term N = (2pi/L)(theta_a V - U_a) - lambda2 (2pi/L)^3 H[eta_aaa]; then the
// integrating-factor step for eta_hat (eq. Fourier-theta2), AB2 (or Euler at n = 0) for
// L and Xbar.
__global__ void __launch_bounds__(kTLThreads)
    k_tl_post(int M, double J, double tau, double lam2, int first,
              const double* __restrict__ tw, const double* __restrict__ X,
              double* __restrict__ aux, const double* __restrict__ dnp,
              const double* __restrict__ dnm, const double* __restrict__ etahat,
              double* __restrict__ nhat_prev, double* __restrict__ scal,
              double* __restrict__ eta, const double* __restrict__ psi, int pw,
              double* __restrict__ hscal) {
  extern __shared__ double lds[];
  TLShared sh;
  sh.setup(lds, M, tw);
  const int tid = threadIdx.x;
  const double invM = 1.0 / M;
  const double L = scal[S_L];
  constexpr int U = kTLMaxM / kTLThreads;
  double uu[U], tha[U], nx[U], ny[U], he[U];
  double gs = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = tid + u * kTLThreads;
    if (j < M) {
      tha[u] = aux[A_THA * M + j];
      he[u] = aux[A_HETA * M + j];
      nx[u] = aux[A_NX * M + j];
      ny[u] = aux[A_NY * M + j];
      const double r2 = aux[A_R2 * M + j];
      const double x = X[j], y = X[M + j];
      uu[u] = psi ? psi[j] : J * (x * nx[u] + y * ny[u]) / r2 - 0.5 * (dnp[j] + dnm[j]);
      aux[A_U * M + j] = uu[u];
      const double g = tha[u] * uu[u];
      sh.xr[j] = g;
      sh.xi[j] = uu[u];
      gs += g;
    }
  }
  gs = block_sum<double>(gs, sh.red);  // (synchronises: the FFT input is complete)
  const double Mdot = kTwoPi * gs * invM;
  fft_lds(sh.xr, sh.xi, sh.yr, sh.yi, sh.twr, sh.twi, M, false);
  // split F = FFT(g + iU) into G_hat and U_hat; spectrum of A[g] + i U_a
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * kTLThreads;
    if (q < M) {
      const int qm = (M - q) & (M - 1);
      const double fr = sh.xr[q], fi = sh.xi[q], cr = sh.xr[qm], ci = -sh.xi[qm];
      const double gr = 0.5 * (fr + cr), gi = 0.5 * (fi + ci);
      const double ur = 0.5 * (fi - ci), ui = -0.5 * (fr - cr);
      const int k = wavenum(q, M);
      sh.yr[q] = (k != 0) ? gi / k - k * ur : 0.0;
      sh.yi[q] = (k != 0) ? -gr / k - k * ui : 0.0;
    }
  }
  __syncthreads();
  fft_lds(sh.yr, sh.yi, sh.xr, sh.xi, sh.twr, sh.twi, M, true);
  const double A0 = sh.yr[0] * invM;
  const double w = kTwoPi / L;
  double qx = 0.0, qy = 0.0;
  double nv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = tid + u * kTLThreads;
    if (j < M) {
      const double A = sh.yr[j] * invM, Ua = sh.yi[j] * invM;
      const double V = -(A - A0);
      const double sx = -ny[u], sy = nx[u];
      qx += uu[u] * nx[u] + V * sx;
      qy += uu[u] * ny[u] + V * sy;
      nv[u] = w * (tha[u] * V - Ua) - lam2 * (pw == 2 ? w * w : w * w * w) * he[u];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = tid + u * kTLThreads;
    if (j < M) {
      sh.xr[j] = nv[u];
      sh.xi[j] = 0.0;
    }
  }
  qx = block_sum<double>(qx, sh.red);
  qy = block_sum<double>(qy, sh.red);
  qx *= invM;
  qy *= invM;
  fft_lds(sh.xr, sh.xi, sh.yr, sh.yi, sh.twr, sh.twi, M, false);
  // scalars (every thread computes the same values)
  const double xbx = scal[S_XBX], xby = scal[S_XBY];
  double Ln, xn, yn;
  if (first) {
    Ln = L + tau * Mdot;
    xn = xbx + tau * qx;
    yn = xby + tau * qy;
  } else {
    Ln = L + 0.5 * tau * (3.0 * Mdot - scal[S_MPREV]);
    xn = xbx + 0.5 * tau * (3.0 * qx - scal[S_QPX]);
    yn = xby + 0.5 * tau * (3.0 * qy - scal[S_QPY]);
  }
  const double Lp = scal[S_LPREV];
  auto ipw = [pw](double x) { return pw == 2 ? 1.0 / (x * x) : 1.0 / (x * x * x); };
  const double c1 = 0.5 * lam2 * tau * (ipw(L) + ipw(Ln));
  const double c2 = first ? 0.0 : lam2 * tau * (0.5 * ipw(Lp) + ipw(L) + 0.5 * ipw(Ln));
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * kTLThreads;
    if (q < M) {
      const double k = fabs(static_cast<double>(wavenum(q, M)));
      const double tk3 = (kTwoPi * k) * (kTwoPi * k) * (pw == 2 ? 1.0 : kTwoPi * k);
      const double e1 = exp(-c1 * tk3);
      const double nr = sh.xr[q], ni = sh.xi[q];
      const double er = etahat[2 * q], ei = etahat[2 * q + 1];
      double hr, hi;
      if (first) {
        hr = e1 * (er + tau * nr);
        hi = e1 * (ei + tau * ni);
      } else {
        const double e2 = exp(-c2 * tk3);
        const double pr = nhat_prev[2 * q], pi = nhat_prev[2 * q + 1];
        hr = e1 * er + 0.5 * tau * (3.0 * e1 * nr - e2 * pr);
        hi = e1 * ei + 0.5 * tau * (3.0 * e1 * ni - e2 * pi);
      }
      if (q == (M >> 1)) hr = hi = 0.0;
      nhat_prev[2 * q] = nr;
      nhat_prev[2 * q + 1] = ni;
      sh.yr[q] = hr;
      sh.yi[q] = hi;
    }
  }
  __syncthreads();
  fft_lds(sh.yr, sh.yi, sh.xr, sh.xi, sh.twr, sh.twi, M, true);
  int bad = 0;
  for (int j = tid; j < M; j += blockDim.x) {
    const double v = sh.yr[j] * invM;
    eta[j] = v;
    bad |= !isfinite(v);
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) {
    double v[S_COUNT];
    for (int q = 0; q < S_COUNT; ++q) v[q] = scal[q];
    v[S_LPREV] = L;
    v[S_MPREV] = Mdot;
    v[S_QPX] = qx;
    v[S_QPY] = qy;
    v[S_L] = Ln;
    v[S_XBX] = xn;
    v[S_XBY] = yn;
    v[S_T] += tau;
    v[S_BAD] = (bad || !isfinite(Ln) || !(Ln > 0.0) || !isfinite(xn) || !isfinite(yn)) ? 1.0 : 0.0;
    for (int q = 0; q < S_COUNT; ++q) scal[q] = v[q];
    if (hscal) {  // the host's copy (mapped memory), pushed out at system scope
      for (int q = 0; q < S_COUNT; ++q) hscal[q] = v[q];
      __threadfence_system();
    }
  }
}

// ---------------------------------------------------------------- equal-arclength start
// Trigonometric interpolation coefficients c_q = (1/Mi) sum_j f_j e^{-2 pi i q j / Mi}
// (Nyquist set to zero) of nf arrays, one block per (q, array).
__global__ void k_dft_coef(int Mi, const double* __restrict__ f, double* __restrict__ c) {
  __shared__ double red[32];
  const int q = blockIdx.x, a = blockIdx.y;
  const double* fa = f + static_cast<size_t>(a) * Mi;
  double sr = 0.0, si = 0.0;
  for (int j = threadIdx.x; j < Mi; j += blockDim.x) {
    const long long m = (static_cast<long long>(q) * j) % Mi;
    double s, co;
    sincospi(2.0 * static_cast<double>(m) / Mi, &s, &co);
    sr += fa[j] * co;
    si -= fa[j] * s;
  }
  sr = block_sum<double>(sr, red);
  si = block_sum<double>(si, red);
  if (threadIdx.x == 0) {
    const bool nyq = (q == Mi / 2);
    c[(static_cast<size_t>(a) * Mi + q) * 2] = nyq ? 0.0 : sr / Mi;
    c[(static_cast<size_t>(a) * Mi + q) * 2 + 1] = nyq ? 0.0 : si / Mi;
  }
}

// Real part of sum_q c_q (i k_q)^d e^{i k_q beta} for one coefficient set.
__device__ double trig_eval(const double* __restrict__ c, int Mi, double beta, int d,
                            double* red) {
  double s = 0.0;
  for (int q = threadIdx.x; q < Mi; q += blockDim.x) {
    const int k = wavenum(q, Mi);
    double sn, cs;
    sincos(k * beta, &sn, &cs);
    double cr = c[2 * q], ci = c[2 * q + 1];
    for (int t = 0; t < d; ++t) {  // multiply by ik
      const double nr = -k * ci, ni = k * cr;
      cr = nr;
      ci = ni;
    }
    s += cr * cs - ci * sn;
  }
  return block_sum<double>(s, red);
}

// |X_beta| at the input samples, one block per sample.
__global__ void k_speed(int Mi, const double* __restrict__ cxy, double* __restrict__ sb) {
  __shared__ double red[32];
  const int j = blockIdx.x;
  const double beta = kTwoPi * j / Mi;
  const double xd = trig_eval(cxy, Mi, beta, 1, red);
  const double yd = trig_eval(cxy + 2 * static_cast<size_t>(Mi), Mi, beta, 1, red);
  if (threadIdx.x == 0) sb[j] = hypot(xd, yd);
}

// Newton for beta_j with s(beta_j) = L j / M, s(beta) = (L/2pi) beta + A(beta) - A(0), A the
// mean-free antiderivative of |X_beta|; then X(beta_j), the raw tangent angle.  One block
// per output point; each point iterates until its own step is below 1e-14 (50 at most).
__global__ void k_newton(int Mi, int M, const double* __restrict__ cxy,
                         const double* __restrict__ cs, double* __restrict__ anti,
                         double* __restrict__ out) {
  __shared__ double red[32];
  const int j = blockIdx.x;
  const double L = kTwoPi * cs[0];
  // A(0) = Re sum anti_q
  const double a0 = trig_eval(anti, Mi, 0.0, 0, red);
  const double target = L * j / M;
  double beta = kTwoPi * j / M;
  for (int it = 0; it < 50; ++it) {
    const double f = L / kTwoPi * beta + trig_eval(anti, Mi, beta, 0, red) - a0 - target;
    const double d = trig_eval(cs, Mi, beta, 0, red);
    const double step = f / d;
    beta -= step;
    if (fabs(step) < 1e-14) break;  // block-uniform
  }
  const double xb = trig_eval(cxy, Mi, beta, 0, red);
  const double yb = trig_eval(cxy + 2 * static_cast<size_t>(Mi), Mi, beta, 0, red);
  const double xd = trig_eval(cxy, Mi, beta, 1, red);
  const double yd = trig_eval(cxy + 2 * static_cast<size_t>(Mi), Mi, beta, 1, red);
  if (threadIdx.x == 0) {
    out[j] = atan2(yd, xd);
    out[M + j] = xb;
    out[2 * M + j] = yb;
  }
}

// anti_q = cs_q / (i k_q) for k_q != 0.
__global__ void k_anti(int Mi, const double* __restrict__ cs, double* __restrict__ anti) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Mi) return;
  const int k = wavenum(q, Mi);
  const double a = cs[2 * q], b = cs[2 * q + 1];
  anti[2 * q] = (k != 0) ? b / k : 0.0;
  anti[2 * q + 1] = (k != 0) ? -a / k : 0.0;
}

// Unwrap the raw angles (add the multiple of 2 pi that keeps consecutive jumps within pi),
// eta = theta - alpha, Xbar = mean of the resampled points, L; reset the scalars.
__global__ void __launch_bounds__(kTLThreads)
    k_unwrap(int M, const double* __restrict__ raw, const double* __restrict__ cs,
             double* __restrict__ eta, double* __restrict__ scal) {
  __shared__ int sc[kTLMaxM];
  __shared__ double red[32];
  const int tid = threadIdx.x;
  // per-sample correction count (numpy's unwrap rule)
  for (int j = tid; j < M; j += blockDim.x) {
    int c = 0;
    if (j > 0) {
      const double dd = raw[j] - raw[j - 1];
      double dm = fmod(dd + M_PI, kTwoPi);
      if (dm < 0) dm += kTwoPi;
      dm -= M_PI;
      if (dm == -M_PI && dd > 0) dm = M_PI;
      const double corr = dm - dd;
      c = (fabs(dd) < M_PI) ? 0 : static_cast<int>(rint(corr / kTwoPi));
    }
    sc[j] = c;
  }
  __syncthreads();
  // inclusive prefix sum (Hillis-Steele over LDS, M <= 2048)
  for (int off = 1; off < M; off <<= 1) {
    int v[2];
    for (int u = 0; u < 2; ++u) {
      const int j = tid + u * kTLThreads;
      v[u] = (j < M && j >= off) ? sc[j - off] : 0;
    }
    __syncthreads();
    for (int u = 0; u < 2; ++u) {
      const int j = tid + u * kTLThreads;
      if (j < M) sc[j] += v[u];
    }
    __syncthreads();
  }
  double sx = 0.0, sy = 0.0;
  for (int j = tid; j < M; j += blockDim.x) {
    eta[j] = raw[j] + kTwoPi * sc[j] - kTwoPi * j / M;
    sx += raw[M + j];
    sy += raw[2 * M + j];
  }
  sx = block_sum<double>(sx, red);
  sy = block_sum<double>(sy, red);
  if (tid == 0) {
    for (int s = 0; s < S_COUNT; ++s) scal[s] = 0.0;
    scal[S_L] = kTwoPi * cs[0];
    scal[S_XBX] = sx / M;
    scal[S_XBY] = sy / M;
  }
}

// Marker refinement M -> 2M: eta, phi, phi2 by trigonometric interpolation (FFT of length
// M, Nyquist dropped, zero padding, inverse FFT of length 2M; the unnormalised DFT doubles),
// the explicit-term history nhat (an unnormalised DFT of length M) by zero padding and
// doubling.  tw holds the twiddles of length 2M; one workgroup.
__global__ void __launch_bounds__(kTLThreads)
    k_tl_refine(int M, const double* __restrict__ tw, double* __restrict__ eta,
                double* __restrict__ phi, double* __restrict__ phi2,
                double* __restrict__ nhat) {
  extern __shared__ double lds[];
  const int M2 = 2 * M, h = M / 2;
  const int tid = threadIdx.x;
  double* xr = lds;        // 2M each
  double* xi = xr + M2;
  double* yr = xi + M2;
  double* yi = yr + M2;
  double* t2r = yi + M2;   // twiddles of length 2M (M entries each)
  double* t2i = t2r + M;
  double* t1r = t2i + M;   // of length M (every other one)
  double* t1i = t1r + h;
  for (int k = tid; k < M; k += blockDim.x) {
    t2r[k] = tw[2 * k];
    t2i[k] = tw[2 * k + 1];
    if (k < h) {
      t1r[k] = tw[4 * k];
      t1i[k] = tw[4 * k + 1];
    }
  }
  // the history: new nhat [2M complex] from the old [M complex], doubled; read all first
  double hr[2 * kTLMaxM / kTLThreads], hi[2 * kTLMaxM / kTLThreads];
  constexpr int UH = 2 * kTLMaxM / kTLThreads;
#pragma unroll
  for (int u = 0; u < UH; ++u) {
    const int q = tid + u * kTLThreads;  // index in the doubled spectrum
    hr[u] = hi[u] = 0.0;
    if (q < M2) {
      int src = -1;
      if (q < h) src = q;
      else if (q > M2 - h) src = q - M;  // negative wavenumbers q - 2M = src - M
      if (src >= 0) {
        hr[u] = 2.0 * nhat[2 * src];
        hi[u] = 2.0 * nhat[2 * src + 1];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UH; ++u) {
    const int q = tid + u * kTLThreads;
    if (q < M2) {
      nhat[2 * q] = hr[u];
      nhat[2 * q + 1] = hi[u];
    }
  }
  double* arrs[3] = {eta, phi, phi2};
  for (int a = 0; a < 3; ++a) {
    double* f = arrs[a];
    double* pr = xr;
    double* pi = xi;
    double* qr = yr;
    double* qi = yi;
    for (int j = tid; j < M; j += blockDim.x) {
      pr[j] = f[j];
      pi[j] = 0.0;
    }
    __syncthreads();
    fft_lds(pr, pi, qr, qi, t1r, t1i, M, false);
    // spectrum of length 2M into (qr, qi): 2 F[q] on |k| < M/2, zero elsewhere
    for (int q = tid; q < M2; q += blockDim.x) {
      int src = -1;
      if (q < h) src = q;
      else if (q > M2 - h) src = q - M;
      qr[q] = src >= 0 ? 2.0 * pr[src] : 0.0;
      qi[q] = src >= 0 ? 2.0 * pi[src] : 0.0;
    }
    __syncthreads();
    fft_lds(qr, qi, pr, pi, t2r, t2i, M2, true);
    const double sc = 1.0 / M2;
    for (int j = tid; j < M2; j += blockDim.x) f[j] = qr[j] * sc;
    __syncthreads();
  }
}
inline size_t refine_lds_bytes(int M) { return sizeof(double) * (8 * static_cast<size_t>(M) + 3 * M); }

__global__ void k_twiddles(int M, double* __restrict__ tw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M / 2) return;
  double s, c;
  sincospi(2.0 * k / M, &s, &c);
  tw[2 * k] = c;
  tw[2 * k + 1] = -s;
}

TLMode hs_mode() { return TLMode{0, 3, Aniso{}, Aniso{}}; }

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace kfbi

using namespace kfbi;

// defined after the Stefan object, whose coefficients it may use
static void tl_pre_launch(thetaL* th, const double* guess, double* xw);

namespace kfbi {
int thetal_refresh(thetaL* th) {
  tl_pre_launch(th, nullptr, nullptr);
  KFBI_HIP(hipGetLastError());
  th->pre_n = th->n;  // the next step of this state need not run the pass again
  return KFBI_OK;
}

// Opens a step: the shape pass with the initial guess copied into the working density,
// or only the copy when a learned guess has just run the pass for this state.
static int tl_open_step(thetaL* th, const double* guess) {
  if (th->pre_n == th->n) {
    KFBI_HIP(hipMemcpyAsync(th->phiw.p, guess, sizeof(double) * th->M, hipMemcpyDeviceToDevice,
                            th->stream));
  } else {
    tl_pre_launch(th, guess, th->phiw.as<double>());
  }
  th->pre_n = -1;
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}
}  // namespace kfbi

static int tl_check(const thetaL* th, bool need_ready) {
  if (!th) {
    set_error("null thetaL object");
    return KFBI_E_INVALID;
  }
  if (need_ready && !th->ready) {
    set_error("thetaL_init (or thetaL_set_state) has not been called");
    return KFBI_E_STATE;
  }
  return KFBI_OK;
}

// Switch the object to M markers (twiddles of length M); state arrays are not touched.
static int tl_set_M(thetaL* th, int M) {
  if (M == th->M) return KFBI_OK;
  hipLaunchKernelGGL(k_twiddles, dim3((M / 2 + 255) / 256), dim3(256), 0, th->stream, M,
                     th->tw.as<double>());
  KFBI_HIP(hipGetLastError());
  th->M = M;
  return KFBI_OK;
}

// Adaptive refinement after a step: double M when the marker spacing L/M of the new state
// exceeds ratio * h and the buffers allow it (eta, the last two densities and the
// explicit-term history are interpolated to the doubled grid).  Synchronises if it refines.
static int tl_maybe_refine(thetaL* th, double ratio, double h) {
  const int M = th->M;
  if (!(ratio > 0.0) || !(th->hscal[S_L] / M > ratio * h) || 2 * M > th->Mcap) return KFBI_OK;
  KFBI_TRY(tl_set_M(th, 2 * M));  // twiddles of length 2M
  hipLaunchKernelGGL(k_tl_refine, dim3(1), dim3(kTLThreads), refine_lds_bytes(M), th->stream, M,
                     th->tw.as<double>(), th->eta.as<double>(), th->phi.as<double>(),
                     th->phi2.as<double>(), th->nhat.as<double>());
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(th->stream));
  return KFBI_OK;
}

static void tl_free(thetaL* th) {
  for (DBuf* b : {&th->tw, &th->eta, &th->scal, &th->X, &th->rhs, &th->aux, &th->etahat, &th->nhat,
                  &th->phi, &th->phi2, &th->phiw, &th->dnp, &th->dnm, &th->init})
    b->release();
  if (th->hscal) (void)hipHostFree(th->hscal);
  th->hscal = th->dscal = nullptr;
  for (hipEvent_t& e : th->tev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (th->kc) kfbi_destroy(th->kc);
  th->kc = nullptr;
}

namespace kfbi {
int thetal_kernel_attrs() {
  KFBI_TRY(allow_full_dyn_lds(reinterpret_cast<const void*>(k_tl_pre)));
  KFBI_TRY(allow_full_dyn_lds(reinterpret_cast<const void*>(k_tl_post)));
  return allow_full_dyn_lds(reinterpret_cast<const void*>(k_tl_refine));
}
}  // namespace kfbi

// Buffers, the KFBI context of the grid solves and the twiddles of an evolution object
// whose parameters have been checked (on failure everything is released).
static int tl_setup(thetaL* th, const thetaL_params* p, int M, int Mcap) {
  th->prm = *p;
  th->M = M;
  th->Mcap = Mcap;
  kfbi_grid g = p->grid;
  g.max_markers = Mcap;
  int st = kfbi_create(&g, &th->kc);
  if (st != KFBI_OK) return st;
  th->stream = static_cast<hipStream_t>(g.stream);
  const int Mi = 4096;  // largest accepted input sampling of thetaL_init
  const int C = Mcap;   // every per-marker buffer is sized for the refinement limit
  if ((st = th->tw.ensure(sizeof(double) * C)) || (st = th->eta.ensure(sizeof(double) * C)) ||
      (st = th->scal.ensure(sizeof(double) * S_COUNT)) ||
      (st = th->X.ensure(sizeof(double) * 2 * C)) || (st = th->rhs.ensure(sizeof(double) * C)) ||
      (st = th->aux.ensure(sizeof(double) * A_COUNT * C)) ||
      (st = th->etahat.ensure(sizeof(double) * 2 * C)) ||
      (st = th->nhat.ensure(sizeof(double) * 2 * C)) ||
      (st = th->phi.ensure(sizeof(double) * C)) || (st = th->phi2.ensure(sizeof(double) * C)) ||
      (st = th->phiw.ensure(sizeof(double) * C)) ||
      (st = th->dnp.ensure(sizeof(double) * C)) || (st = th->dnm.ensure(sizeof(double) * C)) ||
      (st = th->init.ensure(sizeof(double) * (2 * Mi + 4 * Mi + 2 * Mi + 2 * Mi + Mi + 3 * C)))) {
    tl_free(th);
    return st;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&th->hscal), sizeof(double) * S_COUNT,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&th->dscal), th->hscal, 0) !=
          hipSuccess) {
    if (th->hscal) (void)hipHostFree(th->hscal);
    th->hscal = th->dscal = nullptr;
    tl_free(th);
    set_error("hipHostMalloc (coherent scalars) failed");
    return KFBI_E_NOMEM;
  }
  for (hipEvent_t& e : th->tev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      tl_free(th);
      set_error("hipEventCreate failed");
      return KFBI_E_HIP;
    }
  hipLaunchKernelGGL(k_twiddles, dim3((M / 2 + 255) / 256), dim3(256), 0, th->stream, M,
                     th->tw.as<double>());
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(th->stream) != hipSuccess) {
    tl_free(th);
    set_error("thetaL: twiddle kernel failed");
    return KFBI_E_HIP;
  }
  return KFBI_OK;
}

extern "C" {

int thetaL_create(const thetaL_params* p, thetaL** out) {
  if (!p || !out) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *out = nullptr;
  const int M = p->M;
  if (M < 16 || M > kTLMaxM || (M & (M - 1))) {
    set_error("thetaL: M must be a power of two in [16, %d] (M=%d)", kTLMaxM, M);
    return KFBI_E_INVALID;
  }
  if (p->grid.box_bc != KFBI_BOX_FREESPACE || p->grid.c2 != 0.0) {
    set_error("thetaL: the Hele-Shaw pressure solve needs box_bc = KFBI_BOX_FREESPACE, c2 = 0");
    return KFBI_E_INVALID;
  }
  if (!(p->tau > 0.0) || !(p->sigma >= 0.0) || !std::isfinite(p->J)) {
    set_error("thetaL: need tau > 0, sigma >= 0, finite J");
    return KFBI_E_INVALID;
  }
  const int Mcap = p->max_M > 0 ? p->max_M : M;
  if (Mcap < M || Mcap > kTLMaxM || (Mcap & (Mcap - 1)) || !(p->refine >= 0.0)) {
    set_error("thetaL: max_M must be a power of two in [M, %d] and refine >= 0", kTLMaxM);
    return KFBI_E_INVALID;
  }
  thetaL* th = new (std::nothrow) thetaL();
  if (!th) {
    set_error("out of host memory");
    return KFBI_E_NOMEM;
  }
  const int st = tl_setup(th, p, M, Mcap);
  if (st != KFBI_OK) {
    delete th;
    return st;
  }
  *out = th;
  return KFBI_OK;
}

int thetaL_destroy(thetaL* th) {
  if (!th) return KFBI_OK;
  (void)hipStreamSynchronize(th->stream);
  tl_free(th);
  delete th;
  return KFBI_OK;
}

kfbi_ctx* thetaL_kfbi(thetaL* th) { return th ? th->kc : nullptr; }

int thetaL_init(thetaL* th, int Mi, const double* xy) {
  KFBI_TRY(tl_check(th, false));
  if (!xy || Mi < 16 || Mi > 4096 || (Mi & 1)) {
    set_error("thetaL_init: Mi must be even in [16, 4096] with a non-null xy (Mi=%d)", Mi);
    return KFBI_E_INVALID;
  }
  KFBI_TRY(tl_set_M(th, th->prm.M));  // back to the initial markers
  const int M = th->M;
  hipStream_t s = th->stream;
  double* w = th->init.as<double>();
  double* cxy = w;                 // 2 x Mi complex
  double* cs = cxy + 4 * Mi;       // Mi complex
  double* anti = cs + 2 * Mi;      // Mi complex
  double* sb = anti + 2 * Mi;      // Mi
  double* raw = sb + Mi;           // 3 M: raw angle, x, y
  hipLaunchKernelGGL(k_dft_coef, dim3(Mi, 2), dim3(256), 0, s, Mi, xy, cxy);
  hipLaunchKernelGGL(k_speed, dim3(Mi), dim3(256), 0, s, Mi, cxy, sb);
  hipLaunchKernelGGL(k_dft_coef, dim3(Mi, 1), dim3(256), 0, s, Mi, sb, cs);
  hipLaunchKernelGGL(k_anti, dim3((Mi + 255) / 256), dim3(256), 0, s, Mi, cs, anti);
  hipLaunchKernelGGL(k_newton, dim3(M), dim3(256), 0, s, Mi, M, cxy, cs, anti, raw);
  hipLaunchKernelGGL(k_unwrap, dim3(1), dim3(kTLThreads), 0, s, M, raw, cs, th->eta.as<double>(),
                     th->scal.as<double>());
  KFBI_HIP(hipMemsetAsync(th->phi.p, 0, sizeof(double) * M, s));
  KFBI_HIP(hipMemsetAsync(th->phi2.p, 0, sizeof(double) * M, s));
  KFBI_HIP(hipMemsetAsync(th->nhat.p, 0, sizeof(double) * 2 * M, s));
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(th->hscal, th->scal.p, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, s));
  KFBI_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(th->hscal[S_L]) || !(th->hscal[S_L] > 0.0)) {
    set_error("thetaL_init: the curve has no finite positive length");
    return KFBI_E_NONFINITE;
  }
  th->n = 0;
  th->pre_n = -1;
  th->have_phi = 0;
  th->ready = 1;
  return KFBI_OK;
}

int thetaL_markers(thetaL* th, double* xy) {
  KFBI_TRY(tl_check(th, true));
  if (!xy) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  const int M = th->M;
  // the reconstruction kernel writes X straight into the caller's array
  hipLaunchKernelGGL(k_tl_pre, dim3(1), dim3(kTLThreads), tl_lds_bytes(M), th->stream, M,
                     th->prm.sigma, th->prm.J, th->tw.as<double>(), th->eta.as<double>(),
                     th->scal.as<double>(), xy, th->rhs.as<double>(), th->aux.as<double>(),
                     th->etahat.as<double>(), hs_mode(), nullptr, nullptr, nullptr);
  KFBI_HIP(hipGetLastError());
  return KFBI_OK;
}

int thetaL_density(const thetaL* th, double* phi) {
  KFBI_TRY(tl_check(th, true));
  if (!phi) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  KFBI_HIP(hipMemcpyAsync(phi, th->phi.p, sizeof(double) * th->M, hipMemcpyDeviceToDevice,
                          th->stream));
  return KFBI_OK;
}

// After a solve: phi2 <- phi, phi <- phiw (the new density), phiw <- the old phi2 buffer.
static void tl_rotate(thetaL* th) {
  std::swap(th->phi2, th->phi);
  std::swap(th->phi, th->phiw);
}

int thetaL_step(thetaL* th, const double* x0, thetaL_stats* stats) {
  KFBI_TRY(tl_check(th, true));
  const int M = th->M;
  hipStream_t s = th->stream;
  const thetaL_params& p = th->prm;
  auto t0 = std::chrono::steady_clock::now();
  // reconstruction, right-hand side, and the GMRES initial guess (x0, else the previous
  // density, zero before the first solve) into the working density
  const double* guess = x0 ? x0 : th->phi.as<double>();
  KFBI_TRY(tl_open_step(th, guess));
  int st = kfbi_set_interface(th->kc, M, th->X.as<double>());
  if (st != KFBI_OK) return st;
  const double ms_geo = ms_since(t0);
  auto t1 = std::chrono::steady_clock::now();
  const kfbi_bie op{KFBI_DOUBLE, KFBI_MINUS, 0.0, 1.0, 1.0, nullptr};
  kfbi_gmres_stats gs{};
  // the FP64 applies of the solve also write d_n(D x); the last one is the final true
  // residual at the solution, so d_n(D phi) comes with the solve
  kfbi_out o{nullptr, nullptr, th->dnp.as<double>(), th->dnm.as<double>(), nullptr};
  bool dn_ready = false;
  st = gmres_solve_side(th->kc, &op, th->rhs.as<double>(), th->phiw.as<double>(), &p.gmres, &gs,
                        &o, &dn_ready);
  if (st != KFBI_OK) return st;
  const double ms_gm = ms_since(t1);
  // the velocity apply (only when the solve did not end with one at the solution) and the
  // update run without a host synchronisation between them; their times come from events
  KFBI_HIP(hipEventRecord(th->tev[0], s));
  if (!dn_ready) {
    st = kfbi_apply(th->kc, KFBI_DOUBLE, KFBI_FP64, th->phiw.as<double>(), nullptr, &o);
    if (st != KFBI_OK) return st;
  }
  KFBI_HIP(hipEventRecord(th->tev[1], s));
  const double lam2 = p.lambda2 < 0.0 ? p.sigma : p.lambda2;
  hipLaunchKernelGGL(k_tl_post, dim3(1), dim3(kTLThreads), tl_lds_bytes(M), s, M, p.J, p.tau,
                     lam2, th->n == 0 ? 1 : 0, th->tw.as<double>(), th->X.as<double>(),
                     th->aux.as<double>(), th->dnp.as<double>(), th->dnm.as<double>(),
                     th->etahat.as<double>(), th->nhat.as<double>(), th->scal.as<double>(),
                     th->eta.as<double>(), nullptr, 3, th->dscal);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipEventRecord(th->tev[2], s));
  KFBI_HIP(hipStreamSynchronize(s));
  tl_rotate(th);
  float f_ap = 0.f, f_up = 0.f;
  KFBI_HIP(hipEventElapsedTime(&f_ap, th->tev[0], th->tev[1]));
  KFBI_HIP(hipEventElapsedTime(&f_up, th->tev[1], th->tev[2]));
  const double ms_ap = f_ap, ms_up = f_up;
  const int step = th->n;
  th->n += 1;
  th->have_phi = 1;
  if (stats) {
    stats->step = step;
    stats->t = th->hscal[S_T];
    stats->iters = gs.iters;
    stats->applies64 = gs.applies64;
    stats->applies32 = gs.applies32;
    stats->relres = gs.relres;
    stats->area = th->hscal[S_AREA];
    stats->length = th->hscal[S_LEN];
    stats->ms_geometry = ms_geo;
    stats->ms_gmres = ms_gm;
    stats->ms_apply = ms_ap;
    stats->ms_update = ms_up;
    stats->M = M;
    stats->M_next = M;
  }
  if (th->hscal[S_BAD] != 0.0) {
    set_error("thetaL_step: the new state is not finite (step %d)", step);
    return KFBI_E_NONFINITE;
  }
  KFBI_TRY(tl_maybe_refine(th, p.refine, p.grid.side / p.grid.N));
  if (stats) {
    stats->M = M;
    stats->M_next = th->M;
  }
  return KFBI_OK;
}

int thetaL_size(const thetaL* th, int* M) {
  KFBI_TRY(tl_check(th, false));
  if (!M) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *M = th->M;
  return KFBI_OK;
}

int thetaL_run(thetaL* th, int nsteps, thetaL_stats* stats) {
  KFBI_TRY(tl_check(th, true));
  if (nsteps < 0) {
    set_error("nsteps < 0");
    return KFBI_E_INVALID;
  }
  for (int i = 0; i < nsteps; ++i) KFBI_TRY(thetaL_step(th, nullptr, stats ? stats + i : nullptr));
  return KFBI_OK;
}

int thetaL_get_state(const thetaL* th, thetaL_state* st) {
  KFBI_TRY(tl_check(th, true));
  if (!st || !st->eta_dev || !st->phi_prev_dev || !st->phi_prev2_dev || !st->nhat_prev_dev) {
    set_error("thetaL_get_state: null state array");
    return KFBI_E_INVALID;
  }
  const int M = th->M;
  hipStream_t s = th->stream;
  KFBI_HIP(hipMemcpyAsync(st->eta_dev, th->eta.p, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(st->phi_prev_dev, th->phi.p, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(st->phi_prev2_dev, th->phi2.p, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(st->nhat_prev_dev, th->nhat.p, sizeof(double) * 2 * M,
                          hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(th->hscal, th->scal.p, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, s));
  KFBI_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < 8; ++q) st->scal[q] = th->hscal[q];
  st->n = th->n;
  st->M = M;
  return KFBI_OK;
}

int thetaL_set_state(thetaL* th, const thetaL_state* st) {
  KFBI_TRY(tl_check(th, false));
  if (!st || !st->eta_dev || !st->phi_prev_dev || !st->phi_prev2_dev || !st->nhat_prev_dev ||
      st->n < 0) {
    set_error("thetaL_set_state: null state array or negative step count");
    return KFBI_E_INVALID;
  }
  if (!(st->scal[S_L] > 0.0)) {
    set_error("thetaL_set_state: L must be positive");
    return KFBI_E_INVALID;
  }
  const int Ms = st->M == 0 ? th->M : st->M;
  if (Ms < 16 || Ms > th->Mcap || (Ms & (Ms - 1))) {
    set_error("thetaL_set_state: M must be a power of two in [16, max_M] (M=%d)", Ms);
    return KFBI_E_INVALID;
  }
  KFBI_TRY(tl_set_M(th, Ms));
  const int M = th->M;
  hipStream_t s = th->stream;
  KFBI_HIP(hipMemcpyAsync(th->eta.p, st->eta_dev, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(th->phi.p, st->phi_prev_dev, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(th->phi2.p, st->phi_prev2_dev, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
  KFBI_HIP(hipMemcpyAsync(th->nhat.p, st->nhat_prev_dev, sizeof(double) * 2 * M,
                          hipMemcpyDeviceToDevice, s));
  for (int q = 0; q < S_COUNT; ++q) th->hscal[q] = (q < 8) ? st->scal[q] : 0.0;
  KFBI_HIP(hipMemcpyAsync(th->scal.p, th->hscal, sizeof(double) * S_COUNT, hipMemcpyHostToDevice, s));
  KFBI_HIP(hipStreamSynchronize(s));
  th->n = st->n;
  th->pre_n = -1;
  th->have_phi = 1;
  th->ready = 1;
  return KFBI_OK;
}

}  // extern "C"

// ================================================================ Stefan problem (stefan.h)
#include "../../include/stefan.h"

namespace kfbi {
namespace {

// seed field: 0 at nodes inside the interface (label 1), St outside
__global__ void k_seed(int n, const int8_t* __restrict__ lab, double St, double* __restrict__ T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) T[t] = lab[t] ? 0.0 : St;
}

// y = a x + b y (n values); with b = 0, y is only written (its old contents may be
// uninitialised memory, and 0 times a NaN there would be NaN)
__global__ void k_axpby(int n, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = (b != 0.0) ? a * x[t] + b * y[t] : a * x[t];
}

Aniso to_aniso(const stefan_aniso& a) { return Aniso{a.e0, a.e1, a.e2, double(a.m), a.phi0}; }

double aniso_host(const stefan_aniso& a, double phi) {
  return a.e0 * (1.0 + a.e1 * std::cos(a.m * (phi - a.phi0)) +
                 a.e2 * std::cos(2.0 * a.m * (phi - a.phi0)));
}

}  // namespace
}  // namespace kfbi

struct stefan {
  stefan_params prm{};
  thetaL tl;               // interface state; its KFBI context has the mirrored-ghost box
  kfbi::DBuf That, Tprev, Tnew, T1, t1at, amk, neg, grid0;
  kfbi::TLMode md{};
  double lam = 0.0, c2 = 0.0;
  int have_prev = 0;       // T^{n-1} exists (BDF2)
};

// The shape pass of the step of th: the Hele-Shaw right-hand side -sigma kappa + J ln|x|,
// or the Stefan problem's -eps_C kappa with eps_V per marker when th belongs to one.
static void tl_pre_launch(thetaL* th, const double* guess, double* xw) {
  const int M = th->M;
  stefan* o = th->owner;
  hipLaunchKernelGGL(k_tl_pre, dim3(1), dim3(kTLThreads), tl_lds_bytes(M), th->stream, M,
                     o ? 0.0 : th->prm.sigma, o ? 0.0 : th->prm.J, th->tw.as<double>(),
                     th->eta.as<double>(), th->scal.as<double>(), th->X.as<double>(),
                     th->rhs.as<double>(), th->aux.as<double>(), th->etahat.as<double>(),
                     o ? o->md : hs_mode(), o ? o->amk.as<double>() : nullptr,
                     guess, xw);
}

static void st_free(stefan* s) {
  for (DBuf* b : {&s->That, &s->Tprev, &s->Tnew, &s->T1, &s->t1at, &s->amk, &s->neg, &s->grid0})
    b->release();
  tl_free(&s->tl);
}

extern "C" {

int stefan_create(const stefan_params* p, stefan** out) {
  if (!p || !out) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *out = nullptr;
  const int M = p->M;
  if (M < 16 || M > kTLMaxM || (M & (M - 1))) {
    set_error("stefan: M must be a power of two in [16, %d] (M=%d)", kTLMaxM, M);
    return KFBI_E_INVALID;
  }
  if (!(p->tau > 0.0) || (p->ssd != 1 && p->ssd != 2) || !(p->eps_c.e0 >= 0.0) ||
      !(p->eps_v.e0 >= 0.0) || (p->ssd == 1 && !(p->eps_v.e0 > 0.0))) {
    set_error("stefan: need tau > 0, ssd 1 or 2, eps_C, eps_V >= 0 (eps_V > 0 with ssd 1)");
    return KFBI_E_INVALID;
  }
  stefan* s = new (std::nothrow) stefan();
  if (!s) {
    set_error("out of host memory");
    return KFBI_E_NOMEM;
  }
  s->prm = *p;
  s->c2 = p->bdf2 ? 1.5 / p->tau : 1.0 / p->tau;
  if (p->lambda > 0.0) {
    s->lam = p->lambda;
  } else {  // frozen-coefficient maxima over 4096 normal angles
    double mx = 0.0;
    for (int q = 0; q < 4096; ++q) {
      const double phi = 2.0 * M_PI * q / 4096;
      const double ec = aniso_host(p->eps_c, phi), ev = aniso_host(p->eps_v, phi);
      mx = std::max(mx, p->ssd == 1 ? std::fabs(ec / ev) : std::fabs(2.0 * ec));
    }
    s->lam = mx;
  }
  s->md = TLMode{1, p->ssd == 1 ? 2 : 3, to_aniso(p->eps_c), to_aniso(p->eps_v)};
  thetaL_params tp{};
  tp.grid = kfbi_grid{p->x0, p->y0, p->side, p->N, s->c2, KFBI_BOX_NEUMANN, M, p->stream, 0};
  tp.M = M;
  tp.tau = p->tau;
  tp.lambda2 = s->lam;
  tp.gmres = p->gmres;
  const int Mcap = p->max_M > 0 ? p->max_M : M;
  if (Mcap < M || Mcap > kTLMaxM || (Mcap & (Mcap - 1)) || !(p->refine >= 0.0)) {
    delete s;
    set_error("stefan: max_M must be a power of two in [M, %d] and refine >= 0", kTLMaxM);
    return KFBI_E_INVALID;
  }
  int st = tl_setup(&s->tl, &tp, M, Mcap);
  if (st != KFBI_OK) {
    delete s;
    return st;
  }
  s->tl.owner = s;  // its steps and learned guesses use the Stefan coefficients
  const size_t nf = neu_field_size(p->N);
  const size_t n1sq = static_cast<size_t>(p->N + 1) * (p->N + 1);
  if ((st = s->That.ensure(sizeof(double) * nf)) || (st = s->Tprev.ensure(sizeof(double) * nf)) ||
      (st = s->Tnew.ensure(sizeof(double) * nf)) || (st = s->T1.ensure(sizeof(double) * nf)) ||
      (st = s->t1at.ensure(sizeof(double) * Mcap)) || (st = s->amk.ensure(sizeof(double) * Mcap)) ||
      (st = s->neg.ensure(sizeof(double) * Mcap)) || (st = s->grid0.ensure(sizeof(double) * n1sq))) {
    st_free(s);
    delete s;
    return st;
  }
  *out = s;
  return KFBI_OK;
}

int stefan_destroy(stefan* s) {
  if (!s) return KFBI_OK;
  (void)hipStreamSynchronize(s->tl.stream);
  st_free(s);
  delete s;
  return KFBI_OK;
}

int stefan_init(stefan* s, int Mi, const double* xy, const double* T0, double St) {
  if (!s) {
    set_error("null stefan object");
    return KFBI_E_INVALID;
  }
  thetaL* th = &s->tl;
  KFBI_TRY(thetaL_init(th, Mi, xy));
  hipStream_t hs = th->stream;
  const int N = s->prm.N;
  const int n1sq = (N + 1) * (N + 1);
  if (!T0) {  // seed field from the labels of the resampled curve
    hipLaunchKernelGGL(k_tl_pre, dim3(1), dim3(kTLThreads), tl_lds_bytes(th->M), hs, th->M, 0.0,
                       0.0, th->tw.as<double>(), th->eta.as<double>(), th->scal.as<double>(),
                       th->X.as<double>(), th->rhs.as<double>(), th->aux.as<double>(),
                       th->etahat.as<double>(), s->md, s->amk.as<double>(), nullptr, nullptr);
    KFBI_HIP(hipGetLastError());
    KFBI_TRY(kfbi_set_interface(th->kc, th->M, th->X.as<double>()));
    hipLaunchKernelGGL(k_seed, dim3((n1sq + 255) / 256), dim3(256), 0, hs, n1sq,
                       th->kc->lab.as<int8_t>(), St, s->grid0.as<double>());
    KFBI_HIP(hipGetLastError());
    T0 = s->grid0.as<double>();
  }
  KFBI_TRY(neu_from_grid(th->kc, T0, s->That.as<double>()));
  KFBI_HIP(hipStreamSynchronize(hs));
  s->have_prev = 0;
  return KFBI_OK;
}

int stefan_step(stefan* s, const double* x0, stefan_stats* stats) {
  if (!s) {
    set_error("null stefan object");
    return KFBI_E_INVALID;
  }
  thetaL* th = &s->tl;
  KFBI_TRY(tl_check(th, true));
  const int M = th->M;
  hipStream_t hs = th->stream;
  const stefan_params& p = s->prm;
  auto t0 = std::chrono::steady_clock::now();
  // reconstruction, eps_C kappa and eps_V, and the GMRES initial guess (x0, else the last
  // density) into the working density
  const double* guess = x0 ? x0 : th->phi.as<double>();
  KFBI_TRY(tl_open_step(th, guess));
  int st = kfbi_set_interface(th->kc, M, th->X.as<double>());
  if (st != KFBI_OK) return st;
  const double ms_geo = ms_since(t0);
  // T1: the five-point problem with the time-discretisation right-hand side (timed by
  // events; GMRES starts behind it without a host synchronisation)
  KFBI_HIP(hipEventRecord(th->tev[0], hs));
  const double* Fa = s->That.as<double>();
  const double* Fb = nullptr;
  double ca = -1.0 / p.tau, cb = 0.0;
  if (p.bdf2) {
    Fb = s->have_prev ? s->Tprev.as<double>() : s->That.as<double>();
    ca = -2.0 / p.tau;
    cb = 0.5 / p.tau;
  }
  // only T1 at the markers is needed: the solve writes the node rows alone
  const int jlo = th->kc->st.row_lo, jhi = th->kc->st.row_hi;
  KFBI_TRY(neu_dense_solve(th->kc, Fa, Fb, ca, cb, s->T1.as<double>(), jlo, jhi));
  KFBI_TRY(neu_interp(th->kc, s->T1.as<double>(), jlo, jhi, s->t1at.as<double>()));
  hipLaunchKernelGGL(k_axpby, dim3((M + 255) / 256), dim3(256), 0, hs, M, -1.0,
                     s->t1at.as<double>(), 1.0, th->rhs.as<double>());
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipEventRecord(th->tev[1], hs));
  // eq. bie-GT
  auto t2 = std::chrono::steady_clock::now();
  const kfbi_bie op{KFBI_SINGLE, KFBI_AVG, 0.0, -1.0, 0.0, s->amk.as<double>()};
  kfbi_gmres_stats gs{};
  st = kfbi_gmres_solve(th->kc, &op, th->rhs.as<double>(), th->phiw.as<double>(), &p.gmres, &gs);
  if (st != KFBI_OK) return st;
  const double ms_gm = ms_since(t2);
  // T^{n+1} = T1 + T2, T2 = -S psi: one column solve of both right-hand sides; then theta-L
  KFBI_HIP(hipEventRecord(th->tev[2], hs));
  hipLaunchKernelGGL(k_axpby, dim3((M + 255) / 256), dim3(256), 0, hs, M, -1.0,
                     th->phiw.as<double>(), 0.0, s->neg.as<double>());
  KFBI_TRY(neu_apply_full(th->kc, KFBI_SINGLE, s->neg.as<double>(), Fa, Fb, ca, cb,
                          s->Tnew.as<double>()));
  hipLaunchKernelGGL(k_tl_post, dim3(1), dim3(kTLThreads), tl_lds_bytes(M), hs, M, 0.0, p.tau,
                     s->lam, th->n == 0 ? 1 : 0, th->tw.as<double>(), th->X.as<double>(),
                     th->aux.as<double>(), th->dnp.as<double>(), th->dnm.as<double>(),
                     th->etahat.as<double>(), th->nhat.as<double>(), th->scal.as<double>(),
                     th->eta.as<double>(), th->phiw.as<double>(), s->md.pw, th->dscal);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipEventRecord(th->tev[3], hs));
  KFBI_HIP(hipStreamSynchronize(hs));
  tl_rotate(th);
  std::swap(s->Tprev, s->That);  // T^{n-1} <- T^n
  std::swap(s->That, s->Tnew);   // T^n <- T^{n+1}
  s->have_prev = 1;
  float f_t1 = 0.f, f_up = 0.f;
  KFBI_HIP(hipEventElapsedTime(&f_t1, th->tev[0], th->tev[1]));
  KFBI_HIP(hipEventElapsedTime(&f_up, th->tev[2], th->tev[3]));
  const double ms_t1 = f_t1, ms_up = f_up;
  const int step = th->n;
  th->n += 1;
  th->have_phi = 1;
  if (stats) {
    stats->step = step;
    stats->t = th->hscal[S_T];
    stats->iters = gs.iters;
    stats->applies64 = gs.applies64;
    stats->applies32 = gs.applies32;
    stats->relres = gs.relres;
    stats->area = th->hscal[S_AREA];
    stats->length = th->hscal[S_LEN];
    stats->ms_geometry = ms_geo;
    stats->ms_temperature = ms_t1;
    stats->ms_gmres = ms_gm;
    stats->ms_update = ms_up;
    stats->M = M;
    stats->M_next = M;
  }
  if (th->hscal[S_BAD] != 0.0) {
    set_error("stefan_step: the new state is not finite (step %d)", step);
    return KFBI_E_NONFINITE;
  }
  KFBI_TRY(tl_maybe_refine(th, p.refine, p.side / p.N));
  if (stats) stats->M_next = th->M;
  return KFBI_OK;
}

thetaL* stefan_thetal(stefan* s) { return s ? &s->tl : nullptr; }

int stefan_size(const stefan* s, int* M) {
  if (!s || !M) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *M = s->tl.M;
  return KFBI_OK;
}

int stefan_run(stefan* s, int nsteps, stefan_stats* stats) {
  if (!s || nsteps < 0) {
    set_error("null stefan object or nsteps < 0");
    return KFBI_E_INVALID;
  }
  for (int i = 0; i < nsteps; ++i) KFBI_TRY(stefan_step(s, nullptr, stats ? stats + i : nullptr));
  return KFBI_OK;
}

int stefan_temperature(stefan* s, double* grid) {
  if (!s || !grid) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  KFBI_TRY(tl_check(&s->tl, true));
  return neu_to_grid(s->tl.kc, s->That.as<double>(), grid);
}

int stefan_markers(stefan* s, double* xy) {
  if (!s) {
    set_error("null stefan object");
    return KFBI_E_INVALID;
  }
  return thetaL_markers(&s->tl, xy);
}

int stefan_density(const stefan* s, double* psi) {
  if (!s) {
    set_error("null stefan object");
    return KFBI_E_INVALID;
  }
  return thetaL_density(&s->tl, psi);
}

int stefan_interface(const stefan* s, double* eta, double* scal) {
  if (!s || !eta || !scal) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  const thetaL* th = &s->tl;
  KFBI_TRY(tl_check(th, true));
  KFBI_HIP(hipMemcpyAsync(eta, th->eta.p, sizeof(double) * th->M, hipMemcpyDeviceToDevice,
                          th->stream));
  KFBI_HIP(hipMemcpyAsync(th->hscal, th->scal.p, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost,
                          th->stream));
  KFBI_HIP(hipStreamSynchronize(th->stream));
  scal[0] = th->hscal[S_L];
  scal[1] = th->hscal[S_XBX];
  scal[2] = th->hscal[S_XBY];
  scal[3] = th->hscal[S_T];
  return KFBI_OK;
}

int stefan_constants(const stefan* s, double* lambda, double* c2) {
  if (!s || !lambda || !c2) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *lambda = s->lam;
  *c2 = s->c2;
  return KFBI_OK;
}

}  // extern "C"
