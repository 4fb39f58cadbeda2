// Absorption spectrum from dipole traces (Sec. 3.2): the windowed Fourier
// transform of the dipole response of each perturbed run, divided by the
// transform of the applied field, and S(omega) = (2 omega / 3 pi) sum_d Im alpha_dd.
// Dipole power spectrum of a driven run (Sec. 3.5): |windowed transform of mu''|^2.
#include <hip/hip_runtime.h>

#include "device.h"

namespace efe {
namespace {

constexpr int kSpecThreads = 256;

// One workgroup per frequency: the threads stride over the samples of each run
// (trapezoid weights, window exp(-t/tau)) and the sums are reduced in a fixed
// order.  mu: [ndir][nt1][3]; dirs: [ndir] (device copy in the launch args).
struct Dirs {
  int d[3];
};

__global__ void __launch_bounds__(kSpecThreads)
k_spectrum(const double *__restrict__ mu, Dirs dirs, int ndir, int64_t nt1, double dt, double tau, int kind,
           double kappa, double t0, double s, const double *__restrict__ omega, double *__restrict__ S,
           double *__restrict__ alpha, int64_t nw) {
  __shared__ double red[2][kSpecThreads];
  const int64_t iw = blockIdx.x;
  if (iw >= nw) return;
  const double w = omega[iw];
  // F[E](w): kappa for the kick; kappa s sqrt(2 pi) exp(-w^2 s^2 / 2) exp(i w t0) for the Gaussian
  double fr = kappa, fi = 0.0;
  if (kind == 1) {
    const double a = kappa * s * 2.5066282746310002 * exp(-0.5 * w * w * s * s);
    double sn, cs;
    sincos(w * t0, &sn, &cs);
    fr = a * cs;
    fi = a * sn;
  }
  const double fden = fr * fr + fi * fi;
  double sum_im = 0.0;
  for (int r = 0; r < ndir; ++r) {
    const int d = dirs.d[r];
    const double *m = mu + (int64_t)r * nt1 * 3;
    const double m0 = m[d];
    double re = 0.0, im = 0.0;
    for (int64_t n = threadIdx.x; n < nt1; n += kSpecThreads) {
      const double t = dt * (double)n;
      const double wt = (n == 0 || n == nt1 - 1) ? 0.5 * dt : dt;
      const double f = wt * exp(-t / tau) * (m[n * 3 + d] - m0);
      double sn, cs;
      sincos(w * t, &sn, &cs);
      re += f * cs;
      im += f * sn;
    }
    red[0][threadIdx.x] = re;
    red[1][threadIdx.x] = im;
    __syncthreads();
    for (int h = kSpecThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        red[0][threadIdx.x] += red[0][threadIdx.x + h];
        red[1][threadIdx.x] += red[1][threadIdx.x + h];
      }
      __syncthreads();
    }
    // alpha = F[g dmu] / F[E]
    const double ar = (red[0][0] * fr + red[1][0] * fi) / fden;
    const double ai = (red[1][0] * fr - red[0][0] * fi) / fden;
    if (threadIdx.x == 0 && alpha) {
      alpha[((int64_t)r * nw + iw) * 2] = ar;
      alpha[((int64_t)r * nw + iw) * 2 + 1] = ai;
    }
    sum_im += ai;
    __syncthreads();
  }
  if (threadIdx.x == 0) S[iw] = 2.0 * w / (3.0 * 3.14159265358979323846) * sum_im;
}

// Dipole power spectrum (Sec. 3.5): one workgroup per frequency;
// P(omega) = |sum_n w_n exp(-t_n^2 / tau) mu''(t_n) exp(-i omega t_n)|^2 over the interior
// samples n = 1 .. nt1 - 2 (second central difference, trapezoid weights dt, dt/2 at the
// two ends), reduced in a fixed order.  mu: [nt1][3].
__global__ void __launch_bounds__(kSpecThreads)
k_power_spectrum(const double *__restrict__ mu, int dir, int64_t nt1, double dt, double tau,
                 const double *__restrict__ omega, double *__restrict__ P, int64_t nw) {
  __shared__ double red[2][kSpecThreads];
  const int64_t iw = blockIdx.x;
  if (iw >= nw) return;
  const double w = omega[iw];
  const double idt2 = 1.0 / (dt * dt);
  double re = 0.0, im = 0.0;
  for (int64_t n = 1 + threadIdx.x; n <= nt1 - 2; n += kSpecThreads) {
    const double t = dt * (double)n;
    const double acc = (mu[(n + 1) * 3 + dir] - 2.0 * mu[n * 3 + dir] + mu[(n - 1) * 3 + dir]) * idt2;
    const double wt = (n == 1 || n == nt1 - 2) ? 0.5 * dt : dt;
    const double f = wt * exp(-t * t / tau) * acc;
    double sn, cs;
    sincos(w * t, &sn, &cs);
    re += f * cs;
    im -= f * sn;
  }
  red[0][threadIdx.x] = re;
  red[1][threadIdx.x] = im;
  __syncthreads();
  for (int h = kSpecThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) P[iw] = red[0][0] * red[0][0] + red[1][0] * red[1][0];
}

}  // namespace

namespace k {

void power_spectrum(const double *mu, int dir, int64_t nt1, double dt, double tau, const double *omega, int64_t nw,
                    double *P, hipStream_t st) {
  hipLaunchKernelGGL(k_power_spectrum, dim3((unsigned)nw), dim3(kSpecThreads), 0, st, mu, dir, nt1, dt, tau, omega,
                     P, nw);
}


void spectrum(const double *mu, const int *dirs, int ndir, int64_t nt1, double dt, double tau, int kind,
              double kappa, double t0, double s, const double *omega, int64_t nw, double *S, double *alpha,
              hipStream_t st) {
  Dirs dd{{0, 0, 0}};
  for (int r = 0; r < ndir && r < 3; ++r) dd.d[r] = dirs[r];
  hipLaunchKernelGGL(k_spectrum, dim3((unsigned)nw), dim3(kSpecThreads), 0, st, mu, dd, ndir, nt1, dt, tau, kind,
                     kappa, t0, s, omega, S, alpha, nw);
}

}  // namespace k
}  // namespace efe
