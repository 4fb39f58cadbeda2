// Device helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace efe {

#define EFE_HOST_DEVICE __host__ __device__ __forceinline__

__device__ __forceinline__ void cell_ijk(const Geom &g, int64_t c, int e[3]) {
  e[0] = (int)(c % g.nc[0]);
  e[1] = (int)((c / g.nc[0]) % g.nc[1]);
  e[2] = (int)(c / ((int64_t)g.nc[0] * g.nc[1]));
}

// Lower corner and edge lengths of cell e (per-axis cell boundaries of the table).
__device__ __forceinline__ void cell_box(const DevData &d, const int e[3], double lo[3], double h[3]) {
  for (int a = 0; a < 3; ++a) {
    const double b0 = d.tab[d.to.xb[a] + e[a]];
    lo[a] = b0;
    h[a] = d.tab[d.to.xb[a] + e[a] + 1] - b0;
  }
}

// Jacobian h_x h_y h_z / 8 of the affine map from the reference cube onto cell c.
__device__ __forceinline__ double cell_jacobian(const DevData &d, int64_t c) {
  int e[3];
  cell_ijk(d.g, c, e);
  double lo[3], h[3];
  cell_box(d, e, lo, h);
  return 0.125 * h[0] * h[1] * h[2];
}

// global node of cell-local index l = a + P (b + P c)
__device__ __forceinline__ int64_t local_node(const Geom &g, const int e[3], int l) {
  int a = l % g.P, b = (l / g.P) % g.P, c = l / (g.P * g.P);
  return ((int64_t)e[0] * g.p + a) + g.nn[0] * (((int64_t)e[1] * g.p + b) + g.nn[1] * ((int64_t)e[2] * g.p + c));
}

// Out-of-place application of a 1-D operator along one axis of a cell tensor
// in[e2][e1][e0][F] -> out (axis extent replaced by m).  interp: out_o = sum_s T[o][s] in_s
// (T = [m][P] basis at points); proj: out_o = sum_s T[s][o] in_s (T = [e_ax][P]).
__device__ __forceinline__ void apply_axis(const double *__restrict__ in, double *__restrict__ out,
                                           const double *__restrict__ T, int P, bool proj, int e0, int e1,
                                           int e2, int ax, int m, int F) {
  const int o0 = ax == 0 ? m : e0, o1 = ax == 1 ? m : e1, o2 = ax == 2 ? m : e2;
  const int dax = ax == 0 ? e0 : (ax == 1 ? e1 : e2);
  const int total = o0 * o1 * o2 * F;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int f = t % F, r = t / F;
    int x = r % o0;
    r /= o0;
    int y = r % o1, z = r / o1;
    int o = ax == 0 ? x : (ax == 1 ? y : z);
    double s = 0.0;
    for (int k = 0; k < dax; ++k) {
      int ix = ax == 0 ? k : x, iy = ax == 1 ? k : y, iz = ax == 2 ? k : z;
      double mv = proj ? T[k * P + o] : T[o * P + k];
      s += mv * in[((iz * e1 + iy) * e0 + ix) * F + f];
    }
    out[t] = s;
  }
}

// Adiabatic LDA potential: Slater exchange v_x = -(3 rho/pi)^(1/3), optionally
// plus Perdew-Wang 1992 correlation v_c = eps_c - (rs/3) d eps_c/d rs.
__device__ __forceinline__ double vxc_lda(double rho, int kind) {
  if (kind == 0 || !(rho > 1e-30)) return 0.0;
  const double pi = 3.14159265358979323846;
  double v = -cbrt(3.0 * rho / pi);
  if (kind == 2) {
    const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
    double rs = cbrt(3.0 / (4.0 * pi * rho));
    double srs = sqrt(rs);
    double q0 = -2.0 * A * (1.0 + a1 * rs);
    double q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
    double dq1 = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
    double lg = log1p(1.0 / q1);
    double ec = q0 * lg;
    double dec = -2.0 * A * a1 * lg - q0 * dq1 / (q1 * q1 + q1);
    v += ec - rs / 3.0 * dec;
  }
  return v;
}

// f_xc = d v_xc / d rho by the fourth-order central difference in log rho
// (step 1e-3: truncation ~1e-12 relative, rounding ~1e-13).
__device__ __forceinline__ double fxc_lda(double rho, int kind) {
  if (kind == 0 || !(rho > 1e-30)) return 0.0;
  const double h = 1e-3;
  const double e1 = exp(h), e2 = exp(2.0 * h);
  const double d = -vxc_lda(rho * e2, kind) + 8.0 * vxc_lda(rho * e1, kind) - 8.0 * vxc_lda(rho / e1, kind) +
                   vxc_lda(rho / e2, kind);
  return d / (12.0 * h * rho);
}

// block-wide sum of one double per thread (blockDim.x <= 1024), result on all threads
__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// BF16 orbital rows: the products with BF16 blocks read a BF16 copy of their input
// (round to nearest even of the FP32 value, as the products would round it)
struct Bf16 {
  uint16_t v;
};
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(double v) { return (float)v; }
__device__ __forceinline__ float to_float(Bf16 v) { return __uint_as_float((uint32_t)v.v << 16); }
// element of a reduced-precision copy from an FP64 value
template <typename T> __device__ __forceinline__ T narrow(double v);
template <> __device__ __forceinline__ float narrow<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ Bf16 narrow<Bf16>(double v) { return Bf16{bf16_bits((float)v)}; }

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace efe
