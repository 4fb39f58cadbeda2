// HIP kernels of the Krylov part of the Magnus step (the cell products are in
// kernels_cell.hip, the Lanczos vector kernels in kernels_lanczos.hip):
//   enrichment coupling of Hbar X (Sec. 2.2-2.3) on the FP64 MFMA;
//   exp(-i tau T_k) e_1 and the a-posteriori estimate (Sec. 2.6, eqs. (AdaptiveKrylov),
//   (AdaptiveKrylovErr)), and the combination coefficients of a finished run.
// Orbital blocks are node-major with ncol interleaved complex columns.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "common.h"

namespace efe {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// The 16x16x4 MFMA of the coupling in FP64, or in FP32 (G and the orbital rows in
// FP32, FP32 accumulation); Acc is the accumulator, row(kr, r) the row of output
// register r of a lane in row group kr = lane / 16 (the column is lane % 16).
__device__ __forceinline__ double to_wide(double v) { return v; }
__device__ __forceinline__ float to_wide(float v) { return v; }

template <typename T> struct CMfma;
template <> struct CMfma<double> {
  typedef v4d Acc;
  static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kr, int r) { return kr + 4 * r; }
};
template <> struct CMfma<float> {
  typedef v4f Acc;
  static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kr, int r) { return 4 * kr + r; }
};

// ---------------------------------------------------------------------------
// Enrichment coupling (Sec. 2.2-2.3), G = Hbar^ce on the union rows R of the
// cells where an enrichment function is nonzero (row-major n_R x n_k):
//   Y_C[R] += G X_E            (added into the rows the cell products wrote)
//   Y_E     = G^T X[R] + Hbar^ee X_E
// on the 16x16x4 MFMA: FP64, or FP32 for the reduced-precision products (G, X and
// Y in FP32, FP32 accumulation; the workgroup partials of Y_E and Hbar^ee X_E in FP64).
//   k_couple_fused (n_k <= 48): both products in one pass over the rows of R.
//   k_couple_c / k_couple_e (any n_k): Y_C by one wave per block over a contiguous
//               range of 16-row tiles (a block covers KNT 16-column tiles); Y_E by
//               workgroups of kCpWaves waves over a contiguous range of tiles, 48
//               columns (blockIdx.y) and 48 functions (blockIdx.z), each wave keeping
//               its Y_E sums in registers.
// Workgroup partials of Y_E are added in LDS in wave order and written per
// workgroup; two reduction kernels sum them in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kCoupleCWaves = 4096;   // four per SIMD
constexpr int KNT = 6;    // 16-column tiles per block (88 columns = 5.5 tiles)

constexpr int kCcMaxK = 48;   // most enrichment directions of the one-pass kernel

// general n_k: one wave per block, X_E from global memory
template <typename GT, typename XT, typename IO>
__global__ void __launch_bounds__(64)
k_couple_c(const DevData d, const GT *__restrict__ G, const XT *__restrict__ X, int64_t ldx, IO *__restrict__ Y,
           int ncolr, int64_t ldr, int64_t tiles_per_wave, const int *__restrict__ any) {
  if (any && *any == 0) return;
  const int nk = d.nk;
  const int64_t nr = d.nr;
  const int lane = threadIdx.x, kr = lane >> 4, cl = lane & 15;
  const int n0 = blockIdx.y * KNT * 16;
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_wave;
  const int64_t t_end = t_begin + tiles_per_wave < ntiles ? t_begin + tiles_per_wave : ntiles;
  const XT *XE = X + (int64_t)d.g.n_nodes * ldx;
  int col[KNT];
  bool cok[KNT];
#pragma unroll
  for (int nt = 0; nt < KNT; ++nt) {
    col[nt] = n0 + nt * 16 + cl;
    cok[nt] = col[nt] < ncolr;
  }
  const int nks = (nk + 3) / 4;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t r0 = t * 16;
    // A(i, k) = G[r0 + i][k], B(k, j) = X_E[k][j]
    typename CMfma<GT>::Acc acc[KNT];
#pragma unroll
    for (int nt = 0; nt < KNT; ++nt) acc[nt] = typename CMfma<GT>::Acc{0, 0, 0, 0};
    const int64_t ra = r0 + cl;
    const bool rok = ra < nr;
    for (int ks = 0; ks < nks; ++ks) {
      const int k = ks * 4 + kr;
      const bool kok = k < nk;
      const GT a = (rok && kok) ? G[ra * nk + k] : (GT)0;
#pragma unroll
      for (int nt = 0; nt < KNT; ++nt) {
        const GT b = (kok && cok[nt]) ? (GT)to_wide(XE[(int64_t)k * ldx + col[nt]]) : (GT)0;
        acc[nt] = CMfma<GT>::mma(a, b, acc[nt]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + CMfma<GT>::row(kr, r);
      if (row < nr) {
        IO *y = Y + (int64_t)d.urow_node[row] * ldr;
#pragma unroll
        for (int nt = 0; nt < KNT; ++nt)
          if (cok[nt]) y[col[nt]] += (IO)acc[nt][r];
      }
    }
  }
}

constexpr int kCpWaves = 4;
constexpr int kCpBlocks = 512;   // workgroups per 48-column slice
constexpr int kCpNT = 3;         // 16-column tiles per slice
constexpr int kCpMT = 3;         // 16-row tiles of Y_E (n_k <= 48)
constexpr int kCpSlices = 8;     // first-level reduction slices
static_assert(kCpBlocks + kCpSlices <= k::kCoupleScratch, "coupling scratch");

template <typename GT, typename XT>
__global__ void __launch_bounds__(kCpWaves * 64) __attribute__((amdgpu_waves_per_eu(3)))
k_couple_e(const DevData d, const GT *__restrict__ G, const XT *__restrict__ X, int ncolr, int64_t ldx,
           int64_t tiles_per_block, double *__restrict__ part, const int *__restrict__ any) {
  if (any && *any == 0) return;
  __shared__ double red[kCpMT * 16 * kCpNT * 16];
  const int nk = d.nk;
  const int64_t nr = d.nr;
  const int tid = threadIdx.x, lane = tid & 63, kr = lane >> 4, cl = lane & 15;
  const int wave = tid >> 6;
  const int n0 = blockIdx.y * kCpNT * 16, m0 = blockIdx.z * kCpMT * 16;
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_block;
  const int64_t t_end = t_begin + tiles_per_block < ntiles ? t_begin + tiles_per_block : ntiles;
  int col[kCpNT];
  bool cok[kCpNT];
#pragma unroll
  for (int nt = 0; nt < kCpNT; ++nt) {
    col[nt] = n0 + nt * 16 + cl;
    cok[nt] = col[nt] < ncolr;
  }
  typename CMfma<GT>::Acc acc_e[kCpMT][kCpNT];
#pragma unroll
  for (int mt = 0; mt < kCpMT; ++mt)
#pragma unroll
    for (int nt = 0; nt < kCpNT; ++nt) acc_e[mt][nt] = typename CMfma<GT>::Acc{0, 0, 0, 0};
  for (int64_t t = t_begin + wave; t < t_end; t += kCpWaves) {
    const int64_t r0 = t * 16;
    // Y_E sums: A(i, k) = G[r0 + 4 s + k][16 mt + i], B(k, j) = X[node(r0 + 4 s + k)][j]
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int64_t rk = r0 + 4 * s4 + kr;
      const bool ok = rk < nr;
      const XT *xr = X + (ok ? (int64_t)d.urow_node[rk] * ldx : 0);
      GT b[kCpNT];
#pragma unroll
      for (int nt = 0; nt < kCpNT; ++nt) b[nt] = (ok && cok[nt]) ? (GT)to_wide(xr[col[nt]]) : (GT)0;
#pragma unroll
      for (int mt = 0; mt < kCpMT; ++mt) {
        const int m = m0 + mt * 16 + cl;
        const GT a = (ok && m < nk) ? G[rk * nk + m] : (GT)0;
#pragma unroll
        for (int nt = 0; nt < kCpNT; ++nt) acc_e[mt][nt] = CMfma<GT>::mma(a, b[nt], acc_e[mt][nt]);
      }
    }
  }
  // workgroup partial of Y_E: red[m][c] = sum over waves in wave order
  for (int w = 0; w < kCpWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int mt = 0; mt < kCpMT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nt = 0; nt < kCpNT; ++nt) {
            const int idx = (mt * 16 + CMfma<GT>::row(kr, r)) * (kCpNT * 16) + nt * 16 + cl;
            red[idx] = (w == 0 ? 0.0 : red[idx]) + (double)acc_e[mt][nt][r];
          }
    }
    __syncthreads();
  }
  // part[block][m][column]
  double *pb = part + (int64_t)blockIdx.x * nk * ncolr;
  for (int idx = tid; idx < kCpMT * 16 * kCpNT * 16; idx += kCpWaves * 64) {
    const int m = m0 + idx / (kCpNT * 16), c = n0 + idx % (kCpNT * 16);
    if (m < nk && c < ncolr) pb[(int64_t)m * ncolr + c] = red[idx];
  }
}

// Both products in one pass over the union rows (n_k <= 48): per 16-row tile a wave
// loads the tile's G rows, and the X and Y rows of its column slice, once; it adds G X_E
// into the Y rows and accumulates G^T X[R] in registers.  The four rows a lane holds are
// the rows of its output registers for Y_C, and the same rows serve as its k rows for
// Y_E (step s takes row(kr, s)), so one gather of node offsets covers both products.
// The node offsets of the wave's next tile are loaded while the current tile's
// products run.  Workgroup (range, slice) partials of Y_E are summed in LDS in wave
// order and reduced by k_couple_sum as those of k_couple_e.
constexpr int kCfWaves = 4;
constexpr int kCfRanges = kCpBlocks;   // tile ranges: one partial block each

template <typename GT, typename XT, typename IO, int NT>
__global__ void __launch_bounds__(kCfWaves * 64) __attribute__((amdgpu_waves_per_eu(2)))
k_couple_fused(const DevData d, const GT *__restrict__ G, const XT *__restrict__ X, int64_t ldx,
               IO *__restrict__ Y, int ncolr, int64_t ldr, int64_t tiles_per_range, int nranges, int nslice,
               double *__restrict__ part, const int *__restrict__ any) {
  if (any && *any == 0) return;
  constexpr int kMT = kCcMaxK / 16;
  constexpr int kNC = NT * 16;
  __shared__ GT xe[kCcMaxK * kNC];
  __shared__ double red[kMT * 16 * kNC];
  const int nk = d.nk;
  const int64_t nr = d.nr;
  const int b = blockIdx.x, xcd = b & 7, q = b >> 3;
  const int slice = q % nslice, range = (q / nslice) * 8 + xcd;
  if (range >= nranges) return;   // the whole workgroup: no barrier is left waiting
  const int tid = threadIdx.x, lane = tid & 63, kr = lane >> 4, cl = lane & 15, wave = tid >> 6;
  const int n0 = slice * kNC;
  const XT *XE = X + (int64_t)d.g.n_nodes * ldx;
  for (int i = tid; i < kCcMaxK * kNC; i += kCfWaves * 64) {
    const int k = i / kNC, c = n0 + i % kNC;
    xe[i] = (k < nk && c < ncolr) ? (GT)to_wide(XE[(int64_t)k * ldx + c]) : (GT)0;
  }
  __syncthreads();
  int col[NT];
  bool cok[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    col[nt] = n0 + nt * 16 + cl;
    cok[nt] = col[nt] < ncolr;
  }
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)range * tiles_per_range;
  const int64_t t_end = t_begin + tiles_per_range < ntiles ? t_begin + tiles_per_range : ntiles;
  typename CMfma<GT>::Acc acc_e[kMT][NT];
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc_e[mt][nt] = typename CMfma<GT>::Acc{0, 0, 0, 0};
  int64_t nd[4];   // nodes of the lane's rows of the tile (-1 past n_R)
  int64_t t = t_begin + wave;
  if (t < t_end) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = t * 16 + CMfma<GT>::row(kr, r);
      nd[r] = row < nr ? d.urow_node[row] : -1;
    }
  }
  for (; t < t_end; t += kCfWaves) {
    const int64_t r0 = t * 16;
    const int64_t ra = r0 + cl;
    const bool rok = ra < nr;
    GT a[kCcMaxK / 4];   // Y_C: A(i, k) = G[r0 + i][k]
#pragma unroll
    for (int ks = 0; ks < kCcMaxK / 4; ++ks) {
      const int k = ks * 4 + kr;
      a[ks] = (rok && k < nk) ? G[ra * nk + k] : (GT)0;
    }
    GT ae[4][kMT];       // Y_E: A(i, k) = G[row(k, s)][16 mt + i]
    GT xv[4][NT];        //      B(k, j) = X[node(row(k, s))][j]
    IO yv[4][NT];
    int64_t nc[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int64_t row = r0 + CMfma<GT>::row(kr, s4);
      const bool ok = row < nr;
#pragma unroll
      for (int mt = 0; mt < kMT; ++mt) {
        const int m = mt * 16 + cl;
        ae[s4][mt] = (ok && m < nk) ? G[row * nk + m] : (GT)0;
      }
      nc[s4] = nd[s4];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bool v = nc[s4] >= 0 && cok[nt];
        xv[s4][nt] = v ? (GT)to_wide(X[nc[s4] * ldx + col[nt]]) : (GT)0;
        yv[s4][nt] = v ? Y[nc[s4] * ldr + col[nt]] : (IO)0;
      }
    }
    if (t + kCfWaves < t_end) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = (t + kCfWaves) * 16 + CMfma<GT>::row(kr, r);
        nd[r] = row < nr ? d.urow_node[row] : -1;
      }
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc_e[mt][nt] = CMfma<GT>::mma(ae[s4][mt], xv[s4][nt], acc_e[mt][nt]);
    typename CMfma<GT>::Acc acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = typename CMfma<GT>::Acc{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < kCcMaxK / 4; ++ks)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[nt] = CMfma<GT>::mma(a[ks], xe[(ks * 4 + kr) * kNC + nt * 16 + cl], acc[nt]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (nc[r] < 0) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        if (cok[nt]) Y[nc[r] * ldr + col[nt]] = yv[r][nt] + (IO)acc[nt][r];
    }
  }
  // workgroup partial of Y_E: red[m][c] = sum over waves in wave order
  for (int w = 0; w < kCfWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int idx = (mt * 16 + CMfma<GT>::row(kr, r)) * kNC + nt * 16 + cl;
            red[idx] = (w == 0 ? 0.0 : red[idx]) + (double)acc_e[mt][nt][r];
          }
    }
    __syncthreads();
  }
  double *pb = part + (int64_t)range * nk * ncolr;
  for (int i = tid; i < kMT * 16 * kNC; i += kCfWaves * 64) {
    const int m = i / kNC, c = n0 + i % kNC;
    if (m < nk && c < ncolr) pb[(int64_t)m * ncolr + c] = red[i];
  }
}

// first level: lvl1[s][o] = sum of the partials of slice s (a contiguous range
// of workgroups); the four quarters of a block take every fourth partial of
// the range and are combined in a fixed order
__global__ void __launch_bounds__(256)
k_couple_sum(const double *__restrict__ part, int nblk, int nout, double *__restrict__ lvl1,
             const int *__restrict__ any) {
  if (any && *any == 0) return;
  __shared__ double red[4][64];
  const int o = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6, sl = blockIdx.y;
  const int per = (nblk + kCpSlices - 1) / kCpSlices;
  const int b0 = sl * per, b1 = b0 + per < nblk ? b0 + per : nblk;
  double s = 0.0;
  if (o < nout)
    for (int b = b0 + q; b < b1; b += 4) s += part[(int64_t)b * nout + o];
  red[q][threadIdx.x & 63] = s;
  __syncthreads();
  if (q != 0 || o >= nout) return;
  const int lo = threadIdx.x;
  lvl1[(int64_t)sl * nout + o] = red[0][lo] + red[1][lo] + red[2][lo] + red[3][lo];
}

// Y_E[k][c] = sum_s lvl1[s][k][c] + sum_k' Hbar^ee[k][k'] X_E[k'][c].  With aE, also the
// enrichment terms of x^H Hbar x: aE[k][c] = X_E[k][c] (p + Y_E[k][c]) with p = (G^T X[R])[k][c],
// since the rows R add sum_k X_E[k][c] p to it through Y_C[R] += G X_E (G real).
template <typename XT, typename IO>
__global__ void __launch_bounds__(64)
k_couple_final(const DevData d, const double *__restrict__ lvl1, int nsl, const double *__restrict__ Hee,
               const XT *__restrict__ X, int64_t ldx, IO *__restrict__ Y, int ncolr, int64_t ldr,
               const int *__restrict__ any, double *__restrict__ aE) {
  if (any && *any == 0) return;
  const int nk = d.nk, nout = nk * ncolr;
  const int o = blockIdx.x * 64 + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int sl = 0; sl < nsl; ++sl) s += lvl1[(int64_t)sl * nout + o];
  const double p = s;
  const int k = o / ncolr, c = o % ncolr;
  for (int kp = 0; kp < nk; ++kp) s += Hee[k * nk + kp] * (double)to_wide(X[(d.g.n_nodes + kp) * ldx + c]);
  Y[(d.g.n_nodes + k) * ldr + c] = (IO)s;
  if (aE) aE[o] = (double)to_wide(X[(d.g.n_nodes + k) * ldx + c]) * (p + s);
}

// ---------------------------------------------------------------------------
// Per column: eigendecomposition of the j x j symmetric tridiagonal T_j by the
// implicit QL method with Wilkinson-type shifts (Bowdler, Martin, Reinsch and
// Wilkinson, 1968), u = V exp(-i tau Lambda) V^T e_1, the estimate
// |tau| beta_j beta0 |u_j| and the stopping decision.  One wavefront per
// column; lane k owns row k of V (j <= 64).
// ---------------------------------------------------------------------------
// Implicit QL on the n x n tridiagonal (dd diagonal, ee off-diagonal) in LDS,
// accumulating the eigenvectors in Z (initialised to I by the caller).  One
// wavefront; returns false if an eigenvalue needed more than 60 sweeps.
__device__ bool tridiag_ql(int n, double (*Z)[65], double *dd, double *ee, int lane) {
  bool fail = false;
  for (int l = 0; l < n && !fail; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        double s = fabs(dd[m]) + fabs(dd[m + 1]);
        if (fabs(ee[m]) <= DBL_EPSILON * s) break;
      }
      if (m == l) break;
      if (++iter > 60) { fail = true; break; }
      double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
      double r = hypot(g, 1.0);
      g = dd[m] - dd[l] + ee[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
      double s = 1.0, co = 1.0, p = 0.0;
      bool early = false;
      for (int i = m - 1; i >= l; --i) {
        double f = s * ee[i], b = co * ee[i];
        r = hypot(f, g);
        __syncthreads();
        if (lane == 0) ee[i + 1] = r;
        __syncthreads();
        if (r == 0.0) {
          __syncthreads();
          if (lane == 0) { dd[i + 1] -= p; ee[m] = 0.0; }
          __syncthreads();
          early = true;
          break;
        }
        s = f / r;
        co = g / r;
        g = dd[i + 1] - p;
        r = (dd[i] - g) * s + 2.0 * co * b;
        p = s * r;
        __syncthreads();
        if (lane == 0) dd[i + 1] = g + p;
        __syncthreads();
        g = co * r - b;
        if (lane < n) {
          double zf = Z[lane][i + 1], zi = Z[lane][i];
          Z[lane][i + 1] = s * zi + co * zf;
          Z[lane][i] = co * zi - s * zf;
        }
      }
      if (early) continue;
      __syncthreads();
      if (lane == 0) { dd[l] -= p; ee[l] = g; ee[m] = 0.0; }
      __syncthreads();
    }
  }
  __syncthreads();
  return !fail;
}

__global__ void __launch_bounds__(64)
k_tridiag_exp(const double *__restrict__ alpha, const double *__restrict__ beta, int j, int ncol, int kmax,
              double tau, const double *__restrict__ beta0, const int *__restrict__ kforce, double tol,
              int *__restrict__ active, int *__restrict__ kused, double *__restrict__ err, double *__restrict__ ubuf) {
  __shared__ double Z[64][65];
  __shared__ double dd[64], ee[64];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  if (!active[c]) return;
  const int n = j;
  for (int k = 0; k < n; ++k) Z[lane][k] = (lane == k) ? 1.0 : 0.0;
  if (lane < n) {
    dd[lane] = alpha[(int64_t)lane * ncol + c];
    ee[lane] = lane < n - 1 ? beta[(int64_t)lane * ncol + c] : 0.0;
  }
  __syncthreads();
  const bool fail = !tridiag_ql(n, Z, dd, ee, lane);
  __syncthreads();
  // u_k = sum_m Z[k][m] exp(-i tau lam_m) Z[0][m]
  double ur = 0.0, ui = 0.0;
  if (lane < n) {
    for (int m = 0; m < n; ++m) {
      double z0 = Z[0][m], ph = -tau * dd[m];
      double sn, cs;
      sincos(ph, &sn, &cs);
      ur += Z[lane][m] * z0 * cs;
      ui += Z[lane][m] * z0 * sn;
    }
  }
  // broadcast u_{n-1}
  double un_r = __shfl(ur, n - 1, 64), un_i = __shfl(ui, n - 1, 64);
  double bj = beta[(int64_t)(j - 1) * ncol + c];
  double tn = 0.0;
  for (int i = 0; i < n; ++i) {
    double v = fabs(alpha[(int64_t)i * ncol + c]) + (i > 0 ? beta[(int64_t)(i - 1) * ncol + c] : 0.0) +
               beta[(int64_t)i * ncol + c];
    tn = v > tn ? v : tn;
  }
  const double b0 = beta0[c];
  const double est = fabs(tau) * bj * b0 * hypot(un_r, un_i);
  bool done;
  if (kforce) done = j >= kforce[c] || bj == 0.0;
  else done = est <= tol * b0 || bj <= 1e-14 * tn;
  if (fail) done = false;
  if (lane == 0) err[c] = fail ? -1.0 : est;
  if (done) {
    if (lane < n) {
      ubuf[((int64_t)c * kmax + lane) * 2] = ur;
      ubuf[((int64_t)c * kmax + lane) * 2 + 1] = ui;
    }
    if (lane == 0) {
      kused[c] = j;
      active[c] = 0;
    }
  }
}

// Krylov combination coefficients of a finished Lanczos for several times:
//   coef[g][l][c] = beta0 sig_l [exp(-i tau_g T_{k_c}) e_1]_l  (l < k_c; 0 up to kmax)
// with k_c = kused[c], so that sum_l coef[g][l][c] slot_l = exp(-i tau_g A) x_c in
// the Krylov space of the run.  One wavefront per column.
struct TauList {
  double tau[16];
};

__global__ void __launch_bounds__(64)
k_tridiag_coef(const double *__restrict__ alpha, const double *__restrict__ beta, const int *__restrict__ kused,
               int ncol, int kmax, TauList taus, int m, const double *__restrict__ beta0,
               const double *__restrict__ sig, double2 *__restrict__ coef) {
  __shared__ double Z[64][65];
  __shared__ double dd[64], ee[64];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = kused[c];
  if (n > 0) {
    for (int k = 0; k < n; ++k) Z[lane][k] = (lane == k) ? 1.0 : 0.0;
    if (lane < n) {
      dd[lane] = alpha[(int64_t)lane * ncol + c];
      ee[lane] = lane < n - 1 ? beta[(int64_t)lane * ncol + c] : 0.0;
    }
    __syncthreads();
    tridiag_ql(n, Z, dd, ee, lane);
  }
  for (int g = 0; g < m; ++g) {
    for (int l = lane; l < kmax; l += 64) {
      double ur = 0.0, ui = 0.0;
      if (l < n) {
        for (int p = 0; p < n; ++p) {
          double sn, cs;
          sincos(-taus.tau[g] * dd[p], &sn, &cs);
          ur += Z[l][p] * Z[0][p] * cs;
          ui += Z[l][p] * Z[0][p] * sn;
        }
        const double f = beta0[c] * sig[(int64_t)l * ncol + c];
        ur *= f;
        ui *= f;
      }
      coef[((int64_t)g * kmax + l) * ncol + c] = make_double2(ur, ui);
    }
  }
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename GT, typename XT, typename IO>
void couple_apply_t(const DevData &d, const GT *G, const double *Hee, const XT *X, int64_t ldx, IO *Y, int ncolr,
                    int64_t ldr, double *scratch, hipStream_t s, const int *any, double *aE = nullptr) {
  if (d.nk == 0) return;
  const int nout = d.nk * ncolr;
  double *lvl1 = scratch + (int64_t)kCpBlocks * nout;
  int nsl = 1;
  if (d.nr > 0 && d.nk <= kCcMaxK) {
    // one pass: 48-column slices for FP32 rows and blocks, 32-column slices where the
    // G or X values are FP64 (the Y_E sums of a 48-column slice would spill)
    constexpr int NT = (sizeof(GT) == 4 && sizeof(XT) == 4) ? 3 : 2;
    const int64_t ntiles = (d.nr + 15) / 16;
    const int64_t tpr = (ntiles + kCfRanges - 1) / kCfRanges;
    const int nranges = (int)((ntiles + tpr - 1) / tpr);
    const int nslice = (ncolr + NT * 16 - 1) / (NT * 16);
    const unsigned nb = (unsigned)(((nranges + 7) / 8) * 8 * nslice);
    hipLaunchKernelGGL((k_couple_fused<GT, XT, IO, NT>), dim3(nb), dim3(kCfWaves * 64), 0, s, d, G, X, ldx, Y, ncolr, ldr,
                       tpr, nranges, nslice, scratch, any);
    nsl = kCpSlices;
    hipLaunchKernelGGL(k_couple_sum, dim3(nblocks((int64_t)nout, 64), kCpSlices), dim3(256), 0, s, scratch, nranges, nout,
                       lvl1, any);
  } else if (d.nr > 0) {
    const int64_t ntiles = (d.nr + 15) / 16;
    const int64_t tpb = (ntiles + kCpBlocks - 1) / kCpBlocks;
    const int nblk = (int)((ntiles + tpb - 1) / tpb);
    const unsigned ny = (unsigned)((ncolr + kCpNT * 16 - 1) / (kCpNT * 16));
    const unsigned nz = (unsigned)((d.nk + kCpMT * 16 - 1) / (kCpMT * 16));
    const unsigned nyc = (unsigned)((ncolr + KNT * 16 - 1) / (KNT * 16));
    const int64_t tpc = (ntiles + kCoupleCWaves - 1) / kCoupleCWaves;
    hipLaunchKernelGGL((k_couple_c<GT, XT, IO>), dim3((unsigned)((ntiles + tpc - 1) / tpc), nyc), dim3(64), 0, s, d, G, X,
                       ldx, Y, ncolr, ldr, tpc, any);
    hipLaunchKernelGGL((k_couple_e<GT, XT>), dim3((unsigned)nblk, ny, nz), dim3(kCpWaves * 64), 0, s, d, G, X, ncolr,
                       ldx, tpb, scratch, any);
    nsl = kCpSlices;
    hipLaunchKernelGGL(k_couple_sum, dim3(nblocks((int64_t)nout, 64), kCpSlices), dim3(256), 0, s, scratch, nblk, nout,
                       lvl1, any);
  } else {
    k::zero(lvl1, (int64_t)nout, s);
  }
  hipLaunchKernelGGL((k_couple_final<XT, IO>), dim3(nblocks((int64_t)nout, 64)), dim3(64), 0, s, d, lvl1, nsl, Hee, X, ldx,
                     Y, ncolr, ldr, any, aE);
}

}  // namespace

namespace k {

void couple_apply(const DevData &d, const double *G, const double *Hee, const double *X, double *Y, int ncolr,
                  int64_t ldr, double *scratch, hipStream_t s, const int *any, double *aE) {
  couple_apply_t(d, G, Hee, X, ldr, Y, ncolr, ldr, scratch, s, any, aE);
}

void couple_apply_g32(const DevData &d, const float *G, const double *Hee, const double *X, double *Y, int ncolr,
                      int64_t ldr, double *scratch, hipStream_t s, const int *any) {
  couple_apply_t(d, G, Hee, X, ldr, Y, ncolr, ldr, scratch, s, any);
}

void couple_apply_f(const DevData &d, const float *G, const double *Hee, const float *X, const double *X64,
                    float *Y, int ncolr, int64_t ldf, double *scratch, hipStream_t s, const int *any) {
  if (X64) couple_apply_t(d, G, Hee, X64, (int64_t)ncolr, Y, ncolr, ldf, scratch, s, any);
  else couple_apply_t(d, G, Hee, X, ldf, Y, ncolr, ldf, scratch, s, any);
}

void tridiag_coef(const double *alpha, const double *beta, const int *kused, int ncol, int kmax, const double *taus,
                  int m, const double *beta0, const double *sig, double *coef, hipStream_t s) {
  TauList tl{};
  for (int g = 0; g < m && g < 16; ++g) tl.tau[g] = taus[g];
  hipLaunchKernelGGL(k_tridiag_coef, dim3(ncol), dim3(64), 0, s, alpha, beta, kused, ncol, kmax, tl, m < 16 ? m : 16,
                     beta0, sig, (double2 *)coef);
}

void tridiag_exp(const double *alpha, const double *beta, int j, int ncol, int kmax, double tau, const double *beta0,
                 const int *kforce, double tol, int *active, int *kused, double *err, double *u, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_exp, dim3(ncol), dim3(64), 0, s, alpha, beta, j, ncol, kmax, tau, beta0, kforce, tol,
                     active, kused, err, u);
}

}  // namespace k
}  // namespace efe
