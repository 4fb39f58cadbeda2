// HIP kernels of the Krylov part of the Magnus step:
//   Hbar X  = sum_c P_c^T Hbar_c P_c X  (cell blocks on MFMA) + enrichment coupling
//   Lanczos recurrence with full reorthogonalisation (Sec. 2.6, eq. (AdaptiveKrylov))
//   exp(-i tau T_k) e_1 and the a-posteriori estimate (eq. (AdaptiveKrylovErr))
//   Krylov combination beta0 Q_k u.
// Orbital blocks are node-major with ncol interleaved complex columns.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "common.cuh"

namespace efe {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Cell products Y[nodes_c] += Hbar_c X[nodes_c] for the cells of one colour
// (no two cells of a colour share a node; the 8 colours are the parity
// classes of the cell index and run one launch each, in order).  The first
// colour to reach a node stores instead of adding, so Y needs no clearing
// beforehand.  Hbar_c is symmetric, so row k of the row-major block is the
// MFMA A-operand column k; the 16x16x4 MFMA accumulates in registers.
// ---------------------------------------------------------------------------
constexpr int kApplyMaxLoc = 384;   // nloc of degree <= 6 is 343

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double C;
  typedef v4d Acc;
  static __device__ __forceinline__ Acc mma(C a, C b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // output register r of a lane holds row lane/16 + 4 r, column lane%16
  static __device__ __forceinline__ int row(int kr, int r) { return kr + 4 * r; }
};
template <> struct Mfma<float> {
  typedef float C;
  typedef v4f Acc;
  static __device__ __forceinline__ Acc mma(C a, C b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // output register r of a lane holds row 4 (lane/16) + r, column lane%16
  static __device__ __forceinline__ int row(int kr, int r) { return 4 * kr + r; }
};

// One workgroup of 8 waves per (cell, chunk of 96 columns); two workgroups
// share a CU.  Operands pass through LDS in chunks of 8 k-rows, three chunks in
// flight: the chunk's rows of the symmetric cell block (contiguous in memory)
// and the gathered rows of X are copied global -> LDS by the direct-to-LDS
// loads (global_load_lds_dwordx4, 16 B per lane at LDS base + 16 * lane), so
// no registers hold data in flight.  Every wave issues the same number of
// copies per chunk (padding copies land in a scratch line), which lets a
// fixed vmcnt wait certify that the chunk has arrived before the barrier.
// Wave w takes the M tiles (w >> 1) + 4 i and the three 16-column N tiles of
// half (w & 1): every SIMD then carries the same number of tiles.
constexpr int kCellWaves = 8;
constexpr int kCellNT = 3;                  // N tiles per wave
constexpr int kCellCols = 2 * kCellNT * 16; // columns per workgroup
constexpr int kCellKC = 8;                  // k-rows per chunk
constexpr int kCellNS = 3;                  // chunks in flight
constexpr int kCellLDX = 112;               // LDS row stride of X (doubles): the 4 rows of a B read hit disjoint banks
constexpr int kCellXStage = kCellKC * kCellLDX * 8;

// s_waitcnt with vmcnt = N and no wait on the other counters (gfx9 encoding)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

typedef const void __attribute__((address_space(1))) *gptr_t;
typedef void __attribute__((address_space(3))) *lptr_t;

__device__ __forceinline__ void copy16_to_lds(const void *src, void *lds_base) {
  __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)lds_base, 16, 0, 0);
}

template <typename T>
struct CellChunk {
  // A-chunk copies per wave per chunk, sized for the largest cell (nloc <= 384)
  static constexpr int kAIns = (kCellKC * kApplyMaxLoc * (int)sizeof(T) + 1024 * kCellWaves - 1) / (1024 * kCellWaves);
  static constexpr int kPer = kAIns + kCellKC / kCellWaves;   // copies per wave per chunk
};

inline size_t cell_lds_bytes(int nloc, size_t esz) {
  const size_t aseg = (kCellKC * nloc * esz + 1023) / 1024;
  return kCellNS * (aseg * 1024 + kCellXStage) + 1024;
}

template <typename T, int CMT>
__global__ void __launch_bounds__(kCellWaves * 64)
k_cell_apply(const DevData d, const int *__restrict__ cell_list, int slot0, const T *__restrict__ cells,
             const double *__restrict__ X, double *__restrict__ Y, int ncolr, int64_t ldr, const int *__restrict__ any) {
  if (any && *any == 0) return;
  typedef typename Mfma<T>::C C;
  typedef typename Mfma<T>::Acc Acc;
  constexpr int kAIns = CellChunk<T>::kAIns, kPer = CellChunk<T>::kPer;
  __shared__ int64_t rowoff[kApplyMaxLoc];
  __shared__ unsigned char first[kApplyMaxLoc];   // this cell's colour is the first to reach the node
  extern __shared__ __attribute__((aligned(16))) unsigned char cell_sm[];
  const Geom &g = d.g;
  const int nloc = g.nloc;
  const int abytes = kCellKC * nloc * (int)sizeof(T);
  const int aseg = (abytes + 1023) / 1024;
  unsigned char *As = cell_sm;                                   // kCellNS * aseg KB
  unsigned char *Xs = cell_sm + kCellNS * aseg * 1024;           // kCellNS * kCellXStage
  unsigned char *junk = Xs + kCellNS * kCellXStage;              // 1 KB target of padding copies
  const int ci = blockIdx.x;
  const int col0 = blockIdx.y * kCellCols;
  const int wcol = ncolr - col0 < kCellCols ? ncolr - col0 : kCellCols;   // columns of this chunk (even)
  const int64_t cell = cell_list[ci];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kr = lane >> 4, cl = lane & 15;
  const int mg = wave >> 1, nh = wave & 1;
  int e[3];
  cell_ijk(g, cell, e);
  for (int l = tid; l < nloc; l += kCellWaves * 64) {
    rowoff[l] = local_node(g, e, l) * ldr;
    // colours run in the order (e_x & 1) + 2 (e_y & 1) + 4 (e_z & 1); a node on a
    // face shared along some axis is reached first by the even cell of that axis
    const int li[3] = {l % g.P, (l / g.P) % g.P, l / (g.P * g.P)};
    bool later = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const bool shared = (li[ax] == 0 && e[ax] > 0) || (li[ax] == g.p && e[ax] < g.nc[ax] - 1);
      later |= shared && (e[ax] & 1);
    }
    first[l] = later ? 0 : 1;
  }
  // X stages start zeroed: pad columns are never copied into
  for (int i = tid; i < kCellNS * kCellXStage / 8; i += kCellWaves * 64) ((double *)Xs)[i] = 0.0;
  __syncthreads();
  const unsigned char *Ag = (const unsigned char *)(cells + (int64_t)(slot0 + ci) * g.cstride);   // 16-byte aligned
  const int64_t ablock = g.cstride * (int64_t)sizeof(T);   // padded block: copies never cross into the next one
  const int nchunk = (nloc + kCellKC - 1) / kCellKC;
  auto issue = [&](int kc) {
    const int st = kc % kCellNS;
    const int64_t abase = (int64_t)kc * abytes;
#pragma unroll
    for (int i = 0; i < kAIns; ++i) {
      const int seg = wave + kCellWaves * i;
      const int64_t off = abase + (int64_t)seg * 1024 + lane * 16;
      const bool ok = seg < aseg && off + 16 <= ablock;
      copy16_to_lds(Ag + (ok ? off : 0), seg < aseg ? As + (st * aseg + seg) * 1024 : junk);
    }
#pragma unroll
    for (int i = 0; i < kCellKC / kCellWaves; ++i) {
      const int r = wave + kCellWaves * i;
      const int k = kc * kCellKC + r;
      if (k < nloc) {
        if (2 * lane < wcol) copy16_to_lds(X + rowoff[k] + col0 + 2 * lane, Xs + st * kCellXStage + r * kCellLDX * 8);
      } else {
        copy16_to_lds(X, junk);
      }
    }
  };
  const int nmt = (nloc + 15) / 16;
  Acc acc[CMT][kCellNT];
#pragma unroll
  for (int i = 0; i < CMT; ++i)
#pragma unroll
    for (int j = 0; j < kCellNT; ++j) acc[i][j] = Acc{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < kCellNS - 1; ++c)
    if (c < nchunk) issue(c);
  for (int kc = 0; kc < nchunk; ++kc) {
    // this wave's copies of chunk kc are done once at most (chunks issued after it) * kPer remain
    if (kc + 1 < nchunk) wait_vmcnt<kPer * (kCellNS - 2)>();
    else wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (kc + kCellNS - 1 < nchunk) issue(kc + kCellNS - 1);
    const int st = kc % kCellNS;
    const T *Al = (const T *)(As + st * aseg * 1024);
    const double *Xl = (const double *)(Xs + st * kCellXStage);
#pragma unroll
    for (int s4 = 0; s4 < kCellKC / 4; ++s4) {
      const int kl = s4 * 4 + kr;
      const bool kok = kc * kCellKC + kl < nloc;
      C b[kCellNT];
#pragma unroll
      for (int j = 0; j < kCellNT; ++j) b[j] = (C)Xl[kl * kCellLDX + (nh * kCellNT + j) * 16 + cl];
#pragma unroll
      for (int i = 0; i < CMT; ++i) {
        const int t = mg + 4 * i;
        if (t < nmt) {
          const int m = t * 16 + cl;
          const C a = (kok && m < nloc) ? (C)Al[kl * nloc + m] : (C)0;
#pragma unroll
          for (int j = 0; j < kCellNT; ++j) acc[i][j] = Mfma<T>::mma(a, b[j], acc[i][j]);
        }
      }
    }
  }
  // D layout of the 16x16 MFMA (differs between the f64 and f32 forms)
#pragma unroll
  for (int i = 0; i < CMT; ++i) {
    if (mg + 4 * i >= nmt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = (mg + 4 * i) * 16 + Mfma<T>::row(kr, r);
      if (row >= nloc) continue;
      double *yr = Y + rowoff[row];
      const bool f = first[row] != 0;
#pragma unroll
      for (int j = 0; j < kCellNT; ++j) {
        const int col = col0 + (nh * kCellNT + j) * 16 + cl;
        if (col < ncolr) yr[col] = f ? (double)acc[i][j][r] : yr[col] + (double)acc[i][j][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Enrichment coupling: Y_C[r] += G[r] X_E ;  Y_E = G^T X_C[R] + Hbar^ee X_E
// (G = Hbar^ce on the union rows R of the cells where an enrichment function
// is nonzero, row-major n_R x n_k).  One wave per block walks a contiguous
// range of 16-row tiles of R on the FP64 16x16x4 MFMA; a block covers KNT
// 16-column tiles (blockIdx.y).
//   k_couple_c:  Y_C tile (16 x 16 N) += G tile (16 x n_k) . X_E (n_k x 16 N),
//                added into Y.
//   k_couple_e:  Y_E (16 M x 16 N) += G tile^T (16 M x 16 rows) . X[R tile],
//                KMT M tiles per block (blockIdx.z), kept in registers over the
//                range and written as the wave's partial sum; the partials are
//                reduced in a fixed order (deterministic).
constexpr int kCoupleCWaves = 4096;   // four per SIMD
constexpr int KNT = 6;    // 16-column tiles per block (88 columns = 5.5 tiles)
constexpr int KMT = 3;    // 16-row tiles of Y_E per block (48 functions)

__global__ void __launch_bounds__(64)
k_couple_c(const DevData d, const double *__restrict__ G, const double *__restrict__ X, double *__restrict__ Y,
           int ncolr, int64_t ldr, int64_t tiles_per_wave, const int *__restrict__ any) {
  if (any && *any == 0) return;
  const int nk = d.nk;
  const int64_t nr = d.nr;
  const int lane = threadIdx.x, kr = lane >> 4, cl = lane & 15;
  const int n0 = blockIdx.y * KNT * 16;
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_wave;
  const int64_t t_end = t_begin + tiles_per_wave < ntiles ? t_begin + tiles_per_wave : ntiles;
  const double *XE = X + (int64_t)d.g.n_nodes * ldr;
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
    v4d acc[KNT];
#pragma unroll
    for (int nt = 0; nt < KNT; ++nt) acc[nt] = v4d{0, 0, 0, 0};
    const int64_t ra = r0 + cl;
    const bool rok = ra < nr;
    for (int ks = 0; ks < nks; ++ks) {
      const int k = ks * 4 + kr;
      const bool kok = k < nk;
      const double a = (rok && kok) ? G[ra * nk + k] : 0.0;
#pragma unroll
      for (int nt = 0; nt < KNT; ++nt) {
        const double b = (kok && cok[nt]) ? XE[(int64_t)k * ldr + col[nt]] : 0.0;
        acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[nt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + kr + 4 * r;
      if (row < nr) {
        double *y = Y + (int64_t)d.urow_node[row] * ldr;
#pragma unroll
        for (int nt = 0; nt < KNT; ++nt)
          if (cok[nt]) y[col[nt]] += acc[nt][r];
      }
    }
  }
}

__global__ void __launch_bounds__(64)
k_couple_e(const DevData d, const double *__restrict__ G, const double *__restrict__ X, int ncolr, int64_t ldr,
           int64_t tiles_per_wave, double *__restrict__ part, const int *__restrict__ any) {
  if (any && *any == 0) return;
  const int nk = d.nk;
  const int64_t nr = d.nr;
  const int lane = threadIdx.x, kr = lane >> 4, cl = lane & 15;
  const int n0 = blockIdx.y * KNT * 16, m0 = blockIdx.z * KMT * 16;
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_wave;
  const int64_t t_end = t_begin + tiles_per_wave < ntiles ? t_begin + tiles_per_wave : ntiles;
  int col[KNT];
  bool cok[KNT];
#pragma unroll
  for (int nt = 0; nt < KNT; ++nt) {
    col[nt] = n0 + nt * 16 + cl;
    cok[nt] = col[nt] < ncolr;
  }
  v4d acc[KMT][KNT];
#pragma unroll
  for (int mt = 0; mt < KMT; ++mt)
#pragma unroll
    for (int nt = 0; nt < KNT; ++nt) acc[mt][nt] = v4d{0, 0, 0, 0};
  // A(i, k) = G[r + k][m0 + i], B(k, j) = X[node(r + k)][j]; four k-steps per tile
  for (int64_t r4 = t_begin * 4; r4 < t_end * 4; ++r4) {
    const int64_t rk = r4 * 4 + kr;
    const bool rok = rk < nr;
    const double *xr = X + (rok ? (int64_t)d.urow_node[rk] * ldr : 0);
    double b[KNT];
#pragma unroll
    for (int nt = 0; nt < KNT; ++nt) b[nt] = (rok && cok[nt]) ? xr[col[nt]] : 0.0;
#pragma unroll
    for (int mt = 0; mt < KMT; ++mt) {
      const int m = m0 + mt * 16 + cl;
      const double a = (rok && m < nk) ? G[rk * nk + m] : 0.0;
#pragma unroll
      for (int nt = 0; nt < KNT; ++nt) acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[nt], acc[mt][nt], 0, 0, 0);
    }
  }
  // partial Y_E of this wave: part[blockIdx.x][m][col]
  double *pw = part + (int64_t)blockIdx.x * nk * ncolr;
#pragma unroll
  for (int mt = 0; mt < KMT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + mt * 16 + kr + 4 * r;
      if (m < nk) {
#pragma unroll
        for (int nt = 0; nt < KNT; ++nt)
          if (cok[nt]) pw[(int64_t)m * ncolr + col[nt]] = acc[mt][nt][r];
      }
    }
}

// Y_E[k][c] = sum_b part[b][k][c] + sum_k' Hbar^ee[k][k'] X_E[k'][c]; a block of
// 4 x 64 threads reduces 64 consecutive outputs, each quarter over every
// fourth partial, then combines the quarters in a fixed order.
__global__ void __launch_bounds__(256)
k_couple_final(const DevData d, const double *__restrict__ part, int nblk, const double *__restrict__ Hee,
               const double *__restrict__ X, double *__restrict__ Y, int ncolr, int64_t ldr, const int *__restrict__ any) {
  if (any && *any == 0) return;
  __shared__ double red[4][64];
  const int nk = d.nk, nout = nk * ncolr;
  const int o = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
  double s = 0.0;
  if (o < nout)
    for (int b = q; b < nblk; b += 4) s += part[(int64_t)b * nout + o];
  red[q][threadIdx.x & 63] = s;
  __syncthreads();
  if (q != 0 || o >= nout) return;
  const int lo = threadIdx.x;
  s = red[0][lo] + red[1][lo] + red[2][lo] + red[3][lo];
  const int k = o / ncolr, c = o % ncolr;
  for (int kp = 0; kp < nk; ++kp) s += Hee[k * nk + kp] * X[(d.g.n_nodes + kp) * ldr + c];
  Y[(d.g.n_nodes + k) * ldr + c] = s;
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

template <typename T, int CMT>
void launch_apply_m(const DevData &d, const T *cells, const double *X, double *Y, int ncolr, int64_t ldr,
                    hipStream_t s, const int *any) {
  const unsigned ny = (unsigned)((ncolr + kCellCols - 1) / kCellCols);
  const size_t lds = cell_lds_bytes(d.g.nloc, sizeof(T));
  for (int c = 0; c < 8; ++c) {
    const int cnt = d.colour_off[c + 1] - d.colour_off[c];
    if (cnt == 0) continue;
    const int *list = d.colour_cells + d.colour_off[c];
    hipLaunchKernelGGL((k_cell_apply<T, CMT>), dim3((unsigned)cnt, ny), dim3(kCellWaves * 64), lds, s, d, list,
                       d.colour_off[c], cells, X, Y, ncolr, ldr, any);
  }
}

template <typename T>
void launch_apply(const DevData &d, const T *cells, const double *X, double *Y, int ncolr, int64_t ldr, hipStream_t s,
                  const int *any) {
  const int nmt = (d.g.nloc + 15) / 16;     // M tiles per cell; wave group w >> 1 takes ceil(nmt / 4)
  if (nmt <= 8) launch_apply_m<T, 2>(d, cells, X, Y, ncolr, ldr, s, any);
  else if (nmt <= 16) launch_apply_m<T, 4>(d, cells, X, Y, ncolr, ldr, s, any);
  else launch_apply_m<T, 6>(d, cells, X, Y, ncolr, ldr, s, any);
}

}  // namespace

namespace k {

int cell_apply_init(int nloc) {
  const size_t l64 = cell_lds_bytes(nloc, 8), l32 = cell_lds_bytes(nloc, 4);
  int st = 0;
  st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<double, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l64);
  st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<double, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l64);
  st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<double, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l64);
  st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<float, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l32);
  st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<float, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l32);
  st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<float, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l32);
  return st;
}

void cell_apply(const DevData &d, const void *cells, int dtype, const double *X, double *Y, int ncolr, int64_t ldr,
                hipStream_t s, const int *any) {
  if (dtype == 0) launch_apply<double>(d, (const double *)cells, X, Y, ncolr, ldr, s, any);
  else launch_apply<float>(d, (const float *)cells, X, Y, ncolr, ldr, s, any);
}

void couple_apply(const DevData &d, const double *G, const double *Hee, const double *X, double *Y, int ncolr,
                  int64_t ldr, double *scratch, hipStream_t s, const int *any) {
  if (d.nk == 0) return;
  int nblk = 1;
  const int nout = d.nk * ncolr;
  if (d.nr > 0) {
    const int64_t ntiles = (d.nr + 15) / 16;
    const unsigned ny = (unsigned)((ncolr + KNT * 16 - 1) / (KNT * 16));
    const unsigned nz = (unsigned)((d.nk + KMT * 16 - 1) / (KMT * 16));
    const int64_t tpc = (ntiles + kCoupleCWaves - 1) / kCoupleCWaves;
    hipLaunchKernelGGL(k_couple_c, dim3((unsigned)((ntiles + tpc - 1) / tpc), ny), dim3(64), 0, s, d, G, X, Y, ncolr,
                       ldr, tpc, any);
    const int64_t tpe = (ntiles + kCouplePartials - 1) / kCouplePartials;
    nblk = (int)((ntiles + tpe - 1) / tpe);
    hipLaunchKernelGGL(k_couple_e, dim3((unsigned)nblk, ny, nz), dim3(64), 0, s, d, G, X, ncolr, ldr, tpe, scratch,
                       any);
  } else {
    k::zero(scratch, (int64_t)nout, s);
  }
  hipLaunchKernelGGL(k_couple_final, dim3(nblocks((int64_t)nout, 64)), dim3(256), 0, s, d, scratch, nblk, Hee, X, Y,
                     ncolr, ldr, any);
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
