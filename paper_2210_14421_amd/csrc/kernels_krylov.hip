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
// (no two cells of a colour share a node).  One workgroup (4 waves in a 2 x 2
// grid) per (cell, column chunk); the nloc x nloc block is streamed through LDS
// in K-chunks of 8 rows (Hbar_c is symmetric, so rows k of the row-major block
// are the A-operand columns), the gathered X chunk is staged beside it, and the
// 16x16x4 MFMA accumulates in registers.  Double-buffered LDS, one barrier per
// chunk.
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

// One wave per (cell, pair of 16-row M tiles, chunk of NTW 16-column N tiles).
// No LDS staging of operands and no barriers: each lane loads its MFMA
// operands straight from global memory with a PF-deep register pipeline.
//   A operand (row i, k):  Hbar_c[k][i]  (symmetric block, row-major: 16 lanes
//                          read 16 consecutive doubles)
//   B operand (k, col j):  X[node(k)][col0 + j]  (16 consecutive doubles)
// The waves of one cell get block ids congruent mod 8, so they run on the same
// XCD (blocks are dealt to the 8 XCDs round-robin) and share its L2 copy of the
// cell block and of the gathered rows.
template <typename T, int NTW, int PF>
__global__ void __launch_bounds__(64)
k_cell_apply(const DevData d, const int *__restrict__ cell_list, int slot0, int ncells, int npair, int nch,
             const T *__restrict__ cells, const double *__restrict__ X, double *__restrict__ Y, int ncolr,
             int64_t ldr) {
  typedef typename Mfma<T>::C C;
  typedef typename Mfma<T>::Acc Acc;
  constexpr int MTW = 2;
  __shared__ int64_t rowoff[kApplyMaxLoc];
  const Geom &g = d.g;
  const int nloc = g.nloc;
  const int per_cell = npair * nch;
  const int grp = blockIdx.x / (8 * per_cell), rem = blockIdx.x % (8 * per_cell);
  const int ci = grp * 8 + rem % 8;
  if (ci >= ncells) return;
  const int sub = rem / 8;                  // 0 .. per_cell-1
  const int pair = sub % npair, ch = sub / npair;
  const int64_t cell = cell_list[ci];
  const int lane = threadIdx.x;
  const int kr = lane >> 4, cl = lane & 15;
  int e[3];
  cell_ijk(g, cell, e);
  for (int l = lane; l < nloc; l += 64) rowoff[l] = local_node(g, e, l) * ldr;
  __syncthreads();
  // blocks are stored in colour-major order: a colour launch streams them contiguously
  const T *A = cells + (int64_t)(slot0 + ci) * nloc * nloc;
  const int m0 = pair * MTW * 16;
  const int col0 = ch * NTW * 16;
  const int nks = (nloc + 3) / 4;           // k-steps of 4
  // per-lane fixed parts of the operand addresses
  int arow[MTW];
  bool aok[MTW];
#pragma unroll
  for (int mt = 0; mt < MTW; ++mt) {
    arow[mt] = m0 + mt * 16 + cl;
    aok[mt] = arow[mt] < nloc;
  }
  int bcol[NTW];
  bool bok[NTW];
#pragma unroll
  for (int nt = 0; nt < NTW; ++nt) {
    bcol[nt] = col0 + nt * 16 + cl;
    bok[nt] = bcol[nt] < ncolr;
  }
  C a[PF][MTW], b[PF][NTW];
  auto load = [&](int ks, C (&av)[MTW], C (&bv)[NTW]) {
    const int k = ks * 4 + kr;
    const bool kok = k < nloc;
    const T *Ak = A + (int64_t)k * nloc;
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) av[mt] = (kok && aok[mt]) ? (C)Ak[arow[mt]] : (C)0;
    const double *Xk = X + (kok ? rowoff[k] : 0);
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) bv[nt] = (kok && bok[nt]) ? (C)Xk[bcol[nt]] : (C)0;
  };
  Acc acc[MTW][NTW];
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[i][j] = Acc{0, 0, 0, 0};
  const bool mt1 = m0 + 16 < nloc;          // second M tile of the pair in range
#pragma unroll
  for (int p = 0; p < PF; ++p) load(p, a[p], b[p]);
  for (int ks0 = 0; ks0 < nks; ks0 += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      if (ks0 + p < nks) {
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          acc[0][nt] = Mfma<T>::mma(a[p][0], b[p][nt], acc[0][nt]);
          if (mt1) acc[1][nt] = Mfma<T>::mma(a[p][1], b[p][nt], acc[1][nt]);
        }
      }
      if (ks0 + PF + p < nks) load(ks0 + PF + p, a[p], b[p]);
    }
  }
  // D layout of the 16x16 MFMA (differs between the f64 and f32 forms)
#pragma unroll
  for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + mt * 16 + Mfma<T>::row(kr, r);
        const int col = col0 + nt * 16 + cl;
        if (row < nloc && col < ncolr) Y[rowoff[row] + col] += (double)acc[mt][nt][r];
      }
}

// ---------------------------------------------------------------------------
// Enrichment coupling: Y_C[r] += G[r] X_E ;  Y_E = G^T X_C[R] + Hbar^ee X_E
// ---------------------------------------------------------------------------
// Y_C[rows] += G X_E: a block stages 32 rows of G and all of X_E in LDS; a
// thread owns one row and a group of 4 columns.
constexpr int kRowChunk = 32;
constexpr int kCoupleBlocks = 1024;
__global__ void __launch_bounds__(256)
k_couple_c(const DevData d, const double *__restrict__ G, const double *__restrict__ X, double *__restrict__ Y,
           int ncolr, int64_t ldr) {
  extern __shared__ double sm[];
  const int nk = d.nk;
  double *xe = sm;                       // nk * ncolr
  double *gs = xe + nk * ncolr;          // kRowChunk * nk
  for (int t = threadIdx.x; t < nk * ncolr; t += blockDim.x) {
    int k = t / ncolr, c = t % ncolr;
    xe[t] = X[(d.g.n_nodes + k) * ldr + c];
  }
  const int ng = (ncolr + 3) / 4;
  for (int64_t rc = (int64_t)blockIdx.x * kRowChunk; rc < d.nr; rc += (int64_t)gridDim.x * kRowChunk) {
    const int nrow = (int)(d.nr - rc < kRowChunk ? d.nr - rc : kRowChunk);
    __syncthreads();
    for (int t = threadIdx.x; t < nrow * nk; t += blockDim.x) gs[t] = G[rc * nk + t];
    __syncthreads();
    for (int t = threadIdx.x; t < nrow * ng; t += blockDim.x) {
      const int rr = t / ng, c0 = (t % ng) * 4;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      const double *gr = gs + rr * nk;
      for (int k = 0; k < nk; ++k) {
        const double gv = gr[k];
        const double *xr = xe + k * ncolr + c0;
        a0 += gv * xr[0];
        if (c0 + 1 < ncolr) a1 += gv * xr[1];
        if (c0 + 2 < ncolr) a2 += gv * xr[2];
        if (c0 + 3 < ncolr) a3 += gv * xr[3];
      }
      double *y = Y + d.urow_node[rc + rr] * ldr + c0;
      y[0] += a0;
      if (c0 + 1 < ncolr) y[1] += a1;
      if (c0 + 2 < ncolr) y[2] += a2;
      if (c0 + 3 < ncolr) y[3] += a3;
    }
  }
}

// Split-K partial of Y_E = G^T X_C[R]: part[blk][kappa][col] over the block's
// rows; a thread owns a 4 x 4 tile of (kappa, col) outputs.
template <int S>
__global__ void __launch_bounds__(256)
k_couple_e_partial(const DevData d, const double *__restrict__ G, const double *__restrict__ X, int ncolr,
                   int64_t ldr, int64_t rows_per_blk, double *__restrict__ part) {
  extern __shared__ double sm[];
  const int nk = d.nk;
  double *gs = sm;                       // kRowChunk * nk
  double *xs = gs + kRowChunk * nk;      // kRowChunk * ncolr
  const int nout = nk * ncolr;
  const int tk = (nk + 3) / 4, tc = (ncolr + 3) / 4, ntile = tk * tc;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < d.nr ? r0 + rows_per_blk : d.nr;
  double acc[S][4][4];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[s][a][b] = 0.0;
  for (int64_t rc = r0; rc < r1; rc += kRowChunk) {
    const int nrow = (int)(r1 - rc < kRowChunk ? r1 - rc : kRowChunk);
    __syncthreads();
    for (int t = threadIdx.x; t < kRowChunk * nk; t += blockDim.x) gs[t] = t < nrow * nk ? G[rc * nk + t] : 0.0;
    for (int t = threadIdx.x; t < kRowChunk * ncolr; t += blockDim.x) {
      int rr = t / ncolr, c = t % ncolr;
      xs[t] = rr < nrow ? X[d.urow_node[rc + rr] * ldr + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int tile = threadIdx.x + s * 256;
      if (tile < ntile) {
        const int k0 = (tile / tc) * 4, c0 = (tile % tc) * 4;
        for (int rr = 0; rr < nrow; ++rr) {
          double gv[4], xv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) gv[a] = k0 + a < nk ? gs[rr * nk + k0 + a] : 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) xv[b] = c0 + b < ncolr ? xs[rr * ncolr + c0 + b] : 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[s][a][b] += gv[a] * xv[b];
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int tile = threadIdx.x + s * 256;
    if (tile < ntile) {
      const int k0 = (tile / tc) * 4, c0 = (tile % tc) * 4;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (k0 + a < nk && c0 + b < ncolr) part[(int64_t)blockIdx.x * nout + (k0 + a) * ncolr + c0 + b] = acc[s][a][b];
    }
  }
}

__global__ void k_couple_e_final(const DevData d, const double *__restrict__ part, int nblk,
                                 const double *__restrict__ Hee, const double *__restrict__ X, double *__restrict__ Y,
                                 int ncolr, int64_t ldr) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int nk = d.nk, nout = nk * ncolr;
  if (o >= nout) return;
  const int k = o / ncolr, c = o % ncolr;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * nout + o];
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

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, int NTW>
void launch_apply_n(const DevData &d, const T *cells, const double *X, double *Y, int ncolr, int64_t ldr, hipStream_t s) {
  constexpr int PF = 4;
  const int npair = ((d.g.nloc + 15) / 16 + 1) / 2;
  const int nch = (ncolr + NTW * 16 - 1) / (NTW * 16);
  for (int c = 0; c < 8; ++c) {
    int cnt = d.colour_off[c + 1] - d.colour_off[c];
    if (cnt == 0) continue;
    const int *list = d.colour_cells + d.colour_off[c];
    const unsigned nx = (unsigned)(((cnt + 7) / 8) * 8) * npair * nch;
    hipLaunchKernelGGL((k_cell_apply<T, NTW, PF>), dim3(nx), dim3(64), 0, s, d, list, d.colour_off[c], cnt, npair, nch,
                       cells, X, Y, ncolr, ldr);
  }
}

template <typename T>
void launch_apply(const DevData &d, const T *cells, const double *X, double *Y, int ncolr, int64_t ldr, hipStream_t s) {
  if (ncolr <= 16) launch_apply_n<T, 1>(d, cells, X, Y, ncolr, ldr, s);
  else if (ncolr <= 32) launch_apply_n<T, 2>(d, cells, X, Y, ncolr, ldr, s);
  else launch_apply_n<T, 3>(d, cells, X, Y, ncolr, ldr, s);
}

}  // namespace

namespace k {

void cell_apply(const DevData &d, const void *cells, int dtype, const double *X, double *Y, int ncolr, int64_t ldr,
                hipStream_t s) {
  if (dtype == 0) launch_apply<double>(d, (const double *)cells, X, Y, ncolr, ldr, s);
  else launch_apply<float>(d, (const float *)cells, X, Y, ncolr, ldr, s);
}

void couple_apply(const DevData &d, const double *G, const double *Hee, const double *X, double *Y, int ncolr,
                  int64_t ldr, double *scratch, hipStream_t s) {
  if (d.nk == 0) return;
  int nblk = 1;
  const int nout = d.nk * ncolr;
  if (d.nr > 0) {
    size_t lds = ((size_t)d.nk * ncolr + (size_t)kRowChunk * d.nk) * sizeof(double);
    unsigned nb = (unsigned)std::min<int64_t>(kCoupleBlocks, (d.nr + kRowChunk - 1) / kRowChunk);
    hipLaunchKernelGGL(k_couple_c, dim3(nb), dim3(256), lds, s, d, G, X, Y, ncolr, ldr);
    nblk = (int)std::min<int64_t>(kCoupleBlocks, (d.nr + 127) / 128);
    int64_t rpb = (d.nr + nblk - 1) / nblk;
    size_t lds2 = (size_t)kRowChunk * (d.nk + ncolr) * sizeof(double);
    const int ntile = ((d.nk + 3) / 4) * ((ncolr + 3) / 4);
    const int S = (ntile + 255) / 256;
    if (S <= 1)
      hipLaunchKernelGGL(k_couple_e_partial<1>, dim3(nblk), dim3(256), lds2, s, d, G, X, ncolr, ldr, rpb, scratch);
    else if (S <= 2)
      hipLaunchKernelGGL(k_couple_e_partial<2>, dim3(nblk), dim3(256), lds2, s, d, G, X, ncolr, ldr, rpb, scratch);
    else
      hipLaunchKernelGGL(k_couple_e_partial<4>, dim3(nblk), dim3(256), lds2, s, d, G, X, ncolr, ldr, rpb, scratch);
  } else {
    k::zero(scratch, (int64_t)nout, s);
  }
  hipLaunchKernelGGL(k_couple_e_final, dim3(nblocks((int64_t)nout, 128)), dim3(128), 0, s, d, scratch, nblk, Hee, X, Y,
                     ncolr, ldr);
}

void tridiag_exp(const double *alpha, const double *beta, int j, int ncol, int kmax, double tau, const double *beta0,
                 const int *kforce, double tol, int *active, int *kused, double *err, double *u, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_exp, dim3(ncol), dim3(64), 0, s, alpha, beta, j, ncol, kmax, tau, beta0, kforce, tol,
                     active, kused, err, u);
}

}  // namespace k
}  // namespace efe
