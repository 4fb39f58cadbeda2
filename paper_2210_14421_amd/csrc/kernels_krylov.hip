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
// Lanczos vector kernels.  Blocks are n_rows x ncol complex, packed (ld = ncol).
// ---------------------------------------------------------------------------
constexpr int LCH = 8;       // LDS reduction chunk (vectors)
constexpr int kDotBlocks = k::kDotBlocksMax;

// Reduce per-thread accumulators acc[l][2] (l < nv) of the R row groups of a
// block into part[blockIdx.x][l][c][2].  red: LDS of R * LCH * ncol * 2 doubles.
template <int NV>
__device__ __forceinline__ void block_reduce_cols(const double (&acc)[NV][2], int nv, int R, int r0, int c, int ncol,
                                                  double *red, double *__restrict__ part) {
  for (int l0 = 0; l0 < nv; l0 += LCH) {
    __syncthreads();
    if (r0 < R) {
#pragma unroll
      for (int l = 0; l < LCH; ++l) {
        int ll = l0 + l;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k)
          if (k == ll) { re = acc[k][0]; im = acc[k][1]; }
        red[((r0 * LCH + l) * ncol + c) * 2] = re;
        red[((r0 * LCH + l) * ncol + c) * 2 + 1] = im;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < LCH * ncol * 2; t += blockDim.x) {
      int l = t / (ncol * 2);
      if (l0 + l >= nv) continue;
      double sum = 0.0;
      for (int rr = 0; rr < R; ++rr) sum += red[rr * LCH * ncol * 2 + t];
      part[((int64_t)blockIdx.x * nv + l0) * ncol * 2 + t] = sum;
    }
  }
}

// part[blk][l][c] = sum_r conj(Q_l[r][c]) w[r][c] for l < nq (one pass over the
// rows, nq <= NL); with_norm adds entry nq = ||w||^2 per column.
template <int NL>
__global__ void __launch_bounds__(256)
k_dots(const double *__restrict__ Q, int64_t qstride, int nq, const double *__restrict__ w, int64_t nrows, int ncol,
       const int *__restrict__ active, int with_norm, const int *__restrict__ any, double *__restrict__ part) {
  if (any && *any == 0) return;
  extern __shared__ double red[];
  const int R = blockDim.x / ncol;
  const int c = threadIdx.x % ncol, r0 = threadIdx.x / ncol;
  const bool on = r0 < R && (active == nullptr || active[c] != 0);
  double acc[NL + 1][2];
#pragma unroll
  for (int l = 0; l <= NL; ++l) acc[l][0] = acc[l][1] = 0.0;
  if (on) {
    for (int64_t r = (int64_t)blockIdx.x * R + r0; r < nrows; r += (int64_t)gridDim.x * R) {
      const int64_t o = (r * ncol + c) * 2;
      const double wr = w[o], wi = w[o + 1];
#pragma unroll
      for (int l = 0; l < NL; ++l)
        if (l < nq) {
          const double *q = Q + (int64_t)l * qstride + o;
          const double qr = q[0], qi = q[1];
          acc[l][0] += qr * wr + qi * wi;
          acc[l][1] += qr * wi - qi * wr;
        }
      acc[NL][0] += wr * wr + wi * wi;
    }
  }
  if (with_norm) {
    // move the norm to slot nq
#pragma unroll
    for (int l = 0; l < NL; ++l)
      if (l == nq) { acc[l][0] = acc[NL][0]; acc[l][1] = 0.0; }
  }
  block_reduce_cols<NL + 1>(acc, nq + (with_norm ? 1 : 0), R, r0, c, ncol, red, part);
}

// Classical Gram-Schmidt update w -= sum_{l<nq} h[l][c] Q_l for the columns
// with need[c] != 0, and the partial ||w||^2 of the updated vector.  If *any
// is 0 the kernel returns at once.
template <int NL>
__global__ void __launch_bounds__(256)
k_update_norm(const double *__restrict__ Q, int64_t qstride, int nq, const double *__restrict__ h,
              double *__restrict__ w, int64_t nrows, int ncol, const int *__restrict__ need,
              const int *__restrict__ any, double *__restrict__ part) {
  if (*any == 0) return;
  extern __shared__ double sm[];
  const int R = blockDim.x / ncol;
  double *hs = sm;
  double *red = sm + NL * ncol * 2;
  for (int t = threadIdx.x; t < nq * ncol * 2; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  const int c = threadIdx.x % ncol, r0 = threadIdx.x / ncol;
  const bool on = r0 < R && need[c] != 0;
  double acc[1][2] = {{0.0, 0.0}};
  if (on) {
    for (int64_t r = (int64_t)blockIdx.x * R + r0; r < nrows; r += (int64_t)gridDim.x * R) {
      const int64_t o = (r * ncol + c) * 2;
      double wr = w[o], wi = w[o + 1];
#pragma unroll
      for (int l = 0; l < NL; ++l)
        if (l < nq) {
          const double *q = Q + (int64_t)l * qstride + o;
          const double qr = q[0], qi = q[1];
          const double hr = hs[(l * ncol + c) * 2], hi = hs[(l * ncol + c) * 2 + 1];
          wr -= hr * qr - hi * qi;
          wi -= hr * qi + hi * qr;
        }
      w[o] = wr;
      w[o + 1] = wi;
      acc[0][0] += wr * wr + wi * wi;
    }
  }
  block_reduce_cols<1>(acc, 1, R, r0, c, ncol, red, part);
}

// Daniel-Gragg-Kaufman-Stewart test after the first Gram-Schmidt pass: the
// pass lost at most eps ||w|| / ||w'|| of orthogonality, so a second pass is
// made only for columns with ||w'|| < kReorthEta ||w|| (heavy cancellation).
// Sets alpha_j = Re h1_{j-1}, the first-pass norm, need[c] and any.
constexpr double kReorthEta = 1e-3;
__global__ void k_cgs_decide(const double *__restrict__ h1n, const double *__restrict__ nrm1_part, int j, int ncol,
                             const int *__restrict__ active, double *__restrict__ alpha_j, double *__restrict__ nrm1,
                             int *__restrict__ need, int *__restrict__ any) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    int nd = 0;
    if (active[c]) {
      alpha_j[c] = h1n[((j - 1) * ncol + c) * 2];
      const double w2 = h1n[(j * ncol + c) * 2];     // ||w||^2 before the pass
      const double n2 = nrm1_part[2 * c];             // ||w'||^2 after it
      nrm1[c] = n2;
      nd = n2 < kReorthEta * kReorthEta * w2 ? 1 : 0;
    }
    need[c] = nd;
    if (nd) atomicOr(&flag, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *any = flag;
}

__global__ void k_cgs_beta(const double *__restrict__ nrm1, const double *__restrict__ nrm2, const int *__restrict__ need,
                           const int *__restrict__ active, int ncol, double *__restrict__ beta_j) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol || !active[c]) return;
  const double v = need[c] ? nrm2[2 * c] : nrm1[c];
  beta_j[c] = sqrt(v > 0.0 ? v : 0.0);
}

// w[r][c] -= sum_l h[l][c] Q_l[r][c]   (complex), active columns only
__global__ void __launch_bounds__(256)
k_multi_update(const double *__restrict__ Q, int64_t qstride, int nq, const double *__restrict__ h,
               double *__restrict__ w, int64_t nrows, int ncol, const int *__restrict__ active) {
  extern __shared__ double hs[];     // nq * ncol * 2
  for (int t = threadIdx.x; t < nq * ncol * 2; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncol) return;
  const int c = (int)(t % ncol);
  if (active && !active[c]) return;
  double wr = w[2 * t], wi = w[2 * t + 1];
  for (int l = 0; l < nq; ++l) {
    const double qr = Q[(int64_t)l * qstride + 2 * t], qi = Q[(int64_t)l * qstride + 2 * t + 1];
    const double hr = hs[(l * ncol + c) * 2], hi = hs[(l * ncol + c) * 2 + 1];
    wr -= hr * qr - hi * qi;
    wi -= hr * qi + hi * qr;
  }
  w[2 * t] = wr;
  w[2 * t + 1] = wi;
}

// w -= alpha q + beta qm1 (real coefficients per column)
__global__ void k_three_term(double *__restrict__ w, const double *__restrict__ q, const double *__restrict__ qm1,
                             const double *__restrict__ alpha, const double *__restrict__ beta, int64_t nrows,
                             int ncol, const int *__restrict__ active) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncol) return;
  const int c = (int)(t % ncol);
  if (!active[c]) return;
  const double a = alpha[c];
  double wr = w[2 * t] - a * q[2 * t], wi = w[2 * t + 1] - a * q[2 * t + 1];
  if (qm1) {
    const double b = beta[c];
    wr -= b * qm1[2 * t];
    wi -= b * qm1[2 * t + 1];
  }
  w[2 * t] = wr;
  w[2 * t + 1] = wi;
}

// q = w * inv[c]
__global__ void k_scale_cols(const double *__restrict__ w, double *__restrict__ q, const double *__restrict__ nrm,
                             int64_t nrows, int ncol, const int *__restrict__ active) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncol) return;
  const int c = (int)(t % ncol);
  if (active && !active[c]) return;
  const double s = nrm[c] > 0.0 ? 1.0 / nrm[c] : 0.0;
  q[2 * t] = w[2 * t] * s;
  q[2 * t + 1] = w[2 * t + 1] * s;
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

// out[r][c] = beta0[c] sum_{l < k_c} u[c][l] Q_l[r][c]
__global__ void __launch_bounds__(256)
k_combine(const double *__restrict__ Q, int64_t qstride, const double *__restrict__ u, int kmax,
          const int *__restrict__ kused, const double *__restrict__ beta0, double *__restrict__ out, int64_t nrows,
          int ncol) {
  extern __shared__ double us[];   // ncol * kmax * 2
  for (int t = threadIdx.x; t < ncol * kmax * 2; t += blockDim.x) us[t] = u[t];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncol) return;
  const int c = (int)(t % ncol);
  const int kc = kused[c];
  double sr = 0.0, si = 0.0;
  for (int l = 0; l < kc; ++l) {
    const double qr = Q[(int64_t)l * qstride + 2 * t], qi = Q[(int64_t)l * qstride + 2 * t + 1];
    const double ur = us[(c * kmax + l) * 2], ui = us[(c * kmax + l) * 2 + 1];
    sr += ur * qr - ui * qi;
    si += ur * qi + ui * qr;
  }
  const double b = beta0[c];
  out[2 * t] = b * sr;
  out[2 * t + 1] = b * si;
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

template <int NL>
static int launch_dots(const double *Q, int64_t qstride, int nq, const double *w, int64_t nrows, int ncol,
                       const int *active, int with_norm, const int *any, double *part, hipStream_t s) {
  int R = 256 / ncol;
  int nb = (int)std::min<int64_t>(kDotBlocks, (nrows + R - 1) / R);
  if (nb < 1) nb = 1;
  size_t lds = (size_t)R * LCH * ncol * 2 * sizeof(double);
  hipLaunchKernelGGL(k_dots<NL>, dim3(nb), dim3(256), lds, s, Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part);
  return nb;
}

int dots_partials(const double *Q, int64_t qstride, int nq, const double *w, int64_t nrows, int ncol,
                  const int *active, int with_norm, const int *any, double *part, hipStream_t s) {
  if (nq <= 1) return launch_dots<1>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
  if (nq <= 8) return launch_dots<8>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
  if (nq <= 16) return launch_dots<16>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
  if (nq <= 24) return launch_dots<24>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
  if (nq <= 32) return launch_dots<32>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
  if (nq <= 48) return launch_dots<48>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
  return launch_dots<64>(Q, qstride, nq, w, nrows, ncol, active, with_norm, any, part, s);
}

int multidot_partials(const double *Q, int64_t qstride, int nq, const double *w, int64_t nrows, int ncol,
                      const int *active, double *part, hipStream_t s) {
  return dots_partials(Q, qstride, nq, w, nrows, ncol, active, 0, nullptr, part, s);
}

int norm_partials(const double *w, int64_t nrows, int ncol, const int *active, double *part, hipStream_t s) {
  return launch_dots<1>(w, 0, 0, w, nrows, ncol, active, 1, nullptr, part, s);
}

template <int NL>
static int launch_update_norm(const double *Q, int64_t qstride, int nq, const double *h, double *w, int64_t nrows,
                              int ncol, const int *need, const int *any, double *part, hipStream_t s) {
  int R = 256 / ncol;
  int nb = (int)std::min<int64_t>(kDotBlocks, (nrows + R - 1) / R);
  if (nb < 1) nb = 1;
  size_t lds = ((size_t)NL * ncol * 2 + (size_t)R * LCH * ncol * 2) * sizeof(double);
  hipLaunchKernelGGL(k_update_norm<NL>, dim3(nb), dim3(256), lds, s, Q, qstride, nq, h, w, nrows, ncol, need, any, part);
  return nb;
}

int update_norm_partials(const double *Q, int64_t qstride, int nq, const double *h, double *w, int64_t nrows, int ncol,
                         const int *need, const int *any, double *part, hipStream_t s) {
  if (nq <= 8) return launch_update_norm<8>(Q, qstride, nq, h, w, nrows, ncol, need, any, part, s);
  if (nq <= 16) return launch_update_norm<16>(Q, qstride, nq, h, w, nrows, ncol, need, any, part, s);
  if (nq <= 32) return launch_update_norm<32>(Q, qstride, nq, h, w, nrows, ncol, need, any, part, s);
  return launch_update_norm<64>(Q, qstride, nq, h, w, nrows, ncol, need, any, part, s);
}

void cgs_decide(const double *h1n, const double *nrm1_sum, int j, int ncol, const int *active, double *alpha_j,
                double *nrm1, int *need, int *any, hipStream_t s) {
  hipLaunchKernelGGL(k_cgs_decide, dim3(1), dim3(128), 0, s, h1n, nrm1_sum, j, ncol, active, alpha_j, nrm1, need, any);
}

void cgs_beta(const double *nrm1, const double *nrm2, const int *need, const int *active, int ncol, double *beta_j,
              hipStream_t s) {
  hipLaunchKernelGGL(k_cgs_beta, dim3((ncol + 63) / 64), dim3(64), 0, s, nrm1, nrm2, need, active, ncol, beta_j);
}

void multi_update(const double *Q, int64_t qstride, int nq, const double *h, double *w, int64_t nrows, int ncol,
                  const int *active, hipStream_t s) {
  size_t lds = (size_t)nq * ncol * 2 * sizeof(double);
  hipLaunchKernelGGL(k_multi_update, dim3(nblocks(nrows * ncol, 256)), dim3(256), lds, s, Q, qstride, nq, h, w, nrows,
                     ncol, active);
}

void three_term(double *w, const double *q, const double *qm1, const double *alpha, const double *beta, int64_t nrows,
                int ncol, const int *active, hipStream_t s) {
  hipLaunchKernelGGL(k_three_term, dim3(nblocks(nrows * ncol, 256)), dim3(256), 0, s, w, q, qm1, alpha, beta, nrows,
                     ncol, active);
}

void scale_cols(const double *w, double *q, const double *nrm, int64_t nrows, int ncol, const int *active,
                hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cols, dim3(nblocks(nrows * ncol, 256)), dim3(256), 0, s, w, q, nrm, nrows, ncol, active);
}

void tridiag_exp(const double *alpha, const double *beta, int j, int ncol, int kmax, double tau, const double *beta0,
                 const int *kforce, double tol, int *active, int *kused, double *err, double *u, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_exp, dim3(ncol), dim3(64), 0, s, alpha, beta, j, ncol, kmax, tau, beta0, kforce, tol,
                     active, kused, err, u);
}

void combine(const double *Q, int64_t qstride, const double *u, int kmax, const int *kused, const double *beta0,
             double *out, int64_t nrows, int ncol, hipStream_t s) {
  size_t lds = (size_t)ncol * kmax * 2 * sizeof(double);
  hipLaunchKernelGGL(k_combine, dim3(nblocks(nrows * ncol, 256)), dim3(256), lds, s, Q, qstride, u, kmax, kused, beta0,
                     out, nrows, ncol);
}

}  // namespace k
}  // namespace efe

namespace efe {
namespace {

// dst[c] = Re(tmp[c]) or sqrt(max(Re(tmp[c]), 0)) for active columns
__global__ void k_store_re(const double *__restrict__ tmp, double *__restrict__ dst, int ncol, int sqrt_mode,
                           const int *__restrict__ active) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  if (active && !active[c]) return;
  const double v = tmp[2 * c];
  dst[c] = sqrt_mode ? sqrt(v > 0.0 ? v : 0.0) : v;
}

__global__ void k_init_active(const double *__restrict__ beta0, int *__restrict__ active, int *__restrict__ kused,
                              int ncol) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  active[c] = beta0[c] > 0.0 ? 1 : 0;
  kused[c] = 0;
}

}  // namespace

namespace k {

void store_re(const double *tmp, double *dst, int ncol, int sqrt_mode, const int *active, hipStream_t s) {
  hipLaunchKernelGGL(k_store_re, dim3((ncol + 63) / 64), dim3(64), 0, s, tmp, dst, ncol, sqrt_mode, active);
}

void init_active(const double *beta0, int *active, int *kused, int ncol, hipStream_t s) {
  hipLaunchKernelGGL(k_init_active, dim3((ncol + 63) / 64), dim3(64), 0, s, beta0, active, kused, ncol);
}

}  // namespace k
}  // namespace efe
