// Cell part of Hbar X (Sec. 2.3, eq. (TDKSDiscrete2)): Y = sum_c P_c^T Hbar_c P_c X
// with the dense symmetric cell blocks Hbar_c = D_c^-1/2 (K_c / 2 + V_c) D_c^-1/2, on the
// 16x16x4 MFMA (FP64, or FP32 blocks with FP32 accumulation); BF16 products are in
// kernels_cell_bf16.hip.  The orbital rows X and Y are FP64, or, for the FP32 blocks,
// also FP32 (the reduced-precision product reads an FP32 copy of X and leaves its
// FP32-accurate result in FP32: half the gathered and scattered bytes).
#include <hip/hip_runtime.h>

#include <cstdio>

#include "common.h"

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
template <typename T, typename C> __device__ __forceinline__ C widen(T v) { return (C)v; }

template <> struct Mfma<float> {
  typedef float C;
  typedef v4f Acc;
  static __device__ __forceinline__ Acc mma(C a, C b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // output register r of a lane holds row 4 (lane/16) + r, column lane%16
  static __device__ __forceinline__ int row(int kr, int r) { return 4 * kr + r; }
};

// One workgroup of 8 waves per (cell, chunk of 96 columns).  Operands pass
// through LDS in chunks of KC k-rows, NS chunks in flight (the defaults, 8 and 3,
// let two workgroups share a CU; the other (NS, KC) pairs are the autotuner's
// candidates, and all of them add the k terms in the same order, so every
// variant gives the same bits): the chunk's rows of the symmetric cell block (contiguous in memory)
// and the gathered rows of X are copied global -> LDS by the direct-to-LDS
// loads (global_load_lds_dwordx4, 16 B per lane at LDS base + 16 * lane), so
// no registers hold data in flight.  Every wave issues the same number of
// copies per chunk (padding copies land in a scratch line), which lets a
// fixed vmcnt wait certify that the chunk has arrived before the barrier.
// Wave w takes the M tiles (w >> 1) + 4 i and the three 16-column N tiles of
// half (w & 1): every SIMD then carries the same number of tiles.
constexpr int kCellWaves = 8;
constexpr int kCellNT = 3;                  // N tiles per wave (default: 96 columns per workgroup)
// LDS row stride of X in elements: the 4 rows of a B read hit disjoint banks
// (FP64 rows: 112 doubles; FP32 rows: 144 floats, 16 banks apart)
template <typename IO> constexpr int x_ldx() { return sizeof(IO) == 8 ? 112 : 144; }
template <int KC, typename IO> constexpr int x_stage() { return KC * x_ldx<IO>() * (int)sizeof(IO); }

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
// the same, non-temporal (the cell blocks, read once per product: they leave the caches
// to the gathered X rows, which the epilogue reads again)
__device__ __forceinline__ void copy16_to_lds_nt(const void *src, void *lds_base) {
  __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)lds_base, 16, 0, 2);
}

template <typename T, int KC, int NW>
struct CellChunk {
  // A-chunk copies per wave per chunk, sized for the largest cell (nloc <= 384)
  static constexpr int kAIns = (KC * kApplyMaxLoc * (int)sizeof(T) + 1024 * NW - 1) / (1024 * NW);
  static constexpr int kXIns = (KC + NW - 1) / NW;   // X-row copies per wave per chunk
  static constexpr int kPer = kAIns + kXIns;         // copies per wave per chunk
};

inline size_t cell_lds_bytes(int nloc, size_t esz, int ns, int kc, size_t xsz = 8) {
  const size_t aseg = ((size_t)kc * nloc * esz + 1023) / 1024;
  const size_t xrow = xsz == 8 ? (size_t)x_ldx<double>() * 8 : (size_t)x_ldx<float>() * 4;
  return (size_t)ns * (aseg * 1024 + (size_t)kc * xrow) + 1024;
}

// IO: element type of X and Y (double, or float for FP32 blocks); ldr counts IO elements.
// NT: 16-column N tiles per wave, 32 NT columns per workgroup (narrow tiles for blocks of
// few orbitals, whose columns would otherwise be mostly padding).
template <typename T, typename IO, int CMT, int NS, int KC, int WPE, int NT = kCellNT, int NW = kCellWaves>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE)))
k_cell_apply(const DevData d, const int *__restrict__ cell_list, int slot0, const T *__restrict__ cells,
             const IO *__restrict__ X, IO *__restrict__ Y, int ncolr, int64_t ldr, const int *__restrict__ any,
             double *__restrict__ apart, int64_t apld) {
  static_assert(KC % 4 == 0 && NS >= 2, "chunks of whole k-steps, at least one in flight");
  static_assert(sizeof(IO) >= sizeof(T), "X and Y at least as wide as the blocks");
  if (any && *any == 0) return;
  typedef typename Mfma<T>::C C;
  typedef typename Mfma<T>::Acc Acc;
  constexpr int kAIns = CellChunk<T, KC, NW>::kAIns, kXIns = CellChunk<T, KC, NW>::kXIns;
  constexpr int kPer = CellChunk<T, KC, NW>::kPer;
  constexpr int kMG = NW / 2;   // M-tile groups: wave w takes the tiles w / 2 + kMG i
  constexpr int kXStage = x_stage<KC, IO>();
  constexpr int kLDX = x_ldx<IO>();
  constexpr int kEPL = 16 / (int)sizeof(IO);   // elements of an X row per 16-byte copy
  __shared__ int64_t rowoff[kApplyMaxLoc];
  // bit 0: this cell's colour is the first to reach the node; bit 1: the last
  __shared__ unsigned char reach[kApplyMaxLoc];
  extern __shared__ __attribute__((aligned(16))) unsigned char cell_sm[];
  const Geom &g = d.g;
  const int nloc = g.nloc;
  const int abytes = KC * nloc * (int)sizeof(T);
  const int aseg = (abytes + 1023) / 1024;
  unsigned char *As = cell_sm;                                   // NS * aseg KB
  unsigned char *Xs = cell_sm + NS * aseg * 1024;                // NS * kXStage
  unsigned char *junk = Xs + NS * kXStage;                       // 1 KB target of padding copies
  const int ci = blockIdx.x;
  constexpr int kCols = 2 * NT * 16;
  const int col0 = blockIdx.y * kCols;
  const int wcol = ncolr - col0 < kCols ? ncolr - col0 : kCols;   // columns of this chunk (even)
  const int64_t cell = cell_list[ci];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kr = lane >> 4, cl = lane & 15;
  const int mg = wave >> 1, nh = wave & 1;
  int e[3];
  cell_ijk(g, cell, e);
  for (int l = tid; l < nloc; l += NW * 64) {
    rowoff[l] = local_node(g, e, l) * ldr;
    // colours run in the order (e_x & 1) + 2 (e_y & 1) + 4 (e_z & 1); a node on a
    // face shared along some axis is reached first by the even cell of that axis and
    // last by the odd one
    const int li[3] = {l % g.P, (l / g.P) % g.P, l / (g.P * g.P)};
    bool later = false, earlier = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const bool shared = (li[ax] == 0 && e[ax] > 0) || (li[ax] == g.p && e[ax] < g.nc[ax] - 1);
      later |= shared && (e[ax] & 1);
      earlier |= shared && !(e[ax] & 1);
    }
    reach[l] = (later ? 0 : 1) | (earlier ? 0 : 2);
  }
  // X stages start zeroed: pad columns are never copied into
  for (int i = tid; i < NS * kXStage / 8; i += NW * 64) ((double *)Xs)[i] = 0.0;
  __syncthreads();
  const unsigned char *Ag = (const unsigned char *)(cells + (int64_t)(slot0 + ci) * g.cstride);   // 16-byte aligned
  const int64_t ablock = g.cstride * (int64_t)sizeof(T);   // padded block: copies never cross into the next one
  const int nchunk = (nloc + KC - 1) / KC;
  auto issue = [&](int kc) {
    const int st = kc % NS;
    const int64_t abase = (int64_t)kc * abytes;
#pragma unroll
    for (int i = 0; i < kAIns; ++i) {
      const int seg = wave + NW * i;
      const int64_t off = abase + (int64_t)seg * 1024 + lane * 16;
      const bool ok = seg < aseg && off + 16 <= ablock;
      copy16_to_lds_nt(Ag + (ok ? off : 0), seg < aseg ? As + (st * aseg + seg) * 1024 : junk);
    }
#pragma unroll
    for (int i = 0; i < kXIns; ++i) {
      const int r = wave + NW * i;
      const int k = kc * KC + r;
      if (r < KC && k < nloc) {
        if (kEPL * lane < wcol)
          copy16_to_lds(X + rowoff[k] + col0 + kEPL * lane, Xs + st * kXStage + r * kLDX * (int)sizeof(IO));
      } else {
        copy16_to_lds(X, junk);
      }
    }
  };
  const int nmt = (nloc + 15) / 16;
  Acc acc[CMT][NT];
#pragma unroll
  for (int i = 0; i < CMT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = Acc{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < NS - 1; ++c)
    if (c < nchunk) issue(c);
  for (int kc = 0; kc < nchunk; ++kc) {
    // this wave's copies of chunk kc are done once at most (chunks issued after it) * kPer remain
    if (kc + NS - 2 < nchunk) wait_vmcnt<kPer * (NS - 2)>();
    else wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (kc + NS - 1 < nchunk) issue(kc + NS - 1);
    const int st = kc % NS;
    const T *Al = (const T *)(As + st * aseg * 1024);
    const IO *Xl = (const IO *)(Xs + st * kXStage);
    // per k-step: the step's operands first (one LDS wait), then its MFMAs.  Rows m past
    // nloc read neighbouring LDS words: they only reach output rows that are never stored.
    // k-rows past nloc (last chunk) are zeroed, as their X rows are not copied.
#pragma unroll
    for (int s4 = 0; s4 < KC / 4; ++s4) {
      const int kl = s4 * 4 + kr;
      const bool kok = kc * KC + kl < nloc;
      C b[NT], a[CMT];
#pragma unroll
      for (int j = 0; j < NT; ++j) b[j] = (C)Xl[kl * kLDX + (nh * NT + j) * 16 + cl];
#pragma unroll
      for (int i = 0; i < CMT; ++i) {
        const int t = min(mg + kMG * i, nmt - 1);
        const C v = widen<T, C>(Al[kl * nloc + t * 16 + cl]);
        a[i] = kok ? v : (C)0;
      }
#pragma unroll
      for (int i = 0; i < CMT; ++i)
        if (mg + kMG * i < nmt) {
#pragma unroll
          for (int j = 0; j < NT; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
        }
    }
  }
  // D layout of the 16x16 MFMA (differs between the f64 and f32 forms).  Per tile, every
  // earlier value of Y is loaded before any store, so that the loads of the rows a
  // previous colour reached are in flight together.
  // (FP64 accumulators leave room for half a tile's values at a time.)
  // With apart (FP64 blocks and rows only) the workgroup also leaves, per column, the
  // sum of X Y over the nodes this cell's colour reaches last, with Y the sum of all
  // cell products there (the value stored): the cell's share of the cell part of the
  // Lanczos coefficient x^H Hbar x (Sec. 2.6), at apart[(col * apld + cell slot) * 4 + wave
  // group] (one partial per wave of a column half); each node's X is read once per Hbar X.
  // The X values of a wave's first half tile are loaded after its stores, into the
  // registers of the earlier Y values; those of the later halves, whose accumulators the
  // first half's products have freed, together with the earlier Y values, in the same
  // round trip.
  constexpr bool kAlpha = sizeof(T) == 8 && sizeof(IO) == 8;
  const bool wa = kAlpha && apart != nullptr;
  constexpr int kRB = sizeof(C) == 8 ? 2 : 4;
  C pa[NT];   // this lane's running sums per column, over its half tiles in order
#pragma unroll
  for (int j = 0; j < NT; ++j) pa[j] = (C)0;
  if constexpr (kAlpha) static_assert(kMG == k::kAlphaParts, "one partial per wave of a column half");
#pragma unroll
  for (int i = 0; i < CMT; ++i) {
    if (mg + kMG * i >= nmt) continue;
#pragma unroll
    for (int r0 = 0; r0 < 4; r0 += kRB) {
      IO old[kRB][NT], xo[kRB][NT];
      // X at the rows this colour reaches last (zero elsewhere)
      auto load_x = [&]() {
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
          const int row = (mg + kMG * i) * 16 + Mfma<T>::row(kr, r0 + r);
          const bool use = row < nloc && (reach[row] & 2);
          const IO *xr = X + (row < nloc ? rowoff[row] : 0);
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int col = col0 + (nh * NT + j) * 16 + cl;
            xo[r][j] = (use && col < ncolr) ? xr[col] : (IO)0;
          }
        }
      };
      if constexpr (kAlpha) {
        if ((i > 0 || r0 > 0) && wa) load_x();
      }
#pragma unroll
      for (int r = 0; r < kRB; ++r) {
        const int row = (mg + kMG * i) * 16 + Mfma<T>::row(kr, r0 + r);
        const bool add = row < nloc && !(reach[row] & 1);
        const IO *yr = Y + (row < nloc ? rowoff[row] : 0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int col = col0 + (nh * NT + j) * 16 + cl;
          old[r][j] = (add && col < ncolr) ? yr[col] : (IO)0;
        }
      }
#pragma unroll
      for (int r = 0; r < kRB; ++r) {
        const int row = (mg + kMG * i) * 16 + Mfma<T>::row(kr, r0 + r);
        if (row >= nloc) continue;
        IO *yr = Y + rowoff[row];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int col = col0 + (nh * NT + j) * 16 + cl;
          const IO yv = old[r][j] + (IO)acc[i][j][r0 + r];
          if (col < ncolr) yr[col] = yv;
          if constexpr (kAlpha) acc[i][j][r0 + r] = (C)yv;   // the stored value, for the products below
        }
      }
      if constexpr (kAlpha) {
        if (wa) {
          if (i == 0 && r0 == 0) load_x();
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            C t = (C)0;
#pragma unroll
            for (int r = 0; r < kRB; ++r) {
              // rows past nloc hold products of unused LDS words: left out, not multiplied
              const int row = (mg + kMG * i) * 16 + Mfma<T>::row(kr, r0 + r);
              if (row < nloc) t += (C)xo[r][j] * acc[i][j][r0 + r];
            }
            pa[j] += t;
          }
        }
      }
    }
  }
  if constexpr (kAlpha) {
    if (wa) {
      // per column: the four row groups (lanes cl + 16 kr) in a fixed order; each wave of
      // a column half leaves its own partial, apart[col][cell slot][mg]
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        pa[j] += __shfl_xor(pa[j], 16);
        pa[j] += __shfl_xor(pa[j], 32);
      }
      if (kr == 0) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int col = col0 + (nh * NT + j) * 16 + cl;
          if (col < ncolr) apart[((int64_t)col * apld + slot0 + ci) * k::kAlphaParts + mg] = pa[j];
        }
      }
    }
  }
}

template <typename T, int CMT, int NS, int KC, int WPE = (CMT <= 4 ? 4 : 2), int NT = kCellNT, int NW = kCellWaves,
          typename IO>
void launch_apply_m(const DevData &d, const T *cells, const IO *X, IO *Y, int ncolr, int64_t ldr,
                    hipStream_t s, const int *any, double *apart = nullptr) {
  const unsigned ny = (unsigned)((ncolr + 32 * NT - 1) / (32 * NT));
  const size_t lds = cell_lds_bytes(d.g.nloc, sizeof(T), NS, KC, sizeof(IO));
  for (int c = 0; c < 8; ++c) {
    const int cnt = d.colour_off[c + 1] - d.colour_off[c];
    if (cnt == 0) continue;
    const int *list = d.colour_cells + d.colour_off[c];
    hipLaunchKernelGGL((k_cell_apply<T, IO, CMT, NS, KC, WPE, NT, NW>), dim3((unsigned)cnt, ny), dim3(NW * 64), lds,
                       s, d,
                       list, d.colour_off[c], cells, X, Y, ncolr, ldr, any, apart, (int64_t)d.colour_off[8]);
  }
}

// Pipeline variants (chunks in flight NS, k-rows per chunk KC, waves per SIMD the
// registers are budgeted for WPE) for cells of up to 256 nodes (degree <= 5); variant 0
// is the default.  The last three budget registers for six waves per SIMD (three
// workgroups per CU), for FP32 blocks only.  Degree 6 cells use the default only.
constexpr int kCellVariants = 9;
constexpr int kCellVariantsF64 = 6;
constexpr int kVarNS[kCellVariants] = {3, 2, 4, 2, 6, 4, 3, 2, 2};
constexpr int kVarKC[kCellVariants] = {8, 8, 4, 16, 4, 8, 8, 8, 16};
constexpr int kVarWPE[kCellVariants] = {4, 4, 4, 4, 4, 4, 6, 6, 6};
// narrow-tile variants (the default pipeline with 64 or 32 columns per workgroup), for
// blocks of at most that many real columns
constexpr int kNarrow64 = 9, kNarrow32 = 10;
// sixteen-wave variants (FP32 blocks): half the M tiles per wave, registers budgeted for
// eight waves per SIMD (two workgroups per CU)
constexpr int kWide0 = 11, kWideN = 3;
constexpr int kWideNS[kWideN] = {3, 4, 2};
constexpr int kWideKC[kWideN] = {8, 8, 16};

template <typename T, int CMT, int V, typename IO>
void launch_v(const DevData &d, const T *cells, const IO *X, IO *Y, int ncolr, int64_t ldr, hipStream_t s,
              const int *any, double *apart) {
  launch_apply_m<T, CMT, kVarNS[V], kVarKC[V], (CMT <= 4 ? kVarWPE[V] : 2)>(d, cells, X, Y, ncolr, ldr, s, any,
                                                                             apart);
}

template <typename T, int CMT, int W, typename IO>
void launch_w(const DevData &d, const T *cells, const IO *X, IO *Y, int ncolr, int64_t ldr, hipStream_t s,
              const int *any, double *apart) {
  launch_apply_m<T, (CMT + 1) / 2, kWideNS[W], kWideKC[W], 8, kCellNT, 16>(d, cells, X, Y, ncolr, ldr, s, any, apart);
}

template <typename T, int CMT, typename IO>
void launch_variant(int v, const DevData &d, const T *cells, const IO *X, IO *Y, int ncolr, int64_t ldr,
                    hipStream_t s, const int *any, double *apart) {
  switch (v) {
    case kNarrow64: launch_apply_m<T, CMT, kVarNS[0], kVarKC[0], kVarWPE[0], 2>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
    case 1: launch_v<T, CMT, 1>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
    case 2: launch_v<T, CMT, 2>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
    case 3: launch_v<T, CMT, 3>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
    case 4: launch_v<T, CMT, 4>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
    case 5: launch_v<T, CMT, 5>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
    case 6: if constexpr (sizeof(T) == 4) { launch_v<T, CMT, 6>(d, cells, X, Y, ncolr, ldr, s, any, apart); break; } [[fallthrough]];
    case 7: if constexpr (sizeof(T) == 4) { launch_v<T, CMT, 7>(d, cells, X, Y, ncolr, ldr, s, any, apart); break; } [[fallthrough]];
    case 8: if constexpr (sizeof(T) == 4) { launch_v<T, CMT, 8>(d, cells, X, Y, ncolr, ldr, s, any, apart); break; } [[fallthrough]];
    case kWide0:
      if constexpr (sizeof(T) == 4) { launch_w<T, CMT, 0>(d, cells, X, Y, ncolr, ldr, s, any, apart); break; } [[fallthrough]];
    case kWide0 + 1:
      if constexpr (sizeof(T) == 4) { launch_w<T, CMT, 1>(d, cells, X, Y, ncolr, ldr, s, any, apart); break; } [[fallthrough]];
    case kWide0 + 2:
      if constexpr (sizeof(T) == 4) { launch_w<T, CMT, 2>(d, cells, X, Y, ncolr, ldr, s, any, apart); break; } [[fallthrough]];
    case kNarrow32:   // FP32 blocks (the FP64 form of one N tile per wave spills its registers)
      if constexpr (sizeof(T) == 4) {
        launch_apply_m<T, CMT, kVarNS[0], kVarKC[0], kVarWPE[0], 1>(d, cells, X, Y, ncolr, ldr, s, any, apart);
        break;
      }
      [[fallthrough]];
    default: launch_v<T, CMT, 0>(d, cells, X, Y, ncolr, ldr, s, any, apart); break;
  }
}

template <typename T, typename IO>
void launch_apply(const DevData &d, const T *cells, const IO *X, IO *Y, int ncolr, int64_t ldr, hipStream_t s,
                  const int *any, int v, double *apart = nullptr) {
  const int nmt = (d.g.nloc + 15) / 16;     // M tiles per cell; wave group w >> 1 takes ceil(nmt / 4)
  if (nmt <= 8) launch_variant<T, 2>(v, d, cells, X, Y, ncolr, ldr, s, any, apart);
  else if (nmt <= 16) launch_variant<T, 4>(v, d, cells, X, Y, ncolr, ldr, s, any, apart);
  else launch_apply_m<T, 6, 3, 8>(d, cells, X, Y, ncolr, ldr, s, any, apart);
}

template <typename T, typename IO, int CMT, int V>
int set_lds_v(size_t esz, int nloc) {
  return (int)hipFuncSetAttribute((const void *)k_cell_apply<T, IO, CMT, kVarNS[V], kVarKC[V], kVarWPE[V]>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)cell_lds_bytes(nloc, esz, kVarNS[V], kVarKC[V], sizeof(IO)));
}

template <typename T, typename IO, int CMT, int NT>
int set_lds_nt(size_t esz, int nloc) {
  return (int)hipFuncSetAttribute((const void *)k_cell_apply<T, IO, CMT, kVarNS[0], kVarKC[0], kVarWPE[0], NT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)cell_lds_bytes(nloc, esz, kVarNS[0], kVarKC[0], sizeof(IO)));
}

template <typename T, typename IO, int CMT, int W>
int set_lds_w(size_t esz, int nloc) {
  return (int)hipFuncSetAttribute(
      (const void *)k_cell_apply<T, IO, (CMT + 1) / 2, kWideNS[W], kWideKC[W], 8, kCellNT, 16>,
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)cell_lds_bytes(nloc, esz, kWideNS[W], kWideKC[W], sizeof(IO)));
}

template <typename T, typename IO, int CMT>
int set_lds_io(int nloc) {
  const size_t e = sizeof(T);
  int st = set_lds_v<T, IO, CMT, 0>(e, nloc) | set_lds_v<T, IO, CMT, 1>(e, nloc) | set_lds_v<T, IO, CMT, 2>(e, nloc) |
           set_lds_v<T, IO, CMT, 3>(e, nloc) | set_lds_v<T, IO, CMT, 4>(e, nloc) | set_lds_v<T, IO, CMT, 5>(e, nloc);
  if constexpr (sizeof(T) == 4)
    st |= set_lds_v<T, IO, CMT, 6>(e, nloc) | set_lds_v<T, IO, CMT, 7>(e, nloc) | set_lds_v<T, IO, CMT, 8>(e, nloc) |
          set_lds_w<T, IO, CMT, 0>(e, nloc) | set_lds_w<T, IO, CMT, 1>(e, nloc) | set_lds_w<T, IO, CMT, 2>(e, nloc);
  if constexpr (sizeof(T) == 4) st |= set_lds_nt<T, IO, CMT, 1>(e, nloc);
  return st | set_lds_nt<T, IO, CMT, 2>(e, nloc);
}

template <typename T, int CMT>
int set_lds_all(int nloc) {
  if constexpr (sizeof(T) == 4) return set_lds_io<T, double, CMT>(nloc) | set_lds_io<T, float, CMT>(nloc);
  else return set_lds_io<T, double, CMT>(nloc);
}

}  // namespace

namespace k {

int cell_variant_count(int nloc, size_t esz) {
  if ((nloc + 15) / 16 > 16) return 1;
  const int nv = esz == 4 ? kCellVariants : kCellVariantsF64;
  int n = 0;
  while (n < nv && cell_lds_bytes(nloc, esz, kVarNS[n], kVarKC[n]) <= 156 * 1024) ++n;   // + static LDS
  return n;
}

int cell_narrow_variants(int nloc, int ncolr, size_t esz, int *out) {
  if ((nloc + 15) / 16 > 16) return 0;
  int n = 0;
  if (ncolr <= 64) out[n++] = kNarrow64;
  if (ncolr <= 32 && esz == 4) out[n++] = kNarrow32;
  return n;
}

int cell_wide_variants(int nloc, size_t esz, int *out) {
  if (esz != 4 || (nloc + 15) / 16 > 16) return 0;
  int n = 0;
  for (int w = 0; w < kWideN; ++w)
    if (cell_lds_bytes(nloc, esz, kWideNS[w], kWideKC[w]) <= 156 * 1024) out[n++] = kWide0 + w;
  return n;
}

void cell_variant_name(int v, char *out, int len) {
  if (v >= kWide0 && v < kWide0 + kWideN) {
    snprintf(out, len, "dense_ns%d_kc%d_16w", kWideNS[v - kWide0], kWideKC[v - kWide0]);
    return;
  }
  if (v == kNarrow64 || v == kNarrow32) {
    snprintf(out, len, "dense_ns%d_kc%d_cols%d", kVarNS[0], kVarKC[0], v == kNarrow64 ? 64 : 32);
    return;
  }
  if (v < 0 || v >= kCellVariants) v = 0;
  if (kVarWPE[v] == 4) snprintf(out, len, "dense_ns%d_kc%d", kVarNS[v], kVarKC[v]);
  else snprintf(out, len, "dense_ns%d_kc%d_w%d", kVarNS[v], kVarKC[v], kVarWPE[v]);
}

int cell_apply_init(int nloc) {
  int st = 0;
  const int nmt = (nloc + 15) / 16;
  if (nmt <= 8) {
    st |= set_lds_all<double, 2>(nloc) | set_lds_all<float, 2>(nloc);
  } else if (nmt <= 16) {
    st |= set_lds_all<double, 4>(nloc) | set_lds_all<float, 4>(nloc);
  } else {
    st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<double, double, 6, 3, 8, 2>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)cell_lds_bytes(nloc, 8, 3, 8));
    st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<float, double, 6, 3, 8, 2>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)cell_lds_bytes(nloc, 4, 3, 8));
    st |= (int)hipFuncSetAttribute((const void *)k_cell_apply<float, float, 6, 3, 8, 2>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)cell_lds_bytes(nloc, 4, 3, 8, 4));
  }
  return st | cell_bf16_init(nloc);
}

void cell_apply(const DevData &d, const void *cells, int dtype, const double *X, double *Y, int ncolr, int64_t ldr,
                hipStream_t s, const int *any, int variant, double *apart) {
  if (dtype == 0) launch_apply<double, double>(d, (const double *)cells, X, Y, ncolr, ldr, s, any, variant, apart);
  else if (dtype == 1) launch_apply<float, double>(d, (const float *)cells, X, Y, ncolr, ldr, s, any, variant);
  else cell_apply_bf16(d, (const uint16_t *)cells, dtype == 4 ? 2 : 1, X, Y, ncolr, ldr, s, any, variant);
}

void cell_apply_f(const DevData &d, const void *cells, int dtype, const void *X, float *Y, int ncolr, int64_t ldf,
                  hipStream_t s, const int *any, int variant) {
  if (dtype == 1) launch_apply<float, float>(d, (const float *)cells, (const float *)X, Y, ncolr, ldf, s, any, variant);
  else cell_apply_bf16_f(d, (const uint16_t *)cells, dtype == 4 ? 2 : 1, X, dtype == 2 ? 1 : 0, Y, ncolr, ldf, s, any,
                         variant);
}

}  // namespace k
}  // namespace efe
