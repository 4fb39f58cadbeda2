// Cell part of Hbar X (Sec. 2.3, eq. (TDKSDiscrete2)) with BF16 products on the
// 16x16x32 BF16 MFMA and FP32 accumulation: Y = sum_c P_c^T Hbar_c P_c X with the
// symmetric cell blocks stored in BF16 and the gathered rows of X rounded to BF16
// on the way into LDS.  The split form keeps each operand as a pair of BF16 values
// (hi = bf16(x), lo = bf16(x - hi)) and adds hi*hi + hi*lo + lo*hi: three MFMAs
// per product, about 16 significant bits.
//
// X and Y are FP64, or the product reads a reduced-precision copy of X (BF16 for the
// BF16 blocks, FP32 for the split form) and leaves its result in FP32.
//
// Storage of the blocks (both forms): row r of a cell's block at r * lda with lda =
// nloc rounded up to 8 elements (every 8-element chunk of a row is one aligned 16-byte
// copy), nloc * lda elements per plane; the split form stores the hi plane, then
// the lo plane.
#include <hip/hip_runtime.h>

#include "common.h"

namespace efe {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kBCols = 96;       // columns per workgroup (six 16-column N tiles)
constexpr int kBRow = 64;        // LDS bytes per operand row of one k-step (32 BF16)
constexpr int kBXPlane = kBCols * kBRow;

// 16-byte slot of chunk q (8 k-values) in LDS row r: a row-dependent XOR keeps the
// 16 rows read by one MFMA operand load on distinct banks.
__device__ __forceinline__ int slot_of(int r, int q) { return q ^ ((r >> 1) & 3); }

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

typedef const void __attribute__((address_space(1))) *gptr_t;
typedef void __attribute__((address_space(3))) *lptr_t;

__device__ __forceinline__ void copy16(const void *src, void *lds_base) {
  __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)lds_base, 16, 0, 0);
}

inline size_t bf16_lds_bytes(int mmax, int planes, int astages = 2) {
  return (size_t)planes * ((size_t)astages * mmax * kBRow + 2 * kBXPlane) + 1024;
}

// One workgroup per (cell, 96 columns) of 4 * 6 / NPW waves; wave w takes the M tiles
// w / G + 4 i (G = 6 / NPW) and the NPW N tiles NPW (w % G) .. + NPW - 1.  K advances in
// steps of 32 k-rows through LDS: the A operand rows [m][32 k] (copied global -> LDS
// directly, one 16-byte chunk per lane; AS stages, so that with three the copies of step
// s + 2 are in flight during step s) and the B operand [n][32 k] (X rows loaded into
// registers one step ahead, rounded to BF16, written transposed; two stages).  MMAX: rows
// of A staged (nloc rounded up to whole M tiles); PL: 1 (BF16) or 2 (split); NPW 3 (8
// waves) or 2 (12 waves, fewer registers per wave: three waves per SIMD for each of two
// workgroups).
template <int MMAX, int CMT, int PL, int NPW, int WPE, typename XT, typename IO, int AS = 2, bool RA = false>
__global__ void __launch_bounds__(4 * (6 / NPW) * 64) __attribute__((amdgpu_waves_per_eu(WPE)))
k_cell_bf16(const DevData d, const int *__restrict__ cell_list, int slot0, const uint16_t *__restrict__ cells,
            const XT *__restrict__ X, IO *__restrict__ Y, int ncolr, int64_t ldr, const int *__restrict__ any) {
  static_assert(MMAX % 16 == 0 && (MMAX / 16 + 3) / 4 <= CMT, "M tiles per wave");
  static_assert(NPW == 2 || NPW == 3, "N tiles per wave");
  constexpr int G = 6 / NPW;                   // N groups
  constexpr int W = 4 * G;                     // waves per workgroup
  constexpr int T = 64 * W;
  constexpr int H = T / (4 * kBCols);          // threads per (column, chunk) of the B operand
  constexpr int XV = 8 / H;                    // X values per thread and k-step
  if (any && *any == 0) return;
  constexpr int kAIns = (MMAX / 16 + W - 1) / W;   // A copies per wave per plane and step
  constexpr int kAPlane = MMAX * kBRow;
  constexpr int kAStage = PL * kAPlane, kBStage = PL * kBXPlane;
  static_assert(AS == 2 || AS == 3, "A stages");
  static_assert(!RA || AS == 2, "block rows through registers: two stages");
  __shared__ int64_t rowoff[MMAX];
  __shared__ unsigned char first[MMAX];
  extern __shared__ __attribute__((aligned(16))) unsigned char bsm[];
  unsigned char *const bsmB = bsm + AS * kAStage;   // B stages after the A stages
  unsigned char *junk = bsmB + 2 * kBStage;
  const Geom &g = d.g;
  const int nloc = g.nloc;
  const int lda = (nloc + 7) & ~7;
  const int64_t plane = (int64_t)nloc * lda;
  const int nmt = (nloc + 15) / 16;
  const int nks = (nloc + 31) / 32;
  const int ci = blockIdx.x;
  const int col0 = blockIdx.y * kBCols;
  const int wcol = ncolr - col0 < kBCols ? ncolr - col0 : kBCols;
  const int64_t cell = cell_list[ci];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int mg = wave / G, ng = wave % G;
  int e[3];
  cell_ijk(g, cell, e);
  for (int l = tid; l < nloc; l += T) {
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
  __syncthreads();
  const uint16_t *Ag = cells + (int64_t)(slot0 + ci) * PL * plane;
  // A rows of k-step s: instruction i of a wave copies rows 16 (wave + W i) .. +15, lane L
  // row 16 (.) + L / 4 into LDS slot L & 3, which holds chunk slot ^ swizzle of that row.
  // Rows past nloc and chunks past the row end copy the block's first chunk instead
  // (finite values that only meet zero rows of X or output rows never stored).
  auto issueA = [&](int s, int st) {
#pragma unroll
    for (int pl = 0; pl < PL; ++pl)
#pragma unroll
      for (int i = 0; i < kAIns; ++i) {
        const int ins = wave + W * i;
        if (ins < MMAX / 16) {
          const int r = 16 * ins + (lane >> 2), sl = lane & 3;
          const int q = sl ^ ((r >> 1) & 3);
          const int k0 = 32 * s + 8 * q;
          const bool ok = r < nloc && k0 < nloc;
          copy16(Ag + pl * plane + (ok ? (int64_t)r * lda + k0 : 0),
                 bsm + st * kAStage + pl * kAPlane + ins * 1024);
        } else {
          copy16(Ag, junk);
        }
      }
  };
  // RA: the same rows through registers (16-byte loads, written to LDS after the step's
  // MFMAs, beside the B operand) instead of direct copies into LDS
  u32x4 ra[PL][kAIns];
  auto loadA = [&](int s) {
#pragma unroll
    for (int pl = 0; pl < PL; ++pl)
#pragma unroll
      for (int i = 0; i < kAIns; ++i) {
        const int ins = wave + W * i;
        if (ins < MMAX / 16) {
          const int r = 16 * ins + (lane >> 2), sl = lane & 3;
          const int q = sl ^ ((r >> 1) & 3);
          const int k0 = 32 * s + 8 * q;
          const bool ok = r < nloc && k0 < nloc;
          ra[pl][i] = *(const u32x4 *)(Ag + pl * plane + (ok ? (int64_t)r * lda + k0 : 0));
        }
      }
  };
  auto storeA = [&](int st) {
#pragma unroll
    for (int pl = 0; pl < PL; ++pl)
#pragma unroll
      for (int i = 0; i < kAIns; ++i) {
        const int ins = wave + W * i;
        if (ins < MMAX / 16) *(u32x4 *)(bsm + st * kAStage + pl * kAPlane + ins * 1024 + lane * 16) = ra[pl][i];
      }
  };
  // B operand of k-step s: thread t < 384 H takes column n = t % 96, chunk q = (t / 96) % 4
  // (k = 32 s + 8 q .. + 7) and part t / 384 of it (XV of the 8 k-values), rounded (and
  // split) to BF16
  const int xn = tid % kBCols, xq = (tid / kBCols) % 4, xp = tid / (4 * kBCols);
  const bool xthr = tid < 4 * kBCols * H;
  XT xv[XV];
  auto loadX = [&](int s) {
#pragma unroll
    for (int j = 0; j < XV; ++j) {
      const int k = 32 * s + 8 * xq + XV * xp + j;
      xv[j] = (xthr && xn < wcol && k < nloc) ? X[rowoff[k] + col0 + xn] : XT{};
    }
  };
  auto writeX = [&](int st) {
    if (!xthr) return;
    uint32_t hi[XV / 2], lo[XV / 2];
#pragma unroll
    for (int j = 0; j < XV / 2; ++j) {
      const float f0 = to_float(xv[2 * j]), f1 = to_float(xv[2 * j + 1]);
      const uint16_t h0 = bf16_rne(f0), h1 = bf16_rne(f1);
      hi[j] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      if (PL == 2) {
        const uint16_t l0 = bf16_rne(f0 - bf16_val(h0)), l1 = bf16_rne(f1 - bf16_val(h1));
        lo[j] = (uint32_t)l0 | ((uint32_t)l1 << 16);
      }
    }
    unsigned char *xb = bsmB + st * kBStage + xn * kBRow + slot_of(xn, xq) * 16 + xp * 2 * XV;
    if (XV == 8) {
      *(u32x4 *)xb = u32x4{hi[0], hi[1], hi[2], hi[3]};
      if (PL == 2) *(u32x4 *)(xb + kBXPlane) = u32x4{lo[0], lo[1], lo[2], lo[3]};
    } else {
      *(u32x2 *)xb = u32x2{hi[0], hi[1]};
      if (PL == 2) *(u32x2 *)(xb + kBXPlane) = u32x2{lo[0], lo[1]};
    }
  };
  v4f acc[CMT][NPW];
#pragma unroll
  for (int i = 0; i < CMT; ++i)
#pragma unroll
    for (int j = 0; j < NPW; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int cl = lane & 15, kg = lane >> 4;
  if constexpr (RA) {
    loadA(0);
    storeA(0);
  } else {
    issueA(0, 0);
    if (AS == 3 && nks > 1) issueA(1, 1);
  }
  loadX(0);
  writeX(0);
  wait_vm<0>();
  __syncthreads();
  for (int s = 0; s < nks; ++s) {
    const int st = s & 1, sa = AS == 2 ? st : s % 3;
    if constexpr (AS == 2) {
      if (s + 1 < nks) {
        if constexpr (RA) loadA(s + 1);
        else issueA(s + 1, st ^ 1);
        loadX(s + 1);
      }
    } else {
      // the X loads first: the wait the compiler puts before writeX then leaves the A
      // copies of step s + 2, issued after them, in flight
      if (s + 1 < nks) loadX(s + 1);
      if (s + 2 < nks) issueA(s + 2, (s + 2) % 3);
    }
    const unsigned char *Ast = bsm + sa * kAStage;
    const unsigned char *Bst = bsmB + st * kBStage;
    bf16x8 b[NPW], bl[NPW];
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
      const int n = 16 * (NPW * ng + j) + cl;
      b[j] = *(const bf16x8 *)(Bst + n * kBRow + slot_of(n, kg) * 16);
      if (PL == 2) bl[j] = *(const bf16x8 *)(Bst + kBXPlane + n * kBRow + slot_of(n, kg) * 16);
    }
#pragma unroll
    for (int i = 0; i < CMT; ++i) {
      const int t = mg + 4 * i;
      if (t < nmt) {
        const int m = 16 * t + cl;
        const bf16x8 a = *(const bf16x8 *)(Ast + m * kBRow + slot_of(m, kg) * 16);
        bf16x8 al;
        if (PL == 2) al = *(const bf16x8 *)(Ast + kAPlane + m * kBRow + slot_of(m, kg) * 16);
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
          if (PL == 2) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (s + 1 < nks) {
      if constexpr (RA) storeA(st ^ 1);
      writeX(st ^ 1);
    }
    // this wave's copies of step s + 1 have landed once at most the copies of step s + 2
    // (the last ones issued, PL * kAIns per wave, padding copies included) remain
    if (AS == 3 && s + 2 < nks) wait_vm<PL * kAIns>();
    else wait_vm<0>();
    __syncthreads();
  }
  // output register r of a lane holds row 4 (lane / 16) + r, column lane % 16 of its tile.
  // Every earlier value of Y the wave adds to (the rows a previous colour reached) is
  // loaded before any store: with FP32 rows all tiles at once (one memory round trip for
  // the read-modify-write), with FP64 rows tile by tile (the registers of all tiles'
  // values would spill).
  constexpr int TB = sizeof(IO) == 4 ? CMT : 1;   // tiles whose loads are issued together
#pragma unroll
  for (int i0 = 0; i0 < CMT; i0 += TB) {
    IO old[TB][4][NPW];
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      const int t = mg + 4 * (i0 + i);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * t + 4 * kg + r;
        const bool add = t < nmt && row < nloc && !first[row];
        const IO *yr = Y + (add ? rowoff[row] : 0);
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
          const int col = col0 + 16 * (NPW * ng + j) + cl;
          old[i][r][j] = (add && col < ncolr) ? yr[col] : (IO)0;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TB; ++i) {
      const int t = mg + 4 * (i0 + i);
      if (t >= nmt) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * t + 4 * kg + r;
        if (row >= nloc) continue;
        IO *yr = Y + rowoff[row];
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
          const int col = col0 + 16 * (NPW * ng + j) + cl;
          if (col < ncolr) yr[col] = old[i][r][j] + (IO)acc[i0 + i][j][r];
        }
      }
    }
  }
}

template <int MMAX, int CMT, int PL, int NPW, int WPE, typename XT, typename IO, int AS = 2, bool RA = false>
void launch_bf16(const DevData &d, const uint16_t *cells, const XT *X, IO *Y, int ncolr, int64_t ldr,
                 hipStream_t s, const int *any) {
  const unsigned ny = (unsigned)((ncolr + kBCols - 1) / kBCols);
  const size_t lds = bf16_lds_bytes(MMAX, PL, AS);
  for (int c = 0; c < 8; ++c) {
    const int cnt = d.colour_off[c + 1] - d.colour_off[c];
    if (cnt == 0) continue;
    const int *list = d.colour_cells + d.colour_off[c];
    hipLaunchKernelGGL((k_cell_bf16<MMAX, CMT, PL, NPW, WPE, XT, IO, AS, RA>), dim3((unsigned)cnt, ny),
                       dim3(4 * (6 / NPW) * 64), lds, s, d, list, d.colour_off[c], cells, X, Y, ncolr, ldr, any);
  }
}

template <int MMAX, int CMT, int PL, int NPW, int WPE, int AS = 2, bool RA = false>
int set_lds_bf16() {
  const int lds = (int)bf16_lds_bytes(MMAX, PL, AS);
  return (int)hipFuncSetAttribute((const void *)k_cell_bf16<MMAX, CMT, PL, NPW, WPE, double, double, AS, RA>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds) |
         (int)hipFuncSetAttribute((const void *)k_cell_bf16<MMAX, CMT, PL, NPW, WPE, float, float, AS, RA>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds) |
         (int)hipFuncSetAttribute((const void *)k_cell_bf16<MMAX, CMT, PL, NPW, WPE, Bf16, float, AS, RA>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// variant 0: eight waves of three N tiles, four waves per SIMD (two workgroups per CU);
// variant 1: twelve waves of two N tiles, six waves per SIMD; variants 2 and 3: the same
// with the block rows through registers; 4 and 5: with three stages of block rows (2 to 5
// for BF16 blocks, one plane; the split form runs 0 or 1 instead)
template <int MMAX, int CMT, int PL, typename XT, typename IO>
void launch_bf16_v(int v, const DevData &d, const uint16_t *cells, const XT *X, IO *Y, int ncolr,
                   int64_t ldr, hipStream_t s, const int *any) {
  if constexpr (PL == 1) {
    if (v == 5) return launch_bf16<MMAX, CMT, PL, 2, 6, XT, IO, 3>(d, cells, X, Y, ncolr, ldr, s, any);
    if (v == 4) return launch_bf16<MMAX, CMT, PL, 3, 4, XT, IO, 3>(d, cells, X, Y, ncolr, ldr, s, any);
    if (v == 3) return launch_bf16<MMAX, CMT, PL, 2, 6, XT, IO, 2, true>(d, cells, X, Y, ncolr, ldr, s, any);
    if (v == 2) return launch_bf16<MMAX, CMT, PL, 3, 4, XT, IO, 2, true>(d, cells, X, Y, ncolr, ldr, s, any);
  }
  if (v & 1) launch_bf16<MMAX, CMT, PL, 2, 6>(d, cells, X, Y, ncolr, ldr, s, any);
  else launch_bf16<MMAX, CMT, PL, 3, 4>(d, cells, X, Y, ncolr, ldr, s, any);
}

template <int MMAX, int CMT>
int set_lds_bf16_all() {
  return set_lds_bf16<MMAX, CMT, 1, 3, 4>() | set_lds_bf16<MMAX, CMT, 2, 3, 4>() | set_lds_bf16<MMAX, CMT, 1, 2, 6>() |
         set_lds_bf16<MMAX, CMT, 2, 2, 6>() | set_lds_bf16<MMAX, CMT, 1, 3, 4, 3>() | set_lds_bf16<MMAX, CMT, 1, 2, 6, 3>() |
         set_lds_bf16<MMAX, CMT, 1, 3, 4, 2, true>() | set_lds_bf16<MMAX, CMT, 1, 2, 6, 2, true>();
}

}  // namespace

namespace k {

int64_t bf16_block_elems(const Geom &g, int planes) {
  return (int64_t)planes * g.nloc * ((g.nloc + 7) & ~7);
}

int cell_bf16_variant_count(int nloc, int planes) { return nloc <= 224 ? (planes == 1 ? 6 : 2) : 1; }

int cell_bf16_init(int nloc) {
  if (nloc > 352) return 1;
  if (nloc <= 128) return set_lds_bf16_all<128, 2>();
  if (nloc <= 224) return set_lds_bf16_all<224, 4>();
  return set_lds_bf16<352, 6, 1, 3, 2>() | set_lds_bf16<352, 6, 2, 3, 2>();
}

template <typename XT, typename IO>
void cell_apply_bf16_io(const DevData &d, const uint16_t *cells, int planes, const XT *X, IO *Y, int ncolr,
                        int64_t ldr, hipStream_t s, const int *any, int variant) {
  const int nloc = d.g.nloc;
  if (nloc <= 128) {
    if (planes == 1) launch_bf16_v<128, 2, 1>(variant, d, cells, X, Y, ncolr, ldr, s, any);
    else launch_bf16_v<128, 2, 2>(variant, d, cells, X, Y, ncolr, ldr, s, any);
  } else if (nloc <= 224) {
    if (planes == 1) launch_bf16_v<224, 4, 1>(variant, d, cells, X, Y, ncolr, ldr, s, any);
    else launch_bf16_v<224, 4, 2>(variant, d, cells, X, Y, ncolr, ldr, s, any);
  } else {
    if (planes == 1) launch_bf16<352, 6, 1, 3, 2>(d, cells, X, Y, ncolr, ldr, s, any);
    else launch_bf16<352, 6, 2, 3, 2>(d, cells, X, Y, ncolr, ldr, s, any);
  }
}

void cell_apply_bf16(const DevData &d, const uint16_t *cells, int planes, const double *X, double *Y, int ncolr,
                     int64_t ldr, hipStream_t s, const int *any, int variant) {
  cell_apply_bf16_io(d, cells, planes, X, Y, ncolr, ldr, s, any, variant);
}

void cell_apply_bf16_f(const DevData &d, const uint16_t *cells, int planes, const void *X, int x_bf16, float *Y,
                       int ncolr, int64_t ldf, hipStream_t s, const int *any, int variant) {
  if (x_bf16 && planes == 1) cell_apply_bf16_io(d, cells, 1, (const Bf16 *)X, Y, ncolr, ldf, s, any, variant);
  else cell_apply_bf16_io(d, cells, planes, (const float *)X, Y, ncolr, ldf, s, any, variant);
}

}  // namespace k
}  // namespace efe
