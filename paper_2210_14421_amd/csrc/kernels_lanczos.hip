// Lanczos vector kernels (Sec. 2.6): Gram-Schmidt dot products, updates,
// coefficient bookkeeping and the final Krylov combination.
//
// Blocks are n_rows x ncol complex values, row-major (704 B per row at 44
// orbitals).  Every kernel gives each thread one fixed column and walks rows
// with a grid stride, so the per-column sums stay in registers.  The dot
// kernels run 704-thread blocks (16 rows x 44 columns, no idle lane) at six
// waves per SIMD, two blocks per CU; the update and combination kernels,
// which hold their 16 coefficients in LDS and two rows in flight, run
// 448-thread blocks (10 rows x 44 columns).  Measured on the Na8 block
// (1.25 GB): dots 6.3 TB/s, updates 5.0-5.5 TB/s.
//
// The Krylov basis is kept unnormalised: slot 0 is the caller's input block
// itself and slot l >= 1 holds a multiple of the Lanczos vector q_{l+1}; the
// per-column factors sig[l] = 1 / ||slot l|| turn stored slots into q_l.  This
// removes the normalisation pass of every iteration (the Hbar X output is
// written straight into the next slot and orthogonalised in place).
//
// With reduced-precision products the Hbar X output is an FP32 block (row stride
// wld complex values) that the first update reads and writes, orthogonalised, into
// the FP64 slot; the update also leaves an FP32 copy of the slot (the next
// product's input).  The recurrence itself is FP64 throughout.
#include "common.h"

namespace efe {
namespace {

constexpr int kLzThreads = 704;      // dot kernels; also the launch bound of all
constexpr int kLzUpdThreads = 448;   // update and combination kernels
constexpr int kLzChunk = 16;     // basis vectors per streaming pass
constexpr int kLzBlocks = k::kDotBlocksMax;

struct Basis {
  const double2 *q0;      // slot 0
  const double2 *qb;      // slot 1
  int64_t stride2;        // double2 elements between slots >= 1
};

__device__ __forceinline__ const double2 *slot_ptr(const Basis &B, int l) {
  return l == 0 ? B.q0 : B.qb + (int64_t)(l - 1) * B.stride2;
}

__device__ __forceinline__ double2 ldnt(const double2 *p) {
  double2 v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}
__device__ __forceinline__ double2 ldnt(const float2 *p) {
  const float x = __builtin_nontemporal_load(&p->x), y = __builtin_nontemporal_load(&p->y);
  return make_double2((double)x, (double)y);
}
__device__ __forceinline__ void stnt(double2 *p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
// one complex value of the reduced-precision copy of a Lanczos vector (two floats, or
// two BF16 values in one 32-bit word)
__device__ __forceinline__ void stnt(float *p, double2 v) {
  __builtin_nontemporal_store((float)v.x, p);
  __builtin_nontemporal_store((float)v.y, p + 1);
}
__device__ __forceinline__ void stnt(Bf16 *p, double2 v) {
  const uint32_t w = (uint32_t)bf16_bits((float)v.x) | ((uint32_t)bf16_bits((float)v.y) << 16);
  __builtin_nontemporal_store(w, (uint32_t *)p);
}

// part[blk][l0 + v][c] (double2) for v < nl: sum_r conj(slot_{l0+v}[r][c]) w[r][c];
// with_norm adds entry l0 + nl = ||w[:, c]||^2.  Columns with mask[c] == 0
// contribute zeros.  Returns at once when *any == 0.  w: FP64 or FP32 complex, wld
// complex values per row.
template <int NL, typename W2>
__global__ void __launch_bounds__(kLzThreads) __attribute__((amdgpu_waves_per_eu(NL <= 8 ? 6 : 4)))
k_lz_dots(Basis B, int l0, int nl, const W2 *__restrict__ w, int64_t wld, int64_t nrows, int ncol,
          const int *__restrict__ mask, const int *__restrict__ any, int with_norm, int nvtot,
          double2 *__restrict__ part) {
  if (any && *any == 0) return;
  __shared__ double2 red[kLzThreads];
  const int R = blockDim.x / ncol;
  const int c = threadIdx.x % ncol, r0 = threadIdx.x / ncol;
  const bool on = r0 < R && mask[c] != 0;
  double2 acc[NL + 1];
#pragma unroll
  for (int l = 0; l <= NL; ++l) acc[l] = make_double2(0.0, 0.0);
  if (on) {
    const double2 *q[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) q[l] = slot_ptr(B, l0 + (l < nl ? l : 0));
    for (int64_t r = (int64_t)blockIdx.x * R + r0; r < nrows; r += (int64_t)gridDim.x * R) {
      const int64_t o = r * ncol + c;
      const double2 wv = ldnt(w + r * wld + c);
#pragma unroll
      for (int l = 0; l < NL; ++l)
        if (l < nl) {
          const double2 qv = ldnt(q[l] + o);
          acc[l].x += qv.x * wv.x + qv.y * wv.y;
          acc[l].y += qv.x * wv.y - qv.y * wv.x;
        }
      acc[NL].x += wv.x * wv.x + wv.y * wv.y;
    }
  }
#pragma unroll
  for (int v = 0; v <= NL; ++v) {
    const bool is_dot = v < nl, is_norm = with_norm && v == nl;
    if (!is_dot && !is_norm) continue;
    __syncthreads();
    red[threadIdx.x] = on ? (is_dot ? acc[v] : acc[NL]) : make_double2(0.0, 0.0);
    __syncthreads();
    if (threadIdx.x < ncol) {
      double2 s = make_double2(0.0, 0.0);
      for (int rr = 0; rr < R; ++rr) {
        const double2 t = red[rr * ncol + threadIdx.x];
        s.x += t.x;
        s.y += t.y;
      }
      part[((int64_t)blockIdx.x * nvtot + l0 + v) * ncol + threadIdx.x] = s;
    }
  }
}

// w <- gw[c] src - sum_{l < nl} coef[l0 + l][c] slot_{l0+l}  (mask[c] != 0); src is w
// itself (in place) or another block (FP64 or FP32 complex, sld complex values per
// row); sh, when given, receives an FP32 or BF16 copy of the result (shld complex values
// per row).  with_norm writes the partial ||w||^2 of the result to part[blk][c].x and
// that of the pass's input (gw[c] src for a pass of one chunk) to part[blk][c].y.
// gw == nullptr means 1.  zero_masked clears the columns with mask[c] == 0 instead
// (stopped columns: their later slots stay zero).
template <int NL, typename S2, bool INPLACE, typename SHT>
__global__ void __launch_bounds__(kLzThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_lz_update(Basis B, int l0, int nl, const double2 *__restrict__ coef, const double *__restrict__ gw,
            const S2 *__restrict__ src, int64_t sld, double2 *__restrict__ w, SHT *__restrict__ sh, int64_t shld,
            int64_t nrows, int ncol, const int *__restrict__ mask, const int *__restrict__ any, int with_norm,
            int zero_masked, double2 *__restrict__ part) {
  if (any && *any == 0) return;
  extern __shared__ double2 lz_sm[];
  double2 *cs = lz_sm;                       // nl * ncol
  double2 *red = lz_sm + (size_t)NL * ncol;  // blockDim.x
  for (int t = threadIdx.x; t < nl * ncol; t += blockDim.x) cs[t] = coef[(int64_t)l0 * ncol + t];
  __syncthreads();
  const int R = blockDim.x / ncol;
  const int c = threadIdx.x % ncol, r0 = threadIdx.x / ncol;
  const bool on = r0 < R && mask[c] != 0;
  double nrm = 0.0, nin = 0.0;
  if (r0 < R && !on && zero_masked) {
    for (int64_t r = (int64_t)blockIdx.x * R + r0; r < nrows; r += (int64_t)gridDim.x * R) {
      w[r * ncol + c] = make_double2(0.0, 0.0);
      if (sh) stnt(sh + 2 * (r * shld + c), make_double2(0.0, 0.0));
    }
  }
  if (on) {
    const double g = gw ? gw[c] : 1.0;
    const double2 *q[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) q[l] = slot_ptr(B, l0 + (l < nl ? l : 0));
    // RU rows per step (two for the three-term step, one for the long passes, whose
    // loads of NL slots fill the registers)
    constexpr int RU = NL <= 4 ? 2 : 1;
    const int64_t step = (int64_t)gridDim.x * R;
    int64_t r = (int64_t)blockIdx.x * R + r0;
    for (; r + (RU - 1) * step < nrows; r += RU * step) {
      double2 v[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t ru = r + u * step;
        if constexpr (INPLACE) v[u] = ldnt(w + ru * ncol + c);
        else v[u] = ldnt(src + ru * sld + c);
        v[u].x *= g;
        v[u].y *= g;
        nin += v[u].x * v[u].x + v[u].y * v[u].y;
      }
#pragma unroll
      for (int l = 0; l < NL; ++l)
        if (l < nl) {
          const double2 h = cs[l * ncol + c];
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const double2 qv = ldnt(q[l] + (r + u * step) * ncol + c);
            v[u].x -= h.x * qv.x - h.y * qv.y;
            v[u].y -= h.x * qv.y + h.y * qv.x;
          }
        }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t ru = r + u * step;
        stnt(w + ru * ncol + c, v[u]);
        if (sh) stnt(sh + 2 * (ru * shld + c), v[u]);
        nrm += v[u].x * v[u].x + v[u].y * v[u].y;
      }
    }
    for (; r < nrows; r += step) {
      const int64_t oa = r * ncol + c;
      double2 va;
      if constexpr (INPLACE) va = ldnt(w + oa);
      else va = ldnt(src + r * sld + c);
      va.x *= g; va.y *= g;
      nin += va.x * va.x + va.y * va.y;
#pragma unroll
      for (int l = 0; l < NL; ++l)
        if (l < nl) {
          const double2 qa = ldnt(q[l] + oa);
          const double2 h = cs[l * ncol + c];
          va.x -= h.x * qa.x - h.y * qa.y;
          va.y -= h.x * qa.y + h.y * qa.x;
        }
      stnt(w + oa, va);
      if (sh) stnt(sh + 2 * (r * shld + c), va);
      nrm += va.x * va.x + va.y * va.y;
    }
  }
  if (!with_norm) return;
  red[threadIdx.x] = on ? make_double2(nrm, nin) : make_double2(0.0, 0.0);
  __syncthreads();
  if (threadIdx.x < ncol) {
    double s = 0.0, si = 0.0;
    for (int rr = 0; rr < R; ++rr) {
      s += red[rr * ncol + threadIdx.x].x;
      si += red[rr * ncol + threadIdx.x].y;
    }
    part[(int64_t)blockIdx.x * ncol + threadIdx.x] = make_double2(s, si);
  }
}

// out <- (acc ? out : 0) + sum_{l < nl} coef[l0 + l][c] slot_{l0+l}   (all columns)
template <int NL>
__global__ void __launch_bounds__(kLzThreads)
k_lz_combine(Basis B, int l0, int nl, const double2 *__restrict__ coef, double2 *__restrict__ out, int64_t nrows,
             int ncol, int acc_out, const int *__restrict__ nq_dev) {
  if (nq_dev) {
    const int lim = *nq_dev - l0;
    if (lim <= 0 && acc_out) return;
    nl = lim < nl ? (lim > 0 ? lim : 0) : nl;
  }
  extern __shared__ double2 lz_sm[];
  double2 *cs = lz_sm;
  for (int t = threadIdx.x; t < nl * ncol; t += blockDim.x) cs[t] = coef[(int64_t)l0 * ncol + t];
  __syncthreads();
  const int R = blockDim.x / ncol;
  const int c = threadIdx.x % ncol, r0 = threadIdx.x / ncol;
  if (r0 >= R) return;
  const double2 *q[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) q[l] = slot_ptr(B, l0 + (l < nl ? l : 0));
  const int64_t step = (int64_t)gridDim.x * R;
  int64_t r = (int64_t)blockIdx.x * R + r0;
  // slots past a column's k hold unused data: they are not read (their coefficient is
  // zero); the loads of a row's slots are all issued before its first product
  bool use[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const double2 h = l < nl ? cs[l * ncol + c] : make_double2(0.0, 0.0);
    use[l] = h.x != 0.0 || h.y != 0.0;
  }
  for (; r < nrows; r += step) {
    const int64_t oa = r * ncol + c;
    double2 qa[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      qa[l] = make_double2(0.0, 0.0);
      if (use[l]) qa[l] = ldnt(q[l] + oa);
    }
    double2 va = acc_out ? out[oa] : make_double2(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < NL; ++l)
      if (use[l]) {
        const double2 h = cs[l * ncol + c];
        va.x += h.x * qa[l].x - h.y * qa[l].y;
        va.y += h.x * qa[l].y + h.y * qa[l].x;
      }
    stnt(out + oa, va);
  }
}

// ------------------------------------------------------------ coefficients
constexpr double kReorthEta = 1e-3;

// Start: beta0 = ||X||, sig_0 = 1 / beta0, active = beta0 > 0; the partial
// reorthogonalisation state (||T|| estimate, forced pass, omega_1 = 1) restarts.
__global__ void k_lz_init(const double2 *__restrict__ h0, int ncol, double *__restrict__ beta0,
                          double *__restrict__ sig, int *__restrict__ active, int *__restrict__ kused,
                          ProState pro) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double n2 = h0[c].x;
  // a NaN norm stays NaN (the host reports a non-finite input), only a zero column is inactive
  const double b = n2 > 0.0 || n2 != n2 ? sqrt(n2) : 0.0;
  beta0[c] = b;
  sig[c] = b > 0.0 ? 1.0 / b : 0.0;
  active[c] = b > 0.0 ? 1 : 0;
  kused[c] = 0;
  if (pro.om) {
    pro.anorm[c] = 0.0;
    pro.force[c] = 0;
    pro.om[((int64_t)1 * pro.ld) * ncol + c] = 1.0;   // omega_{1,1} (row of q_1: 1 % 3)
  }
}

// After the first dot pass of iteration j (slot j = Hbar slot_{j-1}) over the
// slots first .. j-1: h[l - first][c] = <slot_l, slot_j> and h[j - first][c] =
// ||slot_j||^2.  alpha_j = sig_{j-1}^2 Re <slot_{j-1}, slot_j>; the first update is
// slot_j <- g (slot_j - sum_l sig_l^2 h[l] slot_l) with g = 1 / ||slot_j||,
// after which the Lanczos residual is msc * slot_j with msc = sig_{j-1} / g.
// first = 0: all previous slots; first = j - 2: the two latest (partial scheme).
__global__ void k_lz_coef1(const double2 *__restrict__ h, const double *__restrict__ sig, int j, int first, int ncol,
                           const int *__restrict__ active, double *__restrict__ alpha_j, double2 *__restrict__ coef,
                           double *__restrict__ gsc, double *__restrict__ msc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol || !active[c]) return;
  const double w2 = h[(int64_t)(j - first) * ncol + c].x;
  const double g = w2 > 0.0 ? 1.0 / sqrt(w2) : 0.0;
  const double sj = sig[(int64_t)(j - 1) * ncol + c];
  alpha_j[c] = sj * sj * h[(int64_t)(j - 1 - first) * ncol + c].x;
  for (int l = first; l < j; ++l) {
    const double s = sig[(int64_t)l * ncol + c];
    const double f = g * s * s;
    const double2 v = h[(int64_t)(l - first) * ncol + c];
    coef[(int64_t)(l - first) * ncol + c] = make_double2(f * v.x, f * v.y);
  }
  gsc[c] = g;
  msc[c] = g > 0.0 ? sj / g : 0.0;
}

// Three-term step of iteration j (partial scheme): h[0][c] = <slot_{j-1}, slot_j>, h[1][c] =
// ||slot_j||^2.  alpha_j = sig_{j-1}^2 Re h[0]; the update (slots j-2, j-1) is
// slot_j <- g (slot_j - beta_{j-1} sig_{j-2} / sig_{j-1} slot_{j-2} - sig_{j-1}^2 h[0] slot_{j-1}),
// g = 1 / ||slot_j||: the recurrence's beta_{j-1} q_{j-1} written in the stored slots.
__global__ void k_lz_coef3(const double2 *__restrict__ h, const double *__restrict__ sig,
                           const double *__restrict__ beta, int j, int ncol, const int *__restrict__ active,
                           double *__restrict__ alpha_j, double2 *__restrict__ coef, double *__restrict__ gsc,
                           double *__restrict__ msc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol || !active[c]) return;
  const double w2 = h[ncol + c].x;
  const double g = w2 > 0.0 ? 1.0 / sqrt(w2) : 0.0;
  const double sj = sig[(int64_t)(j - 1) * ncol + c];
  const double2 v = h[c];
  alpha_j[c] = sj * sj * v.x;
  const double f = g * sj * sj;
  if (j >= 2) {
    const double sp = sig[(int64_t)(j - 2) * ncol + c];
    const double bp = beta[(int64_t)(j - 2) * ncol + c];
    coef[c] = make_double2(sj > 0.0 ? g * bp * sp / sj : 0.0, 0.0);
    coef[(int64_t)ncol + c] = make_double2(f * v.x, f * v.y);
  } else {
    coef[c] = make_double2(f * v.x, f * v.y);
  }
  gsc[c] = g;
  msc[c] = g > 0.0 ? sj / g : 0.0;
}

// x^H Hbar x of the product's input, first level: lvl[c][sl] = sum of the cell partials
// apart[c][part] of slice sl (a contiguous range of parts), the last slice with the
// enrichment terms aE[k][c] (k < nk) as well, each summed in a fixed order.  Grid
// (ncolr, kAlphaSlices).
constexpr int kAlphaSlices = k::kAlphaLvl;
__global__ void __launch_bounds__(256)
k_lz_alpha_sum(const double *__restrict__ apart, int nparts, const double *__restrict__ aE, int nk, int ncolr,
               const int *__restrict__ any, double *__restrict__ lvl) {
  if (any && *any == 0) return;
  __shared__ double red[256];
  const int c = blockIdx.x, sl = blockIdx.y;
  const int per = (nparts + kAlphaSlices - 1) / kAlphaSlices;
  const int b0 = sl * per, b1 = b0 + per < nparts ? b0 + per : nparts;
  const double *pc = apart + (int64_t)c * nparts;
  double acc = 0.0;
  for (int i = b0 + threadIdx.x; i < b1; i += 256) acc += pc[i];
  if (sl == kAlphaSlices - 1)
    for (int k = threadIdx.x; k < nk; k += 256) acc += aE[(int64_t)k * ncolr + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lvl[c * kAlphaSlices + sl] = red[0];
}

// The three-term step from hx = x^H Hbar x of slot j - 1 (no dot pass): per real column, the
// slice sums lvl[col][0..kAlphaSlices) in order; alpha_j = sig_{j-1}^2 (hx[2c] + hx[2c + 1]);
// the update scales by g = sig_{j-1}, so that slot j becomes the Lanczos residual itself
// (msc = 1):
// slot_j <- sig_{j-1} slot_j - beta_{j-1} sig_{j-2} slot_{j-2} - sig_{j-1}^3 hx slot_{j-1}.
__global__ void k_lz_coef3x(const double *__restrict__ lvl, const double *__restrict__ sig,
                            const double *__restrict__ beta, int j, int ncol, const int *__restrict__ active,
                            double *__restrict__ alpha_j, double2 *__restrict__ coef, double *__restrict__ gsc,
                            double *__restrict__ msc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol || !active[c]) return;
  const double sj = sig[(int64_t)(j - 1) * ncol + c];
  double hx[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double *lv = lvl + (2 * c + h) * kAlphaSlices;
    double t = 0.0;
#pragma unroll
    for (int sl = 0; sl < kAlphaSlices; ++sl) t += lv[sl];
    hx[h] = t;
  }
  const double v = hx[0] + hx[1];
  alpha_j[c] = sj * sj * v;
  const double f = sj * sj * sj * v;
  if (j >= 2) {
    coef[c] = make_double2(beta[(int64_t)(j - 2) * ncol + c] * sig[(int64_t)(j - 2) * ncol + c], 0.0);
    coef[(int64_t)ncol + c] = make_double2(f, 0.0);
  } else {
    coef[c] = make_double2(f, 0.0);
  }
  gsc[c] = sj;
  msc[c] = 1.0;
}

// Partial reorthogonalisation (Simon 1984): after the local pass of iteration j,
// beta_j ~ msc ||slot_j|| and the omega recurrence estimates omega_{j+1,k} ~
// q_{j+1}^H q_k from alpha_1..j, beta_1..j-1 and the rows omega_j, omega_{j-1}:
//   beta_j omega_{j+1,k} = beta_k omega_{j,k+1} + (alpha_k - alpha_j) omega_{j,k}
//                          + beta_{k-1} omega_{j,k-1} - beta_{j-1} omega_{j-1,k}  (k < j)
// plus 2 eps ||T|| with the sign of the sum; omega_{j+1,j} = eps ||T|| / beta_j and
// omega_{j+1,j+1} = 1 (||T|| = running max of |alpha_i| + beta_i + beta_{i-1}).
// A column needs a pass against every previous slot when an estimate exceeds
// sqrt(eps), when the previous iteration's estimates did (the pass is made for two
// vectors in a row), or when the local pass cancelled most of the vector; the
// estimates of a column that gets the pass restart at eps.  One thread per column.
__global__ void k_lz_pro(const double2 *__restrict__ nrm1, const double *__restrict__ msc,
                         const double *__restrict__ alpha, const double *__restrict__ beta, int j, int ncol,
                         const int *__restrict__ active, ProState pro, int *__restrict__ need, int *__restrict__ any,
                         int rel) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  constexpr double eps = 2.220446049250313e-16, sqrt_eps = 1.4901161193847656e-08;
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    int nd = 0;
    if (active[c]) {
      const double n1 = nrm1[c].x;
      const double bj = msc[c] * sqrt(n1 > 0.0 ? n1 : 0.0);
      const double aj = alpha[(int64_t)(j - 1) * ncol + c];
      const double bjm1 = j > 1 ? beta[(int64_t)(j - 2) * ncol + c] : 0.0;
      double an = fmax(pro.anorm[c], fabs(aj) + bj + bjm1);
      pro.anorm[c] = an;
      // rows by Lanczos index modulo 3: omega_j (cur), omega_{j-1} (old), omega_{j+1} (new)
      const double *cur = pro.om + (int64_t)((j % 3) * pro.ld) * ncol + c;
      const double *old = pro.om + (int64_t)(((j + 2) % 3) * pro.ld) * ncol + c;
      double *nw = pro.om + (int64_t)(((j + 1) % 3) * pro.ld) * ncol + c;
      double mx = 0.0;
      if (bj > 0.0) {
        for (int k = 1; k < j; ++k) {
          const double ojk1 = k + 1 == j ? 1.0 : cur[(int64_t)k * ncol];
          double t = beta[(int64_t)(k - 1) * ncol + c] * ojk1 +
                     (alpha[(int64_t)(k - 1) * ncol + c] - aj) * cur[(int64_t)(k - 1) * ncol];
          if (k > 1) t += beta[(int64_t)(k - 2) * ncol + c] * cur[(int64_t)(k - 2) * ncol];
          const double ojm1 = k == j - 1 ? 1.0 : old[(int64_t)(k - 1) * ncol];
          t -= bjm1 * ojm1;
          t += copysign(2.0 * eps * an, t);
          const double o = t / bj;
          nw[(int64_t)(k - 1) * ncol] = o;
          mx = fmax(mx, fabs(o));
        }
        nw[(int64_t)(j - 1) * ncol] = eps * an / bj;
      } else {
        for (int k = 1; k <= j; ++k) nw[(int64_t)(k - 1) * ncol] = 0.0;
      }
      nw[(int64_t)j * ncol] = 1.0;
      const int exceed = (j > 1 && mx > sqrt_eps) ? 1 : 0;
      // cancellation: ||w'|| < eta ||w|| (the update's input had unit norm unless rel)
      const double lim = kReorthEta * kReorthEta * (rel ? nrm1[c].y : 1.0);
      nd = (bj > 0.0 && (exceed || pro.force[c] || n1 < lim)) ? 1 : 0;
      if (nd)
        for (int k = 1; k <= j; ++k) nw[(int64_t)(k - 1) * ncol] = eps;
      pro.force[c] = exceed;
    }
    need[c] = nd;
    if (nd) atomicOr(&flag, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *any = flag;
}

// Daniel-Gragg-Kaufman-Stewart test: the first pass loses at most
// eps ||w|| / ||w'|| of orthogonality, so a second pass is made only for
// columns where it cancelled most of w (||w'|| < kReorthEta ||w||; the slot was
// scaled to ||w|| = 1).
__global__ void k_lz_decide(const double2 *__restrict__ nrm1, int ncol, const int *__restrict__ active,
                            const double *__restrict__ gsc, int *__restrict__ need, int *__restrict__ any) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    const int nd = (active[c] && gsc[c] > 0.0 && nrm1[c].x < kReorthEta * kReorthEta) ? 1 : 0;
    need[c] = nd;
    if (nd) atomicOr(&flag, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *any = flag;
}

// Second pass: h2[l][c] = <slot_l, slot_j>; slot_j <- g2 (slot_j - sum_l sig_l^2 h2[l] slot_l)
// with g2 = 1 / ||slot_j||.
__global__ void k_lz_coef2(const double2 *__restrict__ h2, const double2 *__restrict__ nrm1,
                           const double *__restrict__ sig, int j, int ncol, const int *__restrict__ need,
                           double2 *__restrict__ coef, double *__restrict__ gsc, double *__restrict__ msc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol || !need[c]) return;
  const double n1 = nrm1[c].x;
  const double g2 = n1 > 0.0 ? 1.0 / sqrt(n1) : 0.0;
  for (int l = 0; l < j; ++l) {
    const double s = sig[(int64_t)l * ncol + c];
    const double f = g2 * s * s;
    const double2 v = h2[(int64_t)l * ncol + c];
    coef[(int64_t)l * ncol + c] = make_double2(f * v.x, f * v.y);
  }
  gsc[c] = g2;
  msc[c] = g2 > 0.0 ? msc[c] / g2 : 0.0;
}

// beta_j = msc ||slot_j||, sig_j = 1 / ||slot_j||.
__global__ void k_lz_beta(const double2 *__restrict__ nrm1, const double2 *__restrict__ nrm2,
                          const int *__restrict__ need, const int *__restrict__ active, const double *__restrict__ msc,
                          int j, int ncol, double *__restrict__ beta_j, double *__restrict__ sig) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol || !active[c]) return;
  const double n2 = need[c] ? nrm2[c].x : nrm1[c].x;
  const double nr = sqrt(n2 > 0.0 ? n2 : 0.0);
  beta_j[c] = msc[c] * nr;
  sig[(int64_t)j * ncol + c] = nr > 0.0 ? 1.0 / nr : 0.0;
}

// coef[l][c] = beta0 sig_l u_l for l < kused[c], else 0  (u from the tridiagonal exponential)
__global__ void k_lz_comb_coef(const double *__restrict__ u, const double *__restrict__ sig,
                               const double *__restrict__ beta0, const int *__restrict__ kused, int kmax, int nl,
                               int ncol, double2 *__restrict__ coef) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nl * ncol) return;
  const int l = t / ncol, c = t % ncol;
  double2 v = make_double2(0.0, 0.0);
  if (l < kused[c]) {
    const double f = beta0[c] * sig[(int64_t)l * ncol + c];
    v.x = f * u[((int64_t)c * kmax + l) * 2];
    v.y = f * u[((int64_t)c * kmax + l) * 2 + 1];
  }
  coef[t] = v;
}

__global__ void k_lz_kmax(const int *__restrict__ kused, int ncol, int *__restrict__ kmaxu) {
  __shared__ int m;
  if (threadIdx.x == 0) m = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) atomicMax(&m, kused[c]);
  __syncthreads();
  if (threadIdx.x == 0) *kmaxu = m;
}

__global__ void k_lz_any(const int *__restrict__ active, int ncol, int *__restrict__ any) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x)
    if (active[c]) atomicOr(&flag, 1);
  __syncthreads();
  if (threadIdx.x == 0) *any = flag;
}

// X (packed FP64, ncolr values per row) -> Xf (FP32, ldf values per row; pad columns zero)
__global__ void __launch_bounds__(256)
k_to_f32(const double *__restrict__ X, int64_t nrows, int ncolr, float *__restrict__ Xf, int64_t ldf) {
  const int64_t n = nrows * ldf;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ldf;
    const int c = (int)(i - r * ldf);
    Xf[i] = c < ncolr ? (float)X[r * ncolr + c] : 0.f;
  }
}

// Xf (FP32, ldf values per row) -> X (packed FP64)
__global__ void __launch_bounds__(256)
k_from_f32(const float *__restrict__ Xf, int64_t ldf, int64_t nrows, int ncolr, double *__restrict__ X) {
  const int64_t n = nrows * (int64_t)ncolr;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ncolr;
    X[i] = (double)Xf[r * ldf + (i - r * ncolr)];
  }
}

inline int lz_grid(int64_t nrows, int ncol, int threads) {
  const int R = threads / ncol;
  const int64_t need = (nrows + R - 1) / R;
  return (int)std::max<int64_t>(1, std::min<int64_t>(kLzBlocks, need));
}

template <typename W2>
int lz_dots_t(const double *q0, const double *qb, int64_t bs, int nq, const W2 *w, int64_t wld, int64_t nrows,
              int ncol, const int *mask, const int *any, int with_norm, double *part, hipStream_t s) {
  const Basis B{(const double2 *)q0, (const double2 *)qb, bs / 2};
  const int nb = lz_grid(nrows, ncol, kLzThreads);
  const int nvtot = nq + (with_norm ? 1 : 0);
  if (nq == 0) {
    hipLaunchKernelGGL((k_lz_dots<1, W2>), dim3(nb), dim3(kLzThreads), 0, s, B, 0, 0, w, wld, nrows, ncol, mask, any,
                       with_norm, nvtot, (double2 *)part);
    return nb;
  }
  for (int l0 = 0; l0 < nq; l0 += kLzChunk) {
    const int nl = std::min(kLzChunk, nq - l0);
    const int wn = (l0 + nl == nq) ? with_norm : 0;
    if (nl <= 4)
      hipLaunchKernelGGL((k_lz_dots<4, W2>), dim3(nb), dim3(kLzThreads), 0, s, B, l0, nl, w, wld, nrows, ncol, mask,
                         any, wn, nvtot, (double2 *)part);
    else if (nl <= 8)
      hipLaunchKernelGGL((k_lz_dots<8, W2>), dim3(nb), dim3(kLzThreads), 0, s, B, l0, nl, w, wld, nrows, ncol, mask,
                         any, wn, nvtot, (double2 *)part);
    else
      hipLaunchKernelGGL((k_lz_dots<kLzChunk, W2>), dim3(nb), dim3(kLzThreads), 0, s, B, l0, nl, w, wld, nrows, ncol,
                         mask, any, wn, nvtot, (double2 *)part);
  }
  return nb;
}

template <typename S2, bool INPLACE, typename SHT>
void lz_update_launch(int nl, int nb, size_t lds, hipStream_t s, const Basis &B, int l0, const double *coef,
                      const double *g, const S2 *src, int64_t sld, double *w, SHT *shc, int64_t shld,
                      int64_t nrows, int ncol, const int *mask, const int *any, int wn, int zm, double *part) {
  if (nl <= 4)
    hipLaunchKernelGGL((k_lz_update<4, S2, INPLACE, SHT>), dim3(nb), dim3(kLzUpdThreads), lds, s, B, l0, nl,
                       (const double2 *)coef, g, src, sld, (double2 *)w, shc, shld, nrows, ncol, mask, any, wn, zm,
                       (double2 *)part);
  else if (nl <= 8)
    hipLaunchKernelGGL((k_lz_update<8, S2, INPLACE, SHT>), dim3(nb), dim3(kLzUpdThreads), lds, s, B, l0, nl,
                       (const double2 *)coef, g, src, sld, (double2 *)w, shc, shld, nrows, ncol, mask, any, wn, zm,
                       (double2 *)part);
  else
    hipLaunchKernelGGL((k_lz_update<kLzChunk, S2, INPLACE, SHT>), dim3(nb), dim3(kLzUpdThreads), lds, s, B, l0, nl,
                       (const double2 *)coef, g, src, sld, (double2 *)w, shc, shld, nrows, ncol, mask, any, wn, zm,
                       (double2 *)part);
}

// src == nullptr: in place on w; sh: the reduced-precision copy (SHT float or Bf16) or nullptr
template <typename S2, typename SHT>
int lz_update_t(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, const double *gw,
                const S2 *src, int64_t sld, double *w, SHT *sh, int64_t shld, int64_t nrows, int ncol,
                const int *mask, const int *any, double *part, hipStream_t s, int zero_masked) {
  const Basis B{(const double2 *)q0, (const double2 *)qb, bs / 2};
  const int nb = lz_grid(nrows, ncol, kLzUpdThreads);
  const size_t lds = ((size_t)kLzChunk * ncol + kLzUpdThreads) * sizeof(double2);
  for (int l0 = 0; l0 < nq; l0 += kLzChunk) {
    const int nl = std::min(kLzChunk, nq - l0);
    const bool last = l0 + nl == nq;
    const int wn = last ? 1 : 0;
    const double *g = l0 == 0 ? gw : nullptr;
    SHT *shc = last ? sh : nullptr;
    // the first chunk reads src; later chunks continue in place on w
    if (l0 == 0 && src)
      lz_update_launch<S2, false, SHT>(nl, nb, lds, s, B, l0, coef, g, src, sld, w, shc, shld, nrows, ncol, mask, any,
                                       wn, zero_masked, part);
    else
      lz_update_launch<double2, true, SHT>(nl, nb, lds, s, B, l0, coef, g, nullptr, 0, w, shc, shld, nrows, ncol,
                                           mask, any, wn, l0 == 0 ? zero_masked : 0, part);
  }
  return nb;
}

// X (packed FP64, ncolr values per row) -> Xs (FP32 or BF16, ldf values per row; pad columns zero)
// (one row per 64-lane group of a 256-thread block; rows of up to 64 lanes x 4 elements)
template <typename SHT>
__global__ void __launch_bounds__(256)
k_to_shadow(const double *__restrict__ X, int64_t nrows, int ncolr, SHT *__restrict__ Xs, int64_t ldf) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nrows; r += (int64_t)gridDim.x * 4)
    for (int c = lane; c < ldf; c += 64) Xs[r * ldf + c] = narrow<SHT>(c < ncolr ? X[r * ncolr + c] : 0.0);
}

}  // namespace

namespace k {

int lz_dots(const double *q0, const double *qb, int64_t bs, int nq, const double *w, int64_t nrows, int ncol,
            const int *mask, const int *any, int with_norm, double *part, hipStream_t s) {
  return lz_dots_t(q0, qb, bs, nq, (const double2 *)w, (int64_t)ncol, nrows, ncol, mask, any, with_norm, part, s);
}

int lz_dots_f(const double *q0, const double *qb, int64_t bs, int nq, const float *w, int64_t ldf, int64_t nrows,
              int ncol, const int *mask, const int *any, int with_norm, double *part, hipStream_t s) {
  return lz_dots_t(q0, qb, bs, nq, (const float2 *)w, ldf / 2, nrows, ncol, mask, any, with_norm, part, s);
}

int lz_update(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, const double *gw, double *w,
              int64_t nrows, int ncol, const int *mask, const int *any, double *part, hipStream_t s, int zero_masked,
              void *sh, int64_t shld, int sh_bf16) {
  if (sh && sh_bf16)
    return lz_update_t(q0, qb, bs, nq, coef, gw, (const double2 *)nullptr, 0, w, (Bf16 *)sh, shld / 2, nrows, ncol,
                       mask, any, part, s, zero_masked);
  return lz_update_t(q0, qb, bs, nq, coef, gw, (const double2 *)nullptr, 0, w, (float *)sh, shld / 2, nrows, ncol,
                     mask, any, part, s, zero_masked);
}

int lz_update_from(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, const double *gw,
                   const float *src, int64_t ldf, double *w, void *sh, int sh_bf16, int64_t nrows, int ncol,
                   const int *mask, const int *any, double *part, hipStream_t s, int zero_masked) {
  if (sh_bf16)
    return lz_update_t(q0, qb, bs, nq, coef, gw, (const float2 *)src, ldf / 2, w, (Bf16 *)sh, ldf / 2, nrows, ncol,
                       mask, any, part, s, zero_masked);
  return lz_update_t(q0, qb, bs, nq, coef, gw, (const float2 *)src, ldf / 2, w, (float *)sh, ldf / 2, nrows, ncol,
                     mask, any, part, s, zero_masked);
}

void to_shadow(const double *X, int64_t nrows, int ncolr, void *Xs, int64_t ldf, int bf16, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>((nrows + 3) / 4, 8192);
  if (bf16) hipLaunchKernelGGL(k_to_shadow<Bf16>, dim3(nb), dim3(256), 0, s, X, nrows, ncolr, (Bf16 *)Xs, ldf);
  else hipLaunchKernelGGL(k_to_shadow<float>, dim3(nb), dim3(256), 0, s, X, nrows, ncolr, (float *)Xs, ldf);
}

void to_f32(const double *X, int64_t nrows, int ncolr, float *Xf, int64_t ldf, hipStream_t s) {
  const int64_t n = nrows * (int64_t)ncolr;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, s, X, nrows, ncolr, Xf, ldf);
}

void from_f32(const float *Xf, int64_t ldf, int64_t nrows, int ncolr, double *X, hipStream_t s) {
  const int64_t n = nrows * (int64_t)ncolr;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_from_f32, dim3(nb), dim3(256), 0, s, Xf, ldf, nrows, ncolr, X);
}

void lz_combine(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, double *out,
                int64_t nrows, int ncol, hipStream_t s, const int *nq_dev) {
  const Basis B{(const double2 *)q0, (const double2 *)qb, bs / 2};
  const int nb = lz_grid(nrows, ncol, kLzUpdThreads);
  const size_t lds = (size_t)kLzChunk * ncol * sizeof(double2);
  if (nq == 0) {
    zero(out, nrows * ncol * 2, s);
    return;
  }
  for (int l0 = 0; l0 < nq; l0 += kLzChunk) {
    const int nl = std::min(kLzChunk, nq - l0);
    const int acc = l0 > 0 ? 1 : 0;
    if (nl <= 4)
      hipLaunchKernelGGL(k_lz_combine<4>, dim3(nb), dim3(kLzUpdThreads), lds, s, B, l0, nl, (const double2 *)coef,
                         (double2 *)out, nrows, ncol, acc, nq_dev);
    else if (nl <= 8)
      hipLaunchKernelGGL(k_lz_combine<8>, dim3(nb), dim3(kLzUpdThreads), lds, s, B, l0, nl, (const double2 *)coef,
                         (double2 *)out, nrows, ncol, acc, nq_dev);
    else
      hipLaunchKernelGGL(k_lz_combine<kLzChunk>, dim3(nb), dim3(kLzUpdThreads), lds, s, B, l0, nl,
                         (const double2 *)coef, (double2 *)out, nrows, ncol, acc, nq_dev);
  }
}

void lz_init(const double *h0, int ncol, double *beta0, double *sig, int *active, int *kused, const ProState &pro,
             hipStream_t s) {
  hipLaunchKernelGGL(k_lz_init, dim3((ncol + 63) / 64), dim3(64), 0, s, (const double2 *)h0, ncol, beta0, sig, active,
                     kused, pro);
}

void lz_coef1(const double *h, const double *sig, int j, int first, int ncol, const int *active, double *alpha_j,
              double *coef, double *gsc, double *msc, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_coef1, dim3((ncol + 63) / 64), dim3(64), 0, s, (const double2 *)h, sig, j, first, ncol,
                     active, alpha_j, (double2 *)coef, gsc, msc);
}

void lz_coef3(const double *h, const double *sig, const double *beta, int j, int ncol, const int *active,
              double *alpha_j, double *coef, double *gsc, double *msc, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_coef3, dim3((ncol + 63) / 64), dim3(64), 0, s, (const double2 *)h, sig, beta, j, ncol,
                     active, alpha_j, (double2 *)coef, gsc, msc);
}

void lz_pro(const double *nrm1, const double *msc, const double *alpha, const double *beta, int j, int ncol,
            const int *active, const ProState &pro, int *need, int *any, hipStream_t s, int rel) {
  hipLaunchKernelGGL(k_lz_pro, dim3(1), dim3(128), 0, s, (const double2 *)nrm1, msc, alpha, beta, j, ncol, active, pro,
                     need, any, rel);
}

void lz_alpha_coef3(const double *apart, int nparts, const double *aE, int nk, double *lvl, const double *sig,
                    const double *beta, int j, int ncol, const int *active, const int *any, double *alpha_j,
                    double *coef, double *gsc, double *msc, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_alpha_sum, dim3(2 * ncol, kAlphaSlices), dim3(256), 0, s, apart, nparts, aE, nk, 2 * ncol,
                     any, lvl);
  hipLaunchKernelGGL(k_lz_coef3x, dim3((ncol + 63) / 64), dim3(64), 0, s, lvl, sig, beta, j, ncol, active, alpha_j,
                     (double2 *)coef, gsc, msc);
}

void lz_decide(const double *nrm1, int ncol, const int *active, const double *gsc, int *need, int *any,
               hipStream_t s) {
  hipLaunchKernelGGL(k_lz_decide, dim3(1), dim3(128), 0, s, (const double2 *)nrm1, ncol, active, gsc, need, any);
}

void lz_coef2(const double *h2, const double *nrm1, const double *sig, int j, int ncol, const int *need, double *coef,
              double *gsc, double *msc, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_coef2, dim3((ncol + 63) / 64), dim3(64), 0, s, (const double2 *)h2, (const double2 *)nrm1,
                     sig, j, ncol, need, (double2 *)coef, gsc, msc);
}

void lz_beta(const double *nrm1, const double *nrm2, const int *need, const int *active, const double *msc, int j,
             int ncol, double *beta_j, double *sig, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_beta, dim3((ncol + 63) / 64), dim3(64), 0, s, (const double2 *)nrm1, (const double2 *)nrm2,
                     need, active, msc, j, ncol, beta_j, sig);
}

void lz_kmax(const int *kused, int ncol, int *kmaxu, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_kmax, dim3(1), dim3(128), 0, s, kused, ncol, kmaxu);
}

void lz_any(const int *active, int ncol, int *any, hipStream_t s) {
  hipLaunchKernelGGL(k_lz_any, dim3(1), dim3(128), 0, s, active, ncol, any);
}

void lz_comb_coef(const double *u, const double *sig, const double *beta0, const int *kused, int kmax, int nl,
                  int ncol, double *coef, hipStream_t s) {
  const int n = nl * ncol;
  hipLaunchKernelGGL(k_lz_comb_coef, dim3((n + 255) / 256), dim3(256), 0, s, u, sig, beta0, kused, kmax, nl, ncol,
                     (double2 *)coef);
}

}  // namespace k
}  // namespace efe
