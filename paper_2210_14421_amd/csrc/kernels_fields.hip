// HIP kernels for the time-dependent fields of the Magnus step:
//   rebuild of the Loewdin cell blocks  Hbar_c = D_c^-1/2 (1/2 K_c + B^T diag(W v) B) D_c^-1/2
//   enrichment coupling  H^ce_{i nu} = int 1/2 grad N_i . grad N^E + v N_i N^E  (and H^ee)
//   density at quadrature points, Poisson right-hand side, stiffness and
//   fast-diagonalisation operators, dipole.
// Sec. 2.1-2.3 of the paper (eqs. (Hmn), (TDKSDiscrete2), (DiscretePoisson)).
#include <hip/hip_runtime.h>

#include "common.h"
#include "plan.h"

namespace efe {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}

// Stored forms of the cell blocks: FP64 / FP32 rows of nloc elements; BF16 rows
// padded to a multiple of 8 elements (one plane), or a hi/lo pair of BF16 planes
// (hi = bf16(v), lo = bf16(v - hi)).  The padding columns are zero from set-up.
struct Bf16Rows { uint16_t v; };
struct Bf16Split { uint16_t v; };
template <typename T> struct Store {
  static constexpr int planes = 1;
  static constexpr bool padded = false;
  static __device__ __forceinline__ void put(T *o, int64_t i, int64_t, double v) { o[i] = (T)v; }
};
template <> struct Store<Bf16Rows> {
  static constexpr int planes = 1;
  static constexpr bool padded = true;
  static __device__ __forceinline__ void put(Bf16Rows *o, int64_t i, int64_t, double v) {
    ((uint16_t *)o)[i] = f32_to_bf16((float)v);
  }
};
template <> struct Store<Bf16Split> {
  static constexpr int planes = 2;
  static constexpr bool padded = true;
  static __device__ __forceinline__ void put(Bf16Split *o, int64_t i, int64_t plane, double v) {
    const float f = (float)v;
    const uint16_t h = f32_to_bf16(f);
    ((uint16_t *)o)[i] = h;
    ((uint16_t *)o)[i + plane] = f32_to_bf16(f - __uint_as_float((uint32_t)h << 16));
  }
};

// ---------------------------------------------------------------------------
// Cell-block rebuild.  One workgroup per cell of one class (all cells of a
// launch share the Gauss rule size n).  The potential part
//   V[(a,b,c),(a',b',c')] = sum_ijk W v(i,j,k) B_i(a)B_i(a') B_j(b)B_j(b') B_k(c)B_k(c')
// depends on the unordered pairs {a,a'}, {b,b'}, {c,c'} only, and is built by
// three contractions over the pair tables G1[i][pair] = B_i(a) B_i(a'): over i
// once for all (k, j), then per z-pair over k and over j, so that no n x NP x NP
// intermediate is held (LDS within 160 KB up to degree 6 with 14 Gauss points).
// mode 0: Hamiltonian (kinetic + v_static + v_H + v_xc - E x_dir); mode 1..3:
// position operator along x/y/z (v = x_d, no kinetic term).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_rebuild(const DevData d, const int *__restrict__ cell_list, int n, int mode, const double *__restrict__ rho,
          const double *__restrict__ phi, const double *__restrict__ efield_p, int fdir, int xc, T *__restrict__ cells,
          double *__restrict__ vq) {
  extern __shared__ double sm[];
  const Geom &g = d.g;
  const int P = g.P, P2 = P * P, nloc = g.nloc, NP = P * (P + 1) / 2;
  const int n3 = n * n * n;
  const bool enr = n == g.qe && g.qe != g.qc ? true : (n == g.qe);
  const double *tab = d.tab;
  double *Bt = sm;                       // n*P
  double *G1 = Bt + n * P;               // n*NP
  double *Kel = G1 + n * NP;             // 3*P2
  double *Mel = Kel + 3 * P2;            // 3*P2
  double *dm = Mel + 3 * P2;             // nloc
  double *wv = dm + nloc;                // n3
  // U: n*n*NP, or the Hartree interpolation's u0, t1, t2 (nloc + P2*n + n*n*P) if larger
  const int usz = n * n * NP > nloc + P2 * n + n * n * P ? n * n * NP : nloc + P2 * n + n * n * P;
  double *U = wv + n3;
  double *Z = U + usz;                   // n*NP
  double *Vc = Z + n * NP;               // NP*NP
  int *pair = (int *)(Vc + NP * NP);     // P2 ints
  double *u0 = U, *t1 = U + nloc, *t2 = t1 + P2 * n;

  const int64_t cell = cell_list[blockIdx.x];
  int e[3];
  cell_ijk(g, cell, e);
  const int toB = enr ? d.to.Be : d.to.Bc, toG = enr ? d.to.G1e : d.to.G1c;
  const int tox = enr ? d.to.xqe : d.to.xqc, tow = enr ? d.to.wqe : d.to.wqc;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) Bt[t] = tab[toB + t];
  for (int t = threadIdx.x; t < n * NP; t += blockDim.x) G1[t] = tab[toG + t];
  double clo[3], ch[3];
  cell_box(d, e, clo, ch);
  for (int t = threadIdx.x; t < 3 * P2; t += blockDim.x) {
    Kel[t] = tab[d.to.Kr + t % P2] * (2.0 / ch[t / P2]);
    Mel[t] = tab[d.to.Mr + t % P2] * (0.5 * ch[t / P2]);
  }
  for (int t = threadIdx.x; t < P2; t += blockDim.x) pair[t] = (int)tab[d.to.pair + t];
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) {
    int64_t node = local_node(g, e, t);
    dm[t] = d.Dm12[node];
    if (mode == 0) u0[t] = phi[node];
  }
  __syncthreads();
  const int64_t q0 = d.q_off[cell];
  if (mode == 0) {
    apply_axis(u0, t1, Bt, P, false, P, P, P, 0, n, 1);      // [c][b][i]
    __syncthreads();
    apply_axis(t1, t2, Bt, P, false, n, P, P, 1, n, 1);      // [c][j][i]
    __syncthreads();
    apply_axis(t2, wv, Bt, P, false, n, n, P, 2, n, 1);      // [k][j][i] = v_H
    __syncthreads();
  }
  const double jac = 0.125 * ch[0] * ch[1] * ch[2];
  const double efield = efield_p ? *efield_p : 0.0;
  for (int q = threadIdx.x; q < n3; q += blockDim.x) {
    int i = q % n, j = (q / n) % n, k = q / (n * n);
    double x[3] = {clo[0] + (tab[tox + i] + 1.0) * 0.5 * ch[0],
                   clo[1] + (tab[tox + j] + 1.0) * 0.5 * ch[1],
                   clo[2] + (tab[tox + k] + 1.0) * 0.5 * ch[2]};
    double w = jac * tab[tow + i] * tab[tow + j] * tab[tow + k];
    double v;
    if (mode == 0) {
      v = d.vstatic[q0 + q] + wv[q] + vxc_lda(rho[q0 + q], xc) - efield * x[fdir];
    } else if (mode == 4) {
      v = rho[q0 + q];                 // potential-only operator of a given g(q)
    } else {
      v = x[mode - 1];
    }
    vq[q0 + q] = v;
    wv[q] = w * v;
  }
  if (!cells) return;   // sum-factorised products: the potential at the points is all they read
  __syncthreads();
  // U[k][j][pa] = sum_i wv[k][j][i] G1[i][pa]
  for (int t = threadIdx.x; t < n * n * NP; t += blockDim.x) {
    int pa = t % NP, kj = t / NP;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += wv[kj * n + i] * G1[i * NP + pa];
    U[t] = s;
  }
  __syncthreads();
  // colour-major storage
  const int64_t lda = Store<T>::padded ? (int64_t)((nloc + 7) & ~7) : (int64_t)nloc;
  const int64_t plane = Store<T>::padded ? (int64_t)nloc * lda : d.g.cstride;
  T *out = cells + (int64_t)d.cell_slot[cell] * Store<T>::planes * plane;
  for (int c = 0; c < P; ++c)
    for (int c2 = c; c2 < P; ++c2) {
      const int pc = pair[c * P + c2];
      // Z[j][pa] = sum_k G1[k][pc] U[k][j][pa]
      for (int t = threadIdx.x; t < n * NP; t += blockDim.x) {
        const int pa = t % NP, j = t / NP;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += G1[k * NP + pc] * U[(k * n + j) * NP + pa];
        Z[t] = s;
      }
      __syncthreads();
      // Vc[pb][pa] = sum_j G1[j][pb] Z[j][pa]
      for (int t = threadIdx.x; t < NP * NP; t += blockDim.x) {
        const int pa = t % NP, pb = t / NP;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += G1[j * NP + pb] * Z[j * NP + pa];
        Vc[t] = s;
      }
      __syncthreads();
      for (int t = threadIdx.x; t < P2 * P2; t += blockDim.x) {
        int rp = t / P2, cp = t % P2;
        int a = rp % P, b = rp / P, a2 = cp % P, b2 = cp / P;
        double val = Vc[pair[b * P + b2] * NP + pair[a * P + a2]];
        if (mode == 0) {
          val += 0.5 * (Kel[0 * P2 + a * P + a2] * Mel[1 * P2 + b * P + b2] * Mel[2 * P2 + c * P + c2] +
                        Mel[0 * P2 + a * P + a2] * Kel[1 * P2 + b * P + b2] * Mel[2 * P2 + c * P + c2] +
                        Mel[0 * P2 + a * P + a2] * Mel[1 * P2 + b * P + b2] * Kel[2 * P2 + c * P + c2]);
        }
        int row = rp + P2 * c, col = cp + P2 * c2;
        Store<T>::put(out, (int64_t)row * lda + col, plane, dm[row] * val * dm[col]);
        if (c2 != c) {
          int row2 = rp + P2 * c2, col2 = cp + P2 * c;
          Store<T>::put(out, (int64_t)row2 * lda + col2, plane, dm[row2] * val * dm[col2]);
        }
      }
      __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Enrichment coupling, per T-cell (a cell where some N^E is nonzero):
//   part[slot][l][nu_local] = sum_q W v N_l(q) N^E_nu(q)
//   hee_part[slot][mu_local][nu_local] = sum_q W v N^E_mu N^E_nu
// ---------------------------------------------------------------------------
template <bool HEE>
__global__ void __launch_bounds__(kThreads)
k_coupling_partials(const DevData d, const double *__restrict__ vq, double *__restrict__ part,
                    double *__restrict__ hee_part) {
  extern __shared__ double sm[];
  const Geom &g = d.g;
  const int slot = blockIdx.x;
  const int64_t cell = d.tcell[slot];
  const bool enr = d.is_enr[cell] != 0;
  const int n = enr ? g.qe : g.qc, n3 = n * n * n, P = g.P, nloc = g.nloc;
  const double *tab = d.tab;
  const int toB = enr ? d.to.Be : d.to.Bc, tow = enr ? d.to.wqe : d.to.wqc;
  double *Bt = sm;             // n*P
  double *wv = Bt + n * P;     // n3
  double *f = wv + n3;         // n3
  double *t1 = f + n3;         // n*n*P
  double *t2 = t1 + n * n * P; // n*P*P
  double *nod = t2 + n * P * P;  // nloc
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) Bt[t] = tab[toB + t];
  const int64_t q0 = d.q_off[cell];
  const double jac = cell_jacobian(d, cell);
  for (int q = threadIdx.x; q < n3; q += blockDim.x) {
    int i = q % n, j = (q / n) % n, k = q / (n * n);
    wv[q] = jac * tab[tow + i] * tab[tow + j] * tab[tow + k] * vq[q0 + q];
  }
  __syncthreads();
  const int k0 = d.tnu_off[slot], k1 = d.tnu_off[slot + 1], nnu = k1 - k0;
  const double *NEs = d.NE + d.tne_off[slot];
  double *ps = part + d.tpart_off[slot];
  double *hs = hee_part + d.thee_off[slot];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int kk = 0; kk < nnu; ++kk) {
    const double *ne = NEs + (int64_t)kk * n3;
    for (int q = threadIdx.x; q < n3; q += blockDim.x) f[q] = wv[q] * ne[q];
    __syncthreads();
    apply_axis(f, t1, Bt, P, true, n, n, n, 0, P, 1);     // [k][j][a]
    __syncthreads();
    apply_axis(t1, t2, Bt, P, true, P, n, n, 1, P, 1);    // [k][b][a]
    __syncthreads();
    apply_axis(t2, nod, Bt, P, true, P, P, n, 2, P, 1);   // [c][b][a]
    // H^ee partial row kk: one wave per mu
    for (int mm = wid; HEE && mm < nnu; mm += nw) {
      const double *nm = NEs + (int64_t)mm * n3;
      double s = 0.0;
      for (int q = lane; q < n3; q += 64) s += f[q] * nm[q];
      s = wave_sum(s);
      if (lane == 0) hs[kk * nnu + mm] = s;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < nloc; l += blockDim.x) ps[(int64_t)l * nnu + kk] = nod[l];
    __syncthreads();
  }
}

// The same partial sums on the FP64 16x16x4 MFMA, one workgroup of 4 waves per
// T-cell, the points streamed through LDS in chunks of 64:
//   part[l][nu] = sum_q B_l(q) F(q, nu),   F(q, nu) = W_q v(q) N^E_nu(q)
//     (A operand B_l(q) = b(i_q, a_l) b(j_q, b_l) b(k_q, c_l) from the 1-D table;
//      wave w takes the M tiles w + 4 i, i < MT, of the nloc node rows, all N
//      tiles: MT = 4 covers nloc <= 256, MT = 6 nloc <= 384);
//   hee[mu][nu] = sum_q N^E_mu(q) F(q, nu)  (the 3 x 3 tiles of 48 functions
//      dealt round-robin to the waves).
constexpr int kCpChunk = 64;
typedef double v4d_t __attribute__((ext_vector_type(4)));

template <int MT, bool PART>
__global__ void __launch_bounds__(256)
k_coupling_mfma(const DevData d, const double *__restrict__ vq, double *__restrict__ part,
                double *__restrict__ hee_part) {
  __shared__ double bt[16 * 8];                       // n x P (n <= 16, P <= 8)
  __shared__ double wq[kCpChunk];
  __shared__ int qoff[kCpChunk];                      // bt row offsets of the point's (i, j, k), packed
  __shared__ double nec[48][kCpChunk + 1];
  const Geom &g = d.g;
  const int slot = blockIdx.x;
  const int64_t cell = d.tcell[slot];
  const bool enr = d.is_enr[cell] != 0;
  const int n = enr ? g.qe : g.qc, n3 = n * n * n, P = g.P, nloc = g.nloc;
  const double *tab = d.tab;
  const int toB = enr ? d.to.Be : d.to.Bc, tow = enr ? d.to.wqe : d.to.wqc;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) bt[t] = tab[toB + t];
  const int k0 = d.tnu_off[slot], nnu = d.tnu_off[slot + 1] - k0;
  const double *NEs = d.NE + d.tne_off[slot];
  const int64_t q0 = d.q_off[cell];
  const double jac = cell_jacobian(d, cell);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane >> 4, cl = lane & 15;
  const int nmt = (nloc + 15) / 16, nnt = (nnu + 15) / 16;
  // node index decomposition of this lane's rows in each of its M tiles
  int la[MT], lb[MT], lc[MT];
  bool lok[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int l = (wave + 4 * i) * 16 + cl;
    lok[i] = wave + 4 * i < nmt && l < nloc;
    la[i] = l % P;
    lb[i] = (l / P) % P;
    lc[i] = l / (P * P);
  }
  v4d_t acc[MT][3], acch[3];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[i][j] = v4d_t{0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < 3; ++j) acch[j] = v4d_t{0, 0, 0, 0};
  for (int qc = 0; qc < n3; qc += kCpChunk) {
    __syncthreads();
    for (int t = threadIdx.x; t < kCpChunk; t += blockDim.x) {
      const int q = qc + t;
      double v = 0.0;
      int off = 0;
      if (q < n3) {
        const int i = q % n, j = (q / n) % n, k = q / (n * n);
        v = jac * tab[tow + i] * tab[tow + j] * tab[tow + k] * vq[q0 + q];
        off = (i * P) | ((j * P) << 8) | ((k * P) << 16);
      }
      wq[t] = v;
      qoff[t] = off;
    }
    for (int t = threadIdx.x; t < 48 * kCpChunk; t += blockDim.x) {
      const int kk = t / kCpChunk, qq = t % kCpChunk;
      nec[kk][qq] = (kk < nnu && qc + qq < n3) ? NEs[(int64_t)kk * n3 + qc + qq] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int s4 = 0; s4 < kCpChunk / 4; ++s4) {
      const int qq = s4 * 4 + kr, q = qc + qq;
      const bool qok = q < n3;
      const int qo = qoff[qq];
      const int oi = qo & 255, oj = (qo >> 8) & 255, ok = qo >> 16;
      const double w = wq[qq];
      double bv[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) bv[j] = w * nec[j * 16 + cl][qq];        // F(q, nu)
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        if (!PART || wave + 4 * i >= nmt) continue;
        const double a = (qok && lok[i]) ? bt[oi + la[i]] * bt[oj + lb[i]] * bt[ok + lc[i]] : 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (j < nnt) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[j], acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int u = wave + 4 * j;             // tile (u / 3, u % 3) of hee
        if (u >= nnt * nnt) continue;
        const int mt = u / nnt, nt = u % nnt;
        const double a = nec[mt * 16 + cl][qq];
        const double b = w * nec[nt * 16 + cl][qq];
        acch[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acch[j], 0, 0, 0);
      }
    }
  }
  double *ps = part + d.tpart_off[slot];
  double *hs = hee_part + d.thee_off[slot];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    if (!PART || wave + 4 * i >= nmt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int l = (wave + 4 * i) * 16 + kr + 4 * r;
      if (l >= nloc) continue;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int kk = j * 16 + cl;
        if (j < nnt && kk < nnu) ps[(int64_t)l * nnu + kk] = acc[i][j][r];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int u = wave + 4 * j;
    if (u >= nnt * nnt) continue;
    const int mt = u / nnt, nt = u % nnt;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = mt * 16 + kr + 4 * r, nu = nt * 16 + cl;
      if (mu < nnu && nu < nnu) hs[mu * nnu + nu] = acch[j][r];
    }
  }
}

// G[r][kappa] = D^-1/2_r sum_nu (Kce[r][nu] + sum_cells part) S[nu][kappa]  (Hbar^ce rows)
// G[r][kp] = D_r^-1/2 sum_nu a[r][nu] S[nu][kp] with a[r][nu] = Kce[r][nu] (kinetic)
// + the partials of the T-cells that contain the node of union row r, on the
// FP64 16x16x4 MFMA: one wave per block walks a contiguous range of 16-row
// tiles for 48 columns of G (blockIdx.y).  Lane (row i, k) forms its entries
// of the A tile a[r0 + i][4 s + k] from the row's cell pairs (at most 8).
constexpr int kGatherWaves = 4096;

template <typename GT>
__global__ void __launch_bounds__(64)
k_coupling_gather(const DevData d, const double *__restrict__ part, int kinetic, GT *__restrict__ G,
                  int64_t tiles_per_wave) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  const int ne = d.ne, nk = d.nk;
  const int64_t nr = d.nr;
  const int lane = threadIdx.x, kr = lane >> 4, cl = lane & 15;
  const int n0 = blockIdx.y * 48;
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_wave;
  const int64_t t_end = t_begin + tiles_per_wave < ntiles ? t_begin + tiles_per_wave : ntiles;
  const int nks = (ne + 3) / 4;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t r0 = t * 16, ra = r0 + cl;
    const bool rok = ra < nr;
    // the row's (slot, local node) pairs: base offset of the partials and the slot
    int cnt = rok ? d.urow_cnt[ra] : 0;
    int slot[8];
    int64_t base[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      slot[p] = 0;
      base[p] = 0;
      if (p < cnt) {
        const int pr = d.urow_pair[ra * 8 + p];
        const int sl = pr >> kPairShift, l = pr & ((1 << kPairShift) - 1);
        const int nnu = d.tnu_off[sl + 1] - d.tnu_off[sl];
        slot[p] = sl;
        base[p] = d.tpart_off[sl] + (int64_t)l * nnu;
      }
    }
    v4d acc[3];
#pragma unroll
    for (int nt = 0; nt < 3; ++nt) acc[nt] = v4d{0, 0, 0, 0};
    for (int ks = 0; ks < nks; ++ks) {
      const int nu = ks * 4 + kr;
      double a = 0.0;
      if (rok && nu < ne) {
        a = kinetic ? d.Kce[ra * ne + nu] : 0.0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          if (p < cnt) {
            const int pos = d.tpos[(int64_t)slot[p] * ne + nu];
            if (pos >= 0) a += part[base[p] + pos];
          }
        }
      }
#pragma unroll
      for (int nt = 0; nt < 3; ++nt) {
        const int kp = n0 + nt * 16 + cl;
        const double bv = (nu < ne && kp < nk) ? d.S[nu * nk + kp] : 0.0;
        acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[nt], 0, 0, 0);
      }
    }
    // output register r of a lane holds row kr + 4 r, column cl
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + kr + 4 * r;
      if (row >= nr) continue;
      const double dm = d.Dm12[d.urow_node[row]];
#pragma unroll
      for (int nt = 0; nt < 3; ++nt) {
        const int kp = n0 + nt * 16 + cl;
        if (kp < nk) G[row * nk + kp] = (GT)(dm * acc[nt][r]);
      }
    }
  }
}

// H^ee partial sums over contiguous ranges of T-cell slots: workgroup b adds the
// nnu x nnu partials of its slots, one slot after another, into an LDS copy of
// the ne x ne matrix (the entries of one slot are distinct) and writes it as
// blk[b]; k_hee_sum adds the blocks in order.
constexpr int kHeeBlocks = 64;

__global__ void __launch_bounds__(256)
k_hee_blocks(const DevData d, const double *__restrict__ hee_part, double *__restrict__ blk) {
  extern __shared__ double hacc[];
  const int ne = d.ne, ne2 = ne * ne;
  for (int t = threadIdx.x; t < ne2; t += blockDim.x) hacc[t] = 0.0;
  const int per = (d.nt + gridDim.x - 1) / gridDim.x;
  const int s0 = blockIdx.x * per, s1 = s0 + per < d.nt ? s0 + per : d.nt;
  __syncthreads();
  for (int sl = s0; sl < s1; ++sl) {
    const int k0 = d.tnu_off[sl], nnu = d.tnu_off[sl + 1] - k0;
    const double *hp = hee_part + d.thee_off[sl];
    for (int t = threadIdx.x; t < nnu * nnu; t += blockDim.x) {
      const int i = t / nnu, j = t % nnu;
      hacc[d.tnu[k0 + i] * ne + d.tnu[k0 + j]] += hp[t];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < ne2; t += blockDim.x) blk[(int64_t)blockIdx.x * ne2 + t] = hacc[t];
}

// H^ee = Kee + the block sums of k_hee_blocks (fixed order)
__global__ void k_hee_sum(const DevData d, const double *__restrict__ blk, int nblk, int kinetic,
                          double *__restrict__ Hraw) {
  const int ne2 = d.ne * d.ne;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne2) return;
  double s = kinetic ? d.Kee[t] : 0.0;
  for (int b = 0; b < nblk; ++b) s += blk[(int64_t)b * ne2 + t];
  Hraw[t] = s;
}

// Hbar^ee = S^T H^ee S in two products: T = H^ee S (ne x nk), then S^T T
__global__ void k_hee_hs(const DevData d, const double *__restrict__ Hraw, double *__restrict__ T) {
  const int ne = d.ne, nk = d.nk;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne * nk) return;
  const int mu = t / nk, b = t % nk;
  double s = 0.0;
  for (int nu = 0; nu < ne; ++nu) s += Hraw[mu * ne + nu] * d.S[nu * nk + b];
  T[t] = s;
}

__global__ void k_hee_loewdin(const DevData d, const double *__restrict__ T, double *__restrict__ Hbar) {
  const int ne = d.ne, nk = d.nk;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nk * nk) return;
  const int a = t / nk, b = t % nk;
  double s = 0.0;
  for (int mu = 0; mu < ne; ++mu) s += d.S[mu * nk + a] * T[mu * nk + b];
  Hbar[t] = s;
}

// ---------------------------------------------------------------------------
// Density rho(q) = sum_a f_a |psi_a(q)|^2, psi = sum_i D_i^-1/2 X_i N_i + sum_nu psiE_nu N^E_nu.
// One workgroup per cell of one class; columns in passes of NCC complex orbitals.
// ---------------------------------------------------------------------------
// CROSS: the block holds column pairs (a, b); out(q) += wcross * sum_pairs Im(conj(a(q)) b(q))
template <int NCC, int MAXS, bool CROSS = false>
__global__ void __launch_bounds__(kThreads)
k_density(const DevData d, const int *__restrict__ cell_list, int n, const double *__restrict__ X, int ncol,
          int64_t ldr, const double *__restrict__ psiE, double *__restrict__ rho, double wcross) {
  extern __shared__ double sm[];
  constexpr int F = 2 * NCC;
  const Geom &g = d.g;
  const int P = g.P, nloc = g.nloc, n3 = n * n * n;
  const bool enr = (n == g.qe);
  const double *tab = d.tab;
  double *Bt = sm;                    // n*P
  double *dm = Bt + n * P;            // nloc
  double *u = dm + nloc;              // nloc*F
  double *t1 = u + nloc * F;          // P*P*n*F
  double *t2 = t1 + P * P * n * F;    // P*n*n*F
  double *occ = t2 + P * n * n * F;   // ncol
  const int64_t cell = cell_list[blockIdx.x];
  int e[3];
  cell_ijk(g, cell, e);
  const int toB = enr ? d.to.Be : d.to.Bc;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) Bt[t] = tab[toB + t];
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) dm[t] = d.Dm12[local_node(g, e, t)];
  if (!CROSS)
    for (int t = threadIdx.x; t < ncol; t += blockDim.x) occ[t] = d.occ[t];
  const int slot = d.tslot_of_cell[cell];
  const int k0 = slot >= 0 ? d.tnu_off[slot] : 0, nnu = slot >= 0 ? d.tnu_off[slot + 1] - k0 : 0;
  const double *NEs = slot >= 0 ? d.NE + d.tne_off[slot] : nullptr;
  double acc[MAXS];
#pragma unroll
  for (int s = 0; s < MAXS; ++s) acc[s] = 0.0;
  const int ncolr = 2 * ncol;
  __syncthreads();
  for (int c0 = 0; c0 < ncol; c0 += NCC) {
    for (int t = threadIdx.x; t < nloc * F; t += blockDim.x) {
      int l = t / F, f = t % F;
      int col = 2 * c0 + f;
      u[t] = col < ncolr ? dm[l] * X[local_node(g, e, l) * ldr + col] : 0.0;
    }
    __syncthreads();
    apply_axis(u, t1, Bt, P, false, P, P, P, 0, n, F);      // [c][b][i][f]
    __syncthreads();
    apply_axis(t1, t2, Bt, P, false, n, P, P, 1, n, F);     // [c][j][i][f]
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      int q = threadIdx.x + s * kThreads;
      if (q < n3) {
        int ji = q % (n * n), k = q / (n * n);
        double val[F];
#pragma unroll
        for (int f = 0; f < F; ++f) val[f] = 0.0;
        for (int c = 0; c < P; ++c) {
          double bk = Bt[k * P + c];
#pragma unroll
          for (int f = 0; f < F; ++f) val[f] += bk * t2[(c * n * n + ji) * F + f];
        }
        for (int kk = 0; kk < nnu; ++kk) {
          double nev = NEs[(int64_t)kk * n3 + q];
          const double *pe = psiE + (int64_t)d.tnu[k0 + kk] * ncolr + 2 * c0;
#pragma unroll
          for (int f = 0; f < F; ++f)
            if (2 * c0 + f < ncolr) val[f] += nev * pe[f];
        }
        if (CROSS) {
#pragma unroll
          for (int cc = 0; cc + 1 < NCC; cc += 2)
            if (c0 + cc + 1 < ncol) acc[s] += val[2 * cc] * val[2 * cc + 3] - val[2 * cc + 1] * val[2 * cc + 2];
        } else {
#pragma unroll
          for (int cc = 0; cc < NCC; ++cc)
            if (c0 + cc < ncol) acc[s] += occ[c0 + cc] * (val[2 * cc] * val[2 * cc] + val[2 * cc + 1] * val[2 * cc + 1]);
        }
      }
    }
    __syncthreads();
  }
  const int64_t q0 = d.q_off[cell];
#pragma unroll
  for (int s = 0; s < MAXS; ++s) {
    int q = threadIdx.x + s * kThreads;
    if (q < n3) {
      if (CROSS) rho[q0 + q] += wcross * acc[s];
      else rho[q0 + q] = acc[s];
    }
  }
}

// Density (or cross density) on cells whose Gauss rule has P points per axis
// (the ordinary cells): the three interpolation stages run in place on a
// nloc x 44 LDS tile of columns (each thread owns whole lines), two passes for
// 88 columns; the enrichment part adds sum_nu N^E_nu(q) psiE[nu] per point.
constexpr int kDenCols = 44;

template <bool CROSS>
__global__ void __launch_bounds__(kThreads)
k_density_sq(const DevData d, const int *__restrict__ cell_list, const double *__restrict__ X, int ncol, int64_t ldr,
             const double *__restrict__ psiE, double *__restrict__ rho, double wcross) {
  extern __shared__ double sm[];
  const Geom &g = d.g;
  const int P = g.P, nloc = g.nloc;
  const double *tab = d.tab;
  double *Bt = sm;                 // P*P
  double *dm = Bt + P * P;         // nloc
  double *occ = dm + nloc;         // 128
  double *u = occ + 128;           // nloc * kDenCols
  const int64_t cell = cell_list[blockIdx.x];
  int e[3];
  cell_ijk(g, cell, e);
  for (int t = threadIdx.x; t < P * P; t += blockDim.x) Bt[t] = tab[d.to.Bc + t];
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) dm[t] = d.Dm12[local_node(g, e, t)];
  if (!CROSS)
    for (int t = threadIdx.x; t < ncol; t += blockDim.x) occ[t] = d.occ[t];
  const int slot = d.tslot_of_cell[cell];
  const int k0 = slot >= 0 ? d.tnu_off[slot] : 0, nnu = slot >= 0 ? d.tnu_off[slot + 1] - k0 : 0;
  const double *NEs = slot >= 0 ? d.NE + d.tne_off[slot] : nullptr;
  const int ncolr = 2 * ncol;
  double acc[2] = {0.0, 0.0};       // points threadIdx.x and threadIdx.x + kThreads (nloc <= 512)
  __syncthreads();
  for (int col0 = 0; col0 < ncolr; col0 += kDenCols) {
    const int w = ncolr - col0 < kDenCols ? ncolr - col0 : kDenCols;
    for (int t = threadIdx.x; t < nloc * kDenCols; t += blockDim.x) {
      const int l = t / kDenCols, f = t % kDenCols;
      u[t] = f < w ? dm[l] * X[local_node(g, e, l) * ldr + col0 + f] : 0.0;
    }
    __syncthreads();
    const int nline = nloc / P;
    for (int ax = 0; ax < 3; ++ax) {
      const int stride = ax == 0 ? 1 : (ax == 1 ? P : P * P);
      for (int t = threadIdx.x; t < nline * kDenCols; t += blockDim.x) {
        const int L = t / kDenCols, f = t % kDenCols;
        const int base = ax == 0 ? L * P : (ax == 1 ? (L % P) + (L / P) * P * P : L);
        double in[8];
        for (int j = 0; j < P; ++j) in[j] = u[(base + j * stride) * kDenCols + f];
        for (int i = 0; i < P; ++i) {
          double v = 0.0;
          for (int j = 0; j < P; ++j) v += Bt[i * P + j] * in[j];
          u[(base + i * stride) * kDenCols + f] = v;
        }
      }
      __syncthreads();
    }
    for (int h = 0; h < 2; ++h) {
      const int q = threadIdx.x + h * kThreads;
      if (q >= nloc) continue;
      double val[kDenCols];
#pragma unroll
      for (int f = 0; f < kDenCols; ++f) val[f] = u[q * kDenCols + f];
      for (int kk = 0; kk < nnu; ++kk) {
        const double nev = NEs[(int64_t)kk * nloc + q];
        const double *pe = psiE + (int64_t)d.tnu[k0 + kk] * ncolr + col0;
#pragma unroll
        for (int f = 0; f < kDenCols; ++f)
          if (f < w) val[f] += nev * pe[f];
      }
      double a = 0.0;
      if (CROSS) {
#pragma unroll
        for (int f = 0; f + 3 < kDenCols; f += 4)
          if (f + 3 < w) a += val[f] * val[f + 3] - val[f + 1] * val[f + 2];
      } else {
#pragma unroll
        for (int f = 0; f + 1 < kDenCols; f += 2)
          if (f + 1 < w) a += occ[(col0 + f) / 2] * (val[f] * val[f] + val[f + 1] * val[f + 1]);
      }
      acc[h] += a;
    }
    __syncthreads();
  }
  const int64_t q0 = d.q_off[cell];
  for (int h = 0; h < 2; ++h) {
    const int q = threadIdx.x + h * kThreads;
    if (q >= nloc) continue;
    if (CROSS) rho[q0 + q] += wcross * acc[h];
    else rho[q0 + q] = acc[h];
  }
}

// ---------------------------------------------------------------------------
// Density through folded nodal values.  The orthogonalised enrichment function
// is N^E_nu = s_nu N^A_nu - sum_i c_{i nu} N_i (Sec. 2.2), so
//   psi(q) = sum_i N_i(q) u_i + sum_{nu atomic on the cell} s_nu N^A_nu(q) psiE_nu,
//   u_i = D_i^-1/2 X_i - sum_nu c_{i nu} psiE_nu.
// The correction of u is nonzero on the union rows only: k_fold_rows writes
// those rows into U (n_R x ncolr); every other node reads D^-1/2 X.  The
// ordinary cells then need no enrichment term at all, and the enrichment
// cells only the atomic parts (stored once, at their points).
// ---------------------------------------------------------------------------
// U = D^-1/2 X[R] - C psiE on the FP64 16x16x4 MFMA: one wave per block walks
// a contiguous range of 16-row tiles of R for 96 columns (blockIdx.y);
// A(i, k) = C[r0 + i][k], B(k, j) = psiE[k][j], the epilogue adds the scaled rows.
constexpr int kFoldWaves = 4096;
constexpr int kFoldNT = 6;

__global__ void __launch_bounds__(64)
k_fold_rows(const DevData d, const double *__restrict__ X, int ncolr, int64_t ldr, const double *__restrict__ psiE,
            double *__restrict__ U, int64_t tiles_per_wave) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  const int ne = d.ne;
  const int64_t nr = d.nr;
  const int lane = threadIdx.x, kr = lane >> 4, cl = lane & 15;
  const int n0 = blockIdx.y * kFoldNT * 16;
  const int64_t ntiles = (nr + 15) / 16;
  const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_wave;
  const int64_t t_end = t_begin + tiles_per_wave < ntiles ? t_begin + tiles_per_wave : ntiles;
  int col[kFoldNT];
  bool cok[kFoldNT];
#pragma unroll
  for (int nt = 0; nt < kFoldNT; ++nt) {
    col[nt] = n0 + nt * 16 + cl;
    cok[nt] = col[nt] < ncolr;
  }
  const int nks = (ne + 3) / 4;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t r0 = t * 16;
    v4d acc[kFoldNT];
#pragma unroll
    for (int nt = 0; nt < kFoldNT; ++nt) acc[nt] = v4d{0, 0, 0, 0};
    const int64_t ra = r0 + cl;
    const bool rok = ra < nr;
    for (int ks = 0; ks < nks; ++ks) {
      const int k = ks * 4 + kr;
      const bool kok = k < ne;
      const double a = (rok && kok) ? d.C[ra * ne + k] : 0.0;
#pragma unroll
      for (int nt = 0; nt < kFoldNT; ++nt) {
        const double bv = (kok && cok[nt]) ? psiE[(int64_t)k * ncolr + col[nt]] : 0.0;
        acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[nt], 0, 0, 0);
      }
    }
    // output register r of a lane holds row kr + 4 r, column cl
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + kr + 4 * r;
      if (row >= nr) continue;
      const int64_t node = d.urow_node[row];
      const double dm = d.Dm12[node];
      const double *xr = X + node * ldr;
      double *ur = U + row * ncolr;
#pragma unroll
      for (int nt = 0; nt < kFoldNT; ++nt)
        if (cok[nt]) ur[col[nt]] = dm * xr[col[nt]] - acc[nt][r];
    }
  }
}

// Density (or cross density) on the cells of one class, NP = P GLL nodes and N
// Gauss points per axis, sum-factorised in passes of F = 8 NFG columns.
//   stage X:  items (c, b, f) load the x-line of folded nodal values and
//             interpolate it to t1[c][b][i][f] (LDS, row stride FS);
//   stage YZ: lanes (j, i, fg) contract t1 along y into t2[c][f] for their 8
//             columns (registers), then along z to the N points (i, j, k), add
//             the atomic part, and sum occupation-weighted squares (or the
//             cross term) over their columns; the NFG lanes of one (j, i) are
//             adjacent and are reduced by shuffles.
// INWG: one workgroup per cell loops over the passes and keeps the point sums
// in registers.  Otherwise one workgroup per (cell, pass) writes a partial
// per pass (part[pass][cell index][q], summed by k_den_sum).  Workgroup b runs
// on XCD b mod 8; each XCD takes a contiguous chunk of the cell list and the
// passes of a cell are consecutive workgroups there, so the cell's atomic
// values and the nodes it shares with its neighbours come from L2 after the
// first read.
// CROSS: the columns hold pairs (a, b); the point value is sum Im(conj(a) b).
template <int NP, int N, int NFG, bool INWG, bool CROSS>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_den(const DevData d, const int *__restrict__ cell_list, int ncells, const double *__restrict__ X, int ncol,
      int64_t ldr, const double *__restrict__ U, const double *__restrict__ psiE, double *__restrict__ out,
      double *__restrict__ part, int npass, double wcross) {
  constexpr int F = 8 * NFG, F2 = F / 2, FS = F + 2, NL = NP * NP * NP, N3 = N * N * N;
  constexpr int NITEM = NP * NP * F2, NIT = (NITEM + kThreads - 1) / kThreads;
  constexpr int kMaxA = 48;
  __shared__ double Bt[N * NP];
  __shared__ __attribute__((aligned(16))) double t1[NP * NP * N * FS];
  __shared__ __attribute__((aligned(16))) double psA[INWG ? 2 : kMaxA * F];
  __shared__ int64_t loff[NL];
  __shared__ double lsc[NL];   // D^-1/2 of the node, or 1 where the value comes from U
  __shared__ int lur[NL];
  __shared__ double locc[CROSS ? 1 : 128];
  const Geom &g = d.g;
  const int tid = threadIdx.x;
  const int ncolr = 2 * ncol;
  if (!CROSS)
    for (int t = tid; t < 128; t += kThreads) locc[t] = t < ncol ? d.occ[t] : 0.0;
  int ci, pass0, pass1;
  if (INWG) {
    ci = blockIdx.x;
    pass0 = 0;
    pass1 = npass;
  } else {
    // XCD x takes the cells [x chunk, (x + 1) chunk) of the list (neighbours share nodes in L2)
    const int b = blockIdx.x, xcd = b & 7, sl = b >> 3, chunk = (ncells + 7) / 8;
    const int cl = sl / npass;
    ci = xcd * chunk + cl;
    pass0 = sl % npass;
    pass1 = pass0 + 1;
    if (cl >= chunk || ci >= ncells) return;
  }
  const int64_t cell = cell_list[ci];
  int e[3];
  cell_ijk(g, cell, e);
  const int toB = N == NP ? d.to.Bc : d.to.Be;
  for (int t = tid; t < N * NP; t += kThreads) Bt[t] = d.tab[toB + t];
  for (int l = tid; l < NL; l += kThreads) {
    const int64_t node = local_node(g, e, l);
    const int ur = d.nr > 0 ? d.node_urow[node] : -1;
    loff[l] = node * ldr;
    lur[l] = ur;
    lsc[l] = ur >= 0 ? 1.0 : d.Dm12[node];
  }
  int na = 0;
  const double *NAc = nullptr;
  int ta0 = 0;
  if (!INWG) {
    const int slot = d.tslot_of_cell[cell];
    if (slot >= 0) {
      ta0 = d.ta_off[slot];
      na = d.ta_off[slot + 1] - ta0;
      NAc = d.NA + d.tna_off[slot];
    }
  }
  // stage-YZ lane
  const int fg = tid % NFG, ij = tid / NFG, jj = ij / N, ii = ij % N;
  (void)NL;
  const bool yz = ij < N * N;
  double acc[INWG ? N : 1];
#pragma unroll
  for (int k = 0; k < (INWG ? N : 1); ++k) acc[k] = 0.0;
  __syncthreads();
  double Bj[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) Bj[b] = yz ? Bt[jj * NP + b] : 0.0;
  for (int pass = pass0; pass < pass1; ++pass) {
    const int c0 = pass * F;
    if (!INWG)
      for (int t = tid; t < ((na + 7) & ~7) * F; t += kThreads) {
        const int a = t / F, f = t % F;
        psA[t] = (a < na && c0 + f < ncolr) ? psiE[(int64_t)d.ta_nu[ta0 + a] * ncolr + c0 + f] : 0.0;
      }
    // stage X: items (c b, column pair); every load of the thread first
    double2 u[NIT][NP];
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int it = tid + r * kThreads;
      const int cb = it / F2, col = c0 + 2 * (it % F2);
      const bool ok = it < NITEM && col < ncolr;
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        const int l = a + NP * cb;
        double2 v = make_double2(0.0, 0.0);
        if (ok) {
          const int ur = lur[l];
          const double *src = ur >= 0 ? U + (int64_t)ur * ncolr + col : X + loff[l] + col;
          v = *(const double2 *)src;
        }
        u[r][a] = v;
      }
    }
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int it = tid + r * kThreads;
      if (it >= NITEM) continue;
      const int cb = it / F2, h = it % F2;
      double sc[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) sc[a] = lsc[a + NP * cb];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          const double bb = Bt[i * NP + a] * sc[a];
          v.x += bb * u[r][a].x;
          v.y += bb * u[r][a].y;
        }
        *(double2 *)(t1 + (cb * N + i) * FS + 2 * h) = v;
        __builtin_amdgcn_sched_barrier(0);   // keeps the table reads of one point at a time in registers
      }
    }
    __syncthreads();
    if (yz) {
      double t2[NP][8];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
#pragma unroll
        for (int f = 0; f < 8; ++f) t2[c][f] = 0.0;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          const double2 *src = (const double2 *)(t1 + ((c * NP + b) * N + ii) * FS + fg * 8);
#pragma unroll
          for (int f2 = 0; f2 < 4; ++f2) {
            const double2 x = src[f2];
            t2[c][2 * f2] += Bj[b] * x.x;
            t2[c][2 * f2 + 1] += Bj[b] * x.y;
          }
          // without the fence the scheduler hoists all NP^2 row reads (8 NP^2 registers)
          if (b & 1) __builtin_amdgcn_sched_barrier(0);
        }
      }
      // weights of the lane's four complex columns (occupations, or 1 per complete pair)
      const int cc0 = (c0 + fg * 8) / 2;
      double w[4];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int cc = cc0 + o;
        if (CROSS) w[o] = (o % 2 == 0 && cc + 1 < ncol) ? 1.0 : 0.0;
        else w[o] = locc[cc < 128 ? cc : 127];
      }
      auto point = [&](int k) -> double {
        double v[8];
#pragma unroll
        for (int f = 0; f < 8; ++f) v[f] = 0.0;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          const double bk = Bt[k * NP + c];
#pragma unroll
          for (int f = 0; f < 8; ++f) v[f] += bk * t2[c][f];
        }
        if (NAc) {
          // atomic values in groups of eight loads in flight (psA rows past na are zero)
          const int q = ii + N * (jj + N * k);
          for (int a0 = 0; a0 < na; a0 += 8) {
            double av[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) av[u] = NAc[(int64_t)(a0 + u < na ? a0 + u : a0) * N3 + q];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const double2 *ps = (const double2 *)(psA + (a0 + u) * F + fg * 8);
#pragma unroll
              for (int f2 = 0; f2 < 4; ++f2) {
                const double2 x = ps[f2];
                v[2 * f2] += av[u] * x.x;
                v[2 * f2 + 1] += av[u] * x.y;
              }
            }
          }
        }
        double r = 0.0;
        if (CROSS) {
#pragma unroll
          for (int pp = 0; pp < 2; ++pp) r += w[2 * pp] * (v[4 * pp] * v[4 * pp + 3] - v[4 * pp + 1] * v[4 * pp + 2]);
        } else {
#pragma unroll
          for (int o = 0; o < 4; ++o) r += w[o] * (v[2 * o] * v[2 * o] + v[2 * o + 1] * v[2 * o + 1]);
        }
        return r;
      };
      if (INWG) {
#pragma unroll
        for (int k = 0; k < (INWG ? N : 1); ++k) acc[k] += point(k);
      } else {
        // the NFG lanes of (j, i) are adjacent and all inside this branch
        double *pp = part + ((int64_t)pass * ncells + ci) * N3 + ii + N * jj;
#pragma unroll 1
        for (int k = 0; k < N; ++k) {
          double r = point(k);
#pragma unroll
          for (int m = 1; m < NFG; m <<= 1) r += __shfl_xor(r, m);
          if (fg == 0) pp[N * N * k] = r;
        }
      }
    }
    __syncthreads();
  }
  if (INWG) {
#pragma unroll
    for (int k = 0; k < (INWG ? N : 1); ++k) {
#pragma unroll
      for (int m = 1; m < NFG; m <<= 1) acc[k] += __shfl_xor(acc[k], m);
    }
    if (yz && fg == 0) {
      const int64_t q0 = d.q_off[cell];
#pragma unroll
      for (int k = 0; k < (INWG ? N : 1); ++k) {
        const int64_t q = q0 + ii + N * (jj + N * k);
        if (CROSS) out[q] += wcross * acc[k];
        else out[q] = acc[k];
      }
    }
  }
}

// out[q] = sum over passes of the partials (fixed order), or += w * that sum
template <bool CROSS>
__global__ void k_den_sum(const DevData d, const int *__restrict__ cell_list, int ncells, int n3,
                          const double *__restrict__ part, int npass, double *__restrict__ out, double wcross) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)ncells * n3;
  if (t >= tot) return;
  const int ci = (int)(t / n3), q = (int)(t - (int64_t)ci * n3);
  double s = 0.0;
  for (int p = 0; p < npass; ++p) s += part[p * tot + t];
  const int64_t o = d.q_off[cell_list[ci]] + q;
  if (CROSS) out[o] += wcross * s;
  else out[o] = s;
}

// psiE[nu][col] = sum_kappa S[nu][kappa] X[n_nodes + kappa][col]
__global__ void k_psiE(const DevData d, const double *__restrict__ X, int ncolr, int64_t ldr, double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.ne * ncolr) return;
  const int nu = t / ncolr, col = t % ncolr;
  double s = 0.0;
  for (int k = 0; k < d.nk; ++k) s += d.S[nu * d.nk + k] * X[(d.g.n_nodes + k) * ldr + col];
  out[t] = s;
}

// ---------------------------------------------------------------------------
// Poisson right-hand side d_i = int rho N_i, one colour of cells per launch
// (cells of one colour share no node, so the scatter needs no atomics).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_poisson_rhs(const DevData d, const int *__restrict__ cell_list, const double *__restrict__ rho, double *__restrict__ dvec) {
  extern __shared__ double sm[];
  const Geom &g = d.g;
  const int64_t cell = cell_list[blockIdx.x];
  const bool enr = d.is_enr[cell] != 0;
  const int n = enr ? g.qe : g.qc, n3 = n * n * n, P = g.P, nloc = g.nloc;
  const double *tab = d.tab;
  const int toB = enr ? d.to.Be : d.to.Bc, tow = enr ? d.to.wqe : d.to.wqc;
  double *Bt = sm, *f = Bt + n * P, *t1 = f + n3, *t2 = t1 + n * n * P, *nod = t2 + n * P * P;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) Bt[t] = tab[toB + t];
  const int64_t q0 = d.q_off[cell];
  const double jac = cell_jacobian(d, cell);
  for (int q = threadIdx.x; q < n3; q += blockDim.x) {
    int i = q % n, j = (q / n) % n, k = q / (n * n);
    f[q] = jac * tab[tow + i] * tab[tow + j] * tab[tow + k] * rho[q0 + q];
  }
  __syncthreads();
  apply_axis(f, t1, Bt, P, true, n, n, n, 0, P, 1);
  __syncthreads();
  apply_axis(t1, t2, Bt, P, true, P, n, n, 1, P, 1);
  __syncthreads();
  apply_axis(t2, nod, Bt, P, true, P, P, n, 2, P, 1);
  __syncthreads();
  int e[3];
  cell_ijk(g, cell, e);
  for (int l = threadIdx.x; l < nloc; l += blockDim.x) dvec[local_node(g, e, l)] += nod[l];
}

// rhs = 4 pi d - lift on interior nodes, 0 on the boundary
__global__ void k_rhs_finish(const DevData d, const double *__restrict__ dvec, double *__restrict__ rhs, int lift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.g.n_nodes) return;
  rhs[i] = d.Dm12[i] != 0.0 ? 4.0 * 3.14159265358979323846 * dvec[i] - (lift ? d.lift[i] : 0.0) : 0.0;
}

// Adjoint potential at the quadrature points of one cell per block:
//   out(q) = (B phibar)(q) + tau f_xc(rho(q)) u(q) + mubar . x(q) + a gin(q)
// (B phibar: the nodal field interpolated to the points; gin may be null).
__global__ void __launch_bounds__(kThreads)
k_adj_potential(const DevData d, const int *__restrict__ cell_list, int n, const double *__restrict__ phibar,
                const double *__restrict__ rho, const double *__restrict__ u, double tau, int xc, double mx, double my,
                double mz, double a, const double *__restrict__ gin, double *__restrict__ out) {
  extern __shared__ double sm[];
  const Geom &g = d.g;
  const int P = g.P, nloc = g.nloc, n3 = n * n * n;
  const bool enr = n == g.qe;
  const double *tab = d.tab;
  double *Bt = sm;                 // n*P
  double *u0 = Bt + n * P;         // nloc
  double *t1 = u0 + nloc;          // P*P*n
  double *t2 = t1 + P * P * n;     // P*n*n
  double *wv = t2 + P * n * n;     // n3
  const int64_t cell = cell_list[blockIdx.x];
  int e[3];
  cell_ijk(g, cell, e);
  const int toB = enr ? d.to.Be : d.to.Bc, tox = enr ? d.to.xqe : d.to.xqc;
  for (int t = threadIdx.x; t < n * P; t += blockDim.x) Bt[t] = tab[toB + t];
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) u0[t] = phibar[local_node(g, e, t)];
  __syncthreads();
  apply_axis(u0, t1, Bt, P, false, P, P, P, 0, n, 1);
  __syncthreads();
  apply_axis(t1, t2, Bt, P, false, n, P, P, 1, n, 1);
  __syncthreads();
  apply_axis(t2, wv, Bt, P, false, n, n, P, 2, n, 1);
  __syncthreads();
  const int64_t q0 = d.q_off[cell];
  double clo[3], ch[3];
  cell_box(d, e, clo, ch);
  for (int q = threadIdx.x; q < n3; q += blockDim.x) {
    const int i = q % n, j = (q / n) % n, k = q / (n * n);
    const double x = clo[0] + (tab[tox + i] + 1.0) * 0.5 * ch[0];
    const double y = clo[1] + (tab[tox + j] + 1.0) * 0.5 * ch[1];
    const double z = clo[2] + (tab[tox + k] + 1.0) * 0.5 * ch[2];
    double v = wv[q] + tau * fxc_lda(rho[q0 + q], xc) * u[q0 + q] + mx * x + my * y + mz * z;
    if (gin) v += a * gin[q0 + q];
    out[q0 + q] = v;
  }
}

// out[r][c] += s[c % ncs] * Y[r][c]  over complex columns (s real; ncs = orbitals)
__global__ void k_axpy_cols(double *__restrict__ out, const double *__restrict__ Y, const double *__restrict__ sc,
                            double s0, int64_t nrows, int ncol) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncol) return;
  const int c = (int)(t % ncol);
  const double f = sc ? s0 * sc[c] : s0;
  out[2 * t] += f * Y[2 * t];
  out[2 * t + 1] += f * Y[2 * t + 1];
}

// Z[r][2c] = a[r][c], Z[r][2c + 1] = b[r][c]  (complex columns)
__global__ void k_interleave(const double2 *__restrict__ a, const double2 *__restrict__ b, double2 *__restrict__ Z,
                             int64_t nrows, int ncol) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncol) return;
  const int64_t r = t / ncol;
  const int c = (int)(t % ncol);
  Z[r * 2 * ncol + 2 * c] = a[t];
  Z[r * 2 * ncol + 2 * c + 1] = b[t];
}

// out = A_axis in (banded 1-D operator, bandwidth p), over all nodes
__global__ void k_axis_band(const DevData d, const double *__restrict__ A, int axis, const double *__restrict__ in,
                            double *__restrict__ out, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const Geom &g = d.g;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_nodes) return;
  int64_t gg[3] = {i % g.nn[0], (i / g.nn[0]) % g.nn[1], i / (g.nn[0] * g.nn[1])};
  const int64_t n = g.nn[axis], gi = gg[axis];
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? g.nn[0] : g.nn[0] * g.nn[1]);
  const int64_t lo = gi - g.p < 0 ? 0 : gi - g.p, hi = gi + g.p > n - 1 ? n - 1 : gi + g.p;
  double s = 0.0;
  for (int64_t k = lo; k <= hi; ++k) s += A[gi * n + k] * in[i + (k - gi) * stride];
  out[i] = s;
}

// y (+)= x on interior nodes; boundary of y zeroed
__global__ void k_interior_acc(const DevData d, const double *__restrict__ x, double *__restrict__ y, int accumulate,
                               const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.g.n_nodes) return;
  double v = d.Dm12[i] != 0.0 ? x[i] : 0.0;
  y[i] = accumulate ? y[i] + v : v;
}

// fast diagonalisation transform along one axis on interior nodes:
// fwd: out_i = sum_a V[a][i] in_a ; back: out_a = sum_i V[a][i] in_i (V: m x m, m = nn - 2)
__global__ void k_fdm_axis(const DevData d, const double *__restrict__ V, int axis, int back,
                           const double *__restrict__ in, double *__restrict__ out, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const Geom &g = d.g;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_nodes) return;
  int64_t gg[3] = {i % g.nn[0], (i / g.nn[0]) % g.nn[1], i / (g.nn[0] * g.nn[1])};
  if (d.Dm12[i] == 0.0) { out[i] = 0.0; return; }
  const int64_t m = g.nn[axis] - 2, o = gg[axis] - 1;
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? g.nn[0] : g.nn[0] * g.nn[1]);
  const double *base = in + i - gg[axis] * stride;   // node with coordinate 0 along axis
  double s = 0.0;
  if (back) {
    for (int64_t k = 0; k < m; ++k) s += V[o * m + k] * base[(k + 1) * stride];
  } else {
    for (int64_t k = 0; k < m; ++k) s += V[k * m + o] * base[(k + 1) * stride];
  }
  out[i] = s;
}

// The same transform on 16 interior lines per workgroup (lines along `axis` at 16 consecutive
// values of the fastest other coordinate u and one value of the slowest v): the lines pass
// through LDS, each thread forms one output o of all 16 lines from the coalesced row W[k][.]
// (W = V for the forward transform, V^T for the back one), and the results leave through LDS.
// For m <= kFdmMaxM; only interior nodes are written.
constexpr int kFdmLines = 16, kFdmMaxM = 256;

__global__ void __launch_bounds__(kFdmMaxM)
k_fdm_lines(const DevData d, const double *__restrict__ W, int axis, const double *__restrict__ in,
            double *__restrict__ out, const int *__restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double tile[kFdmLines][kFdmMaxM + 1];
  const Geom &g = d.g;
  const int m = (int)g.nn[axis] - 2;
  const int au = axis == 0 ? 1 : 0, av = axis == 2 ? 1 : 2;      // the other axes, u fastest
  const int nu = (int)g.nn[au] - 2;
  const int u0 = 1 + kFdmLines * blockIdx.x, v = 1 + blockIdx.y;
  const int64_t st[3] = {1, g.nn[0], g.nn[0] * g.nn[1]};
  const int64_t base = u0 * st[au] + (int64_t)v * st[av];
  const int tid = threadIdx.x;
  // consecutive threads take consecutive addresses: along the line for axis 0, across lines otherwise
  auto at = [&](int idx, int &ln, int &kk) {
    if (axis == 0) { ln = idx / m; kk = idx - ln * m; }
    else { ln = idx % kFdmLines; kk = idx / kFdmLines; }
  };
  for (int idx = tid; idx < kFdmLines * m; idx += kFdmMaxM) {
    int ln, kk;
    at(idx, ln, kk);
    tile[ln][kk] = u0 + ln <= nu ? in[base + ln * st[au] + (int64_t)(kk + 1) * st[axis]] : 0.0;
  }
  __syncthreads();
  double acc[kFdmLines];
#pragma unroll
  for (int l = 0; l < kFdmLines; ++l) acc[l] = 0.0;
  if (tid < m) {
    for (int k = 0; k < m; ++k) {
      const double w = W[(int64_t)k * m + tid];
#pragma unroll
      for (int l = 0; l < kFdmLines; ++l) acc[l] += w * tile[l][k];
    }
  }
  __syncthreads();
  if (tid < m)
#pragma unroll
    for (int l = 0; l < kFdmLines; ++l) tile[l][tid] = acc[l];
  __syncthreads();
  for (int idx = tid; idx < kFdmLines * m; idx += kFdmMaxM) {
    int ln, kk;
    at(idx, ln, kk);
    if (u0 + ln <= nu) out[base + ln * st[au] + (int64_t)(kk + 1) * st[axis]] = tile[ln][kk];
  }
}

__global__ void k_fdm_zero_boundary(const DevData d, double *__restrict__ t, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.g.n_nodes && d.Dm12[i] == 0.0) t[i] = 0.0;
}

__global__ void k_fdm_scale(const DevData d, double *__restrict__ t, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const Geom &g = d.g;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_nodes) return;
  if (d.Dm12[i] == 0.0) { t[i] = 0.0; return; }
  int64_t gg[3] = {i % g.nn[0], (i / g.nn[0]) % g.nn[1], i / (g.nn[0] * g.nn[1])};
  t[i] /= d.fdmL[0][gg[0] - 1] + d.fdmL[1][gg[1] - 1] + d.fdmL[2][gg[2] - 1];
}

__global__ void k_add_boundary(const DevData d, double *__restrict__ phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.g.n_nodes) return;
  if (d.Dm12[i] == 0.0) phi[i] = d.gbnd[i];
}

// deterministic partial dot products
__global__ void __launch_bounds__(kThreads)
k_dot(const double *__restrict__ x, const double *__restrict__ y, int64_t n, double *__restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[v] = sum_b part[b * nval + v] in block order
__global__ void k_reduce(const double *__restrict__ part, int nblk, int nval, double *__restrict__ out) {
  __shared__ double red[16];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(int64_t)b * nval + v];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[v] = s;
}

// dipole partials: one block per cell, part[cell][3]
__global__ void __launch_bounds__(kThreads)
k_dipole(const DevData d, const double *__restrict__ rho, double *__restrict__ part) {
  __shared__ double red[16];
  const Geom &g = d.g;
  const int64_t cell = blockIdx.x;
  const bool enr = d.is_enr[cell] != 0;
  const int n = enr ? g.qe : g.qc, n3 = n * n * n;
  const double *tab = d.tab;
  const int tox = enr ? d.to.xqe : d.to.xqc, tow = enr ? d.to.wqe : d.to.wqc;
  int e[3];
  cell_ijk(g, cell, e);
  const int64_t q0 = d.q_off[cell];
  double clo[3], ch[3];
  cell_box(d, e, clo, ch);
  const double jac = 0.125 * ch[0] * ch[1] * ch[2];
  double s[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < n3; q += blockDim.x) {
    int i = q % n, j = (q / n) % n, k = q / (n * n);
    double w = jac * tab[tow + i] * tab[tow + j] * tab[tow + k] * rho[q0 + q];
    s[0] += w * (clo[0] + (tab[tox + i] + 1.0) * 0.5 * ch[0]);
    s[1] += w * (clo[1] + (tab[tox + j] + 1.0) * 0.5 * ch[1]);
    s[2] += w * (clo[2] + (tab[tox + k] + 1.0) * 0.5 * ch[2]);
  }
  for (int dd = 0; dd < 3; ++dd) {
    double t = block_sum(s[dd], red);
    if (threadIdx.x == 0) part[cell * 3 + dd] = t;
  }
}

__global__ void k_zero(double *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_axpby(const double *x, const double *y, double a, double b, double *out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + b * y[i];
}

// out = a x + (*b) y  (skipped when *skip)
__global__ void k_axpby_dev(const double *x, const double *y, double a, const double *__restrict__ b, double *out,
                            int64_t n, const int *__restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + *b * y[i];
}

// x += alpha p ; r -= alpha q  (skipped when *skip)
__global__ void k_pcg_update(double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
                             const double *__restrict__ q, const double *__restrict__ alpha, int64_t n,
                             const int *__restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double a = *alpha;
    x[i] += a * p[i];
    r[i] -= a * q[i];
  }
}

// Scalar bookkeeping of the preconditioned CG on the device (one thread).
// S: [0] r.z  [1] previous r.z  [2] p.q  [3] r.r  [4] rhs.rhs  [5] alpha  [6] beta  [7] iterations
__global__ void k_pcg_scalar(int op, double *__restrict__ S, double tol2, int *__restrict__ done) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  switch (op) {
    case 0:   // start: converged already?
      *done = (S[3] <= tol2 * S[4] || S[4] == 0.0) ? 1 : 0;
      S[7] = 0.0;
      break;
    case 1:   // beta from r.z (first iteration: 0)
      if (!*done) S[6] = S[7] == 0.0 ? 0.0 : S[0] / S[1];
      break;
    case 2:   // alpha = r.z / p.q
      if (!*done) {
        S[5] = S[0] / S[2];
        S[1] = S[0];
      }
      break;
    case 3:   // after the update: count and test
      if (!*done) {
        S[7] += 1.0;
        if (S[3] <= tol2 * S[4]) *done = 1;
      }
      break;
  }
}

__global__ void k_set_scalar(double *__restrict__ p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_copy_rows(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t nrows, int ncolr) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncolr) return;
  int64_t r = t / ncolr;
  int c = (int)(t % ncolr);
  dst[r * ldd + c] = src[r * lds + c];
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

namespace k {

void zero(double *p, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n);
}

void axpby(const double *x, const double *y, double a, double b, double *out, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpby, dim3(nblocks(n, 256)), dim3(256), 0, s, x, y, a, b, out, n);
}

void copy_rows(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t nrows, int ncolr, hipStream_t s) {
  if (nrows * ncolr > 0)
    hipLaunchKernelGGL(k_copy_rows, dim3(nblocks(nrows * ncolr, 256)), dim3(256), 0, s, src, lds, dst, ldd, nrows, ncolr);
}

static size_t rebuild_lds(const Geom &g, int n) {
  const int P = g.P, NP = P * (P + 1) / 2;
  const size_t ua = (size_t)n * n * NP, ub = (size_t)g.nloc + P * P * n + n * n * P;
  const size_t usz = ua > ub ? ua : ub;   // U, or the interpolation's u0, t1, t2
  const size_t dbl = (size_t)n * P + n * NP + 6 * P * P + g.nloc + n * n * n + usz + n * NP + NP * NP;
  return dbl * sizeof(double) + P * P * sizeof(int) + 64;
}

void rebuild_cells(const DevData &d, int mode, const double *rho, const double *phi, const double *efield, int fdir,
                   int xc, void *cells, int dtype, double *vq, hipStream_t s) {
  for (int cls = 0; cls < 2; ++cls) {
    int nc = cls ? d.n_enr : d.n_ord;
    if (nc == 0) continue;
    int n = cls ? d.g.qe : d.g.qc;
    const int *list = cls ? d.cells_enr : d.cells_ord;
    size_t lds = rebuild_lds(d.g, n);
    if (dtype == 0 || dtype == 3)
      hipLaunchKernelGGL(k_rebuild<double>, dim3(nc), dim3(kThreads), lds, s, d, list, n, mode, rho, phi, efield, fdir,
                         xc, (double *)cells, vq);
    else if (dtype == 1)
      hipLaunchKernelGGL(k_rebuild<float>, dim3(nc), dim3(kThreads), lds, s, d, list, n, mode, rho, phi, efield, fdir,
                         xc, (float *)cells, vq);
    else if (dtype == 2)
      hipLaunchKernelGGL(k_rebuild<Bf16Rows>, dim3(nc), dim3(kThreads), lds, s, d, list, n, mode, rho, phi, efield,
                         fdir, xc, (Bf16Rows *)cells, vq);
    else
      hipLaunchKernelGGL(k_rebuild<Bf16Split>, dim3(nc), dim3(kThreads), lds, s, d, list, n, mode, rho, phi, efield,
                         fdir, xc, (Bf16Split *)cells, vq);
  }
}

void coupling_partials(const DevData &d, const double *vq, double *part, double *hee_part, hipStream_t s) {
  if (d.nt == 0) return;
  const int n = d.g.qe > d.g.qc ? d.g.qe : d.g.qc, P = d.g.P;
  size_t lds = ((size_t)n * P + 2 * n * n * n + n * n * P + n * P * P + d.g.nloc) * sizeof(double);
  if (d.g.qe <= 16 && d.g.qc <= 16 && d.g.P <= 8 && d.max_tnu <= 48) {
    // node part by the three axis contractions, H^ee (a dense product over the points) on MFMA
    hipLaunchKernelGGL(k_coupling_partials<false>, dim3(d.nt), dim3(kThreads), lds, s, d, vq, part, hee_part);
    hipLaunchKernelGGL((k_coupling_mfma<4, false>), dim3(d.nt), dim3(256), 0, s, d, vq, part, hee_part);
    return;
  }
  hipLaunchKernelGGL(k_coupling_partials<true>, dim3(d.nt), dim3(kThreads), lds, s, d, vq, part, hee_part);
}

void coupling_gather(const DevData &d, const double *part, int kinetic, double *G, float *G32, hipStream_t s) {
  if (d.nr == 0 || d.nk == 0) return;
  const int64_t ntiles = (d.nr + 15) / 16;
  const int64_t nw = ntiles < kGatherWaves ? ntiles : kGatherWaves;
  const int64_t tpw = (ntiles + nw - 1) / nw;
  const unsigned ny = (unsigned)((d.nk + 47) / 48);
  if (G)
    hipLaunchKernelGGL(k_coupling_gather<double>, dim3((unsigned)((ntiles + tpw - 1) / tpw), ny), dim3(64), 0, s, d,
                       part, kinetic, G, tpw);
  else
    hipLaunchKernelGGL(k_coupling_gather<float>, dim3((unsigned)((ntiles + tpw - 1) / tpw), ny), dim3(64), 0, s, d,
                       part, kinetic, G32, tpw);
}

int64_t hee_scratch_size(const DevData &d) { return (int64_t)kHeeBlocks * d.ne * d.ne; }

void hee_reduce(const DevData &d, const double *hee_part, int kinetic, double *Hraw, double *Hbar, double *scratch,
                hipStream_t s) {
  if (d.ne == 0) return;
  const int nblk = d.nt > 0 ? kHeeBlocks : 0;
  if (nblk > 0)
    hipLaunchKernelGGL(k_hee_blocks, dim3(nblk), dim3(256), (size_t)d.ne * d.ne * sizeof(double), s, d, hee_part,
                       scratch);
  hipLaunchKernelGGL(k_hee_sum, dim3(nblocks(d.ne * d.ne, 64)), dim3(64), 0, s, d, scratch, nblk, kinetic, Hraw);
  // the block sums are consumed: the scratch holds T = H^ee S next
  hipLaunchKernelGGL(k_hee_hs, dim3(nblocks(d.ne * d.nk, 64)), dim3(64), 0, s, d, Hraw, scratch);
  hipLaunchKernelGGL(k_hee_loewdin, dim3(nblocks(d.nk * d.nk, 64)), dim3(64), 0, s, d, scratch, Hbar);
}

void psiE(const DevData &d, const double *X, int ncolr, int64_t ldr, double *out, hipStream_t s) {
  if (d.ne == 0) return;
  hipLaunchKernelGGL(k_psiE, dim3(nblocks((int64_t)d.ne * ncolr, 128)), dim3(128), 0, s, d, X, ncolr, ldr, out);
}

static size_t density_sq_lds(const Geom &g) {
  return ((size_t)g.P * g.P + g.nloc + 128 + (size_t)g.nloc * kDenCols) * sizeof(double);
}

int density_init(const Geom &g) {
  int st = 0;
  st |= (int)hipFuncSetAttribute((const void *)k_density_sq<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)density_sq_lds(g));
  st |= (int)hipFuncSetAttribute((const void *)k_density_sq<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)density_sq_lds(g));
  return st;
}

template <bool CROSS>
static void density_launch_generic(const DevData &d, const double *X, int ncol, int64_t ldr, const double *psiE,
                                   double *rho, double wcross, hipStream_t s) {
  constexpr int NCC = 4, F = 2 * NCC;
  for (int cls = 0; cls < 2; ++cls) {
    int nc = cls ? d.n_enr : d.n_ord;
    if (nc == 0) continue;
    int n = cls ? d.g.qe : d.g.qc, P = d.g.P;
    const int *list = cls ? d.cells_enr : d.cells_ord;
    if (n == P && d.g.nloc <= 2 * kThreads && ncol <= 128) {
      hipLaunchKernelGGL((k_density_sq<CROSS>), dim3(nc), dim3(kThreads), density_sq_lds(d.g), s, d, list, X, ncol,
                         ldr, psiE, rho, wcross);
      continue;
    }
    size_t lds = ((size_t)n * P + d.g.nloc + (size_t)d.g.nloc * F + (size_t)P * P * n * F + (size_t)P * n * n * F + ncol) *
                 sizeof(double);
    int n3 = n * n * n;
    if (n3 <= 256)
      hipLaunchKernelGGL((k_density<NCC, 1, CROSS>), dim3(nc), dim3(kThreads), lds, s, d, list, n, X, ncol, ldr, psiE,
                         rho, wcross);
    else if (n3 <= 512)
      hipLaunchKernelGGL((k_density<NCC, 2, CROSS>), dim3(nc), dim3(kThreads), lds, s, d, list, n, X, ncol, ldr, psiE,
                         rho, wcross);
    else if (n3 <= 1024)
      hipLaunchKernelGGL((k_density<NCC, 4, CROSS>), dim3(nc), dim3(kThreads), lds, s, d, list, n, X, ncol, ldr, psiE,
                         rho, wcross);
    else if (n3 <= 2048)
      hipLaunchKernelGGL((k_density<NCC, 8, CROSS>), dim3(nc), dim3(kThreads), lds, s, d, list, n, X, ncol, ldr, psiE,
                         rho, wcross);
    else
      hipLaunchKernelGGL((k_density<NCC, 16, CROSS>), dim3(nc), dim3(kThreads), lds, s, d, list, n, X, ncol, ldr,
                         psiE, rho, wcross);
  }
}

constexpr int kDenOrdGroups = 2;   // 8-column groups per pass on ordinary cells

inline int den_passes(int ncolr, int groups) { return (ncolr + 8 * groups - 1) / (8 * groups); }

template <int NP, int N, int NFG, bool CROSS>
static void den_class(const DevData &d, const int *list, int ncells, const double *X, int ncol, int64_t ldr,
                      const double *psiE, double *rho, double wcross, const double *U, double *part, hipStream_t s) {
  if (ncells == 0) return;
  const int np = den_passes(2 * ncol, NFG);
  const unsigned nb = (unsigned)(8 * ((ncells + 7) / 8) * np);
  hipLaunchKernelGGL((k_den<NP, N, NFG, false, CROSS>), dim3(nb), dim3(kThreads), 0, s, d, list, ncells, X, ncol,
                     ldr, U, psiE, rho, part, np, wcross);
  constexpr int N3 = N * N * N;
  hipLaunchKernelGGL((k_den_sum<CROSS>), dim3(nblocks((int64_t)ncells * N3, 256)), dim3(256), 0, s, d, list, ncells,
                     N3, part, np, rho, wcross);
}

template <int NP, bool CROSS>
static void density_launch_folded(const DevData &d, const double *X, int ncol, int64_t ldr, const double *psiE,
                                  double *rho, double wcross, const DenWork &w, hipStream_t s) {
  const int ncolr = 2 * ncol;
  if (d.nr > 0) {
    const int64_t ntiles = (d.nr + 15) / 16;
    const int64_t nw = ntiles < kFoldWaves ? ntiles : kFoldWaves;
    const int64_t tpw = (ntiles + nw - 1) / nw;
    const unsigned ny = (unsigned)((ncolr + 16 * kFoldNT - 1) / (16 * kFoldNT));
    hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)((ntiles + tpw - 1) / tpw), ny), dim3(64), 0, s, d, X, ncolr, ldr,
                       psiE, w.U, tpw);
  }
  // ordinary cells: one workgroup per cell over all passes (no atomic part, no partials)
  if (d.n_ord > 0)
    hipLaunchKernelGGL((k_den<NP, NP, kDenOrdGroups, true, CROSS>), dim3(d.n_ord), dim3(kThreads), 0, s, d,
                       d.cells_ord, d.n_ord, X, ncol, ldr, w.U, psiE, rho, nullptr, den_passes(ncolr, kDenOrdGroups),
                       wcross);
  den_class<NP, 2 * NP, 1, CROSS>(d, d.cells_enr, d.n_enr, X, ncol, ldr, psiE, rho, wcross, w.U, w.part, s);
}

// the folded kernels cover GLL degree 4 and 5 with the default rules (p+1 and
// 2p+2 Gauss points per axis) and at most 48 atomic functions per cell
bool density_folded_ok(const DevData &d) {
  return (d.g.P == 5 || d.g.P == 6) && d.g.qc == d.g.P && d.g.qe == 2 * d.g.P && d.max_ta <= 48;
}

int64_t density_part_size(const DevData &d, int ncolr) {
  return (int64_t)den_passes(ncolr, 1) * d.n_enr * d.g.qe * d.g.qe * d.g.qe;
}

template <bool CROSS>
static void density_launch(const DevData &d, const double *X, int ncol, int64_t ldr, const double *psiE, double *rho,
                           double wcross, const DenWork &w, hipStream_t s) {
  if (!density_folded_ok(d) || !w.U || !w.part || (!CROSS && ncol > 128)) {
    density_launch_generic<CROSS>(d, X, ncol, ldr, psiE, rho, wcross, s);
    return;
  }
  if (d.g.P == 5) density_launch_folded<5, CROSS>(d, X, ncol, ldr, psiE, rho, wcross, w, s);
  else density_launch_folded<6, CROSS>(d, X, ncol, ldr, psiE, rho, wcross, w, s);
}

void density(const DevData &d, const double *X, int ncol, int64_t ldr, const double *psiE, double *rho,
             const DenWork &w, hipStream_t s) {
  density_launch<false>(d, X, ncol, ldr, psiE, rho, 0.0, w, s);
}

void cross_density(const DevData &d, const double *Z, int npair, const double *psiE, double wt, double *out,
                   const DenWork &w, hipStream_t s) {
  density_launch<true>(d, Z, 2 * npair, 4 * npair, psiE, out, wt, w, s);
}

void adj_potential(const DevData &d, const double *phibar, const double *rho, const double *u, double tau, int xc,
                   const double mubar[3], double a, const double *gin, double *out, hipStream_t s) {
  for (int cls = 0; cls < 2; ++cls) {
    int nc = cls ? d.n_enr : d.n_ord;
    if (nc == 0) continue;
    int n = cls ? d.g.qe : d.g.qc, P = d.g.P;
    const int *list = cls ? d.cells_enr : d.cells_ord;
    size_t lds = ((size_t)n * P + d.g.nloc + (size_t)P * P * n + (size_t)P * n * n + (size_t)n * n * n) * sizeof(double);
    hipLaunchKernelGGL(k_adj_potential, dim3(nc), dim3(kThreads), lds, s, d, list, n, phibar, rho, u, tau, xc,
                       mubar[0], mubar[1], mubar[2], a, gin, out);
  }
}

void axpy_cols(double *out, const double *Y, const double *sc, double s0, int64_t nrows, int ncol, hipStream_t s) {
  if (nrows * ncol > 0)
    hipLaunchKernelGGL(k_axpy_cols, dim3(nblocks(nrows * ncol, 256)), dim3(256), 0, s, out, Y, sc, s0, nrows, ncol);
}

void interleave(const double *a, const double *b, double *Z, int64_t nrows, int ncol, hipStream_t s) {
  if (nrows * ncol > 0)
    hipLaunchKernelGGL(k_interleave, dim3(nblocks(nrows * ncol, 256)), dim3(256), 0, s, (const double2 *)a,
                       (const double2 *)b, (double2 *)Z, nrows, ncol);
}

void poisson_rhs(const DevData &d, const double *rho, double *dvec, double *rhs, hipStream_t s, int lift) {
  zero(dvec, d.g.n_nodes, s);
  const int n = d.g.qe > d.g.qc ? d.g.qe : d.g.qc, P = d.g.P;
  size_t lds = ((size_t)n * P + (size_t)n * n * n + (size_t)n * n * P + (size_t)n * P * P + d.g.nloc) * sizeof(double);
  for (int c = 0; c < 8; ++c) {
    int cnt = d.colour_off[c + 1] - d.colour_off[c];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_poisson_rhs, dim3(cnt), dim3(kThreads), lds, s, d, d.colour_cells + d.colour_off[c], rho, dvec);
  }
  hipLaunchKernelGGL(k_rhs_finish, dim3(nblocks(d.g.n_nodes, 256)), dim3(256), 0, s, d, dvec, rhs, lift);
}

// y = K_II x for x with zero boundary: K = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1
void stiffness_apply(const DevData &d, const double *x, double *y, double *t1, double *t2, hipStream_t s,
                     const int *skip) {
  const unsigned nb = nblocks(d.g.n_nodes, 256);
  for (int term = 0; term < 3; ++term) {
    hipLaunchKernelGGL(k_axis_band, dim3(nb), dim3(256), 0, s, d, term == 0 ? d.K1[0] : d.M1[0], 0, x, t1, skip);
    hipLaunchKernelGGL(k_axis_band, dim3(nb), dim3(256), 0, s, d, term == 1 ? d.K1[1] : d.M1[1], 1, t1, t2, skip);
    hipLaunchKernelGGL(k_axis_band, dim3(nb), dim3(256), 0, s, d, term == 2 ? d.K1[2] : d.M1[2], 2, t2, t1, skip);
    hipLaunchKernelGGL(k_interior_acc, dim3(nb), dim3(256), 0, s, d, t1, y, term > 0 ? 1 : 0, skip);
  }
}

// z = K_II^-1 r on interior nodes by fast diagonalisation
void fdm_apply(const DevData &d, const double *r, double *z, double *t1, double *t2, hipStream_t s, const int *skip) {
  const unsigned nb = nblocks(d.g.n_nodes, 256);
  bool lines = d.fdmVT[0] && d.fdmVT[1] && d.fdmVT[2];
  for (int a = 0; a < 3; ++a) lines = lines && d.g.nn[a] - 2 <= kFdmMaxM && d.g.nn[a] >= 3;
  if (lines) {
    auto grid = [&](int axis) {
      const int au = axis == 0 ? 1 : 0, av = axis == 2 ? 1 : 2;
      return dim3((unsigned)((d.g.nn[au] - 2 + kFdmLines - 1) / kFdmLines), (unsigned)(d.g.nn[av] - 2));
    };
    hipLaunchKernelGGL(k_fdm_lines, grid(0), dim3(kFdmMaxM), 0, s, d, d.fdmV[0], 0, r, t1, skip);
    hipLaunchKernelGGL(k_fdm_lines, grid(1), dim3(kFdmMaxM), 0, s, d, d.fdmV[1], 1, t1, t2, skip);
    hipLaunchKernelGGL(k_fdm_lines, grid(2), dim3(kFdmMaxM), 0, s, d, d.fdmV[2], 2, t2, t1, skip);
    hipLaunchKernelGGL(k_fdm_scale, dim3(nb), dim3(256), 0, s, d, t1, skip);
    hipLaunchKernelGGL(k_fdm_lines, grid(2), dim3(kFdmMaxM), 0, s, d, d.fdmVT[2], 2, t1, t2, skip);
    hipLaunchKernelGGL(k_fdm_lines, grid(1), dim3(kFdmMaxM), 0, s, d, d.fdmVT[1], 1, t2, t1, skip);
    hipLaunchKernelGGL(k_fdm_lines, grid(0), dim3(kFdmMaxM), 0, s, d, d.fdmVT[0], 0, t1, z, skip);
    hipLaunchKernelGGL(k_fdm_zero_boundary, dim3(nb), dim3(256), 0, s, d, z, skip);
    return;
  }
  hipLaunchKernelGGL(k_fdm_axis, dim3(nb), dim3(256), 0, s, d, d.fdmV[0], 0, 0, r, t1, skip);
  hipLaunchKernelGGL(k_fdm_axis, dim3(nb), dim3(256), 0, s, d, d.fdmV[1], 1, 0, t1, t2, skip);
  hipLaunchKernelGGL(k_fdm_axis, dim3(nb), dim3(256), 0, s, d, d.fdmV[2], 2, 0, t2, t1, skip);
  hipLaunchKernelGGL(k_fdm_scale, dim3(nb), dim3(256), 0, s, d, t1, skip);
  hipLaunchKernelGGL(k_fdm_axis, dim3(nb), dim3(256), 0, s, d, d.fdmV[2], 2, 1, t1, t2, skip);
  hipLaunchKernelGGL(k_fdm_axis, dim3(nb), dim3(256), 0, s, d, d.fdmV[1], 1, 1, t2, t1, skip);
  hipLaunchKernelGGL(k_fdm_axis, dim3(nb), dim3(256), 0, s, d, d.fdmV[0], 0, 1, t1, z, skip);
}

void axpby_dev(const double *x, const double *y, double a, const double *b, double *out, int64_t n, const int *skip,
               hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpby_dev, dim3(nblocks(n, 256)), dim3(256), 0, s, x, y, a, b, out, n, skip);
}

void pcg_update(double *x, double *r, const double *p, const double *q, const double *alpha, int64_t n,
                const int *skip, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pcg_update, dim3(nblocks(n, 256)), dim3(256), 0, s, x, r, p, q, alpha, n, skip);
}

void pcg_scalar(int op, double *S, double tol2, int *done, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_scalar, dim3(1), dim3(64), 0, s, op, S, tol2, done);
}

void set_scalar(double *p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, p, v);
}

void set_boundary(const DevData &d, double *phi, hipStream_t s) {
  hipLaunchKernelGGL(k_add_boundary, dim3(nblocks(d.g.n_nodes, 256)), dim3(256), 0, s, d, phi);
}

int dot_partials(const double *x, const double *y, int64_t n, double *part, hipStream_t s) {
  int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kThreads), 0, s, x, y, n, part);
  return nb;
}

void reduce_partials(const double *part, int nblk, int nval, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nval), dim3(256), 0, s, part, nblk, nval, out);
}

void dipole_partials(const DevData &d, const double *rho, double *part, int *nblk, hipStream_t s) {
  int64_t nc = (int64_t)d.g.nc[0] * d.g.nc[1] * d.g.nc[2];
  hipLaunchKernelGGL(k_dipole, dim3((unsigned)nc), dim3(kThreads), 0, s, d, rho, part);
  *nblk = (int)nc;
}

}  // namespace k
}  // namespace efe
