// Cell part of Hbar X by sum factorisation (no stored cell blocks): on each cell
//   Hbar_c u = D_c^-1/2 ( 1/2 (K_x x M_y x M_z + M_x x K_y x M_z + M_x x M_y x K_z)
//                         + B^T diag(W v) B ) D_c^-1/2 u
// (Sec. 2.3, eq. (TDKSDiscrete2); the same operator as the dense blocks that
// the rebuild assembles), with K_d, M_d the exact 1-D element matrices, B the
// Lagrange values of the GLL basis at the cell's Gauss points and W v the
// weighted potential at those points.  FP64 on the vector ALU.
#include <hip/hip_runtime.h>

#include "common.h"

namespace efe {
namespace {

constexpr int kSfThreads = 256;

// One workgroup per (cell of one colour, F columns).  Five stages, each a
// loop over lines of the cell tensor, pass the data through LDS ([element][F]):
//   1 x-lines (b, c): u -> M_x u, K_x u, B_x u
//   2 y-lines:        A = M_y K_x u + K_y M_x u, B = M_y M_x u;  B_y B_x u
//   3 z-lines:        y_K = (M_z A + K_z B) / 2;  point values p = B_z B_y B_x u,
//                     p *= W v, back along z: B_z^T p
//   4 y-lines (back): B_y^T
//   5 x-lines (back): B_x^T, add y_K, scale by D^-1/2, store or add into Y
// The first colour to reach a node stores instead of adding (as the dense kernel).
template <int P, int N, int F>
struct SfLayout {
  static constexpr int NL = P * P * P;
  static constexpr int R1 = (2 * NL + N * P * P > NL + N * N * P ? 2 * NL + N * P * P : NL + N * N * P) * F;
  static constexpr int R2 = (2 * NL + N * N * P > N * P * P ? 2 * NL + N * N * P : N * P * P) * F;
};

template <int P, int N, int F>
__global__ void __launch_bounds__(kSfThreads)
k_sf_apply(const DevData d, const int *__restrict__ cell_list, const double *__restrict__ vq, int kinetic,
           const double *__restrict__ X, double *__restrict__ Y, int ncolr, int64_t ldr, const int *__restrict__ any) {
  if (any && *any == 0) return;
  constexpr int P2 = P * P, NL = P * P * P;
  typedef SfLayout<P, N, F> L;
  __shared__ double sB[N * P];                   // B[i][a]
  __shared__ double sK[3][P * P], sM[3][P * P];  // 1-D element matrices per axis
  __shared__ double wv[N * N * N];               // W v at the points, x fastest
  __shared__ int64_t rowoff[NL];
  __shared__ double dm[NL];
  __shared__ unsigned char first[NL];
  extern __shared__ double sf_sm[];
  double *R1 = sf_sm, *R2 = sf_sm + L::R1;
  // stage outputs: 1 -> R1 {mx, kx, px}; 2 -> R2 {A, Bm, py}; 3 -> R1 {yk, rz}; 4 -> R2 {ry}
  double *mx = R1, *kx = R1 + NL * F, *px = R1 + 2 * NL * F;
  double *Ak = R2, *Bk = R2 + NL * F, *py = R2 + 2 * NL * F;
  double *yk = R1, *rz = R1 + NL * F;
  double *ry = R2;
  const Geom &g = d.g;
  const int tid = threadIdx.x;
  const int64_t cell = cell_list[blockIdx.x];
  const int c0 = blockIdx.y * F;
  int e[3];
  cell_ijk(g, cell, e);
  const bool enr = N != P;
  const int toB = enr ? d.to.Be : d.to.Bc, tow = enr ? d.to.wqe : d.to.wqc;
  for (int t = tid; t < N * P; t += kSfThreads) sB[t] = d.tab[toB + t];
  double clo[3], ch[3];
  cell_box(d, e, clo, ch);
  for (int t = tid; t < 3 * P2; t += kSfThreads) {
    sK[t / P2][t % P2] = d.tab[d.to.Kr + t % P2] * (2.0 / ch[t / P2]);
    sM[t / P2][t % P2] = d.tab[d.to.Mr + t % P2] * (0.5 * ch[t / P2]);
  }
  const int64_t q0 = d.q_off[cell];
  const double jac = 0.125 * ch[0] * ch[1] * ch[2];
  for (int q = tid; q < N * N * N; q += kSfThreads) {
    const int i = q % N, j = (q / N) % N, k = q / (N * N);
    wv[q] = jac * d.tab[tow + i] * d.tab[tow + j] * d.tab[tow + k] * vq[q0 + q];
  }
  for (int l = tid; l < NL; l += kSfThreads) {
    const int64_t node = local_node(g, e, l);
    rowoff[l] = node * ldr;
    dm[l] = d.Dm12[node];
    const int li[3] = {l % P, (l / P) % P, l / P2};
    bool later = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const bool shared = (li[ax] == 0 && e[ax] > 0) || (li[ax] == g.p && e[ax] < g.nc[ax] - 1);
      later |= shared && (e[ax] & 1);
    }
    first[l] = later ? 0 : 1;
  }
  __syncthreads();

  // 1: x-lines (b, c) of u = D^-1/2 X; the thread of x-line item tid also loads the
  // output rows it adds to in stage 5 (nodes another colour reached first)
  static_assert(P * P * F <= kSfThreads, "one x-line item per thread");
  const bool xl = tid < P2 * F;
  double yold[P];
  {
    const int it = xl ? tid : 0;
    const int f = it % F, bc = it / F, col = c0 + f;
    const bool ok = xl && col < ncolr;
    double u[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const int l = a + P * bc;
      u[a] = ok ? dm[l] * X[rowoff[l] + col] : 0.0;
      yold[a] = (ok && !first[l]) ? Y[rowoff[l] + col] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < P; ++a) {
      double sm = 0.0, sk = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < P; ++a2) {
        sm += sM[0][a * P + a2] * u[a2];
        sk += sK[0][a * P + a2] * u[a2];
      }
      if (xl) {
        mx[(a + P * bc) * F + f] = sm;
        kx[(a + P * bc) * F + f] = sk;
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < P; ++a) s += sB[i * P + a] * u[a];
      if (xl) px[(i + N * bc) * F + f] = s;       // [c][b][i]
    }
  }
  __syncthreads();
  // 2: y-lines.  Kinetic lines (a, c): A = M_y kx + K_y mx, Bk = M_y mx
  for (int it = tid; it < P2 * F; it += kSfThreads) {
    const int f = it % F, ac = it / F, a = ac % P, c = ac / P;
    double vm[P], vk[P];
#pragma unroll
    for (int b = 0; b < P; ++b) {
      vm[b] = mx[(a + P * b + P2 * c) * F + f];
      vk[b] = kx[(a + P * b + P2 * c) * F + f];
    }
#pragma unroll
    for (int b = 0; b < P; ++b) {
      double sa = 0.0, sb = 0.0;
#pragma unroll
      for (int b2 = 0; b2 < P; ++b2) {
        sa += sM[1][b * P + b2] * vk[b2] + sK[1][b * P + b2] * vm[b2];
        sb += sM[1][b * P + b2] * vm[b2];
      }
      Ak[(a + P * b + P2 * c) * F + f] = sa;
      Bk[(a + P * b + P2 * c) * F + f] = sb;
    }
  }
  // potential lines (i, c): py[c][j][i] = sum_b B[j][b] px[c][b][i]
  for (int it = tid; it < N * P * F; it += kSfThreads) {
    const int f = it % F, ic = it / F, i = ic % N, c = ic / N;
    double v[P];
#pragma unroll
    for (int b = 0; b < P; ++b) v[b] = px[(i + N * b + N * P * c) * F + f];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < P; ++b) s += sB[j * P + b] * v[b];
      py[(i + N * j + N * N * c) * F + f] = s;
    }
  }
  __syncthreads();
  // 3: z-lines.  Kinetic lines (a, b): yk = (M_z A + K_z Bk) / 2 (0 without the kinetic term)
  for (int it = tid; it < P2 * F; it += kSfThreads) {
    const int f = it % F, ab = it / F;
    double va[P], vb[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      va[c] = Ak[(ab + P2 * c) * F + f];
      vb[c] = Bk[(ab + P2 * c) * F + f];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      double s = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < P; ++c2) s += sM[2][c * P + c2] * va[c2] + sK[2][c * P + c2] * vb[c2];
      yk[(ab + P2 * c) * F + f] = kinetic ? 0.5 * s : 0.0;
    }
  }
  // potential lines (i, j): points k, times W v, back along z into rz[c][j][i]
  for (int it = tid; it < N * N * F; it += kSfThreads) {
    const int f = it % F, ij = it / F;
    double v[P];
#pragma unroll
    for (int c = 0; c < P; ++c) v[c] = py[(ij + N * N * c) * F + f];
    double r[P];
#pragma unroll
    for (int c = 0; c < P; ++c) r[c] = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double pk = 0.0;
#pragma unroll
      for (int c = 0; c < P; ++c) pk += sB[k * P + c] * v[c];
      pk *= wv[ij + N * N * k];
#pragma unroll
      for (int c = 0; c < P; ++c) r[c] += sB[k * P + c] * pk;
    }
#pragma unroll
    for (int c = 0; c < P; ++c) rz[(ij + N * N * c) * F + f] = r[c];
  }
  __syncthreads();
  // 4: back along y, lines (i, c): ry[c][b][i] = sum_j B[j][b] rz[c][j][i]
  for (int it = tid; it < N * P * F; it += kSfThreads) {
    const int f = it % F, ic = it / F, i = ic % N, c = ic / N;
    double r[P];
#pragma unroll
    for (int b = 0; b < P; ++b) r[b] = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double v = rz[(i + N * j + N * N * c) * F + f];
#pragma unroll
      for (int b = 0; b < P; ++b) r[b] += sB[j * P + b] * v;
    }
#pragma unroll
    for (int b = 0; b < P; ++b) ry[(i + N * b + N * P * c) * F + f] = r[b];
  }
  __syncthreads();
  // 5: back along x, lines (b, c) (the item of stage 1); add the kinetic part, scale, store
  if (xl) {
    const int it = tid;
    const int f = it % F, bc = it / F, col = c0 + f;
    double r[P];
#pragma unroll
    for (int a = 0; a < P; ++a) r[a] = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double v = ry[(i + N * bc) * F + f];
#pragma unroll
      for (int a = 0; a < P; ++a) r[a] += sB[i * P + a] * v;
    }
    if (col < ncolr) {
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const int l = a + P * bc;
        Y[rowoff[l] + col] = yold[a] + dm[l] * (yk[l * F + f] + r[a]);
      }
    }
  }
}

template <int P, int N, int F>
size_t sf_lds() {
  return (size_t)(SfLayout<P, N, F>::R1 + SfLayout<P, N, F>::R2) * sizeof(double);
}

constexpr int kSfColsOrd = 7;   // columns per workgroup, ordinary cells (P^2 F <= 256)
constexpr int kSfColsEnr = 4;   // enrichment cells (LDS)

template <int P>
void sf_launch(const DevData &d, const double *vq, int kinetic, const double *X, double *Y, int ncolr, int64_t ldr,
               hipStream_t s, const int *any) {
  const unsigned nyo = (unsigned)((ncolr + kSfColsOrd - 1) / kSfColsOrd);
  const unsigned nye = (unsigned)((ncolr + kSfColsEnr - 1) / kSfColsEnr);
  for (int c = 0; c < 8; ++c) {
    const int cnt = d.colour_off[c + 1] - d.colour_off[c];
    if (cnt == 0) continue;
    // the colour's cells in two launches by class (their rules differ); both write disjoint nodes
    for (int cls = 0; cls < 2; ++cls) {
      const int *list = cls ? d.sf_enr + d.sf_off[2 * c + 1] : d.sf_ord + d.sf_off[2 * c];
      const int n = cls ? d.sf_off[2 * c + 3] - d.sf_off[2 * c + 1] : d.sf_off[2 * c + 2] - d.sf_off[2 * c];
      if (n == 0) continue;
      if (cls == 0)
        hipLaunchKernelGGL((k_sf_apply<P, P, kSfColsOrd>), dim3((unsigned)n, nyo), dim3(kSfThreads),
                           (sf_lds<P, P, kSfColsOrd>()), s, d, list, vq, kinetic, X, Y, ncolr, ldr, any);
      else
        hipLaunchKernelGGL((k_sf_apply<P, 2 * P, kSfColsEnr>), dim3((unsigned)n, nye), dim3(kSfThreads),
                           (sf_lds<P, 2 * P, kSfColsEnr>()), s, d, list, vq, kinetic, X, Y, ncolr, ldr, any);
    }
  }
}

}  // namespace

namespace k {

bool sf_supported(const Geom &g) { return (g.P == 5 || g.P == 6) && g.qc == g.P && g.qe == 2 * g.P; }

int sf_init(const Geom &g) {
  int st = 0;
  st |= (int)hipFuncSetAttribute((const void *)k_sf_apply<5, 5, kSfColsOrd>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sf_lds<5, 5, kSfColsOrd>());
  st |= (int)hipFuncSetAttribute((const void *)k_sf_apply<5, 10, kSfColsEnr>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sf_lds<5, 10, kSfColsEnr>());
  st |= (int)hipFuncSetAttribute((const void *)k_sf_apply<6, 6, kSfColsOrd>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sf_lds<6, 6, kSfColsOrd>());
  st |= (int)hipFuncSetAttribute((const void *)k_sf_apply<6, 12, kSfColsEnr>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sf_lds<6, 12, kSfColsEnr>());
  (void)g;
  return st;
}

void sf_apply(const DevData &d, const double *vq, int kinetic, const double *X, double *Y, int ncolr, int64_t ldr,
              hipStream_t s, const int *any) {
  if (d.g.P == 5) sf_launch<5>(d, vq, kinetic, X, Y, ncolr, ldr, s, any);
  else sf_launch<6>(d, vq, kinetic, X, Y, ncolr, ldr, s, any);
}

}  // namespace k
}  // namespace efe
