// Host-side plan of the enriched spectral-FE discretisation (static data).
//
// Basis (Sec. 2.2-2.3 of the paper): degree-p Lagrange polynomials on GLL
// nodes per axis, uniform hex cells, homogeneous Dirichlet boundary; atom
// centred enrichment functions N^E = N^A - sum_l c_l N^C_l orthogonalised
// against the classical functions with the GLL-lumped classical mass, so
// c = D^-1 b with b_i = int N^C_i N^A (eq. (EFEOrtho)); overlap
// M = diag(D, M^ee), M^ee = M^AA - b^T D^-1 b (eq. (M)); Loewdin factor
// S = (M^ee)^-1/2 by eigendecomposition (eq. (MSquareRoot)), canonical when
// an eigenvalue falls below drop_tol * max.
//
// Integrals that involve enrichment functions use the (2p+2)^3 Gauss rule on
// every cell within r_cut of an atom; other Hamiltonian integrals use the
// (p+1)^3 Gauss rule (fixed rules in place of the adaptive quadrature of
// Sec. 2.4).  All cell integrals are evaluated by sum factorisation.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

namespace efe {

namespace {

constexpr double kPi = 3.14159265358979323846;

void parallel_for(int64_t n, const std::function<void(int64_t)> &fn) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 2 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int64_t> next(0);
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= n) break;
        fn(i);
      }
    });
  for (auto &x : th) x.join();
}

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double &Pn, double &dPn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { Pn = 1.0; dPn = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1; p1 = p2;
  }
  Pn = p1;
  // derivative from (x^2 - 1) P_n' = n (x P_n - P_{n-1})
  dPn = (std::fabs(x * x - 1.0) > 1e-300) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.0;
}

void gll_rule(int p, std::vector<double> &x, std::vector<double> &w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  x[0] = -1.0; x[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    double t = -std::cos(kPi * j / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, t, P, dP);
      double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
      double dt = dP / d2P;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[j] = t;
  }
  for (int j = 0; j <= p; ++j) {
    double P, dP;
    legendre(p, x[j], P, dP);
    w[j] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

void gauss_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double t = -std::cos(kPi * (j + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, P, dP);
      double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(n, t, P, dP);
    x[j] = t;
    w[j] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
}

// Lagrange basis on `nodes` at points `pts`: V[i][a], dV[i][a].
void lagrange(const std::vector<double> &nodes, const std::vector<double> &pts,
              std::vector<double> &V, std::vector<double> &dV) {
  int P = (int)nodes.size(), n = (int)pts.size();
  V.assign((size_t)n * P, 1.0);
  dV.assign((size_t)n * P, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = pts[i];
    for (int a = 0; a < P; ++a) {
      double v = 1.0;
      for (int b = 0; b < P; ++b)
        if (b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
      V[(size_t)i * P + a] = v;
      double d = 0.0;
      for (int c = 0; c < P; ++c) {
        if (c == a) continue;
        double t = 1.0 / (nodes[a] - nodes[c]);
        for (int b = 0; b < P; ++b)
          if (b != a && b != c) t *= (x - nodes[b]) / (nodes[a] - nodes[b]);
        d += t;
      }
      dV[(size_t)i * P + a] = d;
    }
  }
}

// nodal u[c][b][a] (P^3) -> point values f[k][j][i] (n^3); tables T*[n][P].
void interp3(int P, int n, const double *Tx, const double *Ty, const double *Tz, const double *u,
             double *f, std::vector<double> &w1, std::vector<double> &w2) {
  w1.resize((size_t)P * P * n);
  w2.resize((size_t)P * n * n);
  for (int cb = 0; cb < P * P; ++cb)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int a = 0; a < P; ++a) s += Tx[i * P + a] * u[cb * P + a];
      w1[(size_t)cb * n + i] = s;
    }
  for (int c = 0; c < P; ++c)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int b = 0; b < P; ++b) s += Ty[j * P + b] * w1[((size_t)c * P + b) * n + i];
        w2[((size_t)c * n + j) * n + i] = s;
      }
  for (int k = 0; k < n; ++k)
    for (int ji = 0; ji < n * n; ++ji) {
      double s = 0.0;
      for (int c = 0; c < P; ++c) s += Tz[k * P + c] * w2[(size_t)c * n * n + ji];
      f[(size_t)k * n * n + ji] = s;
    }
}

// transpose: point values f[k][j][i] -> nodal u[c][b][a] = sum T_x T_y T_z f
void project3(int P, int n, const double *Tx, const double *Ty, const double *Tz, const double *f,
              double *u, std::vector<double> &w1, std::vector<double> &w2) {
  w1.resize((size_t)n * n * P);
  w2.resize((size_t)n * P * P);
  for (int kj = 0; kj < n * n; ++kj)
    for (int a = 0; a < P; ++a) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += Tx[i * P + a] * f[(size_t)kj * n + i];
      w1[(size_t)kj * P + a] = s;
    }
  for (int k = 0; k < n; ++k)
    for (int b = 0; b < P; ++b)
      for (int a = 0; a < P; ++a) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += Ty[j * P + b] * w1[((size_t)k * n + j) * P + a];
        w2[((size_t)k * P + b) * P + a] = s;
      }
  for (int c = 0; c < P; ++c)
    for (int ba = 0; ba < P * P; ++ba) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += Tz[k * P + c] * w2[(size_t)k * P * P + ba];
      u[(size_t)c * P * P + ba] = s;
    }
}

}  // namespace

// Cyclic Jacobi eigendecomposition of a symmetric matrix (row-major n x n).
// evals ascending; evecs column j = eigenvector j (row-major storage).
void sym_eig(int n, std::vector<double> A, std::vector<double> &evals, std::vector<double> &evecs) {
  std::vector<double> V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
      for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = cs * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = cs * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
  evals.resize(n);
  evecs.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    evals[j] = A[(size_t)idx[j] * n + idx[j]];
    for (int i = 0; i < n; ++i) evecs[(size_t)i * n + j] = V[(size_t)i * n + idx[j]];
  }
}

bool Plan::is_boundary(int64_t node) const {
  int64_t g0 = node % nn[0], g1 = (node / nn[0]) % nn[1], g2 = node / (nn[0] * nn[1]);
  return g0 == 0 || g1 == 0 || g2 == 0 || g0 == nn[0] - 1 || g1 == nn[1] - 1 || g2 == nn[2] - 1;
}

void Plan::cell_nodes(int64_t c, int64_t *out) const {
  int e[3];
  cell_ijk(c, e);
  int k = 0;
  for (int cz = 0; cz < P; ++cz)
    for (int by = 0; by < P; ++by)
      for (int ax = 0; ax < P; ++ax)
        out[k++] = node_index((int64_t)e[0] * p + ax, (int64_t)e[1] * p + by, (int64_t)e[2] * p + cz);
}

double Plan::node_coord(int d, int64_t g) const {
  int64_t e = std::min<int64_t>(g / p, nc[d] - 1);
  int64_t a = g - e * p;
  return cell_lo(d, (int)e) + (xg[a] + 1.0) * 0.5 * cell_h(d, (int)e);
}

// Atomic part of enrichment function nu (unnormalised): r^l exp(-zeta r) Y_lm(rhat) u(r),
// u = (1 - (r/rc)^2)^3 inside rc, with Y_00 = 1/sqrt(4 pi), r Y_1m = sqrt(3/(4 pi)) (y, z, x).
double atomic_value(const Plan &pl, int nu, const double x[3], double grad[3]) {
  const double *R = &pl.R[3 * pl.enr_atom[nu]];
  double d[3] = {x[0] - R[0], x[1] - R[1], x[2] - R[2]};
  double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (grad) grad[0] = grad[1] = grad[2] = 0.0;
  if (r >= pl.rc) return 0.0;
  double s = 1.0 - (r / pl.rc) * (r / pl.rc);
  double u = s * s * s, du = -6.0 * r / (pl.rc * pl.rc) * s * s;
  double e = std::exp(-pl.enr_zeta[nu] * r);
  double g = e * u, dg = e * (du - pl.enr_zeta[nu] * u);
  double rh[3] = {0.0, 0.0, 0.0};
  if (r > 0.0) { rh[0] = d[0] / r; rh[1] = d[1] / r; rh[2] = d[2] / r; }
  if (pl.enr_l[nu] == 0) {
    const double Y = 0.28209479177387814;  // 1/sqrt(4 pi)
    if (grad) for (int k = 0; k < 3; ++k) grad[k] = Y * dg * rh[k];
    return Y * g;
  }
  const double Y1 = 0.4886025119029199;    // sqrt(3/(4 pi))
  int comp = pl.enr_m[nu] == -1 ? 1 : (pl.enr_m[nu] == 0 ? 2 : 0);
  if (grad) {
    for (int k = 0; k < 3; ++k) grad[k] = Y1 * d[comp] * dg * rh[k];
    grad[comp] += Y1 * g;
  }
  return Y1 * d[comp] * g;
}

namespace {

double box_dist2(const Plan &pl, int64_t c, const double *R) {
  int e[3];
  pl.cell_ijk(c, e);
  double d2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double lo = pl.cell_lo(d, e[d]), hi = lo + pl.cell_h(d, e[d]);
    double gap = std::max(std::max(lo - R[d], R[d] - hi), 0.0);
    d2 += gap * gap;
  }
  return d2;
}

// Point coordinates and weights of cell c's Gauss rule.
void cell_points(const Plan &pl, int64_t c, std::vector<double> &X, std::vector<double> &W) {
  int e[3];
  pl.cell_ijk(c, e);
  int n = pl.n1d(c);
  const std::vector<double> &xq = pl.is_enr[c] ? pl.xqe : pl.xqc;
  const std::vector<double> &wq = pl.is_enr[c] ? pl.wqe : pl.wqc;
  X.resize((size_t)3 * n * n * n);
  W.resize((size_t)n * n * n);
  const double h[3] = {pl.cell_h(0, e[0]), pl.cell_h(1, e[1]), pl.cell_h(2, e[2])};
  const double l[3] = {pl.cell_lo(0, e[0]), pl.cell_lo(1, e[1]), pl.cell_lo(2, e[2])};
  double jac = 0.125 * h[0] * h[1] * h[2];
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t q = (size_t)i + n * (j + (size_t)n * k);
        X[3 * q + 0] = l[0] + (xq[i] + 1.0) * 0.5 * h[0];
        X[3 * q + 1] = l[1] + (xq[j] + 1.0) * 0.5 * h[1];
        X[3 * q + 2] = l[2] + (xq[k] + 1.0) * 0.5 * h[2];
        W[q] = jac * wq[i] * wq[j] * wq[k];
      }
}

}  // namespace

efe_status build_plan(const efe_system &s, Plan &pl) {
  // ---- validation --------------------------------------------------------
  for (int d = 0; d < 3; ++d) {
    if (s.ncell[d] < 1 || s.ncell[d] > 4096 || !(s.hi[d] > s.lo[d])) {
      pl.error = "invalid mesh: ncell must be 1..4096 and hi > lo";
      return EFE_ERR_ARG;
    }
  }
  if (s.cell_bounds) {
    const double *b = s.cell_bounds;
    for (int d = 0; d < 3; ++d) {
      for (int e = 0; e <= s.ncell[d]; ++e)
        if (!std::isfinite(b[e])) { pl.error = "non-finite cell bounds"; return EFE_ERR_NONFINITE; }
      bool ok = b[0] == s.lo[d] && b[s.ncell[d]] == s.hi[d];
      for (int e = 0; e < s.ncell[d]; ++e) ok = ok && b[e + 1] > b[e];
      if (!ok) {
        pl.error = "cell bounds must increase strictly from lo to hi on every axis";
        return EFE_ERR_ARG;
      }
      b += s.ncell[d] + 1;
    }
  }
  if (s.degree < 2 || s.degree > 6) { pl.error = "degree must be 2..6"; return EFE_ERR_ARG; }
  if (s.natom < 0 || (s.natom > 0 && (!s.R || !s.Z))) { pl.error = "invalid atoms"; return EFE_ERR_ARG; }
  if (s.nenr < 0 || (s.nenr > 0 && (!s.enr_atom || !s.enr_l || !s.enr_m || !s.enr_zeta))) {
    pl.error = "invalid enrichment arrays"; return EFE_ERR_ARG;
  }
  if (s.norb < 0 || s.norb > 128 || (s.norb > 0 && !s.occ)) { pl.error = "norb must be 0..128"; return EFE_ERR_ARG; }
  if (s.xc < 0 || s.xc > 2) { pl.error = "invalid xc kind"; return EFE_ERR_ARG; }
  if (!(s.nuc_sigma > 0.0) && s.natom > 0) { pl.error = "nuc_sigma must be > 0"; return EFE_ERR_ARG; }
  for (int a = 0; a < s.natom; ++a)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(s.R[3 * a + d]) || !std::isfinite(s.Z[a])) { pl.error = "non-finite atom data"; return EFE_ERR_NONFINITE; }
  for (int v = 0; v < s.nenr; ++v) {
    if (s.enr_atom[v] < 0 || s.enr_atom[v] >= s.natom) { pl.error = "enr_atom out of range"; return EFE_ERR_ARG; }
    if (s.enr_l[v] < 0 || s.enr_l[v] > 1) { pl.error = "only l = 0, 1 enrichment"; return EFE_ERR_ARG; }
    if (s.enr_l[v] == 1 && (s.enr_m[v] < -1 || s.enr_m[v] > 1)) { pl.error = "invalid enr_m"; return EFE_ERR_ARG; }
    if (!(s.enr_zeta[v] > 0.0) || !std::isfinite(s.enr_zeta[v])) { pl.error = "enr_zeta must be > 0"; return EFE_ERR_ARG; }
  }
  if (s.nenr > 0 && !(s.r_cut > 0.0)) { pl.error = "r_cut must be > 0"; return EFE_ERR_ARG; }
  int qc = s.quad_cell > 0 ? s.quad_cell : s.degree + 1;
  int qe = s.quad_enr > 0 ? s.quad_enr : 2 * s.degree + 2;
  if (qc < s.degree + 1 || qc > kMaxQ || qe < s.degree + 1 || qe > kMaxQ) {
    pl.error = "quadrature sizes must be degree+1 .. 16"; return EFE_ERR_ARG;
  }

  // ---- copy --------------------------------------------------------------
  pl.p = s.degree; pl.P = s.degree + 1; pl.nloc = pl.P * pl.P * pl.P;
  for (int d = 0; d < 3; ++d) {
    pl.nc[d] = s.ncell[d]; pl.lo[d] = s.lo[d]; pl.hi[d] = s.hi[d];
    pl.xb[d].resize((size_t)s.ncell[d] + 1);
    const double h = (s.hi[d] - s.lo[d]) / s.ncell[d];
    for (int e = 0; e <= s.ncell[d]; ++e) pl.xb[d][e] = s.lo[d] + e * h;
    if (s.cell_bounds) {
      const double *b = s.cell_bounds + (d > 0 ? s.ncell[0] + 1 : 0) + (d > 1 ? s.ncell[1] + 1 : 0);
      pl.xb[d].assign(b, b + s.ncell[d] + 1);
    }
    pl.nn[d] = (int64_t)s.ncell[d] * pl.p + 1;
  }
  pl.n_nodes = pl.nn[0] * pl.nn[1] * pl.nn[2];
  pl.n_cells = (int64_t)pl.nc[0] * pl.nc[1] * pl.nc[2];
  pl.natom = s.natom;
  pl.R.assign(s.R, s.R + 3 * s.natom);
  pl.Z.assign(s.Z, s.Z + s.natom);
  pl.sigma = s.nuc_sigma;
  pl.nenr = s.nenr;
  pl.enr_atom.assign(s.enr_atom, s.enr_atom + s.nenr);
  pl.enr_l.assign(s.enr_l, s.enr_l + s.nenr);
  pl.enr_m.assign(s.enr_m, s.enr_m + s.nenr);
  pl.enr_zeta.assign(s.enr_zeta, s.enr_zeta + s.nenr);
  pl.rc = s.r_cut;
  pl.norb = s.norb;
  pl.occ.assign(s.occ, s.occ + s.norb);
  pl.n_electrons = 0.0;
  for (double f : pl.occ) pl.n_electrons += f;
  pl.xc = s.xc;
  pl.trap_omega = s.trap_omega;
  pl.qc = qc; pl.qe = qe;
  pl.drop_tol = s.enr_drop_tol > 0 ? s.enr_drop_tol : 1e-8;
  const int P = pl.P, p = pl.p;

  // ---- tables ------------------------------------------------------------
  gll_rule(p, pl.xg, pl.wg);
  gauss_rule(qc, pl.xqc, pl.wqc);
  gauss_rule(qe, pl.xqe, pl.wqe);
  lagrange(pl.xg, pl.xqc, pl.Bc, pl.dBc);
  lagrange(pl.xg, pl.xqe, pl.Be, pl.dBe);
  {
    std::vector<double> xe, we, V, dV;
    gauss_rule(P, xe, we);
    lagrange(pl.xg, xe, V, dV);
    pl.Kref.assign((size_t)P * P, 0.0);
    pl.Mref.assign((size_t)P * P, 0.0);
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b) {
        double k = 0, m = 0;
        for (int q = 0; q < P; ++q) {
          k += we[q] * dV[q * P + a] * dV[q * P + b];
          m += we[q] * V[q * P + a] * V[q * P + b];
        }
        pl.Kref[a * P + b] = k;
        pl.Mref[a * P + b] = m;
      }
  }

  // ---- cell classes --------------------------------------------------------
  const int64_t NC = pl.n_cells;
  std::vector<std::vector<uint8_t>> eset(pl.natom, std::vector<uint8_t>(NC, 0));
  std::vector<std::vector<uint8_t>> tset(pl.natom, std::vector<uint8_t>(NC, 0));
  pl.is_enr.assign(NC, 0);
  if (pl.nenr > 0) {
    std::vector<uint8_t> atom_used(pl.natom, 0);
    for (int v = 0; v < pl.nenr; ++v) atom_used[pl.enr_atom[v]] = 1;
    for (int a = 0; a < pl.natom; ++a) {
      if (!atom_used[a]) continue;
      for (int64_t c = 0; c < NC; ++c)
        if (box_dist2(pl, c, &pl.R[3 * a]) < pl.rc * pl.rc) { eset[a][c] = 1; pl.is_enr[c] = 1; }
      for (int64_t c = 0; c < NC; ++c) {
        if (!eset[a][c]) continue;
        int e[3];
        pl.cell_ijk(c, e);
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int f[3] = {e[0] + dx, e[1] + dy, e[2] + dz};
              if (f[0] < 0 || f[1] < 0 || f[2] < 0 || f[0] >= pl.nc[0] || f[1] >= pl.nc[1] || f[2] >= pl.nc[2]) continue;
              tset[a][f[0] + (int64_t)pl.nc[0] * (f[1] + (int64_t)pl.nc[1] * f[2])] = 1;
            }
      }
    }
  }
  pl.q_off.assign(NC + 1, 0);
  for (int64_t c = 0; c < NC; ++c) {
    int n = pl.n1d(c);
    pl.q_off[c + 1] = pl.q_off[c] + (int64_t)n * n * n;
  }
  pl.n_quad = pl.q_off[NC];

  // ---- lumped mass -------------------------------------------------------------
  pl.D.assign(pl.n_nodes, 0.0);
  {
    std::vector<int64_t> nodes(pl.nloc);
    for (int64_t c = 0; c < NC; ++c) {
      int e[3];
      pl.cell_ijk(c, e);
      const double jac = 0.125 * pl.cell_h(0, e[0]) * pl.cell_h(1, e[1]) * pl.cell_h(2, e[2]);
      pl.cell_nodes(c, nodes.data());
      for (int cz = 0; cz < P; ++cz)
        for (int by = 0; by < P; ++by)
          for (int ax = 0; ax < P; ++ax)
            pl.D[nodes[ax + P * (by + P * cz)]] += jac * pl.wg[ax] * pl.wg[by] * pl.wg[cz];
    }
  }

  // ---- static potential at quadrature points ----------------------------------
  pl.vstatic.assign(pl.n_quad, 0.0);
  parallel_for(NC, [&](int64_t c) {
    std::vector<double> X, W;
    cell_points(pl, c, X, W);
    int64_t nq = (int64_t)W.size();
    for (int64_t q = 0; q < nq; ++q) {
      const double *x = &X[3 * q];
      double v = 0.0;
      for (int a = 0; a < pl.natom; ++a) {
        double dx = x[0] - pl.R[3 * a], dy = x[1] - pl.R[3 * a + 1], dz = x[2] - pl.R[3 * a + 2];
        double r = std::sqrt(dx * dx + dy * dy + dz * dz);
        v -= pl.Z[a] * (r > 1e-12 ? std::erf(r / pl.sigma) / r : 2.0 / (pl.sigma * std::sqrt(kPi)));
      }
      if (pl.trap_omega > 0) v += 0.5 * pl.trap_omega * pl.trap_omega * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      pl.vstatic[pl.q_off[c] + q] = v;
    }
  });

  // ---- enrichment --------------------------------------------------------------
  const int ne = pl.nenr;
  pl.tslot_of_cell.assign(NC, -1);
  pl.tcell.clear();
  pl.tnu_off.assign(1, 0);
  pl.tnu.clear();
  pl.tnu_has_atomic.clear();
  for (int64_t c = 0; c < NC && ne > 0; ++c) {
    int cnt = 0;
    for (int v = 0; v < ne; ++v) {
      int a = pl.enr_atom[v];
      if (tset[a][c]) {
        pl.tnu.push_back(v);
        pl.tnu_has_atomic.push_back(eset[a][c]);
        ++cnt;
      }
    }
    if (cnt > 0) {
      pl.tslot_of_cell[c] = (int)pl.tcell.size();
      pl.tcell.push_back((int)c);
      pl.tnu_off.push_back(pl.tnu_off.back() + cnt);
    }
  }
  const int NT = (int)pl.tcell.size();
  if (NT >= (1 << (31 - kPairShift))) { pl.error = "too many enrichment cells for the union-row pairs"; return EFE_ERR_ARG; }
  pl.node_urow.assign(pl.n_nodes, -1);
  pl.urow_node.clear();
  {
    std::vector<int64_t> nodes(pl.nloc);
    std::vector<uint8_t> mark(pl.n_nodes, 0);
    for (int t = 0; t < NT; ++t) {
      pl.cell_nodes(pl.tcell[t], nodes.data());
      for (int64_t i : nodes)
        if (!pl.is_boundary(i)) mark[i] = 1;
    }
    for (int64_t i = 0; i < pl.n_nodes; ++i)
      if (mark[i]) { pl.node_urow[i] = (int)pl.urow_node.size(); pl.urow_node.push_back(i); }
  }
  const int64_t NR = pl.n_urows();
  pl.urow_cnt.assign(NR, 0);
  pl.urow_pair.assign(NR * 8, -1);
  {
    std::vector<int64_t> nodes(pl.nloc);
    for (int t = 0; t < NT; ++t) {
      pl.cell_nodes(pl.tcell[t], nodes.data());
      for (int l = 0; l < pl.nloc; ++l) {
        int r = pl.node_urow[nodes[l]];
        if (r < 0) continue;
        pl.urow_pair[(size_t)r * 8 + pl.urow_cnt[r]++] = (t << kPairShift) | l;
      }
    }
  }
  pl.tne_off.assign(NT + 1, 0);
  pl.ta_off.assign(NT + 1, 0);
  pl.ta_nu.clear();
  pl.tna_off.assign(NT + 1, 0);
  for (int t = 0; t < NT; ++t) {
    int n = pl.n1d(pl.tcell[t]);
    pl.tne_off[t + 1] = pl.tne_off[t] + (int64_t)n * n * n * (pl.tnu_off[t + 1] - pl.tnu_off[t]);
    for (int k = pl.tnu_off[t]; k < pl.tnu_off[t + 1]; ++k)
      if (pl.tnu_has_atomic[k]) pl.ta_nu.push_back(pl.tnu[k]);
    pl.ta_off[t + 1] = (int)pl.ta_nu.size();
    pl.tna_off[t + 1] = pl.tna_off[t] + (int64_t)n * n * n * (pl.ta_off[t + 1] - pl.ta_off[t]);
  }

  pl.enr_scale.assign(ne, 0.0);
  pl.b.assign(NR * ne, 0.0);
  pl.c.assign(NR * ne, 0.0);
  pl.MAA.assign((size_t)ne * ne, 0.0);
  pl.Mee.assign((size_t)ne * ne, 0.0);
  pl.Kce.assign(NR * ne, 0.0);
  pl.Kee.assign((size_t)ne * ne, 0.0);
  pl.NE.assign(pl.tne_off[NT], 0.0);
  pl.NA.assign(pl.tna_off[NT], 0.0);
  pl.nk = 0; pl.ndrop = 0;

  if (ne > 0) {
    // pass 1: norms of the atomic parts (per-slot partials, reduced in slot order)
    std::vector<double> norm_part((size_t)NT * ne, 0.0);
    parallel_for(NT, [&](int64_t t) {
      int64_t c = pl.tcell[t];
      if (!pl.is_enr[c]) return;
      std::vector<double> X, W;
      cell_points(pl, c, X, W);
      for (int k = pl.tnu_off[t]; k < pl.tnu_off[t + 1]; ++k) {
        if (!pl.tnu_has_atomic[k]) continue;
        int v = pl.tnu[k];
        double s = 0.0;
        for (size_t q = 0; q < W.size(); ++q) {
          double a = atomic_value(pl, v, &X[3 * q], nullptr);
          s += W[q] * a * a;
        }
        norm_part[(size_t)t * ne + v] = s;
      }
    });
    for (int v = 0; v < ne; ++v) {
      double s = 0.0;
      for (int t = 0; t < NT; ++t) s += norm_part[(size_t)t * ne + v];
      if (!(s > 0.0)) { pl.error = "an enrichment function vanishes on the mesh"; return EFE_ERR_SINGULAR; }
      pl.enr_scale[v] = 1.0 / std::sqrt(s);
    }

    // pass 2: b (cell-local partials) and M^AA
    std::vector<double> bpart((size_t)NT * pl.nloc * ne, 0.0);
    std::vector<double> maa_part((size_t)NT * ne * ne, 0.0);
    parallel_for(NT, [&](int64_t t) {
      int64_t c = pl.tcell[t];
      if (!pl.is_enr[c]) return;
      std::vector<double> X, W, w1, w2;
      cell_points(pl, c, X, W);
      int n = pl.qe;
      size_t nq = W.size();
      int k0 = pl.tnu_off[t], k1 = pl.tnu_off[t + 1];
      std::vector<double> NA((size_t)(k1 - k0) * nq, 0.0), f(nq), u(pl.nloc);
      for (int k = k0; k < k1; ++k) {
        if (!pl.tnu_has_atomic[k]) continue;
        int v = pl.tnu[k];
        for (size_t q = 0; q < nq; ++q) NA[(size_t)(k - k0) * nq + q] = pl.enr_scale[v] * atomic_value(pl, v, &X[3 * q], nullptr);
        for (size_t q = 0; q < nq; ++q) f[q] = W[q] * NA[(size_t)(k - k0) * nq + q];
        project3(P, n, pl.Be.data(), pl.Be.data(), pl.Be.data(), f.data(), u.data(), w1, w2);
        for (int l = 0; l < pl.nloc; ++l) bpart[((size_t)t * pl.nloc + l) * ne + v] = u[l];
      }
      for (int k = k0; k < k1; ++k)
        for (int kk = k0; kk < k1; ++kk) {
          if (!pl.tnu_has_atomic[k] || !pl.tnu_has_atomic[kk]) continue;
          double s = 0.0;
          for (size_t q = 0; q < nq; ++q) s += W[q] * NA[(size_t)(k - k0) * nq + q] * NA[(size_t)(kk - k0) * nq + q];
          maa_part[((size_t)t * ne + pl.tnu[k]) * ne + pl.tnu[kk]] = s;
        }
    });
    for (int64_t r = 0; r < NR; ++r)
      for (int k = 0; k < pl.urow_cnt[r]; ++k) {
        int pr = pl.urow_pair[(size_t)r * 8 + k];
        int t = pr >> kPairShift, l = pr & ((1 << kPairShift) - 1);
        for (int v = 0; v < ne; ++v) pl.b[(size_t)r * ne + v] += bpart[((size_t)t * pl.nloc + l) * ne + v];
      }
    for (int t = 0; t < NT; ++t)
      for (size_t i = 0; i < (size_t)ne * ne; ++i) pl.MAA[i] += maa_part[(size_t)t * ne * ne + i];
    std::vector<double>().swap(bpart);
    std::vector<double>().swap(maa_part);

    // c = D^-1 b and M^ee = M^AA - b^T D^-1 b
    for (int64_t r = 0; r < NR; ++r) {
      double Dr = pl.D[pl.urow_node[r]];
      for (int v = 0; v < ne; ++v) pl.c[(size_t)r * ne + v] = pl.b[(size_t)r * ne + v] / Dr;
    }
    pl.Mee = pl.MAA;
    for (int64_t r = 0; r < NR; ++r)
      for (int i = 0; i < ne; ++i) {
        double bi = pl.b[(size_t)r * ne + i];
        if (bi == 0.0) continue;
        for (int j = 0; j < ne; ++j) pl.Mee[(size_t)i * ne + j] -= bi * pl.c[(size_t)r * ne + j];
      }
    for (int i = 0; i < ne; ++i)          // exact symmetry
      for (int j = i + 1; j < ne; ++j) {
        double m = 0.5 * (pl.Mee[(size_t)i * ne + j] + pl.Mee[(size_t)j * ne + i]);
        pl.Mee[(size_t)i * ne + j] = pl.Mee[(size_t)j * ne + i] = m;
      }
    sym_eig(ne, pl.Mee, pl.Mee_eval, pl.Mee_evec);
    double lmax = pl.Mee_eval[ne - 1];
    if (!(lmax > 0.0)) { pl.error = "enrichment overlap M^ee has no positive eigenvalue"; return EFE_ERR_SINGULAR; }
    std::vector<int> keep;
    for (int j = 0; j < ne; ++j)
      if (pl.Mee_eval[j] > pl.drop_tol * lmax) keep.push_back(j);
    pl.nk = (int)keep.size();
    pl.ndrop = ne - pl.nk;
    pl.S.assign((size_t)ne * pl.nk, 0.0);
    pl.Splus.assign((size_t)pl.nk * ne, 0.0);
    const std::vector<double> &U = pl.Mee_evec;
    if (pl.ndrop == 0) {      // symmetric Loewdin: S = U L^-1/2 U^T, S^+ = U L^1/2 U^T
      for (int i = 0; i < ne; ++i)
        for (int j = 0; j < ne; ++j) {
          double s = 0.0, sp = 0.0;
          for (int k = 0; k < ne; ++k) {
            s += U[(size_t)i * ne + k] * U[(size_t)j * ne + k] / std::sqrt(pl.Mee_eval[k]);
            sp += U[(size_t)i * ne + k] * U[(size_t)j * ne + k] * std::sqrt(pl.Mee_eval[k]);
          }
          pl.S[(size_t)i * ne + j] = s;
          pl.Splus[(size_t)i * ne + j] = sp;
        }
    } else {                  // canonical: S = U_k L_k^-1/2, S^+ = L_k^1/2 U_k^T
      for (int kk = 0; kk < pl.nk; ++kk) {
        int k = keep[kk];
        for (int i = 0; i < ne; ++i) {
          pl.S[(size_t)i * pl.nk + kk] = U[(size_t)i * ne + k] / std::sqrt(pl.Mee_eval[k]);
          pl.Splus[(size_t)kk * ne + i] = U[(size_t)i * ne + k] * std::sqrt(pl.Mee_eval[k]);
        }
      }
    }

    // pass 3: N^E at T-cell points, static kinetic couplings
    std::vector<double> kce_part((size_t)NT * pl.nloc * ne, 0.0);
    std::vector<double> kee_part((size_t)NT * ne * ne, 0.0);
    parallel_for(NT, [&](int64_t t) {
      int64_t c = pl.tcell[t];
      std::vector<double> X, W, w1, w2;
      cell_points(pl, c, X, W);
      int n = pl.n1d(c);
      const double *Bt = pl.is_enr[c] ? pl.Be.data() : pl.Bc.data();
      const double *dBt = pl.is_enr[c] ? pl.dBe.data() : pl.dBc.data();
      std::vector<double> dBx((size_t)n * P), dBy((size_t)n * P), dBz((size_t)n * P);
      int ec[3];
      pl.cell_ijk(c, ec);
      for (size_t i = 0; i < dBx.size(); ++i) {
        dBx[i] = dBt[i] * 2.0 / pl.cell_h(0, ec[0]);
        dBy[i] = dBt[i] * 2.0 / pl.cell_h(1, ec[1]);
        dBz[i] = dBt[i] * 2.0 / pl.cell_h(2, ec[2]);
      }
      size_t nq = W.size();
      int k0 = pl.tnu_off[t], k1 = pl.tnu_off[t + 1], nv = k1 - k0;
      std::vector<int64_t> nodes(pl.nloc);
      pl.cell_nodes(c, nodes.data());
      std::vector<double> cc(pl.nloc), val(nq), grad(3 * nq * (size_t)nv), tmp(nq), u(pl.nloc);
      for (int k = k0; k < k1; ++k) {
        int v = pl.tnu[k];
        for (int l = 0; l < pl.nloc; ++l) {
          int r = pl.node_urow[nodes[l]];
          cc[l] = r >= 0 ? pl.c[(size_t)r * ne + v] : 0.0;
        }
        double *gx = &grad[(size_t)(k - k0) * 3 * nq], *gy = gx + nq, *gz = gy + nq;
        interp3(P, n, Bt, Bt, Bt, cc.data(), val.data(), w1, w2);
        interp3(P, n, dBx.data(), Bt, Bt, cc.data(), gx, w1, w2);
        interp3(P, n, Bt, dBy.data(), Bt, cc.data(), gy, w1, w2);
        interp3(P, n, Bt, Bt, dBz.data(), cc.data(), gz, w1, w2);
        for (size_t q = 0; q < nq; ++q) { val[q] = -val[q]; gx[q] = -gx[q]; gy[q] = -gy[q]; gz[q] = -gz[q]; }
        if (pl.tnu_has_atomic[k]) {
          int ai = 0;
          for (int kk = k0; kk < k; ++kk) ai += pl.tnu_has_atomic[kk];
          double *na = pl.NA.data() + pl.tna_off[t] + (int64_t)ai * nq;
          for (size_t q = 0; q < nq; ++q) {
            double g3[3];
            double a = atomic_value(pl, v, &X[3 * q], g3);
            na[q] = pl.enr_scale[v] * a;
            val[q] += pl.enr_scale[v] * a;
            gx[q] += pl.enr_scale[v] * g3[0];
            gy[q] += pl.enr_scale[v] * g3[1];
            gz[q] += pl.enr_scale[v] * g3[2];
          }
        }
        std::copy(val.begin(), val.end(), pl.NE.begin() + pl.tne_off[t] + (int64_t)(k - k0) * nq);
        // 1/2 int grad N_i . grad N^E_v
        std::fill(u.begin(), u.end(), 0.0);
        std::vector<double> acc(pl.nloc, 0.0);
        for (int d = 0; d < 3; ++d) {
          const double *g = d == 0 ? gx : (d == 1 ? gy : gz);
          for (size_t q = 0; q < nq; ++q) tmp[q] = 0.5 * W[q] * g[q];
          project3(P, n, d == 0 ? dBx.data() : Bt, d == 1 ? dBy.data() : Bt, d == 2 ? dBz.data() : Bt,
                   tmp.data(), u.data(), w1, w2);
          for (int l = 0; l < pl.nloc; ++l) acc[l] += u[l];
        }
        for (int l = 0; l < pl.nloc; ++l) kce_part[((size_t)t * pl.nloc + l) * ne + v] = acc[l];
      }
      for (int k = k0; k < k1; ++k)
        for (int kk = k0; kk < k1; ++kk) {
          const double *g1 = &grad[(size_t)(k - k0) * 3 * nq], *g2 = &grad[(size_t)(kk - k0) * 3 * nq];
          double s = 0.0;
          for (size_t q = 0; q < nq; ++q)
            s += W[q] * (g1[q] * g2[q] + g1[nq + q] * g2[nq + q] + g1[2 * nq + q] * g2[2 * nq + q]);
          kee_part[((size_t)t * ne + pl.tnu[k]) * ne + pl.tnu[kk]] = 0.5 * s;
        }
    });
    for (int64_t r = 0; r < NR; ++r)
      for (int k = 0; k < pl.urow_cnt[r]; ++k) {
        int pr = pl.urow_pair[(size_t)r * 8 + k];
        int t = pr >> kPairShift, l = pr & ((1 << kPairShift) - 1);
        for (int v = 0; v < ne; ++v) pl.Kce[(size_t)r * ne + v] += kce_part[((size_t)t * pl.nloc + l) * ne + v];
      }
    for (int t = 0; t < NT; ++t)
      for (size_t i = 0; i < (size_t)ne * ne; ++i) pl.Kee[i] += kee_part[(size_t)t * ne * ne + i];
  }

  // ---- Poisson: 1-D operators, FDM, boundary data ----------------------------
  for (int d = 0; d < 3; ++d) {
    int64_t n = pl.nn[d];
    pl.K1[d].assign((size_t)n * n, 0.0);
    pl.M1[d].assign((size_t)n * n, 0.0);
    for (int e = 0; e < pl.nc[d]; ++e) {
      const double h = pl.cell_h(d, e);
      for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
          pl.K1[d][(size_t)(e * p + a) * n + e * p + b] += pl.Kref[a * P + b] * 2.0 / h;
          pl.M1[d][(size_t)(e * p + a) * n + e * p + b] += pl.Mref[a * P + b] * 0.5 * h;
        }
    }
    int m = (int)n - 2;
    // generalised symmetric eigenproblem K v = lam M v on the interior, via M = L L^T
    std::vector<double> L((size_t)m * m, 0.0), K((size_t)m * m), C((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) K[(size_t)i * m + j] = pl.K1[d][(size_t)(i + 1) * n + j + 1];
    for (int j = 0; j < m; ++j) {
      double s = pl.M1[d][(size_t)(j + 1) * n + j + 1];
      for (int k = 0; k < j; ++k) s -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
      L[(size_t)j * m + j] = std::sqrt(s);
      for (int i = j + 1; i < m; ++i) {
        double t = pl.M1[d][(size_t)(i + 1) * n + j + 1];
        for (int k = 0; k < j; ++k) t -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
        L[(size_t)i * m + j] = t / L[(size_t)j * m + j];
      }
    }
    // Y = L^-1 K (forward substitution per column), C = L^-1 Y^T
    std::vector<double> Y((size_t)m * m);
    for (int col = 0; col < m; ++col)
      for (int i = 0; i < m; ++i) {
        double t = K[(size_t)i * m + col];
        for (int k = 0; k < i; ++k) t -= L[(size_t)i * m + k] * Y[(size_t)k * m + col];
        Y[(size_t)i * m + col] = t / L[(size_t)i * m + i];
      }
    for (int col = 0; col < m; ++col)
      for (int i = 0; i < m; ++i) {
        double t = Y[(size_t)col * m + i];
        for (int k = 0; k < i; ++k) t -= L[(size_t)i * m + k] * C[(size_t)k * m + col];
        C[(size_t)i * m + col] = t / L[(size_t)i * m + i];
      }
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) {
        double s = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
        C[(size_t)i * m + j] = C[(size_t)j * m + i] = s;
      }
    std::vector<double> lam, Wv;
    sym_eig(m, C, lam, Wv);
    // V = L^-T W (back substitution)
    pl.fdmV[d].assign((size_t)m * m, 0.0);
    for (int col = 0; col < m; ++col)
      for (int i = m - 1; i >= 0; --i) {
        double t = Wv[(size_t)i * m + col];
        for (int k = i + 1; k < m; ++k) t -= L[(size_t)k * m + i] * pl.fdmV[d][(size_t)k * m + col];
        pl.fdmV[d][(size_t)i * m + col] = t / L[(size_t)i * m + i];
      }
    pl.fdmL[d] = lam;
  }
  pl.gbnd.assign(pl.n_nodes, 0.0);
  double ztot = 0.0;
  for (double z : pl.Z) ztot += z;
  for (int64_t i = 0; i < pl.n_nodes; ++i) {
    if (!pl.is_boundary(i)) continue;
    int64_t g0 = i % pl.nn[0], g1 = (i / pl.nn[0]) % pl.nn[1], g2 = i / (pl.nn[0] * pl.nn[1]);
    double x[3] = {pl.node_coord(0, g0), pl.node_coord(1, g1), pl.node_coord(2, g2)};
    double g = 0.0;
    if (pl.n_electrons != 0.0) {
      if (pl.natom == 0 || ztot == 0.0) {
        g = pl.n_electrons / std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      } else {
        for (int a = 0; a < pl.natom; ++a) {
          double dx = x[0] - pl.R[3 * a], dy = x[1] - pl.R[3 * a + 1], dz = x[2] - pl.R[3 * a + 2];
          g += pl.Z[a] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
        g *= pl.n_electrons / ztot;
      }
    }
    pl.gbnd[i] = g;
  }
  // lift = K g restricted to interior rows, K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1
  pl.lift.assign(pl.n_nodes, 0.0);
  {
    const int64_t n0 = pl.nn[0], n1 = pl.nn[1], n2 = pl.nn[2];
    auto apply_axis = [&](const std::vector<double> &A, int axis, const std::vector<double> &in,
                          std::vector<double> &out) {
      out.assign(in.size(), 0.0);
      int64_t n = pl.nn[axis];
      parallel_for(n2, [&](int64_t z) {
        for (int64_t y = 0; y < n1; ++y)
          for (int64_t x = 0; x < n0; ++x) {
            int64_t g[3] = {x, y, z};
            int64_t gi = g[axis];
            int64_t lo = std::max<int64_t>(0, gi - p), hi = std::min<int64_t>(n - 1, gi + p);
            double s = 0.0;
            for (int64_t k = lo; k <= hi; ++k) {
              int64_t h2[3] = {x, y, z};
              h2[axis] = k;
              s += A[(size_t)gi * n + k] * in[h2[0] + n0 * (h2[1] + n1 * h2[2])];
            }
            out[x + n0 * (y + n1 * z)] = s;
          }
      });
    };
    std::vector<double> t1, t2, t3;
    for (int term = 0; term < 3; ++term) {
      apply_axis(term == 0 ? pl.K1[0] : pl.M1[0], 0, pl.gbnd, t1);
      apply_axis(term == 1 ? pl.K1[1] : pl.M1[1], 1, t1, t2);
      apply_axis(term == 2 ? pl.K1[2] : pl.M1[2], 2, t2, t3);
      for (int64_t i = 0; i < pl.n_nodes; ++i) pl.lift[i] += t3[i];
    }
    for (int64_t i = 0; i < pl.n_nodes; ++i)
      if (pl.is_boundary(i)) pl.lift[i] = 0.0;
  }
  return EFE_OK;
}

efe_status initial_state(const Plan &pl, const int32_t *enr_index, const double *g, double amp,
                         std::vector<double> &X) {
  const int no = pl.norb, ne = pl.nenr, nk = pl.nk;
  const int64_t NN = pl.n_nodes, nrows = NN + nk;
  for (int a = 0; a < no; ++a)
    if (enr_index[a] < 0 || enr_index[a] >= ne) return EFE_ERR_ARG;
  X.assign((size_t)nrows * no, 0.0);
  // per-axis sine tables sin(m pi (x - lo)/(hi - lo)), m = 1..3
  std::vector<double> sn[3];
  for (int d = 0; d < 3; ++d) {
    sn[d].assign((size_t)pl.nn[d] * 3, 0.0);
    for (int64_t gi = 0; gi < pl.nn[d]; ++gi) {
      double x = pl.node_coord(d, gi);
      for (int m = 1; m <= 3; ++m)
        sn[d][(size_t)gi * 3 + m - 1] = std::sin(m * kPi * (x - pl.lo[d]) / (pl.hi[d] - pl.lo[d]));
    }
  }
  std::vector<double> nrm2((size_t)pl.nn[2] * no, 0.0);
  parallel_for(pl.nn[2], [&](int64_t z) {
    for (int64_t y = 0; y < pl.nn[1]; ++y)
      for (int64_t x = 0; x < pl.nn[0]; ++x) {
        int64_t i = pl.node_index(x, y, z);
        if (pl.is_boundary(i)) continue;
        for (int a = 0; a < no; ++a) {
          double f = 0.0;
          int k = 0;
          for (int mx = 0; mx < 3; ++mx)
            for (int my = 0; my < 3; ++my)
              for (int mz = 0; mz < 3; ++mz, ++k)
                f += g[(size_t)a * kNoiseModes + k] * sn[0][x * 3 + mx] * sn[1][y * 3 + my] * sn[2][z * 3 + mz];
          X[(size_t)i * no + a] = f;
          nrm2[(size_t)z * no + a] += pl.D[i] * f * f;
        }
      }
  });
  for (int a = 0; a < no; ++a) {
    double s = 0.0;
    for (int64_t z = 0; z < pl.nn[2]; ++z) s += nrm2[(size_t)z * no + a];
    if (!(s > 0.0)) return EFE_ERR_ARG;
    double scale = amp / std::sqrt(s);
    for (int64_t i = 0; i < NN; ++i) X[(size_t)i * no + a] *= std::sqrt(pl.D[i]) * scale;
    for (int k = 0; k < nk; ++k) X[(size_t)(NN + k) * no + a] = pl.Splus[(size_t)k * ne + enr_index[a]];
  }
  // X <- X (X^T X)^-1/2
  std::vector<double> G((size_t)no * no, 0.0);
  {
    const int64_t chunk = 4096;
    int64_t nch = (nrows + chunk - 1) / chunk;
    std::vector<double> part((size_t)nch * no * no, 0.0);
    parallel_for(nch, [&](int64_t ch) {
      double *Gp = &part[(size_t)ch * no * no];
      for (int64_t r = ch * chunk; r < std::min(nrows, (ch + 1) * chunk); ++r)
        for (int a = 0; a < no; ++a) {
          double xa = X[(size_t)r * no + a];
          if (xa == 0.0) continue;
          for (int b = 0; b < no; ++b) Gp[a * no + b] += xa * X[(size_t)r * no + b];
        }
    });
    for (int64_t ch = 0; ch < nch; ++ch)
      for (size_t i = 0; i < (size_t)no * no; ++i) G[i] += part[(size_t)ch * no * no + i];
  }
  std::vector<double> lam, V;
  sym_eig(no, G, lam, V);
  if (!(lam[0] > 0.0)) return EFE_ERR_SINGULAR;
  std::vector<double> T((size_t)no * no, 0.0);
  for (int a = 0; a < no; ++a)
    for (int b = 0; b < no; ++b) {
      double s = 0.0;
      for (int k = 0; k < no; ++k) s += V[(size_t)a * no + k] * V[(size_t)b * no + k] / std::sqrt(lam[k]);
      T[(size_t)a * no + b] = s;
    }
  parallel_for((nrows + 4095) / 4096, [&](int64_t ch) {
    std::vector<double> row(no);
    for (int64_t r = ch * 4096; r < std::min(nrows, (ch + 1) * 4096); ++r) {
      for (int b = 0; b < no; ++b) {
        double s = 0.0;
        for (int a = 0; a < no; ++a) s += X[(size_t)r * no + a] * T[(size_t)a * no + b];
        row[b] = s;
      }
      for (int b = 0; b < no; ++b) X[(size_t)r * no + b] = row[b];
    }
  });
  return EFE_OK;
}

}  // namespace efe
