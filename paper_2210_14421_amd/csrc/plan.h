// Host-side plan of the enriched spectral-FE discretisation: every quantity
// that does not change during propagation.  Pure C++17, no HIP.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "efe.h"

namespace efe {

constexpr int kMaxP = 7;          // degree <= 6
constexpr int kMaxQ = 16;         // Gauss points per axis
constexpr int kPairShift = 9;     // union-row pair: slot << kPairShift | local node (nloc <= 343 < 512)
constexpr int kNoiseModes = 27;

struct Plan {
  // ---- system -------------------------------------------------------------
  int nc[3] = {0, 0, 0};
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  std::vector<double> xb[3];             // cell boundaries per axis (nc[d] + 1, increasing)
  int p = 0, P = 0, nloc = 0;
  int64_t nn[3] = {0, 0, 0};
  int64_t n_nodes = 0, n_cells = 0;
  int natom = 0;
  std::vector<double> R, Z;
  double sigma = 0.2;
  int nenr = 0;
  std::vector<int> enr_atom, enr_l, enr_m;
  std::vector<double> enr_zeta;
  double rc = 6.0;
  int norb = 0;
  std::vector<double> occ;
  int xc = 0;
  double trap_omega = 0.0;
  int qc = 0, qe = 0;
  double drop_tol = 1e-8;
  double n_electrons = 0.0;

  // ---- 1-D tables (reference cell [-1, 1]) ---------------------------------
  std::vector<double> xg, wg;            // GLL nodes/weights (P)
  std::vector<double> xqc, wqc, xqe, wqe;  // Gauss rules (qc, qe)
  std::vector<double> Bc, dBc, Be, dBe;  // Lagrange values/derivatives [n][P], d/dxi
  // exact 1-D element matrices of the reference cell [P*P]: int dphi_a dphi_b, int phi_a phi_b;
  // a cell of edge h along an axis has (2/h) Kref and (h/2) Mref there
  std::vector<double> Kref, Mref;

  // ---- cells ----------------------------------------------------------------
  std::vector<uint8_t> is_enr;           // n_cells
  std::vector<int64_t> q_off;            // n_cells + 1
  int64_t n_quad = 0;
  std::vector<double> D;                 // lumped GLL mass per node
  std::vector<double> vstatic;           // v_N + v_trap at every quadrature point

  // ---- enrichment -----------------------------------------------------------
  std::vector<double> enr_scale;         // 1/norm of each atomic part
  std::vector<int> tcell;                // T-cells (some N^E nonzero), sorted
  std::vector<int> tslot_of_cell;        // n_cells, -1 if not a T-cell
  std::vector<int> tnu_off, tnu;         // per slot: relevant enrichment indices
  std::vector<uint8_t> tnu_has_atomic;   // per (slot, nu): cell in the atom's cutoff set
  std::vector<int64_t> tne_off;          // per slot: offset of its N^E values
  std::vector<double> NE;                // N^E_nu(q) at T-cell points: [slot][nu_local][q]
  // atomic parts alone, s_nu N^A_nu(q), at the points of the T-cells where they are nonzero
  // (the enrichment cells): [slot][atomic nu in tnu order][q]
  std::vector<int> ta_off, ta_nu;        // per slot: atomic enrichment indices
  std::vector<int64_t> tna_off;          // per slot: offset of its atomic values
  std::vector<double> NA;
  std::vector<int64_t> urow_node;        // union rows (interior nodes of T-cells)
  std::vector<int> node_urow;            // n_nodes, -1 if not a union row
  std::vector<int> urow_cnt;             // cells of the row's node that are T-cells
  std::vector<int> urow_pair;            // [row][8]: slot << kPairShift | local node
  std::vector<double> b, c;              // n_R x nenr
  std::vector<double> MAA, Mee;          // nenr x nenr
  std::vector<double> Mee_eval, Mee_evec;
  std::vector<double> S;                 // nenr x nk
  std::vector<double> Splus;             // nk x nenr: Loewdin coordinates of each N^E
  int nk = 0, ndrop = 0;
  std::vector<double> Kce;               // n_R x nenr: 1/2 int grad N_i . grad N^E_nu
  std::vector<double> Kee;               // nenr x nenr: 1/2 int grad N^E . grad N^E

  // ---- Poisson -------------------------------------------------------------
  std::vector<double> K1[3], M1[3];      // assembled 1-D stiffness/mass (nn x nn, dense)
  std::vector<double> fdmV[3], fdmL[3];  // interior generalised eigenvectors / values
  std::vector<double> gbnd;              // n_nodes: Dirichlet data on boundary, 0 inside
  std::vector<double> lift;              // n_nodes: (K g) on interior nodes, 0 on boundary

  std::string error;

  // helpers
  int64_t node_index(int64_t gx, int64_t gy, int64_t gz) const { return gx + nn[0] * (gy + nn[1] * gz); }
  int n1d(int64_t cell) const { return is_enr[cell] ? qe : qc; }
  bool is_boundary(int64_t node) const;
  void cell_ijk(int64_t c, int e[3]) const {
    e[0] = (int)(c % nc[0]);
    e[1] = (int)((c / nc[0]) % nc[1]);
    e[2] = (int)(c / ((int64_t)nc[0] * nc[1]));
  }
  void cell_nodes(int64_t c, int64_t *out) const;
  double cell_lo(int d, int e) const { return xb[d][e]; }
  double cell_h(int d, int e) const { return xb[d][e + 1] - xb[d][e]; }
  double node_coord(int d, int64_t g) const;
  int64_t n_urows() const { return (int64_t)urow_node.size(); }
};

// Builds the plan; returns an efe_status and fills plan.error on failure.
efe_status build_plan(const efe_system &sys, Plan &plan);

// Loewdin-orthonormalised initial orbitals (real), n_rows x norb row-major.
efe_status initial_state(const Plan &plan, const int32_t *enr_index, const double *g, double amp,
                         std::vector<double> &X);

// Small dense helpers shared by host code.
void sym_eig(int n, std::vector<double> A, std::vector<double> &evals, std::vector<double> &evecs);
double atomic_value(const Plan &pl, int nu, const double x[3], double grad[3]);

}  // namespace efe
