"""EFE discretisation of the TDKS equations (oracle).

Follows Sec. 2.1-2.3 of the paper:

* basis: classical FE functions N^C_i on the interior nodes (Dirichlet boundary,
  Sec. 3.1) plus enrichment functions N^E_nu = N^A_nu - sum_l c_{l nu} N^C_l,
  eq. (EFESplit)-(EFEOrtho), with c chosen so that the overlap of every N^E with
  every N^C vanishes.  Classical-classical mass integrals use GLL quadrature
  (diagonal D, Sec. 2.3), so the condition reads c = D^-1 b, b_i = int N^C_i N^A.
* overlap: block-diagonal M = diag(D, M^ee), eq. (M); M^ee = M^AA - b^T D^-1 b.
* Hamiltonian: H_mn = 1/2 int grad N_m . grad N_n + int v_KS N_m N_n, eq. (Hmn),
  integrated with each cell's Gauss rule.  H^ce and H^ee are computed here by
  evaluating the enrichment functions N^E at quadrature points and integrating
  them directly.
* Loewdin: Hbar = M^-1/2 H M^-1/2, eq. (TDKSDiscrete2); (M^ee)^-1/2 by
  eigendecomposition, eq. (MSquareRoot).  Eigenvalues below drop_tol * max are
  discarded (canonical orthogonalisation), which gives a rectangular S.
* density rho = sum_a f_a |psi_a|^2 (Sec. 2.1), Hartree potential from the
  Poisson problem eq. (Hartree_possion) discretised as eq. (DiscretePoisson) with
  A = (1/4 pi) int grad N . grad N, ALDA (xc.py), nuclear potential of
  Gaussian-smeared nuclei, field potential -E(t) . x, eq. (VField).

Vectors of coefficients use the full row layout: one row per mesh node
(boundary rows are zero) followed by one row per kept enrichment direction.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import erf

from .fe import Mesh, lagrange, gauss_rule
from .enrich import atomic_function
from . import xc as xcmod


@dataclass
class Field:
    """E(t) = dir * sum_k A_k sin(w_k t + phi_k) exp(-(t - t0)^2 / s^2)."""
    direction: int = 2
    A: np.ndarray = None
    w: np.ndarray = None
    phi: np.ndarray = None
    t0: float = 0.0
    s: float = 1.0

    def E(self, t):
        if self.A is None or len(self.A) == 0:
            return 0.0
        env = math.exp(-((t - self.t0) / self.s) ** 2)
        return float(np.sum(self.A * np.sin(self.w * t + self.phi))) * env


class EFEModel:
    def __init__(self, spec, drop_tol: Optional[float] = None):
        self.spec = spec
        self.mesh = m = Mesh(spec.ncell, spec.lo, spec.hi, spec.degree, spec.r_cut,
                             spec.R, spec.qcell, spec.qenr, getattr(spec, "bounds", None))
        self.D = m.lumped_mass()
        self.bnd = m.boundary_mask()
        self.interior = np.nonzero(~self.bnd)[0]
        self.occ = np.asarray(spec.occ, dtype=np.float64)
        self.drop_tol = spec.enr_drop_tol if drop_tol is None else drop_tol
        self._shape_cache = {}
        self._enr_cache = {}
        self._kin_cache = {}
        self._setup_enrichment()
        self.n_rows = m.n_nodes + self.nk
        # static potentials at every quadrature point
        self.qpts, self.qw = m.all_quadrature()
        self.v_nuc = self.nuclear_potential(self.qpts)
        self.v_trap = 0.5 * spec.trap_omega ** 2 * np.sum(self.qpts ** 2, axis=1) \
            if spec.trap_omega > 0 else np.zeros(m.n_quad)
        self._poisson = None

    # ------------------------------------------------------------------ shapes
    def shape(self, c):
        """Points, weights, B, grad B of cell c (B and the reference gradients depend only
        on the class; the gradient along d is scaled by 2 / h_d of the cell)."""
        m = self.mesh
        key = bool(m.is_enr[c])
        if key not in self._shape_cache:
            self._shape_cache[key] = m.reference_shape(key)
        pts, w, _ = m.cell_rule(c)
        B, G = self._shape_cache[key]
        return pts, w, B, G * (2.0 / m.cell_size(c))[:, None, None]

    # ------------------------------------------------------------- enrichment
    def _atomic(self, pts, grad):
        s = self.spec
        vals = np.zeros((len(pts), s.nenr))
        grads = np.zeros((len(pts), s.nenr, 3)) if grad else None
        for nu in range(s.nenr):
            R = s.R[s.enr_atom[nu]]
            out = atomic_function(pts, R, s.enr_l[nu], s.enr_m[nu], s.enr_zeta[nu], s.r_cut, grad)
            if grad:
                vals[:, nu], grads[:, nu, :] = out
            else:
                vals[:, nu] = out
        return vals, grads

    def _setup_enrichment(self):
        """b, c, M^AA, M^ee and its inverse square root S (Sec. 2.2-2.3)."""
        s, m = self.spec, self.mesh
        ne = s.nenr
        self.ecells = np.nonzero(m.is_enr)[0] if ne > 0 else np.zeros(0, dtype=np.int64)
        # unnormalised atomic functions on enrichment cells
        norm2 = np.zeros(ne)
        for c in self.ecells:
            pts, w, _, _ = self.shape(c)
            NA, _ = self._atomic(pts, False)
            norm2 += w @ (NA * NA)
        self.enr_scale = 1.0 / np.sqrt(norm2) if ne > 0 else np.zeros(0)
        b = np.zeros((m.n_nodes, ne))
        MAA = np.zeros((ne, ne))
        for c in self.ecells:
            pts, w, B, _ = self.shape(c)
            NA, _ = self._atomic(pts, False)
            NA = NA * self.enr_scale
            np.add.at(b, m.cell_nodes(c), B.T @ (w[:, None] * NA))
            MAA += NA.T @ (w[:, None] * NA)
        b[self.bnd] = 0.0
        self.b = b
        self.c = np.where(self.bnd[:, None], 0.0, b / self.D[:, None])
        self.MAA = MAA
        self.Mee = MAA - b.T @ (b / self.D[:, None]) if ne > 0 else np.zeros((0, 0))
        if ne > 0:
            lam, U = np.linalg.eigh(self.Mee)
            keep = lam > self.drop_tol * lam.max()
            if np.any(lam[keep] <= 0):
                raise np.linalg.LinAlgError("M^ee not positive definite on kept space")
            self.Mee_eig = (lam, U)
            self.n_dropped = int(np.sum(~keep))
            if self.n_dropped == 0:
                self.S = (U / np.sqrt(lam)) @ U.T
            else:
                self.S = U[:, keep] / np.sqrt(lam[keep])
        else:
            self.S = np.zeros((0, 0))
            self.n_dropped = 0
        self.nk = self.S.shape[1]
        # cells on which some N^E is nonzero: enrichment cells and every cell
        # holding a node with c != 0
        cnz = np.any(self.c != 0.0, axis=1) if ne > 0 else np.zeros(m.n_nodes, bool)
        tc = set(self.ecells.tolist())
        for i in np.nonzero(cnz)[0]:
            tc.update(m.cells_of_node(int(i)))
        self.tcells = np.array(sorted(tc), dtype=np.int64)

    def enrichment_on_cell(self, c, grad=True):
        """N^E_nu and grad N^E_nu at cell c's quadrature points (nq, ne), (3, nq, ne).

        Static data: memoised per cell."""
        key = (int(c), bool(grad))
        if key not in self._enr_cache:
            self._enr_cache[key] = self._enrichment_on_cell(c, grad)
        return self._enr_cache[key]

    def _enrichment_on_cell(self, c, grad):
        pts, w, B, G = self.shape(c)
        nodes = self.mesh.cell_nodes(c)
        cc = self.c[nodes]                          # (nloc, ne)
        if self.mesh.is_enr[c]:
            NA, dNA = self._atomic(pts, grad)
            NA = NA * self.enr_scale
            if grad:
                dNA = dNA * self.enr_scale[None, :, None]
        else:
            NA = np.zeros((len(pts), self.spec.nenr))
            dNA = np.zeros((len(pts), self.spec.nenr, 3))
        NE = NA - B @ cc
        if not grad:
            return NE, None
        dNE = np.stack([dNA[:, :, d] - G[d] @ cc for d in range(3)])
        return NE, dNE

    # ------------------------------------------------------------- potentials
    def nuclear_potential(self, pts):
        """Smeared nuclei: v_N = -sum Z erf(r / sigma) / r, eq. (VN) with Gaussian charges."""
        s = self.spec
        v = np.zeros(len(pts))
        for I in range(s.natom):
            r = np.linalg.norm(pts - s.R[I][None, :], axis=1)
            safe = np.where(r > 1e-12, r, 1.0)
            v -= s.Z[I] * np.where(r > 1e-12, erf(safe / s.nuc_sigma) / safe,
                                   2.0 / (s.nuc_sigma * math.sqrt(math.pi)))
        return v

    def hartree_boundary(self, pts):
        """Dirichlet data of v_H: the far field of the electrons' charge."""
        s = self.spec
        nel = float(np.sum(self.occ))
        if nel == 0.0:
            return np.zeros(len(pts))
        if s.natom == 0:
            return nel / np.linalg.norm(pts, axis=1)
        zt = float(np.sum(s.Z))
        g = np.zeros(len(pts))
        for I in range(s.natom):
            g += s.Z[I] / np.linalg.norm(pts - s.R[I][None, :], axis=1)
        return g * nel / zt

    def ks_potential(self, rho, vH_q, t=0.0, field: Optional[Field] = None):
        v = self.v_nuc + vH_q + xcmod.vxc(rho, self.spec.xc) + self.v_trap
        if field is not None:
            v = v - field.E(t) * self.qpts[:, field.direction]
        return v

    # ------------------------------------------------------------ Hamiltonian
    def cell_block(self, c, v_q, kinetic=True):
        """H_c = 1/2 int grad N . grad N + int v N N on cell c (unscaled, eq. (Hmn))."""
        m = self.mesh
        pts, w, B, G = self.shape(c)
        v = v_q[m.q_off[c]:m.q_off[c + 1]]
        Hc = B.T @ ((w * v)[:, None] * B)
        if kinetic:
            Hc += self.kinetic_block(c)
        return Hc

    def kinetic_block(self, c):
        """1/2 int grad N . grad N on cell c: depends only on the cell's class and edge
        lengths, formed once per (class, edges)."""
        m = self.mesh
        key = (bool(m.is_enr[c]), tuple(m.cell_size(c)))
        K = self._kin_cache.get(key)
        if K is None:
            pts, w, B, G = self.shape(c)
            K = 0.5 * sum(G[d].T @ (w[:, None] * G[d]) for d in range(3))
            K.setflags(write=False)
            self._kin_cache[key] = K
        return K

    def coupling_on_cell(self, c, v_q, kinetic=True):
        """Cell c's contributions to H^ce (nloc x ne) and H^ee (ne x ne), from N^E at its points."""
        m = self.mesh
        pts, w, B, G = self.shape(c)
        v = v_q[m.q_off[c]:m.q_off[c + 1]]
        NE, dNE = self.enrichment_on_cell(c, grad=kinetic)
        part = B.T @ ((w * v)[:, None] * NE)
        pee = NE.T @ ((w * v)[:, None] * NE)
        if kinetic:
            part += 0.5 * sum(G[d].T @ (w[:, None] * dNE[d]) for d in range(3))
            pee += 0.5 * sum(dNE[d].T @ (w[:, None] * dNE[d]) for d in range(3))
        return part, pee

    def coupling(self, v_q, kinetic=True):
        """H^ce (n_nodes x ne, boundary rows zero) and H^ee."""
        m = self.mesh
        ne = self.spec.nenr
        Hce = np.zeros((m.n_nodes, ne))
        Hee = np.zeros((ne, ne))
        for c in self.tcells:
            part, pee = self.coupling_on_cell(c, v_q, kinetic)
            np.add.at(Hce, m.cell_nodes(c), part)
            Hee += pee
        Hce[self.bnd] = 0.0
        return Hce, Hee

    def dm12(self):
        """D^-1/2 with the boundary rows removed."""
        return (~self.bnd).astype(np.float64) / np.sqrt(self.D)

    def hamiltonian(self, v_q, kinetic=True):
        """Hbar as a sparse matrix on the full row layout, eq. (Hmn) + eq. (TDKSDiscrete2)."""
        m = self.mesh
        rows, cols, vals = [], [], []
        for c in range(m.n_cells):
            Hc = self.cell_block(c, v_q, kinetic)
            nodes = m.cell_nodes(c)
            rows.append(np.repeat(nodes, len(nodes)))
            cols.append(np.tile(nodes, len(nodes)))
            vals.append(Hc.reshape(-1))
        N = m.n_nodes
        Hcc = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                            shape=(N, N)).tocsr()
        dm = self.dm12()
        Hbar_cc = sp.diags(dm) @ Hcc @ sp.diags(dm)
        if self.spec.nenr == 0:
            return Hbar_cc.tocsr()
        Hce, Hee = self.coupling(v_q, kinetic)
        Hbar_ce = (dm[:, None] * Hce) @ self.S
        Hbar_ee = self.S.T @ Hee @ self.S
        Hbar = sp.bmat([[Hbar_cc, sp.csr_matrix(Hbar_ce)],
                        [sp.csr_matrix(Hbar_ce.T), sp.csr_matrix(Hbar_ee)]], format="csr")
        return Hbar

    def hamiltonian_rows(self, v_q, X, rows, kinetic=True):
        """(Hbar X) at the given node rows and at every enrichment row, without assembling Hbar.

        Same definitions as `hamiltonian`: cell blocks of the cells that hold each
        requested node, and the full coupling H^ce, H^ee.  Returns (Y_rows, Y_E).
        """
        m = self.mesh
        N = m.n_nodes
        dm = self.dm12()
        Xc = dm[:, None] * X[:N]
        Yr = np.zeros((len(rows), X.shape[1]), dtype=np.result_type(X, np.float64))
        for k, i in enumerate(rows):
            if self.bnd[i]:
                continue
            acc = 0.0
            for c in m.cells_of_node(int(i)):
                nodes = m.cell_nodes(c)
                li = int(np.nonzero(nodes == i)[0][0])
                acc = acc + self.cell_block(c, v_q, kinetic)[li] @ Xc[nodes]
            Yr[k] = dm[i] * acc
        if self.spec.nenr == 0:
            return Yr, np.zeros((0, X.shape[1]))
        Hce, Hee = self.coupling(v_q, kinetic)
        psiE = self.S @ X[N:]
        Yr += dm[rows][:, None] * (Hce[rows] @ psiE)
        YE = self.S.T @ (Hce.T @ Xc + Hee @ psiE)
        return Yr, YE

    def cell_blocks(self, v_q, kinetic=True):
        """Every cell block H_c of `cell_block`, stacked (n_cells, nloc, nloc)."""
        m = self.mesh
        out = np.empty((m.n_cells, m.nloc, m.nloc))
        for c in range(m.n_cells):
            pts, w, B, G = self.shape(c)
            v = v_q[m.q_off[c]:m.q_off[c + 1]]
            Hc = B.T @ ((w * v)[:, None] * B)
            if kinetic:
                Hc += self.kinetic_block(c)
            out[c] = Hc
        return out

    def operator(self, v_q, kinetic=True):
        """Hbar of `hamiltonian` as a matrix-free operator (CellOperator)."""
        return CellOperator(self, v_q, kinetic)

    def position_operator(self, d):
        """Zbar_d: Loewdin position operator (no kinetic term, v = x_d)."""
        return self.hamiltonian(self.qpts[:, d].copy(), kinetic=False)

    # ----------------------------------------------------------------- fields
    def psi_at_quadrature(self, X):
        """psi_a(q) for every quadrature point: (n_quad, norb) complex."""
        m = self.mesh
        X = np.asarray(X)
        psiC = np.where(self.bnd[:, None], 0.0, X[:m.n_nodes] / np.sqrt(self.D)[:, None])
        psiE = self.S @ X[m.n_nodes:] if self.spec.nenr > 0 else None
        out = np.zeros((m.n_quad, X.shape[1]), dtype=np.complex128)
        tset = set(self.tcells.tolist())
        for c in range(m.n_cells):
            pts, w, B, G = self.shape(c)
            val = B @ psiC[m.cell_nodes(c)]
            if psiE is not None and c in tset:
                NE, _ = self.enrichment_on_cell(c, grad=False)
                val = val + NE @ psiE
            out[m.q_off[c]:m.q_off[c + 1]] = val
        return out

    def density(self, X):
        """rho(q) = sum_a f_a |psi_a(q)|^2 (Sec. 2.1)."""
        psi = self.psi_at_quadrature(X)
        return np.real(psi * np.conj(psi)) @ self.occ

    def dipole(self, rho):
        """mu_d = sum_q W_q x_d(q) rho(q): electronic dipole."""
        return self.qpts.T @ (self.qw * rho)

    # ---------------------------------------------------------------- Poisson
    def _poisson_setup(self):
        m = self.mesh
        rows, cols, vals = [], [], []
        for c in range(m.n_cells):
            pts, w, B, G = self.shape(c)
            Kc = sum(G[d].T @ (w[:, None] * G[d]) for d in range(3))
            nodes = m.cell_nodes(c)
            rows.append(np.repeat(nodes, len(nodes)))
            cols.append(np.tile(nodes, len(nodes)))
            vals.append(Kc.reshape(-1))
        N = m.n_nodes
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        I = self.interior
        Bn = np.nonzero(self.bnd)[0]
        self._poisson = dict(K=K, KII=K[I][:, I].tocsc(), KIB=K[I][:, Bn].tocsr(), Bn=Bn,
                             g=self.hartree_boundary(m.node_coords(Bn)))

    def poisson_rhs(self, rho):
        """d_i = int rho N_i with each cell's rule."""
        m = self.mesh
        d = np.zeros(m.n_nodes)
        for c in range(m.n_cells):
            pts, w, B, G = self.shape(c)
            np.add.at(d, m.cell_nodes(c), B.T @ (w * rho[m.q_off[c]:m.q_off[c + 1]]))
        return d

    def stiffness_tensor_apply(self, u):
        """K u over all nodes, K = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1 (exact 1-D matrices)."""
        m = self.mesh
        K = [self.one_d_matrices(d) for d in range(3)]
        U = u.reshape(m.nn[2], m.nn[1], m.nn[0])
        out = np.zeros_like(U)
        for term in range(3):
            Ax = K[0][0] if term == 0 else K[0][1]
            Ay = K[1][0] if term == 1 else K[1][1]
            Az = K[2][0] if term == 2 else K[2][1]
            out += np.einsum("zyx,ax,by,cz->cba", U, Ax, Ay, Az, optimize=True)
        return out.reshape(-1)

    def hartree(self, rho, solver="direct", boundary=None):
        """Nodal v_H: (1/4 pi) K phi = d in the interior, phi = g on the boundary.

        solver "fdm" uses the tensor structure of K for both the Dirichlet lift
        and the interior solve (no assembled matrix; for large meshes)."""
        m = self.mesh
        Bn = np.nonzero(self.bnd)[0]
        if solver == "fdm":
            g = self.hartree_boundary(m.node_coords(Bn)) if boundary is None else boundary
            gf = np.zeros(m.n_nodes)
            gf[Bn] = g
            d = self.poisson_rhs(rho)
            rhs = 4.0 * math.pi * d[self.interior] - self.stiffness_tensor_apply(gf)[self.interior]
            phi = np.zeros(m.n_nodes)
            phi[self.interior] = self.fdm_solve(rhs)
            phi[Bn] = g
            return phi
        if self._poisson is None:
            self._poisson_setup()
        P = self._poisson
        g = P["g"] if boundary is None else boundary
        d = self.poisson_rhs(rho)
        rhs = 4.0 * math.pi * d[self.interior] - P["KIB"] @ g
        if solver == "direct":
            if "lu" not in P:
                P["lu"] = spla.splu(P["KII"])          # K_II is fixed: factorised once
            phiI = P["lu"].solve(rhs)
        elif solver == "cg":
            phiI, info = spla.cg(P["KII"], rhs, rtol=1e-14, atol=0.0, maxiter=20000)
            if info != 0:
                raise RuntimeError("CG did not converge")
        else:
            raise ValueError(solver)
        phi = np.zeros(self.mesh.n_nodes)
        phi[self.interior] = phiI
        phi[P["Bn"]] = g
        return phi

    def fdm_solve(self, rhs_interior):
        """K_II^-1 by fast diagonalisation: K = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1."""
        m = self.mesh
        Vs, lams = [], []
        for d in range(3):
            K1, M1 = self.one_d_matrices(d)
            lam, V = sla.eigh(K1[1:-1, 1:-1], M1[1:-1, 1:-1])
            Vs.append(V)
            lams.append(lam)
        n = [len(l) for l in lams]
        r = rhs_interior.reshape(n[2], n[1], n[0])
        t = np.einsum("zyx,xa,yb,zc->cba", r, Vs[0], Vs[1], Vs[2], optimize=True)
        denom = lams[2][:, None, None] + lams[1][None, :, None] + lams[0][None, None, :]
        t = t / denom
        out = np.einsum("cba,xa,yb,zc->zyx", t, Vs[0], Vs[1], Vs[2], optimize=True)
        return out.reshape(-1)

    def one_d_matrices(self, d):
        """Assembled 1-D stiffness and consistent mass along axis d (exact Gauss rule)."""
        m = self.mesh
        xi, wi = gauss_rule(m.p + 1)
        V, dV = lagrange(m.xg, xi)
        Kr = dV.T @ (wi[:, None] * dV)
        Mr = V.T @ (wi[:, None] * V)
        n = m.nn[d]
        K1 = np.zeros((n, n))
        M1 = np.zeros((n, n))
        for e in range(m.nc[d]):
            h = m.hc[d][e]
            s = slice(e * m.p, e * m.p + m.p + 1)
            K1[s, s] += (2.0 / h) * Kr
            M1[s, s] += (h / 2.0) * Mr
        return K1, M1

    def interpolate_nodal(self, phi):
        """Nodal field -> values at every quadrature point."""
        m = self.mesh
        out = np.empty(m.n_quad)
        for c in range(m.n_cells):
            pts, w, B, G = self.shape(c)
            out[m.q_off[c]:m.q_off[c + 1]] = B @ phi[m.cell_nodes(c)]
        return out

    # ------------------------------------------------------------ composition
    def potential_from_density(self, rho, t=0.0, field=None):
        phi = self.hartree(rho)
        return self.ks_potential(rho, self.interpolate_nodal(phi), t, field), phi

    def hamiltonian_from_density(self, rho, t=0.0, field=None):
        v, _ = self.potential_from_density(rho, t, field)
        return self.hamiltonian(v)

    def operator_from_density(self, rho, t=0.0, field=None):
        """Matrix-free Hbar[rho, t] with the Hartree potential by fast diagonalisation."""
        phi = self.hartree(rho, solver="fdm")
        return self.operator(self.ks_potential(rho, self.interpolate_nodal(phi), t, field))

    def position_operator_free(self, d):
        """Matrix-free Zbar_d (no kinetic term, v = x_d)."""
        return self.operator(self.qpts[:, d].copy(), kinetic=False)

    # -------------------------------------------------------- initial states
    def enrichment_noise_state(self):
        """Enrichment directions plus low-frequency FE noise, Loewdin-orthonormalised.

        Orbital a: enrichment block = S^+ e_nu(a), the Loewdin coordinates of
        N^E_nu(a) (projected on the kept space), classical block = D^1/2 n, with
        n = 0.1 * s / ||s||_M and s(x) = sum_m g_m prod_d sin(m_d pi (x_d - lo_d)/(hi_d - lo_d)).
        Columns are then made orthonormal by X (X^T X)^-1/2.
        """
        from workloads import NOISE_MODES
        s, m = self.spec, self.mesh
        g = s.noise()
        X = np.zeros((self.n_rows, s.norb))
        lam, U = self.Mee_eig
        keep = lam > self.drop_tol * lam.max()
        # T = S^+ (pseudo-inverse of S): kept-space coordinates of each N^E_nu
        if self.n_dropped == 0:
            T = (U * np.sqrt(lam)) @ U.T
        else:
            T = np.sqrt(lam[keep])[:, None] * U[:, keep].T
        xyz = m.node_coords()
        L = m.hi - m.lo
        for a in range(s.norb):
            f = np.zeros(m.n_nodes)
            for k, (mx, my, mz) in enumerate(NOISE_MODES):
                f += g[a, k] * (np.sin(mx * np.pi * (xyz[:, 0] - m.lo[0]) / L[0])
                                * np.sin(my * np.pi * (xyz[:, 1] - m.lo[1]) / L[1])
                                * np.sin(mz * np.pi * (xyz[:, 2] - m.lo[2]) / L[2]))
            f[self.bnd] = 0.0
            nrm = math.sqrt(float(np.sum(self.D * f * f)))
            X[:m.n_nodes, a] = np.sqrt(self.D) * (s.noise_amp * f / nrm)
            X[m.n_nodes:, a] = T[:, s.init_enr[a]]
        G = X.T @ X
        lam_g, V = np.linalg.eigh(G)
        X = X @ ((V / np.sqrt(lam_g)) @ V.T)
        return X.astype(np.complex128)


class CellOperator:
    """Hbar X without the assembled matrix, for meshes too large to assemble.

    The same definitions as `EFEModel.hamiltonian` (eq. (Hmn), eq. (TDKSDiscrete2)):
    Y_C = D^-1/2 sum_c P_c^T H_c P_c D^-1/2 X_C + D^-1/2 H^ce S X_E and
    Y_E = S^T (H^ce)^T D^-1/2 X_C + S^T H^ee S X_E, with the cell blocks H_c of
    `cell_block` (gathered and summed by a scatter matrix) and the coupling of
    `coupling`.  Called on one column (n_rows,) or a block (n_rows, m).
    """

    def __init__(self, model, v_q, kinetic=True):
        m = model.mesh
        self.N = m.n_nodes
        self.n_rows = model.n_rows
        self.nodes = np.stack([m.cell_nodes(c) for c in range(m.n_cells)])
        self.blocks = model.cell_blocks(v_q, kinetic)
        self.dm = model.dm12()
        nl = m.nloc
        self.scatter = sp.csr_matrix((np.ones(m.n_cells * nl), (self.nodes.reshape(-1), np.arange(m.n_cells * nl))),
                                     shape=(self.N, m.n_cells * nl))
        self.has_enr = model.spec.nenr > 0
        if self.has_enr:
            self.Hce, self.Hee = model.coupling(v_q, kinetic)
            self.S = model.S

    def __call__(self, X):
        X = np.asarray(X)
        one = X.ndim == 1
        X2 = (X[:, None] if one else X).astype(np.complex128)
        N, ncol = self.N, X2.shape[1]
        Xc = np.ascontiguousarray(self.dm[:, None] * X2[:N])
        Xr = Xc.view(np.float64)                          # (N, 2 ncol): re and im as real columns
        loc = np.empty((self.blocks.shape[0], self.blocks.shape[1], 2 * ncol))
        step = 512
        for c0 in range(0, self.blocks.shape[0], step):
            c1 = min(c0 + step, self.blocks.shape[0])
            loc[c0:c1] = np.matmul(self.blocks[c0:c1], Xr[self.nodes[c0:c1]])
        Yc = np.ascontiguousarray(self.scatter @ loc.reshape(-1, 2 * ncol)).view(np.complex128)
        Y = np.zeros((self.n_rows, ncol), dtype=np.complex128)
        if self.has_enr:
            psiE = self.S @ X2[N:]
            Yc = Yc + self.Hce @ psiE
            Y[N:] = self.S.T @ (self.Hce.T @ Xc + self.Hee @ psiE)
        Y[:N] = self.dm[:, None] * Yc
        return Y[:, 0] if one else Y
