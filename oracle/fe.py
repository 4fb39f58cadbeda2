"""Spectral hexahedral finite elements on a uniform mesh (oracle).

Follows Sec. 2.2-2.3 of the paper: classical FE basis functions are tensor
products of degree-p Lagrange polynomials on Gauss-Lobatto-Legendre (GLL)
nodes, so that GLL quadrature makes the classical mass matrix diagonal.
Hamiltonian integrals use Gauss-Legendre rules per cell: (p+1)^3 points on
ordinary cells, (2p+2)^3 on cells within the enrichment cutoff of an atom
(fixed high-order rule in place of the paper's adaptive quadrature, Sec. 2.4).

Orderings (shared with the library only as a documented convention):
  global node (gx, gy, gz) -> gx + Nx (gy + Ny gz), Nd = ncell_d p + 1
  cell (ex, ey, ez)        -> ex + nx (ey + ny ez)
  cell-local node (a,b,c)  -> a + (p+1) (b + (p+1) c)
  cell quadrature (i,j,k)  -> i + n (j + n k)
  quadrature arrays are cell-major in cell order, then local point order.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as L


def gll_rule(p: int):
    """GLL nodes and weights on [-1, 1]: endpoints plus the roots of P_p'."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    cp = np.zeros(p + 1)
    cp[p] = 1.0
    interior = np.sort(np.real(L.legroots(L.legder(cp)))) if p > 1 else np.zeros(0)
    # Newton polish of P_p'(x) = 0
    for _ in range(5):
        d1 = L.legval(interior, L.legder(cp))
        d2 = L.legval(interior, L.legder(cp, 2))
        interior = interior - d1 / d2
    x = np.concatenate([[-1.0], interior, [1.0]])
    Pp = L.legval(x, cp)
    w = 2.0 / (p * (p + 1) * Pp * Pp)
    return x, w


@functools.lru_cache(maxsize=None)
def gauss_rule(n: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (NumPy's routine; computed once per n,
    returned read-only)."""
    x, w = L.leggauss(n)
    x.setflags(write=False)
    w.setflags(write=False)
    return x, w


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values and first derivatives of the Lagrange basis on ``nodes`` at ``x``.

    Returns (V, dV) of shape (len(x), len(nodes)).  Plain product formulas.
    """
    n = len(nodes)
    x = np.asarray(x, dtype=np.float64)
    V = np.ones((len(x), n))
    dV = np.zeros((len(x), n))
    for a in range(n):
        for b in range(n):
            if b == a:
                continue
            V[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
        for c in range(n):
            if c == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[c]))
            for b in range(n):
                if b == a or b == c:
                    continue
                term *= (x - nodes[b]) / (nodes[a] - nodes[b])
            dV[:, a] += term
    return V, dV


class Mesh:
    """Tensor-product hex mesh of degree-p spectral elements with Dirichlet boundary.

    Cells are uniform, or graded per axis by the cell boundaries ``bounds[d]``
    (ncell[d] + 1 increasing values from lo[d] to hi[d]); each cell maps its
    reference cube affinely, so every integral keeps its tensor-product form with
    the cell's own sizes.
    """

    def __init__(self, ncell, lo, hi, p, r_cut=0.0, atoms=None, qcell=None, qenr=None, bounds=None):
        self.nc = np.array(ncell, dtype=np.int64)
        self.lo = np.array(lo, dtype=np.float64)
        self.hi = np.array(hi, dtype=np.float64)
        self.p = int(p)
        h = (self.hi - self.lo) / self.nc
        if bounds is None:
            self.bounds = [self.lo[d] + np.arange(self.nc[d] + 1) * h[d] for d in range(3)]
        else:
            self.bounds = [np.asarray(bounds[d], dtype=np.float64) for d in range(3)]
            for d in range(3):
                b = self.bounds[d]
                if len(b) != self.nc[d] + 1 or np.any(np.diff(b) <= 0) or b[0] != self.lo[d] or b[-1] != self.hi[d]:
                    raise ValueError("bounds must be ncell + 1 increasing values from lo to hi per axis")
        self.hc = [np.diff(b) for b in self.bounds]      # cell sizes per axis
        self.nn = self.nc * self.p + 1
        self.n_nodes = int(np.prod(self.nn))
        self.n_cells = int(np.prod(self.nc))
        self.nloc = (self.p + 1) ** 3
        self.xg, self.wg = gll_rule(self.p)
        # 1-D node coordinates per axis
        self.coord1d = []
        for d in range(3):
            g = np.arange(self.nn[d])
            e = np.minimum(g // self.p, self.nc[d] - 1)
            a = g - e * self.p
            self.coord1d.append(self.bounds[d][e] + (self.xg[a] + 1.0) * 0.5 * self.hc[d][e])
        self.qcell = int(qcell) if qcell else self.p + 1
        self.qenr = int(qenr) if qenr else 2 * self.p + 2
        atoms = np.zeros((0, 3)) if atoms is None else np.asarray(atoms, dtype=np.float64)
        self.is_enr = self._classify(atoms, float(r_cut))
        self.nq_cell = np.where(self.is_enr, self.qenr ** 3, self.qcell ** 3)
        self.q_off = np.concatenate([[0], np.cumsum(self.nq_cell)]).astype(np.int64)
        self.n_quad = int(self.q_off[-1])

    # -- indexing ---------------------------------------------------------
    def cell_ijk(self, c):
        nx, ny = self.nc[0], self.nc[1]
        return c % nx, (c // nx) % ny, c // (nx * ny)

    def node_index(self, gx, gy, gz):
        return gx + self.nn[0] * (gy + self.nn[1] * gz)

    def node_ijk(self, i):
        nx, ny = self.nn[0], self.nn[1]
        return i % nx, (i // nx) % ny, i // (nx * ny)

    def cell_nodes(self, c):
        """Global indices of the (p+1)^3 nodes of cell c, in cell-local order."""
        ex, ey, ez = self.cell_ijk(c)
        a = np.arange(self.p + 1)
        gx = ex * self.p + a
        gy = ey * self.p + a
        gz = ez * self.p + a
        GZ, GY, GX = np.meshgrid(gz, gy, gx, indexing="ij")
        return self.node_index(GX, GY, GZ).reshape(-1)

    def node_coords(self, idx=None):
        if idx is None:
            idx = np.arange(self.n_nodes)
        ix, iy, iz = self.node_ijk(np.asarray(idx))
        return np.stack([self.coord1d[0][ix], self.coord1d[1][iy], self.coord1d[2][iz]], axis=-1)

    def boundary_mask(self):
        ix, iy, iz = self.node_ijk(np.arange(self.n_nodes))
        b = np.zeros(self.n_nodes, dtype=bool)
        for g, n in ((ix, self.nn[0]), (iy, self.nn[1]), (iz, self.nn[2])):
            b |= (g == 0) | (g == n - 1)
        return b

    def cells_of_node(self, i):
        """Cells whose closure contains node i."""
        ijk = self.node_ijk(i)
        ranges = []
        for d in range(3):
            g = int(ijk[d])
            es = {min(g // self.p, int(self.nc[d]) - 1)}
            if g % self.p == 0 and g > 0:
                es.add(g // self.p - 1)
            if g % self.p == 0 and g // self.p < self.nc[d]:
                es.add(g // self.p)
            ranges.append(sorted(es))
        out = []
        for ez in ranges[2]:
            for ey in ranges[1]:
                for ex in ranges[0]:
                    out.append(int(ex + self.nc[0] * (ey + self.nc[1] * ez)))
        return out

    # -- cell classes -------------------------------------------------------
    def _classify(self, atoms, r_cut):
        """Enrichment cell: the cell box is closer than r_cut to some atom."""
        flags = np.zeros(self.n_cells, dtype=bool)
        if len(atoms) == 0 or r_cut <= 0:
            return flags
        c = np.arange(self.n_cells)
        ex, ey, ez = self.cell_ijk(c)
        e = [ex, ey, ez]
        for R in atoms:
            d2 = np.zeros(self.n_cells)
            for d in range(3):
                lo = self.bounds[d][e[d]]
                hi = lo + self.hc[d][e[d]]
                gap = np.maximum(np.maximum(lo - R[d], R[d] - hi), 0.0)
                d2 += gap * gap
            flags |= d2 < r_cut * r_cut
        return flags

    # -- per-cell quadrature ------------------------------------------------
    def cell_rule(self, c):
        """Points (nq, 3), weights (nq,), and 1-D reference nodes of cell c's rule."""
        n = self.qenr if self.is_enr[c] else self.qcell
        xi, wi = gauss_rule(n)
        ex, ey, ez = self.cell_ijk(c)
        hc = self.cell_size(c)
        pts1 = [self.bounds[d][e] + (xi + 1.0) * 0.5 * hc[d] for d, e in zip(range(3), (ex, ey, ez))]
        Z, Y, X = np.meshgrid(pts1[2], pts1[1], pts1[0], indexing="ij")
        WZ, WY, WX = np.meshgrid(wi, wi, wi, indexing="ij")
        pts = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
        w = (WX * WY * WZ).reshape(-1) * np.prod(0.5 * hc)
        return pts, w, xi

    def reference_shape(self, enriched):
        """Basis B (nq, nloc) and reference-cube gradients (3, nq, nloc) at the Gauss rule
        of a cell of the given class (the same for every cell of that class)."""
        n = self.qenr if enriched else self.qcell
        xi, _ = gauss_rule(n)
        V, dV = lagrange(self.xg, xi)           # (n, p+1)
        P = self.p + 1
        # point (i,j,k) x fastest, node (a,b,c) x fastest
        B = np.einsum("ia,jb,kc->kjicba", V, V, V).reshape(n ** 3, P ** 3)
        Gx = np.einsum("ia,jb,kc->kjicba", dV, V, V).reshape(n ** 3, P ** 3)
        Gy = np.einsum("ia,jb,kc->kjicba", V, dV, V).reshape(n ** 3, P ** 3)
        Gz = np.einsum("ia,jb,kc->kjicba", V, V, dV).reshape(n ** 3, P ** 3)
        return B, np.stack([Gx, Gy, Gz])

    def cell_shape(self, c):
        """Cell basis at the cell's rule: B (nq, nloc) and grad (3, nq, nloc); the
        affine map of the cell scales the reference gradient along d by 2 / h_d."""
        pts, w, _ = self.cell_rule(c)
        B, G = self.reference_shape(bool(self.is_enr[c]))
        return pts, w, B, G * (2.0 / self.cell_size(c))[:, None, None]

    def all_quadrature(self):
        """Points (n_quad, 3) and weights (n_quad,) over all cells, in cell order."""
        P = np.empty((self.n_quad, 3))
        W = np.empty(self.n_quad)
        for c in range(self.n_cells):
            pts, w, _ = self.cell_rule(c)
            P[self.q_off[c]:self.q_off[c + 1]] = pts
            W[self.q_off[c]:self.q_off[c + 1]] = w
        return P, W

    def lumped_mass(self):
        """Diagonal classical mass from GLL quadrature: sum of cell weights per node."""
        D = np.zeros(self.n_nodes)
        w3 = np.einsum("a,b,c->cba", self.wg, self.wg, self.wg).reshape(-1)
        for c in range(self.n_cells):
            np.add.at(D, self.cell_nodes(c), w3 * np.prod(0.5 * self.cell_size(c)))
        return D

    def cell_size(self, c):
        """Edge lengths (3,) of cell c."""
        e = self.cell_ijk(c)
        return np.array([self.hc[d][e[d]] for d in range(3)])
