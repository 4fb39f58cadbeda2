"""Pins for the oracle on graded tensor-product meshes (per-axis cell boundaries).

Sec. 2.7 refines the FE mesh near the atoms and coarsens it toward the faces; on
a tensor-product mesh this means per-axis cell sizes, with each cell mapped
affinely from the reference cube.  What fixes the discretisation there:
* quadrature: the weights sum to the box volume and integrate x^2, y^4 z exactly;
  every point lies inside its own cell;
* an explicit list of uniform boundaries reproduces the uniform mesh;
* Dirichlet box [0,Lx]x[0,Ly]x[0,Lz] (not a cube, so an axis mix-up shows):
  levels pi^2/2 sum n_d^2/L_d^2, error falling like h^(2p) under halving;
* harmonic oscillator v = |x|^2/2 on a mesh graded toward the centre: 3/2, 5/2;
* Gaussian charge: Hartree potential -> Q erf(r/s)/r, and the FDM, CG and sparse
  direct solves of the graded Poisson operator agree;
* enrichment: S^T M^ee S = I and the energy functional of the Loewdin
  Hamiltonian equals the direct integral on a graded mesh.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy.special import erf

from oracle.fe import Mesh
from oracle.model import EFEModel
from workloads import gaussian_box, trap, tiny, tiny_graded, graded_bounds


def _lowest(m, v, k):
    """Lowest k eigenvalues of Hbar on the active rows (shift-invert Lanczos about the
    bottom of the spectrum; the matrix is symmetric)."""
    H = m.hamiltonian(v)
    act = np.concatenate([m.interior, m.mesh.n_nodes + np.arange(m.nk)])
    A = H[act][:, act].tocsc()
    if A.shape[0] <= 2000:
        return sla.eigh(A.toarray(), eigvals_only=True, subset_by_index=[0, k - 1])
    # a block of 3 k vectors so that every member of a degenerate level is found
    lam = spla.eigsh(A, k=3 * k, sigma=float(np.min(v)) - 1.0, which="LM", tol=1e-13,
                     return_eigenvectors=False, v0=np.random.default_rng(0).standard_normal(A.shape[0]))
    return np.sort(lam)[:k]


def _halve(b):
    b = np.asarray(b)
    return np.sort(np.concatenate([b, 0.5 * (b[1:] + b[:-1])]))


def test_graded_bounds_recipe():
    b = graded_bounds(-35.0, 35.0, 24, 1.93)
    h = np.diff(b)
    assert b[0] == -35.0 and b[-1] == 35.0 and len(b) == 25
    np.testing.assert_allclose(h, h[::-1], rtol=1e-12)            # symmetric
    assert np.all(np.diff(h[:12]) < 0)                           # finest at the centre
    np.testing.assert_allclose(graded_bounds(-2.0, 6.0, 4, 0.0), [-2, 0, 2, 4, 6])


def test_graded_quadrature_and_mass():
    bounds = ([0.0, 0.7, 2.0, 2.4, 5.0], [-1.0, 0.5, 3.0], [2.0, 2.3, 2.9, 4.1])
    m = Mesh((4, 2, 3), (0.0, -1.0, 2.0), (5.0, 3.0, 4.1), 4, bounds=bounds)
    P, W = m.all_quadrature()
    vol = 5.0 * 4.0 * 2.1
    np.testing.assert_allclose(W.sum(), vol, rtol=1e-14)
    np.testing.assert_allclose(m.lumped_mass().sum(), vol, rtol=1e-14)
    # int x^2 dV and int y^4 z dV (exact for the (p+1)-point Gauss rule)
    np.testing.assert_allclose(np.sum(W * P[:, 0] ** 2), 125.0 / 3.0 * 4.0 * 2.1, rtol=1e-13)
    iy4 = (3.0 ** 5 + 1.0) / 5.0
    iz = 0.5 * (4.1 ** 2 - 4.0)
    np.testing.assert_allclose(np.sum(W * P[:, 1] ** 4 * P[:, 2]), 5.0 * iy4 * iz, rtol=1e-13)
    for c in range(m.n_cells):
        e = m.cell_ijk(c)
        lo = np.array([bounds[d][e[d]] for d in range(3)])
        hi = np.array([bounds[d][e[d] + 1] for d in range(3)])
        p = P[m.q_off[c]:m.q_off[c + 1]]
        assert np.all(p > lo) and np.all(p < hi)
        xyz = m.node_coords(m.cell_nodes(c))
        np.testing.assert_allclose(xyz.min(axis=0), lo, atol=1e-14)
        np.testing.assert_allclose(xyz.max(axis=0), hi, atol=1e-14)
        np.testing.assert_allclose(m.cell_size(c), hi - lo, rtol=1e-14)


def test_bad_bounds_rejected():
    with pytest.raises(ValueError):
        Mesh((2, 2, 2), (0, 0, 0), (1, 1, 1), 2, bounds=([0, 0.6, 0.5], [0, 0.5, 1], [0, 0.5, 1]))
    with pytest.raises(ValueError):
        Mesh((2, 2, 2), (0, 0, 0), (1, 1, 1), 2, bounds=([0, 0.5], [0, 0.5, 1], [0, 0.5, 1]))
    with pytest.raises(ValueError):
        Mesh((2, 2, 2), (0, 0, 0), (1, 1, 1), 2, bounds=([0, 0.5, 1.1], [0, 0.5, 1], [0, 0.5, 1]))


def test_uniform_bounds_reproduce_uniform_mesh():
    s = tiny()
    a = EFEModel(s)
    s.bounds = tuple(np.linspace(-8.0, 8.0, 5) for _ in range(3))
    b = EFEModel(s)
    Ha, Hb = a.hamiltonian(a.v_nuc), b.hamiltonian(b.v_nuc)
    assert abs(Ha - Hb).max() < 1e-13 * abs(Ha).max()
    np.testing.assert_allclose(b.S, a.S, atol=1e-13)
    np.testing.assert_allclose(b.D, a.D, rtol=1e-14)


def test_graded_box_levels_converge_at_2p():
    L = np.array([16.0, 12.0, 14.0])
    b0 = ([0.0, 3.0, 8.5, 12.0, 16.0], [0.0, 2.0, 6.5, 12.0], [0.0, 5.0, 7.0, 10.0, 14.0])
    n = np.array([(a, b, c) for a in range(1, 4) for b in range(1, 4) for c in range(1, 4)])
    exact = np.sort(0.5 * math.pi ** 2 * np.sum(n ** 2 / L ** 2, axis=1))[:5]
    errs = []
    for bounds in (b0, tuple(_halve(b) for b in b0)):
        s = gaussian_box(1, 8.0, 4)
        s.ncell = tuple(len(b) - 1 for b in bounds)
        s.lo, s.hi = (0.0, 0.0, 0.0), tuple(L)
        s.bounds = bounds
        m = EFEModel(s)
        lam = _lowest(m, np.zeros(m.mesh.n_quad), 5)
        errs.append(np.abs(lam - exact) / exact)
    assert np.all(errs[1] < 2e-6), errs[1]
    # ground level: rate 2^(2p) = 256 for p = 4 under halving (allow 150)
    assert errs[0][0] / errs[1][0] > 150, errs[0][0] / errs[1][0]


def test_graded_harmonic_oscillator_levels():
    s = trap(omega=1.0, ncell=6, half=6.0, degree=4)
    s.bounds = tuple(graded_bounds(-6.0, 6.0, 6, 1.5) for _ in range(3))
    m = EFEModel(s)
    v = 0.5 * np.sum(m.qpts ** 2, axis=1)
    lam = _lowest(m, v, 4)
    np.testing.assert_allclose(lam, [1.5, 2.5, 2.5, 2.5], rtol=2e-3)
    assert np.ptp(lam[1:]) < 1e-10      # the mesh is the same on every axis


def _gaussian_poisson(bounds, solver):
    Q, s = 2.0, 1.0
    spec = gaussian_box(len(bounds[0]) - 1, 8.0, 4)
    spec.ncell = tuple(len(b) - 1 for b in bounds)
    spec.bounds = bounds
    m = EFEModel(spec)
    r = np.linalg.norm(m.qpts, axis=1)
    rho = Q * (math.pi * s * s) ** -1.5 * np.exp(-r * r / (s * s))
    rn = np.linalg.norm(m.mesh.node_coords(), axis=1)
    exact = np.where(rn > 0, Q * erf(rn / s) / np.where(rn > 0, rn, 1.0), 2 * Q / (s * math.sqrt(math.pi)))
    m._poisson_setup()
    g = exact[m._poisson["Bn"]]
    return m.hartree(rho, solver=solver, boundary=g), exact


def test_graded_poisson_gaussian_charge():
    b0 = tuple(graded_bounds(-8.0, 8.0, 4, 1.2) + 0.0 * d for d in range(3))
    e = []
    for bounds in (b0, tuple(_halve(b) for b in b0)):
        phi, exact = _gaussian_poisson(bounds, "direct")
        e.append(np.abs(phi - exact).max())
    assert e[1] < 5e-3, e
    assert e[0] / e[1] > 16, e
    p1, _ = _gaussian_poisson(b0, "direct")
    p2, _ = _gaussian_poisson(b0, "fdm")
    p3, _ = _gaussian_poisson(b0, "cg")
    assert np.abs(p1 - p2).max() < 1e-12 * np.abs(p1).max()
    assert np.abs(p1 - p3).max() < 1e-10 * np.abs(p1).max()


def test_graded_enrichment_and_energy_functional():
    m = EFEModel(tiny_graded())
    np.testing.assert_allclose(m.S.T @ m.Mee @ m.S, np.eye(m.nk), atol=1e-12)
    np.testing.assert_allclose(np.diag(m.MAA), 1.0, atol=1e-12)
    rng = np.random.default_rng(5)
    X = np.zeros(m.n_rows, dtype=np.complex128)
    X[m.interior] = rng.standard_normal(len(m.interior)) * 0.01
    X[m.mesh.n_nodes:] = rng.standard_normal(m.nk) + 1j * rng.standard_normal(m.nk)
    v = m.v_nuc + 0.1 * np.sin(m.qpts[:, 0])
    e_matrix = np.real(np.vdot(X, m.hamiltonian(v) @ X))
    psiC = np.where(m.bnd, 0.0, X[:m.mesh.n_nodes] / np.sqrt(m.D))
    psiE = m.S @ X[m.mesh.n_nodes:]
    xt = psiC - m.c @ psiE
    e_direct = 0.0
    for c in range(m.mesh.n_cells):
        pts, w, B, G = m.shape(c)
        nodes = m.mesh.cell_nodes(c)
        val = B @ xt[nodes]
        grad = np.stack([G[d] @ xt[nodes] for d in range(3)], axis=1)
        if m.mesh.is_enr[c]:
            NA, dNA = m._atomic(pts, True)
            val = val + (NA * m.enr_scale) @ psiE
            grad = grad + np.einsum("qnd,n,n->qd", dNA, m.enr_scale, psiE)
        vq = v[m.mesh.q_off[c]:m.mesh.q_off[c + 1]]
        e_direct += np.sum(w * (0.5 * np.sum(np.abs(grad) ** 2, axis=1) + vq * np.abs(val) ** 2))
    assert abs(e_matrix - e_direct) < 1e-10 * abs(e_direct)


def test_graded_shape_gradients_against_differences():
    """The per-cell gradient scaling: G[d] of a graded cell against differences of B."""
    m = EFEModel(tiny_graded())
    c = 37
    pts, w, B, G = m.shape(c)
    xt = np.random.default_rng(2).standard_normal(m.mesh.nloc)
    # interpolate at shifted points through the Lagrange basis of the reference cube
    from oracle.fe import lagrange
    e = m.mesh.cell_ijk(c)
    lo = np.array([m.mesh.bounds[d][e[d]] for d in range(3)])
    h = m.mesh.cell_size(c)
    P = m.mesh.p + 1

    def val(x):
        xi = 2.0 * (x - lo) / h - 1.0
        V = [lagrange(m.mesh.xg, xi[:, d])[0] for d in range(3)]
        return np.einsum("qa,qb,qc,cba->q", V[0], V[1], V[2], xt.reshape(P, P, P))

    eps = 1e-6
    for d in range(3):
        dp, dm = pts.copy(), pts.copy()
        dp[:, d] += eps
        dm[:, d] -= eps
        np.testing.assert_allclose(G[d] @ xt, (val(dp) - val(dm)) / (2 * eps), atol=1e-6 * np.abs(G[d] @ xt).max())
    np.testing.assert_allclose(B @ xt, val(pts), atol=1e-12)
