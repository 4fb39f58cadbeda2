"""Pins for the oracle's discretisation: closed forms and invariants.

* Dirichlet box: Hbar eigenvalues -> pi^2 (n1^2+n2^2+n3^2) / (8 L^2) for [-L, L]^3,
  converging like h^(2p) (kinetic term, lumped mass, Loewdin scaling, boundary).
* harmonic oscillator v = |x|^2/2: eigenvalues 3/2, 5/2 (x3) (potential term).
* Gaussian charge: the FE Hartree potential converges to Q erf(r/s)/r (Poisson
  right-hand side, stiffness, Dirichlet lift); FDM, CG and a sparse direct solve
  agree.
* enrichment: M^ee positive definite; S^T M^ee S = I; a duplicated enrichment
  function is dropped by canonical orthogonalisation; energy of a physical
  function computed from the orbital's Loewdin coefficients equals the energy
  functional evaluated directly from the raw (N^C, N^A) representation.
* nuclear potential of a Gaussian-smeared charge: -Z/r far away, -2Z/(sigma sqrt(pi)) at 0.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import erf

from oracle.model import EFEModel
from oracle.enrich import atomic_function
from workloads import gaussian_box, trap, tiny


def _lowest(m, v, k):
    H = m.hamiltonian(v)
    act = np.concatenate([m.interior, m.mesh.n_nodes + np.arange(m.nk)])
    return sla.eigh(H[act][:, act].toarray(), eigvals_only=True, subset_by_index=[0, k - 1])


def test_box_levels_converge_at_2p():
    L = 8.0
    exact = np.array([3, 6, 6, 6, 9]) * math.pi ** 2 / (8 * L * L)
    errs = []
    for nc in (2, 4):
        m = EFEModel(gaussian_box(nc, L, 4))
        lam = _lowest(m, np.zeros(m.mesh.n_quad), 5)
        errs.append(np.abs(lam - exact) / exact)
    assert np.all(errs[1] < 3e-6)
    # ground level: rate h^(2p) = 256 for p = 4 (allow 200)
    assert errs[0][0] / errs[1][0] > 200
    # three-fold degeneracy of the first excited level
    m = EFEModel(gaussian_box(4, L, 4))
    lam = _lowest(m, np.zeros(m.mesh.n_quad), 4)
    assert np.ptp(lam[1:4]) < 1e-12


def test_constant_potential_shifts_levels():
    m = EFEModel(gaussian_box(4, 8.0, 4))
    lam0 = _lowest(m, np.zeros(m.mesh.n_quad), 2)
    lam1 = _lowest(m, np.full(m.mesh.n_quad, 0.7), 2)
    # exact shift up to the lumped-vs-consistent mass gap
    np.testing.assert_allclose(lam1 - lam0, 0.7, rtol=1e-5)


def test_harmonic_oscillator_levels():
    m = EFEModel(trap(omega=1.0, ncell=4, half=6.0, degree=4))
    v = 0.5 * np.sum(m.qpts ** 2, axis=1)
    lam = _lowest(m, v, 4)
    np.testing.assert_allclose(lam, [1.5, 2.5, 2.5, 2.5], rtol=1e-2)
    assert np.ptp(lam[1:]) < 1e-10


def _gaussian_poisson(nc, solver):
    Q, s = 2.0, 1.0
    m = EFEModel(gaussian_box(nc, 8.0, 4))
    r = np.linalg.norm(m.qpts, axis=1)
    rho = Q * (math.pi * s * s) ** -1.5 * np.exp(-r * r / (s * s))
    rn = np.linalg.norm(m.mesh.node_coords(), axis=1)
    exact = np.where(rn > 0, Q * erf(rn / s) / np.where(rn > 0, rn, 1.0), 2 * Q / (s * math.sqrt(math.pi)))
    m._poisson_setup()
    g = exact[m._poisson["Bn"]]
    phi = m.hartree(rho, solver=solver, boundary=g)
    return phi, exact


def test_poisson_gaussian_charge_converges():
    e = []
    for nc in (2, 4):
        phi, exact = _gaussian_poisson(nc, "direct")
        e.append(np.abs(phi - exact).max())
    assert e[1] < 0.03
    assert e[0] / e[1] > 16


def test_poisson_solvers_agree():
    p1, _ = _gaussian_poisson(4, "direct")
    p2, _ = _gaussian_poisson(4, "fdm")
    p3, _ = _gaussian_poisson(4, "cg")
    assert np.abs(p1 - p2).max() < 1e-12 * np.abs(p1).max()
    assert np.abs(p1 - p3).max() < 1e-10 * np.abs(p1).max()


def test_nuclear_potential_limits():
    m = EFEModel(tiny())
    pts = np.array([[0.0, 0.0, 0.0], [7.0, 0.0, 0.0], [0.0, 3.0, 4.0]])
    v = m.nuclear_potential(pts)
    assert abs(v[0] + 2 * 3.0 / (0.2 * math.sqrt(math.pi))) < 1e-12
    assert abs(v[1] + 3.0 / 7.0) < 1e-14
    assert abs(v[2] + 3.0 / 5.0) < 1e-14


def test_enrichment_function_gradient():
    rng = np.random.default_rng(3)
    pts = rng.uniform(-5, 5, size=(50, 3))
    R = np.array([0.3, -0.2, 0.1])
    e = 1e-6
    for (l, mm) in ((0, 0), (1, -1), (1, 0), (1, 1)):
        v, g = atomic_function(pts, R, l, mm, 1.3, 6.0, grad=True)
        for d in range(3):
            dp = pts.copy(); dp[:, d] += e
            dm = pts.copy(); dm[:, d] -= e
            fd = (atomic_function(dp, R, l, mm, 1.3, 6.0) - atomic_function(dm, R, l, mm, 1.3, 6.0)) / (2 * e)
            np.testing.assert_allclose(g[:, d], fd, atol=1e-8)
    # l = 1, m = 0 is the z function
    v = atomic_function(np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]]), np.zeros(3), 1, 0, 1.0, 6.0)
    assert v[0] > 0 and v[1] == 0.0


def test_enrichment_overlap_and_loewdin():
    m = EFEModel(tiny())
    lam = np.linalg.eigvalsh(m.Mee)
    assert np.all(lam > 0)
    np.testing.assert_allclose(m.S.T @ m.Mee @ m.S, np.eye(m.nk), atol=1e-12)
    # unit norm of the atomic parts under the enrichment rule
    np.testing.assert_allclose(np.diag(m.MAA), 1.0, atol=1e-13)


def test_duplicate_enrichment_is_dropped():
    s = tiny()
    s.enr_atom = np.concatenate([s.enr_atom, [0]]).astype(np.int32)
    s.enr_l = np.concatenate([s.enr_l, [0]]).astype(np.int32)
    s.enr_m = np.concatenate([s.enr_m, [0]]).astype(np.int32)
    s.enr_zeta = np.concatenate([s.enr_zeta, [3.0]])   # same as the 1s
    m = EFEModel(s)
    assert m.n_dropped == 1 and m.nk == 5
    np.testing.assert_allclose(m.S.T @ m.Mee @ m.S, np.eye(5), atol=1e-10)


def test_energy_functional_matches_loewdin_hamiltonian():
    """X^H Hbar X equals int 1/2 |grad psi|^2 + v |psi|^2 of the physical function."""
    m = EFEModel(tiny())
    rng = np.random.default_rng(5)
    X = np.zeros(m.n_rows, dtype=np.complex128)
    X[m.interior] = rng.standard_normal(len(m.interior)) * 0.01
    X[m.mesh.n_nodes:] = rng.standard_normal(m.nk) + 1j * rng.standard_normal(m.nk)
    v = m.v_nuc + 0.1 * np.sin(m.qpts[:, 0])
    H = m.hamiltonian(v)
    e_matrix = np.real(np.vdot(X, H @ X))
    # direct: raw representation psi = sum xt_i N_i + sum psiE_nu N^A_nu
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


def test_hamiltonian_symmetric_and_boundary_free():
    m = EFEModel(tiny())
    H = m.hamiltonian(m.v_nuc)
    assert abs(H - H.T).max() < 1e-13
    bn = np.nonzero(m.bnd)[0]
    assert abs(H[bn]).max() == 0.0


def test_hamiltonian_rows_match_full_matrix():
    """The row-restricted route (used at full Na8 size) equals the assembled Hbar."""
    m = EFEModel(tiny())
    rng = np.random.default_rng(8)
    v = m.v_nuc + 0.2 * np.cos(m.qpts[:, 1])
    X = rng.standard_normal((m.n_rows, 2)) + 1j * rng.standard_normal((m.n_rows, 2))
    X[:m.mesh.n_nodes][m.bnd] = 0.0
    rows = rng.choice(m.mesh.n_nodes, size=40, replace=False)
    Yr, YE = m.hamiltonian_rows(v, X, rows)
    Y = m.hamiltonian(v) @ X
    np.testing.assert_allclose(Yr, Y[rows], rtol=0, atol=1e-12 * np.abs(Y).max())
    np.testing.assert_allclose(YE, Y[m.mesh.n_nodes:], rtol=0, atol=1e-12 * np.abs(Y).max())
