"""Host logic of the library (no GPU): the C-ABI loads, exports every declared
symbol, and its host plan of the discretisation agrees with the FP64 oracle.

The plan is the library's own C++ set-up (enrichment normalisation, the
orthogonalising coefficients c = D^-1 b, M^ee and S = (M^ee)^-1/2, static
kinetic couplings, Poisson boundary data); the oracle computes the same
quantities independently in NumPy.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from workloads import tiny, tiny_graded, trap, na_cluster

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    path = os.path.join(ROOT, "paper_2210_14421_amd", "libefe.so")
    if not os.path.exists(path):
        pytest.skip("libefe.so not built")
    return path


def test_exports_every_declared_symbol():
    path = _lib()
    lib = ctypes.CDLL(path)
    header = open(os.path.join(ROOT, "include", "efe.h")).read()
    names = re.findall(r"^(?:efe_status|const char \*)\s*(\w+)\(", header, flags=re.M)
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    from paper_2210_14421_amd import efe
    assert sorted(names) == sorted(efe.EXPORTED)


@pytest.fixture(scope="module", params=["uniform", "graded"])
def tiny_pair(request):
    """The tiny system on its uniform mesh and on a graded, axis-dependent one (Sec. 2.7)."""
    _lib()
    from paper_2210_14421_amd.efe import Plan
    from oracle.model import EFEModel
    s = tiny() if request.param == "uniform" else tiny_graded()
    return Plan(s), EFEModel(s)


def test_plan_sizes(tiny_pair):
    p, m = tiny_pair
    assert p.n_nodes == m.mesh.n_nodes
    assert p.n_quad == m.mesh.n_quad
    assert p.n_kept == m.nk
    assert p.n_tcells == len(m.tcells)
    np.testing.assert_array_equal(p.get("is_enr", p.n_cells).astype(bool), m.mesh.is_enr)


def test_plan_mass_and_enrichment(tiny_pair):
    p, m = tiny_pair
    ne = m.spec.nenr
    np.testing.assert_allclose(p.get("D", p.n_nodes), m.D, rtol=1e-14)
    np.testing.assert_allclose(p.get("enr_scale", ne), m.enr_scale, rtol=1e-12)
    np.testing.assert_allclose(p.get("MAA", ne * ne).reshape(ne, ne), m.MAA, atol=1e-13)
    np.testing.assert_allclose(p.get("Mee", ne * ne).reshape(ne, ne), m.Mee, atol=1e-13)
    c = p.get("c", p.n_nodes * ne).reshape(-1, ne)
    assert np.abs(c - m.c).max() < 1e-12 * np.abs(m.c).max()
    S = p.get("S", ne * m.nk).reshape(ne, m.nk)
    assert np.abs(S - m.S).max() < 1e-11 * np.abs(m.S).max()


@pytest.mark.parametrize("degree", [2, 3, 6])
def test_plan_enrichment_every_degree(degree):
    """The enrichment set-up at the degrees the workloads do not use.  Degree 6
    has 343 local nodes per cell: the (T-cell slot, local node) pairs of the
    union rows must keep local indices past 255 (a byte-wide field wrapped them
    and gave an indefinite M^ee with fewer than five directions kept)."""
    import dataclasses
    _lib()
    from paper_2210_14421_amd.efe import Plan
    from oracle.model import EFEModel
    s = dataclasses.replace(tiny(), degree=degree)
    p, m = Plan(s), EFEModel(s)
    ne = s.nenr
    assert p.n_nodes == m.mesh.n_nodes and p.n_kept == m.nk == ne
    np.testing.assert_allclose(p.get("MAA", ne * ne).reshape(ne, ne), m.MAA, atol=1e-13)
    np.testing.assert_allclose(p.get("Mee", ne * ne).reshape(ne, ne), m.Mee, atol=1e-13)
    c = p.get("c", p.n_nodes * ne).reshape(-1, ne)
    assert np.abs(c - m.c).max() < 1e-12 * np.abs(m.c).max()
    S = p.get("S", ne * m.nk).reshape(ne, m.nk)
    assert np.abs(S - m.S).max() < 1e-10 * np.abs(m.S).max()
    Kce = np.zeros((m.mesh.n_nodes, ne))
    for cell in m.tcells:
        pts, w, B, G = m.shape(cell)
        NE, dNE = m.enrichment_on_cell(cell, grad=True)
        np.add.at(Kce, m.mesh.cell_nodes(cell), 0.5 * sum(G[d].T @ (w[:, None] * dNE[d]) for d in range(3)))
    Kce[m.bnd] = 0.0
    got = p.get("Kce", p.n_nodes * ne).reshape(-1, ne)
    assert np.abs(got - Kce).max() < 1e-11 * np.abs(Kce).max()


def test_plan_many_enrichment_functions():
    """lattice13: 52 enrichment functions, all kept, 52 nonzero on a central T-cell."""
    _lib()
    from paper_2210_14421_amd.efe import Plan
    from oracle.model import EFEModel
    from workloads import lattice13
    s = lattice13()
    p, m = Plan(s), EFEModel(s)
    ne = s.nenr
    assert p.n_kept == m.nk == ne == 52
    np.testing.assert_allclose(p.get("Mee", ne * ne).reshape(ne, ne), m.Mee, atol=1e-13)
    c = p.get("c", p.n_nodes * ne).reshape(-1, ne)
    assert np.abs(c - m.c).max() < 1e-12 * np.abs(m.c).max()
    S = p.get("S", ne * m.nk).reshape(ne, m.nk)
    assert np.abs(S - m.S).max() < 1e-11 * np.abs(m.S).max()


def test_plan_static_potential(tiny_pair):
    p, m = tiny_pair
    np.testing.assert_allclose(p.get("vstatic", p.n_quad), m.v_nuc + m.v_trap, rtol=1e-13, atol=1e-13)


def test_plan_kinetic_coupling(tiny_pair):
    """Kce = 1/2 int grad N_i . grad N^E, Kee = 1/2 int grad N^E . grad N^E (oracle basis functions)."""
    p, m = tiny_pair
    ne = m.spec.nenr
    Kce = np.zeros((m.mesh.n_nodes, ne))
    Kee = np.zeros((ne, ne))
    for c in m.tcells:
        pts, w, B, G = m.shape(c)
        NE, dNE = m.enrichment_on_cell(c, grad=True)
        np.add.at(Kce, m.mesh.cell_nodes(c), 0.5 * sum(G[d].T @ (w[:, None] * dNE[d]) for d in range(3)))
        Kee += 0.5 * sum(dNE[d].T @ (w[:, None] * dNE[d]) for d in range(3))
    Kce[m.bnd] = 0.0
    got = p.get("Kce", p.n_nodes * ne).reshape(-1, ne)
    assert np.abs(got - Kce).max() < 1e-11 * np.abs(Kce).max()
    np.testing.assert_allclose(p.get("Kee", ne * ne).reshape(ne, ne), Kee, rtol=1e-11, atol=1e-12)


def test_plan_poisson_boundary(tiny_pair):
    p, m = tiny_pair
    m._poisson_setup()
    P = m._poisson
    g = p.get("gbnd", p.n_nodes)
    np.testing.assert_allclose(g[P["Bn"]], P["g"], rtol=1e-14)
    assert np.all(g[m.interior] == 0.0)
    lift = p.get("lift", p.n_nodes)
    np.testing.assert_allclose(lift[m.interior], P["KIB"] @ P["g"], rtol=1e-11, atol=1e-12)


def test_plan_trap_without_enrichment():
    _lib()
    from paper_2210_14421_amd.efe import Plan
    from oracle.model import EFEModel
    s = trap(omega=1.0, ncell=4, half=6.0, degree=4)
    p, m = Plan(s), EFEModel(s)
    assert p.n_kept == 0 and p.n_tcells == 0
    np.testing.assert_allclose(p.get("vstatic", p.n_quad), m.v_nuc + m.v_trap, rtol=1e-13)


def test_plan_duplicate_enrichment_dropped():
    _lib()
    from paper_2210_14421_amd.efe import Plan
    s = tiny()
    s.enr_atom = np.concatenate([s.enr_atom, [0]]).astype(np.int32)
    s.enr_l = np.concatenate([s.enr_l, [0]]).astype(np.int32)
    s.enr_m = np.concatenate([s.enr_m, [0]]).astype(np.int32)
    s.enr_zeta = np.concatenate([s.enr_zeta, [3.0]])
    p = Plan(s)
    assert p.n_kept == 5


def test_plan_rejects_bad_input():
    _lib()
    from paper_2210_14421_amd.efe import Plan, EfeError
    s = tiny()
    s.degree = 9
    with pytest.raises(EfeError) as e:
        Plan(s)
    assert e.value.status == -1
    s = tiny()
    s.enr_zeta = np.array([3.0, -1.0, 1.0, 1.0, 1.0])
    with pytest.raises(EfeError):
        Plan(s)
    # graded meshes: boundaries must run strictly from lo to hi, and be finite
    for bad in ([-8.0, -2.0, -2.0, 3.0, 8.0], [-7.0, -2.0, 0.0, 3.0, 8.0], [-8.0, -2.0, 0.0, 3.0, 8.5]):
        s = tiny_graded()
        s.bounds = (np.array(bad), s.bounds[1], s.bounds[2])
        with pytest.raises(EfeError) as e:
            Plan(s)
        assert e.value.status == -1
    s = tiny_graded()
    s.bounds = (s.bounds[0], np.array([-8.0, np.nan, 0.0, 3.0, 8.0]), s.bounds[2])
    with pytest.raises(EfeError) as e:
        Plan(s)
    assert e.value.status == -6


def test_plan_na2_matches_oracle_setup():
    """A degree-5 cluster with overlapping atoms: c, M^ee, S against the oracle."""
    _lib()
    from paper_2210_14421_amd.efe import Plan
    from oracle.model import EFEModel
    s = na_cluster(2, seed=2)
    p, m = Plan(s), EFEModel(s)
    ne = s.nenr
    assert p.n_kept == m.nk
    np.testing.assert_allclose(p.get("Mee", ne * ne).reshape(ne, ne), m.Mee, atol=1e-13)
    # the 3s functions are nearly in the classical span: lambda_min/lambda_max of
    # M^ee is ~1e-6, so S = (M^ee)^-1/2 is reproducible only to ~kappa * eps
    lam = np.linalg.eigvalsh(m.Mee)
    kappa = lam[-1] / lam[0]
    assert kappa > 1e5
    S = p.get("S", ne * m.nk).reshape(ne, m.nk)
    assert np.abs(S - m.S).max() < 1e-12 * kappa * np.abs(m.S).max()


def test_field_vjp_against_oracle_derivatives():
    """efe_field_vjp (host arithmetic of the library) against the oracle's dE/dtheta
    and central differences of the oracle's field E(t), on the 24-parameter pulse
    of the adjoint workload and at the step and midpoint times of 40 steps."""
    _lib()
    from paper_2210_14421_amd.efe import make_field, field_vjp, EfeError
    from oracle.adjoint import field_derivatives, field_from_params
    from workloads import adjoint_field_params
    theta = adjoint_field_params(7, 8, (1e-3, 1e-2), (0.05, 0.5))
    m = len(theta) // 3
    t0, s, dt = 4.0, 2.0, 0.02
    f, keep = make_field(2, theta[:m], theta[m:2 * m], theta[2 * m:], t0, s)
    t = np.sort(np.concatenate([dt * np.arange(40), dt * np.arange(40) + 0.5 * dt]))
    g = np.random.default_rng(3).standard_normal(len(t))
    got = field_vjp(f, t, g)
    ref = sum(gi * field_derivatives(theta, t0, s, ti) for gi, ti in zip(g, t))
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-16 * np.max(np.abs(ref)))
    h = 1e-6
    fd = np.zeros_like(theta)
    for p in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        Fp, Fm = field_from_params(tp, t0, s), field_from_params(tm, t0, s)
        fd[p] = sum(gi * (Fp.E(ti) - Fm.E(ti)) for gi, ti in zip(g, t)) / (2 * h)
    np.testing.assert_allclose(got, fd, rtol=1e-6, atol=1e-8 * np.max(np.abs(fd)))
    f0, k0 = make_field(2)                                 # no field: nothing to differentiate
    with pytest.raises(EfeError):
        field_vjp(f0, t, g)
    with pytest.raises(EfeError):
        field_vjp(f, t, np.where(np.arange(len(t)) == 3, np.nan, g))
    del keep, k0
