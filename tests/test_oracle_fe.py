"""Pins for the oracle's FE layer: quadrature exactness, Lagrange basis, mesh sums.

Closed forms: int_{-1}^{1} x^k dx = 2/(k+1) for even k, 0 for odd k; GLL with
p+1 points is exact to degree 2p-1, Gauss with n points to degree 2n-1.
"""
import numpy as np
import pytest

from oracle.fe import gll_rule, gauss_rule, lagrange, Mesh
from workloads import tiny, na8


def _moment(k):
    return 0.0 if k % 2 else 2.0 / (k + 1)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_gll_exactness(p):
    x, w = gll_rule(p)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    for k in range(2 * p):
        assert abs(np.sum(w * x ** k) - _moment(k)) < 1e-14
    # degree 2p is NOT exact for p >= 1 (the lumped mass is an approximation)
    assert abs(np.sum(w * x ** (2 * p)) - _moment(2 * p)) > 1e-6


def test_gll_known_values():
    # p = 2: nodes -1, 0, 1 with weights 1/3, 4/3, 1/3 (Simpson)
    x, w = gll_rule(2)
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    # p = 3: interior nodes +-1/sqrt(5), weights 1/6, 5/6
    x, w = gll_rule(3)
    np.testing.assert_allclose(x[1:3], [-1 / np.sqrt(5), 1 / np.sqrt(5)], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("n", [2, 5, 6, 10, 12])
def test_gauss_exactness(n):
    x, w = gauss_rule(n)
    for k in range(2 * n):
        assert abs(np.sum(w * x ** k) - _moment(k)) < 1e-13


@pytest.mark.parametrize("p", [2, 4, 5])
def test_lagrange_basis(p):
    nodes, _ = gll_rule(p)
    V, dV = lagrange(nodes, nodes)
    np.testing.assert_allclose(V, np.eye(p + 1), atol=1e-14)
    x = np.linspace(-1, 1, 37)
    V, dV = lagrange(nodes, x)
    np.testing.assert_allclose(V.sum(axis=1), 1.0, atol=1e-13)     # partition of unity
    np.testing.assert_allclose(dV.sum(axis=1), 0.0, atol=1e-11)
    # interpolation of x^p is exact, its derivative too
    np.testing.assert_allclose(V @ nodes ** p, x ** p, atol=1e-13)
    np.testing.assert_allclose(dV @ nodes ** p, p * x ** (p - 1), atol=1e-11)
    # derivative against central differences
    e = 1e-6
    Vp, _ = lagrange(nodes, x + e)
    Vm, _ = lagrange(nodes, x - e)
    np.testing.assert_allclose((Vp - Vm) / (2 * e), dV, atol=1e-7)


def test_tiny_mesh_sums_and_classes():
    s = tiny()
    m = Mesh(s.ncell, s.lo, s.hi, s.degree, s.r_cut, s.R, s.qcell, s.qenr)
    assert m.n_nodes == 17 ** 3 == 4913
    assert int(m.is_enr.sum()) == 56          # all but the 8 corner cells
    assert m.n_quad == 8 * 125 + 56 * 1000
    P, W = m.all_quadrature()
    np.testing.assert_allclose(W.sum(), 16.0 ** 3, rtol=1e-14)
    np.testing.assert_allclose(m.lumped_mass().sum(), 16.0 ** 3, rtol=1e-14)
    # every quadrature point lies inside its cell
    for c in range(m.n_cells):
        ex, ey, ez = m.cell_ijk(c)
        p = P[m.q_off[c]:m.q_off[c + 1]]
        lo = m.lo + np.array([ex, ey, ez]) * 4.0
        assert np.all(p > lo) and np.all(p < lo + 4.0)
        np.testing.assert_allclose(m.cell_size(c), 4.0, rtol=1e-15)
    # cell nodes sit on the cell box, local order x fastest
    xyz = m.node_coords(m.cell_nodes(5))
    ex, ey, ez = m.cell_ijk(5)
    lo = m.lo + np.array([ex, ey, ez]) * 4.0
    assert np.all(xyz >= lo - 1e-12) and np.all(xyz <= lo + 4.0 + 1e-12)
    assert xyz[1, 0] > xyz[0, 0] and xyz[1, 1] == xyz[0, 1]


def test_na8_mesh_sizes():
    s = na8()
    m = Mesh(s.ncell, s.lo, s.hi, s.degree, s.r_cut, s.R, s.qcell, s.qenr)
    assert m.n_nodes == 121 ** 3 == 1771561
    assert int((~m.boundary_mask()).sum()) == 119 ** 3
    assert m.nloc == 216
    ne = int(m.is_enr.sum())
    assert 800 < ne < 2000
    assert m.n_quad == (m.n_cells - ne) * 216 + ne * 1728


def test_cells_of_node():
    m = Mesh((3, 2, 2), (0, 0, 0), (3, 2, 2), 2)
    # a vertex shared by 8 cells
    i = m.node_index(2, 2, 2)
    assert len(m.cells_of_node(i)) == 8
    # a cell-interior node
    assert m.cells_of_node(m.node_index(1, 1, 1)) == [0]
    # every node is in the closure of each listed cell
    for i in range(m.n_nodes):
        for c in m.cells_of_node(i):
            assert i in m.cell_nodes(c)
