"""The oracle's matrix-free route for large meshes, pinned to its assembled route.

`EFEModel.operator` applies Hbar cell by cell (eq. (Hmn) blocks summed into the
classical rows, the coupling, the Loewdin scaling of eq. (TDKSDiscrete2)) without
the global matrix; the assembled `EFEModel.hamiltonian` is itself pinned by the
box levels, the oscillator levels and the energy functional.  The lockstep
Lanczos driver advances independent columns together with one block product per
iteration; each column must equal its own column-by-column run.  A matrix-free
Magnus step (Hartree by fast diagonalisation) must equal the assembled step.
"""
import os

import numpy as np
import pytest

from oracle.model import EFEModel
from oracle.propagate import Propagator, lanczos_expm
from workloads import tiny, tiny_graded


@pytest.fixture(scope="module")
def model():
    return EFEModel(tiny())


def _rand_block(n, m, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))


@pytest.mark.parametrize("kinetic", [True, False])
def test_operator_equals_assembled_matrix(model, kinetic):
    rng = np.random.default_rng(5)
    v = model.v_nuc + rng.uniform(-0.3, 0.3, model.mesh.n_quad)
    H = model.hamiltonian(v, kinetic)
    Op = model.operator(v, kinetic)
    X = _rand_block(model.n_rows, 3, 6)
    X[:model.mesh.n_nodes][model.bnd] = 0.0
    Y = Op(X)
    ref = H @ X
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))
    np.testing.assert_allclose(Op(X[:, 1]), ref[:, 1], rtol=0, atol=1e-12 * np.max(np.abs(ref)))


def test_operator_on_graded_cells():
    m = EFEModel(tiny_graded())
    v = m.v_nuc + 0.1 * m.qpts[:, 0]
    X = _rand_block(m.n_rows, 2, 7)
    X[:m.mesh.n_nodes][m.bnd] = 0.0
    ref = m.hamiltonian(v) @ X
    assert np.max(np.abs(m.operator(v)(X) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_position_operator_free(model):
    X = _rand_block(model.n_rows, 2, 8)
    X[:model.mesh.n_nodes][model.bnd] = 0.0
    for d in range(3):
        ref = model.position_operator(d) @ X
        assert np.max(np.abs(model.position_operator_free(d)(X) - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("reorth", ["full", "partial"])
def test_lockstep_columns_equal_column_by_column(model, reorth):
    H = model.hamiltonian(model.v_nuc)
    X = _rand_block(model.n_rows, 4, 9)
    X[:model.mesh.n_nodes][model.bnd] = 0.0
    X[:, 2] = 0.0                               # a zero column stops at once on both routes
    Y1, k1, e1 = lanczos_expm(H, 0.2, X, tol=1e-10, kmax=64, reorth=reorth)
    Y2, k2, e2 = lanczos_expm(H, 0.2, X, tol=1e-10, kmax=64, reorth=reorth, block=True)
    assert list(k1) == list(k2) and k1[2] == 0
    assert np.max(np.abs(Y2 - Y1)) <= 1e-13 * np.max(np.abs(Y1))
    kf = np.maximum(k1 - 2, 1)
    Y3, k3, _ = lanczos_expm(H, 0.2, X, tol=1e-10, kmax=64, k_force=kf, reorth=reorth, block=True)
    Y4, k4, _ = lanczos_expm(H, 0.2, X, tol=1e-10, kmax=64, k_force=kf, reorth=reorth)
    assert list(k3) == list(k4) and np.max(np.abs(Y3 - Y4)) <= 1e-13 * np.max(np.abs(Y4))
    # at most three columns together: the same columns
    Y5, k5, _ = lanczos_expm(H, 0.2, X, tol=1e-10, kmax=64, reorth=reorth, block=True, block_cols=3)
    assert list(k5) == list(k1) and np.max(np.abs(Y5 - Y1)) <= 1e-13 * np.max(np.abs(Y1))


def test_matrix_free_step_equals_assembled_step(model, golden_dir):
    X0 = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]
    spec = model.spec
    Pa = Propagator(model, X0, tol=spec.krylov_tol, kmax=spec.kmax)
    Pm = Propagator(model, X0, tol=spec.krylov_tol, kmax=spec.kmax, matrix_free=True)
    ka, km = Pa.kick(spec.kick, 2), Pm.kick(spec.kick, 2)
    assert list(ka) == list(km)
    for _ in range(2):
        mua, kpa, kca = Pa.step(spec.dt)
        mum, kpm, kcm = Pm.step(spec.dt)
        assert list(kpa) == list(kpm) and list(kca) == list(kcm)
        assert np.linalg.norm(mum - mua) <= 1e-11 * np.linalg.norm(mua)
    assert np.max(np.abs(Pm.X - Pa.X)) <= 1e-11
