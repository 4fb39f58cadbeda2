"""Edge cases of the Lanczos exponential and the products on the GPU (tiny system).

* a zero column among live ones: it stays zero with k = 0, the others equal the
  oracle's exponential with identical k (the oracle returns zero for it too);
* ragged blocks: Hbar X and exp(-i tau Hbar) X of a single column and of
  one-column slices equal the oracle's, with the same k as inside the full block;
* error paths: a Krylov limit below the needed dimension gives EFE_ERR_NOCONV
  (-4) and leaves X unchanged, a NaN in X gives EFE_ERR_NONFINITE (-6); the
  context stays usable after both (a following exponential matches the oracle).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


@pytest.fixture(scope="module")
def env(golden_dir):
    from workloads import tiny
    from oracle.model import EFEModel
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    model = EFEModel(spec)
    X0 = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]
    ctx = Context(spec, dtype="f64", kmax=64)
    ctx.set_hamiltonian(_dev(X0), 0.0)
    H = model.hamiltonian_from_density(model.density(X0))
    yield spec, model, X0, ctx, H
    ctx.close()


def _block(model, ncol, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((model.n_rows, ncol), dtype=np.complex128)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X[act] = rng.standard_normal((len(act), ncol)) + 1j * rng.standard_normal((len(act), ncol))
    return X / np.linalg.norm(X, axis=0)


def test_zero_column(env):
    from oracle.propagate import lanczos_expm
    spec, model, X0, ctx, H = env
    X = _block(model, 2, 31)
    X[:, 0] = 0.0
    ref, kref, _ = lanczos_expm(H, 0.1, X, tol=1e-10, kmax=64)
    Xd = _dev(X)
    ku, er = ctx.lanczos_expm(Xd, 0.1)
    Y = Xd.cpu().numpy()
    assert ku[0] == 0 and kref[0] == 0 and er[0] == 0.0
    assert np.abs(Y[:, 0]).max() == 0.0
    assert ku[1] == kref[1]
    assert _rel(Y[:, 1], ref[:, 1]) < 1e-11


def test_ragged_columns(env):
    from oracle.propagate import lanczos_expm
    spec, model, X0, ctx, H = env
    X = _block(model, 2, 32)
    Y1 = ctx.apply_H(_dev(X[:, 1:2].copy())).cpu().numpy()
    assert _rel(Y1[:, 0], H @ X[:, 1]) < 1e-12
    full = _dev(X)
    kfull, _ = ctx.lanczos_expm(full, 0.2)
    for c in range(2):
        col = _dev(X[:, c:c + 1].copy())
        kc, _ = ctx.lanczos_expm(col, 0.2)
        ref, kref, _ = lanczos_expm(H, 0.2, X[:, c:c + 1], tol=1e-10, kmax=64)
        assert kc[0] == kref[0] == kfull[c]
        assert _rel(col.cpu().numpy()[:, 0], ref[:, 0]) < 1e-11
        assert _rel(col.cpu().numpy()[:, 0], full.cpu().numpy()[:, c]) < 1e-12


def test_error_paths_leave_the_context_usable(env):
    from oracle.propagate import lanczos_expm
    from paper_2210_14421_amd.efe import Context, EfeError
    spec, model, X0, _, H = env
    ctx = Context(spec, dtype="f64", kmax=3)
    try:
        ctx.set_hamiltonian(_dev(X0), 0.0)
        X = _block(model, 2, 33)
        Xd = _dev(X)
        with pytest.raises(EfeError) as e:
            ctx.lanczos_expm(Xd, 0.5)                       # needs k = 19
        assert e.value.status == -4
        assert np.array_equal(Xd.cpu().numpy(), X)          # untouched on error
        bad = X.copy()
        bad[model.interior[5], 1] = np.nan
        with pytest.raises(EfeError) as e:
            ctx.lanczos_expm(_dev(bad), 1e-4)
        assert e.value.status == -6
        # still usable: a short exponential within kmax = 3 matches the oracle
        ref, kref, _ = lanczos_expm(H, 1e-4, X, tol=1e-6, kmax=3)
        ctx.set_options(tol=1e-6)
        ku, _ = ctx.lanczos_expm(Xd, 1e-4)
        assert list(ku) == list(kref)
        assert _rel(Xd.cpu().numpy(), ref) < 1e-11
    finally:
        ctx.close()


def test_captured_step_reports_a_non_finite_orbital(env):
    """The device-driven step cannot stop early: a NaN orbital comes back as
    EFE_ERR_NONFINITE from its statistics, and a later step from good orbitals works."""
    from paper_2210_14421_amd.efe import Context, EfeError
    spec, model, X0, _, H = env
    ctx = Context(spec, dtype="f64", kmax=40)
    try:
        Psi = _dev(X0)
        ctx.set_hamiltonian(Psi, 0.0)
        Psi[model.interior[9], 0] = float("nan")
        with pytest.raises(EfeError) as e:
            ctx.magnus_step(Psi, 0.0, spec.dt, graph=True)
        assert e.value.status == -6
        Psi = _dev(X0)
        ctx.set_hamiltonian(Psi, 0.0)
        st = ctx.magnus_step(Psi, 0.0, spec.dt, graph=True)
        assert np.all(np.isfinite(st["mu"]))
    finally:
        ctx.close()
