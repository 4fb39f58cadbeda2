"""Sum-factorised cell products (prod_dtype EFE_F64_SF) against the oracle and the dense path.

The sum-factorised apply evaluates the same operator as the stored FP64 blocks
(Sec. 2.3): D^-1/2 (1/2 K + B^T W v B) D^-1/2 per cell, by three 1-D
contractions each way.  Bars are FP64 rounding level, as for the dense path:
* tiny: Hbar X (random block) vs the oracle's assembled matrix, 1e-12; the
  position operator (no kinetic term) through the kick, 1e-11 with identical k;
  10 Magnus steps: same k and a dipole within 1e-10 of the dense context;
* Na8: Hbar X at the sampled rows of the oracle fixture (1e-8 / 1e-7 as the
  dense test) and against the dense FP64 context on every row.
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
def tiny_env(golden_dir):
    from workloads import tiny
    from oracle.model import EFEModel
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    print("tiny: oracle model, dense and sum-factorised contexts", flush=True)
    model = EFEModel(spec)
    X0 = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]
    sf = Context(spec, dtype="f64sf", kmax=64)
    dense = Context(spec, dtype="f64", kmax=64)
    yield spec, model, X0, sf, dense
    sf.close()
    dense.close()


def test_sf_apply_H_tiny(tiny_env):
    spec, model, X0, sf, _ = tiny_env
    sf.set_hamiltonian(_dev(X0), 0.0)
    rng = np.random.default_rng(11)
    X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    Y = sf.apply_H(_dev(X)).cpu().numpy()
    ref = model.hamiltonian_from_density(model.density(X0)) @ X
    e = _rel(Y, ref)
    print(f"tiny sum-factorised Hbar X rel err {e:.2e}")
    assert e < 1e-12
    assert np.abs(Y[:model.mesh.n_nodes][model.bnd]).max() == 0.0


def test_sf_kick_tiny(tiny_env):
    from oracle.propagate import lanczos_expm
    spec, model, X0, sf, _ = tiny_env
    Z = model.position_operator(2)
    ref, kref, _ = lanczos_expm(Z, -1e-3, X0, tol=1e-10, kmax=64)
    Xd = _dev(X0)
    ku, _ = sf.lanczos_expm(Xd, -1e-3, op="z")
    assert list(ku) == list(kref)
    assert _rel(Xd.cpu().numpy(), ref) < 1e-11


def test_sf_steps_match_dense_tiny(tiny_env):
    spec, model, X0, sf, dense = tiny_env
    Ps = []
    for c in (sf, dense):
        P = _dev(X0)
        c.lanczos_expm(P, -spec.kick, op="z")
        c.set_hamiltonian(P, 0.0)
        Ps.append(P)
    t = 0.0
    for n in range(10):
        a = sf.magnus_step(Ps[0], t, spec.dt)
        b = dense.magnus_step(Ps[1], t, spec.dt)
        t += spec.dt
        assert list(a["k_pred"]) == list(b["k_pred"]) and list(a["k_corr"]) == list(b["k_corr"])
        d = np.max(np.abs(a["mu"] - b["mu"])) / np.max(np.abs(b["mu"]))
        assert d < 1e-10, (n, d)
    assert _rel(Ps[0].cpu().numpy(), Ps[1].cpu().numpy()) < 1e-10


def test_sf_apply_H_na8(golden_dir):
    from workloads import na8
    from paper_2210_14421_amd.efe import Context
    gold = np.load(os.path.join(golden_dir, "na8_sampled.npz"))
    spec = na8()
    print("na8: sum-factorised and dense contexts", flush=True)
    sf = Context(spec, dtype="f64sf", kmax=4)
    try:
        Psi = sf.initial_state()
        sf.set_hamiltonian(Psi, 0.0)
        Y = sf.apply_H(Psi).cpu().numpy()
        N = sf.n_nodes
        e_rows = _rel(Y[gold["rows"]], gold["Y_rows"])
        e_enr = _rel(Y[N:], gold["Y_E"])
        print(f"Na8 sum-factorised Hbar X: sampled node rows {e_rows:.2e}, enrichment rows {e_enr:.2e}")
        assert e_rows < 1e-8
        assert e_enr < 1e-7
    finally:
        sf.close()
    dense = Context(spec, dtype="f64", kmax=4)
    try:
        P2 = dense.initial_state()
        dense.set_hamiltonian(P2, 0.0)
        Yd = dense.apply_H(P2).cpu().numpy()
        e = _rel(Y, Yd)
        print(f"Na8 sum-factorised vs dense Hbar X, all rows: {e:.2e}")
        assert e < 1e-12
    finally:
        dense.close()
