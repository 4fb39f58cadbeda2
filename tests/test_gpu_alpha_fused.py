"""The three-term Lanczos step with alpha_j taken from the products (FP64 blocks, the
partial scheme's default) against the same scheme with alpha_j from a dot pass over the
new vector (reorth="partial_dot").

The products leave, per column, each cell's sum of X (Hbar_c X_c) and the coupling's
enrichment terms X_E (G^T X[R] + Y_E) (Sec. 2.2-2.3); their fixed-order sum is x^H Hbar x,
the Lanczos coefficient of Sec. 2.6, up to rounding.  The two forms must choose the same
Krylov dimensions and agree to rounding:
* tiny (one-pass coupling) and lattice13 (52 functions: the row-tile coupling kernels),
  a random block, tau = 0.3: identical k per column, results within 1e-12;
* Na2 and Na8 at full size: one kicked Magnus step each: identical k, dipoles within
  1e-11 relative, orbitals within 1e-10.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


def _spec(name):
    import workloads
    if name == "tiny":
        return workloads.tiny()
    return workloads.lattice13()


@pytest.mark.parametrize("name", ["tiny", "lattice13"])
def test_alpha_from_products_lanczos(name):
    from oracle.model import EFEModel
    from paper_2210_14421_amd.efe import Context
    spec = _spec(name)
    print(f"{name}: oracle model (for the active rows and the initial state)", flush=True)
    model = EFEModel(spec)
    rng = np.random.default_rng(31)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X0 = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    X0[act] = np.linalg.qr(rng.standard_normal((len(act), spec.norb)) +
                           1j * rng.standard_normal((len(act), spec.norb)))[0]
    X = np.zeros_like(X0)
    X[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    out = []
    for reorth in ("partial", "partial_dot"):
        ctx = Context(spec, dtype="f64", kmax=64, reorth=reorth)
        try:
            ctx.set_hamiltonian(_dev(X0), 0.0)
            Xd = _dev(X)
            ku, _ = ctx.lanczos_expm(Xd, 0.3)
            out.append((list(ku), Xd.cpu().numpy()))
        finally:
            ctx.close()
    e = _rel(out[0][1], out[1][1])
    print(f"{name}: k {out[0][0]} / {out[1][0]}, rel diff {e:.2e}")
    assert out[0][0] == out[1][0]
    assert e < 1e-12


@pytest.mark.parametrize("name", ["na2", "na8"])
def test_alpha_from_products_step(name):
    from workloads import na8, na_cluster
    from paper_2210_14421_amd.efe import Context
    spec = na8() if name == "na8" else na_cluster(2, seed=2)
    res = []
    for reorth in ("partial", "partial_dot"):
        print(f"{name} {reorth}: context", flush=True)
        ctx = Context(spec, dtype="f64", kmax=40, reorth=reorth)
        try:
            Psi = ctx.initial_state()
            ctx.lanczos_expm(Psi, -spec.kick, op="z")
            ctx.set_hamiltonian(Psi, 0.0)
            st = ctx.magnus_step(Psi, 0.0, spec.dt)
            res.append((list(st["k_pred"]), list(st["k_corr"]), np.array(st["mu"]), Psi.cpu().numpy()))
        finally:
            ctx.close()
    (kp0, kc0, mu0, P0), (kp1, kc1, mu1, P1) = res
    d = float(np.max(np.abs(mu0 - mu1)) / np.max(np.abs(mu1)))
    e = _rel(P0, P1)
    print(f"{name} one step: k {kp0[:3]}.. / {kp1[:3]}..; dipole rel diff {d:.2e}; orbitals {e:.2e}")
    assert kp0 == kp1 and kc0 == kc1
    assert d < 1e-11
    assert e < 1e-10
