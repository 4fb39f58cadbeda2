"""GPU parity on the tiny system (one Li-like atom, 4^3 cells of degree 4).

Each stage of the HIP path is compared element by element with the FP64 oracle
on the same inputs: the oracle's SCF ground state (golden fixture written by the
oracle) and the system of workloads.tiny().  Tolerances are FP64 rounding-level
(relative 1e-11 .. 1e-12); the 200-step trajectory is compared against the
oracle's stored trajectory with the oracle's Krylov dimensions replayed, at the
dipole bar e_mu <= 1e-8.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def env(golden_dir):
    from workloads import tiny
    from oracle.model import EFEModel
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    print("tiny: building oracle model and GPU context", flush=True)
    model = EFEModel(spec)
    gs = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))
    ctx = Context(spec, dtype="f64", kmax=64)
    yield spec, model, gs["X"], ctx
    ctx.close()


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


def test_dims(env):
    from paper_2210_14421_amd.efe import Plan
    spec, model, X0, ctx = env
    assert ctx.n_rows == model.n_rows
    assert ctx.n_nodes == model.mesh.n_nodes
    assert ctx.n_quad == model.mesh.n_quad
    assert ctx.n_union_rows == Plan(spec).n_union_rows > 0


def test_density_parity(env):
    spec, model, X0, ctx = env
    rho = ctx.density(_dev(X0)).cpu().numpy()
    ref = model.density(X0)
    assert _rel(rho, ref) < 1e-12


def test_hartree_parity(env):
    spec, model, X0, ctx = env
    ref_rho = model.density(X0)
    phi, it = ctx.hartree(_dev(ref_rho))
    ref = model.hartree(ref_rho)
    assert _rel(phi.cpu().numpy(), ref) < 1e-11
    assert it <= 3


def test_apply_H_parity(env):
    spec, model, X0, ctx = env
    Xd = _dev(X0)
    ctx.set_hamiltonian(Xd, 0.0)
    rng = np.random.default_rng(11)
    X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    Y = ctx.apply_H(_dev(X)).cpu().numpy()
    H = model.hamiltonian_from_density(model.density(X0))
    ref = H @ X
    assert _rel(Y, ref) < 1e-12
    # boundary rows stay zero
    assert np.abs(Y[:model.mesh.n_nodes][model.bnd]).max() == 0.0


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("bf16", 1e-2), ("bf16x3", 1e-4)])
def test_apply_H_reduced_precision(env, dtype, tol):
    """FP32 products (FP32 blocks and operands, FP32 accumulation), BF16 products
    (BF16 blocks and orbital rows on the BF16 MFMA) and split BF16 products (hi/lo
    pairs, three BF16 MFMAs): Hbar X against the FP64 oracle.  The bound is the
    operand rounding (2^-24, 2^-9 and about 2^-16 relative per entry) amplified by
    the cancellation in the kinetic rows."""
    from paper_2210_14421_amd.efe import Context
    spec, model, X0, _ = env
    ctx = Context(spec, dtype=dtype, kmax=64)
    try:
        ctx.set_hamiltonian(_dev(X0), 0.0)
        rng = np.random.default_rng(11)
        X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
        act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
        X[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
        Y = ctx.apply_H(_dev(X)).cpu().numpy()
        ref = model.hamiltonian_from_density(model.density(X0)) @ X
        e = _rel(Y, ref)
        print(f"{dtype} Hbar X rel err {e:.2e}")
        assert e < tol
    finally:
        ctx.close()


def test_lanczos_parity(env):
    from oracle.propagate import lanczos_expm
    spec, model, X0, ctx = env
    ctx.set_hamiltonian(_dev(X0), 0.0)
    H = model.hamiltonian_from_density(model.density(X0))
    rng = np.random.default_rng(12)
    X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    X[model.interior] = rng.standard_normal((len(model.interior), spec.norb))
    X[model.mesh.n_nodes:] = rng.standard_normal((model.nk, spec.norb))
    X /= np.linalg.norm(X, axis=0)
    ref, kref, eref = lanczos_expm(H, 0.05, X, tol=1e-10, kmax=64)
    Xd = _dev(X)
    ku, er = ctx.lanczos_expm(Xd, 0.05)
    assert list(ku) == list(kref)
    assert _rel(Xd.cpu().numpy(), ref) < 1e-11
    # The estimate |tau| beta_k beta0 |u_k| takes u_k = [exp(-i tau T_k)]_{k,1}
    # from a sum of O(1) terms that cancels down to ~1e-10, so two correct
    # implementations agree in it only to ~k eps / |u_k| ~ 1e-5 relative.
    np.testing.assert_allclose(er, eref, rtol=1e-5, atol=1e-22)


def test_kick_parity(env):
    from oracle.propagate import lanczos_expm
    spec, model, X0, ctx = env
    Z = model.position_operator(2)
    ref, kref, _ = lanczos_expm(Z, -1e-3, X0, tol=1e-10, kmax=64)
    Xd = _dev(X0)
    ku, _ = ctx.lanczos_expm(Xd, -1e-3, op="z")
    assert list(ku) == list(kref)
    assert _rel(Xd.cpu().numpy(), ref) < 1e-11


def test_magnus_trajectory_parity(env, golden_dir):
    """200 Magnus-2 steps after a z kick, Krylov dimensions replayed from the oracle."""
    spec, model, X0, ctx = env
    traj = np.load(os.path.join(golden_dir, "tiny_traj.npz"))
    Psi = _dev(X0)
    kk = traj["k_kick"]
    ctx.lanczos_expm(Psi, -spec.kick, op="z", k_force=kk)
    ctx.set_hamiltonian(Psi, 0.0)
    mus = [ctx.dipole(Psi)]
    t = 0.0
    ks = traj["k"]
    for n in range(spec.nsteps):
        st = ctx.magnus_step(Psi, t, spec.dt, k_force=ks[n])
        t += spec.dt
        mus.append(st["mu"])
        if n % 50 == 0:
            print(f"step {n}: mu_z {st['mu'][2]:.9e} ref {traj['mu'][n + 1][2]:.9e}", flush=True)
    mus = np.array(mus)
    ref = traj["mu"]
    e_mu = np.max(np.linalg.norm(mus - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    print("tiny 200-step e_mu =", e_mu)
    assert e_mu <= 1e-8
    Xf = Psi.cpu().numpy()
    assert _rel(Xf, traj["X_final"]) < 1e-7
    G = Xf.conj().T @ Xf
    assert np.abs(G - np.eye(spec.norb)).max() < 1e-9


def test_magnus_adaptive_close(env, golden_dir):
    """Adaptive Krylov dimensions on both sides: same k, same trace to 1e-8 over 20 steps."""
    spec, model, X0, ctx = env
    traj = np.load(os.path.join(golden_dir, "tiny_traj.npz"))
    Psi = _dev(X0)
    ctx.lanczos_expm(Psi, -spec.kick, op="z")
    ctx.set_hamiltonian(Psi, 0.0)
    t = 0.0
    for n in range(20):
        st = ctx.magnus_step(Psi, t, spec.dt)
        t += spec.dt
        assert list(st["k_pred"]) == list(traj["k"][n][0])
        assert list(st["k_corr"]) == list(traj["k"][n][1])
    ref = traj["mu"][20]
    assert np.linalg.norm(st["mu"] - ref) / np.linalg.norm(ref) < 1e-8
