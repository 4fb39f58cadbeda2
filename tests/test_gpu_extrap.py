"""Magnus-2 with the extrapolated midpoint Hamiltonian on the GPU (magnus_step_extrap).

* tiny: kick, then 100 steps against the oracle's stored trajectory of the same
  scheme (tests/golden/tiny_extrap.npz), Krylov dimensions replayed: the first
  two steps are predictor-corrector steps, the rest extrapolated (k_pred = 0);
  the second half runs without rebuilding the end-of-step Hamiltonian, which
  the extrapolated step does not read.  Bar: e_mu <= 1e-8, as for the
  predictor-corrector trajectory.
* the record of densities restarts on efe_set_hamiltonian and on a new dt; a
  predictor-corrector start without a current Hamiltonian is refused.
* Na8: two predictor-corrector and two extrapolated steps; orthonormality, the
  first two steps identical, and the dipole of the extrapolated steps within 1%
  of the predictor-corrector's.  The Na8 state (enrichment directions plus
  noise) is far from stationary: core-valence beats turn by about 0.8 rad per
  step of 0.02 au, so the two midpoint rules differ at the 0.1-1% level here
  (parity of the extrapolated scheme itself is the tiny test).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def tiny_env(golden_dir):
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    print("tiny extrapolated: GPU context", flush=True)
    ctx = Context(spec, dtype="f64", kmax=64)
    X0 = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]
    yield spec, ctx, X0
    ctx.close()


def test_extrap_trajectory_parity(tiny_env, golden_dir):
    spec, ctx, X0 = tiny_env
    traj = np.load(os.path.join(golden_dir, "tiny_extrap.npz"))
    Psi = _dev(X0)
    ctx.lanczos_expm(Psi, -spec.kick, op="z", k_force=traj["k_kick"])
    ctx.set_hamiltonian(Psi, 0.0)
    mus = [ctx.dipole(Psi)]
    ks = traj["k"]
    t = 0.0
    for n in range(len(ks)):
        st = ctx.magnus_step(Psi, t, spec.dt, k_force=ks[n], scheme="extrap", keep_ham=n < 50)
        t += spec.dt
        mus.append(st["mu"])
        if n < 2:
            assert np.all(st["k_pred"] > 0)
        else:
            assert np.all(st["k_pred"] == 0)
        if n % 25 == 0:
            print(f"step {n}: mu_z {st['mu'][2]:.9e} ref {traj['mu'][n + 1][2]:.9e}", flush=True)
    mus = np.array(mus)
    ref = traj["mu"]
    e_mu = np.max(np.linalg.norm(mus - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    print("tiny extrapolated 100-step e_mu =", e_mu)
    assert e_mu <= 1e-8
    Xf = Psi.cpu().numpy()
    assert _rel(Xf, traj["X_final"]) < 1e-7
    G = Xf.conj().T @ Xf
    assert np.abs(G - np.eye(spec.norb)).max() < 1e-9


def test_extrap_history_restarts(tiny_env):
    from paper_2210_14421_amd.efe import EfeError
    spec, ctx, X0 = tiny_env
    Psi = _dev(X0)
    ctx.lanczos_expm(Psi, -spec.kick, op="z")
    ctx.set_hamiltonian(Psi, 0.0)
    kinds = []
    t = 0.0
    for dt in (0.05, 0.05, 0.05, 0.05, 0.025, 0.025):
        st = ctx.magnus_step(Psi, t, dt, scheme="extrap")
        t += dt
        kinds.append("pc" if np.all(st["k_pred"] > 0) else "ex")
    # three densities of dt = 0.05 after two steps; a new dt keeps one
    assert kinds == ["pc", "pc", "ex", "ex", "pc", "pc"]
    # set_hamiltonian restarts the record
    ctx.set_hamiltonian(Psi, t)
    st = ctx.magnus_step(Psi, t, 0.025, scheme="extrap")
    assert np.all(st["k_pred"] > 0)
    # without the end-of-step Hamiltonian a predictor-corrector start is refused
    ctx.set_hamiltonian(Psi, t)
    ctx.magnus_step(Psi, t, 0.05, scheme="extrap", keep_ham=False)   # a predictor-corrector step keeps it
    ctx.magnus_step(Psi, t + 0.05, 0.05, scheme="extrap", keep_ham=False)
    ctx.magnus_step(Psi, t + 0.1, 0.05, scheme="extrap", keep_ham=False)   # extrapolated, Hamiltonian dropped
    with pytest.raises(EfeError):
        ctx.magnus_step(Psi, t + 0.15, 0.05)
    with pytest.raises(EfeError):
        ctx.magnus_step(Psi, t + 0.15, 0.025, scheme="extrap")
    ctx.magnus_step(Psi, t + 0.15, 0.05, scheme="extrap", keep_ham=False)   # still extrapolated: fine
    G = Psi.cpu().numpy()
    G = G.conj().T @ G
    assert np.abs(G - np.eye(spec.norb)).max() < 1e-9


def test_extrap_na8_steps():
    from workloads import na8
    from paper_2210_14421_amd.efe import Context
    spec = na8()
    print("na8: predictor-corrector vs extrapolated steps", flush=True)
    ctx = Context(spec, kmax=24)
    try:
        P0 = ctx.initial_state()
        ctx.lanczos_expm(P0, -spec.kick, op="z")
        Pa, Pb = P0.clone(), P0.clone()
        mus = {}
        for name, P, scheme in (("pc", Pa, "pc"), ("ex", Pb, "extrap")):
            ctx.set_hamiltonian(P, 0.0)
            out = []
            for n in range(4):
                st = ctx.magnus_step(P, n * spec.dt, spec.dt, scheme=scheme, keep_ham=False)
                out.append(st["mu"])
                if scheme == "extrap":
                    assert np.all(st["k_pred"] > 0) == (n < 2)
            mus[name] = np.array(out)
        for P in (Pa, Pb):
            G = P.conj().T @ P
            assert float((G - torch.eye(G.shape[0], dtype=G.dtype, device=G.device)).abs().max()) < 1e-11
        d = np.abs(mus["ex"] - mus["pc"]).max() / np.abs(mus["pc"][:, 2]).max()
        print("Na8 dipole, extrapolated vs predictor-corrector (4 steps):", d, mus["ex"][:, 2], mus["pc"][:, 2])
        assert np.array_equal(mus["ex"][:2], mus["pc"][:2])
        assert d < 1e-2
    finally:
        ctx.close()
