"""GPU parity on graded tensor-product meshes (per-axis cell boundaries, Sec. 2.7).

Every kernel that maps a cell from the reference cube (the point coordinates and
weights of the rebuild, the 1-D stiffness and mass of the cell blocks and of the
sum-factorised apply, the coupling partials, the Poisson right-hand side, the
dipole) takes its cell's own edge lengths; the same checks as on the uniform
mesh hold at the same bars:
* tiny_graded (axis-dependent boundaries): density 1e-12, Hartree 1e-11, Hbar X
  1e-12 for the stored FP64 blocks and the sum-factorised apply, the z kick with
  identical k, and 50 Magnus steps with the oracle's k replayed (e_mu <= 1e-8),
  the oracle's values stored by the golden script;
* Na8 in a 70-bohr box on a sinh-graded 24^3 mesh: the sampled rows of Hbar X,
  the density at sampled points, the dipole and the Hartree potential at sampled
  nodes against the oracle at full size.
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
    from workloads import tiny_graded
    from oracle.model import EFEModel
    from paper_2210_14421_amd.efe import Context
    spec = tiny_graded()
    print("tiny_graded: oracle model and GPU context", flush=True)
    model = EFEModel(spec)
    X0 = np.load(os.path.join(golden_dir, "tiny_graded_ground_state.npz"))["X"]
    ctx = Context(spec, dtype="f64", kmax=64)
    yield spec, model, X0, ctx
    ctx.close()


def _random_block(model, norb, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((model.n_rows, norb), dtype=np.complex128)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X[act] = rng.standard_normal((len(act), norb)) + 1j * rng.standard_normal((len(act), norb))
    return X


def test_graded_fields(env):
    spec, model, X0, ctx = env
    assert ctx.n_rows == model.n_rows and ctx.n_quad == model.mesh.n_quad
    rho = ctx.density(_dev(X0)).cpu().numpy()
    ref = model.density(X0)
    assert _rel(rho, ref) < 1e-12
    phi, it = ctx.hartree(_dev(ref))
    e = _rel(phi.cpu().numpy(), model.hartree(ref))
    print(f"tiny_graded: density ok, Hartree rel err {e:.2e}")
    assert e < 1e-11
    np.testing.assert_allclose(ctx.dipole(_dev(X0)), model.dipole(ref), rtol=0, atol=1e-12)


def test_graded_apply_H(env):
    spec, model, X0, ctx = env
    ctx.set_hamiltonian(_dev(X0), 0.0)
    X = _random_block(model, spec.norb, 11)
    Y = ctx.apply_H(_dev(X)).cpu().numpy()
    ref = model.hamiltonian_from_density(model.density(X0)) @ X
    e = _rel(Y, ref)
    print(f"tiny_graded Hbar X rel err {e:.2e}")
    assert e < 1e-12
    assert np.abs(Y[:model.mesh.n_nodes][model.bnd]).max() == 0.0


def test_graded_sum_factorised_apply_H(env):
    from paper_2210_14421_amd.efe import Context
    spec, model, X0, _ = env
    sf = Context(spec, dtype="f64sf", kmax=64)
    try:
        sf.set_hamiltonian(_dev(X0), 0.0)
        X = _random_block(model, spec.norb, 12)
        Y = sf.apply_H(_dev(X)).cpu().numpy()
        ref = model.hamiltonian_from_density(model.density(X0)) @ X
        e = _rel(Y, ref)
        print(f"tiny_graded sum-factorised Hbar X rel err {e:.2e}")
        assert e < 1e-12
    finally:
        sf.close()


def test_graded_kick(env):
    from oracle.propagate import lanczos_expm
    spec, model, X0, ctx = env
    ref, kref, _ = lanczos_expm(model.position_operator(2), -1e-3, X0, tol=1e-10, kmax=64)
    Xd = _dev(X0)
    ku, _ = ctx.lanczos_expm(Xd, -1e-3, op="z")
    assert list(ku) == list(kref)
    assert _rel(Xd.cpu().numpy(), ref) < 1e-11


def test_graded_trajectory(env, golden_dir):
    """50 Magnus-2 steps after a z kick, Krylov dimensions replayed from the oracle."""
    spec, model, X0, ctx = env
    traj = np.load(os.path.join(golden_dir, "tiny_graded_traj.npz"))
    Psi = _dev(X0)
    ctx.lanczos_expm(Psi, -spec.kick, op="z", k_force=traj["k_kick"])
    ctx.set_hamiltonian(Psi, 0.0)
    mus = [ctx.dipole(Psi)]
    t = 0.0
    for n in range(len(traj["k"])):
        st = ctx.magnus_step(Psi, t, spec.dt, k_force=traj["k"][n])
        t += spec.dt
        mus.append(st["mu"])
    mus = np.array(mus)
    ref = traj["mu"]
    e_mu = np.max(np.linalg.norm(mus - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    print(f"tiny_graded 50-step e_mu = {e_mu:.2e}")
    assert e_mu <= 1e-8
    assert _rel(Psi.cpu().numpy(), traj["X_final"]) < 1e-7
    # adaptive run from the same start takes the oracle's Krylov dimensions
    P2 = _dev(X0)
    ctx.lanczos_expm(P2, -spec.kick, op="z")
    ctx.set_hamiltonian(P2, 0.0)
    st = ctx.magnus_step(P2, 0.0, spec.dt)
    assert list(st["k_pred"]) == list(traj["k"][0][0]) and list(st["k_corr"]) == list(traj["k"][0][1])


def test_graded_na8_sampled(golden_dir):
    from workloads import na8_graded
    from paper_2210_14421_amd.efe import Context
    path = os.path.join(golden_dir, "na8_graded_sampled.npz")
    gold = np.load(path)
    spec = na8_graded()
    print("Na8_graded: GPU context", flush=True)
    ctx = Context(spec, dtype="f64", kmax=4)
    try:
        assert ctx.n_kept == int(gold["nk"])
        Psi = ctx.initial_state()
        N = ctx.n_nodes
        X = Psi.cpu().numpy()
        assert _rel(X[gold["rows"]], gold["X0_rows"]) < 1e-10
        assert _rel(X[N:], gold["X0_E"]) < 1e-8
        rho = ctx.density(Psi).cpu().numpy()
        e_rho = _rel(rho[gold["q_idx"]], gold["rho_q"])
        mu = ctx.dipole(Psi)
        e_mu = float(np.max(np.abs(mu - gold["mu"])) / np.max(np.abs(gold["mu"])))
        phi, _ = ctx.hartree(torch.from_numpy(rho).to("cuda"))
        e_phi = _rel(phi.cpu().numpy()[gold["phi_idx"]], gold["phi"])
        ctx.set_hamiltonian(Psi, 0.0)
        Y = ctx.apply_H(Psi).cpu().numpy()
        e_rows = _rel(Y[gold["rows"]], gold["Y_rows"])
        e_enr = _rel(Y[N:], gold["Y_E"])
        print(f"Na8_graded: rho {e_rho:.2e} mu {e_mu:.2e} phi {e_phi:.2e} "
              f"Hbar X node rows {e_rows:.2e} enrichment rows {e_enr:.2e}")
        assert e_rho < 1e-11 and e_mu < 1e-10 and e_phi < 1e-10
        assert e_rows < 1e-8 and e_enr < 1e-7
    finally:
        ctx.close()
