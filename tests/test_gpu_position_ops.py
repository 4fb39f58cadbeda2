"""The position operators along x, y and z on the GPU (the kick exp(i kappa Xbar_d)
of Sec. 3.2 for each direction), against the oracle's, on tiny_graded, whose
cell boundaries differ per axis so that an exchanged axis shows: for each
direction, the exponential of a seeded random block with identical Krylov
dimensions per column (1e-11; this is the check that separates the axes), and
a kick of the stored ground state followed by the dipole (1e-12 absolute; a
kick is nearly a pointwise phase, so it moves the density only slightly).
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


@pytest.mark.parametrize("direction", [0, 1, 2])
def test_position_operator_parity(direction, golden_dir):
    from workloads import tiny_graded
    from oracle.model import EFEModel
    from oracle.propagate import lanczos_expm
    from paper_2210_14421_amd.efe import Context
    spec = tiny_graded()
    model = EFEModel(spec)
    op = "xyz"[direction]
    Zd = model.position_operator(direction)
    rng = np.random.default_rng(90 + direction)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    X[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    X /= np.linalg.norm(X, axis=0)
    X0 = np.load(os.path.join(golden_dir, "tiny_graded_ground_state.npz"))["X"]
    ctx = Context(spec, dtype="f64", kmax=64)
    try:
        ref, kref, _ = lanczos_expm(Zd, 0.3, X, tol=1e-10, kmax=64)
        Xd = _dev(X)
        ku, _ = ctx.lanczos_expm(Xd, 0.3, op=op)
        e = _rel(Xd.cpu().numpy(), ref)
        print(f"{op}: exp(-0.3 i {op}bar) k {list(ku)} (oracle {list(kref)}), rel err {e:.1e}", flush=True)
        assert list(ku) == list(kref) and e < 1e-11
        kicked, _, _ = lanczos_expm(Zd, -1e-2, X0, tol=1e-10, kmax=64)
        P = _dev(X0)
        ctx.lanczos_expm(P, -1e-2, op=op)
        mu = ctx.dipole(P)
        mu_ref = model.dipole(model.density(kicked))
        print(f"{op}: kicked dipole {mu} (oracle {mu_ref})", flush=True)
        np.testing.assert_allclose(mu, mu_ref, rtol=0, atol=1e-12)
    finally:
        ctx.close()


@pytest.mark.parametrize("direction", [0, 1, 2])
def test_driven_step_along_each_axis(direction, golden_dir):
    """Three Magnus-2 steps of tiny_graded under a Gaussian pulse along x, y or z
    (E = 0.05 sin(0.4 t + 0.3) exp(-(t - 0.1)^2), the potential -E x_d of eq.
    (VField)), the oracle's Krylov dimensions replayed: dipoles and orbitals 1e-10,
    and the dipole moves most along the field."""
    from workloads import tiny_graded
    from oracle.model import EFEModel, Field
    from oracle.propagate import Propagator
    from paper_2210_14421_amd.efe import Context, make_field
    spec = tiny_graded()
    model = EFEModel(spec)
    X0 = np.load(os.path.join(golden_dir, "tiny_graded_ground_state.npz"))["X"]
    A, w, phi, t0, s = [0.05], [0.4], [0.3], 0.1, 1.0
    fo = Field(direction=direction, A=np.array(A), w=np.array(w), phi=np.array(phi), t0=t0, s=s)
    prop = Propagator(model, X0, t=0.0, field=fo)
    fg, keep = make_field(direction, A, w, phi, t0, s)
    ctx = Context(spec, dtype="f64", kmax=64)
    try:
        P = _dev(X0)
        ctx.set_hamiltonian(P, 0.0, field=fg)
        mu0 = model.dipole(model.density(X0))
        t = 0.0
        for n in range(3):
            mu_ref, kp, kc = prop.step(spec.dt)
            st = ctx.magnus_step(P, t, spec.dt, field=fg, k_force=np.array([kp, kc]))
            t += spec.dt
            e_mu = float(np.max(np.abs(np.array(st["mu"]) - mu_ref)) / np.max(np.abs(mu_ref)))
            e_x = _rel(P.cpu().numpy(), prop.X)
            print(f"{'xyz'[direction]} field, step {n}: dipole {e_mu:.1e}, orbitals {e_x:.1e}", flush=True)
            assert e_mu < 1e-10 and e_x < 1e-10
        dmu = np.abs(np.array(st["mu"]) - mu0)
        assert int(np.argmax(dmu)) == direction
        del keep
    finally:
        ctx.close()
