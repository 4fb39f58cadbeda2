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
