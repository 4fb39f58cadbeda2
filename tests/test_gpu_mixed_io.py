"""Reduced-precision products (FP32, BF16 and split BF16 blocks) at orbital counts
whose row lengths are awkward for their FP32 / BF16 rows: 1 orbital (2 real columns,
rows padded to 4), 3 (6 -> 8) and 60 (120 real columns: two column chunks of the
cell products).  The products read a reduced-precision copy of the Lanczos vector
kept in the memory of the next Krylov slot and leave their result in the output
block of the exponential; these checks cover that placement against the FP64
oracle of the tiny system with occupations (2, 1, 0, ...):

* Hbar X (the standalone product: efe_apply_H) against the assembled oracle
  operator;
* the exponential of a seeded block with the oracle's Krylov dimensions replayed;
* one Magnus-2 step with the oracle's Krylov dimensions replayed (dipole and
  orbitals), then the captured (hipGraph) step bitwise equal to the host-driven
  one from the same state.

Bounds by product type (relative, max norm): FP32 products 1e-6, split BF16
2e-4, BF16 2e-2 (operands rounded to 2^-9: H Hbar X errors of a few 1e-3).
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

BOUND = {"f32": 1e-6, "bf16x3": 2e-4, "bf16": 2e-2}


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


@pytest.mark.parametrize("dtype", ["f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("norb", [1, 3, 60])
def test_reduced_precision_rows(dtype, norb):
    from workloads import tiny
    from oracle.model import EFEModel
    from oracle.propagate import Propagator, lanczos_expm
    from paper_2210_14421_amd.efe import Context
    occ = np.concatenate([[2.0, 1.0][:norb], np.zeros(max(0, norb - 2))])
    spec = dataclasses.replace(tiny(), occ=occ)
    print(f"{dtype}, {norb} orbitals: oracle model", flush=True)
    model = EFEModel(spec)
    rng = np.random.default_rng(700 + norb)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])

    def block():
        Z = rng.standard_normal((len(act), norb)) + 1j * rng.standard_normal((len(act), norb))
        Xb = np.zeros((model.n_rows, norb), dtype=np.complex128)
        Xb[act] = np.linalg.qr(Z)[0]
        return Xb

    X, B = block(), block()
    H = model.hamiltonian_from_density(model.density(X))
    bound = BOUND[dtype]
    ctx = Context(spec, dtype=dtype, kmax=64)
    try:
        ctx.set_hamiltonian(_dev(X), 0.0)
        e_hx = _rel(ctx.apply_H(_dev(B)).cpu().numpy(), H @ B)
        ref, kref, _ = lanczos_expm(H, 0.2, B, tol=1e-10, kmax=64)
        Bd = _dev(B)
        ctx.lanczos_expm(Bd, 0.2, k_force=kref)
        e_lz = _rel(Bd.cpu().numpy(), ref)
        prop = Propagator(model, X)
        mu_ref, kp, kc = prop.step(spec.dt)
        Psi = _dev(X)
        st = ctx.magnus_step(Psi, 0.0, spec.dt, k_force=np.array([kp, kc]))
        e_mu = float(np.max(np.abs(np.array(st["mu"]) - mu_ref)) / np.max(np.abs(mu_ref)))
        e_x = _rel(Psi.cpu().numpy(), prop.X)
        print(f"{dtype}, {norb} orbitals: Hbar X {e_hx:.1e}, exp {e_lz:.1e}, step dipole {e_mu:.1e}, "
              f"orbitals {e_x:.1e} (bound {bound:.0e})", flush=True)
        assert e_hx < bound and e_lz < bound and e_mu < bound and e_x < bound
        # the captured step from the same state equals the host-driven step bit for bit
        P1, P2 = _dev(X), _dev(X)
        ctx.set_hamiltonian(P1, 0.0)
        s1 = ctx.magnus_step(P1, 0.0, spec.dt)
        ctx.set_hamiltonian(P2, 0.0)
        s2 = ctx.magnus_step(P2, 0.0, spec.dt, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(P1, P2), float((P1 - P2).abs().max())
        assert np.array_equal(s1["mu"], s2["mu"])
        assert list(s1["k_pred"]) == list(s2["k_pred"]) and list(s1["k_corr"]) == list(s2["k_corr"])
    finally:
        ctx.close()
