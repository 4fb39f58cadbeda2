"""GPU parity at orbital counts the workloads do not use: one orbital, and 60
(120 real columns: two 96-column chunks of the cell products, and Lanczos
kernels whose rows-per-block mapping is not a multiple of the workloads').

The tiny system with occupations (2) or (2, 1, 0, ..., 0), a seeded orthonormal
block, against the oracle: density and Hbar X (1e-12), the exponential of a
random block with identical Krylov dimensions per column (1e-11), one Magnus-2
step with the oracle's Krylov dimensions replayed (1e-10) and chosen
adaptively.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


@pytest.mark.parametrize("norb", [1, 60])
def test_orbital_count_parity(norb):
    from workloads import tiny
    from oracle.model import EFEModel
    from oracle.propagate import Propagator, lanczos_expm
    from paper_2210_14421_amd.efe import Context
    occ = np.array([2.0]) if norb == 1 else np.concatenate([[2.0, 1.0], np.zeros(norb - 2)])
    spec = dataclasses.replace(tiny(), occ=occ)
    print(f"{norb} orbitals: oracle model", flush=True)
    model = EFEModel(spec)
    rng = np.random.default_rng(60 + norb)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])

    def block():
        Z = rng.standard_normal((len(act), norb)) + 1j * rng.standard_normal((len(act), norb))
        Xb = np.zeros((model.n_rows, norb), dtype=np.complex128)
        Xb[act] = np.linalg.qr(Z)[0]
        return Xb

    X, B = block(), block()
    rho_ref = model.density(X)
    H = model.hamiltonian_from_density(rho_ref)
    ctx = Context(spec, dtype="f64", kmax=64)
    try:
        e_rho = _rel(ctx.density(_dev(X)).cpu().numpy(), rho_ref)
        ctx.set_hamiltonian(_dev(X), 0.0)
        e_hx = _rel(ctx.apply_H(_dev(B)).cpu().numpy(), H @ B)
        ref, kref, _ = lanczos_expm(H, 0.2, B, tol=1e-10, kmax=64)
        Bd = _dev(B)
        ku, _ = ctx.lanczos_expm(Bd, 0.2)
        e_lz = _rel(Bd.cpu().numpy(), ref)
        print(f"{norb} orbitals: rho {e_rho:.1e} Hbar X {e_hx:.1e} exp {e_lz:.1e} (k {sorted(set(kref.tolist()))})",
              flush=True)
        assert e_rho < 1e-12 and e_hx < 1e-12
        assert list(ku) == list(kref) and e_lz < 1e-11
        prop = Propagator(model, X)
        mu_ref, kp, kc = prop.step(spec.dt)
        Psi = _dev(X)
        st = ctx.magnus_step(Psi, 0.0, spec.dt, k_force=np.array([kp, kc]))
        e_mu = float(np.max(np.abs(np.array(st["mu"]) - mu_ref)) / np.max(np.abs(mu_ref)))
        e_x = _rel(Psi.cpu().numpy(), prop.X)
        print(f"{norb} orbitals: step dipole {e_mu:.1e}, orbitals {e_x:.1e}", flush=True)
        assert e_mu < 1e-10 and e_x < 1e-10
        Psi = _dev(X)
        ctx.set_hamiltonian(Psi, 0.0)
        st = ctx.magnus_step(Psi, 0.0, spec.dt)
        assert list(st["k_pred"]) == list(kp) and list(st["k_corr"]) == list(kc)
    finally:
        ctx.close()
