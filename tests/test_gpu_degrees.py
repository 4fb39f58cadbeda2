"""GPU parity at the FE degrees the workloads do not use: 2, 3 and 6 (degrees 4
and 5 are the tiny and Na clusters' own).

The tiny system (4^3 cells on [-8, 8]^3, one Z = 3 atom, five enrichment
functions) at each degree, with a seeded orthonormal two-orbital block, against
the oracle at the same degree:
* density at the points and Hbar X with FP64 blocks (bound b below), Hartree
  potential (1e-11), dipole (1e-12); Hbar X with FP32 blocks (1e-6) and BF16
  blocks (1e-2);
* one Magnus-2 step with the oracle's Krylov dimensions replayed (dipole and
  orbitals 1e-10), and the same dimensions chosen adaptively;
* the sum-factorised products, built for degrees 4 and 5 only, are refused
  with EFE_ERR_ARG.
Degree 6 (343 local nodes, 22 M tiles) runs the cell kernel's six-tile form at
one workgroup per CU; degrees 2 and 3
(27 and 64 local nodes) the two-tile form with most M tiles empty, and the
smallest Poisson grids (7^3 and 11^3 unknowns).

Bound b: the enrichment directions come from M^ee = M^AA - b^T D^-1 b, a
cancellation between terms of unit size whose result has smallest eigenvalue
lambda (5.7e-2 at degree 2 down to 7.8e-5 at degree 6, where the FE space
nearly contains the atomic functions).  Rounding in the enrichment rows then
grows as eps / lambda; b = max(1e-12, 50 eps / lambda) (measured errors are
2 to 11 eps / lambda).
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


@pytest.mark.parametrize("degree", [2, 3, 6])
def test_degree_parity(degree):
    from workloads import tiny
    from oracle.model import EFEModel
    from oracle.propagate import Propagator
    from paper_2210_14421_amd.efe import Context, EfeError
    spec = dataclasses.replace(tiny(), degree=degree)
    print(f"degree {degree}: oracle model", flush=True)
    model = EFEModel(spec)
    rng = np.random.default_rng(100 + degree)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    Z = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    X[act] = np.linalg.qr(Z)[0]
    rho_ref = model.density(X)
    H = model.hamiltonian_from_density(rho_ref)
    bound = max(1e-12, 50 * np.finfo(float).eps / float(np.min(model.Mee_eig[0])))
    ctx = Context(spec, dtype="f64", kmax=64)
    try:
        assert ctx.n_rows == model.n_rows and ctx.n_quad == model.mesh.n_quad
        rho = ctx.density(_dev(X)).cpu().numpy()
        e_rho = _rel(rho, rho_ref)
        phi, _ = ctx.hartree(_dev(rho_ref))
        e_phi = _rel(phi.cpu().numpy(), model.hartree(rho_ref))
        mu = ctx.dipole(_dev(X))
        ctx.set_hamiltonian(_dev(X), 0.0)
        B = np.zeros_like(X)
        B[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
        e_hx = _rel(ctx.apply_H(_dev(B)).cpu().numpy(), H @ B)
        print(f"degree {degree}: rho {e_rho:.1e} phi {e_phi:.1e} Hbar X {e_hx:.1e} (bound {bound:.1e})", flush=True)
        assert e_rho < bound and e_phi < 1e-11 and e_hx < bound
        np.testing.assert_allclose(mu, model.dipole(rho_ref), rtol=0, atol=1e-12)
        # one step, Krylov dimensions replayed, then adaptive from the same start
        prop = Propagator(model, X)
        mu_ref, kp, kc = prop.step(spec.dt)
        Psi = _dev(X)
        st = ctx.magnus_step(Psi, 0.0, spec.dt, k_force=np.array([kp, kc]))
        e_mu = float(np.max(np.abs(np.array(st["mu"]) - mu_ref)) / np.max(np.abs(mu_ref)))
        e_x = _rel(Psi.cpu().numpy(), prop.X)
        print(f"degree {degree}: step k {list(kp)}/{list(kc)}, dipole {e_mu:.1e}, orbitals {e_x:.1e}", flush=True)
        assert e_mu < 1e-10 and e_x < 1e-10
        Psi = _dev(X)
        ctx.set_hamiltonian(Psi, 0.0)
        st = ctx.magnus_step(Psi, 0.0, spec.dt)
        assert list(st["k_pred"]) == list(kp) and list(st["k_corr"]) == list(kc)
    finally:
        ctx.close()
    for dtype, tol in (("f32", 1e-6), ("bf16", 1e-2), ("bf16x3", 1e-4)):
        c = Context(spec, dtype=dtype, kmax=64)
        try:
            c.set_hamiltonian(_dev(X), 0.0)
            e = _rel(c.apply_H(_dev(B)).cpu().numpy(), H @ B)
            print(f"degree {degree}: {dtype} Hbar X {e:.1e}", flush=True)
            assert e < tol
        finally:
            c.close()
    with pytest.raises(EfeError) as e:
        Context(spec, dtype="f64sf", kmax=64)
    assert e.value.status == -1
