"""GPU parity on the tiny system with Gauss rules and cell counts that the
workloads do not use:
* "rules": degree 4 with 6 points per axis on ordinary cells and 12 on
  enrichment cells (the workloads take p + 1 and 2p + 2), which sends the
  density to its general interpolation path;
* "rules16": degree 5 with 6 and 16 points (16 is the largest rule: the
  rebuild's and the MFMA coupling partials' largest point sets);
* "odd": 3 x 5 x 2 cells, non-cubic (16/3 x 16/5 x 8 bohr): colour classes of
  unequal size, the last cell of an axis odd or even;
* "thin": 1 x 2 x 5 cells: a single cell along x, so two of the eight colour
  classes are empty and no x face is shared.
Each against the oracle on the same seeded orthonormal two-orbital block:
density and Hbar X (1e-12), Hartree (1e-11), dipole (1e-12), one Magnus-2 step
with the oracle's Krylov dimensions replayed (1e-10) and chosen adaptively;
FP32 blocks (1e-6); the sum-factorised products where they are built (degree
4 or 5 with the default rules), refused with EFE_ERR_ARG elsewhere.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CASES = {
    "rules": dict(quad_cell=6, quad_enr=12),
    "rules16": dict(degree=5, quad_cell=6, quad_enr=16),
    "odd": dict(ncell=(3, 5, 2)),
    "thin": dict(ncell=(1, 2, 5)),
}


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


@pytest.mark.parametrize("case", list(CASES))
def test_mesh_and_rule_parity(case):
    from workloads import tiny
    from oracle.model import EFEModel
    from oracle.propagate import Propagator
    from paper_2210_14421_amd.efe import Context, EfeError
    spec = dataclasses.replace(tiny(), **CASES[case])
    print(f"{case}: oracle model", flush=True)
    model = EFEModel(spec)
    rng = np.random.default_rng(7)
    act = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    X = np.zeros((model.n_rows, spec.norb), dtype=np.complex128)
    Z = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    X[act] = np.linalg.qr(Z)[0]
    B = np.zeros_like(X)
    B[act] = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
    rho_ref = model.density(X)
    H = model.hamiltonian_from_density(rho_ref)
    ctx = Context(spec, dtype="f64", kmax=64)
    try:
        assert ctx.n_rows == model.n_rows and ctx.n_quad == model.mesh.n_quad
        e_rho = _rel(ctx.density(_dev(X)).cpu().numpy(), rho_ref)
        phi, _ = ctx.hartree(_dev(rho_ref))
        e_phi = _rel(phi.cpu().numpy(), model.hartree(rho_ref))
        np.testing.assert_allclose(ctx.dipole(_dev(X)), model.dipole(rho_ref), rtol=0, atol=1e-12)
        ctx.set_hamiltonian(_dev(X), 0.0)
        e_hx = _rel(ctx.apply_H(_dev(B)).cpu().numpy(), H @ B)
        print(f"{case}: rho {e_rho:.1e} phi {e_phi:.1e} Hbar X {e_hx:.1e}", flush=True)
        assert e_rho < 1e-12 and e_phi < 1e-11 and e_hx < 1e-12
        prop = Propagator(model, X)
        mu_ref, kp, kc = prop.step(spec.dt)
        Psi = _dev(X)
        st = ctx.magnus_step(Psi, 0.0, spec.dt, k_force=np.array([kp, kc]))
        e_mu = float(np.max(np.abs(np.array(st["mu"]) - mu_ref)) / np.max(np.abs(mu_ref)))
        e_x = _rel(Psi.cpu().numpy(), prop.X)
        print(f"{case}: step k {list(kp)}/{list(kc)}, dipole {e_mu:.1e}, orbitals {e_x:.1e}", flush=True)
        assert e_mu < 1e-10 and e_x < 1e-10
        Psi = _dev(X)
        ctx.set_hamiltonian(Psi, 0.0)
        st = ctx.magnus_step(Psi, 0.0, spec.dt)
        assert list(st["k_pred"]) == list(kp) and list(st["k_corr"]) == list(kc)
    finally:
        ctx.close()
    c = Context(spec, dtype="f32", kmax=64)
    try:
        c.set_hamiltonian(_dev(X), 0.0)
        assert _rel(c.apply_H(_dev(B)).cpu().numpy(), H @ B) < 1e-6
    finally:
        c.close()
    default_rules = spec.quad_cell in (0, spec.degree + 1) and spec.quad_enr in (0, 2 * spec.degree + 2)
    if spec.degree in (4, 5) and default_rules:
        c = Context(spec, dtype="f64sf", kmax=64)
        try:
            c.set_hamiltonian(_dev(X), 0.0)
            e = _rel(c.apply_H(_dev(B)).cpu().numpy(), H @ B)
            print(f"{case}: sum-factorised Hbar X {e:.1e}", flush=True)
            assert e < 1e-12
        finally:
            c.close()
    else:
        with pytest.raises(EfeError) as e:
            Context(spec, dtype="f64sf", kmax=64)
        assert e.value.status == -1
