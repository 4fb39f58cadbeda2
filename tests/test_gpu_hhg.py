"""Dipole power spectrum (power_spectrum, Sec. 3.5) and the sinusoidally driven
step on the GPU.

* power spectrum against the oracle, element by element (relative 1e-12): the
  tiny system's stored kicked trajectory, a cubic dipole (exact second
  differences) and an oscillation; argument checks;
* the driven step: the tiny system (one atom at the centre of a symmetric mesh,
  s and p enrichment) under kappa sin(pi t/T) sin(omega t) and under the
  opposite field; inversion symmetry makes the dipole odd in the field, so the
  two traces are opposite to rounding and the even harmonics of their power
  spectrum come only from the pulse envelope.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_power_spectrum_parity(golden_dir):
    from oracle.spectrum import power_spectrum as P_ref
    from paper_2210_14421_amd.efe import power_spectrum
    traj = np.load(os.path.join(golden_dir, "tiny_traj.npz"))
    mu, dt = traj["mu"], float(traj["dt"])
    w = np.linspace(0.0, 12.0, 300)
    P = power_spectrum(_gpu(mu), 2, dt, _gpu(w), 1e5).cpu().numpy()
    e = _rel(P, P_ref(mu, 2, dt, w, 1e5))
    print(f"tiny kicked trajectory: power spectrum rel err {e:.2e}")
    assert e < 1e-12
    t = 0.005 * np.arange(4001)
    cubic = np.zeros((4001, 3))
    cubic[:, 1] = 2.0 + 0.5 * t - 0.3 * t ** 2 + 0.07 * t ** 3
    osc = np.zeros((4001, 3))
    osc[:, 0] = np.sin(0.7 * t) + 0.2 * np.sin(2.1 * t)
    for mu, d in ((cubic, 1), (osc, 0)):
        w = np.linspace(0.0, 3.0, 257)
        P = power_spectrum(_gpu(mu), d, 0.005, _gpu(w), 50.0).cpu().numpy()
        assert _rel(P, P_ref(mu, d, 0.005, w, 50.0)) < 1e-12
    # three samples: one interior point with the half weight at both ends
    mu3 = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 5.0]])
    P = power_spectrum(_gpu(mu3), 2, 0.5, _gpu(np.array([0.0, 1.0])), 10.0).cpu().numpy()
    np.testing.assert_allclose(P, P_ref(mu3, 2, 0.5, [0.0, 1.0], 10.0), rtol=1e-14)


def test_power_spectrum_argument_checks():
    from paper_2210_14421_amd.efe import power_spectrum, EfeError
    mu = _gpu(np.zeros((10, 3)))
    w = _gpu(np.linspace(0.1, 1.0, 4))
    with pytest.raises(EfeError):
        power_spectrum(mu, 3, 0.1, w, 1e5)
    with pytest.raises(EfeError):
        power_spectrum(mu, 0, 0.0, w, 1e5)
    with pytest.raises(EfeError):
        power_spectrum(mu, 0, 0.1, w, -1.0)
    with pytest.raises(EfeError):
        power_spectrum(_gpu(np.zeros((2, 3))), 0, 0.1, w, 1e5)


def test_driven_tiny_is_odd_in_the_field(golden_dir):
    from workloads import tiny, hhg_field
    from paper_2210_14421_amd.efe import Context, make_field, power_spectrum
    spec = tiny()
    X0 = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]
    omega, ncyc, dt = 0.3, 3, 0.05
    traces = []
    for sign in (1.0, -1.0):
        p = hhg_field(kappa=sign * 0.01, omega=omega, ncycles=ncyc, direction=2)
        nsteps = int(round(p["T"] / dt))
        f, keep = make_field(p["direction"], p["A"], p["w"], p["phi"], p["t0"], p["s"])
        ctx = Context(spec, kmax=40)
        try:
            Psi = torch.from_numpy(np.ascontiguousarray(X0)).to("cuda")
            ctx.set_hamiltonian(Psi, 0.0, field=f)
            mus = [ctx.dipole(Psi)]
            t = 0.0
            for n in range(nsteps):
                st = ctx.magnus_step(Psi, t, dt, field=f)
                t += dt
                mus.append(st["mu"])
            traces.append(np.array(mus))
        finally:
            ctx.close()
        print(f"driven tiny ({'+' if sign > 0 else '-'}E): {nsteps} steps, mu_z(T) = {traces[-1][-1][2]:.6e}",
              flush=True)
    a, b = traces
    odd = float(np.max(np.abs(a[:, 2] + b[:, 2])) / np.max(np.abs(a[:, 2] - a[0, 2])))
    print(f"|mu_z(+E) + mu_z(-E)| / max |mu_z(+E) - mu_z(0)| = {odd:.2e}")
    assert odd < 1e-9
    # transverse components stay at zero (the field and the system are symmetric about z)
    assert np.max(np.abs(a[:, :2])) < 1e-10
    w = np.array([k * omega for k in range(1, 8)])
    P = power_spectrum(_gpu(a), 2, dt, _gpu(w), 1e5).cpu().numpy()
    print("harmonic intensities P(k omega), k = 1..7:", " ".join(f"{x:.2e}" for x in P))
    assert np.all(np.isfinite(P)) and P[0] > 0.0
