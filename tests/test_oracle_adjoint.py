"""Pins of the oracle's field-parameter gradient (central differences with k replay).

Harmonic-potential (Kohn) theorem: in a harmonic trap the dipole of any
electron system obeys the driven classical oscillator
    mu_z'' = -w0^2 mu_z + N E(t),  so from rest  mu_z(t) = (N/w0) int_0^t sin(w0 (t - t')) E(t') dt'.
With the target mu* = 0 the loss is L = sum_n mu_z(t_n)^2, linear-response in the
amplitudes A_k, and its exact gradient is dL/dA_k = sum_n 2 mu_n G_nk with
G_nk = (N/w0) int_0^{t_n} sin(w0 (t_n - t')) sin(w_k t' + phi_k) env(t') dt'.
The FE trap reproduces the theorem to a few per cent (h = 3, p = 4), which
bounds the comparison; a sign error in the field coupling or the loss flips
the gradient.
"""
import numpy as np
import pytest

from oracle.adjoint import fd_gradient, field_derivatives, field_from_params, loss
from oracle.model import EFEModel
from workloads import trap

TRAP_ARGS = dict(omega=1.0, ncell=4, half=6.0, degree=4)


@pytest.fixture(scope="module")
def trap_model(golden_dir):
    import os
    m = EFEModel(trap(**TRAP_ARGS))
    X0 = np.load(os.path.join(golden_dir, "trap_ground_state.npz"))["X"]
    return m, X0


def _kohn_G(theta, t0, s, ts, w0=1.0, N=2.0, nq=4001):
    m = len(theta) // 3
    A, w, ph = theta[:m], theta[m:2 * m], theta[2 * m:]
    G = np.zeros((len(ts), m))
    for n, tn in enumerate(ts):
        tp = np.linspace(0.0, tn, nq)
        env = np.exp(-((tp - t0) / s) ** 2)
        for k in range(m):
            f = np.sin(w0 * (tn - tp)) * np.sin(w[k] * tp + ph[k]) * env
            G[n, k] = (N / w0) * np.trapezoid(f, tp)
    return G


def test_field_derivatives_match_differences():
    theta = np.array([3e-3, 5e-3, 1.3, 2.1, 0.4, 1.9])
    t0, s, t = 0.4, 0.3, 0.37
    d = field_derivatives(theta, t0, s, t)
    h = 1e-6
    for p in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (field_from_params(tp, t0, s).E(t) - field_from_params(tm, t0, s).E(t)) / (2 * h)
        assert abs(fd - d[p]) <= 1e-8 * max(1e-3, abs(d[p]))


def test_gradient_kohn_theorem(trap_model):
    m, X0 = trap_model
    dt, nsteps, t0, s = 0.05, 10, 0.3, 0.2
    theta = np.array([4e-3, 6e-3, 3.0, 5.0, 0.3, 1.1])
    mu_target = np.zeros(nsteps)
    g, L, mus, ks = fd_gradient(m, X0, theta, t0, s, dt, nsteps, mu_target, params=[0, 1])
    ts = dt * np.arange(1, nsteps + 1)
    G = _kohn_G(theta, t0, s, ts)
    mu_k = G @ theta[:2]
    assert np.abs(mus[:, 2] - mu_k).max() < 0.05 * np.abs(mu_k).max()
    g_k = 2.0 * G.T @ mu_k
    err = np.abs(g[:2] - g_k).max() / np.abs(g_k).max()
    print("Kohn gradient (A):", g[:2], g_k, err)
    assert err < 0.1
    # loss is quadratic in A at linear response: L(2A) = 4 L(A) to the same accuracy
    L2 = loss(m, X0, np.concatenate([2 * theta[:2], theta[2:]]), t0, s, dt, nsteps, mu_target)[0]
    assert abs(L2 / L - 4.0) < 0.01
