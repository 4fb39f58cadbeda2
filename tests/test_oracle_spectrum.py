"""Pins for the oracle's absorption spectrum (Sec. 3.2).

* closed form: the windowed transform of a kicked harmonic response
  N kappa sin(w0 t)/w0 is N / (w0^2 + (1/tau - i w)^2) (trapezoid error O(dt^2));
* Thomas-Reiche-Kuhn: int_0^inf (2 w / pi) Im alpha dw = N for that response
  (the normalisation of S), with the analytic 4 N / (pi tau W) tail beyond W;
* Gaussian pulse: for the linear oscillator driven by kappa exp(-(t-t0)^2/2s^2)
  the window factors through the convolution, alpha = alpha_kick F[gE]/F[E]
  with F[gE](w) = F[E](w + i/tau) (pins the phase exp(+i w t0) of F[E]);
* physics: the kicked two-electron harmonic trap (Kohn mode) propagated by the
  oracle's Magnus step gives the spectrum of N kappa sin(w0 t)/w0 (one peak,
  carrying N = 2 with the analytic tail beyond the grid) to 5%, the
  discretisation limit of the trap mesh.
"""
import math
import os

import numpy as np
from scipy.signal import fftconvolve
import pytest

from oracle.spectrum import absorption_spectrum, polarizability, pulse_transform, windowed_transform


def _oscillator_alpha(w, w0, N, tau):
    a = 1.0 / tau - 1j * np.asarray(w)
    return N / (w0 ** 2 + a * a)


def test_windowed_transform_closed_form():
    w0, N, kappa, tau, dt = 1.3, 3.0, 1e-3, 4.0, 0.005
    t = np.arange(0.0, 30 * tau, dt)
    mu = np.zeros((len(t), 3))
    mu[:, 1] = 0.2 + N * kappa * np.sin(w0 * t) / w0      # offset: the ground-state dipole is subtracted
    w = np.linspace(0.05, 3.0, 60)
    alpha = polarizability(mu, 1, dt, w, tau, dict(kind="kick", kappa=kappa))
    ref = _oscillator_alpha(w, w0, N, tau)
    assert np.max(np.abs(alpha - ref)) / np.max(np.abs(ref)) < 1e-4
    # three isotropic runs: S = (2 w / pi) Im alpha
    traces = []
    for d in range(3):
        m = np.zeros_like(mu)
        m[:, d] = mu[:, 1]
        traces.append(m)
    S = absorption_spectrum(traces, [0, 1, 2], dt, w, tau, dict(kind="kick", kappa=kappa))
    np.testing.assert_allclose(S, 2 * w / math.pi * np.imag(ref), rtol=2e-4, atol=1e-6 * np.max(np.abs(S)))
    # second order in dt
    e = []
    for h in (0.02, 0.01):
        tt = np.arange(0.0, 30 * tau, h)
        f = N * kappa * np.sin(w0 * tt) / w0
        e.append(np.max(np.abs(windowed_transform(f, h, w, tau) / kappa - ref)))
    assert 3.6 < e[0] / e[1] < 4.4


def test_trk_sum_rule_normalisation():
    w0, N, tau, W = 1.7, 2.0, 10.0, 400.0
    w = np.linspace(0.0, W, 400001)
    f = 2 * w / math.pi * np.imag(_oscillator_alpha(w, w0, N, tau))
    integral = float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(w)))
    tail = 4 * N / (math.pi * tau * W)
    assert abs(integral + tail - N) < 1e-4 * N


def test_gaussian_pulse_convention():
    w0, N, kappa, tau, t0, s, dt = 0.9, 2.0, 2e-5, 40.0, 3.0, 0.2, 0.002
    t = np.arange(0.0, 12 * tau, dt)
    E = kappa * np.exp(-((t - t0) ** 2) / (2 * s * s))
    G = N * np.sin(w0 * t) / w0
    resp = fftconvolve(G, E)[: len(t)] * dt             # mu(t) = int_0^t G(t - t') E(t') dt'
    mu = np.zeros((len(t), 3))
    mu[:, 0] = resp
    w = np.linspace(0.1, 2.5, 40)
    pulse = dict(kind="gauss", kappa=kappa, t0=t0, s=s)
    alpha = polarizability(mu, 0, dt, w, tau, pulse)
    ref = _oscillator_alpha(w, w0, N, tau) * pulse_transform(w + 1j / tau, **pulse) / pulse_transform(w, **pulse)
    assert np.max(np.abs(alpha - ref)) / np.max(np.abs(ref)) < 2e-3


def test_kohn_mode_spectrum_in_trap(golden_dir):
    from oracle.model import EFEModel
    from oracle.propagate import Propagator
    from workloads import trap
    m = EFEModel(trap(omega=1.0, ncell=4, half=6.0, degree=4))
    X0 = np.load(os.path.join(golden_dir, "trap_ground_state.npz"))["X"]
    kappa, dt, nsteps, tau = 1e-3, 0.1, 120, 2.5
    P = Propagator(m, X0, tol=1e-12)
    mu = [m.dipole(P.rho)]
    P.kick(kappa, 2)
    for _ in range(nsteps):
        mu.append(P.step(dt)[0])
    mu = np.array(mu)
    w = np.linspace(0.01, 6.0, 600)
    # the trap response is isotropic: use the z run for all three directions
    S = absorption_spectrum([mu[:, [2, 2, 2]]] * 3, [0, 1, 2], dt, w, tau, dict(kind="kick", kappa=kappa))
    # the ideal response N kappa sin(t) windowed: the peak sits at sqrt(1 + 1/tau^2), not at 1
    ideal = 2 * w / math.pi * np.imag(_oscillator_alpha(w, 1.0, 2.0, tau))
    err = np.max(np.abs(S - ideal)) / np.max(ideal)
    total = float(np.sum(0.5 * (S[1:] + S[:-1]) * np.diff(w))) + 4 * 2.0 / (math.pi * tau * w[-1])
    print("trap spectrum: peak", w[np.argmax(S)], "max deviation from the ideal", err, "sum rule", total)
    assert err < 0.05
    assert abs(total - 2.0) < 0.1


# ---------------------------------------------------------------- power spectrum (Sec. 3.5)

def _windowed_exact(f, t_a, t_b, omega, tau):
    """|int_{t_a}^{t_b} exp(-i w t) exp(-t^2/tau) f(t) dt|^2 by adaptive quadrature."""
    from scipy.integrate import quad
    out = []
    g = lambda t: math.exp(-t * t / tau) * f(t)
    for w in omega:
        if w == 0.0:
            re, im = quad(g, t_a, t_b, limit=400, epsabs=0, epsrel=1e-12)[0], 0.0
        else:      # QAWO: the oscillatory factor is integrated exactly against the polynomial fits
            re = quad(g, t_a, t_b, weight="cos", wvar=w, limit=800, epsabs=0, epsrel=1e-12)[0]
            im = -quad(g, t_a, t_b, weight="sin", wvar=w, limit=800, epsabs=0, epsrel=1e-12)[0]
        out.append(re * re + im * im)
    return np.array(out)


def test_power_spectrum_of_a_cubic_dipole():
    """mu = 2 + t/2 - 0.3 t^2 + 0.07 t^3: the second difference is exact (mu'' = -0.6 + 0.42 t),
    so P equals the windowed integral of mu'' over [t_1, t_{N-1}] to the trapezoid error."""
    from oracle.spectrum import power_spectrum, dipole_acceleration
    dt, N, tau = 0.005, 4000, 50.0
    t = dt * np.arange(N + 1)
    mu = np.zeros((N + 1, 3))
    mu[:, 1] = 2.0 + 0.5 * t - 0.3 * t ** 2 + 0.07 * t ** 3
    np.testing.assert_allclose(dipole_acceleration(mu[:, 1], dt), -0.6 + 0.42 * t[1:-1], rtol=0, atol=2e-7)
    omega = np.array([0.0, 0.4, 1.3, 2.9])
    P = power_spectrum(mu, 1, dt, omega, tau)
    ref = _windowed_exact(lambda x: -0.6 + 0.42 * x, t[1], t[-2], omega, tau)
    np.testing.assert_allclose(P, ref, rtol=1e-4)
    # the window is exp(-t^2/tau): with exp(-t/tau) the value differs by orders
    alt = _windowed_exact(lambda x: (-0.6 + 0.42 * x) * math.exp(x * x / tau - x / tau), t[1], t[-2], omega[:1], tau)
    assert abs(alt[0] - P[0]) > 0.5 * P[0]


def test_power_spectrum_of_linear_dipole_vanishes():
    from oracle.spectrum import power_spectrum
    dt = 0.05
    t = dt * np.arange(2001)
    mu = np.stack([3.0 - 0.2 * t, 0.1 * t, np.full_like(t, 7.0)], axis=1)
    P = power_spectrum(mu, 0, dt, np.linspace(0.0, 3.0, 7), 1e5)
    assert np.max(P) < 1e-16


def test_power_spectrum_peaks_at_the_oscillation():
    """mu = sin(w0 t): |F[mu'']|^2 peaks at w0 (not at w0/2 or 2 w0) and equals
    w0^4 |F[sin]|^2 there up to the O((w0 dt)^2) error of the difference."""
    from oracle.spectrum import power_spectrum
    w0, dt, N, tau = 0.7, 0.02, 20000, 1e5
    t = dt * np.arange(N + 1)
    mu = np.zeros((N + 1, 3))
    mu[:, 2] = np.sin(w0 * t)
    omega = np.linspace(0.05, 2.0, 391)
    P = power_spectrum(mu, 2, dt, omega, tau)
    assert abs(omega[np.argmax(P)] - w0) <= 0.005 + 1e-12
    # at omega = w0: sin(w0 t) exp(-i w0 t) = sin(2 w0 t)/2 - i (1 - cos(2 w0 t))/2
    from scipy.integrate import quad
    g0 = lambda x: -w0 * w0 * math.exp(-x * x / tau)
    a, b = t[1], t[-2]
    re = 0.5 * quad(g0, a, b, weight="sin", wvar=2 * w0, limit=800)[0]
    im = -0.5 * quad(g0, a, b, limit=400)[0] + 0.5 * quad(g0, a, b, weight="cos", wvar=2 * w0, limit=800)[0]
    np.testing.assert_allclose(P[np.argmin(np.abs(omega - w0))], re * re + im * im, rtol=1e-3)


def test_hhg_field_is_the_sinusoidal_pulse():
    """The sum-of-sines parameters reproduce kappa sin(pi t/T) sin(omega t) on [0, T]."""
    from oracle.model import Field
    from workloads import hhg_field
    p = hhg_field(kappa=0.01, omega=0.03, ncycles=5)
    f = Field(direction=p["direction"], A=p["A"], w=p["w"], phi=p["phi"], t0=p["t0"], s=p["s"])
    T = p["T"]
    assert abs(T - 5 * 2 * math.pi / 0.03) < 1e-9
    for t in np.linspace(0.0, T, 97):
        assert abs(f.E(t) - 0.01 * math.sin(math.pi * t / T) * math.sin(0.03 * t)) < 1e-15
