"""Field-parameter gradients of a dipole-tracking loss (oracle; test infrastructure only).

The propagation is the Magnus-2 predictor-corrector of ``oracle.propagate``
(Sec. 2.5-2.6) driven by the external field of eq. (VField),
E(t) z_hat with E(t) = sum_k A_k sin(w_k t + phi_k) exp(-(t - t0)^2 / s^2)
(no kick).  The loss compares the z dipole with a target trace:

    L(theta) = sum_{n=1}^{N} (mu_z(t_n) - mu*_n)^2,   theta = (A_1..A_m, w_1..w_m, phi_1..phi_m).

The oracle's gradient is the plain definition of the derivative of this
discrete forward map, taken by central differences with the Krylov dimension
of every column frozen to the base run (k replay), so that L(theta +- h) are
smooth functions of theta.  Truncation error O(h^2).
"""
from __future__ import annotations

import numpy as np

from .model import Field
from .propagate import Propagator


def field_from_params(theta, t0, s, direction=2):
    """Field with theta = concatenation of (A, w, phi), m components each."""
    theta = np.asarray(theta, dtype=np.float64)
    m = len(theta) // 3
    return Field(direction=direction, A=theta[:m].copy(), w=theta[m:2 * m].copy(), phi=theta[2 * m:].copy(),
                 t0=float(t0), s=float(s))


def run_dipole(model, X0, field, dt, nsteps, k_force=None):
    """mu(t_1..t_N) of the field-driven propagation from X0 at t = 0, and the k per step."""
    P = Propagator(model, X0, t=0.0, field=field)
    return P.run(dt, nsteps, k_force)


def loss(model, X0, theta, t0, s, dt, nsteps, mu_target, k_force=None):
    mus, ks = run_dipole(model, X0, field_from_params(theta, t0, s), dt, nsteps, k_force)
    return float(np.sum((mus[:, 2] - mu_target) ** 2)), mus, ks


def fd_gradient(model, X0, theta, t0, s, dt, nsteps, mu_target, h=1e-6, params=None):
    """Central-difference gradient of `loss` with the base run's k replayed
    (components `params`, default all; the others are left at zero).

    Returns (g, L, mus, ks)."""
    theta = np.asarray(theta, dtype=np.float64)
    L0, mus, ks = loss(model, X0, theta, t0, s, dt, nsteps, mu_target)
    g = np.zeros_like(theta)
    for p in (range(len(theta)) if params is None else params):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        Lp = loss(model, X0, tp, t0, s, dt, nsteps, mu_target, ks)[0]
        Lm = loss(model, X0, tm, t0, s, dt, nsteps, mu_target, ks)[0]
        g[p] = (Lp - Lm) / (2.0 * h)
    return g, L0, mus, ks


def field_derivatives(theta, t0, s, t):
    """dE(t)/dtheta for theta = (A, w, phi)."""
    theta = np.asarray(theta, dtype=np.float64)
    m = len(theta) // 3
    A, w, ph = theta[:m], theta[m:2 * m], theta[2 * m:]
    env = np.exp(-((t - t0) / s) ** 2)
    arg = w * t + ph
    return np.concatenate([np.sin(arg) * env, A * t * np.cos(arg) * env, A * np.cos(arg) * env])
