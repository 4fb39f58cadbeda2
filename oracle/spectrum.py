"""Absorption spectrum from dipole traces (oracle; test infrastructure only).

Sec. 3.2: the dynamic polarizability is the Fourier transform of the dipole
response divided by that of the applied field, the trace is damped by an
exponential window g(t) = exp(-t / tau) to broaden the peaks, and the
absorption spectrum is proportional to omega Tr Im alpha(omega).

Readings (the printed formula divides by the field transform twice):
* F[f](omega) = int_0^T f(t) exp(i omega t) dt, by the trapezoid rule on the
  samples t_n = n dt, n = 0..N, with t = 0 the start of the run;
* alpha_dd(omega) = F[g (mu_d - mu_d(0))](omega) / F[E_d](omega) for the run
  perturbed along d (mu_d its d component);
* S(omega) = (2 omega / (3 pi)) sum_d Im alpha_dd(omega), normalised so that the
  Thomas-Reiche-Kuhn sum rule reads int_0^inf S d omega = N_e for an isotropic
  response (the paper's prefactor 4 omega / (3 pi) belongs to another Fourier
  convention; this normalisation is fixed by the sum rule);
* pulses: a delta kick of strength kappa at t = 0 (F[E] = kappa), or the
  Gaussian kappa exp(-(t - t0)^2 / (2 s^2)) of Sec. 3.1-3.2, whose transform is
  kappa s sqrt(2 pi) exp(-omega^2 s^2 / 2) exp(i omega t0).
"""
from __future__ import annotations

import math

import numpy as np


def pulse_transform(omega, kind, kappa, t0=0.0, s=1.0):
    """F[E](omega) of a delta kick ("kick") or a Gaussian pulse ("gauss"); omega may be complex."""
    omega = np.asarray(omega)
    if kind == "kick":
        return np.full(omega.shape, complex(kappa))
    if kind == "gauss":
        return kappa * s * math.sqrt(2.0 * math.pi) * np.exp(-0.5 * (omega * s) ** 2) * np.exp(1j * omega * t0)
    raise ValueError(f"unknown pulse {kind!r}")


def windowed_transform(f, dt, omega, tau):
    """int_0^T g(t) f(t) exp(i omega t) dt (trapezoid rule), f sampled at n dt."""
    f = np.asarray(f, dtype=np.float64)
    t = dt * np.arange(len(f))
    w = np.full(len(f), dt)
    w[0] = w[-1] = 0.5 * dt
    gf = w * np.exp(-t / tau) * f
    return np.exp(1j * np.outer(np.asarray(omega, dtype=np.float64), t)) @ gf


def polarizability(mu, direction, dt, omega, tau, pulse):
    """alpha_dd(omega) from the trace mu[n][3] of the run perturbed along direction d."""
    mu = np.asarray(mu, dtype=np.float64)
    dmu = mu[:, direction] - mu[0, direction]
    return windowed_transform(dmu, dt, omega, tau) / pulse_transform(omega, **pulse)


def absorption_spectrum(traces, directions, dt, omega, tau, pulse):
    """S(omega) = (2 omega / 3 pi) sum_d Im alpha_dd(omega) over the given runs."""
    omega = np.asarray(omega, dtype=np.float64)
    acc = np.zeros(len(omega))
    for mu, d in zip(traces, directions):
        acc += np.imag(polarizability(mu, d, dt, omega, tau, pulse))
    return 2.0 * omega / (3.0 * math.pi) * acc
