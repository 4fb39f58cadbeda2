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

Sec. 3.5 (high-harmonic generation): the dipole power spectrum is the squared
modulus of the windowed Fourier transform of the dipole acceleration.  Readings
(the printed derivative reads d/dt^2): P(omega) = |int_0^T exp(-i omega t)
exp(-t^2/tau) mu_d''(t) dt|^2 with the Gaussian window as printed, mu_d'' by the
second central difference at the interior samples t_1 .. t_{N-1}, and the
trapezoid rule over those samples.  The sinusoidal pulse of that section is
kappa sin(pi t/T) sin(omega t) on [0, T].
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


def dipole_acceleration(mu_d, dt):
    """mu''(t_n), n = 1 .. N-1, by the second central difference of the samples mu_d[0..N]."""
    mu_d = np.asarray(mu_d, dtype=np.float64)
    return (mu_d[2:] - 2.0 * mu_d[1:-1] + mu_d[:-2]) / (dt * dt)


def power_spectrum(mu, direction, dt, omega, tau):
    """P(omega) = |int exp(-i omega t) exp(-t^2 / tau) mu_d''(t) dt|^2 over t_1 .. t_{N-1}
    (trapezoid rule), mu[n][3] sampled at t_n = n dt."""
    mu = np.asarray(mu, dtype=np.float64)
    acc = dipole_acceleration(mu[:, direction], dt)
    t = dt * np.arange(1, len(mu) - 1)
    w = np.full(len(t), dt)
    w[0] = w[-1] = 0.5 * dt
    f = w * np.exp(-t * t / tau) * acc
    F = np.exp(-1j * np.outer(np.asarray(omega, dtype=np.float64), t)) @ f
    return np.abs(F) ** 2
