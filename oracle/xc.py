"""Adiabatic LDA exchange-correlation potential (oracle).

Sec. 2.1: the paper uses the adiabatic LDA in the Ceperley-Alder form.  Here the
exchange part is Slater's, and correlation (optional) is the Perdew-Wang 1992
parametrisation of the same Ceperley-Alder data, spin-unpolarised.  Densities
below 1e-30 give a zero potential.
"""
from __future__ import annotations

import numpy as np

RHO_FLOOR = 1e-30

# Perdew & Wang, PRB 45, 13244 (1992), unpolarised correlation, with p = 1
PW_A = 0.031091
PW_ALPHA1 = 0.21370
PW_BETA = (7.5957, 3.5876, 1.6382, 0.49294)


def slater_energy_density(rho):
    """Exchange energy per electron, eps_x = -(3/4)(3 rho / pi)^(1/3)."""
    rho = np.asarray(rho, dtype=np.float64)
    return np.where(rho > RHO_FLOOR, -0.75 * np.cbrt(3.0 * np.clip(rho, 0, None) / np.pi), 0.0)


def slater_potential(rho):
    """v_x = d(rho eps_x)/d rho = -(3 rho / pi)^(1/3)."""
    rho = np.asarray(rho, dtype=np.float64)
    return np.where(rho > RHO_FLOOR, -np.cbrt(3.0 * np.clip(rho, 0, None) / np.pi), 0.0)


def pw92_eps_c(rs):
    """Correlation energy per electron as a function of the Wigner-Seitz radius."""
    rs = np.asarray(rs, dtype=np.float64)
    b1, b2, b3, b4 = PW_BETA
    q0 = -2.0 * PW_A * (1.0 + PW_ALPHA1 * rs)
    q1 = 2.0 * PW_A * (b1 * np.sqrt(rs) + b2 * rs + b3 * rs ** 1.5 + b4 * rs * rs)
    return q0 * np.log1p(1.0 / q1)


def pw92_deps_drs(rs):
    """Analytic d eps_c / d rs."""
    rs = np.asarray(rs, dtype=np.float64)
    b1, b2, b3, b4 = PW_BETA
    q0 = -2.0 * PW_A * (1.0 + PW_ALPHA1 * rs)
    dq0 = -2.0 * PW_A * PW_ALPHA1
    q1 = 2.0 * PW_A * (b1 * np.sqrt(rs) + b2 * rs + b3 * rs ** 1.5 + b4 * rs * rs)
    dq1 = PW_A * (b1 / np.sqrt(rs) + 2.0 * b2 + 3.0 * b3 * np.sqrt(rs) + 4.0 * b4 * rs)
    return dq0 * np.log1p(1.0 / q1) - q0 * dq1 / (q1 * q1 + q1)


def pw92_potential(rho):
    """v_c = eps_c - (rs/3) d eps_c/d rs, rs = (3 / (4 pi rho))^(1/3)."""
    rho = np.asarray(rho, dtype=np.float64)
    ok = rho > RHO_FLOOR
    rs = np.cbrt(3.0 / (4.0 * np.pi * np.where(ok, rho, 1.0)))
    v = pw92_eps_c(rs) - rs / 3.0 * pw92_deps_drs(rs)
    return np.where(ok, v, 0.0)


def pw92_energy_density(rho):
    rho = np.asarray(rho, dtype=np.float64)
    ok = rho > RHO_FLOOR
    rs = np.cbrt(3.0 / (4.0 * np.pi * np.where(ok, rho, 1.0)))
    return np.where(ok, pw92_eps_c(rs), 0.0)


def vxc(rho, kind):
    if kind == "none":
        return np.zeros_like(np.asarray(rho, dtype=np.float64))
    if kind == "slater":
        return slater_potential(rho)
    if kind == "slater_pw92":
        return slater_potential(rho) + pw92_potential(rho)
    raise ValueError(kind)
