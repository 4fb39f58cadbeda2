"""Pins of the oracle's adiabatic LDA (Sec. 2.1: the exchange-correlation potential in
the adiabatic local density approximation, Ceperley-Alder correlation).

Nothing here re-types the oracle's formulas.  Each part is held against something
fixed outside it:

* Slater exchange: the textbook Dirac exchange energy per electron of the uniform
  gas, eps_x = -(3 / 4 pi) k_F with k_F = (3 pi^2 rho)^(1/3), and the potential as
  the derivative d(rho eps_x)/d rho by central differences; the closed value
  v_x(pi / 3) = -1.
* PW92 correlation (Perdew-Wang 1992, spin-unpolarised):
  - the exact high-density limit of the electron gas (Gell-Mann-Brueckner):
    d eps_c / d ln r_s -> (1 - ln 2) / pi^2 and eps_c - c0 ln r_s -> -c1 with the
    published c1 = 0.046644;
  - the low-density expansion eps_c = -d0 / r_s + d1 / r_s^(3/2) + ... with the
    published d0 = 0.4335 and d1 = 1.4408;
  - an independent parametrisation of the same Ceperley-Alder data (Perdew-Zunger
    1981, r_s >= 1 branch): agreement within 1% for r_s in [1, 10];
  - the potential v_c = d(rho eps_c)/d rho and the analytic d eps_c / d r_s against
    central differences.
* The density floor: no potential at or below 1e-30.

The last tests plant the mistakes these pins exist for (the 3/4 energy-density
factor in the Slater potential, a sign flip in d eps_c / d r_s, a wrong PW92
constant) into a private copy of the oracle module and check that a pin fails.
"""
from __future__ import annotations

import importlib.util
import math
import os

import numpy as np
import pytest

from oracle import xc

ORACLE_XC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "xc.py")

RHOS = np.logspace(-8, 3, 45)


def dirac_eps_x(rho):
    """Textbook exchange energy per electron of the uniform electron gas."""
    kf = np.cbrt(3.0 * math.pi ** 2 * rho)
    return -3.0 / (4.0 * math.pi) * kf


def central_diff_rho(f, rho, rel=1e-4):
    """d f / d rho by a fourth-order central difference with relative step rel."""
    h = rel * rho
    return (-f(rho + 2 * h) + 8 * f(rho + h) - 8 * f(rho - h) + f(rho - 2 * h)) / (12 * h)


def pz81_eps_c(rs):
    """Perdew-Zunger 1981 unpolarised correlation, r_s >= 1 branch (its own constants)."""
    return -0.1423 / (1.0 + 1.0529 * np.sqrt(rs) + 0.3334 * rs)


# ---------------------------------------------------------------- pin checks (module in)
def check_slater(m):
    rho = RHOS
    np.testing.assert_allclose(m.slater_energy_density(rho), dirac_eps_x(rho), rtol=1e-13)
    v_fd = central_diff_rho(lambda r: r * dirac_eps_x(r), rho)
    np.testing.assert_allclose(m.slater_potential(rho), v_fd, rtol=1e-9)
    assert abs(float(m.slater_potential(math.pi / 3.0)) + 1.0) < 1e-14


def check_pw92_high_density(m):
    c0 = (1.0 - math.log(2.0)) / math.pi ** 2
    for rs in (1e-8, 1e-10):
        h = 1e-3
        slope = (float(m.pw92_eps_c(rs * math.exp(h))) - float(m.pw92_eps_c(rs * math.exp(-h)))) / (2 * h)
        assert abs(slope - c0) < 1e-4 * c0, (rs, slope, c0)
        c1 = -(float(m.pw92_eps_c(rs)) - c0 * math.log(rs))
        assert abs(c1 - 0.046644) < 2e-5, (rs, c1)


def check_pw92_low_density(m):
    d0, d1 = 0.4335, 1.4408

    def f(rs):                      # -r_s eps_c = d0 - d1 r_s^(-1/2) + O(1/r_s)
        return -float(m.pw92_eps_c(rs)) * rs

    for rs in (1e8, 1e10):
        assert abs(f(rs) + d1 / math.sqrt(rs) - d0) < 1e-4, (rs, f(rs))
    r1, r2 = 1e8, 1e10
    d1_est = (f(r2) - f(r1)) / (r1 ** -0.5 - r2 ** -0.5)
    assert abs(d1_est - d1) < 1e-3, d1_est


def check_pw92_vs_pz81(m):
    rs = np.linspace(1.0, 10.0, 37)
    np.testing.assert_allclose(m.pw92_eps_c(rs), pz81_eps_c(rs), rtol=1e-2)


def check_pw92_potential(m):
    rs = np.logspace(-3, 2, 41)
    h = 1e-5 * rs
    d_fd = (-m.pw92_eps_c(rs + 2 * h) + 8 * m.pw92_eps_c(rs + h) - 8 * m.pw92_eps_c(rs - h)
            + m.pw92_eps_c(rs - 2 * h)) / (12 * h)
    np.testing.assert_allclose(m.pw92_deps_drs(rs), d_fd, rtol=1e-8)
    rho = RHOS

    def e_c(r):
        return m.pw92_eps_c(np.cbrt(3.0 / (4.0 * math.pi * r)))

    v_fd = central_diff_rho(lambda r: r * e_c(r), rho)
    np.testing.assert_allclose(m.pw92_potential(rho), v_fd, rtol=1e-8)
    np.testing.assert_allclose(m.pw92_energy_density(rho), e_c(rho), rtol=1e-14)


PINS = [check_slater, check_pw92_high_density, check_pw92_low_density, check_pw92_vs_pz81, check_pw92_potential]


# ---------------------------------------------------------------------------- tests
@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_oracle_xc_pin(pin):
    pin(xc)


def test_sum_and_floor():
    rho = np.array([0.0, 1e-31, 1e-30, 2e-30, 1e-3, 1.0])
    np.testing.assert_array_equal(xc.vxc(rho, "none"), 0.0)
    np.testing.assert_array_equal(xc.vxc(rho, "slater"), xc.slater_potential(rho))
    np.testing.assert_allclose(xc.vxc(rho, "slater_pw92"), xc.slater_potential(rho) + xc.pw92_potential(rho),
                               rtol=0, atol=0)
    for kind in ("slater", "slater_pw92"):
        v = xc.vxc(rho, kind)
        assert v[0] == 0.0 and v[1] == 0.0 and v[2] == 0.0     # at or below the floor
        assert v[3] < 0.0 and np.all(v[3:] < 0.0)
    with pytest.raises(ValueError):
        xc.vxc(rho, "pbe")


def test_exchange_dominates_correlation():
    """v_c is a small negative correction to v_x at the densities of the workloads."""
    rho = np.logspace(-4, 2, 13)
    vx, vc = xc.slater_potential(rho), xc.pw92_potential(rho)
    assert np.all(vc < 0.0) and np.all(np.abs(vc) < np.abs(vx))


# --------------------------------------------------------------- planted mistakes
def _copy_of_oracle_xc():
    spec = importlib.util.spec_from_file_location("oracle_xc_copy", ORACLE_XC)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _fails(m):
    failed = []
    for pin in PINS:
        try:
            pin(m)
        except AssertionError:
            failed.append(pin.__name__)
    return failed


def test_pins_pass_on_an_unmodified_copy():
    assert _fails(_copy_of_oracle_xc()) == []


def test_pins_catch_energy_density_factor_in_slater_potential():
    m = _copy_of_oracle_xc()
    good = m.slater_potential
    m.slater_potential = lambda rho: 0.75 * good(rho)
    assert "check_slater" in _fails(m)


def test_pins_catch_sign_flip_in_correlation_derivative():
    m = _copy_of_oracle_xc()
    good = m.pw92_deps_drs
    m.pw92_deps_drs = lambda rs: -good(rs)
    assert "check_pw92_potential" in _fails(m)


@pytest.mark.parametrize("which,value", [("A", 0.0311), ("alpha1", 0.2137 * 1.1), ("beta", 0), ("beta", 1),
                                         ("beta", 2), ("beta", 3)])
def test_pins_catch_a_wrong_pw92_constant(which, value):
    m = _copy_of_oracle_xc()
    if which == "A":
        m.PW_A = value
    elif which == "alpha1":
        m.PW_ALPHA1 = value
    else:
        b = list(m.PW_BETA)
        b[value] *= 1.02
        m.PW_BETA = tuple(b)
    assert _fails(m), f"a wrong {which} passed every pin"
