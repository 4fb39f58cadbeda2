"""Atomic part of the enrichment functions (oracle).

Sec. 2.2, eq. (EFEAtomic): an enrichment function's atomic part is an atomic
orbital times a smooth cutoff u(r).  The atomic orbitals themselves are not
available, so Slater-type stand-ins are used,

    N^A_nu(x) = r^l exp(-zeta r) Y_lm(r_hat) u(r),  r = |x - R_I|,
    u(r) = (1 - (r/r_c)^2)^3 for r < r_c, else 0,

with real spherical harmonics Y_00 = 1/sqrt(4 pi) and
r Y_1m = sqrt(3/(4 pi)) * (y, z, x) for m = (-1, 0, +1).  Normalisation to unit
norm happens in the model, under the enrichment quadrature.
"""
from __future__ import annotations

import numpy as np

_Y00 = 1.0 / np.sqrt(4.0 * np.pi)
_Y1 = np.sqrt(3.0 / (4.0 * np.pi))
_COMP = {-1: 1, 0: 2, 1: 0}   # m -> Cartesian component (y, z, x)


def cutoff(r, rc):
    s = np.clip(1.0 - (r / rc) ** 2, 0.0, None)
    u = s ** 3
    du = np.where(r < rc, -6.0 * r / (rc * rc) * s * s, 0.0)
    return u, du


def atomic_function(pts, R, l, m, zeta, rc, grad=False):
    """Values (nq,) and optionally gradients (nq, 3) of one unnormalised N^A."""
    d = pts - R[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    u, du = cutoff(r, rc)
    e = np.exp(-zeta * r)
    g = e * u                      # radial factor
    dg = e * (du - zeta * u)       # its r-derivative
    with np.errstate(invalid="ignore", divide="ignore"):
        rhat = np.where(r[:, None] > 0, d / np.where(r > 0, r, 1.0)[:, None], 0.0)
    if l == 0:
        val = _Y00 * g
        gr = (_Y00 * dg)[:, None] * rhat if grad else None
    elif l == 1:
        k = _COMP[int(m)]
        val = _Y1 * d[:, k] * g
        if grad:
            gr = (_Y1 * d[:, k] * dg)[:, None] * rhat
            gr[:, k] += _Y1 * g
        else:
            gr = None
    else:
        raise ValueError("only l = 0, 1 enrichment functions are supported")
    return (val, gr) if grad else val
