"""Maxwell equal-area construction (test infrastructure).

The paper quotes coexistence densities from the Maxwell equal-area law for
both pseudopotential forms (Sec. IV.A for the exponential form with
G = -10/3; Sec. IV.D for the Carnahan-Starling EOS of Eq. (58)).  With the
pseudopotential the bulk pressure is p = rho c_s^2 + G c^2 psi^2 / 2, which
for the square-root form is p_EOS itself.

``maxwell`` takes any pressure function p(rho) (normally the C oracle's psi,
see ``oracle.ref.pressure_fn``), so the printed coexistence values pin the
oracle's EOS and psi code directly.

Method: locate the two spinodals (dp/drho = 0), then solve for the
coexistence pressure p* at which the equal-area condition in specific volume
v = 1/rho holds,  integral_{rho_V}^{rho_L} (p(rho) - p*) / rho^2 drho = 0,
with rho_V < rho_L the outer roots of p(rho) = p*.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq


def _spinodals(p, lo, hi, n=20001):
    r = np.linspace(lo, hi, n)
    pv = np.array([p(x) for x in r])
    d = np.diff(pv)
    sign = np.sign(d)
    idx = np.nonzero(sign[:-1] != sign[1:])[0]
    if len(idx) < 2:
        raise ValueError("pressure curve has no van der Waals loop in range")
    h = 1e-7

    def dp(x):
        return (p(x + h * x) - p(x - h * x)) / (2 * h * x)

    ext = []
    for i in idx[:2]:
        ext.append(brentq(dp, r[i], r[i + 2], xtol=1e-15, rtol=1e-14))
    return ext[0], ext[1]  # local max (vapour side), local min (liquid side)


def _finite_upper(p, lo, hi, n=4001):
    """Largest grid point below the first density where p is not finite (the
    square-root pseudopotential is real only while its radicand is >= 0)."""
    r = np.linspace(lo, hi, n)
    ok = np.array([np.isfinite(p(x)) for x in r])
    if ok.all():
        return hi
    first_bad = int(np.argmin(ok))
    return r[max(first_bad - 1, 1)]


def maxwell(p, lo, hi):
    """Coexistence (rho_L, rho_V) for pressure function p on (lo, hi)."""
    hi = _finite_upper(p, lo, hi)
    r_max, r_min = _spinodals(p, lo, hi)
    p_hi = p(r_max)
    p_lo = max(p(r_min), p(lo))

    def roots(ps):
        rv = brentq(lambda x: p(x) - ps, lo, r_max, xtol=1e-16, rtol=1e-15)
        rl = brentq(lambda x: p(x) - ps, r_min, hi, xtol=1e-16, rtol=1e-15)
        return rv, rl

    def area(ps):
        rv, rl = roots(ps)
        val, _ = quad(lambda x: (p(x) - ps) / (x * x), rv, rl, epsabs=1e-14, epsrel=1e-11, limit=400)
        return val

    eps = 1e-12 * abs(p_hi - p_lo)
    ps = brentq(area, p_lo + eps, p_hi - eps, xtol=1e-17, rtol=1e-14)
    rv, rl = roots(ps)
    return rl, rv
