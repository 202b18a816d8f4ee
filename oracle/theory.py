"""Leading-order theory used to pin the oracle (TEST INFRASTRUCTURE ONLY).

Everything here evaluates the EOS through the oracle's own C routine
(``oracle.eos``) and integrates with scipy quadrature.

* ``critical_point``      -- (rho_c, T_c) of the Carnahan-Starling EOS from
  dp/drho = d2p/drho2 = 0 (the EOS is named in Section II; its form is the
  reading stated in ``lbm_oracle.c``).
* ``coexistence``         -- liquid/vapour densities from the mechanical-stability
  condition, Eq. (16), with G2 = 0 and exponent epsilon:
  p(rho_V) = p(rho_L) = p_b and
  integral_{rho_V}^{rho_L} (p_b - p_EOS) psi' / psi^(1+epsilon) drho = 0.
  (For the psi forms used here p_EOS = rho cs^2 + G c^2 psi^2 / 2.)
* ``maxwell``             -- the thermodynamic (Maxwell equal-area) coexistence,
  integral (p_b - p) drho / rho^2 = 0, quoted in Section III.B.
* ``flat_surface_tension`` -- surface tension of a flat interface from the
  pressure tensor of Eq. (22) plus the isotropic 2 sigma |F|^2 / psi^2 term of
  the Eq. (8) forcing: with u = (d psi / dn)^2 the normal balance
  (G/4) psi psi'' + 2 sigma G^2 psi'^2 = p_b - p_EOS integrates to
  u(psi) = (8/G) psi^eps integral_{psi_V}^{psi} (p_b - p) s^(-1-eps) ds,
  and P_n - P_t = (G/6)(1 - kappa) psi psi'' gives
  surface tension = -(G/6)(1 - kappa) integral sqrt(u) dpsi.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize

import oracle as O


def _p(P, rho):
    return O.eos(P, np.asarray(rho, dtype=float))[0]


def _psi(P, rho):
    return O.eos(P, np.asarray(rho, dtype=float))[1]


def _dpsi(P, rho):
    rho = np.asarray(rho, dtype=float)
    h = 1e-6 * rho
    return (_psi(P, rho + h) - _psi(P, rho - h)) / (2.0 * h)


def critical_point(a: float, b: float, R: float = 1.0):
    """(rho_c, T_c) of the Carnahan-Starling EOS p = T A(rho) - a rho^2."""
    P = O.Params(nx=1, ny=1, eos_kind=O.EOS_CS, eos=(a, b, R, 1.0), G=-1.0)

    def A(r):  # p at T = 1 plus a rho^2
        return _p(P, r) + a * r * r

    def d1(r, h):
        return (A(r + h) - A(r - h)) / (2 * h)

    def d2(r, h):
        return (A(r + h) - 2 * A(r) + A(r - h)) / (h * h)

    # critical point: T A' = 2 a rho and T A'' = 2 a  =>  A' - rho A'' = 0
    def g(r):
        h = 1e-4 * r
        return float(d1(r, h) - r * d2(r, h))

    rho_c = optimize.brentq(g, 0.02 / b * 4, 0.3 / b * 4, xtol=1e-14)
    h = 1e-4 * rho_c
    T_c = 2 * a * rho_c / float(d1(rho_c, h))
    return rho_c, T_c


def _spinodals(P, rho_max):
    """Local maximum (vapour side) and minimum (liquid side) of p(rho) on (0, rho_max)."""
    r = np.linspace(rho_max * 1e-5, rho_max, 200001)
    p = _p(P, r)
    ok = np.isfinite(p)
    dp = np.diff(p)
    i_max = None
    for i in range(1, len(dp)):
        if ok[i] and dp[i - 1] > 0 and dp[i] <= 0:
            i_max = i
            break
    if i_max is None:
        raise ValueError("EOS has no van der Waals loop on (0, %g)" % rho_max)
    i_min = None
    for i in range(i_max + 1, len(dp)):
        if ok[i] and dp[i - 1] < 0 and dp[i] >= 0:
            i_min = i
            break
    if i_min is None:
        raise ValueError("no liquid branch found")
    return r[i_max], r[i_min], r


def _branch_roots(P, pb, ra, rb, rho_hi):
    lo = 1e-12
    rv = optimize.brentq(lambda x: float(_p(P, x)) - pb, lo, ra, xtol=1e-15, rtol=1e-14)
    rl = optimize.brentq(lambda x: float(_p(P, x)) - pb, rb, rho_hi, xtol=1e-15, rtol=1e-14)
    return rv, rl


def _breaks(P, a, b):
    if P.eos_kind == O.EOS_PIECEWISE:
        return [x for x in (P.eos[3], P.eos[4]) if a < x < b]
    return None


def _solve(P, weight, rho_max):
    ra, rb, _ = _spinodals(P, rho_max)
    p_hi = float(_p(P, ra))
    p_lo = max(float(_p(P, rb)), 0.0) + 1e-9 * abs(p_hi)
    # largest density on the liquid branch where the EOS (and psi) is defined
    rho_hi = rb
    step = (rho_max - rb) / 2000.0
    while rho_hi + step < rho_max and np.isfinite(_psi(P, rho_hi + step)):
        rho_hi += step

    def I(pb):
        rv, rl = _branch_roots(P, pb, ra, rb, rho_hi)
        val, _ = integrate.quad(lambda x: (pb - float(_p(P, x))) * weight(x), rv, rl,
                                points=_breaks(P, rv, rl), limit=400, epsabs=0, epsrel=1e-11)
        return val

    a_, b_ = p_lo, p_hi * (1 - 1e-12)
    fa, fb = I(a_), I(b_)
    if np.sign(fa) == np.sign(fb):
        raise ValueError("no coexistence root (I(p_lo)=%g, I(p_hi)=%g)" % (fa, fb))
    pb = optimize.brentq(I, a_, b_, xtol=1e-16, rtol=1e-13)
    rv, rl = _branch_roots(P, pb, ra, rb, rho_hi)
    return rl, rv, pb


def _rho_max(P):
    if P.eos_kind == O.EOS_CS:
        return 4.0 / P.eos[1] * 0.999
    if P.eos_kind == O.EOS_PIECEWISE:
        return P.eos[4] * 1.5
    return 50.0 * P.eos[1]


def coexistence(P: "O.Params", epsilon: float):
    """(rho_L, rho_V, p_b) from the mechanical-stability condition, Eq. (16) with G2 = 0."""
    def w(x):
        ps = float(_psi(P, x))
        return float(_dpsi(P, x)) / ps ** (1.0 + epsilon)
    return _solve(P, w, _rho_max(P))


def maxwell(P: "O.Params"):
    """(rho_L, rho_V, p_b) from the Maxwell equal-area construction in 1/rho."""
    return _solve(P, lambda x: 1.0 / (x * x), _rho_max(P))


def flat_surface_tension(P: "O.Params", epsilon: float, kappa: float = 0.0, n: int = 40001):
    """Leading-order surface tension of a flat interface (see module docstring)."""
    rl, rv, pb = coexistence(P, epsilon)
    G = P.G
    # dense grid in rho, refined near both ends where psi changes fastest
    t = np.linspace(0.0, 1.0, n)
    s = 0.5 - 0.5 * np.cos(np.pi * t)
    rho = rv + (rl - rv) * s
    brk = _breaks(P, rv, rl) or []
    rho = np.unique(np.concatenate([rho, np.array(brk, dtype=float)]))
    psi = _psi(P, rho)
    dpsi = _dpsi(P, rho)
    integrand = (pb - _p(P, rho)) * dpsi * psi ** (-1.0 - epsilon)
    J = integrate.cumulative_trapezoid(integrand, rho, initial=0.0)
    u = (8.0 / G) * psi ** epsilon * J
    root = np.sqrt(np.clip(u, 0.0, None))
    tension = -(G / 6.0) * (1.0 - kappa) * integrate.trapezoid(root * dpsi, rho)
    return float(tension)
