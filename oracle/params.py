"""ORACLE -- test infrastructure only.

Plan-time parameters of the complex-coordinate FMM written from their
definitions (Sec. 4.1, Sec. 5.1, Sec. 6.3):

* ``lipschitz_bound_2d(c)``: the 2D convergence condition L < (R - r)/(R + r)
  with c = R/r (the lemma of Sec. 4.1);
* ``lipschitz_bound_3d(c)``: the 3D condition L < z_c =
  (c^2 + 5 - sqrt(12 c^2 + 24)) / (c^2 - 1) (the lemma of Sec. 5.1);
* ``nterms``: the expansion length of a level, the smallest n with
  |f_n(R) g_n(r)| <= eps (Sec. 6.3, prefactors dropped as the paper does in
  practice), R = (0.5 + k) w, r = sqrt(d)/2 w, required at n and n + 1 so a
  zero of g_n cannot end the search early.  Laplace uses (r/R)^n (the
  scale-free form of r^n / R^(n+1)); Helmholtz |H_n(kR) J_n(kr)| in 2D and
  |h_n(kR) j_n(kr)| in 3D, evaluated with scipy's library routines.  Where
  those over- or underflow (small kappa w at high order: |h_n| ~ (2n-1)!!/z^(n+1)
  leaves the FP64 range) the same product is evaluated in mpmath at 30 digits.
"""
from __future__ import annotations

import math

import mpmath
import scipy.special as sp


def lipschitz_bound_2d(c: float) -> float:
    return (c - 1.0) / (c + 1.0)


def lipschitz_bound_3d(c: float) -> float:
    return (c * c + 5.0 - math.sqrt(12.0 * c * c + 24.0)) / (c * c - 1.0)


def separation_ratio(dim: int, sep: int) -> float:
    """c = R / r with R = (0.5 + k) w and r = sqrt(dim)/2 w."""
    return (0.5 + sep) / (math.sqrt(dim) / 2.0)


def _normal(*xs) -> bool:
    """Every factor finite and of normal magnitude (no overflow, no underflow)."""
    return all(math.isfinite(abs(x)) and abs(x) >= 1e-300 for x in xs)


def _crit_mp(dim, kappa, R, r, n):
    with mpmath.workdps(30):
        X, x = mpmath.mpf(kappa) * R, mpmath.mpf(kappa) * r
        if dim == 2:
            v = mpmath.hankel1(n, X) * mpmath.besselj(n, x)
        else:
            h = mpmath.sqrt(mpmath.pi / (2 * X)) * mpmath.hankel1(n + 0.5, X)
            j = mpmath.sqrt(mpmath.pi / (2 * x)) * mpmath.besselj(n + 0.5, x)
            v = h * j
        return float(abs(v))


def _crit(dim, kernel, kappa, R, r, n):
    if kernel == "laplace":
        return (r / R) ** n
    if dim == 2:
        h, j = sp.hankel1(n, kappa * R), sp.jv(n, kappa * r)
    else:
        h = sp.spherical_jn(n, kappa * R) + 1j * sp.spherical_yn(n, kappa * R)
        j = sp.spherical_jn(n, kappa * r)
    if _normal(h, j):
        return abs(h * j)
    return _crit_mp(dim, kappa, R, r, n)


def nterms(dim: int, kernel: str, kappa: float, w: float, sep: int, eps: float,
           pmax: int) -> int:
    """Expansion length for boxes of width w; pmax + 1 if none <= pmax works."""
    R = (0.5 + sep) * w
    r = math.sqrt(dim) / 2.0 * w
    for n in range(1, pmax + 1):
        if _crit(dim, kernel, kappa, R, r, n) <= eps and _crit(dim, kernel, kappa, R, r, n + 1) <= eps:
            return n
    return pmax + 1
