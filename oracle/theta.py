"""Truncation-error bounds and the theta tables (oracle, test infrastructure).

Section 3 of the paper writes the truncation error of each scheme as a power
series (newtyerrsertay), bounds its norm by the series of absolute values
evaluated at theta = ||A|| (newtyerrnorm), and defines theta_{2m} as the
largest theta for which that bound does not exceed the unit roundoff u
(u = 2^-53 for double, 2^-24 for single), truncating the series after 150
terms. Tables 1 and 2 list the results.

Here the error series is formed from the scalar polynomial each scheme
represents (``schemes.scheme_polynomials``) and the Taylor coefficients of
cos / sin, in mpmath at 60 digits, and theta is found by bisection on the
increasing function theta -> sum_k |alpha_k| theta^k.

Reading taken (the paper is at odds with itself here): the bound starts at
the first power where the scheme actually differs from the Taylor series,
found from the coefficients. For the 7-product sine that is A^23 (the printed
coefficients match Taylor through A^21 only), which gives theta = 1.8548 in
double precision instead of the printed 1.97; starting the sum at A^25, as
the order 2m~+1 = 23 of the paper's error formula would, reproduces 1.97
(``theta(..., start='paper')``). Low-order residuals that come only from the
20-digit rounding of printed coefficients are excluded from the bound, as they
would be with exact coefficients.

Pins (tests/test_oracle_theta.py): the 16 printed theta values of Tables 1
and 2 (tests/golden/theta_tables.json) to their printed digits, with the
single documented exception above.
"""
from __future__ import annotations

import math

import mpmath

from .schemes import scheme_polynomials

__all__ = ["taylor_coeff", "error_series", "first_mismatch", "theta",
           "PAPER_START", "U_DOUBLE", "U_SINGLE", "table"]

U_DOUBLE = mpmath.mpf(2) ** -53
U_SINGLE = mpmath.mpf(2) ** -24

# First power of A in the paper's error series (newtyerrsertay):
# 2m+2 with 2m in {4, 8, 16, 24} for cosine, 2m~+3 with 2m~+1 in {5, 7, 17, 23} for sine.
PAPER_START = {("c", 3): 6, ("c", 4): 10, ("c", 6): 18, ("c", 7): 26,
               ("s", 3): 7, ("s", 4): 9, ("s", 6): 19, ("s", 7): 25}


def taylor_coeff(kind: str, k: int):
    """Coefficient of x^k in the Maclaurin series of cos (kind 'c') or sin ('s')."""
    if kind == "c":
        return mpmath.mpf(0) if k % 2 else mpmath.mpf((-1) ** (k // 2)) / math.factorial(k)
    if kind == "s":
        return mpmath.mpf(0) if k % 2 == 0 else mpmath.mpf((-1) ** ((k - 1) // 2)) / math.factorial(k)
    raise ValueError(kind)


def error_series(level: int, kind: str, nterms: int = 150, dps: int = 60):
    """alpha_k = Taylor_k - scheme_k for k = 0 .. nterms-1 (mpmath numbers)."""
    with mpmath.workdps(dps):
        pc, ps = scheme_polynomials(level, dps)
        p = pc if kind == "c" else ps
        return [taylor_coeff(kind, k) - p.coeff(k) for k in range(nterms)]


def first_mismatch(level: int, kind: str, rel_tol: float = 1e-15) -> int:
    """First power k at which the scheme differs from Taylor by more than rel_tol * k!^-1."""
    alpha = error_series(level, kind, nterms=60)
    for k, a in enumerate(alpha):
        if abs(a) * math.factorial(k) > rel_tol:
            return k
    return 60


def theta(level: int, kind: str, u, start="actual", nterms: int = 150, dps: int = 60):
    """Largest theta with sum_{k >= start} |alpha_k| theta^k <= u (bisection).

    ``start`` is 'actual' (first power where the scheme differs from Taylor),
    'paper' (the order stated in the paper's error formula) or an integer.
    """
    if start == "actual":
        k0 = first_mismatch(level, kind)
    elif start == "paper":
        k0 = PAPER_START[(kind, level)]
    else:
        k0 = int(start)
    with mpmath.workdps(dps):
        alpha = error_series(level, kind, nterms=nterms, dps=dps)
        mags = [abs(a) for a in alpha[k0:]]
        u = mpmath.mpf(u)

        def bound(t):
            return mpmath.fsum(m * t ** (k0 + i) for i, m in enumerate(mags))

        lo, hi = mpmath.mpf(0), mpmath.mpf(1)
        while bound(hi) <= u:
            hi *= 2
        for _ in range(200):
            mid = (lo + hi) / 2
            if bound(mid) <= u:
                lo = mid
            else:
                hi = mid
        return float(lo)


def table(u, start="actual"):
    """{(kind, level): theta} for all eight schemes at unit roundoff u."""
    return {(k, lv): theta(lv, k, u, start=start) for k in ("c", "s") for lv in (3, 4, 6, 7)}
