"""Plain reference algorithm for cos(A) and sin(A) (oracle, test infrastructure).

This is deliberately NOT the paper's factorized scheme: it is the textbook
scaling + Taylor + double-angle method, so that it checks the paper's method
from outside.

Steps (definitions from Section 2.1 and Section 1 of the paper):

1. theta = ||A||_1, the maximum absolute column sum.
2. s = smallest integer >= 0 with theta * 2^-s <= 1.
3. X = 2^-s A and Y = X X.
4. Cosine Taylor polynomial sum_{k=0}^{m} (-1)^k Y^k / (2k)!  and the sine
   inner sum sum_{k=0}^{m} (-1)^k Y^k / (2k+1)!, both by Horner's rule in Y
   (the definitions of T^c_{2m} and T^s_{2m+1}).  With ||X||_1 <= 1 the
   neglected tails are below 1/(2m+2)!:  m = 9 in float64 (1/20! < 2^-53/8),
   m = 11 in long double (1/24! < 2^-64/8).
5. S = X * inner.
6. s times, from the old pair: C <- I - 2 S S,  S <- 2 S C  (Section 1).

Pins (tests/test_oracle_reference.py): diagonal matrices against elementwise
cos/sin; symmetric matrices against an eigendecomposition; strictly upper
triangular integer matrices against the exact finite Taylor sum in rationals;
the 2x2 overscaling family [[c, c*lam], [0, -c]] (A^2 = c^2 I) and the
rotation generator tJ (cos(tJ) = cosh(t) I, sin(tJ) = sinh(t) J) in closed
form; 1x1 matrices against libm; random 8x8 matrices against mpmath's
cosm/sinm at 60 digits; nonnormal matrices with ||A||_1 <= 1e-3 against 40-term
Taylor sums in mpmath at 50 digits (C - I to a few units of rounding);
cos^2 + sin^2 = I and CS = SC.
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np

__all__ = ["norm1", "scaling_power", "taylor_terms", "sincosm", "sincosm_ld"]


def norm1(A: np.ndarray) -> float:
    """Maximum absolute column sum of A (the matrix 1-norm), plain loops in numpy."""
    A = np.asarray(A)
    if A.size == 0:
        return 0.0
    return float(np.max(np.sum(np.abs(A), axis=0)))


def scaling_power(theta: float, limit: float = 1.0) -> int:
    """Smallest s >= 0 with theta * 2^-s <= limit, by exact halving."""
    if not math.isfinite(theta):
        raise ValueError("non-finite norm")
    s = 0
    t = float(theta)
    while t > limit:
        t *= 0.5
        s += 1
    return s


def taylor_terms(m: int):
    """Exact coefficients 1/(2k)! and 1/(2k+1)! with sign (-1)^k, k = 0..m."""
    cos_c = [Fraction((-1) ** k, math.factorial(2 * k)) for k in range(m + 1)]
    sin_c = [Fraction((-1) ** k, math.factorial(2 * k + 1)) for k in range(m + 1)]
    return cos_c, sin_c


def _horner(Y, coeffs, I, dtype):
    """sum_k coeffs[k] Y^k by Horner's rule, coefficients given as Fractions."""
    acc = I * dtype(coeffs[-1].numerator) / dtype(coeffs[-1].denominator)
    for c in reversed(coeffs[:-1]):
        acc = Y @ acc + I * (dtype(c.numerator) / dtype(c.denominator))
    return acc


def _sincosm(A, dtype, m):
    A = np.asarray(A, dtype=dtype)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    I = np.eye(n, dtype=dtype)
    theta = norm1(A)
    s = scaling_power(theta)
    X = A * dtype(2.0) ** (-s)
    Y = X @ X
    cos_c, sin_c = taylor_terms(m)
    C = _horner(Y, cos_c, I, dtype)
    S = X @ _horner(Y, sin_c, I, dtype)
    for _ in range(s):
        C, S = I - dtype(2) * (S @ S), dtype(2) * (S @ C)
    return C, S, s


def sincosm(A: np.ndarray):
    """cos(A), sin(A) in float64 (numpy matmul, host BLAS). Returns (C, S)."""
    C, S, _ = _sincosm(A, np.float64, 9)
    return C, S


def sincosm_ld(A: np.ndarray):
    """cos(A), sin(A) in 80-bit long double (numpy's non-BLAS matmul loop).

    Returns long-double arrays. Meant for n <= 512; cost grows like n^3 at a
    few hundred MFLOP/s.
    """
    C, S, _ = _sincosm(np.asarray(A, dtype=np.longdouble), np.longdouble, 11)
    return C, S


def scaling_used(A: np.ndarray) -> int:
    """The scaling power this reference uses for A (for reporting)."""
    return scaling_power(norm1(A))
