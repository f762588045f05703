"""Wave-equation functions c(t^2 A) and s(t, A) (oracle, test infrastructure).

Section 1 of the paper writes the solution of y'' + A y = 0 through
  c(t^2 A) = cos(sqrt(t^2 A)) = sum_k (-1)^k (t^2 A)^k / (2k)!,
  s(t, A)  = (sqrt A)^-1 sin(t sqrt A) = t sum_k (-1)^k (t^2 A)^k / (2k+1)!,
and the double angle c(4 t^2 A) = 2 c(t^2 A)^2 - I, s(2t, A) = 2 s(t, A) c(t^2 A).
Section 2.2 adapts the factorized schemes: with B = t^2 A in the role of A_2
and the scalar t in the role of the final factor A, each scheme needs one
product fewer:
  2 products: P^c_4 and P^s_{3,4}            (from Algorithm4cA/4sA)
  3 products: P^c_4 and P^s_4                (adds the Algorithm5sA sine)
  4 products: P^c_8 and P^s_{8,12}           (from Algorithm6cA/6sA, eq:cosm8)
  5 products: P^c_12 and P^s_{11,24}         (from Algorithm7cA/7sA)

Readings (the paper is garbled or silent here):
* P^s_{3,4} is printed with -(6!/7!) B_4; the B^3 coefficient of the sine
  series requires +(6!/7!) B_4 (as in Algorithm4sA), which is used.
* The 5-product sine writes z_11 P^c_12(A) inside C_24; read as P^c_12(B).
* The 4-product cosine writes y_0 I + y_1 B + y_2 B_2 + B_8 "with the same
  coefficients" as eq:cosm8: read as y_0 = 1, y_1 = -1/2, y_2 = x_8 (the
  Algorithm6cA cosine with A_2 -> B).
* Error bounds (no tables in the paper): with B_s = 4^-s B the cosine
  truncation error is sum_k |alpha_k| ||B_s||^k and the sine's, relative to
  the factor t, sum_k |beta_k| ||B_s||^k; theta_B is where the sum reaches u.
  Because the wave cosine polynomial in B equals the cos scheme's polynomial
  in A^2, theta_B^c = (theta^c)^2 exactly.
* Scaling: B_s = 4^-s t^2 A (t halved s times), s double-angle steps.

Pins (tests/test_oracle_wave.py): A = X^2 for random nonsymmetric X, where
c(t^2 X^2) = cos(tX) and s(t, X^2) X = sin(tX) by the independent cos/sin
reference; symmetric positive definite A against an eigendecomposition;
the block exponential e^{tM}, M = [[0, I], [-A, 0]], against scipy's expm;
scalar closed forms (cos/cosh, sin/sinh); scheme polynomials against the
Taylor coefficients in B.
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np

from . import schemes as _schemes
from .reference import norm1, taylor_terms
from .theta import U_DOUBLE, U_SINGLE

__all__ = ["reference", "wave2", "wave3", "wave4", "wave5", "WAVE_SCHEMES", "WAVE_PRODUCTS",
           "wave_polynomials", "theta_wave", "wave_table", "wave_plan", "paper_wave"]

WAVE_PRODUCTS = {2: 2, 3: 3, 4: 4, 5: 5}


def _horner(Y, coeffs, I):
    acc = I * (coeffs[-1].numerator / coeffs[-1].denominator)
    for c in reversed(coeffs[:-1]):
        acc = Y @ acc + I * (c.numerator / c.denominator)
    return acc


def reference(A: np.ndarray, t: float, m: int = 9):
    """c(t^2 A), s(t, A) by scaling ||B_s||_1 <= 1, Horner in B_s, and doubling t."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    I = np.eye(n)
    B = (t * t) * A
    th = norm1(B)
    s = 0
    while th > 1.0:
        th *= 0.25
        s += 1
    Bs = B * 4.0 ** (-s)
    ts = t * 2.0 ** (-s)
    cos_c, sin_c = taylor_terms(m)
    C = _horner(Bs, cos_c, I)
    S = ts * _horner(Bs, sin_c, I)
    for _ in range(s):
        C, S = 2.0 * (C @ C) - I, 2.0 * (S @ C)
    return C, S


# ---------------------------------------------------------------------------
# Schemes of Section 2.2 over a generic algebra: B (= t^2 A, scaled), I, and the
# scalar t. Each returns (cosine part, sine part including the factor t).
# ---------------------------------------------------------------------------

def wave2(B, I, t, c=None):
    """2 products: P^c_4(B) and P^s_{3,4}(t, A) (sign of the B_4 term as in Algorithm4sA)."""
    B2 = B @ B
    B4 = B2 @ (-B / 720 + B2 / 40320)
    Pc = I - B / 2 + B2 / 24 + B4
    Ps = (I - B / 6 + B2 / 120 + B4 / 7) * t
    return Pc, Ps


def wave3(B, I, t, c=None):
    """3 products: P^c_4(B) and P^s_4(t, A)."""
    B2 = B @ B
    B4 = B2 @ (-B / 720 + B2 / 40320)
    Pc = I - B / 2 + B2 / 24 + B4
    B4s = B2 @ (-B / 5040 + B2 / 362880)
    Ps = (I - B / 6 + B2 / 120 + B4s) * t
    return Pc, Ps


def wave4(B, I, t, c):
    """4 products: P^c_8(B) and P^s_{8,12}(t, A) with the coefficients of eq:cosm8 and Algorithm6sA."""
    x, z = c["x"], c["z6"]
    B2 = B @ B
    B4 = B2 @ (x[1] * B + x[2] * B2)
    B8 = (x[3] * B2 + B4) @ (x[4] * I + x[5] * B + x[6] * B2 + x[7] * B4)
    Pc = I - B / 2 + x[8] * B2 + B8
    C12 = (z[5] * I + z[5] * B + z[6] * B2 + z[7] * B4 + z[8] * Pc) @ B4
    Ps = (z[0] * I + z[1] * B + z[2] * B2 + z[3] * B4 + z[4] * Pc + C12) * t
    return Pc, Ps


def wave5(B, I, t, c):
    """5 products: P^c_12(B) and P^s_{11,24}(t, A) with the coefficients of Coefs7cA and Coefs7sA."""
    a, z = c["a"], c["z7"]
    B2 = B @ B
    B3 = B2 @ B
    D = {j: a[(0, j)] * I + a[(1, j)] * B + a[(2, j)] * B2 + a[(3, j)] * B3 for j in (1, 2, 3, 4)}
    B6 = D[3] + D[4] @ D[4]
    Pc = D[1] + (D[2] + B6) @ B6
    C24 = (z[6] * I + z[7] * B + z[8] * B2 + z[9] * B3 + z[10] * B6 + z[11] * Pc) @ Pc
    Ps = (z[0] * I + z[1] * B + z[2] * B2 + z[3] * B3 + z[4] * B6 + z[5] * Pc + C24) * t
    return Pc, Ps


WAVE_SCHEMES = {2: wave2, 3: wave3, 4: wave4, 5: wave5}


def wave_polynomials(level: int, dps: int = 60):
    """Scalar polynomials in b (cosine part, sine part divided by t) of a wave scheme."""
    with mpmath.workdps(dps):
        c = _schemes.coefficients(dps)
        Pc, Ps = WAVE_SCHEMES[level](_schemes.Poly.x(), _schemes.Poly.one(), mpmath.mpf(1), c)
        return Pc, Ps


def _series_coeff(kind: str, k: int):
    f = math.factorial(2 * k) if kind == "c" else math.factorial(2 * k + 1)
    return mpmath.mpf((-1) ** k) / f


def theta_wave(level: int, kind: str, u, nterms: int = 75, dps: int = 60) -> float:
    """Largest ||B|| with sum_{k >= k0} |alpha_k| ||B||^k <= u, k0 = first power where the scheme
    differs from the series (75 terms in B = 150 terms in sqrt(B), as in Section 3)."""
    with mpmath.workdps(dps):
        Pc, Ps = wave_polynomials(level, dps)
        p = Pc if kind == "c" else Ps
        alpha = [_series_coeff(kind, k) - p.coeff(k) for k in range(nterms)]
        k0 = next(k for k, a in enumerate(alpha) if abs(a) * math.factorial(2 * k + (kind == "s")) > 1e-15)
        mags = [abs(a) for a in alpha[k0:]]
        u = mpmath.mpf(u)

        def bound(x):
            return mpmath.fsum(m * x ** (k0 + i) for i, m in enumerate(mags))

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


def wave_table(accuracy: str = "double"):
    """min(theta^c_B, theta^s_B) per wave scheme, rounded down to 5 significant digits."""
    u = U_DOUBLE if accuracy == "double" else U_SINGLE
    out = {}
    for level in (2, 3, 4, 5):
        th = min(theta_wave(level, "c", u), theta_wave(level, "s", u))
        e = math.floor(math.log10(th))
        out[level] = math.floor(th / 10 ** (e - 4)) * 10 ** (e - 4)
    return out


# Rounded-down combined bounds on ||B||_1 (computed by wave_table; pinned in tests).
WAVE_THETA = {
    "double": {2: 3.4458e-3, 3: 1.3213e-2, 4: 9.6251e-1, 5: 3.6404},
    "single": {2: 5.2237e-1, 3: 7.354e-1, 4: 8.9612, 5: 2.1848e1},
}


def wave_plan(normB: float, accuracy: str = "double"):
    """(level, s, products) minimising products + 2 s, s least with ||B|| 4^-s <= theta_level."""
    if not math.isfinite(normB) or normB < 0:
        raise ValueError("norm must be finite and >= 0")
    best = None
    for level in (2, 3, 4, 5):
        s = 0
        t = float(normB)
        while t > WAVE_THETA[accuracy][level]:
            t *= 0.25
            s += 1
        cand = (WAVE_PRODUCTS[level] + 2 * s, s, level)
        if best is None or cand[:2] < best[:2]:
            best = cand
    cost, s, level = best
    return level, s, cost


def paper_wave(A: np.ndarray, t: float, accuracy: str = "double", return_plan=False):
    """c(t^2 A), s(t, A) by the Section 2.2 schemes with the plan above, in float64."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    I = np.eye(n)
    B = (t * t) * A
    level, s, products = wave_plan(norm1(B), accuracy)
    Bs = B * 4.0 ** (-s)
    ts = t * 2.0 ** (-s)
    C, S = WAVE_SCHEMES[level](Bs, I, ts, _schemes.float_coefficients())
    for _ in range(s):
        C, S = 2.0 * (C @ C) - I, 2.0 * (S @ C)
    if return_plan:
        return C, S, (level, s, products)
    return C, S
