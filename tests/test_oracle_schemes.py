"""Pins for oracle/schemes.py: each factorized scheme of Section 2.1 against the
Taylor series of cos / sin (closed form 1/(2k)!, 1/(2k+1)!), and its product
count against Tables 1-2."""
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import schemes

GOLD = os.path.join(os.path.dirname(__file__), "golden", "theta_tables.json")

# (level) -> (cosine exact through x^k, sine exact through x^k) as stated in
# Section 2.1: T^c_4/T^s_5, T^c_8/T^s_7, T^c_8/T^s_9 (Algorithm5sA), T^c_16/T^s_17,
# T^c_24/T^s through x^21.
ORDERS = {3: (5, 6), 4: (9, 8), 5: (9, 10), 6: (17, 18), 7: (25, 22)}


def taylor(kind, k):
    if kind == "c":
        return Fraction(0) if k % 2 else Fraction((-1) ** (k // 2), math.factorial(k))
    return Fraction(0) if k % 2 == 0 else Fraction((-1) ** ((k - 1) // 2), math.factorial(k))


def max_rel_mismatch(poly, kind, upto):
    """max_k<upto |coef_k - taylor_k| * k! (relative to the Taylor magnitude 1/k!)."""
    worst = 0.0
    with mpmath.workdps(60):
        for k in range(upto):
            t = taylor(kind, k)
            d = poly.coeff(k) - mpmath.mpf(t.numerator) / t.denominator
            worst = max(worst, float(abs(d) * math.factorial(k)))
    return worst


@pytest.mark.parametrize("level", [3, 4, 5, 6, 7])
def test_scheme_matches_taylor(level):
    pc, ps = schemes.scheme_polynomials(level)
    oc, os_ = ORDERS[level]
    # level 7: coefficients printed to 20 digits; cancellation lifts the relative
    # residual of the highest matched orders to a few 1e-16 (absolute < 1e-35)
    tol = 1e-30 if level in (3, 4, 5, 6) else 1e-15
    assert max_rel_mismatch(pc, "c", oc) <= tol
    assert max_rel_mismatch(ps, "s", os_) <= tol


@pytest.mark.parametrize("level", [3, 4, 5, 6, 7])
def test_scheme_differs_at_next_order(level):
    """The first mismatch is exactly where the paper's orders end (x^23 for the k=7 sine)."""
    pc, ps = schemes.scheme_polynomials(level)
    oc, os_ = ORDERS[level]
    t = taylor("c", oc + 1)
    assert abs(pc.coeff(oc + 1) - mpmath.mpf(t.numerator) / t.denominator) * math.factorial(oc + 1) > 1e-6
    t = taylor("s", os_ + 1)
    assert abs(ps.coeff(os_ + 1) - mpmath.mpf(t.numerator) / t.denominator) * math.factorial(os_ + 1) > 1e-6


def test_scheme_degrees():
    """Degrees: cos 4/8/16/24 and sine 5/9/25/49 (T^s_{7,9}, T^s_{17,25}, degree-49 sine)."""
    got = {lv: tuple(p.degree for p in schemes.scheme_polynomials(lv)) for lv in (3, 4, 6, 7)}
    assert got == {3: (4, 5), 4: (8, 9), 6: (16, 25), 7: (24, 49)}


def test_product_counts_match_tables():
    with open(GOLD) as f:
        g = json.load(f)
    for level, pi in zip(g["columns_products"], g["columns_products"]):
        assert schemes.count_products(level) == pi


def test_level6_duplicate_z5_is_consistent():
    """Reading of (Algorithm6sA): replacing the identity coefficient of C_24 by any
    other value breaks the x^17 match, so the printed z_5 on both terms is needed."""
    mpmath.mp.dps = 60
    try:
        _check_duplicate_z5()
    finally:
        mpmath.mp.dps = 15


def _check_duplicate_z5():
    c = schemes.coefficients()
    c["z6"] = dict(c["z6"])
    x = schemes.Poly.x()
    one = schemes.Poly.one()
    pc, ps = schemes.level6(x, one, c)
    assert max_rel_mismatch(ps, "s", 18) < 1e-30
    # perturb: identity coefficient differs from z5 by 1e-6 relative
    pert = dict(c)
    z = dict(c["z6"])

    def level6_mod(A, I, cc):
        xx = cc["x"]
        A2 = A @ A
        A4 = A2 @ A2
        A8 = A4 @ (xx[1] * A2 + xx[2] * A4)
        A16 = (xx[3] * A4 + A8) @ (xx[4] * I + xx[5] * A2 + xx[6] * A4 + xx[7] * A8)
        Tc = I - A2 / 2 + xx[8] * A4 + A16
        C24 = (z[5] * (1 + mpmath.mpf("1e-6")) * I + z[5] * A2 + z[6] * A4 + z[7] * A8 + z[8] * Tc) @ A8
        return Tc, A @ (z[0] * I + z[1] * A2 + z[2] * A4 + z[3] * A8 + z[4] * Tc + C24)

    _, ps2 = level6_mod(x, one, pert)
    assert max_rel_mismatch(ps2, "s", 18) > 1e-12


def test_float_scheme_on_scalar_matrix():
    """On a 1x1 matrix the float64 schemes reproduce math.cos/sin within the theta bounds."""
    for level, th in ((3, 6.5e-3), (4, 8.0e-2), (6, 0.98), (7, 1.85)):
        for x in (th, -th, th / 3):
            C, S = schemes.evaluate(level, np.array([[x]]))
            assert abs(C[0, 0] - math.cos(x)) <= 8e-16   # truncation <= u plus a few roundings
            assert abs(S[0, 0] - math.sin(x)) <= 8e-16   # truncation <= u plus a few roundings


def test_level5_product_count_and_shared_cosine():
    """The 5-product scheme spends one product more than k = 4 (Algorithm5sA's own A_8) and
    keeps the k = 4 cosine polynomial exactly."""
    assert schemes.count_products(5) == 5
    with mpmath.workdps(60):
        c4, _ = schemes.scheme_polynomials(4)
        c5, _ = schemes.scheme_polynomials(5)
        for k in range(40):
            assert c4.coeff(k) == c5.coeff(k)
