"""Plant mistakes in the oracle (on the CPU) and check that its pins catch them.

Each mutation patches one ingredient of the oracle and runs the check that is
supposed to detect it; the test passes when the check fails."""
from fractions import Fraction
import math

import numpy as np
import pytest

import workloads as W
from oracle import plan as P
from oracle import reference as R
from oracle import schemes


def diag_pin_error():
    d = np.linspace(-3.0, 3.0, 13)
    C, S = R.sincosm(np.diag(d))
    return max(np.max(np.abs(np.diag(C) - np.cos(d))), np.max(np.abs(np.diag(S) - np.sin(d))))


def nilpotent_pin_error():
    A = np.triu(np.ones((4, 4)), 1)
    A[0, 3] = 2.0
    # exact: A^2, A^3 by hand in rationals via numpy ints (small exact integers)
    A2 = A @ A
    A3 = A2 @ A
    Cx = np.eye(4) - A2 / 2
    Sx = A - A3 / 6
    C, S = R.sincosm(A)
    return max(np.max(np.abs(C - Cx)), np.max(np.abs(S - Sx)))


def test_pins_pass_unmutated():
    assert diag_pin_error() < 1e-14
    assert nilpotent_pin_error() < 1e-14


@pytest.mark.parametrize("mut", ["drop_term", "flip_sign", "wrong_factorial"])
def test_taylor_mutations_caught(monkeypatch, mut):
    orig = R.taylor_terms

    def bad(m):
        c, s = orig(m)
        c, s = list(c), list(s)
        if mut == "drop_term":
            c[2] = Fraction(0)
        elif mut == "flip_sign":
            s[1] = -s[1]
        else:
            c[1] = Fraction(-1, 3)
        return c, s

    monkeypatch.setattr(R, "taylor_terms", bad)
    assert diag_pin_error() > 1e-8


def test_scaling_off_by_one_caught(monkeypatch):
    orig = R.scaling_power
    monkeypatch.setattr(R, "scaling_power", lambda t, limit=1.0: max(orig(t, limit) - 2, 0))
    # norm 6 needs s = 3; using s = 1 leaves ||X|| = 3 and m = 9 truncation error ~ 3^20/20!
    d = np.linspace(-6.0, 6.0, 13)
    C, _ = R.sincosm(np.diag(d))
    assert np.max(np.abs(np.diag(C) - np.cos(d))) > 1e-12


def test_transposed_operand_caught(monkeypatch):
    """A transposed product (X^T instead of X) is caught by the nilpotent pin."""
    orig = R._horner

    def transposing_horner(Y, coeffs, I, dtype):
        return orig(Y.T.copy(), coeffs, I, dtype)

    monkeypatch.setattr(R, "_horner", transposing_horner)
    assert nilpotent_pin_error() > 1e-3


def test_scheme_coefficient_typo_caught(monkeypatch):
    import mpmath
    orig = schemes.coefficients

    def bad(dps=60):
        c = orig(dps)
        c["x"] = dict(c["x"])
        c["x"][8] = c["x"][8] * (1 + mpmath.mpf("1e-9"))
        return c

    monkeypatch.setattr(schemes, "coefficients", bad)
    with mpmath.workdps(60):
        pc, _ = schemes.scheme_polynomials(6)
        k = 4
        err = abs(pc.coeff(k) - mpmath.mpf(1) / math.factorial(k)) * math.factorial(k)
    assert err > 1e-12


def test_plan_tie_rule_caught():
    """Preferring the larger s on a tie changes the plan: at norm 0.1 both (6, 0) and
    (4, 1) cost 6 products; the rule picks (6, 0)."""
    t = 0.1
    assert P.plan(t) == (6, 0, 6)
    lv, s, cost = P.plan(t)
    cands = []
    for level, th in P.THETA["double"].items():
        pi = P.PRODUCTS[level]
        ss = P.scaling_for(t, th)
        cands.append((pi + 2 * ss, -ss, level))
    wrong = min(cands)
    assert (lv, s) != (wrong[2], -wrong[1]) or cost != wrong[0]
