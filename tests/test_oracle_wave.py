"""Pins for oracle/wave.py (c(t^2 A), s(t, A) of Sections 1 and 2.2)."""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import reference as R
from oracle import wave as Wv
from oracle.theta import U_DOUBLE, U_SINGLE
from tests.conftest import rel_fro


@pytest.mark.parametrize("t", [0.3, 1.0, 2.5])
@pytest.mark.parametrize("e", [-3, 0, 3])
def test_square_of_nonsymmetric(t, e):
    """A = X^2: c(t^2 A) = cos(tX) and s(t, A) X = sin(tX) (independent cos/sin reference)."""
    X = W.gaussian(30, 2.0 ** e, key=(100, e + 5))
    A = X @ X
    C, S = Wv.reference(A, t)
    Cx, Sx = R.sincosm(t * X)
    assert rel_fro(C, Cx) <= 1e-12
    assert rel_fro(S @ X, Sx) <= 1e-12
    Cp, Sp = Wv.paper_wave(A, t)
    assert rel_fro(Cp, Cx) <= 1e-12
    assert rel_fro(Sp @ X, Sx) <= 1e-12


@pytest.mark.parametrize("target", [0.5, 8.0, 200.0])
def test_spd_eigh(target):
    A = W.laplacian_1d(40, target)
    lam, Q = np.linalg.eigh(A)
    t = 1.7
    r = np.sqrt(np.maximum(lam, 0.0))
    Cr = (Q * np.cos(t * r)) @ Q.T
    Sr = (Q * np.where(r > 0, np.sin(t * r) / np.where(r > 0, r, 1.0), t)) @ Q.T
    for fn in (Wv.reference, Wv.paper_wave):
        C, S = fn(A, t)
        assert rel_fro(C, Cr) <= 1e-12 * max(1.0, target)
        assert rel_fro(S, Sr) <= 1e-12 * max(1.0, target)


def test_block_exponential():
    """e^{tM}, M = [[0, I], [-A, 0]] equals [[c, s], [-A s, c]] (scipy expm)."""
    n = 12
    A = W.gaussian(n, 6.0, key=(101,))
    t = 0.8
    M = np.zeros((2 * n, 2 * n))
    M[:n, n:] = np.eye(n)
    M[n:, :n] = -A
    E = scipy.linalg.expm(t * M)
    for fn in (Wv.reference, Wv.paper_wave):
        C, S = fn(A, t)
        assert rel_fro(C, E[:n, :n]) <= 1e-12
        assert rel_fro(S, E[:n, n:]) <= 1e-12
        assert rel_fro(-A @ S, E[n:, :n]) <= 1e-12
        assert rel_fro(C, E[n:, n:]) <= 1e-12


@pytest.mark.parametrize("a", [0.0, 1e-6, 0.7, 30.0, -4.0])
def test_scalar(a):
    t = 1.3
    C, S = Wv.reference(np.array([[a]]), t)
    if a > 0:
        r = math.sqrt(a)
        cr, sr = math.cos(t * r), math.sin(t * r) / r
    elif a < 0:
        r = math.sqrt(-a)
        cr, sr = math.cosh(t * r), math.sinh(t * r) / r
    else:
        cr, sr = 1.0, t
    assert abs(C[0, 0] - cr) <= 1e-14 * max(1, abs(cr))
    assert abs(S[0, 0] - sr) <= 1e-14 * max(1, abs(sr))


ORDERS = {2: (4, 3), 3: (4, 4), 4: (8, 8), 5: (12, 10)}


@pytest.mark.parametrize("level", [2, 3, 4, 5])
def test_wave_polynomials_match_series(level):
    """Cosine part equals sum (-1)^k b^k/(2k)! and sine part sum (-1)^k b^k/(2k+1)! through the
    orders of Section 2.2 (the 5-product sine through b^10, i.e. A^21 in the cos/sin scheme)."""
    with mpmath.workdps(60):
        Pc, Ps = Wv.wave_polynomials(level)
        oc, os_ = ORDERS[level]
        tol = 1e-30 if level != 5 else 1e-15
        for k in range(oc + 1):
            want = mpmath.mpf((-1) ** k) / math.factorial(2 * k)
            assert abs(Pc.coeff(k) - want) * math.factorial(2 * k) <= tol, ("c", k)
        for k in range(os_ + 1):
            want = mpmath.mpf((-1) ** k) / math.factorial(2 * k + 1)
            assert abs(Ps.coeff(k) - want) * math.factorial(2 * k + 1) <= tol, ("s", k)
        k = os_ + 1
        want = mpmath.mpf((-1) ** k) / math.factorial(2 * k + 1)
        assert abs(Ps.coeff(k) - want) * math.factorial(2 * k + 1) > 1e-8


def test_printed_sign_of_p34_is_wrong():
    """With -(6!/7!) B_4, as printed, the b^3 coefficient of the sine part is wrong."""
    with mpmath.workdps(60):
        from oracle.schemes import Poly
        b = Poly.x()
        one = Poly.one()
        B2 = b @ b
        B4 = B2 @ (-b / 720 + B2 / 40320)
        printed = one - b / 6 + B2 / 120 - B4 / 7
        assert abs(printed.coeff(3) - mpmath.mpf(-1) / 5040) > 1e-5


def test_cosine_theta_is_square_of_cos_table():
    from oracle import theta as T
    for level, lv in ((3, 4), (4, 6), (5, 7)):
        for u in (U_DOUBLE, U_SINGLE):
            assert abs(Wv.theta_wave(level, "c", u) - T.theta(lv, "c", u) ** 2) <= 1e-9 * Wv.theta_wave(level, "c", u)


@pytest.mark.parametrize("acc", ["double", "single"])
def test_wave_table_constants(acc):
    assert Wv.WAVE_THETA[acc] == pytest.approx(Wv.wave_table(acc), rel=1e-12)


def test_wave_plan_brute_force():
    g = np.random.default_rng(3)
    for t in np.exp2(g.uniform(-20, 30, size=2000)):
        for acc in ("double", "single"):
            cands = []
            for level in (2, 3, 4, 5):
                for s in range(0, 200):
                    if t <= Wv.WAVE_THETA[acc][level] * 4.0 ** s:
                        cands.append((level + 2 * s, s, level))
                        break
            cost, s, level = min(cands)
            assert Wv.wave_plan(float(t), acc) == (level, s, cost)
