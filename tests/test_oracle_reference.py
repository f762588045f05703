"""Pins for oracle/reference.py (the independent Taylor + double-angle oracle).

Each test compares with something fixed by mathematics, not by the oracle:
elementwise cos/sin on diagonal matrices, eigendecomposition for symmetric
matrices, exact rational finite sums for nilpotent matrices, closed forms for
matrices with A^2 = c^2 I and for the rotation generator, libm on 1x1
matrices, mpmath's arbitrary-precision cosm/sinm on random matrices, 40-term
Taylor sums at 50 digits on tiny nonnormal matrices, and the identities
cos^2 + sin^2 = I, CS = SC.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import workloads as W
from oracle import reference as R
from tests.conftest import rel_fro

NORM_EXPS = [-8, -4, 0, 1, 4, 7, 10]


@pytest.mark.parametrize("e", NORM_EXPS)
def test_diagonal(e):
    d = W.rng(11, e + 20).uniform(-1, 1, size=24)
    d *= 2.0 ** e / np.max(np.abs(d))
    C, S = R.sincosm(np.diag(d))
    tol = 1e-15 * max(1.0, 2.0 ** e)
    assert np.max(np.abs(np.diag(C) - np.cos(d))) <= tol
    assert np.max(np.abs(np.diag(S) - np.sin(d))) <= tol
    assert np.count_nonzero(C - np.diag(np.diag(C))) == 0
    assert np.count_nonzero(S - np.diag(np.diag(S))) == 0


@pytest.mark.parametrize("e", NORM_EXPS)
def test_symmetric_eigh(e):
    A = W.symmetric_gaussian(48, 2.0 ** e, key=(12, e + 20))
    lam, Q = np.linalg.eigh(A)
    Cr = (Q * np.cos(lam)) @ Q.T
    Sr = (Q * np.sin(lam)) @ Q.T
    C, S = R.sincosm(A)
    tol = 4e-15 * max(1.0, 2.0 ** e) * 48 ** 0.5
    assert rel_fro(C, Cr) <= tol
    assert np.linalg.norm(S - Sr) <= tol * max(np.linalg.norm(Sr), 1e-300)


def _frac_matmul(X, Y):
    n = len(X)
    return [[sum(X[i][k] * Y[k][j] for k in range(n)) for j in range(n)] for i in range(n)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_nilpotent_exact(seed):
    """Strictly upper triangular integer matrices: finite Taylor sums in exact rationals.

    A transposed operand or a wrong sign would produce a lower-triangular or
    sign-flipped result and fail here."""
    n = 7
    A = W.nilpotent_upper(n, key=(13, seed))
    Af = [[Fraction(int(v)) for v in row] for row in A]
    I = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    powers = [I]
    for _ in range(n):
        powers.append(_frac_matmul(powers[-1], Af))
    Cex = [[Fraction(0)] * n for _ in range(n)]
    Sex = [[Fraction(0)] * n for _ in range(n)]
    for k in range(n):
        c = Fraction((-1) ** (k // 2), math.factorial(k))
        target = Cex if k % 2 == 0 else Sex
        for i in range(n):
            for j in range(n):
                target[i][j] += c * powers[k][i][j]
    Cx = np.array([[float(v) for v in r] for r in Cex])
    Sx = np.array([[float(v) for v in r] for r in Sex])
    C, S = R.sincosm(A)
    assert rel_fro(C, Cx) <= 1e-13
    assert rel_fro(S, Sx) <= 1e-13


@pytest.mark.parametrize("c", [0.1, 1.0, 3.0])
@pytest.mark.parametrize("lam", [1.0, 10.0, 100.0])
def test_squares_to_scalar(c, lam):
    """A = c [[1, lam], [0, -1]] has A^2 = c^2 I: cos A = cos(c) I, sin A = sin(c)/c A."""
    A = c * W.overscale_2x2(lam)
    C, S = R.sincosm(A)
    Cr = math.cos(c) * np.eye(2)
    Sr = (math.sin(c) / c) * A
    tol = 1e-15 * (1 + lam) * max(1, R.scaling_used(A)) * 8
    assert np.max(np.abs(C - Cr)) <= tol
    assert np.max(np.abs(S - Sr)) <= tol * (1 + lam)


@pytest.mark.parametrize("t", [0.01, 0.5, 2.0, 10.0])
def test_rotation_generator_hyperbolic(t):
    """cos(tJ) = cosh(t) I and sin(tJ) = sinh(t) J for J = [[0,-1],[1,0]] (J^2 = -I)."""
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    C, S = R.sincosm(t * J)
    assert rel_fro(C, math.cosh(t) * np.eye(2)) <= 1e-14 * max(1, t)
    assert rel_fro(S, math.sinh(t) * J) <= 1e-14 * max(1, t)


def test_scalar_libm():
    for x in np.concatenate([np.linspace(-20, 20, 81), [1e-9, 0.3, 700.0, -1000.0]]):
        C, S = R.sincosm(np.array([[x]]))
        tol = 2e-16 * max(1.0, abs(x)) * 8
        assert abs(C[0, 0] - math.cos(x)) <= tol, x
        assert abs(S[0, 0] - math.sin(x)) <= tol, x


@pytest.mark.parametrize("e", [-3, 1, 3, 5])
def test_mpmath_random_nonsymmetric(e):
    """Random 8x8 nonsymmetric matrices against mpmath cosm/sinm at 40 digits."""
    A = W.gaussian(8, 2.0 ** e, key=(14, e + 10))
    with mpmath.workdps(40):
        M = mpmath.matrix(A.tolist())
        Cm = np.array(mpmath.cosm(M).tolist(), dtype=float)
        Sm = np.array(mpmath.sinm(M).tolist(), dtype=float)
    C, S = R.sincosm(A)
    assert rel_fro(C, Cm) <= 1e-14 * max(1, 2.0 ** e)
    assert rel_fro(S, Sm) <= 1e-14 * max(1, 2.0 ** e)


def _mp_taylor(A, terms=40, dps=50):
    """cos A and sin A as the plain Taylor sums that define them (Section 2.1), powers A^0 ..
    A^(2 terms - 1), every product and sum in mpmath at `dps` digits; also C - I."""
    with mpmath.workdps(dps):
        n = A.shape[0]
        M = mpmath.matrix(A.tolist())
        P = mpmath.eye(n)
        C = mpmath.zeros(n, n)
        S = mpmath.zeros(n, n)
        fact = mpmath.mpf(1)
        for k in range(2 * terms):
            if k > 0:
                P = P * M
                fact *= k
            term = P / fact
            if k % 2 == 0:
                C += term if (k // 2) % 2 == 0 else -term
            else:
                S += term if (k // 2) % 2 == 0 else -term
        I = mpmath.eye(n)
        to_np = lambda X: np.array([[float(X[i, j]) for j in range(n)] for i in range(n)])
        return to_np(C), to_np(S), to_np(C - I)


@pytest.mark.parametrize("norm", [1e-3, 1e-5, 1e-8])
@pytest.mark.parametrize("kind", ["gaussian", "triangular"])
def test_tiny_norm_mpmath_taylor(norm, kind):
    """||A||_1 <= 1e-3, nonnormal: the oracle (s = 0, Horner to degree 18/19) against a
    40-term Taylor sum at 50 digits. C - I is compared separately, with an absolute bar of a
    few units of rounding of C (its entries are near those of I), so that the A^2 term
    beneath the identity is pinned: at ||A||_1 = 1e-3 it is 1e-7, nine orders of magnitude
    above the bar, so a wrong sign or factorial there fails (measured: at most 1.5 u)."""
    if kind == "gaussian":
        A = W.gaussian(10, norm, key=(16, int(-math.log10(norm))))
    else:
        G = np.triu(W.rng(17, int(-math.log10(norm))).standard_normal((10, 10)))
        G[np.triu_indices(10, 1)] *= 30.0        # strongly nonnormal, not nilpotent
        A = W.rescale(G, norm)
    Cm, Sm, CmI = _mp_taylor(A)
    C, S = R.sincosm(A)
    assert R.scaling_used(A) == 0
    u = 2.0 ** -53
    assert rel_fro(C, Cm) <= 2e-16
    assert rel_fro(S, Sm) <= 4e-16
    assert np.linalg.norm((C - np.eye(10)) - CmI) <= 4 * u * 10 ** 0.5


def test_long_double_agrees_with_mpmath():
    A = W.gaussian(6, 3.0, key=(15,))
    with mpmath.workdps(40):
        M = mpmath.matrix(A.tolist())
        Cm = mpmath.cosm(M)
        Sm = mpmath.sinm(M)
    C, S = R.sincosm_ld(A)
    errc = max(abs(mpmath.mpf(float(C[i, j])) - Cm[i, j]) for i in range(6) for j in range(6))
    # long double carries ~19 digits; compare beyond float64 resolution
    errc_ld = max(abs(mpmath.mpf(str(C[i, j])) - Cm[i, j]) for i in range(6) for j in range(6))
    assert errc_ld < 1e-16
    assert errc < 1e-14


@pytest.mark.parametrize("e", [-2, 2, 6, 10])
def test_identities(e):
    n = 40
    A = W.gaussian(n, 2.0 ** e, key=(16, e + 10))
    C, S = R.sincosm(A)
    I = np.eye(n)
    u = 2.0 ** -53
    denom = np.linalg.norm(C) ** 2 + np.linalg.norm(S) ** 2 + n ** 0.5
    assert np.linalg.norm(C @ C + S @ S - I) / denom <= 64 * n * u
    assert np.linalg.norm(C @ S - S @ C) / denom <= 64 * n * u


def test_parity_bitwise():
    A = W.gaussian(32, 5.0, key=(17,))
    C1, S1 = R.sincosm(A)
    C2, S2 = R.sincosm(-A)
    assert np.array_equal(C1, C2)
    assert np.array_equal(S1, -S2)


def test_zero_and_empty():
    C, S = R.sincosm(np.zeros((5, 5)))
    assert np.array_equal(C, np.eye(5)) and not S.any()
    C, S = R.sincosm(np.zeros((0, 0)))
    assert C.shape == (0, 0) and S.shape == (0, 0)


def test_fp64_vs_long_double_close():
    A = W.gaussian(64, 2.0, key=(1, 64, 0, 0))
    C, S = R.sincosm(A)
    Cl, Sl = R.sincosm_ld(A)
    assert rel_fro(C, Cl.astype(np.float64)) <= 1e-14
    assert rel_fro(S, Sl.astype(np.float64)) <= 1e-14
