"""Pins for oracle/paper_algorithm.py: the paper's method (plan + scheme + double
angle) against the independent reference oracle, mpmath, and closed forms."""
import mpmath
import numpy as np
import pytest

import workloads as W
from oracle import paper_algorithm as PA
from oracle import plan as P
from oracle import reference as R
from tests.conftest import rel_fro


@pytest.mark.parametrize("family", ["gaussian", "symmetric", "laplacian1d"])
@pytest.mark.parametrize("e", [-7, -4, -1, 0, 1, 2, 4, 7, 10])
def test_against_reference(family, e):
    A = W.family(family, 64, 2.0 ** e, key=(21, e + 10))
    C, S, plan = PA.sincosm(A, return_plan=True)
    Cr, Sr = R.sincosm(A)
    assert plan == P.plan(np.linalg.norm(A, 1))
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


@pytest.mark.parametrize("level_norm", [(3, 5e-3), (4, 6e-2), (6, 0.9), (7, 1.8)])
def test_each_level_mpmath(level_norm):
    level, t = level_norm
    A = W.gaussian(6, t, key=(22, level))
    C, S, plan = PA.sincosm(A, return_plan=True)
    assert plan[0] == level and plan[1] == 0
    with mpmath.workdps(40):
        M = mpmath.matrix(A.tolist())
        Cm = np.array(mpmath.cosm(M).tolist(), dtype=float)
        Sm = np.array(mpmath.sinm(M).tolist(), dtype=float)
    assert rel_fro(C, Cm) <= 4e-16 * 6
    assert rel_fro(S, Sm) <= 4e-16 * 6


@pytest.mark.parametrize("acc", ["double", "single"])
def test_single_table_accuracy(acc):
    """With the single table, the float64 evaluation still reaches about 2^-24."""
    A = W.gaussian(32, 64.0, key=(23,))
    C, S = PA.sincosm(A, accuracy=acc)
    Cl, Sl = R.sincosm_ld(A)
    tol = 1e-12 if acc == "double" else 5e-6
    assert rel_fro(C, Cl.astype(float)) <= tol
    assert rel_fro(S, Sl.astype(float)) <= tol


def test_float32_single_accuracy():
    A64 = W.gaussian(48, 16.0, key=(24,))
    A32 = A64.astype(np.float32)
    C, S = PA.sincosm(A32.astype(np.float32), accuracy="single", dtype=np.float32)
    Cr, Sr = R.sincosm(A32.astype(np.float64))
    assert rel_fro(C, Cr) <= 5e-5
    assert rel_fro(S, Sr) <= 5e-5


@pytest.mark.parametrize("acc,theta,tol", [("double", 0.1, 1e-15), ("double", 0.1149, 1e-15),
                                           ("single", 0.8, 2e-7)])
def test_extended_level5_against_mpmath(acc, theta, tol):
    """The 5-product scheme at the top of its band against mpmath's cosm/sinm at 40 digits."""
    A = W.gaussian(8, theta, key=(30, int(theta * 1e5)))
    C, S, plan = PA.sincosm(A, acc, return_plan=True, extended=True)
    assert plan == (5, 0, 5)
    with mpmath.workdps(40):
        M = mpmath.matrix(A.tolist())
        Cm = np.array(mpmath.cosm(M).tolist(), dtype=float)
        Sm = np.array(mpmath.sinm(M).tolist(), dtype=float)
    assert rel_fro(C, Cm) <= tol and rel_fro(S, Sm) <= tol


@pytest.mark.parametrize("lam", [1e2, 1e4, 1e8])
def test_refined_norm_removes_overscaling(lam):
    """Section 4's [[1, lambda], [0, -1]]: A^2 = I, so cos A = cos(1) I and sin A = sin(1) A exactly.
    The tables' plan scales by about lambda and loses accuracy; the refined plan needs s = 0."""
    import math
    A = np.array([[1.0, lam], [0.0, -1.0]])
    Cx, Sx = math.cos(1.0) * np.eye(2), math.sin(1.0) * A
    C0, S0, p0 = PA.sincosm(A, return_plan=True)
    C1, S1, p1 = PA.sincosm(A, return_plan=True, refined=True)
    assert p1 == (7, 0, 7) and p0[1] >= int(math.log2(lam)) - 1
    assert rel_fro(C1, Cx) <= 1e-15 and rel_fro(S1, Sx) <= 1e-15
    if lam >= 1e8:
        assert max(rel_fro(C0, Cx), rel_fro(S0, Sx)) > 1e-12    # the overscaling the paper notes


def test_refined_norm_block_family_and_random():
    """[[I, B], [0, -I]] squares to I for any B (closed form at any size); on Gaussian matrices the
    refined plan never takes more products and stays within 1e-12 of the reference."""
    import math
    n = 24
    B = W.gaussian(n // 2, 300.0, key=(31,))
    A = np.block([[np.eye(n // 2), B], [np.zeros((n // 2, n // 2)), -np.eye(n // 2)]])
    assert np.array_equal(A @ A, np.eye(n))
    C, S, p = PA.sincosm(A, return_plan=True, refined=True)
    assert p == (7, 0, 7)
    assert rel_fro(C, math.cos(1.0) * np.eye(n)) <= 1e-15 and rel_fro(S, math.sin(1.0) * A) <= 1e-15
    for e in (-3, 1, 5, 9):
        A = W.gaussian(40, 2.0 ** e, key=(32, e + 10))
        C, S, p = PA.sincosm(A, return_plan=True, refined=True)
        assert p[2] <= P.plan(np.linalg.norm(A, 1))[2]
        Cr, Sr = R.sincosm(A)
        assert rel_fro(C, Cr) <= 1e-12 and rel_fro(S, Sr) <= 1e-12
