"""Pins for oracle/closed_forms.py (the 1-D Laplacian family in closed form)."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import propagators as Pr
from oracle import reference as R
from oracle import wave as Wv
from tests.conftest import rel_fro


@pytest.mark.parametrize("n", [3, 10, 64])
def test_eigenpairs(n):
    T = np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    lam, V = CF.laplacian_1d_eig(n)
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-14)
    assert np.abs(T @ V - V * lam).max() <= 1e-14
    assert np.allclose(np.sort(lam), np.linalg.eigvalsh(T), atol=1e-14)


@pytest.mark.parametrize("target", [2.0 ** -3, 4.0, 2.0 ** 7])
def test_sincos_rows_against_reference(target):
    n = 60
    A = W.laplacian_1d(n, target)
    c = target / 4.0
    assert np.array_equal(A, c * W.laplacian_1d(n, 4.0))
    rows = [0, 7, 31, 59]
    Cr, Sr = CF.sincos_rows(n, c, rows)
    C, S = R.sincosm(A)
    assert rel_fro(Cr, C[rows]) <= 1e-12 * max(1.0, target / 8)
    assert rel_fro(Sr, S[rows]) <= 1e-12 * max(1.0, target / 8)


def test_wave_and_unitary_rows():
    n, target, t = 50, 16.0, 1.3
    A = W.laplacian_1d(n, target)
    c = target / 4.0
    rows = [0, 10, 49]
    Cw, Sw = CF.wave_rows(n, c, t, rows)
    C, S = Wv.reference(A, t)
    assert rel_fro(Cw, C[rows]) <= 1e-12 and rel_fro(Sw, S[rows]) <= 1e-12
    U = CF.unitary_rows(n, c, t, rows)
    assert rel_fro(U, Pr.unitary(A, t)[rows]) <= 1e-12


def test_large_argument_reduction():
    """At n = 4000 the eigenvectors stay orthonormal to rounding (no loss from j k pi / (n + 1))."""
    n = 4000
    lam, V = CF.laplacian_1d_eig(n)
    idx = [0, 1999, 3999]
    G = V[:, idx].T @ V[:, idx]
    assert np.abs(G - np.eye(3)).max() <= 1e-13


@pytest.mark.parametrize("target", [4.0, 64.0])
def test_laplacian_2d_rows_against_reference(target):
    m = 9
    A = W.laplacian_2d(m, target)
    c = target / 8.0
    L = W.laplacian_2d(m, 8.0)
    assert np.array_equal(A, c * L)
    rows = [0, 13, 40, 80]
    C, S = R.sincosm(A)
    assert rel_fro(CF.laplacian_2d_rows(m, c, rows, np.cos), C[rows]) <= 1e-12 * max(1.0, target / 8)
    assert rel_fro(CF.laplacian_2d_rows(m, c, rows, np.sin), S[rows]) <= 1e-12 * max(1.0, target / 8)
