"""Pins for oracle/propagators.py (eq:unitary and eq:symplectic of Section 1)."""
import cmath
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import propagators as Pr
from tests.conftest import rel_fro


@pytest.mark.parametrize("family", ["gaussian", "symmetric", "laplacian1d"])
@pytest.mark.parametrize("t", [0.4, 3.0, -2.2])
def test_unitary_against_complex_expm(family, t):
    A = W.family(family, 40, 6.0, key=(80, int(10 * t) + 50))
    E = scipy.linalg.expm(-1j * t * A)
    for fn in (Pr.unitary, Pr.unitary_paper):
        assert rel_fro(fn(A, t), E) <= 1e-12


def test_unitarity_for_symmetric():
    A = W.symmetric_gaussian(60, 30.0, key=(81,))
    U = Pr.unitary_paper(A, 1.7)
    assert np.linalg.norm(U @ U.conj().T - np.eye(60)) <= 1e-12 * 60


def test_group_law():
    A = W.gaussian(30, 4.0, key=(82,))
    U1, U2, U12 = Pr.unitary(A, 0.3), Pr.unitary(A, 0.9), Pr.unitary(A, 1.2)
    assert rel_fro(U1 @ U2, U12) <= 1e-12
    E1, E2, E12 = Pr.symplectic(A, 0.3), Pr.symplectic(A, 0.9), Pr.symplectic(A, 1.2)
    assert rel_fro(E1 @ E2, E12) <= 1e-12


@pytest.mark.parametrize("family", ["gaussian", "symmetric", "laplacian1d"])
@pytest.mark.parametrize("t", [0.5, 2.0])
def test_symplectic_against_block_expm(family, t):
    n = 30
    A = W.family(family, n, 9.0, key=(83, int(10 * t)))
    M = np.zeros((2 * n, 2 * n))
    M[:n, n:] = np.eye(n)
    M[n:, :n] = -A
    E = scipy.linalg.expm(t * M)
    for fn in (Pr.symplectic, Pr.symplectic_paper):
        assert rel_fro(fn(A, t), E) <= 1e-12


def test_symplectic_structure_for_symmetric():
    """For symmetric A, M is Hamiltonian, so E = e^{tM} satisfies E^T J E = J."""
    n = 25
    A = W.symmetric_gaussian(n, 5.0, key=(84,))
    E = Pr.symplectic_paper(A, 1.3)
    J = np.zeros((2 * n, 2 * n))
    J[:n, n:] = np.eye(n)
    J[n:, :n] = -np.eye(n)
    assert np.linalg.norm(E.T @ J @ E - J) <= 1e-12 * n


@pytest.mark.parametrize("a", [0.0, 0.3, -1.5, 25.0])
def test_scalar_closed_forms(a):
    t = 0.7
    U = Pr.unitary(np.array([[a]]), t)[0, 0]
    assert abs(U - cmath.exp(-1j * t * a)) <= 1e-15 * max(1.0, abs(t * a))
    E = Pr.symplectic(np.array([[a]]), t)
    if a > 0:
        r = math.sqrt(a)
        want = [[math.cos(t * r), math.sin(t * r) / r], [-r * math.sin(t * r), math.cos(t * r)]]
    elif a < 0:
        r = math.sqrt(-a)
        want = [[math.cosh(t * r), math.sinh(t * r) / r], [r * math.sinh(t * r), math.cosh(t * r)]]
    else:
        want = [[1.0, t], [0.0, 1.0]]
    assert np.allclose(E, want, rtol=1e-14, atol=1e-15)


def test_planted_mistakes_are_caught(monkeypatch):
    """A wrong sign in the assembly of either propagator fails the expm pins."""
    A = W.gaussian(20, 5.0, key=(85,))
    t = 0.9
    n = 20
    M = np.zeros((2 * n, 2 * n))
    M[:n, n:] = np.eye(n)
    M[n:, :n] = -A
    E = scipy.linalg.expm(t * M)
    U = scipy.linalg.expm(-1j * t * A)

    def bad_block(A_, C, S):
        B = np.block([[C, S], [A_ @ S, C]])   # sign of -A s dropped
        return B

    monkeypatch.setattr(Pr, "assemble_block", bad_block)
    assert rel_fro(Pr.symplectic(A, t), E) > 1e-3
    monkeypatch.undo()
    from oracle import reference as R
    orig = R.sincosm
    monkeypatch.setattr(R, "sincosm", lambda X, *a, **k: (orig(X)[0], -orig(X)[1]))  # sin sign flipped
    assert rel_fro(Pr.unitary(A, t), U) > 1e-3
