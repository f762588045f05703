"""Propagators assembled from the matrix cosine and sine (oracle, test infrastructure).

Section 1 of the paper motivates the method with two evolution operators:
* eq:unitary - for real A, the solution operator of i u' = A u is
  U(t) = e^{-itA} = cos(tA) - i sin(tA), formed from the real pair of tA
  (two real products per double-angle step instead of a complex squaring);
* eq:symplectic - the first-order form of y'' + A y = 0 (eq.2a) has
  e^{tM}, M = [[0, I], [-A, 0]], equal to [[c(t^2 A), s(t, A)], [-A s(t, A), c(t^2 A)]].

Each propagator comes in two forms: from the independent Taylor references
(`reference.sincosm`, `wave.reference`) and from the paper's schemes with
their plans (`paper_algorithm.sincosm`, `wave.paper_wave`), in float64.

Pins (tests/test_oracle_propagators.py): scipy's complex matrix exponential
expm(-itA) and its real block exponential expm(tM) (a Pade method, independent
of this code); unitarity of e^{-itA} for symmetric A; the group law
U(t1) U(t2) = U(t1 + t2) and its block analogue; closed forms for 1 x 1 A.
"""
from __future__ import annotations

import numpy as np

from . import paper_algorithm as _pa
from . import reference as _ref
from . import wave as _wave

__all__ = ["unitary", "unitary_paper", "symplectic", "symplectic_paper", "assemble_block"]


def unitary(A: np.ndarray, t: float) -> np.ndarray:
    """e^{-itA} = cos(tA) - i sin(tA) from the Taylor reference of the cos/sin pair (eq:unitary)."""
    X = float(t) * np.asarray(A, dtype=np.float64)
    C, S = _ref.sincosm(X)
    return C - 1j * S


def unitary_paper(A: np.ndarray, t: float, accuracy: str = "double", return_plan=False):
    """e^{-itA} by the paper's cos/sin method on tA (plan on ||tA||_1)."""
    X = float(t) * np.asarray(A, dtype=np.float64)
    C, S, plan = _pa.sincosm(X, accuracy, return_plan=True)
    U = C - 1j * S
    return (U, plan) if return_plan else U


def assemble_block(A: np.ndarray, C: np.ndarray, S: np.ndarray) -> np.ndarray:
    """[[C, S], [-A S, C]] (eq:symplectic) from c(t^2 A) and s(t, A)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    E = np.empty((2 * n, 2 * n))
    E[:n, :n] = C
    E[:n, n:] = S
    E[n:, :n] = -(A @ S)
    E[n:, n:] = C
    return E


def symplectic(A: np.ndarray, t: float) -> np.ndarray:
    """e^{tM}, M = [[0, I], [-A, 0]], from the Taylor reference of c(t^2 A), s(t, A)."""
    C, S = _wave.reference(A, t)
    return assemble_block(A, C, S)


def symplectic_paper(A: np.ndarray, t: float, accuracy: str = "double", return_plan=False):
    """e^{tM} from the Section 2.2 schemes and their plan."""
    C, S, plan = _wave.paper_wave(A, t, accuracy, return_plan=True)
    E = assemble_block(A, C, S)
    return (E, plan) if return_plan else E
