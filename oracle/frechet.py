"""Derivative references for L(A) = <Gc, cos A> + <Gs, sin A> (oracle, test infrastructure).

The paper does not differentiate its method; these references follow the
standard facts used to check an adjoint:

* Block form: for a power series f, f([[A, E], [0, A]]) = [[f(A), L_f(A, E)],
  [0, f(A)]], where L_f(A, E) is the Frechet derivative of f at A in the
  direction E.
* Adjoint: for a real power series, <G, L_f(A, E)> = <L_f(A^T, G), E>, so
  dL/dA = L_cos(A^T, Gc) + L_sin(A^T, Gs).
* Dual numbers: products of pairs (X, dX)(Z, dZ) = (XZ, X dZ + dX Z) carry the
  directional derivative through any sequence of products and sums.
* Central finite differences (L(A + hE) - L(A - hE)) / 2h.

``block_gradient`` evaluates f on the 2n x 2n block matrix with the
independent ``reference`` algorithm, the direction scaled to the norm of A
and the result divided back. ``dual_gradient`` runs the same Taylor /
double-angle steps as ``reference`` on dual pairs.

Pins (tests/test_oracle_frechet.py): the directional identity
L_cos(A, A) = -A sin A and L_sin(A, A) = A cos A; diagonal A with diagonal E
(derivative = elementwise -sin, cos times E); agreement of block and dual
forms; central finite differences on small matrices.
"""
from __future__ import annotations

import numpy as np

from .reference import norm1, scaling_power, sincosm, taylor_terms

__all__ = ["frechet_block", "block_gradient", "dual_frechet", "dual_gradient",
           "loss", "fd_directional"]


def frechet_block(A: np.ndarray, E: np.ndarray):
    """(L_cos(A, E), L_sin(A, E)) from the 2n x 2n block matrix, float64."""
    A = np.asarray(A, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    n = A.shape[0]
    ne = norm1(E)
    if ne == 0.0:
        z = np.zeros_like(A)
        return z, z.copy()
    tau = max(norm1(A), 1e-3) / ne
    B = np.zeros((2 * n, 2 * n))
    B[:n, :n] = A
    B[n:, n:] = A
    B[:n, n:] = tau * E
    C, S = sincosm(B)
    return C[:n, n:] / tau, S[:n, n:] / tau


def block_gradient(A: np.ndarray, Gc, Gs):
    """dL/dA = L_cos(A^T, Gc) + L_sin(A^T, Gs) via the block form."""
    At = np.asarray(A, dtype=np.float64).T.copy()
    g = np.zeros_like(At)
    if Gc is not None:
        g += frechet_block(At, Gc)[0]
    if Gs is not None:
        g += frechet_block(At, Gs)[1]
    return g


def dual_frechet(A: np.ndarray, E: np.ndarray, m: int = 9):
    """(L_cos(A, E), L_sin(A, E)) by dual-number arithmetic on the reference steps."""
    A = np.asarray(A, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    n = A.shape[0]
    I = np.eye(n)
    Z = np.zeros((n, n))
    s = scaling_power(norm1(A))
    f = 2.0 ** (-s)
    X, dX = A * f, E * f
    Y, dY = X @ X, X @ dX + dX @ X
    cos_c, sin_c = taylor_terms(m)

    def horner(coeffs):
        acc = I * (coeffs[-1].numerator / coeffs[-1].denominator)
        dacc = Z.copy()
        for c in reversed(coeffs[:-1]):
            acc, dacc = (Y @ acc + I * (c.numerator / c.denominator),
                         Y @ dacc + dY @ acc)
        return acc, dacc

    C, dC = horner(cos_c)
    P, dP = horner(sin_c)
    S, dS = X @ P, X @ dP + dX @ P
    for _ in range(s):
        C, dC, S, dS = (I - 2.0 * (S @ S), -2.0 * (S @ dS + dS @ S),
                        2.0 * (S @ C), 2.0 * (S @ dC + dS @ C))
    return dC, dS


def dual_gradient(A: np.ndarray, Gc, Gs):
    """dL/dA via dual numbers at A^T with directions Gc and Gs."""
    At = np.asarray(A, dtype=np.float64).T.copy()
    g = np.zeros_like(At)
    if Gc is not None:
        g += dual_frechet(At, Gc)[0]
    if Gs is not None:
        g += dual_frechet(At, Gs)[1]
    return g


def loss(fn, A, Gc, Gs):
    """<Gc, C> + <Gs, S> for (C, S) = fn(A)."""
    C, S = fn(A)
    out = 0.0
    if Gc is not None:
        out += float(np.sum(Gc * C))
    if Gs is not None:
        out += float(np.sum(Gs * S))
    return out


def fd_directional(fn, A, Gc, Gs, E, h=1e-6):
    """Central difference of the loss along E: (L(A+hE) - L(A-hE)) / 2h."""
    return (loss(fn, A + h * E, Gc, Gs) - loss(fn, A - h * E, Gc, Gs)) / (2 * h)
