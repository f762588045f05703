"""Closed forms for the 1-D Laplacian family (oracle, test infrastructure).

The wave-equation family of Section 1 (and of the test workloads) is
A = c T with T = tridiag(-1, 2, -1) of order n. T has the eigenvalues
lambda_k = 2 - 2 cos(k pi / (n + 1)) = 4 sin^2(k pi / (2 (n + 1))) and the
orthonormal eigenvectors v_k(j) = sqrt(2 / (n + 1)) sin(j k pi / (n + 1)),
j, k = 1..n (the discrete sine transform). Every matrix function is then
f(A) = V f(c Lambda) V^T, so selected rows of cos A, sin A, c(t^2 A), s(t, A)
and e^{-itA} can be formed exactly (to rounding) at any order, including the
full sizes where no general-purpose oracle finishes in seconds.

Accuracy: the sine arguments j k pi / (n + 1) are reduced exactly with
integer arithmetic (j k mod 2 (n + 1)) before the multiplication by pi, and
lambda_k uses the 4 sin^2 form, so no entry loses accuracy to cancellation or
to large arguments.

The 2-D 5-point Laplacian on an m x m grid, L = I (x) T + T (x) I (n = m^2),
has the eigenvectors v_i (x) v_j with eigenvalues lambda_i + lambda_j, so a
row (a, b) of f(c L) is sum_i v_i(a) v_i (x) [sum_j f(c (lambda_i + lambda_j))
v_j(b) v_j], O(m^3) per row.

Pins (tests/test_oracle_closed_forms.py): eigenpairs against numpy's eigh and
T V = V Lambda; rows of cos/sin against the Taylor reference; the wave and
unitary rows against their oracles; 2-D rows against the Taylor reference.
"""
from __future__ import annotations

import numpy as np

__all__ = ["laplacian_1d_eig", "function_rows", "sincos_rows", "wave_rows", "unitary_rows",
           "laplacian_2d_rows"]


def laplacian_1d_eig(n: int, c: float = 1.0):
    """(lam, V): eigenvalues of c T (ascending) and the orthonormal eigenvectors as columns."""
    k = np.arange(1, n + 1, dtype=np.int64)
    lam = 4.0 * np.sin(k * (np.pi / (2 * (n + 1)))) ** 2 * float(c)
    jk = np.outer(k, k) % (2 * (n + 1))          # exact argument reduction
    V = np.sqrt(2.0 / (n + 1)) * np.sin(jk * (np.pi / (n + 1)))
    return lam, V


def function_rows(n: int, c: float, rows, f) -> np.ndarray:
    """Rows `rows` of f(c T) = V diag(f(lam)) V^T (f applied to the eigenvalue vector)."""
    lam, V = laplacian_1d_eig(n, c)
    rows = np.asarray(rows, dtype=np.int64)
    return (V[rows] * f(lam)) @ V.T


def sincos_rows(n: int, c: float, rows):
    """Rows of cos(c T) and sin(c T)."""
    lam, V = laplacian_1d_eig(n, c)
    rows = np.asarray(rows, dtype=np.int64)
    Vr = V[rows]
    return (Vr * np.cos(lam)) @ V.T, (Vr * np.sin(lam)) @ V.T


def wave_rows(n: int, c: float, t: float, rows):
    """Rows of c(t^2 A) = cos(t sqrt A) and s(t, A) = sin(t sqrt A) / sqrt A for A = c T (SPD)."""
    lam, V = laplacian_1d_eig(n, c)
    r = np.sqrt(lam)
    rows = np.asarray(rows, dtype=np.int64)
    Vr = V[rows]
    return (Vr * np.cos(t * r)) @ V.T, (Vr * (np.sin(t * r) / r)) @ V.T


def unitary_rows(n: int, c: float, t: float, rows):
    """Rows of e^{-itA} for A = c T."""
    lam, V = laplacian_1d_eig(n, c)
    rows = np.asarray(rows, dtype=np.int64)
    Vr = V[rows]
    return ((Vr * np.cos(t * lam)) @ V.T) - 1j * ((Vr * np.sin(t * lam)) @ V.T)


def laplacian_2d_rows(m: int, c: float, rows, f) -> np.ndarray:
    """Rows (flattened grid index a m + b) of f(c (I (x) T + T (x) I)) for an m x m grid."""
    lam, V = laplacian_1d_eig(m)
    F = f(float(c) * (lam[:, None] + lam[None, :]))          # F[i, j] = f(c (lam_i + lam_j))
    out = np.empty((len(rows), m * m), dtype=np.result_type(F, V))
    for k, r in enumerate(rows):
        a, b = divmod(int(r), m)
        Wb = (F * V[b, :][None, :]) @ V.T                     # [i, b'] = sum_j F_ij v_j(b) v_j(b')
        out[k] = ((V * V[a, :][None, :]) @ Wb).ravel()        # [a', b'] = sum_i v_i(a) v_i(a') Wb[i, b']
    return out
