"""Seeded synthetic input matrices for the matrix cosine/sine workloads.

This module only draws and rescales random matrices. It holds none of the
matrix-function arithmetic: the product path and the CPU oracle both take
their inputs from here and from nowhere else.

Every generator is deterministic in its seed key. Matrices are generated in
float64, row-major, and rescaled so that their 1-norm (maximum absolute
column sum, computed with ``numpy.linalg.norm(., 1)``) equals the requested
target. Float32 variants are produced by casting the float64 matrix.

The families follow the test sets of the paper's numerical experiments
(Section 4: normally and uniformly distributed random matrices, triangular
nilpotent matrices, and the 2x2 matrices [[1, lam], [0, -1]]) and the
wave-equation motivation of Section 1 (scaled discrete Laplacians). The
MATLAB gallery matrices of Section 4 are not available; these families
stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "rescale",
    "gaussian",
    "symmetric_gaussian",
    "uniform",
    "laplacian_1d",
    "laplacian_2d",
    "nilpotent_upper",
    "overscale_2x2",
    "headline_anchor_exponents",
    "log_uniform_exponents",
    "batched_sizes",
    "batched_gaussian",
    "family",
]


def rng(*key: int) -> np.random.Generator:
    """A numpy Generator seeded by an integer key tuple."""
    return np.random.default_rng([int(k) for k in key])


def rescale(G: np.ndarray, target_norm1: float) -> np.ndarray:
    """Return G * (target / ||G||_1); G is returned unchanged when it is zero."""
    nrm = float(np.linalg.norm(G, 1)) if G.size else 0.0
    if nrm == 0.0:
        return G.copy()
    return G * (float(target_norm1) / nrm)


def gaussian(n: int, target_norm1: float, key=(0,)) -> np.ndarray:
    """n x n matrix with i.i.d. N(0,1) entries, rescaled to the target 1-norm."""
    G = rng(*key).standard_normal((n, n))
    return rescale(G, target_norm1)


def symmetric_gaussian(n: int, target_norm1: float, key=(0,)) -> np.ndarray:
    """(G + G^T)/2 for Gaussian G, rescaled to the target 1-norm."""
    G = rng(*key).standard_normal((n, n))
    return rescale(0.5 * (G + G.T), target_norm1)


def uniform(n: int, target_norm1: float, key=(0,), lo=0.0, hi=1.0) -> np.ndarray:
    """n x n matrix with i.i.d. U(lo, hi) entries, rescaled to the target 1-norm."""
    G = rng(*key).uniform(lo, hi, size=(n, n))
    return rescale(G, target_norm1)


def _tridiag(n: int) -> np.ndarray:
    T = 2.0 * np.eye(n)
    if n > 1:
        i = np.arange(n - 1)
        T[i, i + 1] = -1.0
        T[i + 1, i] = -1.0
    return T


def laplacian_1d(n: int, target_norm1: float) -> np.ndarray:
    """t^2 * tridiag(-1, 2, -1)/h^2 stored dense, rescaled to the target 1-norm.

    The scale factor t^2/h^2 is absorbed into the rescaling; the matrix is the
    wave-equation operator of Section 1 for a 1-D grid.
    """
    return rescale(_tridiag(n), target_norm1)


def laplacian_2d(m: int, target_norm1: float) -> np.ndarray:
    """2-D 5-point Laplacian on an m x m grid, (I (x) T + T (x) I), dense, n = m^2."""
    T = _tridiag(m)
    I = np.eye(m)
    L = np.kron(I, T) + np.kron(T, I)
    return rescale(L, target_norm1)


def nilpotent_upper(n: int, key=(0,), integer=True, rank_band=None) -> np.ndarray:
    """Strictly upper-triangular (hence nilpotent) matrix.

    With ``integer=True`` the entries are small integers in [-3, 3], so every
    power of the matrix is exact in float64 for the sizes used in tests.
    ``rank_band`` limits the nonzeros to the first ``rank_band`` superdiagonals
    (a banded nilpotent matrix as built by spdiags in the paper's Section 4).
    """
    g = rng(*key)
    if integer:
        M = g.integers(-3, 4, size=(n, n)).astype(np.float64)
    else:
        M = g.standard_normal((n, n))
    M = np.triu(M, 1)
    if rank_band is not None:
        M = np.triu(M, 1) - np.triu(M, 1 + int(rank_band))
    return M


def overscale_2x2(lam: float) -> np.ndarray:
    """The matrix [[1, lam], [0, -1]] of Section 4 (overscaling family)."""
    return np.array([[1.0, float(lam)], [0.0, -1.0]])


def headline_anchor_exponents():
    """1-norm exponents e of the fixed anchors, ||A||_1 = 2^e."""
    return (-4, 0, 4, 10)


def log_uniform_exponents(count: int, lo: float, hi: float, key=(0,)) -> np.ndarray:
    """``count`` exponents drawn uniformly in [lo, hi] (so 2^e is log-uniform)."""
    return rng(*key).uniform(lo, hi, size=count)


def batched_sizes(count: int, key=(3, 0), sizes=tuple(range(8, 257, 4))) -> np.ndarray:
    """Matrix orders drawn uniformly from ``sizes`` (default {8, 12, ..., 256})."""
    g = rng(*key)
    return np.asarray(sizes, dtype=np.int64)[g.integers(0, len(sizes), size=count)]


def batched_gaussian(count: int, key=(3,), lo_exp=-6.0, hi_exp=8.0, sizes=None,
                     dtype=np.float64):
    """A packed batch of Gaussian matrices of uneven order.

    Returns ``(ns, offsets, packed, norms)``: the orders, element offsets of
    each matrix in ``packed`` (row-major, leading dimension n), the packed
    values, and the target 1-norms 2^e with e ~ U(lo_exp, hi_exp).
    """
    ns = batched_sizes(count, key=tuple(key) + (0,)) if sizes is None else np.asarray(sizes, np.int64)
    count = len(ns)
    exps = log_uniform_exponents(count, lo_exp, hi_exp, key=tuple(key) + (1,))
    norms = np.exp2(exps)
    offsets = np.zeros(count, dtype=np.int64)
    if count:
        offsets[1:] = np.cumsum(ns[:-1] ** 2)
    total = int((ns ** 2).sum())
    packed = np.empty(total, dtype=dtype)
    g = rng(*(tuple(key) + (2,)))
    for i, (n, off) in enumerate(zip(ns, offsets)):
        n = int(n)
        G = g.standard_normal((n, n))
        packed[off:off + n * n] = rescale(G, norms[i]).astype(dtype).ravel()
    return ns, offsets, packed, norms


def family(name: str, n: int, target_norm1: float, key=(0,)) -> np.ndarray:
    """Dispatch by family name: gaussian, symmetric, laplacian1d."""
    if name == "gaussian":
        return gaussian(n, target_norm1, key)
    if name == "symmetric":
        return symmetric_gaussian(n, target_norm1, key)
    if name == "laplacian1d":
        return laplacian_1d(n, target_norm1)
    raise ValueError(f"unknown family {name!r}")
