"""Pins for oracle/frechet.py: closed-form directional derivatives, the diagonal
case, block vs dual agreement, and central finite differences."""
import numpy as np
import pytest

import workloads as W
from oracle import frechet as F
from oracle import reference as R
from tests.conftest import rel_fro


@pytest.mark.parametrize("e", [-3, 0, 3, 6])
def test_directional_identity(e):
    """d/dt f(A + tA) at 0 = A f'(A): L_cos(A, A) = -A sin A, L_sin(A, A) = A cos A."""
    A = W.gaussian(24, 2.0 ** e, key=(31, e + 10))
    C, S = R.sincosm(A)
    for fn in (F.frechet_block, F.dual_frechet):
        Lc, Ls = fn(A, A)
        assert rel_fro(Lc, -A @ S) <= 1e-11
        assert rel_fro(Ls, A @ C) <= 1e-11


def test_diagonal_elementwise():
    d = np.array([0.3, -1.2, 2.5, 0.01, 5.0])
    e = np.array([1.0, -0.5, 0.25, 2.0, -1.0])
    for fn in (F.frechet_block, F.dual_frechet):
        Lc, Ls = fn(np.diag(d), np.diag(e))
        assert np.allclose(np.diag(Lc), -np.sin(d) * e, rtol=0, atol=1e-13)
        assert np.allclose(np.diag(Ls), np.cos(d) * e, rtol=0, atol=1e-13)


@pytest.mark.parametrize("e", [-1, 3, 7])
def test_block_vs_dual(e):
    A = W.gaussian(20, 2.0 ** e, key=(32, e + 10))
    g = W.rng(33, e + 10)
    Gc, Gs = g.standard_normal((20, 20)), g.standard_normal((20, 20))
    gb = F.block_gradient(A, Gc, Gs)
    gd = F.dual_gradient(A, Gc, Gs)
    assert rel_fro(gb, gd) <= 1e-10


@pytest.mark.parametrize("e", [-1, 3])
def test_fd(e):
    n = 12
    A = W.gaussian(n, 2.0 ** e, key=(34, e + 10))
    g = W.rng(35, e + 10)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    grad = F.dual_gradient(A, Gc, Gs)
    for i in range(3):
        E = g.standard_normal((n, n))
        E /= np.linalg.norm(E)
        fd = F.fd_directional(R.sincosm, A, Gc, Gs, E, h=1e-6)
        an = float(np.sum(grad * E))
        scale = np.linalg.norm(grad)
        assert abs(fd - an) <= 1e-6 * max(scale, 1.0)


def test_adjoint_identity_transpose():
    """<G, L_f(A, E)> = <L_f(A^T, G), E> checked numerically."""
    n = 10
    A = W.gaussian(n, 3.0, key=(36,))
    g = W.rng(37)
    G, E = g.standard_normal((n, n)), g.standard_normal((n, n))
    Lc, Ls = F.dual_frechet(A, E)
    Lc_t, Ls_t = F.dual_frechet(A.T.copy(), G)
    assert abs(np.sum(G * Lc) - np.sum(Lc_t * E)) <= 1e-11 * np.linalg.norm(G) * np.linalg.norm(Lc)
    assert abs(np.sum(G * Ls) - np.sum(Ls_t * E)) <= 1e-11 * np.linalg.norm(G) * np.linalg.norm(Ls)
