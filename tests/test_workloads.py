"""Input generators: deterministic, correctly rescaled, right structure."""
import numpy as np

import workloads as W


def test_deterministic_and_norm():
    A = W.gaussian(50, 3.5, key=(1, 2))
    B = W.gaussian(50, 3.5, key=(1, 2))
    assert np.array_equal(A, B)
    assert abs(np.abs(A).sum(axis=0).max() - 3.5) <= 1e-14 * 3.5


def test_families():
    S = W.symmetric_gaussian(20, 2.0, key=(3,))
    assert np.array_equal(S, S.T)
    L = W.laplacian_1d(16, 8.0)
    assert np.count_nonzero(np.triu(L, 2)) == 0 and abs(np.abs(L).sum(0).max() - 8.0) < 1e-14
    L2 = W.laplacian_2d(8, 64.0)
    assert L2.shape == (64, 64) and abs(np.abs(L2).sum(0).max() - 64.0) < 1e-12
    N = W.nilpotent_upper(9, key=(4,))
    assert np.count_nonzero(np.tril(N)) == 0


def test_batched_layout():
    ns, offs, packed, norms = W.batched_gaussian(30, key=(9,))
    assert len(ns) == 30 and set(ns.tolist()) <= set(range(8, 257, 4))
    assert offs[0] == 0 and packed.size == int((ns ** 2).sum())
    for n, o, t in zip(ns, offs, norms):
        A = packed[o:o + n * n].reshape(n, n)
        assert abs(np.abs(A).sum(0).max() - t) <= 1e-13 * t
