"""Every kernel configuration the autotuner may choose computes the same
products (GPU, through the C ABI): each one is forced with sincosm_tune_set
and checked against float64 numpy with the elementwise bound of the product
kernel, and a whole sincosm_eval under a non-default configuration matches
the oracle."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import reference as R
from tests.conftest import rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_00465_amd as sc
    return torch, sc


def configs(lib, arith):
    out = []
    info = (ctypes.c_int32 * 7)()
    for i in range(lib.sincosm_tune_num_configs(arith)):
        lib.sincosm_tune_config_info(arith, i, info)
        out.append((i, info[0], info[1]))
    return out


@pytest.mark.parametrize("arith,dt", [(0, "f64"), (1, "f32")])
def test_every_config_matmul(env, arith, dt):
    torch, sc = env
    lib = sc.lib
    n = 512                      # padded to 512: divisible by every tile of the table
    tdt = torch.float64 if dt == "f64" else torch.float32
    g = W.rng(90, arith)
    X = torch.from_numpy(g.standard_normal((n, n))).to(tdt).cuda()
    Y = torch.from_numpy(g.standard_normal((n, n))).to(tdt).cuda()
    Xd, Yd = X.cpu().double().numpy(), Y.cpu().double().numpy()
    ref = Xd @ Yd
    bound = np.abs(Xd) @ np.abs(Yd)
    u = 2.0 ** -53 if dt == "f64" else 2.0 ** -24
    try:
        for idx, bm, bn in configs(lib, arith):
            print("[case] config", arith, idx, bm, bn, flush=True)
            assert lib.sincosm_tune_set(arith, n, n, idx) == 0
            Z = torch.empty_like(X)
            sc.sincosm_matmul(X, Y, Z)
            torch.cuda.synchronize()
            err = np.max(np.abs(Z.cpu().double().numpy() - ref) / bound)
            assert err <= 2 * n * u, (idx, err)
    finally:
        lib.sincosm_tune_set(arith, n, n, -1)
        sc._autotune.apply_cache()


def test_eval_under_forced_config(env):
    torch, sc = env
    lib = sc.lib
    n = 512
    A = W.gaussian(n, 40.0, key=(91,))
    Cr, Sr = R.sincosm(A)
    At = torch.from_numpy(A).cuda()
    try:
        for idx in (5, 6, 7):
            lib.sincosm_tune_set(0, n, n, idx)
            C = torch.empty_like(At)
            S = torch.empty_like(At)
            sc.sincosm_eval(At, C, S)
            torch.cuda.synchronize()
            assert rel_fro(C.cpu().numpy(), Cr) <= 1e-12 and rel_fro(S.cpu().numpy(), Sr) <= 1e-12
    finally:
        lib.sincosm_tune_set(0, n, n, -1)
        sc._autotune.apply_cache()
