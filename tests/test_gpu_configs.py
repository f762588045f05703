"""Every kernel configuration the autotuner may choose computes the same
products (GPU, through the C ABI): each one is forced with sincosm_tune_set
and checked against float64 numpy with the elementwise bound of the product
kernel; a whole sincosm_eval under each configuration matches the oracle, and
the reverse pass under each configuration matches the default one."""
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
    info = (ctypes.c_int32 * 8)()
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


def force(lib, arith, n, idx):
    """Make every launch of this arithmetic at padded order n use configuration idx
    (all three launch classes); idx = -1 removes the forcing."""
    for code in (arith, arith | 16, arith | 32):
        assert lib.sincosm_tune_set(code, n, n, idx) == 0


@pytest.mark.parametrize("arith", [0, 1])
def test_eval_under_every_config(env, arith):
    """A whole sincosm_eval (scaled first and last scheme products, two-problem double-angle
    launches) under each configuration against the oracle: float64 storage with the double
    plan, float32 storage with the single plan."""
    torch, sc = env
    lib = sc.lib
    n = 512
    A = W.gaussian(n, 40.0, key=(91,))
    Cr, Sr = R.sincosm(A)
    dt, acc = (torch.float64, "double") if arith == 0 else (torch.float32, "single")
    At = torch.from_numpy(A).to(dt).cuda()
    if arith == 1:
        Cr, Sr = R.sincosm(At.cpu().double().numpy())
    try:
        for idx, bm, bn in configs(lib, arith):
            print("[case] eval config", arith, idx, bm, bn, flush=True)
            force(lib, arith, n, idx)
            C = torch.empty_like(At)
            S = torch.empty_like(At)
            plan = sc.sincosm_eval(At, C, S, acc)
            torch.cuda.synchronize()
            assert plan.s > 0
            tol = 1e-12 if arith == 0 else 5e-6
            ec = rel_fro(C.cpu().double().numpy(), Cr)
            es = rel_fro(S.cpu().double().numpy(), Sr)
            assert ec <= tol and es <= tol, (idx, ec, es)
    finally:
        force(lib, arith, n, -1)
        sc._autotune.apply_cache()


def test_backward_under_every_config(env):
    """The reverse pass (launches with up to 3 + 1 k-segments and operand scales) under each
    float64 configuration agrees with the default configuration's gradient."""
    torch, sc = env
    lib = sc.lib
    n = 256
    A = torch.from_numpy(W.gaussian(n, 8.0, key=(92,))).cuda()
    g = W.rng(93)
    Gc = torch.from_numpy(g.standard_normal((n, n))).cuda()
    Gs = torch.from_numpy(g.standard_normal((n, n))).cuda()
    ref = torch.empty_like(A)
    sc.sincosm_backward(A, Gc, Gs, ref)
    torch.cuda.synchronize()
    try:
        for idx, bm, bn in configs(lib, 0):
            print("[case] backward config", idx, bm, bn, flush=True)
            force(lib, 0, n, idx)
            gA = torch.empty_like(A)
            sc.sincosm_backward(A, Gc, Gs, gA)
            torch.cuda.synchronize()
            err = float((gA - ref).norm() / ref.norm())
            assert err <= 1e-13, (idx, err)
    finally:
        force(lib, 0, n, -1)
        sc._autotune.apply_cache()
