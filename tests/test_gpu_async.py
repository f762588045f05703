"""sincosm_eval_async and sincosm_backward_async (plan decided on the device, fixed launch
sequence, no read-back) through the C ABI: bitwise equal to sincosm_eval and sincosm_backward,
whose plan is read back first (the launches that do work are the same, with the 2^-s operand
scales resolved on the device);
against the oracle at 1e-12 (double plan, Sections 1 and 2.1, Tables 1-2) and 5e-6 (float32
storage, single plan); the plan record; s_max, non-finite input; HIP-graph capture with no
plan known at capture, replayed on matrices whose plans differ."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import plan as P
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


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def both(env, A, accuracy="double", products="native", s_max=16, extended=False):
    torch, sc = env
    C0, S0 = torch.empty_like(A), torch.empty_like(A)
    p0 = sc.sincosm_eval(A, C0, S0, accuracy, products, extended=extended)
    C1, S1 = torch.full_like(A, 5.0), torch.full_like(A, 5.0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_eval_async(A, C1, S1, s_max, accuracy, products, plan_dev=pd, extended=extended)
    torch.cuda.synchronize()
    return (C0, S0, p0), (C1, S1, sc.plan_from_device(pd))


EXPS = [-9.0, -5.0, -1.0, 0.5, 1.0, 2.0, 5.0, 10.0]


@pytest.mark.parametrize("n", [33, 257, 1000])
@pytest.mark.parametrize("e", EXPS)
def test_async_equals_sync_f64(env, n, e):
    torch, sc = env
    say("async f64", n, e)
    A_np = W.gaussian(n, 2.0 ** e, key=(100, n, int(e * 2) + 40))
    A = torch.from_numpy(A_np).cuda()
    (C0, S0, p0), (C1, S1, p1) = both(env, A)
    assert (p1.level, p1.s, p1.products, p1.status) == (p0.level, p0.s, p0.products, 0)
    assert p1.norm1 == p0.norm1
    assert torch.equal(C0, C1) and torch.equal(S0, S1), (n, e, p0)
    if n <= 257:
        Cr, Sr = R.sincosm(A_np)
        assert rel_fro(C1.cpu().numpy(), Cr) <= 1e-12 and rel_fro(S1.cpu().numpy(), Sr) <= 1e-12


@pytest.mark.parametrize("n,e", [(64, 1.0), (300, 4.0), (777, 8.0)])
def test_async_equals_sync_f32_single(env, n, e):
    torch, sc = env
    say("async f32", n, e)
    A32 = W.gaussian(n, 2.0 ** e, key=(101, n)).astype(np.float32)
    A = torch.from_numpy(A32).cuda()
    (C0, S0, p0), (C1, S1, p1) = both(env, A, "single")
    assert (p1.level, p1.s) == (p0.level, p0.s)
    assert torch.equal(C0, C1) and torch.equal(S0, S1)
    Cr, Sr = R.sincosm(A32.astype(np.float64))
    assert rel_fro(C1.double().cpu().numpy(), Cr) <= 5e-6 and rel_fro(S1.double().cpu().numpy(), Sr) <= 5e-6


@pytest.mark.parametrize("products", ["f32", "bf16x3"])
@pytest.mark.parametrize("e", [-3.0, 6.0])
def test_async_equals_sync_tiers(env, products, e):
    torch, sc = env
    say("async tier", products, e)
    A = torch.from_numpy(W.gaussian(400, 2.0 ** e, key=(102, int(e) + 10))).cuda()
    (C0, S0, p0), (C1, S1, p1) = both(env, A, "single", products)
    assert (p1.level, p1.s) == (p0.level, p0.s)
    assert torch.equal(C0, C1) and torch.equal(S0, S1)


@pytest.mark.parametrize("norm", [0.1, 0.9])
def test_async_extended_plan(env, norm):
    """With the 5-product scheme among the candidates (it wins on (theta_4, theta_5])."""
    torch, sc = env
    A = torch.from_numpy(W.gaussian(200, norm, key=(103, int(norm * 10)))).cuda()
    (C0, S0, p0), (C1, S1, p1) = both(env, A, "double" if norm < 0.5 else "single", extended=True)
    assert (p1.level, p1.s) == (p0.level, p0.s)
    assert torch.equal(C0, C1) and torch.equal(S0, S1)


def test_async_headline_anchor(env):
    """n = 4096, ||A||_1 = 2^10 (level 7, s = 10): 27 of the enqueued launches do work."""
    torch, sc = env
    say("async 4096 e=10")
    A = torch.from_numpy(W.gaussian(4096, 2.0 ** 10, key=(2, 4096, 0, 20))).cuda()
    (C0, S0, p0), (C1, S1, p1) = both(env, A, s_max=12)
    assert (p1.level, p1.s) == (7, 10)
    assert torch.equal(C0, C1) and torch.equal(S0, S1)


def test_async_s_max_and_nonfinite(env):
    torch, sc = env
    A = torch.from_numpy(W.gaussian(50, 2.0 ** 6, key=(104,))).cuda()   # double plan: s = 6
    C, S = torch.empty_like(A), torch.empty_like(A)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_eval_async(A, C, S, 5, plan_dev=pd)
    rec = sc.plan_from_device(pd)
    assert (rec.level, rec.s, rec.status) == (7, 6, sc._lib.E_SCALING)
    assert bool(torch.isnan(C).all()) and bool(torch.isnan(S).all())
    sc.sincosm_eval_async(A, C, S, 6, plan_dev=pd)                   # exactly enough steps
    assert sc.plan_from_device(pd).status == 0
    Cr, Sr = R.sincosm(A.cpu().numpy())
    assert rel_fro(C.cpu().numpy(), Cr) <= 1e-12 and rel_fro(S.cpu().numpy(), Sr) <= 1e-12
    A[3, 4] = float("inf")
    sc.sincosm_eval_async(A, C, S, 8, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_NONFINITE
    assert bool(torch.isnan(C).all()) and bool(torch.isnan(S).all())
    Z = torch.zeros(40, 40, dtype=torch.float64, device="cuda")   # A = 0: C = I, S = 0 exactly
    sc.sincosm_eval_async(Z, C[:40, :40], S[:40, :40], 0)
    assert torch.equal(C[:40, :40], torch.eye(40, dtype=torch.float64, device="cuda"))
    assert not bool(S[:40, :40].any())
    with pytest.raises(sc.SincosmError):
        sc.sincosm_eval_async(A, C, S, -1)
    with pytest.raises(sc.SincosmError):
        sc.sincosm_eval_async(A, C, S, 1101)


def test_async_graph_capture_no_plan(env):
    """Capture once with no plan known; replay on inputs whose plans differ (levels 4, 6, 7 and
    s = 0 .. 8) with eager work between the replays: each replay equals sincosm_eval bitwise."""
    torch, sc = env
    n = 320
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(A), torch.empty_like(A)
    ws = torch.empty(sc.workspace_size(n), dtype=torch.uint8, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_eval_async(A, C, S, 8, ws=ws, plan_dev=pd)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_eval_async(A, C, S, 8, ws=ws, plan_dev=pd)
    seen = set()
    for k, e in enumerate([-5.0, -1.0, 0.5, 3.0, 8.0]):
        say("async graph replay", e)
        A_np = W.gaussian(n, 2.0 ** e, key=(105, k))
        A.copy_(torch.from_numpy(A_np).cuda())
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        junk = junk @ junk                                             # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rec = sc.plan_from_device(pd)
        Ce, Se = torch.empty_like(A), torch.empty_like(A)
        pe = sc.sincosm_eval(A, Ce, Se)
        torch.cuda.synchronize()
        assert (rec.level, rec.s, rec.status) == (pe.level, pe.s, 0)
        assert torch.equal(C, Ce) and torch.equal(S, Se), e
        seen.add((rec.level, rec.s))
    assert len(seen) == 5


# ---------------------------------------------------------------------------
# Reverse pass with the plan decided on the device
# ---------------------------------------------------------------------------
def _grads(env, A, Gc, Gs, s_max):
    torch, sc = env
    At = torch.from_numpy(A).cuda()
    gc = torch.from_numpy(Gc).cuda() if Gc is not None else None
    gs = torch.from_numpy(Gs).cuda() if Gs is not None else None
    g0 = torch.empty_like(At)
    p0 = sc.sincosm_backward(At, gc, gs, g0)
    g1 = torch.full_like(At, 9.0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_backward_async(At, gc, gs, g1, s_max, plan_dev=pd)
    torch.cuda.synchronize()
    return g0, g1, p0, sc.plan_from_device(pd)


@pytest.mark.parametrize("n", [16, 70, 130])
@pytest.mark.parametrize("e", [-9.0, -5.0, -1.0, 1.0, 2.0, 3.0, 7.0])
def test_backward_async_equals_sync(env, n, e):
    """Every level and s = 0 .. 7 (odd and even s: the adjoint pair's starting place)."""
    from oracle import frechet as F
    say("backward async", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(110, n, int(e * 2) + 40))
    g = W.rng(111, n, int(e * 2) + 40)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    g0, g1, p0, p1 = _grads(env, A, Gc, Gs, 8)
    assert (p1.level, p1.s, p1.status) == (p0.level, p0.s, 0)
    import torch
    assert torch.equal(g0, g1), (n, e, p0)
    if n <= 70:
        assert rel_fro(g1.cpu().numpy(), F.dual_gradient(A, Gc, Gs)) <= 1e-12


@pytest.mark.parametrize("which", ["cos", "sin"])
def test_backward_async_one_sided_and_config(env, which):
    import torch
    n = 256
    A = W.gaussian(n, 128.0, key=(4, n, 256))          # the configured n = 256, ||A||_1 = 128 case (s = 7)
    G = W.rng(112).standard_normal((n, n))
    Gc, Gs = (G, None) if which == "cos" else (None, G)
    g0, g1, p0, p1 = _grads(env, A, Gc, Gs, 7)          # exactly enough steps
    assert p1.s == 7 and p1.status == 0
    assert torch.equal(g0, g1)


def test_backward_async_s_max_and_nonfinite(env):
    torch, sc = env
    n = 40
    A = torch.from_numpy(W.gaussian(n, 2.0 ** 6, key=(113,))).cuda()   # s = 6
    G = torch.from_numpy(W.rng(114).standard_normal((n, n))).cuda()
    gA = torch.empty_like(A)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_backward_async(A, G, G, gA, 5, plan_dev=pd)
    rec = sc.plan_from_device(pd)
    assert (rec.s, rec.status) == (6, sc._lib.E_SCALING)
    assert bool(torch.isnan(gA).all())
    A[2, 3] = float("nan")
    sc.sincosm_backward_async(A, G, G, gA, 8, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_NONFINITE
    assert bool(torch.isnan(gA).all())
    with pytest.raises(sc.SincosmError):
        sc.sincosm_backward_async(A, G, G, gA, -1)
    with pytest.raises(sc.SincosmError):
        sc.sincosm_backward_async(A.float(), G.float(), G.float(), gA.float(), 4)


def test_backward_async_graph_capture_no_plan(env):
    """Captured once with no plan known; replayed on inputs whose plans differ: every replay equals
    sincosm_backward bitwise."""
    torch, sc = env
    n = 200
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    Gc = torch.from_numpy(W.rng(115).standard_normal((n, n))).cuda()
    Gs = torch.from_numpy(W.rng(116).standard_normal((n, n))).cuda()
    gA = torch.empty_like(A)
    ws = torch.empty(sc.lib.sincosm_backward_workspace_size(n, 0, 0, 8), dtype=torch.uint8, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_backward_async(A, Gc, Gs, gA, 8, ws=ws, plan_dev=pd)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_backward_async(A, Gc, Gs, gA, 8, ws=ws, plan_dev=pd)
    seen = set()
    for k, e in enumerate([-6.0, -1.0, 1.0, 4.0, 7.0]):
        say("backward async graph replay", e)
        A.copy_(torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(117, k))).cuda())
        junk = torch.randn(128, 128, device="cuda", dtype=torch.float64)
        junk = junk @ junk
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rec = sc.plan_from_device(pd)
        ge = torch.empty_like(A)
        pe = sc.sincosm_backward(A, Gc, Gs, ge)
        torch.cuda.synchronize()
        assert (rec.level, rec.s, rec.status) == (pe.level, pe.s, 0)
        assert torch.equal(gA, ge), e
        seen.add((rec.level, rec.s))
    assert len(seen) == 5
