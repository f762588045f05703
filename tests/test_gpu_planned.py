"""sincosm_eval_planned (GPU, through the C ABI): the caller's plan gives bitwise the
results of sincosm_eval for the same plan, the device-side plan check reports and
NaN-fills when the plan does not cover ||A||_1 or A is not finite, and the call is
captured in a HIP graph and replayed with new inputs."""
import math

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


def plan_buffer(torch):
    import paper_2010_00465_amd as sc
    return torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("n,e,dt,acc,prod,ext", [
    (64, -3, "f64", "double", "native", False),
    (300, 4, "f64", "double", "native", False),
    (1000, 10, "f64", "double", "native", False),
    (257, 4, "f32", "single", "native", False),
    (300, 6, "f64", "single", "f32", False),
    (300, 6, "f64", "single", "bf16x3", False),
    (200, -3.25, "f64", "double", "native", True),
])
def test_bitwise_equal_to_eval(env, n, e, dt, acc, prod, ext):
    torch, sc = env
    say("planned vs eval", n, e, dt, acc, prod, ext)
    tdt = torch.float64 if dt == "f64" else torch.float32
    A = torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(120, n))).to(tdt).cuda()
    C0, S0 = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_eval(A, C0, S0, acc, prod, extended=ext)
    C, S = torch.full_like(A, 7.0), torch.full_like(A, 7.0)
    pd = plan_buffer(torch)
    sc.sincosm_eval_planned(A, C, S, plan, acc, prod, plan_dev=pd, extended=ext)
    rec = sc.plan_from_device(pd)
    assert (rec.level, rec.s, rec.products, rec.status) == (plan.level, plan.s, plan.products, 0)
    assert rec.norm1 == plan.norm1
    assert torch.equal(C, C0) and torch.equal(S, S0)


def test_extra_scaling_is_accepted(env):
    """A plan with more double-angle steps than needed still covers A: status OK, results
    near the oracle (each extra step may add about one rounding of growth)."""
    torch, sc = env
    n = 200
    A = W.gaussian(n, 8.0, key=(121,))
    level, s, _ = P.plan(8.0)
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    pd = plan_buffer(torch)
    sc.sincosm_eval_planned(At, C, S, (level, s + 3), plan_dev=pd)
    rec = sc.plan_from_device(pd)
    assert (rec.level, rec.s, rec.status) == (level, s + 3, 0)
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C.cpu().numpy(), Cr) <= 1e-11 and rel_fro(S.cpu().numpy(), Sr) <= 1e-11


@pytest.mark.parametrize("prod,acc,tol", [("native", "double", 1e-13), ("f32", "single", 2e-5),
                                           ("bf16x3", "single", 8 * 7 * 2.0 ** -18)])
def test_extra_scaling_beyond_fold_range(env, prod, acc, tol):
    """A plan with s = 35 on a symmetric A with ||A||_1 = 1: the first product's operand scale
    4^-35 lies outside the range in which a power-of-two scale moves into the epilogue, so
    the product kernels (float64, float32 and split-bf16) scale the staged operands
    themselves. For this A the extra double-angle steps add no error beyond rounding
    (checked on the host with the oracle's schemes), so the bars are those of the
    arithmetic: float64 near u, float32 and bf16x3 at their product error."""
    torch, sc = env
    print("[case] planned s=35", prod, acc, flush=True)
    n = 64
    A = W.symmetric_gaussian(n, 1.0, key=(61,))
    w, V = np.linalg.eigh(A)
    Cr, Sr = (V * np.cos(w)) @ V.T, (V * np.sin(w)) @ V.T
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    pd = plan_buffer(torch)
    sc.sincosm_eval_planned(At, C, S, (7, 35), acc, prod, plan_dev=pd)
    rec = sc.plan_from_device(pd)
    assert (rec.level, rec.s, rec.status) == (7, 35, 0)
    assert rel_fro(C.cpu().numpy(), Cr) <= tol and rel_fro(S.cpu().numpy(), Sr) <= tol


@pytest.mark.parametrize("acc", ["double", "single"])
def test_plan_that_does_not_cover(env, acc):
    """||A||_1 2^-s just above the level's theta: status SINCOSM_E_PLAN, C and S all NaN;
    exactly at theta: covered."""
    torch, sc = env
    n = 96
    th = P.THETA[acc][7]
    for scale, want in ((math.nextafter(th * 4.0, math.inf), -6), (th * 4.0, 0)):
        A = 1e-3 * W.gaussian(n, 1.0, key=(122,))
        A[:, 5] = 0.0
        A[7, 5] = scale                          # the 1-norm is exactly `scale`
        At = torch.from_numpy(A).cuda()
        assert float(At.abs().sum(0).max()) == scale
        C, S = torch.empty_like(At), torch.empty_like(At)
        pd = plan_buffer(torch)
        sc.sincosm_eval_planned(At, C, S, (7, 2), acc, plan_dev=pd)
        rec = sc.plan_from_device(pd)
        assert rec.status == want, (acc, scale, rec)
        if want:
            assert torch.isnan(C).all() and torch.isnan(S).all()
        else:
            assert torch.isfinite(C).all() and torch.isfinite(S).all()


def test_nonfinite_input(env):
    torch, sc = env
    n = 80
    A = torch.from_numpy(W.gaussian(n, 1.0, key=(123,))).cuda()
    A[3, 5] = float("inf")
    C, S = torch.empty_like(A), torch.empty_like(A)
    pd = plan_buffer(torch)
    sc.sincosm_eval_planned(A, C, S, (7, 0), plan_dev=pd)
    rec = sc.plan_from_device(pd)
    assert rec.status == -4
    assert torch.isnan(C).all() and torch.isnan(S).all()


def test_graph_capture_and_replay(env):
    """Capture sincosm_eval_planned (n = 384, plan for ||A||_1 = 16) in a graph; replay it on
    three new inputs of the same norm with eager work between the replays; every replay
    equals the eager call bitwise and the oracle to 1e-12, and updates the plan record."""
    torch, sc = env
    n, target = 384, 16.0
    plan = sc.plan_host(target)
    inputs = [W.gaussian(n, target, key=(124, k)) for k in range(4)]
    A = torch.from_numpy(inputs[0]).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    ws = torch.empty(sc.workspace_size(n, torch.float64), dtype=torch.uint8, device="cuda")
    pd = plan_buffer(torch)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_eval_planned(A, C, S, plan, ws=ws, plan_dev=pd)     # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_eval_planned(A, C, S, plan, ws=ws, plan_dev=pd)
    for k in (1, 2, 3):
        say("graph replay", k)
        A.copy_(torch.from_numpy(inputs[k]).cuda())
        pd.zero_()
        junk = torch.randn(512, 512, device="cuda", dtype=torch.float64)
        junk = junk @ junk                                             # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rec = sc.plan_from_device(pd)
        assert (rec.level, rec.s, rec.status) == (plan.level, plan.s, 0)
        assert rec.norm1 == sc.plan_device(A).norm1      # the library's own fixed-order 1-norm
        Cg, Sg = C.clone(), S.clone()
        Ce, Se = torch.empty_like(A), torch.empty_like(A)
        sc.sincosm_eval_planned(A, Ce, Se, plan, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(Cg, Ce) and torch.equal(Sg, Se)
        Cr, Sr = R.sincosm(inputs[k])
        assert rel_fro(Cg.cpu().numpy(), Cr) <= 1e-12 and rel_fro(Sg.cpu().numpy(), Sr) <= 1e-12


def test_argument_errors(env):
    torch, sc = env
    A = torch.zeros(32, 32, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(A), torch.empty_like(A)
    for bad in ((5, 0), (7, -1), (7, 1101), (1, 0)):
        with pytest.raises(sc.SincosmError):
            sc.sincosm_eval_planned(A, C, S, bad)
    with pytest.raises(ValueError):
        sc.sincosm_eval_planned(A, C, S, (7, 0), plan_dev=torch.zeros(8, dtype=torch.uint8, device="cuda"))
