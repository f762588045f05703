"""sincosm_eval_planned_noalloc (the entry point that allocates nothing: its workspace is
the library's static device scratch) against sincosm_eval_planned on a caller workspace,
through the C ABI: the same launches, so the results must be bitwise equal; both are also
held to the oracle's 1e-12 (double plan, Section 2.1 schemes and Section 1 double angle).
Two calls in a row, the second on a smaller matrix, so stale contents of the shared
scratch from the first call would show."""
import sys

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


def _pair(env, A_np, dtype, accuracy):
    torch, sc = env
    A = torch.from_numpy(A_np).cuda().to(dtype)
    plan = sc.plan_host(float(A.double().abs().sum(0).max()), accuracy)
    C0, S0 = torch.empty_like(A), torch.empty_like(A)
    C1, S1 = torch.full_like(A, 7.0), torch.full_like(A, 7.0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_eval_planned(A, C0, S0, plan, accuracy)
    sc.sincosm_eval_planned_noalloc(A, C1, S1, plan, accuracy, plan_dev=pd)
    torch.cuda.synchronize()
    rec = sc.plan_from_device(pd)
    assert (rec.level, rec.s, rec.status) == (plan.level, plan.s, 0)
    return A, (C0, S0), (C1, S1), plan


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_matches_planned_two_calls(env, dt):
    torch, sc = env
    dtype = torch.float64 if dt == "f64" else torch.float32
    accuracy = "double" if dt == "f64" else "single"
    tol = 1e-12 if dt == "f64" else 5e-6
    for n, e in [(512 if dt == "f64" else 768, 4.0), (77, 1.0)]:   # the largest order, then a smaller one
        print("[case] noalloc", dt, n, e, flush=True)
        A_np = W.gaussian(n, 2.0 ** e, key=(90, n))
        A, (C0, S0), (C1, S1), plan = _pair(env, A_np, dtype, accuracy)
        assert torch.equal(C0, C1) and torch.equal(S0, S1), (n, plan)
        Cr, Sr = R.sincosm(A.double().cpu().numpy())
        assert rel_fro(C1.double().cpu().numpy(), Cr) <= tol
        assert rel_fro(S1.double().cpu().numpy(), Sr) <= tol


def test_noalloc_rejects_large_and_bad_plan(env):
    torch, sc = env
    A = torch.from_numpy(W.gaussian(1024, 1.0, key=(91,))).cuda()
    C, S = torch.full_like(A, 3.0), torch.full_like(A, 3.0)
    with pytest.raises(sc.SincosmError) as ei:
        sc.sincosm_eval_planned_noalloc(A, C, S, (7, 0))
    assert ei.value.status == sc._lib.E_TOO_LARGE
    torch.cuda.synchronize()
    assert bool((C == 3.0).all()) and bool((S == 3.0).all())   # nothing enqueued
    # a plan that does not cover ||A||_1: NaN outputs and the status in the record
    A = torch.from_numpy(W.gaussian(64, 8.0, key=(92,))).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_eval_planned_noalloc(A, C, S, (7, 0), plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_PLAN
    assert bool(torch.isnan(C).all()) and bool(torch.isnan(S).all())
    # n = 0 is a no-op
    Z = torch.empty(0, 0, dtype=torch.float64, device="cuda")
    sc.sincosm_eval_planned_noalloc(Z, Z.clone(), Z.clone(), (3, 0))


def test_noalloc_graph_capture(env):
    """Captured in a HIP graph and replayed on new inputs with eager work between the
    replays: every replay equals the eager sincosm_eval_planned call bitwise."""
    torch, sc = env
    n = 200
    plan = sc.plan_host(8.0)   # covers ||A||_1 <= 8 with the double table
    A = torch.from_numpy(W.gaussian(n, 4.0, key=(93,))).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_eval_planned_noalloc(A, C, S, plan)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_eval_planned_noalloc(A, C, S, plan)
    for k in range(3):
        print("[case] noalloc graph replay", k, flush=True)
        A.copy_(torch.from_numpy(W.gaussian(n, 2.0 + k, key=(94, k))).cuda())
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        junk = junk @ junk                                             # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Cg, Sg = C.clone(), S.clone()
        Ce, Se = torch.empty_like(A), torch.empty_like(A)
        sc.sincosm_eval_planned(A, Ce, Se, plan)
        torch.cuda.synchronize()
        assert torch.equal(Cg, Ce) and torch.equal(Sg, Se), k
