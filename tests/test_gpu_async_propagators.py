"""sincosm_wave_eval_async, sincosm_wave_block_eval_async and sincosm_expi_eval_async (plan decided
on the device, fixed launch sequence, no read-back) through the C ABI.

expi: bitwise equal to sincosm_expi_eval (the same products as sincosm_eval_async on tA, then
U = C - i S).
wave: C bitwise equal to sincosm_wave_eval (B_s = 4^-s t^2 A formed exactly instead of through
operand scales and coefficients); S carried as s / t_s through the steps (Section 1's step
s(2t, A) = 2 s(t, A) c(t^2 A) in those units has coefficient 1) and multiplied by t at the end,
so S differs from the synchronous call by rounding only: both are held to the oracle's bar
(1e-12 relative, the Section 2.2 schemes with the same plan) and to each other at 1e-13.
Also: the plan record, s_max and non-finite input, float32 storage at the single bar 5e-6,
and HIP-graph capture with no plan known at capture, replayed on inputs whose plans differ."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import plan as P
from oracle import propagators as Pr
from oracle import wave as Wv
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


def wave_both(env, A, t, accuracy="double", products="native", s_max=8):
    torch, sc = env
    C0, S0 = torch.empty_like(A), torch.empty_like(A)
    p0 = sc.sincosm_wave_eval(A, t, C0, S0, accuracy, products)
    C1, S1 = torch.full_like(A, 5.0), torch.full_like(A, 5.0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_wave_eval_async(A, t, C1, S1, s_max, accuracy, products, plan_dev=pd)
    torch.cuda.synchronize()
    return (C0, S0, p0), (C1, S1, sc.plan_from_device(pd))


def np64(x):
    return x.double().cpu().numpy()


B_EXPS = [-9, -7, -2, 1, 4, 8, 12]


@pytest.mark.parametrize("n", [33, 257])
@pytest.mark.parametrize("e", B_EXPS)
def test_wave_async_vs_sync_and_oracle(env, n, e):
    """||t^2 A||_1 = 2^e: wave levels 2, 3, 4, 5 and s = 0 .. 6."""
    torch, sc = env
    say("wave async", n, e)
    t = 1.3
    A_np = W.gaussian(n, 2.0 ** e / (t * t), key=(160, n, e + 20))
    A = torch.from_numpy(A_np).cuda()
    (C0, S0, p0), (C1, S1, p1) = wave_both(env, A, t)
    assert (p1.level, p1.s, p1.products, p1.status) == (p0.level, p0.s, p0.products, 0)
    assert p1.norm1 == p0.norm1
    assert torch.equal(C0, C1), (n, e, p0)
    d = rel_fro(np64(S1), np64(S0))
    say("wave async S vs sync", d)
    assert d <= 1e-13
    Cp, Sp = Wv.paper_wave(A_np, t)
    assert rel_fro(np64(C1), Cp) <= 1e-12 and rel_fro(np64(S1), Sp) <= 1e-12


def test_wave_async_every_level(env):
    torch, sc = env
    seen = set()
    for e in B_EXPS:
        A = torch.from_numpy(W.gaussian(40, 2.0 ** e, key=(161, e + 20))).cuda()
        _, (_, _, p1) = wave_both(env, A, 1.0)
        seen.add(p1.level)
    assert seen == {2, 3, 4, 5}


@pytest.mark.parametrize("n,e", [(1000, 6), (1536, 10)])
def test_wave_async_larger_n(env, n, e):
    torch, sc = env
    say("wave async large", n, e)
    t = 0.7
    A_np = W.gaussian(n, 2.0 ** e / (t * t), key=(162, n))
    A = torch.from_numpy(A_np).cuda()
    (C0, S0, p0), (C1, S1, p1) = wave_both(env, A, t)
    assert (p1.level, p1.s) == (p0.level, p0.s)
    assert torch.equal(C0, C1)
    assert rel_fro(np64(S1), np64(S0)) <= 1e-13
    Cp, Sp = Wv.paper_wave(A_np, t)
    assert rel_fro(np64(C1), Cp) <= 1e-12 and rel_fro(np64(S1), Sp) <= 1e-12


def test_wave_async_t_zero_negative_t(env):
    torch, sc = env
    A = torch.from_numpy(W.gaussian(48, 50.0, key=(163,))).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    sc.sincosm_wave_eval_async(A, 0.0, C, S, 0)
    assert torch.equal(C, torch.eye(48, dtype=torch.float64, device="cuda"))
    assert not bool(S.any())
    Cn, Sn = torch.empty_like(A), torch.empty_like(A)
    sc.sincosm_wave_eval_async(A, 0.9, C, S, 8)
    sc.sincosm_wave_eval_async(A, -0.9, Cn, Sn, 8)
    assert torch.equal(C, Cn) and torch.equal(S, -Sn)


@pytest.mark.parametrize("n,e", [(64, 1), (300, 7)])
def test_wave_async_float32_single(env, n, e):
    torch, sc = env
    say("wave async f32", n, e)
    t = 0.8
    A32 = W.gaussian(n, 2.0 ** e / (t * t), key=(164, n)).astype(np.float32)
    A = torch.from_numpy(A32).cuda()
    (C0, S0, p0), (C1, S1, p1) = wave_both(env, A, t, "single")
    assert (p1.level, p1.s) == (p0.level, p0.s)
    assert torch.equal(C0, C1)
    Cp, Sp = Wv.paper_wave(A32.astype(np.float64), t, "single")
    assert rel_fro(np64(C1), Cp) <= 5e-6 and rel_fro(np64(S1), Sp) <= 5e-6


@pytest.mark.parametrize("products", ["f32", "bf16x3"])
def test_wave_async_tiers(env, products):
    """Lower-precision products on float64 data: same plan as the synchronous call, results within
    the sync result's own distance from the oracle."""
    torch, sc = env
    say("wave async tier", products)
    t = 1.1
    A_np = W.gaussian(300, 2.0 ** 6 / (t * t), key=(165,))
    A = torch.from_numpy(A_np).cuda()
    (C0, S0, p0), (C1, S1, p1) = wave_both(env, A, t, "single", products)
    assert (p1.level, p1.s) == (p0.level, p0.s)
    Cp, Sp = Wv.paper_wave(A_np, t, "single")
    for X1, X0, Xp in ((C1, C0, Cp), (S1, S0, Sp)):
        e1, e0 = rel_fro(np64(X1), Xp), rel_fro(np64(X0), Xp)
        say("tier", products, e1, e0)
        assert e1 <= 2.0 * e0 + 1e-14


def test_wave_async_s_max_and_nonfinite(env):
    torch, sc = env
    t = 1.0
    A = torch.from_numpy(W.gaussian(50, 2.0 ** 8, key=(166,))).cuda()   # wave double plan: s = 4
    p = sc.wave_plan_host(float(A.abs().sum(0).max()))
    C, S = torch.empty_like(A), torch.empty_like(A)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_wave_eval_async(A, t, C, S, p.s - 1, plan_dev=pd)
    rec = sc.plan_from_device(pd)
    assert (rec.level, rec.s, rec.status) == (p.level, p.s, sc._lib.E_SCALING)
    assert bool(torch.isnan(C).all()) and bool(torch.isnan(S).all())
    sc.sincosm_wave_eval_async(A, t, C, S, p.s, plan_dev=pd)             # exactly enough steps
    assert sc.plan_from_device(pd).status == 0
    Cp, Sp = Wv.paper_wave(A.cpu().numpy(), t)
    assert rel_fro(np64(C), Cp) <= 1e-12 and rel_fro(np64(S), Sp) <= 1e-12
    A[1, 2] = float("nan")
    sc.sincosm_wave_eval_async(A, t, C, S, 8, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_NONFINITE
    assert bool(torch.isnan(C).all()) and bool(torch.isnan(S).all())
    with pytest.raises(sc.SincosmError):
        sc.sincosm_wave_eval_async(A, t, C, S, -1)
    with pytest.raises(sc.SincosmError):
        sc.sincosm_wave_eval_async(A, float("inf"), C, S, 4)


def test_wave_async_graph_capture_no_plan(env):
    """Captured once with no plan known; replayed on inputs whose wave plans differ (levels and s)
    with eager work between the replays: C equals sincosm_wave_eval bitwise, S to 1e-13."""
    torch, sc = env
    n = 200
    t = 0.9
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(A), torch.empty_like(A)
    ws = torch.empty(sc.workspace_size(n), dtype=torch.uint8, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_wave_eval_async(A, t, C, S, 8, ws=ws, plan_dev=pd)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_wave_eval_async(A, t, C, S, 8, ws=ws, plan_dev=pd)
    seen = set()
    for k, e in enumerate([-8, -2, 1, 5, 11]):
        say("wave async graph replay", e)
        A.copy_(torch.from_numpy(W.gaussian(n, 2.0 ** e / (t * t), key=(167, k))).cuda())
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        junk = junk @ junk                                             # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rec = sc.plan_from_device(pd)
        Ce, Se = torch.empty_like(A), torch.empty_like(A)
        pe = sc.sincosm_wave_eval(A, t, Ce, Se)
        torch.cuda.synchronize()
        assert (rec.level, rec.s, rec.status) == (pe.level, pe.s, 0)
        assert torch.equal(C, Ce), e
        assert rel_fro(np64(S), np64(Se)) <= 1e-13
        seen.add((rec.level, rec.s))
    assert len(seen) == 5


# ---------------------------------------------------------------------------
# e^{tM}, M = [[0, I], [-A, 0]]
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [33, 257])
@pytest.mark.parametrize("e", [-8, -2, 1, 4, 8, 11])
def test_wave_block_async(env, n, e):
    """Odd and even s (the pair is moved to fixed buffers on the device before the last product)."""
    torch, sc = env
    say("block async", n, e)
    t = 1.3
    A_np = W.gaussian(n, 2.0 ** e / (t * t), key=(168, n, e + 20))
    A = torch.from_numpy(A_np).cuda()
    E0 = torch.empty(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    p0 = sc.sincosm_wave_block_eval(A, t, E0)
    E1 = torch.full_like(E0, 7.0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_wave_block_eval_async(A, t, E1, 8, plan_dev=pd)
    torch.cuda.synchronize()
    p1 = sc.plan_from_device(pd)
    assert (p1.level, p1.s, p1.status) == (p0.level, p0.s, 0)
    assert torch.equal(E1[:n, :n], E0[:n, :n]) and torch.equal(E1[n:, n:], E0[n:, n:])
    assert rel_fro(np64(E1), np64(E0)) <= 1e-13
    assert rel_fro(np64(E1), Pr.symplectic_paper(A_np, t)) <= 1e-12


def test_wave_block_async_failures(env):
    torch, sc = env
    n = 30
    A = torch.from_numpy(W.gaussian(n, 2.0 ** 9, key=(169,))).cuda()
    p = sc.wave_plan_host(float(A.abs().sum(0).max()))
    E = torch.empty(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_wave_block_eval_async(A, 1.0, E, p.s - 1, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_SCALING
    assert bool(torch.isnan(E).all())
    sc.sincosm_wave_block_eval_async(A, 1.0, E, p.s, plan_dev=pd)
    assert sc.plan_from_device(pd).status == 0
    assert rel_fro(np64(E), Pr.symplectic_paper(A.cpu().numpy(), 1.0)) <= 1e-12
    A[0, 0] = float("inf")
    sc.sincosm_wave_block_eval_async(A, 1.0, E, 8, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_NONFINITE
    assert bool(torch.isnan(E).all())


# ---------------------------------------------------------------------------
# e^{-itA}
# ---------------------------------------------------------------------------
def expi_both(env, A, t, accuracy="double", products="native", s_max=16):
    torch, sc = env
    ct = torch.complex128 if A.dtype == torch.float64 else torch.complex64
    U0 = torch.empty(A.shape, dtype=ct, device="cuda")
    p0 = sc.sincosm_expi_eval(A, t, U0, accuracy, products)
    U1 = torch.full(A.shape, 3.0, dtype=ct, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_expi_eval_async(A, t, U1, s_max, accuracy, products, plan_dev=pd)
    torch.cuda.synchronize()
    return (U0, p0), (U1, sc.plan_from_device(pd))


@pytest.mark.parametrize("n", [33, 257])
@pytest.mark.parametrize("e", [-6, -1, 1, 5, 9])
def test_expi_async_equals_sync(env, n, e):
    torch, sc = env
    say("expi async", n, e)
    t = 0.75
    A_np = W.gaussian(n, 2.0 ** e / t, key=(170, n, e + 20))
    A = torch.from_numpy(A_np).cuda()
    (U0, p0), (U1, p1) = expi_both(env, A, t)
    assert (p1.level, p1.s, p1.products, p1.status) == (p0.level, p0.s, p0.products, 0)
    assert torch.equal(U0, U1), (n, e, p0)
    th = float(np.abs(t * A_np).sum(0).max())
    assert any((p1.level, p1.s) == P.plan(th * f)[:2] for f in (1.0, 1 - 1e-12, 1 + 1e-12))
    assert rel_fro(U1.cpu().numpy(), Pr.unitary_paper(A_np, t)) <= 1e-12


def test_expi_async_float32_and_failures(env):
    torch, sc = env
    A32 = W.gaussian(120, 40.0, key=(171,)).astype(np.float32)
    A = torch.from_numpy(A32).cuda()
    (U0, p0), (U1, p1) = expi_both(env, A, 0.5, "single")
    assert (p1.level, p1.s) == (p0.level, p0.s) and torch.equal(U0, U1)
    assert rel_fro(U1.cpu().numpy().astype(np.complex128), Pr.unitary(A32.astype(np.float64), 0.5)) <= 5e-6
    Ad = torch.from_numpy(W.gaussian(40, 2.0 ** 6, key=(172,))).cuda()   # double plan: s = 6
    U = torch.empty(40, 40, dtype=torch.complex128, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_expi_eval_async(Ad, 1.0, U, 5, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_SCALING
    assert bool(torch.isnan(U.real).all()) and bool(torch.isnan(U.imag).all())
    Ad[5, 5] = float("nan")
    sc.sincosm_expi_eval_async(Ad, 1.0, U, 8, plan_dev=pd)
    assert sc.plan_from_device(pd).status == sc._lib.E_NONFINITE
    assert bool(torch.isnan(U.real).all())
    with pytest.raises(sc.SincosmError):
        sc.sincosm_expi_eval_async(Ad, float("nan"), U, 8)


def test_expi_async_graph_capture_no_plan(env):
    torch, sc = env
    n = 160
    t = 1.25
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    U = torch.empty(n, n, dtype=torch.complex128, device="cuda")
    ws = torch.empty(sc.workspace_size(n), dtype=torch.uint8, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_expi_eval_async(A, t, U, 10, ws=ws, plan_dev=pd)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_expi_eval_async(A, t, U, 10, ws=ws, plan_dev=pd)
    seen = set()
    for k, e in enumerate([-4.0, 0.5, 2.0, 7.0]):
        say("expi async graph replay", e)
        A.copy_(torch.from_numpy(W.gaussian(n, 2.0 ** e / t, key=(173, k))).cuda())
        junk = torch.randn(128, 128, device="cuda", dtype=torch.float64)
        junk = junk @ junk
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rec = sc.plan_from_device(pd)
        Ue = torch.empty_like(U)
        pe = sc.sincosm_expi_eval(A, t, Ue)
        torch.cuda.synchronize()
        assert (rec.level, rec.s, rec.status) == (pe.level, pe.s, 0)
        assert torch.equal(U, Ue), e
        seen.add((rec.level, rec.s))
    assert len(seen) == 4


@pytest.mark.parametrize("products", ["f32", "bf16x3"])
def test_expi_async_tiers_bitwise(env, products):
    """Lowered-product tiers on float64 data: the device-planned e^{-itA} equals the synchronous
    call bitwise (same launches, plan decided on the device)."""
    torch, sc = env
    say("expi async tier", products)
    A = torch.from_numpy(W.gaussian(300, 2.0 ** 5, key=(174,))).cuda()
    (U0, p0), (U1, p1) = expi_both(env, A, 0.8, "single", products)
    assert (p1.level, p1.s) == (p0.level, p0.s)
    assert torch.equal(U0, U1)


@pytest.mark.parametrize("norm", [0.1, 0.81])
def test_expi_async_extended_plan(env, norm):
    """With the 5-product scheme among the candidates (it wins on (theta_4, theta_5])."""
    torch, sc = env
    A = torch.from_numpy(W.gaussian(150, norm, key=(175, int(norm * 10)))).cuda()
    acc = "double" if norm < 0.5 else "single"
    U0 = torch.empty(A.shape, dtype=torch.complex128, device="cuda")
    p0 = sc.sincosm_expi_eval(A, 1.0, U0, acc, extended=True)
    U1 = torch.empty_like(U0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_expi_eval_async(A, 1.0, U1, 8, acc, plan_dev=pd, extended=True)
    torch.cuda.synchronize()
    p1 = sc.plan_from_device(pd)
    assert (p1.level, p1.s) == (p0.level, p0.s) and p0.level == 5
    assert torch.equal(U0, U1)


@pytest.mark.parametrize("n", [64, 257])
def test_wave_block_async_float32(env, n):
    """Float32 storage, single plan: the device-planned block propagator against the synchronous
    one (C blocks bitwise, the s blocks to float32 rounding) and against the oracle at 5e-6."""
    torch, sc = env
    say("block async f32", n)
    t = 0.9
    A32 = W.gaussian(n, 2.0 ** 4 / (t * t), key=(176, n)).astype(np.float32)
    A = torch.from_numpy(A32).cuda()
    E0 = torch.empty(2 * n, 2 * n, dtype=torch.float32, device="cuda")
    sc.sincosm_wave_block_eval(A, t, E0, "single")
    E1 = torch.empty_like(E0)
    sc.sincosm_wave_block_eval_async(A, t, E1, 8, "single")
    torch.cuda.synchronize()
    assert torch.equal(E1[:n, :n], E0[:n, :n]) and torch.equal(E1[n:, n:], E0[n:, n:])
    assert rel_fro(np64(E1), np64(E0)) <= 1e-6
    assert rel_fro(np64(E1), Pr.symplectic_paper(A32.astype(np.float64), t, "single")) <= 5e-6


def test_wave_async_n4096(env):
    """The headline order (tuned 256 x 128 double-angle launches): ||t^2 A||_1 = 2^10, s = 4;
    C bitwise equal to the synchronous call, S to 1e-13, both against the closed form of the
    1-D Laplacian family on sampled rows."""
    torch, sc = env
    say("wave async n=4096")
    n, t = 4096, 1.0
    A_np = W.laplacian_1d(n, 2.0 ** 10)
    A = torch.from_numpy(A_np).cuda()
    (C0, S0, p0), (C1, S1, p1) = wave_both(env, A, t)
    assert (p1.level, p1.s, p1.status) == (p0.level, p0.s, 0) and p1.s >= 3
    assert torch.equal(C0, C1)
    assert rel_fro(np64(S1), np64(S0)) <= 1e-13
    del C0, S0
    # A = c tridiag(-1, 2, -1): its eigenpairs are known in closed form
    rows = [0, 1, 2047, 4095]
    c = 2.0 ** 10 / 4.0
    k = np.arange(1, n + 1)
    mu = 2.0 * c * (1.0 - np.cos(k * np.pi / (n + 1)))        # eigenvalues of A
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(np.arange(1, n + 1), k) * np.pi / (n + 1))
    r = np.sqrt(mu)
    Cr = (V[rows] * np.cos(t * r)) @ V.T
    Sr = (V[rows] * (np.sin(t * r) / r)) @ V.T
    C1r, S1r = np64(C1[rows]), np64(S1[rows])
    assert rel_fro(C1r, Cr) <= 1e-12 and rel_fro(S1r, Sr) <= 1e-12
