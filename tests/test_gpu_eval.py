"""GPU parity of sincosm_eval (through the C ABI) against the CPU oracle.

Bars: relative Frobenius error <= 1e-12 against the float64 oracle for the
double-accuracy float64 path; the plan integers (level, s) equal the oracle's
(either neighbour accepted within 1e-12 relative of a breakpoint, where the two
1-norm summation orders may round differently)."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import paper_algorithm as PA
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


def run(env, A_np, accuracy="double", products="native", dtype=None):
    torch, sc = env
    t = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    if dtype is not None:
        t = t.to(dtype)
    C = torch.empty_like(t)
    S = torch.empty_like(t)
    plan = sc.sincosm_eval(t, C, S, accuracy, products)
    torch.cuda.synchronize()
    return C.cpu().double().numpy(), S.cpu().double().numpy(), plan


def plan_ok(plan, A, acc="double"):
    t = float(np.abs(A).sum(0).max())
    want = P.plan(t, acc)
    if (plan.level, plan.s, plan.products) == want:
        return True
    for f in (1 - 1e-12, 1 + 1e-12):
        if (plan.level, plan.s, plan.products) == P.plan(t * f, acc):
            return True
    return False


# ---------------------------------------------------------------------------
# Products
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 16, 37, 64, 100, 128, 300, 777, 1000, 1600])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_matmul(env, n, dt):
    torch, sc = env
    say("matmul", n, dt)
    g = W.rng(40, n)
    X = g.standard_normal((n, n))
    Y = g.standard_normal((n, n))
    tdt = torch.float64 if dt == "f64" else torch.float32
    Xt = torch.from_numpy(X).cuda().to(tdt)
    Yt = torch.from_numpy(Y).cuda().to(tdt)
    Z = torch.empty_like(Xt)
    sc.sincosm_matmul(Xt, Yt, Z)
    torch.cuda.synchronize()
    Xr = Xt.cpu().double().numpy()
    Yr = Yt.cpu().double().numpy()
    ref = Xr @ Yr
    bound = np.abs(Xr) @ np.abs(Yr)
    u = 2.0 ** -53 if dt == "f64" else 2.0 ** -24
    err = np.max(np.abs(Z.cpu().double().numpy() - ref) / bound)
    assert err <= 2 * n * u, err


def test_matmul_strided(env):
    torch, sc = env
    say("matmul strided")
    g = W.rng(41)
    big = torch.from_numpy(g.standard_normal((90, 120))).cuda()
    X = big[:70, 5:75]
    Y = big[10:80, 40:110]
    Zb = torch.zeros(80, 100, dtype=torch.float64, device="cuda")
    Z = Zb[3:73, 7:77]
    sc.sincosm_matmul(X, Y, Z)
    torch.cuda.synchronize()
    ref = X.cpu().numpy() @ Y.cpu().numpy()
    assert np.max(np.abs(Z.cpu().numpy() - ref)) < 1e-12
    # outside the written window stays zero
    Zc = Zb.cpu().numpy().copy()
    Zc[3:73, 7:77] = 0
    assert not Zc.any()


# ---------------------------------------------------------------------------
# Whole path, float64
# ---------------------------------------------------------------------------
def test_config_small_n64(env):
    """n = 64 Gaussian rescaled to ||A||_1 = 2 (7 products, s = 1: 9 products)."""
    say("config n=64 norm=2")
    A = W.gaussian(64, 2.0, key=(1, 64, 0, 0))
    C, S, plan = run(env, A)
    assert (plan.level, plan.s, plan.products) == (7, 1, 9)
    Cl, Sl = R.sincosm_ld(A)
    assert rel_fro(C, Cl.astype(float)) <= 1e-12
    assert rel_fro(S, Sl.astype(float)) <= 1e-12
    Cp, Sp = PA.sincosm(A)
    assert rel_fro(C, Cp) <= 1e-13
    assert rel_fro(S, Sp) <= 1e-13


LEVEL_EXPS = [-9.0, -5.0, -1.0, 0.5, 1.0, 2.0, 5.0, 10.0]


@pytest.mark.parametrize("family", ["gaussian", "symmetric", "laplacian1d"])
@pytest.mark.parametrize("n", [33, 64, 257])
@pytest.mark.parametrize("e", LEVEL_EXPS)
def test_levels_and_scaling(env, family, n, e):
    say("eval", family, n, e)
    A = W.family(family, n, 2.0 ** e, key=(42, n, int(e * 2) + 40))
    C, S, plan = run(env, A)
    assert plan_ok(plan, A)
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


def test_every_level_reached(env):
    seen = set()
    for e in LEVEL_EXPS:
        A = W.gaussian(48, 2.0 ** e, key=(43, int(e * 2) + 40))
        seen.add(run(env, A)[2].level)
    assert seen == {3, 4, 6, 7}


@pytest.mark.parametrize("n,e", [(1000, 0.0), (1000, 4.0), (1536, 10.0), (2100, 3.0)])
def test_larger_n(env, n, e):
    say("eval large", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(44, n))
    C, S, plan = run(env, A)
    assert plan_ok(plan, A)
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


def test_n4096_oracle_small_norm(env):
    say("eval 4096 oracle e=-4")
    A = W.gaussian(4096, 2.0 ** -4, key=(2, 4096, 0, 0))
    C, S, plan = run(env, A)
    assert (plan.level, plan.s) == (4, 0)
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


@pytest.mark.parametrize("e", [-4, 0, 4, 10])
def test_n4096_anchors_vs_oracle(env, e):
    """The headline workload: n = 4096 Gaussian at ||A||_1 = 2^e (plans (4,0), (7,0), (7,4),
    (7,10)), the same seeded matrices the throughput figure is measured on, against the
    float64 oracle. At this order the scheme products run the tuned 128 x 128 direct-load
    configuration and the double-angle launches the 256 x 128 one."""
    say("eval 4096 anchor oracle", e)
    A = W.gaussian(4096, 2.0 ** e, key=(2, 4096, 0, e + 10))
    C, S, plan = run(env, A)
    assert (plan.level, plan.s) == {-4: (4, 0), 0: (7, 0), 4: (7, 4), 10: (7, 10)}[e]
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12, rel_fro(C, Cr)
    assert rel_fro(S, Sr) <= 1e-12, rel_fro(S, Sr)


@pytest.mark.parametrize("n", [1536, 2048, 3000])
@pytest.mark.parametrize("e", [-9.0, -5.0, -1.0])
def test_levels_3_4_6_padded_128(env, n, e):
    """Levels 3, 4 and 6 (s = 0) at orders padded to 128-wide tiles, against the oracle."""
    say("eval levels 128-padded", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(45, n, int(e) + 20))
    C, S, plan = run(env, A)
    assert plan_ok(plan, A) and plan.level == {-9.0: 3, -5.0: 4, -1.0: 6}[e]
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


@pytest.mark.parametrize("e", [4.0, 10.0])
def test_n4096_identities(env, e):
    """At full size: cos^2 + sin^2 = I and CS = SC (scaled residuals), on the GPU."""
    torch, sc = env
    say("eval 4096 identities", e)
    n = 4096
    A = torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(2, n, 0, int(e)))).cuda()
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    plan = sc.sincosm_eval(A, C, S)
    assert plan.products == P.plan(float(A.abs().sum(0).max()))[2]
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    denom = float(C.norm() ** 2 + S.norm() ** 2 + n ** 0.5)
    r1 = float((C @ C + S @ S - I).norm()) / denom
    r2 = float((C @ S - S @ C).norm()) / denom
    u = 2.0 ** -53
    assert r1 <= 8 * n * u and r2 <= 8 * n * u, (r1, r2)


# ---------------------------------------------------------------------------
# Closed forms, edge cases, invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("e", [33.0, 40.0])
def test_large_norm_scaled_operands(env, e):
    """||A||_1 = 2^e needs s > 30: the first product's operand scale 4^-s then lies outside
    the range in which it moves into the epilogue, so the kernels scale the operands
    themselves. Against eigh of a symmetric A; the s double-angle steps amplify rounding by
    about 2^s, so the bar is 2^s 64 u (a missing or doubled scale gives errors of order 1)."""
    say("eval large norm", e)
    A = W.symmetric_gaussian(48, 2.0 ** e, key=(60, int(e)))
    w, V = np.linalg.eigh(A)
    Cr, Sr = (V * np.cos(w)) @ V.T, (V * np.sin(w)) @ V.T
    C, S, plan = run(env, A)
    assert plan_ok(plan, A) and plan.s > 30
    tol = 2.0 ** plan.s * 64 * 2.0 ** -53
    assert rel_fro(C, Cr) <= tol and rel_fro(S, Sr) <= tol
    Cp, Sp = PA.sincosm(A)     # the same algorithm in float64 on the host
    assert rel_fro(C, Cp) <= tol and rel_fro(S, Sp) <= tol


def test_n1(env):
    for x in (0.0, 1e-3, 0.7, -2.5, 40.0):
        C, S, plan = run(env, np.array([[x]]))
        assert abs(C[0, 0] - math.cos(x)) <= 1e-15 * max(1, abs(x)) * 16
        assert abs(S[0, 0] - math.sin(x)) <= 1e-15 * max(1, abs(x)) * 16


def test_rotation_generator(env):
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    for t in (0.3, 2.0, 9.0):
        C, S, _ = run(env, t * J)
        assert rel_fro(C, math.cosh(t) * np.eye(2)) <= 1e-14 * max(1, t)
        assert rel_fro(S, math.sinh(t) * J) <= 1e-14 * max(1, t)


def test_nilpotent(env):
    A = W.nilpotent_upper(40, key=(45,), rank_band=3) * 0.5
    C, S, _ = run(env, A)
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12 and rel_fro(S, Sr) <= 1e-12
    assert not np.tril(C, -1).any() and not np.tril(S, -1).any()


def test_zero_matrix_exact(env):
    C, S, plan = run(env, np.zeros((50, 50)))
    assert (plan.level, plan.s) == (3, 0)
    assert np.array_equal(C, np.eye(50)) and not S.any()


def test_parity_bitwise(env):
    A = W.gaussian(130, 9.0, key=(46,))
    C1, S1, _ = run(env, A)
    C2, S2, _ = run(env, -A)
    assert np.array_equal(C1, C2) and np.array_equal(S1, -S2)


def test_deterministic(env):
    A = W.gaussian(300, 30.0, key=(47,))
    a = run(env, A)
    b = run(env, A)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_transpose_consistency(env):
    A = W.gaussian(90, 3.0, key=(48,))
    C, S, _ = run(env, A)
    Ct, St, _ = run(env, A.T.copy())
    # the plan may differ (1-norm vs infinity-norm), the functions agree
    assert rel_fro(Ct, C.T) <= 1e-12 and rel_fro(St, S.T) <= 1e-12


def test_nonfinite_input(env):
    torch, sc = env
    A = torch.zeros(20, 20, dtype=torch.float64, device="cuda")
    A[3, 4] = float("nan")
    C = torch.zeros_like(A)
    S = torch.zeros_like(A)
    plan = sc.sincosm_eval(A, C, S, raise_nonfinite=False)
    assert plan.status == -4
    assert torch.isnan(C).all() and torch.isnan(S).all()
    A[3, 4] = float("inf")
    with pytest.raises(sc.SincosmError):
        sc.sincosm_eval(A, C, S)


def test_strided_views_and_errors(env):
    torch, sc = env
    g = W.rng(49)
    big = torch.from_numpy(g.standard_normal((80, 90)) * 0.05).cuda()
    A = big[5:65, 10:70]
    Cb = torch.zeros(70, 75, dtype=torch.float64, device="cuda")
    Sb = torch.zeros(70, 75, dtype=torch.float64, device="cuda")
    C = Cb[2:62, 3:63]
    S = Sb[2:62, 3:63]
    sc.sincosm_eval(A, C, S)
    Cr, Sr = R.sincosm(A.cpu().numpy())
    assert rel_fro(C.cpu().numpy(), Cr) <= 1e-12 and rel_fro(S.cpu().numpy(), Sr) <= 1e-12
    Cc = Cb.cpu().numpy().copy()
    Cc[2:62, 3:63] = 0
    assert not Cc.any()
    # aliasing and workspace errors
    with pytest.raises(sc.SincosmError) as ei:
        sc.sincosm_eval(A, A, S)
    assert ei.value.status == -1
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(sc.SincosmError) as ei:
        sc.sincosm_eval(A, C, S, ws=small)
    assert ei.value.status == -3


def test_device_plan_matches_oracle(env):
    torch, sc = env
    for i, e in enumerate(np.linspace(-12, 30, 43)):
        A = W.gaussian(24, 2.0 ** e, key=(50, i))
        p = sc.plan_device(torch.from_numpy(A).cuda())
        assert plan_ok(p, A), (e, p)
        p = sc.plan_device(torch.from_numpy(A).cuda(), "single")
        assert plan_ok(p, A, "single"), (e, p)


# ---------------------------------------------------------------------------
# Single accuracy / float32 storage / float32 products
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,e", [(64, 1.0), (257, 4.0), (1000, 6.0)])
def test_float32_single(env, n, e):
    torch, sc = env
    say("eval f32", n, e)
    A32 = W.gaussian(n, 2.0 ** e, key=(51, n)).astype(np.float32)
    C, S, plan = run(env, A32, accuracy="single", dtype=torch.float32)
    assert plan_ok(plan, A32.astype(np.float64), "single")
    Cr, Sr = R.sincosm(A32.astype(np.float64))
    assert rel_fro(C, Cr) <= 5e-6
    assert rel_fro(S, Sr) <= 5e-6


@pytest.mark.parametrize("n,e", [(64, 1.0), (500, 6.0)])
def test_tier_f32_products(env, n, e):
    torch, sc = env
    say("eval tier f32 products", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(52, n))
    C, S, plan = run(env, A, accuracy="single", products="f32")
    assert plan_ok(plan, A, "single")
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 5e-6 and rel_fro(S, Sr) <= 5e-6


# ---------------------------------------------------------------------------
# Split BF16 x3 products (precision tier)
# ---------------------------------------------------------------------------
U_BF = 2.0 ** -18   # |x - (hi + lo)| <= 2^-9 |lo| <= 2^-18 |x| ; dropped lo*lo ~ 2^-18 |x||y|


@pytest.mark.parametrize("n", [16, 100, 300, 1000, 1600])
def test_matmul_bf16x3(env, n):
    """Elementwise bound |Z - XY| <= (4 * 2^-18 + 2 n 2^-24) (|X||Y|)_ij: split error of both
    operands, the dropped lo*lo term, and float32 accumulation."""
    torch, sc = env
    g = W.rng(53, n)
    X = g.standard_normal((n, n)).astype(np.float32)
    Y = g.standard_normal((n, n)).astype(np.float32)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    Z = torch.empty_like(Xt)
    sc.sincosm_matmul(Xt, Yt, Z, products="bf16x3")
    torch.cuda.synchronize()
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    err = np.max(np.abs(Z.cpu().double().numpy() - Xd @ Yd) / (np.abs(Xd) @ np.abs(Yd)))
    assert err <= 4 * U_BF + 2 * n * 2.0 ** -24, err


@pytest.mark.parametrize("n,e", [(64, 1.0), (300, 4.0), (1000, 6.0), (2100, 6.0)])
def test_tier_bf16x3_products(env, n, e):
    """float64 storage, bf16x3 scheme products, float64 squarings, single-accuracy plan.

    Stated bound: each of the Pi scheme products carries a relative error of a few 2^-18
    (test_matmul_bf16x3), the float32 intermediates 2^-24, and the s double-angle steps
    amplify an error of the scheme's output by at most about 2^s relative to cos/sin of
    norm-1 arguments: rel err <= 8 Pi 2^-18 2^s (checked with Pi = 7)."""
    torch, sc = env
    print("[case] eval tier bf16x3", n, e, flush=True)
    A = W.gaussian(n, 2.0 ** e, key=(54, n))
    C, S, plan = run(env, A, accuracy="single", products="bf16x3")
    assert plan_ok(plan, A, "single")
    Cr, Sr = R.sincosm(A)
    tol = 8 * 7 * U_BF * 2 ** plan.s
    ec, es = rel_fro(C, Cr), rel_fro(S, Sr)
    print(f"bf16x3 n={n} e={e} plan=({plan.level},{plan.s}) rel err cos {ec:.2e} sin {es:.2e} tol {tol:.1e}")
    assert ec <= tol and es <= tol


def test_tier_bf16x3_float32_storage(env):
    torch, sc = env
    A32 = W.gaussian(200, 8.0, key=(55,)).astype(np.float32)
    C, S, plan = run(env, A32, accuracy="single", products="bf16x3", dtype=torch.float32)
    Cr, Sr = R.sincosm(A32.astype(np.float64))
    tol = 8 * 7 * U_BF * 2 ** plan.s
    assert rel_fro(C, Cr) <= tol and rel_fro(S, Sr) <= tol


# ---------------------------------------------------------------------------
# Extended plan: the 5-product scheme (Algorithm4cA cosine, Algorithm5sA sine)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [33, 257, 1000])
@pytest.mark.parametrize("acc,norm", [("double", 0.1), ("double", 0.114), ("single", 0.8)])
def test_extended_level5(env, n, acc, norm):
    torch, sc = env
    say("eval level5", n, acc, norm)
    A = W.gaussian(n, norm, key=(56, n, int(norm * 1000)))
    At = torch.from_numpy(A).cuda()
    C = torch.empty_like(At)
    S = torch.empty_like(At)
    plan = sc.sincosm_eval(At, C, S, acc, extended=True)
    torch.cuda.synchronize()
    assert (plan.level, plan.s, plan.products) == (5, 0, 5)
    assert sc.plan_device(At, acc).products == 6          # the paper's tables take one more
    C, S = C.cpu().numpy(), S.cpu().numpy()
    Cp, Sp = PA.sincosm(A, acc, extended=True)
    assert rel_fro(C, Cp) <= 1e-12 and rel_fro(S, Sp) <= 1e-12
    Cr, Sr = R.sincosm(A)
    tol = 1e-12 if acc == "double" else 5e-6
    assert rel_fro(C, Cr) <= tol and rel_fro(S, Sr) <= tol


def test_extended_level5_tiers_and_expi(env):
    torch, sc = env
    A = W.gaussian(300, 0.8, key=(57,))
    C, S, plan = None, None, None
    At = torch.from_numpy(A).cuda()
    C = torch.empty_like(At)
    S = torch.empty_like(At)
    plan = sc.sincosm_eval(At, C, S, "single", "bf16x3", extended=True)
    assert plan.level == 5
    Cr, Sr = R.sincosm(A)
    tol = 8 * 5 * U_BF
    assert rel_fro(C.cpu().numpy(), Cr) <= tol and rel_fro(S.cpu().numpy(), Sr) <= tol
    U = torch.empty(300, 300, dtype=torch.complex128, device="cuda")
    p = sc.sincosm_expi_eval(At, 1.0, U, "double", extended=False)
    assert p.level == 6
    p = sc.sincosm_expi_eval(At * 0.125, 1.0, U, "double", extended=True)
    assert p.level == 5
    Ur = R.sincosm(A * 0.125)
    assert rel_fro(U.cpu().numpy(), Ur[0] - 1j * Ur[1]) <= 1e-12


# ---------------------------------------------------------------------------
# Refined-norm plan (min(||A||_1, ||A^2||_1^(1/2))) against overscaling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [1e2, 1e4, 1e8])
def test_refined_paper_overscaling_matrix(env, lam):
    """Section 4's [[1, lambda], [0, -1]]: cos A = cos(1) I, sin A = sin(1) A; 7 products, s = 0."""
    torch, sc = env
    A = np.array([[1.0, lam], [0.0, -1.0]])
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    plan = sc.sincosm_eval(At, C, S, refined=True)
    assert (plan.level, plan.s, plan.products) == (7, 0, 7)
    assert rel_fro(C.cpu().numpy(), math.cos(1.0) * np.eye(2)) <= 1e-15
    assert rel_fro(S.cpu().numpy(), math.sin(1.0) * A) <= 1e-15


@pytest.mark.parametrize("n,norm", [(300, 1e3), (1000, 1e6), (4096, 1024.0)])
def test_refined_block_family(env, n, norm):
    """[[I, B], [0, -I]] squares to I exactly: closed form at any size, including n = 4096."""
    torch, sc = env
    say("refined block", n, norm)
    h = n // 2
    B = torch.from_numpy(W.gaussian(h, norm, key=(58, n))).cuda()
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    A[:h, :h] = torch.eye(h, dtype=torch.float64, device="cuda")
    A[h:, h:] = -torch.eye(h, dtype=torch.float64, device="cuda")
    A[:h, h:] = B
    C, S = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_eval(A, C, S, refined=True)
    assert (plan.level, plan.s) == (7, 0)
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    ec = float((C - math.cos(1.0) * I).norm() / (math.cos(1.0) * n ** 0.5))
    es = float((S - math.sin(1.0) * A).norm() / (math.sin(1.0) * A.norm()))
    assert ec <= 1e-15 and es <= 1e-15, (ec, es)
    # the tables' plan on the same matrix scales by about ||A||_1
    assert sc.plan_device(A).s >= 9


@pytest.mark.parametrize("e", [-3, 1, 5, 9])
def test_refined_random_matches_oracle(env, e):
    """Gaussian matrices: plan = the oracle's refined plan; within 1e-12 of both oracles; and
    bitwise equal to the unrefined call whenever the plans agree (same products, A^2 reused)."""
    torch, sc = env
    A = W.gaussian(257, 2.0 ** e, key=(59, e + 10))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    plan = sc.sincosm_eval(At, C, S, refined=True)
    th = P.refined_theta(A)
    got = (plan.level, plan.s, plan.products)
    assert any(got == P.plan(th * f) for f in (1.0, 1 - 1e-12, 1 + 1e-12)), (got, th)
    C, S = C.cpu().numpy(), S.cpu().numpy()
    Cp, Sp = PA.sincosm(A, refined=True)
    assert rel_fro(C, Cp) <= 1e-12 and rel_fro(S, Sp) <= 1e-12
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C, Cr) <= 1e-12 and rel_fro(S, Sr) <= 1e-12
    C0, S0, plan0 = run(env, A)
    if (plan0.level, plan0.s) == (plan.level, plan.s):
        assert np.array_equal(C0, C) and np.array_equal(S0, S)


def test_refined_tiers_and_flags(env):
    torch, sc = env
    A = np.kron(np.eye(50), np.array([[1.0, 1e6], [0.0, -1.0]]))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    plan = sc.sincosm_eval(At, C, S, "single", "f32", refined=True, extended=True)
    assert plan.s == 0
    tol = 5e-6
    assert rel_fro(C.cpu().numpy(), math.cos(1.0) * np.eye(100)) <= tol
    assert rel_fro(S.cpu().numpy(), math.sin(1.0) * A) <= tol
    # the flag is for sincosm_eval only
    U = torch.empty(100, 100, dtype=torch.complex128, device="cuda")
    st = sc.lib.sincosm_expi_eval(100, 0, At.data_ptr(), 100, 1.0, U.data_ptr(), 100, 32, 0, None, 0, None, None)
    assert st == -1


def test_refined_edge_cases(env):
    torch, sc = env
    # n = 1: A^2 = a^2, theta' = |a|
    for x in (0.0, -0.3, 40.0):
        At = torch.tensor([[x]], dtype=torch.float64, device="cuda")
        C, S = torch.empty_like(At), torch.empty_like(At)
        plan = sc.sincosm_eval(At, C, S, refined=True)
        assert abs(plan.norm1 - abs(x)) <= 1e-15 * max(1.0, abs(x))
        assert abs(float(C) - math.cos(x)) <= 1e-15 * 16 * max(1, abs(x))
        assert abs(float(S) - math.sin(x)) <= 1e-15 * 16 * max(1, abs(x))
    # zero matrix: exact identity / zero
    Z = torch.zeros(40, 40, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(Z), torch.empty_like(Z)
    plan = sc.sincosm_eval(Z, C, S, refined=True)
    assert (plan.level, plan.s) == (3, 0)
    assert torch.equal(C, torch.eye(40, dtype=torch.float64, device="cuda")) and not S.any()
    # non-finite input: status and NaN outputs, as without the flag
    Z[3, 7] = float("nan")
    plan = sc.sincosm_eval(Z, C, S, refined=True, raise_nonfinite=False)
    assert plan.status == -4 and torch.isnan(C).all() and torch.isnan(S).all()
    # A^2 overflows while A is finite: plan on ||A||_1, A^2 recomputed from the scaled operands
    A = torch.full((8, 8), 1e160, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(A), torch.empty_like(A)
    p0 = sc.sincosm_eval(A.clone(), C.clone(), S.clone())
    plan = sc.sincosm_eval(A, C, S, refined=True)
    assert (plan.level, plan.s) == (p0.level, p0.s)
    C0, S0 = torch.empty_like(A), torch.empty_like(A)
    sc.sincosm_eval(A, C0, S0)
    # (about 530 double-angle steps: the values are not meaningful, but both calls run the
    # same launches, so they agree bit for bit, NaN and Inf included)
    same = lambda X, Y: torch.equal(torch.nan_to_num(X), torch.nan_to_num(Y))
    assert same(C, C0) and same(S, S0)


def test_plan_log_env(env):
    """SINCOSM_LOG=1: each plan read back to the host is printed to stderr (a child process,
    since the variable is read once per process)."""
    import os
    import subprocess
    import sys as _sys
    code = ("import torch, numpy as np, paper_2010_00465_amd as sc, workloads as W\n"
            "A = torch.from_numpy(W.gaussian(64, 8.0, key=(5,))).cuda()\n"
            "C, S = torch.empty_like(A), torch.empty_like(A)\n"
            "sc.sincosm_eval(A, C, S)\n"
            "sc.sincosm_wave_eval(A, 0.5, C, S)\n"
            "torch.cuda.synchronize()\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    envv = dict(os.environ, SINCOSM_LOG="1", PYTHONPATH=root)
    r = subprocess.run([_sys.executable, "-c", code], cwd=root, env=envv, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("[sincosm]")]
    assert any(l.startswith("[sincosm] sincosm_eval n=64: level 7 s 3 products 13") for l in lines), lines
    assert any(l.startswith("[sincosm] wave n=64: level") for l in lines), lines
