"""GPU parity of sincosm_wave_eval (c(t^2 A), s(t, A) of Sections 1 and 2.2) against the oracle.

Bars: relative Frobenius error <= 1e-12 against the float64 wave oracle (the Section 2.2
schemes with the same plan, oracle/wave.py paper_wave) for the double-accuracy float64
path, and against the independent Taylor reference (oracle/wave.py reference) where the
two oracles themselves agree to well below that (||t^2 A||_1 <= 2^8); plan integers equal
the oracle's wave plan (either neighbour accepted within 1e-12 relative of a breakpoint).
Float32 storage / single accuracy: 5e-6 relative (the single-accuracy bar)."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import reference as R
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


def run(env, A_np, t, accuracy="double", products="native", dtype=None):
    torch, sc = env
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    if dtype is not None:
        A = A.to(dtype)
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    plan = sc.sincosm_wave_eval(A, t, C, S, accuracy, products)
    torch.cuda.synchronize()
    return C.cpu().double().numpy(), S.cpu().double().numpy(), plan


def plan_ok(plan, A, t, acc="double"):
    nb = float(np.abs((t * t) * A).sum(0).max())
    got = (plan.level, plan.s, plan.products)
    return any(got == Wv.wave_plan(nb * f, acc) for f in (1.0, 1 - 1e-12, 1 + 1e-12))


B_EXPS = [-9, -7, -2, 1, 4, 8, 12]


@pytest.mark.parametrize("family", ["gaussian", "symmetric", "laplacian1d"])
@pytest.mark.parametrize("n", [33, 64, 257])
@pytest.mark.parametrize("e", B_EXPS)
def test_levels_and_scaling(env, family, n, e):
    """||t^2 A||_1 = 2^e: every wave scheme (2, 3, 4, 5 products) and s up to 6."""
    say("wave", family, n, e)
    t = 1.3
    A = W.family(family, n, 2.0 ** e / (t * t), key=(60, n, e + 20))
    C, S, plan = run(env, A, t)
    assert plan_ok(plan, A, t), plan
    Cp, Sp = Wv.paper_wave(A, t)
    assert rel_fro(C, Cp) <= 1e-12
    assert rel_fro(S, Sp) <= 1e-12
    if e <= 8:
        Cr, Sr = Wv.reference(A, t)
        assert rel_fro(C, Cr) <= 1e-12
        assert rel_fro(S, Sr) <= 1e-12


def test_every_level_reached(env):
    seen = set()
    for e in B_EXPS:
        A = W.gaussian(40, 2.0 ** e, key=(61, e + 20))
        seen.add(run(env, A, 1.0)[2].level)
    assert seen == {2, 3, 4, 5}


@pytest.mark.parametrize("n,e", [(1000, 0), (1000, 6), (1536, 10), (2100, 3)])
def test_larger_n(env, n, e):
    say("wave large", n, e)
    t = 0.7
    A = W.gaussian(n, 2.0 ** e / (t * t), key=(62, n))
    C, S, plan = run(env, A, t)
    assert plan_ok(plan, A, t)
    Cp, Sp = Wv.paper_wave(A, t)
    assert rel_fro(C, Cp) <= 1e-12
    assert rel_fro(S, Sp) <= 1e-12


def test_square_of_nonsymmetric(env):
    """A = X^2: c(t^2 A) = cos(tX) and s(t, A) X = sin(tX), with cos/sin from the independent
    Taylor reference of the cos/sin oracle."""
    say("wave X^2")
    X = W.gaussian(150, 3.0, key=(63,))
    A = X @ X
    t = 1.1
    C, S, _ = run(env, A, t)
    Cx, Sx = R.sincosm(t * X)
    assert rel_fro(C, Cx) <= 1e-12
    assert rel_fro(S @ X, Sx) <= 1e-12


def test_spd_eigendecomposition(env):
    """Symmetric positive definite A (1-D Laplacian): C = Q cos(t sqrt L) Q^T, S = Q sin(t sqrt L)/sqrt L Q^T."""
    say("wave spd")
    A = W.laplacian_1d(200, 400.0)
    t = 0.9
    C, S, _ = run(env, A, t)
    lam, Q = np.linalg.eigh(A)
    r = np.sqrt(np.maximum(lam, 0.0))
    Cr = (Q * np.cos(t * r)) @ Q.T
    Sr = (Q * (np.sin(t * r) / r)) @ Q.T
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


def test_block_exponential(env):
    """e^{tM} for M = [[0, I], [-A, 0]] equals [[C, S], [-A S, C]] (scipy's expm)."""
    import scipy.linalg
    say("wave block expm")
    n = 60
    A = W.gaussian(n, 5.0, key=(64,))
    t = 0.8
    C, S, _ = run(env, A, t)
    M = np.zeros((2 * n, 2 * n))
    M[:n, n:] = np.eye(n)
    M[n:, :n] = -A
    E = scipy.linalg.expm(t * M)
    assert rel_fro(C, E[:n, :n]) <= 1e-12
    assert rel_fro(S, E[:n, n:]) <= 1e-12


def test_n1_closed_forms(env):
    t = 1.3
    for a in (0.0, 1e-6, 0.7, 30.0, -4.0, 900.0):
        C, S, _ = run(env, np.array([[a]]), t)
        if a > 0:
            r = math.sqrt(a)
            cr, sr = math.cos(t * r), math.sin(t * r) / r
        elif a < 0:
            r = math.sqrt(-a)
            cr, sr = math.cosh(t * r), math.sinh(t * r) / r
        else:
            cr, sr = 1.0, t
        tol = 64 * 2.0 ** -53 * max(1.0, t * t * abs(a))
        assert abs(C[0, 0] - cr) <= tol * max(1, abs(cr)), (a, C[0, 0], cr)
        assert abs(S[0, 0] - sr) <= tol * max(1, abs(sr)), (a, S[0, 0], sr)


def test_t_zero_exact(env):
    A = W.gaussian(70, 3.0, key=(65,))
    C, S, plan = run(env, A, 0.0)
    assert (plan.level, plan.s) == (2, 0)
    assert np.array_equal(C, np.eye(70)) and not S.any()


def test_negative_t_bitwise(env):
    A = W.gaussian(130, 9.0, key=(66,))
    C1, S1, _ = run(env, A, 1.7)
    C2, S2, _ = run(env, A, -1.7)
    assert np.array_equal(C1, C2) and np.array_equal(S1, -S2)


def test_agrees_with_cos_sin_path(env):
    """c(t^2 X^2) = cos(tX): the wave path against the library's own cos/sin path at n = 400."""
    torch, sc = env
    say("wave vs sincosm")
    X = torch.from_numpy(W.gaussian(400, 6.0, key=(67,))).cuda()
    A = X @ X
    t = 0.6
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    sc.sincosm_wave_eval(A, t, C, S)
    Cx = torch.empty_like(A)
    Sx = torch.empty_like(A)
    sc.sincosm_eval((t * X).contiguous(), Cx, Sx)
    assert float((C - Cx).norm() / Cx.norm()) <= 1e-12
    assert float((S @ X - Sx).norm() / Sx.norm()) <= 1e-12


def test_double_angle_identity_n4096(env):
    """At full size: c(4 t^2 A) = 2 c(t^2 A)^2 - I and s(2t, A) = 2 s(t, A) c(t^2 A),
    from two independent calls (different plans), scaled residuals on the GPU."""
    torch, sc = env
    say("wave 4096 double angle")
    n = 4096
    A = torch.from_numpy(W.gaussian(n, 64.0, key=(68, n))).cuda()
    t = 0.5
    C1 = torch.empty_like(A)
    S1 = torch.empty_like(A)
    C2 = torch.empty_like(A)
    S2 = torch.empty_like(A)
    p1 = sc.sincosm_wave_eval(A, t, C1, S1)
    p2 = sc.sincosm_wave_eval(A, 2 * t, C2, S2)
    assert p2.products >= p1.products
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    u = 2.0 ** -53
    rc = float((2 * (C1 @ C1) - I - C2).norm() / (2 * C1.norm() ** 2 + n ** 0.5))
    rs = float((2 * (S1 @ C1) - S2).norm() / (2 * S1.norm() * C1.norm()))
    assert rc <= 8 * n * u and rs <= 8 * n * u, (rc, rs)


def test_n4096_oracle_small_norm(env):
    """Full size against the Taylor reference where no double-angle step is taken."""
    say("wave 4096 oracle")
    n = 4096
    A = W.gaussian(n, 2.0, key=(69, n))
    C, S, plan = run(env, A, 1.0)
    assert (plan.level, plan.s) == (5, 0)
    Cr, Sr = Wv.reference(A, 1.0)
    assert rel_fro(C, Cr) <= 1e-12
    assert rel_fro(S, Sr) <= 1e-12


def test_nonfinite_and_errors(env):
    torch, sc = env
    A = torch.zeros(20, 20, dtype=torch.float64, device="cuda")
    A[3, 4] = float("nan")
    C = torch.zeros_like(A)
    S = torch.zeros_like(A)
    plan = sc.sincosm_wave_eval(A, 1.0, C, S, raise_nonfinite=False)
    assert plan.status == -4
    assert torch.isnan(C).all() and torch.isnan(S).all()
    A[3, 4] = 1.0
    with pytest.raises(sc.SincosmError):
        sc.sincosm_wave_eval(A, float("inf"), C, S)
    plan = sc.sincosm_wave_eval(A, 1e200, C, S, raise_nonfinite=False)   # t^2 overflows
    assert plan.status == -4
    with pytest.raises(sc.SincosmError):
        sc.sincosm_wave_eval(A, 1.0, A, S)   # output aliases the input


@pytest.mark.parametrize("n,e", [(64, 1), (257, 6), (1000, 9)])
def test_float32_single(env, n, e):
    say("wave f32", n, e)
    t = 1.0
    A32 = W.gaussian(n, 2.0 ** e, key=(70, n)).astype(np.float32)
    import torch
    C, S, plan = run(env, A32, t, accuracy="single", dtype=torch.float32)
    assert plan_ok(plan, A32.astype(np.float64), t, "single")
    Cr, Sr = Wv.reference(A32.astype(np.float64), t)
    tol = 5e-6
    assert rel_fro(C, Cr) <= tol and rel_fro(S, Sr) <= tol


U_BF = 2.0 ** -18


@pytest.mark.parametrize("n,e", [(64, 1), (300, 6)])
def test_tier_bf16x3_products(env, n, e):
    """float64 storage, bf16x3 scheme products, float64 double-angle steps: the bound of the
    cos/sin bf16x3 tier, 8 Pi 2^-18 2^s with Pi = 5."""
    say("wave bf16x3", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(71, n))
    C, S, plan = run(env, A, 1.0, accuracy="single", products="bf16x3")
    Cr, Sr = Wv.reference(A, 1.0)
    tol = 8 * 5 * U_BF * 2 ** plan.s
    assert rel_fro(C, Cr) <= tol and rel_fro(S, Sr) <= tol


def test_strided_views(env):
    """Inputs and outputs as views with leading dimension > n; memory outside stays untouched."""
    torch, sc = env
    g = W.rng(72)
    big = torch.from_numpy(g.standard_normal((80, 90)) * 0.05).cuda()
    A = big[5:65, 10:70]
    Cb = torch.zeros(70, 75, dtype=torch.float64, device="cuda")
    Sb = torch.zeros(70, 75, dtype=torch.float64, device="cuda")
    C = Cb[2:62, 3:63]
    S = Sb[4:64, 10:70]
    sc.sincosm_wave_eval(A, 1.4, C, S)
    torch.cuda.synchronize()
    Cp, Sp = Wv.paper_wave(A.cpu().numpy(), 1.4)
    assert rel_fro(C.cpu().numpy(), Cp) <= 1e-12 and rel_fro(S.cpu().numpy(), Sp) <= 1e-12
    rc, rs = Cb.cpu().numpy().copy(), Sb.cpu().numpy().copy()
    rc[2:62, 3:63] = 0
    rs[4:64, 10:70] = 0
    assert not rc.any() and not rs.any()


def test_block_n1(env):
    """n = 1: e^{tM} for M = [[0, 1], [-a, 0]] against the oracle's block (closed forms there)."""
    from oracle import propagators as Pr
    torch, sc = env
    for a in (0.0, 2.5, -3.0):
        A = torch.tensor([[a]], dtype=torch.float64, device="cuda")
        E = sc.wave_block(A, 0.9).cpu().numpy()
        assert rel_fro(E, Pr.symplectic(np.array([[a]]), 0.9)) <= 1e-14


def test_wave_helper_matches_entry_point(env):
    """sc.wave allocates and calls sincosm_wave_eval on a contiguous copy: bitwise the same
    results for a strided view."""
    torch, sc = env
    big = torch.from_numpy(W.gaussian(150, 3.0, key=(95,))).cuda()
    A = big[5:133, 7:135]
    C, S = sc.wave(A, 0.75)
    Ac = A.contiguous()
    C1, S1 = torch.empty_like(Ac), torch.empty_like(Ac)
    sc.sincosm_wave_eval(Ac, 0.75, C1, S1)
    torch.cuda.synchronize()
    assert torch.equal(C, C1) and torch.equal(S, S1)
