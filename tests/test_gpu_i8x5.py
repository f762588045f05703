"""Products on the int8 matrix cores by error-free splitting (SINCOSM_PROD_I8X5) through the C ABI.

The product alone (sincosm_matmul): every operand entry is kept to 35 bits below its row's
(left operand) or column's (right operand) largest power of two, and the digit products of
weight below 2^-42 are left out, so the elementwise error of Z = X Y is at most
  T1 + T2,  T1 = 2^-34 (rowmax_i |X| colsum_j |Y| + rowsum_i |X| colmax_j |Y|),
            T2 = 2^-31 n rowmax_i |X| colmax_j |Y|
plus the float64 combination. T2 is reached only when digits agree in sign along the inner
dimension (tested with every digit at 127); for uncorrelated digits (Gaussian and graded
operands) its sums grow like n^(1/2) and the tests gate at 2 T1 alone.
Whole evaluations (sincosm_eval, float64 storage, intermediates and epilogues in float64, the
squarings in float64): against the float64 oracle at the single-accuracy bar 5e-6 for the
single plan (Table 2), and for the double plan at a bound derived from the product's: in the
Frobenius norm T1 gives at most 2^-33 n^(1/2) ||X|| ||Y|| (a row maximum is at most the row's
norm, a column sum at most n^(1/2) times the column's norm) and T2 at most 2^-31 n ||X|| ||Y||,
so the schemes' Pi products and the s squarings, each at most doubling what came before, keep
the relative error below 8 Pi (2^-33 n^(1/2) + 2^-31 n) 2^s (8 covering the growth of the
intermediates, as for the tiers' bounds in float32)."""
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


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [64, 100, 257, 1000])
@pytest.mark.parametrize("kind", ["gaussian", "graded"])
def test_i8x5_product_bound(env, n, kind):
    torch, sc = env
    say("i8x5 product", n, kind)
    g = W.rng(180, n, 0 if kind == "gaussian" else 1)
    X = g.standard_normal((n, n))
    Y = g.standard_normal((n, n))
    if kind == "graded":   # rows and columns of very different magnitudes
        X *= np.exp2(g.integers(-20, 20, size=(n, 1)))
        Y *= np.exp2(g.integers(-20, 20, size=(1, n)))
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    Z = torch.empty_like(Xt)
    sc.sincosm_matmul(Xt, Yt, Z, products="i8x5")
    torch.cuda.synchronize()
    Zr = X @ Y
    aX, aY = np.abs(X), np.abs(Y)
    bound = 2.0 ** -34 * (np.outer(aX.max(1), aY.sum(0)) + np.outer(aX.sum(1), aY.max(0)))
    err = np.abs(Z.cpu().numpy() - Zr)
    ratio = float((err / (2.0 * bound + 1e-300)).max())
    say("i8x5 product worst error / (2 bound)", ratio)
    assert ratio <= 1.0


@pytest.mark.parametrize("n", [64, 257, 1000])
@pytest.mark.parametrize("e", [-6.0, -1.0, 1.0, 4.0, 8.0])
def test_i8x5_eval_single(env, n, e):
    """Single plan, every level reached over the norms: <= 5e-6 against the float64 oracle."""
    torch, sc = env
    say("i8x5 eval single", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(181, n, int(e) + 10))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    p = sc.sincosm_eval(At, C, S, "single", "i8x5")
    torch.cuda.synchronize()
    Cr, Sr = R.sincosm(A)
    ec, es = rel_fro(C.cpu().numpy(), Cr), rel_fro(S.cpu().numpy(), Sr)
    say("i8x5 single errors", p.level, p.s, ec, es)
    assert ec <= 5e-6 and es <= 5e-6


@pytest.mark.parametrize("e", [-4.0, 0.0, 4.0, 10.0])
def test_i8x5_eval_double_plan_bound(env, e):
    torch, sc = env
    n = 512
    say("i8x5 eval double plan", e)
    A = W.gaussian(n, 2.0 ** e, key=(182, int(e) + 10))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    p = sc.sincosm_eval(At, C, S, "double", "i8x5")
    torch.cuda.synchronize()
    Cr, Sr = R.sincosm(A)
    bound = 8.0 * p.level * (2.0 ** -33 * np.sqrt(n) + 2.0 ** -31 * n) * 2.0 ** p.s
    ec, es = rel_fro(C.cpu().numpy(), Cr), rel_fro(S.cpu().numpy(), Sr)
    say("i8x5 double-plan errors", p.level, p.s, ec, es, bound)
    assert ec <= bound and es <= bound


def test_i8x5_laplacian_tier_workload(env):
    """The precision tiers' workload at reduced order (2-D Laplacian on a 32 x 32 grid,
    ||A||_1 = 64, single plan): within the single-accuracy bar with room to spare."""
    torch, sc = env
    A = W.laplacian_2d(32, 64.0)
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    p = sc.sincosm_eval(At, C, S, "single", "i8x5")
    torch.cuda.synchronize()
    Cr, Sr = R.sincosm(A)
    ec, es = rel_fro(C.cpu().numpy(), Cr), rel_fro(S.cpu().numpy(), Sr)
    say("i8x5 laplacian", p.level, p.s, ec, es)
    assert ec <= 5e-7 and es <= 5e-7


def test_i8x5_planned_and_refined(env):
    """sincosm_eval_planned with I8X5 products equals sincosm_eval bitwise; the refined-norm
    plan (its scaling pass is an epilogue-only launch) runs too."""
    torch, sc = env
    n = 300
    A = torch.from_numpy(W.gaussian(n, 20.0, key=(183,))).cuda()
    C0, S0, C1, S1 = (torch.empty_like(A) for _ in range(4))
    p = sc.sincosm_eval(A, C0, S0, "single", "i8x5")
    sc.sincosm_eval_planned(A, C1, S1, p, "single", "i8x5")
    torch.cuda.synchronize()
    assert torch.equal(C0, C1) and torch.equal(S0, S1)
    sc.sincosm_eval(A, C1, S1, "single", "i8x5", refined=True)
    torch.cuda.synchronize()
    Cr, Sr = R.sincosm(A.cpu().numpy())
    assert rel_fro(C1.cpu().numpy(), Cr) <= 5e-6 and rel_fro(S1.cpu().numpy(), Sr) <= 5e-6


def test_i8x5_largest_order_int32_range(env):
    """n = 16384, the largest order the int8 products take, with every digit at its largest
    magnitude (all entries 1 - 2^-36: five digits of 127 each), so each of the five int32 sums
    reaches its bound 5 n 127^2 = 1.32e9 < 2^31 and the digit products left out reach theirs
    (gate T1 + T2); sampled rows of a Gaussian product of the same order against the float64 host
    product (gate 2 T1)."""
    torch, sc = env
    n = 16384
    say("i8x5 largest order", n)
    v = 1.0 - 2.0 ** -36
    X = torch.full((n, n), v, dtype=torch.float64, device="cuda")
    Z = torch.empty_like(X)
    sc.sincosm_matmul(X, X, Z, products="i8x5")
    torch.cuda.synchronize()
    exact = n * v * v
    zr = Z[::4097, ::4097].cpu().numpy()
    bound = 2.0 ** -34 * 2 * n * v * v + 2.0 ** -31 * n * v * v
    say("constant product worst error / (T1 + T2)", float(np.abs(zr - exact).max() / bound))
    assert np.abs(zr - exact).max() <= bound
    del X
    g = W.rng(184, n)
    Xg = torch.from_numpy(g.standard_normal((n, n))).cuda()
    Yg = torch.from_numpy(g.standard_normal((n, n))).cuda()
    sc.sincosm_matmul(Xg, Yg, Z, products="i8x5")
    torch.cuda.synchronize()
    rows = np.array([0, 1, 5000, 9999, n - 2, n - 1])
    Xr = Xg[rows].cpu().numpy()
    Yh = Yg.cpu().numpy()
    Zr = Xr @ Yh
    aY = np.abs(Yh)
    bound = 2.0 ** -34 * (np.outer(np.abs(Xr).max(1), aY.sum(0)) + np.outer(np.abs(Xr).sum(1), aY.max(0)))
    err = np.abs(Z[rows].cpu().numpy() - Zr)
    ratio = float((err / (2.0 * bound)).max())
    say("sampled rows worst error / (2 bound)", ratio)
    assert ratio <= 1.0


@pytest.mark.parametrize("n", [1, 63, 64, 65])
def test_i8x5_small_orders(env, n):
    """Orders at and around one 64 x 64 tile (and n = 1) against the float64 oracle at the
    single bar."""
    torch, sc = env
    say("i8x5 small order", n)
    A = W.gaussian(n, 3.0, key=(185, n))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    sc.sincosm_eval(At, C, S, "single", "i8x5")
    torch.cuda.synchronize()
    Cr, Sr = R.sincosm(A)
    assert rel_fro(C.cpu().numpy(), Cr) <= 5e-6 and rel_fro(S.cpu().numpy(), Sr) <= 5e-6


def test_i8x5_noalloc_matches_planned(env):
    """The entry point that allocates nothing with int8 products: bitwise equal to
    sincosm_eval_planned, on two calls in a row (the second of smaller order) sharing the
    library's scratch."""
    torch, sc = env
    for n in (300, 130):
        say("i8x5 noalloc", n)
        A = torch.from_numpy(W.gaussian(n, 12.0, key=(186, n))).cuda()
        plan = sc.plan_host(float(A.abs().sum(0).max()), "single")
        C0, S0 = torch.empty_like(A), torch.empty_like(A)
        C1, S1 = torch.full_like(A, 7.0), torch.full_like(A, 7.0)
        sc.sincosm_eval_planned(A, C0, S0, plan, "single", "i8x5")
        sc.sincosm_eval_planned_noalloc(A, C1, S1, plan, "single", "i8x5")
        torch.cuda.synchronize()
        assert torch.equal(C0, C1) and torch.equal(S0, S1)


@pytest.mark.parametrize("n,e", [(64, 1), (300, 6), (1000, 9)])
def test_i8x5_wave_pair(env, n, e):
    """The wave pair c(t^2 A), s(t, A) (Section 2.2) with int8 scheme products: the
    single-accuracy bar against the oracle (s up to 4 here: ||B||_1 = 2^9)."""
    from oracle import wave as Wv
    torch, sc = env
    say("i8x5 wave", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(187, n))
    C, S = sc.wave(torch.from_numpy(A).cuda(), 1.0, "single", "i8x5")
    Cr, Sr = Wv.reference(A, 1.0)
    assert rel_fro(C.cpu().numpy(), Cr) <= 5e-6 and rel_fro(S.cpu().numpy(), Sr) <= 5e-6


@pytest.mark.parametrize("n,e", [(64, 1), (300, 6)])
def test_i8x5_propagators(env, n, e):
    """e^{-itA} and the block propagator e^{tM} with int8 scheme products against the oracle
    at the single-accuracy bar; the device-planned e^{-itA} gives bitwise the same result."""
    from oracle import propagators as Pr
    torch, sc = env
    say("i8x5 propagators", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(188, n))
    At = torch.from_numpy(A).cuda()
    U = sc.expi(At, 1.0, "single", "i8x5")
    assert rel_fro(U.cpu().numpy(), Pr.unitary(A, 1.0)) <= 5e-6
    E = sc.wave_block(At, 1.0, "single", "i8x5")
    assert rel_fro(E.cpu().numpy(), Pr.symplectic(A, 1.0)) <= 5e-6
    Ua = torch.full((n, n), 3.0, dtype=torch.complex128, device="cuda")
    sc.sincosm_expi_eval_async(At, 1.0, Ua, accuracy="single", products="i8x5")
    torch.cuda.synchronize()
    assert torch.equal(Ua, U)


def _sync_async(env, A, s_max=16):
    torch, sc = env
    C0, S0 = torch.empty_like(A), torch.empty_like(A)
    p0 = sc.sincosm_eval(A, C0, S0, "single", "i8x5")
    C1, S1 = torch.full_like(A, 5.0), torch.full_like(A, 5.0)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    sc.sincosm_eval_async(A, C1, S1, s_max, "single", "i8x5", plan_dev=pd)
    torch.cuda.synchronize()
    return (C0, S0, p0), (C1, S1, sc.plan_from_device(pd))


@pytest.mark.parametrize("n", [100, 400])
@pytest.mark.parametrize("e", [-7.0, -2.0, 0.5, 3.0, 8.0])
def test_i8x5_async_equals_sync(env, n, e):
    """sincosm_eval_async with int8 products (the plan decided on the device; slot launches of
    alternative levels, each int8 kernel leaving when the record rules it out): the same plan
    and bitwise the same cos and sin as sincosm_eval."""
    torch, sc = env
    say("i8x5 async", n, e)
    A = torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(189, n, int(e) + 10))).cuda()
    (C0, S0, p0), (C1, S1, p1) = _sync_async(env, A)
    assert (p1.level, p1.s, p1.status) == (p0.level, p0.s, 0)
    assert torch.equal(C0, C1) and torch.equal(S0, S1)


def test_i8x5_async_graph_capture(env):
    """Captured once with no plan known, replayed on inputs whose plans differ, with eager work
    between the replays: each replay equals sincosm_eval with int8 products bitwise."""
    torch, sc = env
    n = 192
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(A), torch.empty_like(A)
    ws = torch.empty(sc.workspace_size(n, torch.float64, "single", "i8x5"), dtype=torch.uint8, device="cuda")
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.sincosm_eval_async(A, C, S, 8, "single", "i8x5", ws=ws, plan_dev=pd)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sincosm_eval_async(A, C, S, 8, "single", "i8x5", ws=ws, plan_dev=pd)
    seen = set()
    for k, e in enumerate([-5.0, 0.5, 3.0, 7.0]):
        say("i8x5 async graph replay", e)
        A.copy_(torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(190, k))).cuda())
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        junk = junk @ junk
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rec = sc.plan_from_device(pd)
        Ce, Se = torch.empty_like(A), torch.empty_like(A)
        pe = sc.sincosm_eval(A, Ce, Se, "single", "i8x5")
        torch.cuda.synchronize()
        assert (rec.level, rec.s, rec.status) == (pe.level, pe.s, 0)
        assert torch.equal(C, Ce) and torch.equal(S, Se), e
        seen.add((rec.level, rec.s))
    assert len(seen) == 4


@pytest.mark.parametrize("n,e", [(64, 1), (300, 6)])
def test_i8x5_wave_async(env, n, e):
    """The device-planned wave pair and block with int8 products against the oracle at the
    single-accuracy bar."""
    from oracle import wave as Wv
    from oracle import propagators as Pr
    torch, sc = env
    say("i8x5 wave async", n, e)
    A = W.gaussian(n, 2.0 ** e, key=(191, n))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    sc.sincosm_wave_eval_async(At, 1.0, C, S, 8, "single", "i8x5")
    E = torch.empty(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    sc.sincosm_wave_block_eval_async(At, 1.0, E, 8, "single", "i8x5")
    torch.cuda.synchronize()
    Cr, Sr = Wv.reference(A, 1.0)
    assert rel_fro(C.cpu().numpy(), Cr) <= 5e-6 and rel_fro(S.cpu().numpy(), Sr) <= 5e-6
    assert rel_fro(E.cpu().numpy(), Pr.symplectic(A, 1.0)) <= 5e-6


def test_i8x5_product_nonfinite_rows_and_columns(env):
    """sincosm_matmul with int8 products: a row of X holding NaN and a column of Y holding Inf
    give a NaN row and column of Z (where a float64 product is non-finite too); every other
    entry stays within the product bound."""
    torch, sc = env
    n = 130
    g = W.rng(192, n)
    X = g.standard_normal((n, n))
    Y = g.standard_normal((n, n))
    Zr = X @ Y
    X[5, 7] = np.nan
    Y[3, 11] = np.inf
    Z = torch.empty(n, n, dtype=torch.float64, device="cuda")
    sc.sincosm_matmul(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), Z, products="i8x5")
    torch.cuda.synchronize()
    Zg = Z.cpu().numpy()
    assert np.isnan(Zg[5]).all() and np.isnan(Zg[:, 11]).all()
    keep = np.ones((n, n), bool)
    keep[5] = False
    keep[:, 11] = False
    assert np.isfinite(Zg[keep]).all()
    Xf, Yf = np.nan_to_num(X, nan=0.0), np.nan_to_num(Y, posinf=0.0)
    aX, aY = np.abs(Xf), np.abs(Yf)
    bound = 2.0 ** -34 * (np.outer(aX.max(1), aY.sum(0)) + np.outer(aX.sum(1), aY.max(0)))
    assert (np.abs(Zg - Zr)[keep] <= 2.0 * bound[keep]).all()


@pytest.mark.parametrize("norm", [0.1, 0.8, 40.0])
def test_i8x5_extended_plan(env, norm):
    """The extended plan (the 5-product scheme among the candidates) with int8 products:
    against the float64 oracle at the single-accuracy bar, and the device-planned form
    bitwise equal to the synchronous one."""
    torch, sc = env
    n = 200
    say("i8x5 extended", norm)
    A = W.gaussian(n, norm, key=(193, int(norm * 10)))
    At = torch.from_numpy(A).cuda()
    C, S = torch.empty_like(At), torch.empty_like(At)
    p = sc.sincosm_eval(At, C, S, "single", "i8x5", extended=True)
    C1, S1 = torch.full_like(At, 2.0), torch.full_like(At, 2.0)
    sc.sincosm_eval_async(At, C1, S1, 8, "single", "i8x5", extended=True)
    torch.cuda.synchronize()
    Cr, Sr = R.sincosm(A)
    say("i8x5 extended plan", p.level, p.s)
    assert rel_fro(C.cpu().numpy(), Cr) <= 5e-6 and rel_fro(S.cpu().numpy(), Sr) <= 5e-6
    assert torch.equal(C, C1) and torch.equal(S, S1)


def _emulate_i8x5(X, Y):
    """The int8 product's arithmetic on the CPU: per-row (X) and per-column (Y) exponents from
    the largest magnitude, five 7-bit digits d = trunc(128 y) with y <- 128 y - d (exact in
    float64), the digit products of each weight k + l <= 4 (slice indices from 0) summed
    exactly (int64 here), and the five sums combined in float64 from the smallest weight up,
    then scaled by 2^(e_i + f_j)."""
    def digits(M, axis):
        m = np.abs(M).max(axis=axis, keepdims=True)
        e = np.where(m > 0, np.frexp(m)[1], 0)
        y = np.ldexp(M, -e)
        ds = []
        for _ in range(5):
            t = y * 128.0
            q = np.trunc(t)
            ds.append(q.astype(np.int64))
            y = t - q
        return ds, e
    D, e = digits(X, 1)
    E, f = digits(Y, 0)
    v = np.zeros((X.shape[0], Y.shape[1]))
    for g in range(4, -1, -1):
        S = sum(D[k] @ E[g - k] for k in range(g + 1))
        v = v + np.ldexp(S.astype(np.float64), -7 * (g + 2))
    return np.ldexp(v, e + f)


@pytest.mark.parametrize("n,kind", [(64, "gaussian"), (100, "graded"), (257, "gaussian")])
def test_i8x5_product_bitwise_emulation(env, n, kind):
    """sincosm_matmul with int8 products equals the CPU emulation of its arithmetic bit for bit
    (the int32 sums are exact, and the float64 combination has a fixed order)."""
    torch, sc = env
    say("i8x5 emulation", n, kind)
    g = W.rng(194, n, 0 if kind == "gaussian" else 1)
    X = g.standard_normal((n, n))
    Y = g.standard_normal((n, n))
    if kind == "graded":
        X *= np.exp2(g.integers(-30, 30, size=(n, 1)))
        Y *= np.exp2(g.integers(-30, 30, size=(1, n)))
    Z = torch.empty(n, n, dtype=torch.float64, device="cuda")
    sc.sincosm_matmul(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), Z, products="i8x5")
    torch.cuda.synchronize()
    assert np.array_equal(Z.cpu().numpy(), _emulate_i8x5(X, Y))


def test_i8x5_seeded_sweep(env):
    """24 seeded draws (order uniform on 16 ... 400, ||A||_1 = 2^e with e uniform on [-6, 8],
    Gaussian, symmetric and 1-D Laplacian families): every single-plan evaluation with int8
    products within the single-accuracy bar against the float64 oracle."""
    torch, sc = env
    g = W.rng(195)
    worst = 0.0
    for k in range(24):
        n = int(g.integers(16, 401))
        e = float(g.uniform(-6.0, 8.0))
        fam = ("gaussian", "symmetric", "laplacian1d")[k % 3]
        A = W.family(fam, n, 2.0 ** e, key=(195, k))
        At = torch.from_numpy(A).cuda()
        C, S = torch.empty_like(At), torch.empty_like(At)
        p = sc.sincosm_eval(At, C, S, "single", "i8x5")
        torch.cuda.synchronize()
        Cr, Sr = R.sincosm(A)
        err = max(rel_fro(C.cpu().numpy(), Cr), rel_fro(S.cpu().numpy(), Sr))
        say("i8x5 sweep", k, fam, n, round(e, 2), p.level, p.s, err)
        worst = max(worst, err)
        assert err <= 5e-6, (k, fam, n, e)
    say("i8x5 sweep worst", worst)
