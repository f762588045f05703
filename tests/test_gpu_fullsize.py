"""Full-size parity (n = 8192, and the 2n = 8192 block at n = 4096) on the wave-equation
family A = c tridiag(-1, 2, -1), whose matrix functions have the closed form
V f(c Lambda) V^T (oracle/closed_forms.py): sampled rows of every output are compared with
the exact values, in the launch configuration the product kernels use at that order.

The precision tiers are checked the same way on the 2-D Laplacian of a 90 x 90 grid
(n = 8100), whose eigenvectors are Kronecker products of the 1-D ones.

Bars: relative Frobenius error over the sampled rows <= 1e-12 for the float64 double-accuracy
paths (the float64 CPU oracle itself stays at 4e-13 on this family up to ||A||_1 = 2^10);
<= 5e-6 for float32 storage with the single-accuracy plan; the tier bounds stated at
test_tiers_laplacian_2d_n8100."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import plan as P
from oracle import wave as Wv
from tests.conftest import rel_fro

pytestmark = pytest.mark.gpu

N = 8192


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_00465_amd as sc
    return torch, sc


@pytest.fixture(scope="module")
def eig():
    cache = {}

    def get(n):
        if n not in cache:
            cache[n] = CF.laplacian_1d_eig(n)
        return cache[n]
    return get


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def sample_rows(n, seed):
    g = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, 1, n // 2, n - 1], g.integers(0, n, size=4)]))


def rows_of(eig, n, rows, f):
    lam, V = eig(n)
    return (V[rows] * f(lam)) @ V.T


def lap(torch, n, target, dtype):
    return torch.from_numpy(W.laplacian_1d(n, target)).cuda().to(dtype)


@pytest.mark.parametrize("e", [-4, 4, 10])
def test_sincosm_f64_n8192(env, eig, e):
    torch, sc = env
    say("full size sincosm f64", N, e)
    A = lap(torch, N, 2.0 ** e, torch.float64)
    C, S = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_eval(A, C, S)
    assert (plan.level, plan.s, plan.products) == P.plan(2.0 ** e)
    c = 2.0 ** e / 4.0
    rows = sample_rows(N, 1 + e + 10)
    Cr = rows_of(eig, N, rows, lambda l: np.cos(c * l))
    Sr = rows_of(eig, N, rows, lambda l: np.sin(c * l))
    ec = rel_fro(C[rows].cpu().numpy(), Cr)
    es = rel_fro(S[rows].cpu().numpy(), Sr)
    print(f"n={N} e={e} plan={plan.level},{plan.s} rel err rows cos {ec:.2e} sin {es:.2e}")
    assert ec <= 1e-12 and es <= 1e-12


def test_sincosm_f32_single_n8192(env, eig):
    torch, sc = env
    say("full size sincosm f32", N)
    e = 4
    A = lap(torch, N, 2.0 ** e, torch.float32)
    C, S = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_eval(A, C, S, "single")
    c = 2.0 ** e / 4.0
    rows = sample_rows(N, 2)
    Cr = rows_of(eig, N, rows, lambda l: np.cos(c * l))
    Sr = rows_of(eig, N, rows, lambda l: np.sin(c * l))
    tol = 5e-6
    assert rel_fro(C[rows].double().cpu().numpy(), Cr) <= tol
    assert rel_fro(S[rows].double().cpu().numpy(), Sr) <= tol


def test_sincosm_gaussian_identities_n8192(env):
    """Gaussian n = 8192 at ||A||_1 = 16 (15 products): cos^2 + sin^2 = I and CS = SC."""
    torch, sc = env
    say("full size gaussian identities", N)
    A = torch.from_numpy(W.gaussian(N, 16.0, key=(2, N, 0, 4))).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_eval(A, C, S)
    assert plan.products == 15
    I = torch.eye(N, dtype=torch.float64, device="cuda")
    denom = float(C.norm() ** 2 + S.norm() ** 2 + N ** 0.5)
    r1 = float((C @ C + S @ S - I).norm()) / denom
    r2 = float((C @ S - S @ C).norm()) / denom
    assert r1 <= 8 * N * 2.0 ** -53 and r2 <= 8 * N * 2.0 ** -53, (r1, r2)


def test_wave_f64_n8192(env, eig):
    torch, sc = env
    say("full size wave", N)
    target, t = 64.0, 2.0          # ||t^2 A||_1 = 256
    A = lap(torch, N, target, torch.float64)
    C, S = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_wave_eval(A, t, C, S)
    assert (plan.level, plan.s, plan.products) == Wv.wave_plan(t * t * target)
    c = target / 4.0
    rows = sample_rows(N, 3)
    Cr = rows_of(eig, N, rows, lambda l: np.cos(t * np.sqrt(c * l)))
    Sr = rows_of(eig, N, rows, lambda l: np.sin(t * np.sqrt(c * l)) / np.sqrt(c * l))
    assert rel_fro(C[rows].cpu().numpy(), Cr) <= 1e-12
    assert rel_fro(S[rows].cpu().numpy(), Sr) <= 1e-12


def test_expi_f64_n8192(env, eig):
    torch, sc = env
    say("full size expi", N)
    target, t = 64.0, 1.0
    A = lap(torch, N, target, torch.float64)
    U = torch.empty(N, N, dtype=torch.complex128, device="cuda")
    plan = sc.sincosm_expi_eval(A, t, U)
    assert (plan.level, plan.s, plan.products) == P.plan(t * target)
    c = target / 4.0
    rows = sample_rows(N, 4)
    Ur = rows_of(eig, N, rows, lambda l: np.cos(t * c * l)) - 1j * rows_of(eig, N, rows, lambda l: np.sin(t * c * l))
    assert rel_fro(U[rows].cpu().numpy(), Ur) <= 1e-12


def test_wave_block_n4096(env, eig):
    """e^{tM}, 2n = 8192: the four blocks' rows against c, s and -A s in closed form."""
    torch, sc = env
    n = 4096
    say("full size wave block", n)
    target, t = 64.0, 1.0
    A = lap(torch, n, target, torch.float64)
    E = torch.empty(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    sc.sincosm_wave_block_eval(A, t, E)
    c = target / 4.0
    rows = sample_rows(n, 5)
    r = lambda l: np.sqrt(c * l)
    Cr = rows_of(eig, n, rows, lambda l: np.cos(t * r(l)))
    Sr = rows_of(eig, n, rows, lambda l: np.sin(t * r(l)) / r(l))
    ASr = rows_of(eig, n, rows, lambda l: r(l) * np.sin(t * r(l)))
    Eh = E.cpu().numpy()
    assert rel_fro(Eh[rows, :n], Cr) <= 1e-12
    assert rel_fro(Eh[rows, n:], Sr) <= 1e-12
    assert rel_fro(Eh[n + rows, :n], -ASr) <= 1e-12
    assert rel_fro(Eh[n + rows, n:], Cr) <= 1e-12


U32 = 2.0 ** -24
U_BF = 2.0 ** -18


@pytest.mark.parametrize("acc,prod", [("double", "native"), ("single", "native"), ("single", "f32"),
                                      ("single", "bf16x3"), ("single", "i8x5")])
def test_tiers_laplacian_2d_n8100(env, acc, prod):
    """Precision tiers on the 2-D Laplacian of a 90 x 90 grid (n = 8100), ||A||_1 = 64, float64
    storage, against the closed form (sampled rows). Bounds: 1e-12 for the float64 double path;
    5e-6 for float64 with the single table and for the int8 five-slice products (float64
    intermediates; their product error, 2^-34 of row maxima times column sums, stays far below
    the single table's); the FP32-product tier 16 Pi u_32 2^s and the BF16x3 tier 8 Pi 2^-18 2^s
    (each scheme product rounds to float32 / carries the split error, and the s float64
    double-angle steps amplify an error by about 2 each)."""
    torch, sc = env
    m = 90
    say("tiers 8100", acc, prod)
    A = torch.from_numpy(W.laplacian_2d(m, 64.0)).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    plan = sc.sincosm_eval(A, C, S, acc, prod)
    c = 64.0 / 8.0
    rows = sample_rows(m * m, 6)
    Cr = CF.laplacian_2d_rows(m, c, rows, np.cos)
    Sr = CF.laplacian_2d_rows(m, c, rows, np.sin)
    ec = rel_fro(C[rows].cpu().numpy(), Cr)
    es = rel_fro(S[rows].cpu().numpy(), Sr)
    pi = plan.level
    tol = {("double", "native"): 1e-12, ("single", "native"): 5e-6, ("single", "i8x5"): 5e-6,
           ("single", "f32"): 16 * pi * U32 * 2 ** plan.s,
           ("single", "bf16x3"): 8 * pi * U_BF * 2 ** plan.s}[(acc, prod)]
    print(f"n=8100 {acc}/{prod} plan=({plan.level},{plan.s}) rows rel err cos {ec:.2e} sin {es:.2e} tol {tol:.1e}")
    assert ec <= tol and es <= tol
