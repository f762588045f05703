"""GPU parity of sincosm_backward (through the C ABI) against the oracle's
derivative references: the dual-number Frechet derivative at A^T (equal to the
block-triangular form, pinned in tests/test_oracle_frechet.py), central finite
differences, and the directional identity <dL/dA, A> = <Gc, -A sin A> + <Gs, A cos A>.

Bar: relative Frobenius error <= 1e-12 against the oracle gradient (both are
float64 evaluations of the same derivative; the oracle uses its own Taylor
degree and scaling, so the two differ by rounding amplified by the s squarings;
measured at most 9.1e-15 over these cases, at n = 2048, ||A||_1 = 128, s = 7)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import frechet as F
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


def grad(env, A, Gc, Gs):
    torch, sc = env
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    gc = torch.from_numpy(Gc).cuda() if Gc is not None else None
    gs = torch.from_numpy(Gs).cuda() if Gs is not None else None
    gA = torch.empty_like(At)
    plan = sc.sincosm_backward(At, gc, gs, gA)
    torch.cuda.synchronize()
    return gA.cpu().numpy(), plan


@pytest.mark.parametrize("n", [16, 70, 130])
@pytest.mark.parametrize("e", [-9.0, -5.0, -1.0, 0.5, 1.0, 3.0, 7.0])
def test_backward_vs_oracle(env, n, e):
    print("[case] backward", n, e, flush=True)
    A = W.gaussian(n, 2.0 ** e, key=(60, n, int(e * 2) + 40))
    g = W.rng(61, n, int(e * 2) + 40)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    gA, plan = grad(env, A, Gc, Gs)
    ref = F.dual_gradient(A, Gc, Gs)
    assert rel_fro(gA, ref) <= 1e-12, (plan, rel_fro(gA, ref))


@pytest.mark.parametrize("which", ["cos", "sin"])
def test_backward_one_sided(env, which):
    n = 50
    A = W.gaussian(n, 5.0, key=(62,))
    G = W.rng(63).standard_normal((n, n))
    Gc, Gs = (G, None) if which == "cos" else (None, G)
    gA, _ = grad(env, A, Gc, Gs)
    ref = F.dual_gradient(A, Gc, Gs)
    assert rel_fro(gA, ref) <= 1e-12


@pytest.mark.parametrize("n,norm", [(256, 0.5), (256, 8.0), (256, 128.0), (1024, 0.5), (1024, 8.0), (1024, 128.0),
                                    (2048, 0.5), (2048, 8.0), (2048, 128.0)])
def test_backward_config_sizes(env, n, norm):
    print("[case] backward config", n, norm, flush=True)
    A = W.gaussian(n, norm, key=(4, n, int(norm * 2)))
    g = W.rng(64, n, int(norm * 2))
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    gA, plan = grad(env, A, Gc, Gs)
    ref = F.dual_gradient(A, Gc, Gs)
    assert rel_fro(gA, ref) <= 1e-12, (plan, rel_fro(gA, ref))


@pytest.mark.parametrize("n,e", [(16, 1.0), (40, -3.0), (70, 3.0), (130, 7.0)])
def test_backward_vs_block_form(env, n, e):
    """Against the block-triangular form: L_f(A^T, G) is the top-right block of
    f([[A^T, G], [0, A^T]]), evaluated by the independent Taylor reference on 2n x 2n."""
    print("[case] backward block", n, e, flush=True)
    A = W.gaussian(n, 2.0 ** e, key=(71, n, int(e * 2) + 40))
    g = W.rng(72, n, int(e * 2) + 40)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    gA, plan = grad(env, A, Gc, Gs)
    ref = F.block_gradient(A, Gc, Gs)
    assert rel_fro(gA, ref) <= 1e-12, (plan, rel_fro(gA, ref))


@pytest.mark.parametrize("n,norm", [(256, 0.5), (256, 8.0), (256, 128.0)])
def test_backward_config_block_form(env, n, norm):
    """The configured n = 256 cases against the block form (a 512 x 512 reference)."""
    print("[case] backward config block", n, norm, flush=True)
    A = W.gaussian(n, norm, key=(4, n, int(norm * 2)))
    g = W.rng(64, n, int(norm * 2))
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    gA, plan = grad(env, A, Gc, Gs)
    ref = F.block_gradient(A, Gc, Gs)
    assert rel_fro(gA, ref) <= 1e-12, (plan, rel_fro(gA, ref))


def _fd_check(env, A, Gc, Gs, g, directions, h=1e-6):
    """Central differences of the loss along unit-Frobenius directions E, with the plan
    frozen along the difference, against <dL/dA, E>. Returns the worst relative gap."""
    torch, sc = env
    gA, plan = grad(env, A, Gc, Gs)
    gct = torch.from_numpy(Gc).cuda()
    gst = torch.from_numpy(Gs).cuda()

    def loss(M):
        t = torch.from_numpy(M).cuda()
        C = torch.empty_like(t)
        S = torch.empty_like(t)
        p = sc.sincosm_eval(t, C, S)
        assert p.s == plan.s and p.level == plan.level   # plan frozen along the difference
        return float((C * gct).sum() + (S * gst).sum())

    worst = 0.0
    for _ in range(directions):
        E = g.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (loss(A + h * E) - loss(A - h * E)) / (2 * h)
        an = float((gA * E).sum())
        worst = max(worst, abs(fd - an) / max(1.0, np.linalg.norm(gA)))
    return worst


def test_backward_finite_differences(env):
    torch, sc = env
    n = 40
    A = W.gaussian(n, 6.0, key=(65,))
    g = W.rng(66)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    gA, plan = grad(env, A, Gc, Gs)

    def loss(M):
        t = torch.from_numpy(M).cuda()
        C = torch.empty_like(t)
        S = torch.empty_like(t)
        p = sc.sincosm_eval(t, C, S)
        assert p.s == plan.s and p.level == plan.level   # plan frozen along the difference
        return float((C.cpu().numpy() * Gc).sum() + (S.cpu().numpy() * Gs).sum())

    for i in range(3):
        E = g.standard_normal((n, n))
        E /= np.linalg.norm(E)
        h = 1e-6
        fd = (loss(A + h * E) - loss(A - h * E)) / (2 * h)
        an = float((gA * E).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, np.linalg.norm(gA)), (fd, an)


def test_backward_directional_identity(env):
    n = 64
    A = W.gaussian(n, 3.0, key=(67,))
    g = W.rng(68)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    gA, _ = grad(env, A, Gc, Gs)
    C, S = R.sincosm(A)
    lhs = float((gA * A).sum())
    rhs = float((Gc * (-A @ S)).sum() + (Gs * (A @ C)).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))


def test_autograd_function(env):
    torch, sc = env
    n = 33
    A = torch.from_numpy(W.gaussian(n, 2.5, key=(69,))).cuda().requires_grad_(True)
    C, S = sc.sincosm(A)
    g = W.rng(70)
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    loss = (C * torch.from_numpy(Gc).cuda()).sum() + (S * torch.from_numpy(Gs).cuda()).sum()
    loss.backward()
    ref = F.dual_gradient(A.detach().cpu().numpy(), Gc, Gs)
    assert rel_fro(A.grad.cpu().numpy(), ref) <= 1e-12


def test_backward_nonfinite_and_errors(env):
    torch, sc = env
    A = torch.zeros(10, 10, dtype=torch.float64, device="cuda")
    A[1, 1] = float("nan")
    gA = torch.zeros_like(A)
    G = torch.ones_like(A)
    with pytest.raises(sc.SincosmError) as ei:
        sc.sincosm_backward(A, G, G, gA, s=0)
    assert ei.value.status == -4
    assert torch.isnan(gA).all()
    with pytest.raises(sc.SincosmError) as ei:
        sc.sincosm_backward(A.float(), G.float(), G.float(), gA.float(), s=0)
    assert ei.value.status == -2


@pytest.mark.parametrize("n,norm", [(256, 0.5), (256, 8.0), (256, 128.0), (1024, 0.5), (1024, 8.0), (1024, 128.0),
                                    (2048, 0.5), (2048, 8.0), (2048, 128.0)])
def test_backward_finite_differences_config_sizes(env, n, norm):
    """Central differences (h = 1e-6) along 4 seeded directions at the configured sizes.
    The gap is FD's own truncation (h^2) and cancellation (u |L| / h) error, so the bar
    is 1e-6 relative to ||dL/dA||_F."""
    print("[case] backward fd", n, norm, flush=True)
    A = W.gaussian(n, norm, key=(4, n, int(norm * 2)))
    g = W.rng(64, n, int(norm * 2))
    Gc, Gs = g.standard_normal((n, n)), g.standard_normal((n, n))
    worst = _fd_check(env, A, Gc, Gs, W.rng(73, n, int(norm * 2)), 4)
    assert worst <= 1e-6, worst
