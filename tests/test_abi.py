"""C-ABI library checks that need no GPU: it loads, exports every function the
header declares, and its host plan rule agrees with the oracle's."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sincosm.h")
LIB = os.path.join(ROOT, "paper_2010_00465_amd", "libsincosm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sincosm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsincosm.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2010_00465_amd import _lib
    assert sorted(_lib.SYMBOLS) == declared_functions()


class Plan(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("s", ctypes.c_int32), ("products", ctypes.c_int32),
                ("status", ctypes.c_int32), ("norm1", ctypes.c_double)]


def host_plan(lib, t, acc):
    p = Plan()
    lib.sincosm_plan_host.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.POINTER(Plan)]
    assert lib.sincosm_plan_host(t, acc, ctypes.byref(p)) == 0
    return p


def test_host_plan_matches_oracle_fixture(lib):
    with open(os.path.join(ROOT, "tests", "golden", "plan_breakpoints.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        t = float.fromhex(c["norm1"])
        p = host_plan(lib, t, 0 if c["accuracy"] == "double" else 1)
        assert (p.level, p.s, p.products, p.status) == (c["level"], c["s"], c["products"], 0), c


def test_host_plan_matches_oracle_random(lib):
    from oracle import plan as P
    ts = np.exp2(np.random.default_rng(5).uniform(-40, 60, size=4000))
    for t in ts:
        for acc, name in ((0, "double"), (1, "single")):
            p = host_plan(lib, float(t), acc)
            assert (p.level, p.s, p.products) == P.plan(float(t), name)


def test_host_plan_nonfinite(lib):
    for t in (math.nan, math.inf, -1.0):
        p = host_plan(lib, t, 0)
        assert p.status == -4


def test_argument_errors_without_gpu(lib):
    lib.sincosm_workspace_size.restype = ctypes.c_size_t
    lib.sincosm_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    assert lib.sincosm_workspace_size(0, 0, 0, 0) == 0
    assert lib.sincosm_workspace_size(64, 7, 0, 0) == 0          # bad dtype
    assert lib.sincosm_workspace_size(64, 0, 0, 0) > 10 * 64 * 64 * 8
    lib.sincosm_strerror.restype = ctypes.c_char_p
    assert lib.sincosm_strerror(-3) == b"workspace missing or too small"
    lib.sincosm_plan_host.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
    assert lib.sincosm_plan_host(1.0, 5, None) == -1


def test_wave_host_plan_matches_oracle(lib):
    """The library's wave plan rule against the oracle's, including values at and next to every
    bound times a power of four (where s steps)."""
    from oracle import wave as Wv
    lib.sincosm_wave_plan_host.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.POINTER(Plan)]
    xs = list(np.exp2(np.random.default_rng(6).uniform(-40, 80, size=3000)))
    for acc in ("double", "single"):
        for th in Wv.WAVE_THETA[acc].values():
            for k in range(0, 12):
                b = th * 4.0 ** k
                xs += [b, math.nextafter(b, math.inf), math.nextafter(b, 0.0)]
    for x in xs:
        for code, name in ((0, "double"), (1, "single")):
            p = Plan()
            assert lib.sincosm_wave_plan_host(float(x), code, ctypes.byref(p)) == 0
            assert (p.level, p.s, p.products, p.status) == (*Wv.wave_plan(float(x), name), 0), (x, name)
    p = Plan()
    assert lib.sincosm_wave_plan_host(math.nan, 0, ctypes.byref(p)) == 0 and p.status == -4


def test_host_plan_extended_matches_oracle(lib):
    """With SINCOSM_PLAN_EXTENDED the host rule equals the oracle's extended plan; flagged
    accuracy codes are rejected by the wave plan."""
    from oracle import plan as P
    ext = 16
    xs = list(np.exp2(np.random.default_rng(9).uniform(-30, 40, size=3000)))
    for acc in ("double", "single"):
        for th in list(P.THETA[acc].values()) + [P.THETA_LEVEL5[acc]]:
            for k in range(10):
                b = math.ldexp(th, k)
                xs += [b, math.nextafter(b, math.inf), math.nextafter(b, 0.0)]
    for x in xs:
        for code, name in ((0, "double"), (1, "single")):
            p = host_plan(lib, float(x), code | ext)
            assert (p.level, p.s, p.products) == P.plan(float(x), name, extended=True), (x, name)
    lib.sincosm_wave_plan_host.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.POINTER(Plan)]
    assert lib.sincosm_wave_plan_host(1.0, ext, ctypes.byref(Plan())) == -1


def test_planned_argument_errors_without_gpu(lib):
    """sincosm_eval_planned rejects a bad plan or arguments before any device work."""
    f = lib.sincosm_eval_planned
    f.restype = ctypes.c_int
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    f.argtypes = [i64, ctypes.c_int, vp, i64, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Plan),
                  vp, ctypes.c_size_t, vp, vp]
    fake = 1 << 40            # never dereferenced: every call below fails validation first

    def call(level, s, acc=0, n=64, plan=True, ws=fake):
        p = Plan(level, s, 0, 0, 0.0)
        return f(n, 0, fake, n, fake + 2 ** 20, n, fake + 2 ** 21, n, acc, 0, ctypes.byref(p) if plan else None,
                 ws, 1 << 30, None, None)

    assert call(5, 0) == -1                  # level 5 without the extended flag
    assert call(2, 0) == -1 and call(8, 0) == -1
    assert call(7, -1) == -1 and call(7, 1101) == -1
    assert call(7, 3, plan=False) == -1
    assert call(7, 3, acc=32) == -1          # the refined flag is not accepted here
    assert call(7, 3, acc=7) == -1
    assert call(7, 3, n=-1) == -1
    assert call(7, 3, ws=None) == -3         # workspace missing
    assert call(7, 3, n=0) == 0              # n = 0 is a no-op
    lib.sincosm_strerror.restype = ctypes.c_char_p
    assert lib.sincosm_strerror(-6) == b"the given plan does not cover the matrix 1-norm"


def test_batched_argument_errors_without_gpu(lib):
    """Argument checks of the batched entry points that come before any device work."""
    i32 = ctypes.c_int32
    ns = (i32 * 3)(4, 17, 256)
    bad_n = (i32 * 2)(4, 257)
    zero_n = (i32 * 2)(0, 5)
    lib.sincosm_batched_workspace_size.restype = ctypes.c_size_t
    assert lib.sincosm_batched_workspace_size(0, ns, 0, 0, 0) == 0          # empty batch
    assert lib.sincosm_batched_workspace_size(2, bad_n, 0, 0, 0) == 0       # order above 256
    assert lib.sincosm_batched_workspace_size(2, zero_n, 0, 0, 0) == 0      # order 0
    assert lib.sincosm_batched_workspace_size(3, ns, 7, 0, 0) == 0          # bad dtype
    assert lib.sincosm_batched_workspace_size(3, ns, 0, 0, 2) == 0          # products other than native
    # sincosm_eval_batched: an empty batch is a no-op; bad sizes, enums and workspaces fail
    i64 = ctypes.c_int64
    call = lib.sincosm_eval_batched
    call.argtypes = [i64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, i64, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                     ctypes.c_void_p, ctypes.c_void_p]
    buf = ctypes.create_string_buffer(1024)
    p = ctypes.cast(buf, ctypes.c_void_p).value
    aligned = (p + 255) // 256 * 256
    assert call(0, 0, None, None, 0, None, None, None, 0, 0, None, 0, None, None) == 0
    assert call(-1, 0, p, p, 9, p, p, p, 0, 0, p, 64, None, None) == -1         # negative batch
    assert call(3, 0, p, p, -1, p, p, p, 0, 0, p, 64, None, None) == -1         # negative extent
    assert call(3, 0, p, p, 9, p, p, p, 9, 0, p, 64, None, None) == -1          # bad accuracy
    assert call(3, 5, p, p, 9, p, p, p, 0, 0, p, 64, None, None) == -1          # bad dtype
    assert call(3, 0, p, p, 9, p, p, p, 0, 2, p, 64, None, None) == -2          # unsupported products
    assert call(3, 0, None, p, 9, p, p, p, 0, 0, p, 64, None, None) == -1       # missing order array
    assert call(3, 0, p, None, 9, p, p, p, 0, 0, p, 64, None, None) == -1       # missing offsets
    assert call(3, 0, p, p, 9, p, p, p, 0, 0, None, 64, None, None) == -3      # no workspace
    assert call(3, 0, p, p, 9, p, p, p, 0, 0, aligned + 8, 64, None, None) == -3   # misaligned


def test_python_host_plan_helpers():
    """The package's host plan helpers marshal to the C ABI: same integers as the oracle."""
    import paper_2010_00465_amd as sc
    from oracle import plan as P
    from oracle import wave as Wv
    for x in (0.0, 1e-3, 0.5, 1.0, 2.0, 37.5, 2.0 ** 10):
        for acc in ("double", "single"):
            p = sc.plan_host(x, acc)
            assert (p.level, p.s, p.products, p.status) == (*P.plan(x, acc), 0)
            q = sc.wave_plan_host(x, acc)
            assert (q.level, q.s, q.products, q.status) == (*Wv.wave_plan(x, acc), 0)


def test_autograd_rejects_unsupported_gradients_up_front():
    """The reverse pass is the float64 adjoint of the float64 products: asking sincosm for a
    gradient of a float32 input, or with lowered products, fails before any device work."""
    import torch
    import paper_2010_00465_amd as sc
    A32 = torch.zeros(4, 4, dtype=torch.float32, requires_grad=True)
    with pytest.raises(TypeError):
        sc.sincosm(A32)
    A64 = torch.zeros(4, 4, dtype=torch.float64, requires_grad=True)
    with pytest.raises(TypeError):
        sc.sincosm(A64, "single", "f32")


def test_device_planned_and_noalloc_argument_errors_without_gpu(lib):
    """Synchronous argument checks of sincosm_eval_async, sincosm_backward_async and
    sincosm_eval_planned_noalloc, all taken before any device work."""
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    buf = ctypes.create_string_buffer(4096)
    p = ctypes.cast(buf, vp).value
    aligned = (p + 255) // 256 * 256
    ea = lib.sincosm_eval_async
    ea.argtypes = [i64, ctypes.c_int, vp, i64, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, i32, vp,
                   ctypes.c_size_t, vp, vp]
    assert ea(0, 0, None, 0, None, 0, None, 0, 0, 0, 8, None, 0, None, None) == 0       # n = 0: no-op
    assert ea(-1, 0, p, 4, p, 4, p, 4, 0, 0, 8, p, 64, None, None) == -1                # negative n
    assert ea(4, 0, p, 4, p, 4, p, 4, 0, 0, -1, p, 64, None, None) == -1                # negative s_max
    assert ea(4, 0, p, 4, p, 4, p, 4, 0, 0, 1101, p, 64, None, None) == -1              # s_max too large
    assert ea(4, 0, p, 4, p, 4, p, 4, 32, 0, 8, p, 64, None, None) == -1                # refined flag
    assert ea(4, 0, None, 4, p, 4, p, 4, 0, 0, 8, p, 64, None, None) == -1              # no A
    assert ea(4, 0, aligned, 4, aligned + 4096, 4, aligned + 8192, 4, 0, 0, 8, None, 0, None, None) == -3
    ba = lib.sincosm_backward_async
    ba.argtypes = [i64, ctypes.c_int, vp, i64, vp, i64, vp, i64, vp, i64, ctypes.c_int, i32, vp,
                   ctypes.c_size_t, vp, vp]
    assert ba(0, 0, None, 0, None, 0, None, 0, None, 0, 0, 4, None, 0, None, None) == 0
    assert ba(4, 0, p, 4, None, 4, None, 4, p, 4, 0, -1, p, 64, None, None) == -1      # negative s_max
    assert ba(4, 1, p, 4, None, 4, None, 4, p, 4, 0, 4, p, 64, None, None) == -2       # float32
    assert ba(4, 0, p, 4, None, 4, None, 4, p, 4, 0, 4, p, 64, None, None) == -1       # gA aliases A
    na = lib.sincosm_eval_planned_noalloc
    plan = Plan()
    plan.level, plan.s = 7, 0
    na.argtypes = [i64, ctypes.c_int, vp, i64, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int,
                   ctypes.POINTER(Plan), vp, vp]
    assert na(1024, 0, p, 1024, p, 1024, p, 1024, 0, 0, ctypes.byref(plan), None, None) == -7   # too large
    assert na(-1, 0, p, 4, p, 4, p, 4, 0, 0, ctypes.byref(plan), None, None) == -1
    lib.sincosm_strerror.restype = ctypes.c_char_p
    assert b"scratch" in lib.sincosm_strerror(-7)
    assert b"double-angle" in lib.sincosm_strerror(-8)


def test_async_propagator_argument_errors_without_gpu(lib):
    """Synchronous argument checks of the device-planned wave, block and expi entry points."""
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    buf = ctypes.create_string_buffer(4096)
    p = ctypes.cast(buf, vp).value
    we = lib.sincosm_wave_eval_async
    we.argtypes = [i64, ctypes.c_int, vp, i64, dbl, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, i32, vp,
                   ctypes.c_size_t, vp, vp]
    assert we(0, 0, None, 0, 1.0, None, 0, None, 0, 0, 0, 4, None, 0, None, None) == 0
    assert we(4, 0, p, 4, 1.0, p + 1024, 4, p + 2048, 4, 0, 0, -1, p, 64, None, None) == -1   # s_max < 0
    assert we(4, 0, p, 4, float("inf"), p + 1024, 4, p + 2048, 4, 0, 0, 4, p, 64, None, None) == -1
    assert we(4, 0, p, 4, 1.0, p, 4, p + 2048, 4, 0, 0, 4, p, 64, None, None) == -1           # C aliases A
    assert we(4, 0, p, 4, 1.0, p + 1024, 4, p + 2048, 4, 0, 0, 4, None, 0, None, None) == -3  # no workspace
    wb = lib.sincosm_wave_block_eval_async
    wb.argtypes = [i64, ctypes.c_int, vp, i64, dbl, vp, i64, ctypes.c_int, ctypes.c_int, i32, vp,
                   ctypes.c_size_t, vp, vp]
    assert wb(0, 0, None, 0, 1.0, None, 0, 0, 0, 4, None, 0, None, None) == 0
    assert wb(4, 0, p, 4, 1.0, p + 1024, 7, 0, 0, 4, p, 64, None, None) == -1                # lde < 2n
    assert wb(4, 0, p, 4, 1.0, p + 1024, 8, 0, 0, 1101, p, 64, None, None) == -1             # s_max too large
    ex = lib.sincosm_expi_eval_async
    ex.argtypes = [i64, ctypes.c_int, vp, i64, dbl, vp, i64, ctypes.c_int, ctypes.c_int, i32, vp,
                   ctypes.c_size_t, vp, vp]
    assert ex(0, 0, None, 0, 1.0, None, 0, 0, 0, 4, None, 0, None, None) == 0
    assert ex(4, 0, p, 4, float("nan"), p + 1024, 4, 0, 0, 4, p, 64, None, None) == -1
    u_odd = (p + 1024) // 16 * 16 + 8                                                      # not 16-byte aligned
    assert ex(4, 0, p, 4, 1.0, u_odd, 4, 0, 0, 4, p, 64, None, None) == -1
    assert ex(4, 0, p, 4, 1.0, p + 1024, 4, 32, 0, 4, p, 64, None, None) == -1               # refined flag
    assert ex(4, 0, p, 4, 1.0, p + 1024, 4, 0, 0, 4, None, 0, None, None) == -3


def test_int8_product_tier_sizes_and_rejections_without_gpu(lib):
    """SINCOSM_PROD_I8X5: float64 storage only, n <= 16384 (int32 accumulation of the slice
    products); its workspace adds the slice planes (10 np^2 bytes and the exponents); the
    batched pass rejects it before any GPU call."""
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    ws = lib.sincosm_workspace_size
    ws.restype, ws.argtypes = sz, [i64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    for n in (64, 1000, 4096):
        np_ = 64 * ((n + 63) // 64) if n < 1536 else 128 * ((n + 127) // 128)
        assert ws(n, 0, 1, 3) >= ws(n, 0, 1, 0) + 10 * np_ * np_
    assert ws(64, 1, 1, 3) == 0              # float32 storage
    assert ws(16384, 0, 1, 3) > 0 and ws(16385, 0, 1, 3) == 0
    mw = lib.sincosm_matmul_workspace_size
    mw.restype, mw.argtypes = sz, [i64, ctypes.c_int, ctypes.c_int]
    assert mw(1000, 0, 3) >= mw(1000, 0, 0) + 10 * 1024 * 1024
    bws = lib.sincosm_batched_workspace_size
    bws.restype, bws.argtypes = sz, [i64, ctypes.POINTER(i32), ctypes.c_int, ctypes.c_int, ctypes.c_int]
    ns = (i32 * 2)(16, 32)
    assert bws(2, ns, 0, 0, 3) == 0          # the batched pass takes native products only
