"""Simultaneous matrix cosine and sine on MI355X (gfx950).

Python face of libsincosm.so. The functions named after the C ABI
(``sincosm_eval``, ``sincosm_eval_batched``, ``sincosm_backward``,
``sincosm_matmul``, ``plan_host``) only marshal torch tensors into pointers,
sizes and the current HIP stream. ``sincosm`` adds output/workspace
allocation through torch and an autograd.Function whose backward calls
``sincosm_backward``.

Method: Seydaoglu, Bader, Blanes, Casas, arXiv 2010.00465 (scaling by 2^-s,
the factorized Taylor schemes of Section 2.1 with 3/4/6/7 products chosen
from the bounds of Tables 1-2, and s double-angle steps of Section 1).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import ACC, PROD, Plan, SincosmError, check, lib
from . import autotune as _autotune

# kernel configurations measured by the autotuner on the target (JSON cache)
TUNED_ENTRIES = _autotune.apply_cache()

__all__ = ["sincosm", "sincosm_eval", "sincosm_eval_batched", "sincosm_backward", "sincosm_matmul",
           "plan_host", "plan_device", "workspace_size", "Plan", "SincosmError", "sincosm_batched",
           "wave_plan_host", "sincosm_wave_eval", "wave", "sincosm_wave_block_eval", "wave_block",
           "sincosm_expi_eval", "expi", "sincosm_eval_planned", "plan_from_device", "PLAN_BYTES",
           "sincosm_eval_planned_noalloc", "sincosm_eval_async", "sincosm_backward_async"]


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.F64
    if t.dtype == torch.float32:
        return _lib.F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("expected a 2-D row-major tensor (unit column stride)")
    return t.stride(0)


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")


def _acc(accuracy: str, extended: bool = False, refined: bool = False) -> int:
    return ACC[accuracy] | (_lib.PLAN_EXTENDED if extended else 0) | (_lib.PLAN_REFINED if refined else 0)


def plan_host(norm1: float, accuracy: str = "double", extended: bool = False) -> Plan:
    """The library's plan for a given 1-norm (host computation, same rule as the device).
    ``extended`` adds the 5-product scheme (Algorithm4cA + Algorithm5sA) to the candidates."""
    p = Plan()
    check(lib.sincosm_plan_host(float(norm1), _acc(accuracy, extended), ctypes.byref(p)), "sincosm_plan_host")
    return p


def plan_device(A: torch.Tensor, accuracy: str = "double", extended: bool = False) -> Plan:
    """The plan sincosm_eval would choose for A (1-norm and rule on the device)."""
    _require_cuda(A)
    n = A.shape[0]
    ws = _workspace(lib.sincosm_plan_workspace_size(n), A.device)
    p = Plan()
    check(lib.sincosm_plan_device(n, _dtype_code(A), A.data_ptr(), _ld(A), _acc(accuracy, extended),
                                  ws.data_ptr(), ws.numel(), ctypes.byref(p), _stream(A)), "sincosm_plan_device")
    return p


def workspace_size(n: int, dtype=torch.float64, accuracy="double", products="native") -> int:
    code = _lib.F64 if dtype == torch.float64 else _lib.F32
    return int(lib.sincosm_workspace_size(int(n), code, ACC[accuracy], PROD[products]))


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch allocations are 512-byte aligned, as the library requires (256)
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sincosm_eval(A: torch.Tensor, C: torch.Tensor, S: torch.Tensor, accuracy: str = "double",
                 products: str = "native", ws: torch.Tensor | None = None, raise_nonfinite=True,
                 extended: bool = False, refined: bool = False) -> Plan:
    """C-ABI sincosm_eval on torch tensors (writes C and S in place). Returns the plan.
    ``products``: the scheme products' arithmetic, "native" (the storage type), "f32",
    "bf16x3" or "i8x5" (float64 storage only: int8 matrix cores on five 7-bit slices per
    operand, float64 intermediates; meant for the single-accuracy plan).
    ``extended``: the plan may also use the 5-product scheme; ``refined``: plan on
    min(||A||_1, ||A^2||_1^(1/2)) (against overscaling of nonnormal A)."""
    _require_cuda(A, C, S)
    n = A.shape[0]
    dt = _dtype_code(A)
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    plan = Plan()
    st = lib.sincosm_eval(n, dt, A.data_ptr(), _ld(A), C.data_ptr(), _ld(C), S.data_ptr(), _ld(S),
                          _acc(accuracy, extended, refined), PROD[products], ws.data_ptr(), ws.numel(),
                          ctypes.byref(plan), _stream(A))
    if st == _lib.E_NONFINITE and not raise_nonfinite:
        return plan
    check(st, "sincosm_eval")
    return plan


PLAN_BYTES = ctypes.sizeof(Plan)


def sincosm_eval_planned(A: torch.Tensor, C: torch.Tensor, S: torch.Tensor, plan, accuracy: str = "double",
                         products: str = "native", ws: torch.Tensor | None = None,
                         plan_dev: torch.Tensor | None = None, extended: bool = False) -> None:
    """C-ABI sincosm_eval_planned: cos and sin with the caller's plan (a Plan or (level, s)).
    Only enqueues work on the current stream (graph-capturable when ``ws`` and ``plan_dev``
    are given); C and S become NaN if the plan does not cover ||A||_1 or A is not finite.
    ``plan_dev``: optional device uint8 tensor of at least PLAN_BYTES bytes that receives
    the call's plan record (read it with ``plan_from_device``)."""
    _require_cuda(A, C, S)
    n = A.shape[0]
    dt = _dtype_code(A)
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    p = Plan()
    if isinstance(plan, Plan):
        p.level, p.s = plan.level, plan.s
    else:
        p.level, p.s = int(plan[0]), int(plan[1])
    pd = None
    if plan_dev is not None:
        _require_cuda(plan_dev)
        if plan_dev.numel() * plan_dev.element_size() < PLAN_BYTES:
            raise ValueError("plan_dev holds fewer than PLAN_BYTES bytes")
        pd = plan_dev.data_ptr()
    check(lib.sincosm_eval_planned(n, dt, A.data_ptr(), _ld(A), C.data_ptr(), _ld(C), S.data_ptr(), _ld(S),
                                   _acc(accuracy, extended), PROD[products], ctypes.byref(p), ws.data_ptr(),
                                   ws.numel(), pd, _stream(A)), "sincosm_eval_planned")


def sincosm_eval_async(A: torch.Tensor, C: torch.Tensor, S: torch.Tensor, s_max: int = 16,
                       accuracy: str = "double", products: str = "native", ws: torch.Tensor | None = None,
                       plan_dev: torch.Tensor | None = None, extended: bool = False) -> None:
    """C-ABI sincosm_eval_async: cos and sin with the plan decided on the device. Only
    enqueues work on the current stream (no read-back; graph-capturable when ``ws`` and
    ``plan_dev`` are given). ``s_max`` bounds the double-angle steps enqueued (the double
    table's plan needs s <= s_max for ||A||_1 <= 1.8548 * 2^s_max); beyond it, and for
    non-finite A, C and S become NaN and the plan record's status says why."""
    _require_cuda(A, C, S)
    n = A.shape[0]
    dt = _dtype_code(A)
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    pd = None
    if plan_dev is not None:
        _require_cuda(plan_dev)
        if plan_dev.numel() * plan_dev.element_size() < PLAN_BYTES:
            raise ValueError("plan_dev holds fewer than PLAN_BYTES bytes")
        pd = plan_dev.data_ptr()
    check(lib.sincosm_eval_async(n, dt, A.data_ptr(), _ld(A), C.data_ptr(), _ld(C), S.data_ptr(), _ld(S),
                                 _acc(accuracy, extended), PROD[products], int(s_max), ws.data_ptr(),
                                 ws.numel(), pd, _stream(A)), "sincosm_eval_async")


def sincosm_eval_planned_noalloc(A: torch.Tensor, C: torch.Tensor, S: torch.Tensor, plan,
                                 accuracy: str = "double", products: str = "native",
                                 plan_dev: torch.Tensor | None = None, extended: bool = False) -> None:
    """C-ABI sincosm_eval_planned_noalloc: sincosm_eval_planned on the library's static device
    scratch (no workspace, nothing allocated by the call). Raises SincosmError with status
    E_TOO_LARGE when the order needs more than NOALLOC_SCRATCH_BYTES of workspace. Calls
    that overlap in time on one GPU share the scratch and race."""
    _require_cuda(A, C, S)
    n = A.shape[0]
    p = Plan()
    if isinstance(plan, Plan):
        p.level, p.s = plan.level, plan.s
    else:
        p.level, p.s = int(plan[0]), int(plan[1])
    pd = None
    if plan_dev is not None:
        _require_cuda(plan_dev)
        if plan_dev.numel() * plan_dev.element_size() < PLAN_BYTES:
            raise ValueError("plan_dev holds fewer than PLAN_BYTES bytes")
        pd = plan_dev.data_ptr()
    check(lib.sincosm_eval_planned_noalloc(n, _dtype_code(A), A.data_ptr(), _ld(A), C.data_ptr(), _ld(C),
                                           S.data_ptr(), _ld(S), _acc(accuracy, extended), PROD[products],
                                           ctypes.byref(p), pd, _stream(A)), "sincosm_eval_planned_noalloc")


def plan_from_device(plan_dev: torch.Tensor) -> Plan:
    """Read a plan record that sincosm_eval_planned wrote (synchronises with its stream)."""
    raw = plan_dev.view(torch.uint8).flatten()[:PLAN_BYTES].cpu().numpy().tobytes()
    return Plan.from_buffer_copy(raw)


def wave_plan_host(normB: float, accuracy: str = "double") -> Plan:
    """The library's wave plan for a given ||t^2 A||_1 (host computation, same rule as the device)."""
    p = Plan()
    check(lib.sincosm_wave_plan_host(float(normB), ACC[accuracy], ctypes.byref(p)), "sincosm_wave_plan_host")
    return p


def sincosm_wave_eval(A: torch.Tensor, t: float, C: torch.Tensor, S: torch.Tensor, accuracy: str = "double",
                      products: str = "native", ws: torch.Tensor | None = None, raise_nonfinite=True) -> Plan:
    """C-ABI sincosm_wave_eval: C = cos(t sqrt A), S = sin(t sqrt A)/sqrt A, in place. Returns the plan."""
    _require_cuda(A, C, S)
    n = A.shape[0]
    dt = _dtype_code(A)
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    plan = Plan()
    st = lib.sincosm_wave_eval(n, dt, A.data_ptr(), _ld(A), float(t), C.data_ptr(), _ld(C), S.data_ptr(),
                               _ld(S), ACC[accuracy], PROD[products], ws.data_ptr(), ws.numel(),
                               ctypes.byref(plan), _stream(A))
    if st == _lib.E_NONFINITE and not raise_nonfinite:
        return plan
    check(st, "sincosm_wave_eval")
    return plan


def _plan_dev_ptr(plan_dev: torch.Tensor | None):
    if plan_dev is None:
        return None
    _require_cuda(plan_dev)
    if plan_dev.numel() * plan_dev.element_size() < PLAN_BYTES:
        raise ValueError("plan_dev holds fewer than PLAN_BYTES bytes")
    return plan_dev.data_ptr()


def sincosm_wave_eval_async(A: torch.Tensor, t: float, C: torch.Tensor, S: torch.Tensor, s_max: int = 8,
                            accuracy: str = "double", products: str = "native", ws: torch.Tensor | None = None,
                            plan_dev: torch.Tensor | None = None) -> None:
    """C-ABI sincosm_wave_eval_async: sincosm_wave_eval with the wave plan decided on the device
    (enqueue only; graph-capturable when ``ws`` and ``plan_dev`` are given). A plan needing more
    than ``s_max`` steps (double table: ||t^2 A||_1 > 3.6404 * 4^s_max), or non-finite t^2 A,
    gives NaN in C and S and the reason in the plan record's status."""
    _require_cuda(A, C, S)
    n = A.shape[0]
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    check(lib.sincosm_wave_eval_async(n, _dtype_code(A), A.data_ptr(), _ld(A), float(t), C.data_ptr(), _ld(C),
                                      S.data_ptr(), _ld(S), ACC[accuracy], PROD[products], int(s_max),
                                      ws.data_ptr(), ws.numel(), _plan_dev_ptr(plan_dev), _stream(A)),
          "sincosm_wave_eval_async")


def sincosm_wave_block_eval_async(A: torch.Tensor, t: float, E: torch.Tensor, s_max: int = 8,
                                  accuracy: str = "double", products: str = "native",
                                  ws: torch.Tensor | None = None, plan_dev: torch.Tensor | None = None) -> None:
    """C-ABI sincosm_wave_block_eval_async: E = e^{tM} (2n x 2n) with the plan decided on the device."""
    _require_cuda(A, E)
    n = A.shape[0]
    if E.dtype != A.dtype or E.shape[0] != 2 * n or E.shape[1] != 2 * n:
        raise ValueError("E must be 2n x 2n of A's dtype")
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    check(lib.sincosm_wave_block_eval_async(n, _dtype_code(A), A.data_ptr(), _ld(A), float(t), E.data_ptr(),
                                            _ld(E), ACC[accuracy], PROD[products], int(s_max), ws.data_ptr(),
                                            ws.numel(), _plan_dev_ptr(plan_dev), _stream(A)),
          "sincosm_wave_block_eval_async")


def wave(A: torch.Tensor, t: float, accuracy: str = "double", products: str = "native"):
    """(c(t^2 A), s(t, A)) for a square float64/float32 GPU tensor: the propagator of y'' + A y = 0."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    A = A.contiguous()
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    sincosm_wave_eval(A, t, C, S, accuracy, products)
    return C, S


def sincosm_wave_block_eval(A: torch.Tensor, t: float, E: torch.Tensor, accuracy: str = "double",
                            products: str = "native", ws: torch.Tensor | None = None,
                            raise_nonfinite=True) -> Plan:
    """C-ABI sincosm_wave_block_eval: E (2n x 2n) = e^{tM}, M = [[0, I], [-A, 0]], in place."""
    _require_cuda(A, E)
    n = A.shape[0]
    if E.dtype != A.dtype or E.shape[0] != 2 * n or E.shape[1] != 2 * n:
        raise ValueError("E must be 2n x 2n of A's dtype")
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    plan = Plan()
    st = lib.sincosm_wave_block_eval(n, _dtype_code(A), A.data_ptr(), _ld(A), float(t), E.data_ptr(), _ld(E),
                                     ACC[accuracy], PROD[products], ws.data_ptr(), ws.numel(),
                                     ctypes.byref(plan), _stream(A))
    if st == _lib.E_NONFINITE and not raise_nonfinite:
        return plan
    check(st, "sincosm_wave_block_eval")
    return plan


def wave_block(A: torch.Tensor, t: float, accuracy: str = "double", products: str = "native"):
    """e^{tM} for M = [[0, I], [-A, 0]] (2n x 2n), the propagator of (y, y') for y'' + A y = 0."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    A = A.contiguous()
    n = A.shape[0]
    E = torch.empty(2 * n, 2 * n, dtype=A.dtype, device=A.device)
    sincosm_wave_block_eval(A, t, E, accuracy, products)
    return E


_COMPLEX_OF = {torch.float64: torch.complex128, torch.float32: torch.complex64}


def sincosm_expi_eval(A: torch.Tensor, t: float, U: torch.Tensor, accuracy: str = "double",
                      products: str = "native", ws: torch.Tensor | None = None, raise_nonfinite=True,
                      extended: bool = False) -> Plan:
    """C-ABI sincosm_expi_eval: U = e^{-itA} = cos(tA) - i sin(tA) (complex tensor, written in place)."""
    _require_cuda(A, U)
    n = A.shape[0]
    if U.dtype != _COMPLEX_OF.get(A.dtype) or U.dim() != 2 or U.stride(1) != 1:
        raise ValueError("U must be a row-major complex tensor matching A's precision")
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    plan = Plan()
    st = lib.sincosm_expi_eval(n, _dtype_code(A), A.data_ptr(), _ld(A), float(t), U.data_ptr(), U.stride(0),
                               _acc(accuracy, extended), PROD[products], ws.data_ptr(), ws.numel(),
                               ctypes.byref(plan), _stream(A))
    if st == _lib.E_NONFINITE and not raise_nonfinite:
        return plan
    check(st, "sincosm_expi_eval")
    return plan


def sincosm_expi_eval_async(A: torch.Tensor, t: float, U: torch.Tensor, s_max: int = 16,
                            accuracy: str = "double", products: str = "native", ws: torch.Tensor | None = None,
                            plan_dev: torch.Tensor | None = None, extended: bool = False) -> None:
    """C-ABI sincosm_expi_eval_async: U = e^{-itA} with the plan decided on the device (enqueue
    only; bitwise the result of sincosm_expi_eval). s_max and the plan record as in
    sincosm_eval_async."""
    _require_cuda(A, U)
    n = A.shape[0]
    if U.dtype != _COMPLEX_OF.get(A.dtype) or U.dim() != 2 or U.stride(1) != 1:
        raise ValueError("U must be a row-major complex tensor matching A's precision")
    if ws is None:
        ws = _workspace(workspace_size(n, A.dtype, accuracy, products), A.device)
    check(lib.sincosm_expi_eval_async(n, _dtype_code(A), A.data_ptr(), _ld(A), float(t), U.data_ptr(),
                                      U.stride(0), _acc(accuracy, extended), PROD[products], int(s_max),
                                      ws.data_ptr(), ws.numel(), _plan_dev_ptr(plan_dev), _stream(A)),
          "sincosm_expi_eval_async")


def expi(A: torch.Tensor, t: float = 1.0, accuracy: str = "double", products: str = "native"):
    """e^{-itA} for a real square GPU tensor, as a complex tensor (the unitary propagator of i u' = A u)."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    A = A.contiguous()
    U = torch.empty(A.shape, dtype=_COMPLEX_OF[A.dtype], device=A.device)
    sincosm_expi_eval(A, t, U, accuracy, products)
    return U


def sincosm_matmul(X: torch.Tensor, Y: torch.Tensor, Z: torch.Tensor, products: str = "native",
                   ws: torch.Tensor | None = None) -> None:
    """C-ABI sincosm_matmul: Z = X Y with the library's product kernels."""
    _require_cuda(X, Y, Z)
    n = X.shape[0]
    dt = _dtype_code(X)
    if ws is None:
        ws = _workspace(lib.sincosm_matmul_workspace_size(n, dt, PROD[products]), X.device)
    check(lib.sincosm_matmul(n, dt, X.data_ptr(), _ld(X), Y.data_ptr(), _ld(Y), Z.data_ptr(), _ld(Z),
                             PROD[products], ws.data_ptr(), ws.numel(), _stream(X)), "sincosm_matmul")


def sincosm_backward(A: torch.Tensor, Gc: torch.Tensor | None, Gs: torch.Tensor | None, gA: torch.Tensor,
                     accuracy: str = "double", s: int | None = None, ws: torch.Tensor | None = None) -> Plan:
    """C-ABI sincosm_backward: gA = d/dA (<Gc, cos A> + <Gs, sin A>)."""
    _require_cuda(A, Gc, Gs, gA)
    n = A.shape[0]
    dt = _dtype_code(A)
    if s is None:
        s = plan_device(A, accuracy).s
    if ws is None:
        ws = _workspace(lib.sincosm_backward_workspace_size(n, dt, ACC[accuracy], int(s)), A.device)
    plan = Plan()
    gc_ptr, gc_ld = (Gc.data_ptr(), _ld(Gc)) if Gc is not None else (None, n)
    gs_ptr, gs_ld = (Gs.data_ptr(), _ld(Gs)) if Gs is not None else (None, n)
    check(lib.sincosm_backward(n, dt, A.data_ptr(), _ld(A), gc_ptr, gc_ld, gs_ptr, gs_ld, gA.data_ptr(),
                               _ld(gA), ACC[accuracy], ws.data_ptr(), ws.numel(), ctypes.byref(plan),
                               _stream(A)), "sincosm_backward")
    return plan


def sincosm_backward_async(A: torch.Tensor, Gc: torch.Tensor | None, Gs: torch.Tensor | None, gA: torch.Tensor,
                           s_max: int = 16, accuracy: str = "double", ws: torch.Tensor | None = None,
                           plan_dev: torch.Tensor | None = None) -> None:
    """C-ABI sincosm_backward_async: gA = d/dA (<Gc, cos A> + <Gs, sin A>) with the plan decided on
    the device (no read-back; graph-capturable when ``ws`` and ``plan_dev`` are given). ``s_max``
    bounds the double-angle steps and sizes the workspace; beyond it, and for non-finite A, gA
    becomes NaN and the plan record's status says why."""
    _require_cuda(A, Gc, Gs, gA)
    n = A.shape[0]
    dt = _dtype_code(A)
    if ws is None:
        ws = _workspace(lib.sincosm_backward_workspace_size(n, dt, ACC[accuracy], int(s_max)), A.device)
    pd = None
    if plan_dev is not None:
        _require_cuda(plan_dev)
        if plan_dev.numel() * plan_dev.element_size() < PLAN_BYTES:
            raise ValueError("plan_dev holds fewer than PLAN_BYTES bytes")
        pd = plan_dev.data_ptr()
    gc_ptr, gc_ld = (Gc.data_ptr(), _ld(Gc)) if Gc is not None else (None, n)
    gs_ptr, gs_ld = (Gs.data_ptr(), _ld(Gs)) if Gs is not None else (None, n)
    check(lib.sincosm_backward_async(n, dt, A.data_ptr(), _ld(A), gc_ptr, gc_ld, gs_ptr, gs_ld, gA.data_ptr(),
                                     _ld(gA), ACC[accuracy], int(s_max), ws.data_ptr(), ws.numel(), pd,
                                     _stream(A)), "sincosm_backward_async")


class BatchedWorkspace:
    """Device metadata and workspace for one packed batch (C-ABI sincosm_eval_batched).

    ``ns`` and ``offsets`` (host sequences or int32 / int64 GPU tensors) are kept on the
    device; ``run`` enqueues the batched call's fixed launch sequence (no read-back), so it
    may be captured in a CUDA/HIP graph. ``nmax`` bounds the orders when ``ns`` is a device
    tensor (default 256).
    """

    def __init__(self, ns, offsets, dtype=torch.float64, device="cuda", accuracy="double", nmax=None):
        self.dtype = dtype
        self.accuracy = accuracy
        dt = _lib.F64 if dtype == torch.float64 else _lib.F32
        if isinstance(ns, torch.Tensor):
            self.n_dev = ns.to(device=device, dtype=torch.int32).contiguous()
            n_host = None
            self.batch = int(self.n_dev.numel())
        else:
            n_list = [int(v) for v in ns]
            self.batch = len(n_list)
            self.n_dev = torch.tensor(n_list, dtype=torch.int32, device=device)
            n_host = n_list if nmax is None else None
        if isinstance(offsets, torch.Tensor):
            self.off_dev = offsets.to(device=device, dtype=torch.int64).contiguous()
        else:
            self.off_dev = torch.tensor([int(v) for v in offsets], dtype=torch.int64, device=device)
        if self.off_dev.numel() != self.batch:
            raise ValueError("ns and offsets differ in length")
        if n_host is not None:
            arr = (ctypes.c_int32 * self.batch)(*n_host)
        elif nmax is not None:
            arr = (ctypes.c_int32 * self.batch)(*([int(nmax)] * self.batch))
        else:
            arr = None
        size = lib.sincosm_batched_workspace_size(self.batch, arr, dt, ACC[accuracy], PROD["native"])
        if size == 0:
            raise SincosmError(_lib.E_ARG, "sincosm_batched_workspace_size")
        self.ws = _workspace(size, device)

    def run(self, A: torch.Tensor, C: torch.Tensor, S: torch.Tensor, plans: torch.Tensor | None = None):
        _require_cuda(A, C, S)
        if C.numel() < A.numel() or S.numel() < A.numel():
            raise ValueError("C and S must hold as many elements as A")
        plans_ptr = plans.data_ptr() if plans is not None else None
        check(lib.sincosm_eval_batched(self.batch, _dtype_code(A), self.n_dev.data_ptr(), self.off_dev.data_ptr(),
                                       A.numel(), A.data_ptr(), C.data_ptr(), S.data_ptr(), ACC[self.accuracy],
                                       PROD["native"], self.ws.data_ptr(), self.ws.numel(), plans_ptr, _stream(A)),
              "sincosm_eval_batched")


def plans_from_bytes(buf: torch.Tensor):
    """Decode a device uint8 tensor of sincosm_plan records into Plan objects."""
    raw = bytes(buf.cpu().numpy().tobytes())
    return [Plan.from_buffer_copy(raw[i:i + PLAN_BYTES]) for i in range(0, len(raw), PLAN_BYTES)]


def sincosm_eval_batched(ns, offsets, A: torch.Tensor, C: torch.Tensor, S: torch.Tensor,
                         accuracy: str = "double", products: str = "native",
                         plans: torch.Tensor | None = None) -> BatchedWorkspace:
    """Set up the batch's device metadata and workspace (ns, offsets: host sequences or GPU
    tensors) and run it once."""
    if products != "native":
        raise SincosmError(_lib.E_UNSUPPORTED, "sincosm_eval_batched")
    w = BatchedWorkspace(ns, offsets, A.dtype, A.device, accuracy)
    w.run(A, C, S, plans)
    return w


class _SinCosM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, accuracy, products):
        C = torch.empty_like(A)
        S = torch.empty_like(A)
        plan = sincosm_eval(A, C, S, accuracy, products)
        ctx.save_for_backward(A)
        ctx.accuracy = accuracy
        ctx.s = plan.s
        return C, S

    @staticmethod
    def backward(ctx, gC, gS):
        (A,) = ctx.saved_tensors
        gA = torch.empty_like(A)
        gC = gC.contiguous() if gC is not None else None
        gS = gS.contiguous() if gS is not None else None
        sincosm_backward(A, gC, gS, gA, ctx.accuracy, s=ctx.s)
        return gA, None, None


def sincosm(A: torch.Tensor, accuracy: str = "double", products: str = "native"):
    """(cos A, sin A) for a square float64/float32 GPU tensor, differentiable in A."""
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    A = A.contiguous()
    if A.requires_grad and torch.is_grad_enabled():
        if A.dtype != torch.float64 or products != "native":
            # the reverse pass (sincosm_backward) is the float64 adjoint of the float64 products
            raise TypeError("sincosm: gradients are provided for float64 input with native products only")
        return _SinCosM.apply(A, accuracy, products)
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    sincosm_eval(A, C, S, accuracy, products)
    return C, S


def sincosm_batched(mats, accuracy: str = "double", products: str = "native"):
    """cos and sin of a list of square GPU matrices of one dtype (packed into one batched call)."""
    if not mats:
        return [], []
    dev, dt = mats[0].device, mats[0].dtype
    ns = [int(m.shape[0]) for m in mats]
    offs, o = [], 0
    for n in ns:
        offs.append(o)
        o += n * n
    A = torch.empty(max(o, 1), dtype=dt, device=dev)
    for m, off, n in zip(mats, offs, ns):
        A[off:off + n * n].copy_(m.reshape(-1))
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    sincosm_eval_batched(ns, offs, A, C, S, accuracy, products)
    Cs = [C[off:off + n * n].view(n, n) for off, n in zip(offs, ns)]
    Ss = [S[off:off + n * n].view(n, n) for off, n in zip(offs, ns)]
    return Cs, Ss
