"""ctypes binding of libsincosm.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module only turns
torch tensors into device pointers, sizes and the current HIP stream. It
raises at import time when the library has not been built, so nothing can
silently fall back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsincosm.so")

OK = 0
E_ARG = -1
E_UNSUPPORTED = -2
E_WORKSPACE = -3
E_NONFINITE = -4
E_HIP = -5
E_PLAN = -6
E_TOO_LARGE = -7
E_SCALING = -8
NOALLOC_SCRATCH_BYTES = 32 << 20   # SINCOSM_NOALLOC_SCRATCH_BYTES

F64, F32 = 0, 1
ACC = {"double": 0, "single": 1}
PLAN_EXTENDED = 16   # OR-ed into the accuracy code: the 5-product scheme joins the plan
PLAN_REFINED = 32    # OR-ed into the accuracy code of sincosm_eval: plan on min(||A||_1, ||A^2||_1^(1/2))
PROD = {"native": 0, "f32": 1, "bf16x3": 2, "i8x5": 3}


class Plan(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("s", ctypes.c_int32), ("products", ctypes.c_int32),
                ("status", ctypes.c_int32), ("norm1", ctypes.c_double)]

    def as_tuple(self):
        return (self.level, self.s, self.products)

    def __repr__(self):
        return (f"Plan(level={self.level}, s={self.s}, products={self.products}, "
                f"status={self.status}, norm1={self.norm1!r})")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "or python paper_2010_00465_amd/build.py")

lib = ctypes.CDLL(LIB_PATH)

_i64, _i32, _int, _sz, _vp, _dbl = (ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_double)
_PlanP = ctypes.POINTER(Plan)

SYMBOLS = {
    "sincosm_plan_host": (_int, [_dbl, _int, _PlanP]),
    "sincosm_strerror": (ctypes.c_char_p, [_int]),
    "sincosm_workspace_size": (_sz, [_i64, _int, _int, _int]),
    "sincosm_plan_workspace_size": (_sz, [_i64]),
    "sincosm_plan_device": (_int, [_i64, _int, _vp, _i64, _int, _vp, _sz, _PlanP, _vp]),
    "sincosm_eval": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _int, _int, _vp, _sz, _PlanP, _vp]),
    "sincosm_eval_planned": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _int, _int, _PlanP, _vp, _sz,
                                    _vp, _vp]),
    "sincosm_eval_async": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _int, _int, _i32, _vp, _sz, _vp,
                                  _vp]),
    "sincosm_eval_planned_noalloc": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _int, _int, _PlanP,
                                            _vp, _vp]),
    "sincosm_wave_plan_host": (_int, [_dbl, _int, _PlanP]),
    "sincosm_wave_eval": (_int, [_i64, _int, _vp, _i64, _dbl, _vp, _i64, _vp, _i64, _int, _int, _vp, _sz, _PlanP,
                                 _vp]),
    "sincosm_wave_block_eval": (_int, [_i64, _int, _vp, _i64, _dbl, _vp, _i64, _int, _int, _vp, _sz, _PlanP, _vp]),
    "sincosm_expi_eval": (_int, [_i64, _int, _vp, _i64, _dbl, _vp, _i64, _int, _int, _vp, _sz, _PlanP, _vp]),
    "sincosm_wave_eval_async": (_int, [_i64, _int, _vp, _i64, _dbl, _vp, _i64, _vp, _i64, _int, _int, _i32, _vp,
                                       _sz, _vp, _vp]),
    "sincosm_wave_block_eval_async": (_int, [_i64, _int, _vp, _i64, _dbl, _vp, _i64, _int, _int, _i32, _vp, _sz,
                                             _vp, _vp]),
    "sincosm_expi_eval_async": (_int, [_i64, _int, _vp, _i64, _dbl, _vp, _i64, _int, _int, _i32, _vp, _sz, _vp,
                                       _vp]),
    "sincosm_batched_workspace_size": (_sz, [_i64, ctypes.POINTER(_i32), _int, _int, _int]),
    "sincosm_eval_batched": (_int, [_i64, _int, _vp, _vp, _i64, _vp, _vp, _vp, _int, _int, _vp, _sz, _vp, _vp]),
    "sincosm_backward_workspace_size": (_sz, [_i64, _int, _int, _i32]),
    "sincosm_backward": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int, _vp, _sz,
                                _PlanP, _vp]),
    "sincosm_backward_async": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int, _i32, _vp, _sz,
                                      _vp, _vp]),
    "sincosm_tune_num_configs": (_int, [_int]),
    "sincosm_tune_config_info": (_int, [_int, _int, ctypes.POINTER(_i32)]),
    "sincosm_tune_set": (_int, [_int, _i64, _i64, _int]),
    "sincosm_tune_lookup": (_int, [_int, _i64]),
    "sincosm_timing_enable": (_int, [_int]),
    "sincosm_timing_read": (_int, [_int, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
    "sincosm_matmul_workspace_size": (_sz, [_i64, _int, _int]),
    "sincosm_matmul": (_int, [_i64, _int, _vp, _i64, _vp, _i64, _vp, _i64, _int, _vp, _sz, _vp]),
}

for _name, (_res, _args) in SYMBOLS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SincosmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.sincosm_strerror(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def check(status: int, where: str) -> None:
    if status != OK:
        raise SincosmError(status, where)
