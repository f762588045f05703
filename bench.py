"""Throughput of the simultaneous matrix cosine/sine on one MI355X.

One step = cos(A) and sin(A) (sincosm_eval through the C ABI, float64,
double-accuracy plan) for four dense n = 4096 Gaussian matrices rescaled to
||A||_1 = 2^-4, 2^0, 2^4, 2^10: the anchors of the n = 4096 float64 workload,
taking 4, 7, 15 and 27 products. Inputs, outputs and workspaces are resident
in device memory before the timed region.

Printed: one JSON line with evaluations/s, algorithmic TFLOP/s
((Pi + 2 s) 2 n^3 per evaluation) against the float64 MFMA peak, the
roofline of the dominant kernel (the double-angle product launch, timed with
HIP events on its stream), the relative errors of the anchors against the
float64 CPU oracle, and the oracle's own throughput on the host cores (all
threads, and one thread). Beside the step (unless --no-extras): the mean over
8 seeded draws of ||A||_1 = 2^e, e ~ U(-4, 10); the float32 single-accuracy
path on the anchors; the float64 oracle's and the GPU's discrepancy against the
long-double oracle at n = 256; and the secondary workloads (batched, reverse
pass, precision tiers, wave pair, propagators, other orders).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
N = 4096
ANCHORS = (-4, 0, 4, 10)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (batched, backward, tiers, wave, propagators, "
                         "5-product scheme, refined norm, other orders)")
    ap.add_argument("--only", choices=["batched", "batched_call", "backward", "tiers", "wave", "propagators",
                                       "level5", "refined", "sizes"],
                    help="run and print only one of the secondary measurements (batched_call: the 20,000-matrix "
                         "batched calls alone, float64 and float32, without the comparison loops; for counters)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run sincosm_matmul once at --n: its two pad/convert copy kernels read and "
                         "write n*n float64 each, a known byte count for scaling HBM counters")
    return ap.parse_args()


def copy_calibration(n):
    import torch
    import paper_2010_00465_amd as sc
    X = torch.ones(n, n, dtype=torch.float64, device="cuda:0")
    Z = torch.empty_like(X)
    torch.cuda.synchronize()
    sc.sincosm_matmul(X, X, Z)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"n": n, "copy_kernel_bytes_read": 8 * n * n,
                                           "copy_kernel_bytes_written": 8 * n * n}}))


def product_config(lib, n, flags):
    """The product-kernel configuration the tuning table gives launches of this class at
    padded order n (the bench's n is a multiple of 128, so it is its own padded order)."""
    import ctypes
    idx = lib.sincosm_tune_lookup(flags, n)
    if idx < 0:
        return "default configuration"
    info = (ctypes.c_int32 * 8)()
    lib.sincosm_tune_config_info(0, idx, info)
    return (f"configuration {idx}: {info[0]}x{info[1]} tile, k step {info[2]}, {info[3] * info[4] * info[7]} waves"
            + (", direct loads" if info[6] else "") + (f", {info[7]} k groups" if info[7] > 1 else ""))


def cpu_baseline(mats):
    """Time the float64 oracle on one whole step (every anchor matrix once).

    Returns (seconds, threads, [(C, S) per matrix])."""
    from oracle import reference as R
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover - informational only
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    out = [R.sincosm(A) for A in mats]
    return time.perf_counter() - t0, threads, out


def cpu_host(n, products_per_step):
    """The host CPU and the like-for-like CPU figure for the method: one float64 DGEMM of
    order n through numpy (all threads, then one thread) times the step's product count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, n))
    Y = rng.standard_normal((n, n))
    X @ Y
    t0 = time.perf_counter()
    X @ Y
    t_all = time.perf_counter() - t0
    t_one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            t0 = time.perf_counter()
            X @ Y
            t_one = time.perf_counter() - t0
    except Exception:  # pragma: no cover - informational only
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "dgemm_s": t_all, "dgemm_1thread_s": t_one,
            "products_per_step": products_per_step,
            "paper_algorithm_evals_per_s": len(products_per_step) / (sum(products_per_step) * t_all),
            "paper_algorithm_evals_per_s_1thread":
                (len(products_per_step) / (sum(products_per_step) * t_one)) if t_one else None,
            "note": f"(products per evaluation) x (one n={n} numpy DGEMM on this host): the CPU time of "
                    "the method's own products, without its O(n^2) work"}


KERNEL_SOURCES = ("gemm.hip", "epilogue.hpp")


def kernel_sources_sha256():
    """sha256 over the product kernel's sources (gemm.hip, then epilogue.hpp)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_00465_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per double-angle launch from the committed counter summary,
    or None when the product kernel's sources changed since it was taken."""
    prof = os.path.join(ROOT, "profiles", "gemm_f64_n4096.md")
    try:
        text = open(prof).read()
        sha = kernel_sources_sha256()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch (double-angle step)",
                                                   "kernel_sources_sha256"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if vals.get("kernel_sources_sha256") != sha:
        return None
    try:
        return float(vals["traffic_bytes_per_launch (double-angle step)"])
    except (KeyError, ValueError):
        return None


def batched_traffic():
    """Counter bytes (HBM reads + writes, copy-calibrated) per 20,000-matrix batched call, float64
    and float32, from the committed counter summary; None once csrc/batched.hip has changed."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "batched_mixed_20k.md")
    try:
        text = open(prof).read()
        with open(os.path.join(ROOT, "paper_2010_00465_amd", "csrc", "batched.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("batched_sources_sha256") != sha:
        return None
    try:
        return {"f64": float(vals["traffic_bytes_per_call (float64)"]),
                "f32": float(vals["traffic_bytes_per_call (float32)"])}
    except (KeyError, ValueError):
        return None


def _hbm_roofline(traffic, seconds):
    """HBM roofline of a batched call: counter bytes per call over the timed call, against 8 TB/s."""
    if traffic is None:
        return None
    achieved = traffic / seconds / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}


def _elapsed(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def bench_batched(torch, sc, W):
    """20,000 matrices, n uniform on {8,...,256}, ||A||_1 = 2^U(-6,8), float64, double accuracy;
    against a loop of single-matrix calls over the first 400 matrices of the same batch."""
    ns, offs, packed, _ = W.batched_gaussian(20000, key=(3,))
    A = torch.from_numpy(packed).cuda()
    C = torch.empty_like(A)
    S = torch.empty_like(A)
    plans = torch.zeros(len(ns) * sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    w = sc.BatchedWorkspace(ns, offs, A.dtype, A.device)
    w.run(A, C, S, plans)
    pl = sc.plans_from_bytes(plans)
    flops = float(sum(p.products * 2.0 * int(n) ** 3 for p, n in zip(pl, ns)))
    t = _elapsed(torch, lambda: w.run(A, C, S, plans), 3)
    # per-matrix loop on a prefix of the same batch
    k = 400
    mats = [A[int(o):int(o) + int(n) * int(n)].view(int(n), int(n)) for n, o in zip(ns[:k], offs[:k])]
    outs = [(torch.empty_like(m), torch.empty_like(m)) for m in mats]
    wsz = max(sc.workspace_size(int(n), torch.float64) for n in ns[:k])
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")

    def loop():
        for m, (c, s_) in zip(mats, outs):
            sc.sincosm_eval(m, c, s_, ws=ws)

    loop()
    t_loop = _elapsed(torch, loop, 1)
    loop_flops = float(sum(p.products * 2.0 * int(n) ** 3 for p, n in zip(pl[:k], ns[:k])))
    # the same loop with the plan decided on the device (no read-back; s <= 8 for these norms),
    # eagerly and as one captured HIP graph of all 400 calls
    s_max = 8

    def loop_async():
        for m, (c, s_) in zip(mats, outs):
            sc.sincosm_eval_async(m, c, s_, s_max, ws=ws)

    loop_async()
    t_loop_async = _elapsed(torch, loop_async, 1)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        loop_async()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g_loop = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_loop):
        loop_async()
    g_loop.replay()
    t_loop_graph = _elapsed(torch, g_loop.replay, 3)
    del g_loop
    # the same call captured in a HIP graph and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        w.run(A, C, S, plans)
    g.replay()
    t_graph = _elapsed(torch, g.replay, 3)
    # float32 storage with the single-accuracy plans, same orders and norms
    A32 = A.to(torch.float32)
    C32, S32 = torch.empty_like(A32), torch.empty_like(A32)
    plans32 = torch.zeros_like(plans)
    w32 = sc.BatchedWorkspace(ns, offs, torch.float32, A.device, accuracy="single")
    w32.run(A32, C32, S32, plans32)
    pl32 = sc.plans_from_bytes(plans32)
    flops32 = float(sum(p.products * 2.0 * int(n) ** 3 for p, n in zip(pl32, ns)))
    t32 = _elapsed(torch, lambda: w32.run(A32, C32, S32, plans32), 3)
    return {"workload": "20000 float64 Gaussian matrices, n uniform on {8,...,256}, ||A||_1 = 2^U(-6,8), "
                        "double-accuracy plans, one sincosm_eval_batched call",
            "ms_per_batch": 1e3 * t, "evals_per_s": len(ns) / t, "tflops_algorithmic": flops / t / 1e12,
            "mean_products": float(np.mean([p.products for p in pl])),
            "graph_replay_ms": 1e3 * t_graph,
            "loop_of_sincosm_eval": {"matrices": k, "evals_per_s": k / t_loop,
                                     "tflops_algorithmic": loop_flops / t_loop / 1e12},
            "loop_of_sincosm_eval_async": {"matrices": k, "s_max": s_max, "evals_per_s": k / t_loop_async,
                                           "tflops_algorithmic": loop_flops / t_loop_async / 1e12,
                                           "graph_replay_evals_per_s": k / t_loop_graph,
                                           "graph_replay_tflops_algorithmic": loop_flops / t_loop_graph / 1e12},
            "speedup_vs_loop": (len(ns) / t) / (k / t_loop),
            "hbm_roofline": _hbm_roofline((batched_traffic() or {}).get("f64"), t),
            "float32_single": {"ms_per_batch": 1e3 * t32, "evals_per_s": len(ns) / t32,
                               "tflops_algorithmic": flops32 / t32 / 1e12,
                               "mean_products": float(np.mean([p.products for p in pl32])),
                               "hbm_roofline": _hbm_roofline((batched_traffic() or {}).get("f32"), t32)}}


def bench_batched_call(torch, sc, W):
    """The 20,000-matrix batched call alone (float64 double plans, then float32 single plans),
    three timed calls each after one warm-up: the workload of the batched counter passes."""
    ns, offs, packed, _ = W.batched_gaussian(20000, key=(3,))
    out = {}
    for dt, acc in ((torch.float64, "double"), (torch.float32, "single")):
        A = torch.from_numpy(packed).cuda().to(dt)
        C, S = torch.empty_like(A), torch.empty_like(A)
        plans = torch.zeros(len(ns) * sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
        w = sc.BatchedWorkspace(ns, offs, dt, A.device, accuracy=acc)
        w.run(A, C, S, plans)
        pl = sc.plans_from_bytes(plans)
        flops = float(sum(p.products * 2.0 * int(n) ** 3 for p, n in zip(pl, ns)))
        t = _elapsed(torch, lambda: w.run(A, C, S, plans), 3)
        out["f64_double" if dt == torch.float64 else "f32_single"] = {
            "ms_per_batch": 1e3 * t, "tflops_algorithmic": flops / t / 1e12,
            "hbm_roofline": _hbm_roofline((batched_traffic() or {}).get("f64" if dt == torch.float64 else "f32"),
                                          t)}
        del A, C, S, w
    return out


def bench_backward(torch, sc, W):
    """Gradient of <Gc, cos A> + <Gs, sin A>, n = 2048 Gaussian, ||A||_1 = 128 (float64)."""
    n = 2048
    A = torch.from_numpy(W.gaussian(n, 128.0, key=(4, n, 256))).cuda()
    g = W.rng(64, n, 256)
    Gc = torch.from_numpy(g.standard_normal((n, n))).cuda()
    Gs = torch.from_numpy(g.standard_normal((n, n))).cuda()
    gA = torch.empty_like(A)
    plan = sc.plan_device(A)
    ws = torch.empty(sc.lib.sincosm_backward_workspace_size(n, 0, 0, plan.s), dtype=torch.uint8, device="cuda")
    sc.sincosm_backward(A, Gc, Gs, gA, s=plan.s, ws=ws)
    t = _elapsed(torch, lambda: sc.sincosm_backward(A, Gc, Gs, gA, s=plan.s, ws=ws), 3)
    prods = 3 * plan.level + 6 * plan.s - 2
    # the same with the plan decided on the device (no read-back), s_max = 8
    wsa = torch.empty(sc.lib.sincosm_backward_workspace_size(n, 0, 0, 8), dtype=torch.uint8, device="cuda")
    sc.sincosm_backward_async(A, Gc, Gs, gA, 8, ws=wsa)
    ta = _elapsed(torch, lambda: sc.sincosm_backward_async(A, Gc, Gs, gA, 8, ws=wsa), 3)
    return {"workload": f"sincosm_backward, n={n} Gaussian, ||A||_1=128, plan (level {plan.level}, s {plan.s})",
            "ms": 1e3 * t, "products": prods, "tflops_algorithmic": prods * 2.0 * n ** 3 / t / 1e12,
            "forward_products": plan.products,
            "async_s_max8_ms": 1e3 * ta}


def bench_tiers(torch, sc, W):
    """n = 4096: 2-D 5-point Laplacian on a 64 x 64 grid scaled to ||A||_1 = 64, and a Gaussian
    matrix of the same norm; each product arithmetic with its plan table: time and relative error
    against the float64 CPU oracle; for each lowered tier, the float64 path with the error closest
    to it from below (matched accuracy: the same or better error)."""
    from oracle import reference as R
    from paper_2010_00465_amd import _lib

    def one(Anp):
        A = torch.from_numpy(Anp).cuda()
        Cr, Sr = R.sincosm(Anp)
        out = {}
        for name, acc, prod in (("fp64_double", "double", "native"), ("fp64_single_plan", "single", "native"),
                                ("fp32_products", "single", "f32"), ("bf16x3_products", "single", "bf16x3"),
                                ("int8x5_products", "single", "i8x5")):
            C = torch.empty_like(A)
            S = torch.empty_like(A)
            ws = torch.empty(sc.workspace_size(4096, torch.float64, acc, prod), dtype=torch.uint8, device="cuda")
            plan = sc.sincosm_eval(A, C, S, acc, prod, ws=ws)
            t = _elapsed(torch, lambda: sc.sincosm_eval(A, C, S, acc, prod, ws=ws), 3)
            ec = float(np.linalg.norm(C.cpu().numpy() - Cr) / np.linalg.norm(Cr))
            es = float(np.linalg.norm(S.cpu().numpy() - Sr) / np.linalg.norm(Sr))
            out[name] = {"ms": 1e3 * t, "plan": [plan.level, plan.s], "products": plan.products,
                         "rel_err_cos": ec, "rel_err_sin": es}
            # per-launch durations of one more evaluation (HIP events around each product launch;
            # an int8 scheme product's launch includes its slicing kernels)
            _lib.lib.sincosm_timing_enable(1)
            sc.sincosm_eval(A, C, S, acc, prod, ws=ws)
            per = {}
            for kind, key in ((0, "scheme_product_ms"), (1, "double_angle_step_ms")):
                ms, cnt = ctypes.c_double(), ctypes.c_int64()
                _lib.lib.sincosm_timing_read(kind, ctypes.byref(ms), ctypes.byref(cnt))
                per[key] = ms.value / cnt.value if cnt.value else None
            _lib.lib.sincosm_timing_enable(0)
            out[name].update(per)
            if prod == "i8x5" and per["scheme_product_ms"]:
                out[name]["int8_pops_per_scheme_product"] = 15 * 2.0 * 4096 ** 3 / per["scheme_product_ms"] / 1e12
            del ws
        fp64 = [k for k in ("fp64_single_plan", "fp64_double")]
        for tier in ("fp32_products", "bf16x3_products", "int8x5_products"):
            err = max(out[tier]["rel_err_cos"], out[tier]["rel_err_sin"])
            ok = [k for k in fp64 if max(out[k]["rel_err_cos"], out[k]["rel_err_sin"]) <= err]
            best = min(ok, key=lambda k: out[k]["ms"]) if ok else None
            out[tier]["matched_accuracy_fp64"] = None if best is None else {
                "path": best, "ms": out[best]["ms"],
                "rel_err": max(out[best]["rel_err_cos"], out[best]["rel_err_sin"]),
                "speedup_of_tier": out[best]["ms"] / out[tier]["ms"]}
            out[tier]["meets_single_accuracy_5e-6"] = err <= 5e-6
        return out

    out = {"workload": "n=4096 2-D Laplacian (64 x 64 grid), ||A||_1 = 64, float64 storage; errors relative "
                       "to the float64 CPU oracle"}
    out.update(one(W.laplacian_2d(64, 64.0)))
    out["gaussian"] = dict(workload="n=4096 Gaussian N(0,1) rescaled to ||A||_1 = 64, float64 storage; errors "
                                    "relative to the float64 CPU oracle",
                           **one(W.gaussian(4096, 64.0, key=(7, 4096))))
    return out


def bench_draws(torch, sc, W, n, ws):
    """The n = 4096 float64 Gaussian workload at 8 seeded draws e ~ U(-4, 10), ||A||_1 = 2^e:
    each evaluation timed on its own after a warm-up; mean throughput over the draws."""
    exps = W.log_uniform_exponents(8, -4.0, 10.0, key=(2, n, 0, 100))
    A = torch.empty(n, n, dtype=torch.float64, device="cuda")
    C, S = torch.empty_like(A), torch.empty_like(A)
    per, t_sum, f_sum = [], 0.0, 0.0
    for d, e in enumerate(exps):
        A.copy_(torch.from_numpy(W.gaussian(n, 2.0 ** float(e), key=(2, n, 0, 1000 + d))))
        p = sc.sincosm_eval(A, C, S, ws=ws)
        t = _elapsed(torch, lambda: sc.sincosm_eval(A, C, S, ws=ws), 2)
        flops = p.products * 2.0 * n ** 3
        per.append({"log2_norm1": float(e), "plan": [p.level, p.s], "products": p.products, "ms": 1e3 * t,
                    "tflops_algorithmic": flops / t / 1e12})
        t_sum += t
        f_sum += flops
    return {"workload": f"sincosm_eval of 8 dense n={n} float64 Gaussian matrices, ||A||_1 = 2^e with e drawn "
                        "uniformly in [-4, 10] (seeded), double-accuracy plan",
            "evals_per_s": len(exps) / t_sum, "tflops_algorithmic": f_sum / t_sum / 1e12,
            "pct_fp64_mfma_peak": 100.0 * f_sum / t_sum / 1e12 / FP64_MFMA_PEAK_TFLOPS, "draws": per}


def bench_fp32_single(torch, sc, W, n, mats, with_oracle):
    """Float32 storage with the single-accuracy plan (Table 2) on the four anchor matrices cast
    to float32: throughput against the FP32 MFMA peak and, when asked, the relative error against
    the float64 oracle run on the float32 values promoted (the single-accuracy bar is 5e-6)."""
    from oracle import reference as R
    A = [torch.from_numpy(m.astype(np.float32)).cuda() for m in mats]
    C = [torch.empty_like(a) for a in A]
    S = [torch.empty_like(a) for a in A]
    ws = torch.empty(sc.workspace_size(n, torch.float32, "single"), dtype=torch.uint8, device="cuda")
    plans = [sc.sincosm_eval(a, c, s_, "single", ws=ws) for a, c, s_ in zip(A, C, S)]

    def step():
        for a, c, s_ in zip(A, C, S):
            sc.sincosm_eval(a, c, s_, "single", ws=ws)

    t = _elapsed(torch, step, 3)
    flops = sum(p.products for p in plans) * 2.0 * n ** 3
    out = {"workload": f"sincosm_eval of the four n={n} anchor matrices cast to float32, single-accuracy plan",
           "evals_per_s": len(A) / t, "tflops_algorithmic": flops / t / 1e12,
           "pct_fp32_mfma_peak": 100.0 * flops / t / 1e12 / FP32_MFMA_PEAK_TFLOPS,
           "plans": [[p.level, p.s] for p in plans], "products": [p.products for p in plans]}
    if with_oracle:
        errs = {}
        for e, m, c, s_ in zip(ANCHORS, mats, C, S):
            Cr, Sr = R.sincosm(m.astype(np.float32).astype(np.float64))
            errs[f"2^{e}"] = {"cos": float(np.linalg.norm(c.double().cpu().numpy() - Cr) / np.linalg.norm(Cr)),
                              "sin": float(np.linalg.norm(s_.double().cpu().numpy() - Sr) / np.linalg.norm(Sr))}
        out["rel_err_vs_oracle"] = errs
        out["rel_err_max"] = max(max(v.values()) for v in errs.values())
    return out


def oracle_vs_long_double(torch, sc, W, n=256):
    """The float64 oracle's own discrepancy against the 80-bit long-double oracle (the best
    available reference for a general matrix), and the GPU's, on the four anchors at order n."""
    from oracle import reference as R
    out = {"n": n, "reference": "oracle in 80-bit long double (Taylor m=11 + double angle)", "per_anchor": {}}
    for e in ANCHORS:
        A = W.gaussian(n, 2.0 ** e, key=(2, n, 0, e + 10))
        Cl, Sl = (x.astype(np.float64) for x in R.sincosm_ld(A))
        Co, So = R.sincosm(A)
        At = torch.from_numpy(A).cuda()
        Cg, Sg = torch.empty_like(At), torch.empty_like(At)
        sc.sincosm_eval(At, Cg, Sg)
        Cg, Sg = Cg.cpu().numpy(), Sg.cpu().numpy()

        def rel(X, Y):
            return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))

        out["per_anchor"][f"2^{e}"] = {"fp64_oracle": max(rel(Co, Cl), rel(So, Sl)),
                                       "gpu": max(rel(Cg, Cl), rel(Sg, Sl)),
                                       "gpu_vs_fp64_oracle": max(rel(Cg, Co), rel(Sg, So))}
    return out


def cpu_baseline_1core(mat):
    """The float64 oracle on one thread, on the cheapest anchor (||A||_1 = 2^-4)."""
    from oracle import reference as R
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover - informational only
        return None
    with threadpool_limits(1):
        t0 = time.perf_counter()
        R.sincosm(mat)
        secs = time.perf_counter() - t0
    return {"value": 1.0 / secs, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"the ||A||_1 = 2^-4 anchor (n={mat.shape[0]}) once through the float64 oracle on one "
                      f"host thread, {secs:.1f} s"}


def bench_wave(torch, sc, W):
    """Wave-equation pair c(t^2 A), s(t, A) (sincosm_wave_eval), n = 4096 float64.

    (a) A = X^2 for a Gaussian X with ||X||_1 = 2^e (e = 0, 4), t = 1: the wave call gives
        cos(X) (and s(1, A) X = sin(X)) and is timed against sincosm_eval(X), which returns the
        same cosine, with the products each plan takes and the relative difference of the two
        cosines; (b) A = 2-D 5-point Laplacian on a 64 x 64 grid with ||A||_1 = 64 and t = 1/2, 4
        (the semi-discrete wave equation y'' + A y = 0)."""
    n = 4096
    out = {"workload": "sincosm_wave_eval, n=4096 float64, double-accuracy wave plan"}
    ws = torch.empty(sc.workspace_size(n, torch.float64), dtype=torch.uint8, device="cuda")
    for e in (0, 4):
        X = torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(5, n, e))).cuda()
        A = torch.empty_like(X)
        sc.sincosm_matmul(X, X, A)
        C, S, Cx, Sx = (torch.empty_like(X) for _ in range(4))
        pw = sc.sincosm_wave_eval(A, 1.0, C, S, ws=ws)
        pc = sc.sincosm_eval(X, Cx, Sx, ws=ws)
        tw = _elapsed(torch, lambda: sc.sincosm_wave_eval(A, 1.0, C, S, ws=ws), 3)
        tc = _elapsed(torch, lambda: sc.sincosm_eval(X, Cx, Sx, ws=ws), 3)
        diff = float((C - Cx).norm() / Cx.norm())
        out[f"X^2_gaussian_2^{e}"] = {
            "wave": {"ms": 1e3 * tw, "plan": [pw.level, pw.s], "products": pw.products,
                     "norm1_B": pw.norm1, "tflops_algorithmic": pw.products * 2.0 * n ** 3 / tw / 1e12},
            "sincosm_eval_of_X": {"ms": 1e3 * tc, "plan": [pc.level, pc.s], "products": pc.products},
            "speedup": tc / tw, "rel_diff_cos": diff}
    A = torch.from_numpy(W.laplacian_2d(64, 64.0)).cuda()
    C, S = torch.empty_like(A), torch.empty_like(A)
    pd = torch.zeros(sc.PLAN_BYTES, dtype=torch.uint8, device="cuda")
    for t in (0.5, 4.0):
        p = sc.sincosm_wave_eval(A, t, C, S, ws=ws)
        tw = _elapsed(torch, lambda: sc.sincosm_wave_eval(A, t, C, S, ws=ws), 3)
        # the device-planned call with s_max = 8 (the plan decided on the device, nothing read back)
        sc.sincosm_wave_eval_async(A, t, C, S, 8, ws=ws, plan_dev=pd)
        ta = _elapsed(torch, lambda: sc.sincosm_wave_eval_async(A, t, C, S, 8, ws=ws, plan_dev=pd), 3)
        out[f"laplacian2d_t{t}"] = {"ms": 1e3 * tw, "plan": [p.level, p.s], "products": p.products,
                                    "tflops_algorithmic": p.products * 2.0 * n ** 3 / tw / 1e12,
                                    "async_s_max8_ms": 1e3 * ta}
    return out


def bench_level5(torch, sc, W):
    """n = 4096 Gaussian with ||A||_1 = 0.1 (double) and 0.8 (single accuracy), float64: the
    paper's plan (6 products) against the extended plan with the 5-product scheme; relative
    difference of the results."""
    n = 4096
    out = {"workload": "n=4096 float64 Gaussian; paper plan vs plan with the 5-product scheme"}
    ws = torch.empty(sc.workspace_size(n, torch.float64), dtype=torch.uint8, device="cuda")
    for acc, norm in (("double", 0.1), ("single", 0.8)):
        A = torch.from_numpy(W.gaussian(n, norm, key=(7, n, int(norm * 10)))).cuda()
        res = {}
        outs = {}
        for ext in (False, True):
            C, S = torch.empty_like(A), torch.empty_like(A)
            p = sc.sincosm_eval(A, C, S, acc, ws=ws, extended=ext)
            t = _elapsed(torch, lambda: sc.sincosm_eval(A, C, S, acc, ws=ws, extended=ext), 5)
            res["extended" if ext else "paper"] = {"ms": 1e3 * t, "plan": [p.level, p.s], "products": p.products}
            outs[ext] = (C, S)
        (C0, S0), (C1, S1) = outs[False], outs[True]
        res["speedup"] = res["paper"]["ms"] / res["extended"]["ms"]
        res["rel_diff_cos"] = float((C1 - C0).norm() / C0.norm())
        res["rel_diff_sin"] = float((S1 - S0).norm() / S0.norm())
        out[f"{acc}_norm_{norm}"] = res
    return out


def bench_sizes(torch, sc, W):
    """The anchor matrices (Gaussian, ||A||_1 = 2^e, e in {-4, 0, 4, 10}) at n = 1024 and 8192,
    float64 with the double-accuracy plans and float32 storage with the single-accuracy plans:
    evaluations/s and algorithmic TFLOP/s over the four anchors; at n = 1024 also through a
    HIP graph of sincosm_eval_planned with the same plans."""
    out = {"workload": "four Gaussian anchor matrices per order and storage type"}
    for n in (1024, 8192):
        for dt, acc in ((torch.float64, "double"), (torch.float32, "single")):
            mats = [torch.from_numpy(W.gaussian(n, 2.0 ** e, key=(2, n, 0, e + 10))).cuda().to(dt) for e in ANCHORS]
            outs = [(torch.empty_like(m), torch.empty_like(m)) for m in mats]
            ws = torch.empty(sc.workspace_size(n, dt, acc), dtype=torch.uint8, device="cuda")
            plans = [sc.sincosm_eval(m, c, s_, acc, ws=ws) for m, (c, s_) in zip(mats, outs)]

            def run():
                for m, (c, s_) in zip(mats, outs):
                    sc.sincosm_eval(m, c, s_, acc, ws=ws)

            t = _elapsed(torch, run, 2)
            flops = sum(p.products for p in plans) * 2.0 * n ** 3
            key = f"n{n}_{'f64' if dt == torch.float64 else 'f32'}_{acc}"
            out[key] = {"evals_per_s": len(mats) / t, "tflops_algorithmic": flops / t / 1e12,
                        "products": [p.products for p in plans]}
            if n <= 1024:
                # the same four evaluations with the plans given (sincosm_eval_planned), captured
                # once in a HIP graph and replayed: no plan read-back, no host gaps between calls
                def run_planned():
                    for m, (c, s_), p in zip(mats, outs, plans):
                        sc.sincosm_eval_planned(m, c, s_, p, acc, ws=ws)

                run_planned()
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    run_planned()
                tg = _elapsed(torch, g.replay, 5)
                out[key]["graph_replay"] = {"evals_per_s": len(mats) / tg, "tflops_algorithmic": flops / tg / 1e12}
                del g
            del mats, outs, ws
    return out


def bench_refined(torch, sc, W):
    """Overscaling (Section 4's [[1, lambda], [0, -1]] family at n = 4096): A = [[I, B], [0, -I]]
    with B Gaussian, ||B||_1 = 1024, so A^2 = I and cos A = cos(1) I, sin A = sin(1) A exactly.
    The tables' plan on ||A||_1 against the refined plan on min(||A||_1, ||A^2||_1^(1/2)); errors
    against the closed forms (computed on the GPU)."""
    import math
    n, h = 4096, 2048
    B = torch.from_numpy(W.gaussian(h, 1024.0, key=(8, n))).cuda()
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    A[:h, :h] = torch.eye(h, dtype=torch.float64, device="cuda")
    A[h:, h:] = -torch.eye(h, dtype=torch.float64, device="cuda")
    A[:h, h:] = B
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    Cx, Sx = math.cos(1.0) * I, math.sin(1.0) * A
    ws = torch.empty(sc.workspace_size(n, torch.float64), dtype=torch.uint8, device="cuda")
    out = {"workload": "n=4096 float64 [[I, B], [0, -I]], B Gaussian with ||B||_1 = 1024 (A^2 = I)"}
    for name, ref in (("paper_plan", False), ("refined_plan", True)):
        C, S = torch.empty_like(A), torch.empty_like(A)
        p = sc.sincosm_eval(A, C, S, ws=ws, refined=ref)
        t = _elapsed(torch, lambda: sc.sincosm_eval(A, C, S, ws=ws, refined=ref), 3)
        out[name] = {"ms": 1e3 * t, "plan": [p.level, p.s], "products": p.products, "norm_used": p.norm1,
                     "rel_err_cos": float((C - Cx).norm() / Cx.norm()),
                     "rel_err_sin": float((S - Sx).norm() / Sx.norm())}
    out["speedup"] = out["paper_plan"]["ms"] / out["refined_plan"]["ms"]
    return out


def bench_propagators(torch, sc, W):
    """n = 4096 float64 propagators against torch.linalg.matrix_exp on the same operator.

    e^{-itA} (eq:unitary): symmetric Gaussian A with ||A||_1 = 64 and the 2-D Laplacian with
    ||A||_1 = 64, t = 1: sincosm_expi_eval (real products, two per double-angle step) against
    matrix_exp of the complex128 matrix -itA (a general exponential with complex products).
    e^{tM} (eq:symplectic): the 2-D Laplacian, t = 1: sincosm_wave_block_eval (n x n products)
    against matrix_exp of the real 2n x 2n block M. Reported: times, the ratio, and the relative
    difference of the two results."""
    n = 4096
    out = {"workload": "n=4096 float64; library comparison: torch.linalg.matrix_exp on the same operator"}
    ws = torch.empty(sc.workspace_size(n, torch.float64), dtype=torch.uint8, device="cuda")
    ops = {"symmetric_gaussian": torch.from_numpy(W.symmetric_gaussian(n, 64.0, key=(6, n))).cuda(),
           "laplacian2d": torch.from_numpy(W.laplacian_2d(64, 64.0)).cuda()}
    for name, A in ops.items():
        U = torch.empty(n, n, dtype=torch.complex128, device="cuda")
        p = sc.sincosm_expi_eval(A, 1.0, U, ws=ws)
        t_ours = _elapsed(torch, lambda: sc.sincosm_expi_eval(A, 1.0, U, ws=ws), 3)
        Z = (-1j) * A.to(torch.complex128)
        R = torch.linalg.matrix_exp(Z)
        t_ref = _elapsed(torch, lambda: torch.linalg.matrix_exp(Z), 2)
        # the device-planned call (s_max = 8: nothing read back)
        sc.sincosm_expi_eval_async(A, 1.0, U, 8, ws=ws)
        t_async = _elapsed(torch, lambda: sc.sincosm_expi_eval_async(A, 1.0, U, 8, ws=ws), 3)
        out[f"expi_{name}"] = {"ms": 1e3 * t_ours, "plan": [p.level, p.s], "real_products": p.products,
                               "async_s_max8_ms": 1e3 * t_async,
                               "matrix_exp_complex128_ms": 1e3 * t_ref, "speedup": t_ref / t_ours,
                               "rel_diff": float((U - R).norm() / R.norm())}
    A = ops["laplacian2d"]
    E = torch.empty(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    p = sc.sincosm_wave_block_eval(A, 1.0, E, ws=ws)
    t_ours = _elapsed(torch, lambda: sc.sincosm_wave_block_eval(A, 1.0, E, ws=ws), 3)
    M = torch.zeros(2 * n, 2 * n, dtype=torch.float64, device="cuda")
    M[:n, n:] = torch.eye(n, dtype=torch.float64, device="cuda")
    M[n:, :n] = -A
    R = torch.linalg.matrix_exp(M)
    t_ref = _elapsed(torch, lambda: torch.linalg.matrix_exp(M), 2)
    sc.sincosm_wave_block_eval_async(A, 1.0, E, 8, ws=ws)
    t_async = _elapsed(torch, lambda: sc.sincosm_wave_block_eval_async(A, 1.0, E, 8, ws=ws), 3)
    out["block_laplacian2d"] = {"ms": 1e3 * t_ours, "plan": [p.level, p.s], "products_n": p.products + 1,
                                "async_s_max8_ms": 1e3 * t_async,
                                "matrix_exp_2n_ms": 1e3 * t_ref, "speedup": t_ref / t_ours,
                                "rel_diff": float((E - R).norm() / R.norm())}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library and this benchmark run on one GPU; --gpus must be 1 "
              "(the batched path shards by matrix and a single large matrix by row blocks, "
              "but no multi-GPU code is built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.n)
        return
    if args.only:
        import torch
        import paper_2010_00465_amd as sc
        import workloads as W
        fn = {"batched": bench_batched, "batched_call": bench_batched_call, "backward": bench_backward,
              "tiers": bench_tiers,
              "wave": bench_wave, "propagators": bench_propagators, "level5": bench_level5,
              "refined": bench_refined, "sizes": bench_sizes}[args.only]
        print(json.dumps({args.only: fn(torch, sc, W)}))
        return
    import torch
    import paper_2010_00465_amd as sc
    import workloads as W
    from paper_2010_00465_amd import _lib

    n = args.n
    dev = torch.device("cuda:0")
    mats = [W.gaussian(n, 2.0 ** e, key=(2, n, 0, e + 10)) for e in ANCHORS]
    A = [torch.from_numpy(m).to(dev) for m in mats]
    C = [torch.empty_like(a) for a in A]
    S = [torch.empty_like(a) for a in A]
    ws = torch.empty(sc.workspace_size(n, torch.float64), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        return [sc.sincosm_eval(a, c, s_, ws=ws) for a, c, s_ in zip(A, C, S)]

    plans = None
    for _ in range(max(args.warmup, 1)):
        plans = step()
    torch.cuda.synchronize()
    products = [p.products for p in plans]

    _lib.lib.sincosm_timing_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = [t0]
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()     # each call already waits for its plan; this closes the step
        marks.append(time.perf_counter())
    elapsed = marks[-1] - t0
    step_ms = np.diff(np.asarray(marks)) * 1e3
    tot = {}
    for kind in (0, 1):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        _lib.lib.sincosm_timing_read(kind, ctypes.byref(ms), ctypes.byref(cnt))
        tot[kind] = (ms.value, cnt.value)
    _lib.lib.sincosm_timing_enable(0)

    ms_per_step = 1e3 * elapsed / args.steps
    evals = len(ANCHORS) * args.steps
    value = evals / elapsed
    flops_per_step = sum(products) * 2.0 * n ** 3
    tflops = flops_per_step * args.steps / elapsed / 1e12

    # Dominant kernel: the double-angle launch (two n x n x n products per launch).
    sq_ms, sq_cnt = tot[1]
    sq_flops = 2 * 2.0 * n ** 3
    sq_avg_s = (sq_ms / sq_cnt) / 1e3 if sq_cnt else float("nan")
    sq_tflops = sq_flops / sq_avg_s / 1e12 if sq_cnt else None
    sch_ms, sch_cnt = tot[0]

    # plan read-back alone (1-norm, plan kernel, 24-byte copy and stream sync), outside the timed region
    pw = torch.empty(sc.lib.sincosm_plan_workspace_size(n), dtype=torch.uint8, device=dev)
    plan_ms = []
    for _ in range(10):
        torch.cuda.synchronize()
        tp = time.perf_counter()
        p_ = sc.Plan()
        _lib.check(sc.lib.sincosm_plan_device(n, 0, A[1].data_ptr(), n, 0, pw.data_ptr(), pw.numel(),
                                              ctypes.byref(p_), torch.cuda.current_stream(dev).cuda_stream),
                   "sincosm_plan_device")
        plan_ms.append((time.perf_counter() - tp) * 1e3)

    draws = bench_draws(torch, sc, W, n, ws) if (n == N and not args.no_extras) else None
    fp32 = (bench_fp32_single(torch, sc, W, n, mats, not args.no_cpu_baseline)
            if (n == N and not args.no_extras) else None)

    rel = None
    cpu = None
    cpu1 = None
    host = None
    ld = None
    if not args.no_cpu_baseline:
        secs, threads, ref = cpu_baseline(mats)
        rel = {"reference": "float64 CPU oracle (Taylor m=9 + double angle), same inputs",
               "per_anchor": {}}
        worst = 0.0
        for e, (Cr, Sr), Cg, Sg in zip(ANCHORS, ref, C, S):
            ec = float(np.linalg.norm(Cg.cpu().numpy() - Cr) / np.linalg.norm(Cr))
            es = float(np.linalg.norm(Sg.cpu().numpy() - Sr) / np.linalg.norm(Sr))
            rel["per_anchor"][f"2^{e}"] = {"cos": ec, "sin": es}
            worst = max(worst, ec, es)
        rel["max"] = worst
        cpu = {"value": len(mats) / secs, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"one whole step (the four n={n} anchor matrices once each) through the float64 "
                         f"oracle on the host, {secs:.1f} s"}
        host = cpu_host(n, products)
        if not args.no_extras:
            cpu1 = cpu_baseline_1core(mats[0])
            ld = oracle_vs_long_double(torch, sc, W)

    extras = {}
    if not args.no_extras and n == N:
        extras["batched"] = bench_batched(torch, sc, W)
        extras["backward"] = bench_backward(torch, sc, W)
        extras["tiers"] = bench_tiers(torch, sc, W)
        extras["wave"] = bench_wave(torch, sc, W)
        extras["propagators"] = bench_propagators(torch, sc, W)
        extras["level5"] = bench_level5(torch, sc, W)
        extras["refined"] = bench_refined(torch, sc, W)
        extras["sizes"] = bench_sizes(torch, sc, W)

    out = {
        "metric": "cos+sin evals/sec & % MFMA peak at n=4096 FP64; rel err vs FP64 oracle",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sincosm_eval of four dense n={n} float64 Gaussian matrices per step, "
                               f"||A||_1 = 2^e for e in {list(ANCHORS)} (double-accuracy plan)",
                   "n": n, "anchors_log2_norm1": list(ANCHORS), "products": products,
                   "plans": [[p.level, p.s] for p in plans], "evals_per_step": len(ANCHORS)},
        "step_ms_median": float(np.median(step_ms)),
        "step_ms_iqr": float(np.percentile(step_ms, 75) - np.percentile(step_ms, 25)),
        "plan_readback_ms_median": float(np.median(plan_ms)),
        "tflops_algorithmic": tflops,
        "pct_fp64_mfma_peak": 100.0 * tflops / FP64_MFMA_PEAK_TFLOPS,
        "roofline": {"bound": "mfma", "kernel": "double-angle product launch (FP64 MFMA product kernel, "
                                                "2 problems, " + product_config(_lib.lib, n, 16) + ")",
                     "achieved": sq_tflops, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (sq_tflops / FP64_MFMA_PEAK_TFLOPS) if sq_tflops else None,
                     "traffic": measured_traffic(), "launches": sq_cnt,
                     "avg_ms": (sq_ms / sq_cnt) if sq_cnt else None},
        "scheme_products": {"launches": sch_cnt, "avg_ms": (sch_ms / sch_cnt) if sch_cnt else None,
                            "tflops": (2.0 * n ** 3 / (sch_ms / sch_cnt / 1e3) / 1e12) if sch_cnt else None},
        "draws": draws,
        "rel_err": rel,
        "oracle_vs_long_double": ld,
        "fp32_single": fp32,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
        "cpu_host": host,
    }
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
