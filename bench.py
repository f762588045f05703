"""Throughput of the simultaneous matrix cosine/sine on one MI355X.

One step = cos(A) and sin(A) (sincosm_eval through the C ABI, float64,
double-accuracy plan) for four dense n = 4096 Gaussian matrices rescaled to
||A||_1 = 2^-4, 2^0, 2^4, 2^10: the anchors of the n = 4096 float64 workload,
taking 4, 7, 15 and 27 products. Inputs, outputs and workspaces are resident
in device memory before the timed region.

Printed: one JSON line with evaluations/s, algorithmic TFLOP/s
((Pi + 2 s) 2 n^3 per evaluation) against the float64 MFMA peak, the
roofline of the dominant kernel (the double-angle product launch, timed with
HIP events on its stream), the relative error of the 2^0 anchor against the
float64 CPU oracle, and the oracle's own throughput on the host cores.
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
N = 4096
ANCHORS = (-4, 0, 4, 10)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(A: np.ndarray):
    """Time the float64 oracle on one anchor matrix; returns (seconds, threads, C, S)."""
    from oracle import reference as R
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover - informational only
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    C, S = R.sincosm(A)
    return time.perf_counter() - t0, threads, C, S


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(the batched path shards by matrix and a single large matrix by row blocks, "
              "but no multi-GPU code is built)", file=sys.stderr)
        sys.exit(2)
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
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
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

    rel = None
    cpu = None
    if not args.no_cpu_baseline:
        a_idx = ANCHORS.index(0)
        secs, threads, Cr, Sr = cpu_baseline(mats[a_idx])
        Cg, Sg = C[a_idx].cpu().numpy(), S[a_idx].cpu().numpy()
        rel = {"cos": float(np.linalg.norm(Cg - Cr) / np.linalg.norm(Cr)),
               "sin": float(np.linalg.norm(Sg - Sr) / np.linalg.norm(Sr)),
               "anchor": "2^0", "reference": "float64 CPU oracle (Taylor m=9 + double angle)"}
        # scale the sample to the 4-anchor mix by the oracle's own product counts
        # (s_o = ceil(log2 ||A||_1) halvings; 11 products + 2 s_o per evaluation)
        from oracle import reference as R
        oracle_products = [11 + 2 * R.scaling_power(2.0 ** e) for e in ANCHORS]
        mix = sum(oracle_products) / len(oracle_products)
        cpu = {"value": (1.0 / secs) * (oracle_products[a_idx] / mix), "unit": "evals/s", "cores": threads,
               "kind": "oracle",
               "sample": f"one float64 oracle evaluation of the 2^0 anchor at n={n} ({secs:.1f} s, "
                         f"{oracle_products[a_idx]} products), scaled to the 4-anchor mix by the oracle's "
                         f"product counts {oracle_products}"}

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
        "tflops_algorithmic": tflops,
        "pct_fp64_mfma_peak": 100.0 * tflops / FP64_MFMA_PEAK_TFLOPS,
        "roofline": {"bound": "mfma", "kernel": "double-angle product launch (gemm_kernel<double,128,...>, "
                                                "2 problems)",
                     "achieved": sq_tflops, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (sq_tflops / FP64_MFMA_PEAK_TFLOPS) if sq_tflops else None,
                     "traffic": None, "launches": sq_cnt,
                     "avg_ms": (sq_ms / sq_cnt) if sq_cnt else None},
        "scheme_products": {"launches": sch_cnt, "avg_ms": (sch_ms / sch_cnt) if sch_cnt else None,
                            "tflops": (2.0 * n ** 3 / (sch_ms / sch_cnt / 1e3) / 1e12) if sch_cnt else None},
        "rel_err": rel,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
