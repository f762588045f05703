"""Autotuner for the product kernel's configuration (tile shape, k depth,
wave grid, occupancy) per arithmetic and padded matrix order.

For each arithmetic and each probe order n it times every configuration the
library offers whose tile divides the padded order (C-ABI
``sincosm_tune_num_configs`` / ``sincosm_tune_config_info``), by forcing it
with ``sincosm_tune_set`` and timing ``sincosm_matmul`` with HIP events. A
second pass tunes the launches of several equal problems (the double-angle
steps): it forces each configuration for that class only
(``SINCOSM_TUNE_MULTI``) and times the double-angle launches of a
``sincosm_eval`` call with the library's launch timing. A third pass (float64)
tunes the launches of unequal problems or several k-segments, which only the
reverse pass makes (``SINCOSM_TUNE_UNEVEN``): it times whole
``sincosm_backward`` calls with each configuration forced for that class. A
fourth pass picks the product mode of the batched kernel's per-matrix products
(``SINCOSM_TUNE_BATCHED``: 64 x 64 or 32 x 32 output tiles, or for padded
orders up to 32 the LDS-resident kernel) per padded order, timing
``sincosm_eval_batched`` on batches of one order. The fastest
configuration per probe and class is written to a JSON cache with the range of
padded orders it covers (midpoints between probes); for the single-product and
double-angle classes the choice is then settled on whole evaluations (every
pairing of each class's three fastest configurations on four anchor
evaluations). ``apply_cache`` installs a
cache in the library; the package calls it at import for the cache shipped
next to this file (``tune_gfx950.json``) or the file named by
``SINCOSM_TUNE_CACHE``. Entries of an arithmetic whose recorded configuration
table differs from the library's are skipped.

Usage on the GPU:  python -m paper_2010_00465_amd.autotune --out paper_2010_00465_amd/tune_gfx950.json
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import time

from ._lib import lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_gfx950.json")
ARITH = {"f64": 0, "f32": 1}
MULTI = 16          # SINCOSM_TUNE_MULTI: the table of launches of several equal problems
UNEVEN = 32         # SINCOSM_TUNE_UNEVEN: launches of unequal problems or several k-segments
BATCHED = 64        # SINCOSM_TUNE_BATCHED: the batched kernel's output tile per padded order
CLASS_FLAG = {"": 0, "multi": MULTI, "uneven": UNEVEN, "batched": BATCHED}
UNEVEN_PROBES = (256, 512, 1024, 2048, 4096)
BATCHED_PROBES = (16, 32, 48, 64, 96, 128, 144, 160, 176, 192, 208, 224, 240, 256)
PROBES = (256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144, 8192)


def padded(n: int) -> int:
    g = 128 if n >= 1536 else (64 if n >= 256 else 32)
    return (n + g - 1) // g * g


def configs(arith: str, flags: int = 0):
    out = []
    for i in range(lib.sincosm_tune_num_configs(ARITH[arith] | flags)):
        info = (ctypes.c_int32 * 8)()
        lib.sincosm_tune_config_info(ARITH[arith] | flags, i, info)
        out.append({"idx": i, "bm": info[0], "bn": info[1], "bk": info[2], "wgm": info[3], "wgn": info[4],
                    "wpe": info[5], "direct": info[6], "kgroups": info[7]})
    return out


def apply_cache(path: str | None = None) -> int:
    """Install the entries of a tuning cache; returns how many were applied."""
    path = path or os.environ.get("SINCOSM_TUNE_CACHE") or DEFAULT_CACHE
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    count = 0
    for key, entries in data.get("entries", {}).items():
        arith, _, cls = key.partition("_")
        if arith not in ARITH or cls not in CLASS_FLAG:
            continue
        table = arith + "_batched" if cls == "batched" else arith
        tuned, have = data.get("configs", {}).get(table), configs(arith, CLASS_FLAG[cls] & BATCHED)
        if not tuned or tuned != have[:len(tuned)]:
            # tuned against another configuration table: its indices mean other kernels (a table
            # that only appended configurations keeps the indices of the ones the cache knows)
            continue
        code = ARITH[arith] | CLASS_FLAG[cls]
        for e in entries:
            if lib.sincosm_tune_set(code, int(e["np_lo"]), int(e["np_hi"]), int(e["idx"])) == 0:
                count += 1
    return count


def time_config(torch, sc, arith: str, n: int, idx: int, reps: int) -> float:
    np_ = padded(n)
    lib.sincosm_tune_set(ARITH[arith], np_, np_, idx)
    dt = torch.float64 if arith == "f64" else torch.float32
    X = torch.randn(n, n, dtype=dt, device="cuda")
    Y = torch.randn(n, n, dtype=dt, device="cuda")
    Z = torch.empty_like(X)
    ws = torch.empty(lib.sincosm_matmul_workspace_size(n, ARITH[arith], 0), dtype=torch.uint8, device="cuda")
    sc.sincosm_matmul(X, Y, Z, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sc.sincosm_matmul(X, Y, Z, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    lib.sincosm_tune_set(ARITH[arith], np_, np_, -1)
    return e0.elapsed_time(e1) / reps


def time_config_multi(torch, sc, arith: str, n: int, idx: int, reps: int) -> float:
    """Average duration (ms) of the double-angle launches of sincosm_eval at order n with
    configuration idx forced for the two-product class only (||A||_1 = 16: 4 steps)."""
    np_ = padded(n)
    dt = torch.float64 if arith == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(n)
    A = torch.randn(n, n, dtype=dt, device="cuda", generator=g)
    A *= 16.0 / float(A.abs().sum(0).max())
    C, S = torch.empty_like(A), torch.empty_like(A)
    ws = torch.empty(sc.workspace_size(n, dt), dtype=torch.uint8, device="cuda")
    lib.sincosm_tune_set(ARITH[arith] | MULTI, np_, np_, idx)
    sc.sincosm_eval(A, C, S, ws=ws)
    torch.cuda.synchronize()
    lib.sincosm_timing_enable(1)
    for _ in range(reps):
        sc.sincosm_eval(A, C, S, ws=ws)
    torch.cuda.synchronize()
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    lib.sincosm_timing_read(1, ctypes.byref(ms), ctypes.byref(cnt))
    lib.sincosm_timing_enable(0)
    lib.sincosm_tune_set(ARITH[arith] | MULTI, np_, np_, -1)
    return ms.value / max(cnt.value, 1)


def time_config_uneven(torch, sc, n: int, idx: int, reps: int) -> float:
    """Average duration (ms) of a whole float64 sincosm_backward call at order n (Gaussian,
    ||A||_1 = 128: plan level 7, s = 7) with configuration idx forced for the uneven class."""
    np_ = padded(n)
    g = torch.Generator(device="cuda").manual_seed(n)
    A = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    A *= 128.0 / float(A.abs().sum(0).max())
    Gc = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    Gs = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    gA = torch.empty_like(A)
    lib.sincosm_tune_set(ARITH["f64"] | UNEVEN, np_, np_, idx)
    s = sc.plan_device(A).s
    ws = torch.empty(lib.sincosm_backward_workspace_size(n, 0, 0, s), dtype=torch.uint8, device="cuda")
    sc.sincosm_backward(A, Gc, Gs, gA, s=s, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sc.sincosm_backward(A, Gc, Gs, gA, s=s, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    lib.sincosm_tune_set(ARITH["f64"] | UNEVEN, np_, np_, -1)
    return e0.elapsed_time(e1) / reps


def time_config_batched(torch, sc, arith: str, n: int, idx: int, reps: int) -> float:
    """Average duration (ms) of sincosm_eval_batched on a batch of Gaussian matrices of order
    n (||A||_1 = 8: level 7 with s = 3 in double, s = 1 in single) with batched tile
    configuration idx forced for that order."""
    np_ = (n + 15) // 16 * 16
    dt = torch.float64 if arith == "f64" else torch.float32
    count = 4096   # several matrices per resident workgroup
    g = torch.Generator(device="cuda").manual_seed(n)
    A = torch.randn(count, n, n, dtype=dt, device="cuda", generator=g)
    A *= 8.0 / A.abs().sum(1).amax(1).view(count, 1, 1)
    C, S = torch.empty_like(A), torch.empty_like(A)
    ns, offs = [n] * count, [k * n * n for k in range(count)]
    lib.sincosm_tune_set(ARITH[arith] | BATCHED, np_, np_, idx)
    w = sc.BatchedWorkspace(ns, offs, dt, "cuda", "double" if arith == "f64" else "single")
    w.run(A, C, S)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        w.run(A, C, S)
    e1.record()
    torch.cuda.synchronize()
    lib.sincosm_tune_set(ARITH[arith] | BATCHED, np_, np_, -1)
    return e0.elapsed_time(e1) / reps


def _ranges(nps, k):
    lo = 1 if k == 0 else (nps[k - 1] + nps[k]) // 2 + 1
    hi = 1 << 30 if k == len(nps) - 1 else (nps[k] + nps[k + 1]) // 2
    return lo, hi


def tune_batched(torch, sc, arith: str, reps: int, log):
    entries, timings = [], {}
    nps = sorted({(n + 15) // 16 * 16 for n in BATCHED_PROBES})
    for k, np_ in enumerate(nps):
        best = None
        timings[str(np_)] = {}
        for c in configs(arith, BATCHED):
            if c["direct"] == 2 and np_ > c["bm"]:
                continue   # the LDS-resident mode takes padded orders up to its size only
            ms = time_config_batched(torch, sc, arith, np_, c["idx"], reps)
            timings[str(np_)][str(c["idx"])] = ms
            if best is None or ms < best[1]:
                best = (c["idx"], ms)
        lo, hi = _ranges(nps, k)
        entries.append({"np_lo": lo, "np_hi": hi, "idx": best[0], "probe_np": np_, "ms": best[1]})
        cb = configs(arith, BATCHED)[best[0]]
        mode = "LDS-resident" if cb["direct"] == 2 else f"tile {cb['bm']}"
        log(f"{arith} batched np={np_}: best {mode} {best[1]:.3f} ms")
    return entries, timings


def tune(ariths=("f64", "f32"), probes=PROBES, reps=5, log=print, batched_only=False):
    import torch
    import paper_2010_00465_amd as sc
    result = {"device": torch.cuda.get_device_name(0), "created": time.strftime("%Y-%m-%d %H:%M:%S"),
              "configs": {} if batched_only else {a: configs(a) for a in ariths}, "entries": {}, "timings": {}}
    for arith in ariths:
        result["configs"][arith + "_batched"] = configs(arith, BATCHED)
        result["entries"][arith + "_batched"], result["timings"][arith + "_batched"] = \
            tune_batched(torch, sc, arith, reps, log)
        if batched_only:
            continue
        entries, timings = [], {}
        nps = sorted({padded(n) for n in probes})
        for k, np_ in enumerate(nps):
            best = None
            timings[str(np_)] = {}
            for c in configs(arith):
                if np_ % c["bm"] or np_ % c["bn"]:
                    continue
                ms = time_config(torch, sc, arith, np_, c["idx"], reps)
                timings[str(np_)][str(c["idx"])] = ms
                if best is None or ms < best[1]:
                    best = (c["idx"], ms)
            lo = 1 if k == 0 else (nps[k - 1] + np_) // 2 + 1
            hi = 1 << 30 if k == len(nps) - 1 else (np_ + nps[k + 1]) // 2
            flops = 2.0 * np_ ** 3
            entries.append({"np_lo": lo, "np_hi": hi, "idx": best[0], "probe_np": np_, "ms": best[1],
                            "tflops": flops / (best[1] * 1e-3) / 1e12})
            log(f"{arith} np={np_}: best config {best[0]} {best[1]:.3f} ms "
                f"({flops / (best[1] * 1e-3) / 1e12:.1f} TFLOP/s incl. padding copies)")
        result["entries"][arith] = entries
        result["timings"][arith] = timings
        # two-product launches, with the single-product table just measured installed
        for e in entries:
            lib.sincosm_tune_set(ARITH[arith], int(e["np_lo"]), int(e["np_hi"]), int(e["idx"]))
        entries_m, timings_m = [], {}
        for k, np_ in enumerate(nps):
            best = None
            timings_m[str(np_)] = {}
            for c in configs(arith):
                if np_ % c["bm"] or np_ % c["bn"]:
                    continue
                ms = time_config_multi(torch, sc, arith, np_, c["idx"], reps)
                timings_m[str(np_)][str(c["idx"])] = ms
                if best is None or ms < best[1]:
                    best = (c["idx"], ms)
            lo, hi = _ranges(nps, k)
            flops = 4.0 * np_ ** 3
            entries_m.append({"np_lo": lo, "np_hi": hi, "idx": best[0], "probe_np": np_, "ms": best[1],
                              "tflops": flops / (best[1] * 1e-3) / 1e12})
            log(f"{arith} two-product launches np={np_}: best config {best[0]} {best[1]:.3f} ms "
                f"({flops / (best[1] * 1e-3) / 1e12:.1f} TFLOP/s)")
        result["entries"][arith + "_multi"] = entries_m
        result["timings"][arith + "_multi"] = timings_m
        refine_whole(torch, sc, result, arith, log=log)
        if arith != "f64":
            continue
        # launches of the reverse pass, with both tables above installed
        for e in entries_m:
            lib.sincosm_tune_set(ARITH[arith] | MULTI, int(e["np_lo"]), int(e["np_hi"]), int(e["idx"]))
        nps_u = sorted({padded(n) for n in UNEVEN_PROBES})
        entries_u, timings_u = [], {}
        for k, np_ in enumerate(nps_u):
            best = None
            timings_u[str(np_)] = {}
            for c in configs(arith):
                if np_ % c["bm"] or np_ % c["bn"]:
                    continue
                ms = time_config_uneven(torch, sc, np_, c["idx"], max(1, reps // 2))
                timings_u[str(np_)][str(c["idx"])] = ms
                if best is None or ms < best[1]:
                    best = (c["idx"], ms)
            lo, hi = _ranges(nps_u, k)
            entries_u.append({"np_lo": lo, "np_hi": hi, "idx": best[0], "probe_np": np_, "ms": best[1]})
            log(f"{arith} reverse-pass launches np={np_}: best config {best[0]}, whole backward {best[1]:.3f} ms")
        result["entries"][arith + "_uneven"] = entries_u
        result["timings"][arith + "_uneven"] = timings_u
    return result


def time_whole(torch, sc, arith: str, n: int, reps: int) -> float:
    """Average duration (ms) of the four anchor evaluations (Gaussian, ||A||_1 = 2^-4, 2^0,
    2^4, 2^10; 4, 7, 15 and 27 products in double) at order n, with the current table."""
    dt = torch.float64 if arith == "f64" else torch.float32
    acc = "double" if arith == "f64" else "single"
    g = torch.Generator(device="cuda").manual_seed(n)
    mats = []
    for e in (-4, 0, 4, 10):
        A = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
        mats.append((A * (2.0 ** e / float(A.abs().sum(0).max()))).to(dt))
    C, S = torch.empty_like(mats[0]), torch.empty_like(mats[0])
    ws = torch.empty(sc.workspace_size(n, dt, acc), dtype=torch.uint8, device="cuda")
    for A in mats:
        sc.sincosm_eval(A, C, S, acc, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for A in mats:
            sc.sincosm_eval(A, C, S, acc, ws=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def refine_whole(torch, sc, result, arith: str, top: int = 3, reps: int = 2, log=print):
    """Whole-evaluation pass: per probe order, the `top` fastest configurations of the
    single-product and the double-angle classes (from the launch timings above) are tried in
    every pairing on four anchor evaluations, and the fastest pairing replaces the entries of
    that probe's range. The launch timings alone miss what consecutive launches of one
    evaluation do to each other (caches, the other class's tail)."""
    ent, ent_m = result["entries"][arith], result["entries"][arith + "_multi"]
    tim, tim_m = result["timings"][arith], result["timings"][arith + "_multi"]
    code = ARITH[arith]
    for e, em in zip(ent, ent_m):
        np_ = e["probe_np"]
        c0 = sorted(tim[str(np_)], key=lambda k: tim[str(np_)][k])[:top]
        c1 = sorted(tim_m[str(np_)], key=lambda k: tim_m[str(np_)][k])[:top]
        best = None
        for a in c0:
            for b in c1:
                lib.sincosm_tune_set(code, np_, np_, int(a))
                lib.sincosm_tune_set(code | MULTI, np_, np_, int(b))
                ms = time_whole(torch, sc, arith, np_, reps)
                if best is None or ms < best[2]:
                    best = (int(a), int(b), ms)
        lib.sincosm_tune_set(code, np_, np_, -1)
        lib.sincosm_tune_set(code | MULTI, np_, np_, -1)
        lib.sincosm_tune_set(code, int(e["np_lo"]), int(e["np_hi"]), best[0])
        lib.sincosm_tune_set(code | MULTI, int(em["np_lo"]), int(em["np_hi"]), best[1])
        log(f"{arith} np={np_}: whole evaluations best with configs {best[0]} / {best[1]} "
            f"({best[2]:.2f} ms for four anchors; launch timings chose {e['idx']} / {em['idx']})")
        e["idx"], em["idx"] = best[0], best[1]
        e["whole_ms"] = em["whole_ms"] = best[2]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--arith", default="f64,f32")
    ap.add_argument("--batched-only", action="store_true",
                    help="tune only the batched kernel's tiles and merge them into the --out cache")
    args = ap.parse_args()
    res = tune(tuple(args.arith.split(",")), reps=args.reps, log=lambda s: print(s, flush=True),
               batched_only=args.batched_only)
    if args.batched_only and os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        for key in ("configs", "entries", "timings"):
            old.setdefault(key, {}).update(res[key])
        res = old
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
