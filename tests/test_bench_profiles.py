"""The bench reads HBM traffic from the committed rocprofv3 summaries only while the kernel
sources they were taken from are unchanged (a hash recorded in each summary); these checks
keep the summaries and the sources in step, and check the bench's own contract pieces that
need no GPU."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_product_kernel_profile_is_current():
    """profiles/gemm_f64_n4096.md carries the hash of csrc/gemm.hip + epilogue.hpp; the bench's
    roofline traffic comes from it."""
    b = _bench()
    t = b.measured_traffic()
    assert t is not None and t > 0


def test_batched_profile_is_current():
    """profiles/batched_mixed_20k.md carries the hash of csrc/batched.hip; the bench's batched HBM
    roofline comes from it."""
    b = _bench()
    t = b.batched_traffic()
    assert t is not None and t["f64"] > t["f32"] > 0
    r = b._hbm_roofline(t["f64"], 0.070)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and 0 < r["frac"] < 1


def test_bench_refuses_several_gpus():
    """One GPU here: --gpus N with N > 1 exits with a message, before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
