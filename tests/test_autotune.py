"""Autotuner plumbing (no GPU): the configuration table, the tuning hooks of
the C ABI, and the shipped cache file."""
import ctypes
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2010_00465_amd import _lib
    return _lib.lib


def test_config_table(lib):
    for arith in (0, 1):
        n = lib.sincosm_tune_num_configs(arith)
        assert n >= 3
        info = (ctypes.c_int32 * 8)()
        for i in range(n):
            assert lib.sincosm_tune_config_info(arith, i, info) == 0
            bm, bn, bk, wgm, wgn, wpe, direct, kgroups = list(info)
            assert bm % (16 * wgm) == 0 and bn % (16 * wgn) == 0 and bk % 4 == 0 and wpe >= 1
            assert direct in (0, 1) and kgroups in (1, 2, 4)
        # the three defaults are the square tiles of the padding granularities
        sizes = []
        for i in range(3):
            lib.sincosm_tune_config_info(arith, i, info)
            sizes.append((info[0], info[1]))
        assert sizes == [(128, 128), (64, 64), (32, 32)]
    assert lib.sincosm_tune_config_info(0, 999, info) == -1
    assert lib.sincosm_tune_num_configs(7) == 0


def test_tune_set_validation(lib):
    assert lib.sincosm_tune_set(0, 100, 50, 0) == -1     # empty range
    assert lib.sincosm_tune_set(0, 1, 10, 999) == -1     # unknown configuration
    assert lib.sincosm_tune_set(9, 1, 10, 0) == -1       # unknown arithmetic
    assert lib.sincosm_tune_set(0, 1 << 40, 1 << 41, 1) == 0
    assert lib.sincosm_tune_set(0, 1 << 40, 1 << 41, -1) == 0


def test_shipped_cache_is_consistent(lib):
    from paper_2010_00465_amd import autotune
    path = autotune.DEFAULT_CACHE
    assert os.path.exists(path)
    data = json.load(open(path))
    for key, entries in data["entries"].items():
        arith, _, cls = key.partition("_")
        assert cls in ("", "multi", "uneven", "batched"), key
        flag = autotune.CLASS_FLAG[cls] & autotune.BATCHED
        n = lib.sincosm_tune_num_configs(autotune.ARITH[arith] | flag)
        prev_hi = 0
        for e in entries:
            assert 0 <= e["idx"] < n
            assert e["np_lo"] == prev_hi + 1 and e["np_hi"] >= e["np_lo"]
            prev_hi = e["np_hi"]
            if flag:     # batched orders are padded to 16; the tile need not divide them
                assert e["probe_np"] % 16 == 0 and e["probe_np"] <= 256
                continue
            info = data["configs"][arith][e["idx"]]
            assert e["probe_np"] % info["bm"] == 0 and e["probe_np"] % info["bn"] == 0


def test_shipped_cache_matches_table_and_applies(lib):
    from paper_2010_00465_amd import autotune
    data = json.load(open(autotune.DEFAULT_CACHE))
    for arith in autotune.ARITH:
        have = autotune.configs(arith)
        assert data["configs"][arith] == have[:len(data["configs"][arith])]   # the library may append
        if arith + "_batched" in data["configs"]:
            tuned = data["configs"][arith + "_batched"]
            assert tuned == autotune.configs(arith, autotune.BATCHED)[:len(tuned)]
    expected = sum(len(v) for v in data["entries"].values())
    assert autotune.apply_cache() == expected


def test_cache_of_another_table_is_skipped(lib, tmp_path):
    """A cache whose configuration list is not a prefix of the library's table is skipped for
    that table (a prefix is accepted: appending configurations keeps the earlier indices)."""
    from paper_2010_00465_amd import autotune
    data = json.load(open(autotune.DEFAULT_CACHE))
    data["configs"]["f64"][0] = dict(data["configs"]["f64"][0], bk=99)   # an entry that means another kernel
    p = tmp_path / "cache.json"
    p.write_text(json.dumps(data))
    try:
        applied = autotune.apply_cache(str(p))
        # the f64 product-kernel classes are skipped; the batched tile table is its own
        skipped = [k for k in data["entries"] if k.startswith("f64") and not k.endswith("_batched")]
        assert applied == sum(len(v) for k, v in data["entries"].items() if k not in skipped)
    finally:
        for arith in autotune.ARITH.values():
            for code in (arith, arith | autotune.MULTI, arith | autotune.UNEVEN, arith | autotune.BATCHED):
                lib.sincosm_tune_set(code, 1, 1 << 30, -1)
        autotune.apply_cache()


def test_multi_class_flag(lib):
    """SINCOSM_TUNE_MULTI addresses a second table; the configuration list is the same."""
    from paper_2010_00465_amd import autotune
    assert lib.sincosm_tune_num_configs(autotune.MULTI) == lib.sincosm_tune_num_configs(0)
    assert lib.sincosm_tune_set(autotune.MULTI, 1 << 40, 1 << 41, 1) == 0
    assert lib.sincosm_tune_set(autotune.MULTI, 1 << 40, 1 << 41, -1) == 0
    assert lib.sincosm_tune_set(autotune.MULTI | 9, 1, 10, 0) == -1


def test_uneven_class_flag(lib):
    """SINCOSM_TUNE_UNEVEN addresses a third table (float64 reverse-pass launches); both
    class flags together are rejected."""
    from paper_2010_00465_amd import autotune
    assert lib.sincosm_tune_num_configs(autotune.UNEVEN) == lib.sincosm_tune_num_configs(0)
    info = (ctypes.c_int32 * 8)()
    assert lib.sincosm_tune_config_info(autotune.UNEVEN, 0, info) == 0
    assert lib.sincosm_tune_set(autotune.UNEVEN, 1 << 40, 1 << 41, 1) == 0
    assert lib.sincosm_tune_set(autotune.UNEVEN, 1 << 40, 1 << 41, -1) == 0
    assert lib.sincosm_tune_set(autotune.UNEVEN | autotune.MULTI, 1 << 40, 1 << 41, 1) == -1
    data = json.load(open(autotune.DEFAULT_CACHE))
    assert "f64_uneven" in data["entries"] and "f32_uneven" not in data["entries"]


def test_batched_class_flag(lib):
    """SINCOSM_TUNE_BATCHED addresses the batched kernel's mode table: three configurations
    (64 x 64 and 32 x 32 output tiles, and the LDS-resident kernel, which reports the largest
    order it holds, 32 in float64 and 64 in float32, as its size and 2 as its "direct" field);
    no other class flag may accompany it."""
    from paper_2010_00465_amd import autotune
    info = (ctypes.c_int32 * 8)()
    for arith, lds in ((0, 32), (1, 64)):
        code = arith | autotune.BATCHED
        assert lib.sincosm_tune_num_configs(code) == 3
        modes = []
        for i in range(3):
            assert lib.sincosm_tune_config_info(code, i, info) == 0
            modes.append((info[0], info[1], info[3], info[4], info[6]))
        assert modes == [(64, 64, 2, 2, 0), (32, 32, 2, 2, 0), (lds, lds, lds // 16, lds // 16, 2)]
        assert lib.sincosm_tune_config_info(code, 3, info) == -1
        assert lib.sincosm_tune_set(code, 1 << 40, 1 << 41, 3) == -1
        assert lib.sincosm_tune_set(code, 1 << 40, 1 << 41, 2) == 0
        assert lib.sincosm_tune_set(code, 1 << 40, 1 << 41, -1) == 0
        for other in (autotune.MULTI, autotune.UNEVEN):
            assert lib.sincosm_tune_set(code | other, 1 << 40, 1 << 41, 0) == -1
    assert lib.sincosm_tune_num_configs(7 | autotune.BATCHED) == 0


def test_padding_rule_matches_library(lib):
    from paper_2010_00465_amd import autotune
    lib.sincosm_matmul_workspace_size.restype = ctypes.c_size_t
    for n in (1, 31, 200, 256, 1000, 1535, 1536, 4096, 4100):
        np_ = autotune.padded(n)
        assert lib.sincosm_matmul_workspace_size(n, 0, 0) == 2 * ((np_ * np_ * 8 + 255) // 256 * 256)


def test_tune_lookup(lib):
    """sincosm_tune_lookup reports what the launches use: later entries win (an entry set
    again for the same range becomes the latest), clearing removes the range, the classes of
    several or unequal problems fall back to the plain table, and the batched tile table
    stands alone (no fallback: its indices are not product-kernel configurations)."""
    from paper_2010_00465_amd import autotune
    lo, hi = 1 << 40, (1 << 40) + 1000          # orders no cache entry covers
    for code in (0, autotune.MULTI, autotune.UNEVEN, autotune.BATCHED):
        assert lib.sincosm_tune_lookup(code, lo) == -1
    try:
        assert lib.sincosm_tune_set(0, lo, hi, 1) == 0
        assert lib.sincosm_tune_lookup(0, lo + 5) == 1
        assert lib.sincosm_tune_lookup(autotune.MULTI, lo + 5) == 1     # falls back to the plain table
        assert lib.sincosm_tune_lookup(autotune.UNEVEN, lo + 5) == 1
        assert lib.sincosm_tune_lookup(autotune.BATCHED, lo + 5) == -1  # no fallback for the batched tile
        assert lib.sincosm_tune_set(0, lo, lo + 10, 2) == 0               # later, narrower entry wins
        assert lib.sincosm_tune_lookup(0, lo + 5) == 2 and lib.sincosm_tune_lookup(0, lo + 500) == 1
        assert lib.sincosm_tune_set(0, lo, hi, 0) == 0                    # the first range again: now the latest
        assert lib.sincosm_tune_lookup(0, lo + 5) == 0 and lib.sincosm_tune_lookup(0, lo + 500) == 0
        assert lib.sincosm_tune_set(autotune.MULTI, lo, hi, 3) == 0
        assert lib.sincosm_tune_lookup(autotune.MULTI, lo + 500) == 3
        assert lib.sincosm_tune_lookup(autotune.UNEVEN, lo + 500) == 0
        assert lib.sincosm_tune_set(autotune.BATCHED, lo, hi, 1) == 0
        assert lib.sincosm_tune_lookup(autotune.BATCHED, lo + 500) == 1
        assert lib.sincosm_tune_lookup(1, lo + 500) == -1                 # other arithmetic untouched
        assert lib.sincosm_tune_lookup(autotune.MULTI | autotune.UNEVEN, lo) == -1
        assert lib.sincosm_tune_lookup(7, lo) == -1
    finally:
        for code in (0, autotune.MULTI, autotune.BATCHED):
            assert lib.sincosm_tune_set(code, lo, hi, -1) == 0
    for code in (0, autotune.MULTI, autotune.BATCHED):
        assert lib.sincosm_tune_lookup(code, lo + 5) == -1
