"""Pins for oracle/plan.py: an independent brute-force enumeration of all
(level, s) candidates, and the committed breakpoint fixture."""
import json
import math
import os

import numpy as np
import pytest

from oracle import plan

GOLD = os.path.join(os.path.dirname(__file__), "golden", "plan_breakpoints.json")


def brute_force(t, acc, extended=False):
    """Enumerate every (level, s) with t <= theta_level * 2^s, s < 2000; pick min products then min s."""
    cands = []
    levels = ((3, 3), (4, 4), (5, 5), (6, 6), (7, 7)) if extended else ((3, 3), (4, 4), (6, 6), (7, 7))
    for level, pi in levels:
        th = plan.THETA_LEVEL5[acc] if level == 5 else plan.THETA[acc][level]
        for s in range(0, 2000):
            if t <= math.ldexp(th, s):
                cands.append((pi + 2 * s, s, level))
                break
    cands.sort()
    cost, s, level = cands[0]
    return level, s, cost


@pytest.mark.parametrize("acc", ["double", "single"])
def test_plan_matches_brute_force(acc):
    g = np.random.default_rng(7)
    ts = list(np.exp2(g.uniform(-30, 40, size=3000))) + [0.0, 1e-300, 1.0, 2.0, 1e300]
    for level, th in plan.THETA[acc].items():
        for s in range(0, 20):
            x = math.ldexp(th, s)
            ts += [x, math.nextafter(x, math.inf), math.nextafter(x, 0.0)]
    for t in ts:
        assert plan.plan(float(t), acc) == brute_force(float(t), acc), t


@pytest.mark.parametrize("acc", ["double", "single"])
def test_extended_plan_matches_brute_force(acc):
    g = np.random.default_rng(8)
    ts = list(np.exp2(g.uniform(-30, 40, size=3000))) + [0.0, 1.0, 2.0]
    bounds = list(plan.THETA[acc].values()) + [plan.THETA_LEVEL5[acc]]
    for th in bounds:
        for s in range(0, 12):
            x = math.ldexp(th, s)
            ts += [x, math.nextafter(x, math.inf), math.nextafter(x, 0.0)]
    for t in ts:
        got = plan.plan(float(t), acc, extended=True)
        assert got == brute_force(float(t), acc, extended=True), t
        assert got[2] <= plan.plan(float(t), acc)[2]


def test_extended_plan_band():
    """The 5-product scheme wins exactly on (theta_4, theta_5] at s = 0 and nowhere else."""
    for acc in ("double", "single"):
        lo, hi = plan.THETA[acc][4], plan.THETA_LEVEL5[acc]
        assert plan.plan(math.nextafter(lo, math.inf), acc, extended=True) == (5, 0, 5)
        assert plan.plan(hi, acc, extended=True) == (5, 0, 5)
        assert plan.plan(math.nextafter(hi, math.inf), acc, extended=True) == (6, 0, 6)
        assert plan.plan(lo, acc, extended=True) == (4, 0, 4)
    for t in np.exp2(np.linspace(-30, 40, 20000)):
        lv = plan.plan(float(t), "double", extended=True)[0]
        assert lv != 5 or plan.THETA["double"][4] < t <= plan.THETA_LEVEL5["double"]


def test_plan_fixture():
    with open(GOLD) as f:
        d = json.load(f)
    for c in d["cases"]:
        t = float.fromhex(c["norm1"])
        assert plan.plan(t, c["accuracy"]) == (c["level"], c["s"], c["products"])


def test_known_points():
    # config anchors ||A||_1 = 2^e, e in {-4, 0, 4, 10}, double table: 4 / 7 / 15 / 27 products
    assert [plan.plan(2.0 ** e)[2] for e in (-4, 0, 4, 10)] == [4, 7, 15, 27]
    assert plan.plan(2.0) == (7, 1, 9)
    assert plan.plan(64.0, "single") == (7, 4, 15)
    assert plan.plan(64.0, "double") == (7, 6, 19)


def test_plan_rejects_nonfinite():
    for t in (math.nan, math.inf, -1.0):
        with pytest.raises(ValueError):
            plan.plan(t)
