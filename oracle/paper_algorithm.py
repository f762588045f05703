"""The paper's method written out plainly (oracle, test infrastructure).

cos(A), sin(A) by (Section 1, Section 2.1, Tables 1-2, Section 4):

1. theta = ||A||_1 (exact, ``reference.norm1``).
2. (level, s) from ``plan.plan``.
3. X = 2^-s A.
4. The level's scheme on X (``schemes``), giving C ~ cos X and S ~ sin X.
5. s double-angle steps from the old pair: C <- I - 2 S S, S <- 2 S C.

This replica uses exactly the integers (level, s) the product path must
choose, so the product path can be compared with it more tightly than with
the independent ``reference`` algorithm. It is evaluated in float64 (or long
double) with numpy matmul.

Pins: at s = 0 it is checked against ``reference`` (independent Taylor /
Horner) and against mpmath's cosm/sinm; its plans against ``plan``'s
brute-force pin (tests/test_oracle_paper_algorithm.py).
"""
from __future__ import annotations

import numpy as np

from . import plan as _plan
from . import schemes as _schemes
from .reference import norm1

__all__ = ["sincosm", "plan_for"]


def plan_for(A: np.ndarray, accuracy: str = "double", extended: bool = False, refined: bool = False):
    """(level, s, products) for A (``extended``: the 5-product scheme is a candidate too;
    ``refined``: plan on min(||A||_1, ||A^2||_1^(1/2)))."""
    theta = _plan.refined_theta(A) if refined else norm1(A)
    return _plan.plan(theta, accuracy, extended)


def sincosm(A: np.ndarray, accuracy: str = "double", dtype=np.float64, return_plan=False, extended=False,
            refined=False):
    """cos(A), sin(A) by the paper's method in ``dtype`` arithmetic."""
    A = np.asarray(A, dtype=dtype)
    n = A.shape[0]
    I = np.eye(n, dtype=dtype)
    level, s, products = plan_for(A, accuracy, extended, refined)
    X = A * dtype(2.0) ** (-s)
    C, S = _schemes.evaluate(level, X, dtype=dtype)
    for _ in range(s):
        C, S = I - dtype(2) * (S @ S), dtype(2) * (S @ C)
    if return_plan:
        return C, S, (level, s, products)
    return C, S
