"""Choice of scheme and scaling power (oracle, test infrastructure).

Tables 1 and 2 give, for each scheme k in {3, 4, 6, 7} products, the largest
norms theta^c and theta^s for which the cosine and sine truncation errors stay
below the unit roundoff, and Section 4 combines the schemes with scaling by
2^-s and s double-angle steps (2 products each, Section 1).

Readings taken (the paper only shows the resulting staircase in its Figure 1):

* Both outputs share one scaling, so a scheme is usable for theta <= the
  smaller of its two bounds.
* (level, s) minimises the total number of products Pi_level + 2 s, where s
  is the smallest integer >= 0 with theta 2^-s <= theta_level; ties go to the
  smaller s. s is found by exact halving, never through a floating log2.
* The 7-product sine bound in double precision is 1.8548 (re-derived from the
  printed coefficients) instead of the printed 1.97.
* Extended plan (opt-in, not the paper's tables): the 5-product scheme of
  Algorithm4cA + Algorithm5sA joins the candidates. Its sine bound (T^s_9,
  derived as for the tables: 1.7401e-1 double, 1.0812 single) exceeds its
  cosine's, so its combined bound is the printed T^c_8 bound of Tables 1-2:
  1.1495e-1 (double), 8.5756e-1 (single).
* Refined norm (opt-in, not in the paper): Section 4 tests [[1, lambda],
  [0, -1]] up to lambda = 1e8, where ||A||_1 is huge but A^2 = I, and notes
  the overscaling this causes. Every scheme is a polynomial in Y = X^2 (the
  sine times X), so its truncation error is bounded by the same series in
  ||Y||^(1/2): the plan may use theta' = min(||A||_1, ||A^2||_1^(1/2)), with A^2
  the product the schemes form first anyway. The cosine bound then holds as
  in Tables 1-2; the sine's bound becomes u ||X|| / theta_level relative to X
  (Al-Mohy and Higham's use of ||A^p||^(1/p), restricted to p = 2).

Pins (tests/test_oracle_plan.py): a brute-force enumeration over all
(level, s) candidates written independently, and the table constants against
the theta re-derivation of ``theta``.
"""
from __future__ import annotations

import math

__all__ = ["THETA", "THETA_LEVEL5", "PRODUCTS", "plan", "scaling_for", "refined_theta"]

PRODUCTS = {3: 3, 4: 4, 5: 5, 6: 6, 7: 7}

# min(theta^c, theta^s) per scheme; Table 1 (u = 2^-53) and Table 2 (u = 2^-24).
THETA = {
    "double": {3: 6.5633e-3, 4: 8.0438e-2, 6: 9.8108e-1, 7: 1.8548},
    "single": {3: 1.8709e-1, 4: 7.492e-1, 6: 2.9935, 7: 4.3819},
}
# combined bound of the 5-product scheme (extended plan only)
THETA_LEVEL5 = {"double": 1.1495e-1, "single": 8.5756e-1}


def scaling_for(theta: float, limit: float) -> int:
    """Smallest s >= 0 with theta * 2^-s <= limit (exact halving)."""
    s = 0
    t = float(theta)
    while t > limit:
        t *= 0.5
        s += 1
    return s


def plan(theta: float, accuracy: str = "double", extended: bool = False):
    """Return (level, s, products) for a matrix of 1-norm ``theta``.

    ``extended`` adds the 5-product scheme to the candidates.
    Raises ValueError for a non-finite or negative norm.
    """
    if not math.isfinite(theta) or theta < 0:
        raise ValueError("norm must be finite and >= 0")
    bounds = dict(THETA[accuracy])
    if extended:
        bounds[5] = THETA_LEVEL5[accuracy]
    best = None
    for level in sorted(bounds):
        s = scaling_for(theta, bounds[level])
        cand = (PRODUCTS[level] + 2 * s, s, level)
        if best is None or cand[:2] < best[:2]:
            best = cand
    cost, s, level = best
    return level, s, cost


def refined_theta(A) -> float:
    """min(||A||_1, ||A^2||_1^(1/2)) with A^2 formed in float64 (NaN or Inf propagate)."""
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    t1 = float(np.abs(A).sum(axis=0).max()) if A.size else 0.0
    if not math.isfinite(t1):
        return t1
    t2 = float(np.abs(A @ A).sum(axis=0).max()) if A.size else 0.0
    if not math.isfinite(t2):
        return t1
    return min(t1, math.sqrt(t2))
