"""The paper's factorized Taylor schemes (oracle, test infrastructure).

Section 2.1 of the paper gives, for k = 3, 4, 6, 7 matrix products, a scheme
that evaluates an approximation of cos(A) and sin(A) simultaneously:

* k = 3: equations (Algorithm3cA) and (Algorithm3sA): T^c_4 and T^s_5.
* k = 4: equations (Algorithm4cA) and (Algorithm4sA): T^c_8 and T^s_{7,9}.
* k = 5: (Algorithm4cA) with the sine raised to order nine by (Algorithm5sA):
  T^c_8 and T^s_9 (not in Tables 1-2; used only by the extended plan).
* k = 6: equations (Algorithm6cA) with coefficients (eq:cosm8), and
  (Algorithm6sA) with the rational z_0..z_8: T^c_16 and T^s_{17,25}.
* k = 7: equations (Algorithm7cA) with (Coefs7cA), and (Algorithm7sA) with
  (Coefs7sA): T^c_24 and the degree-49 sine approximation.

The scheme functions are written once over a generic algebra: they use ``@``
for the matrix product, ``+``/``-`` and multiplication by scalars, and an
identity element ``I``. Passing numpy matrices evaluates the scheme on a
matrix; passing ``Poly`` objects (scalar polynomials with mpmath coefficients)
yields the polynomial each scheme represents, which the tests compare with
the Taylor coefficients and which ``theta`` uses to bound the truncation
error.

Reading of the paper taken here:

* In (Algorithm6sA) the identity and A_2 terms of C_24 carry the same
  coefficient z_5, as printed (solving for two separate unknowns gives the
  same value).
* In (Algorithm7sA) the left-hand side is written T^s_{23,49}(B); it is read
  as a function of A.
* The 20-digit decimals of (Coefs7cA) and (Coefs7sA) are parsed exactly
  (mpmath) and rounded only when a float scheme is built.

Pins (tests/test_oracle_schemes.py): the scalar polynomial of each scheme
equals the Taylor series of cos / sin through the order the paper states
(exact rational identity for k = 3, 4, 6; relative 1e-17 for k = 7 whose
coefficients are printed to 20 digits), and each scheme's product count
matches Tables 1 and 2.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np

__all__ = ["Poly", "coefficients", "float_coefficients", "level3", "level4", "level5",
           "level6", "level7", "SCHEMES", "PRODUCTS", "CountingMatrix"]

# Products per scheme (Tables 1 and 2, row Pi_{2m}; k = 5 from Algorithm5sA).
PRODUCTS = {3: 3, 4: 4, 5: 5, 6: 6, 7: 7}


def coefficients(dps: int = 60):
    """Coefficient sets of the k = 6 and k = 7 schemes as mpmath numbers.

    Returns a dict with keys 'x' (x_1..x_8 of eq:cosm8), 'z6' (z_0..z_8 of the
    k = 6 sine), 'a' (a_{i,j}, i = 0..3, j = 1..4 of Coefs7cA) and 'z7'
    (z_0..z_11 of Coefs7sA).
    """
    with mpmath.workdps(dps):
        r = mpmath.sqrt(36681)
        F = mpmath.mpf
        x = {
            1: F(7) / 500,
            2: F(-7) / 60000,
            3: (F(-1533) + 7 * r) / 2500,
            4: -5 * (F(124581) + 391 * r) / 10594584,
            5: F(9775) / 10594584,
            6: -5 * (F(1001) + r) / 508540032,
            7: F(3125) / 889945056,
            8: (F(1549211) + 3246 * r) / 63063000,
        }
        z6 = {
            0: F(8887) / 4794,
            1: F(-1897) / 3196,
            2: F(25259) / 575280,
            3: F(-965093875) / 9674368704,
            4: F(-4093) / 4794,
            5: F(25698275) / 29023106112,
            6: F(-3907675) / 348277273344,
            7: F(11865625) / 3656911370112,
            8: F(25) / 308756448,
        }
        a = {
            (0, 1): F("0"),
            (1, 1): F("0"),
            (2, 1): F("0.02264979811206039519"),
            (3, 1): F("-0.00013110924142135755"),
            (0, 2): F("0.55751443809990408029"),
            (1, 2): F("-0.61577924683458386455"),
            (2, 2): F("0.00747198841446687051"),
            (3, 2): F("-0.00003362444420476012"),
            (0, 3): F("0.75936877868464999248"),
            (1, 3): F("-0.01560333979813817129"),
            (2, 3): F("0.00010936989591908396"),
            (3, 3): F("-1.03893360877457159499e-6"),
            (0, 4): F("0"),
            (1, 4): F("-0.039649968743474473091"),
            (2, 4): F("0.000155490073503821463"),
            (3, 4): F("-1.126739663071170022488e-6"),
        }
        z7 = {
            0: F("0.10090808375109885598"),
            1: F("-0.07668753546445299316"),
            2: F("0.00084924846993243257"),
            3: F("-0.00001220406904464391"),
            4: F("0.98499703159318860027"),
            5: F("-0.84925233648155398756"),
            6: F("1"),
            7: F("0.00095544138280925799"),
            8: F("4.56337109377154270633e-6"),
            9: F("2.73461259403000427141e-8"),
            10: F("0.00048550288474842477"),
            11: F("-4.15891109384923342531e-7"),
        }
    return {"x": x, "z6": z6, "a": a, "z7": z7}


def float_coefficients():
    """The same sets rounded to float64 (correct rounding of the mp values)."""
    c = coefficients()
    return {k: {kk: float(v) for kk, v in d.items()} for k, d in c.items()}


class Poly:
    """Scalar polynomial with mpmath coefficients, closed under the scheme ops."""

    __array_priority__ = 100

    def __init__(self, coeffs):
        self.c = [mpmath.mpf(v) if not isinstance(v, mpmath.mpf) else v for v in coeffs]

    @staticmethod
    def x():
        return Poly([0, 1])

    @staticmethod
    def one():
        return Poly([1])

    def _lift(self, other):
        if isinstance(other, Poly):
            return other
        if isinstance(other, Fraction):
            other = mpmath.mpf(other.numerator) / other.denominator
        return Poly([other])

    def __add__(self, other):
        o = self._lift(other)
        n = max(len(self.c), len(o.c))
        a = self.c + [mpmath.mpf(0)] * (n - len(self.c))
        b = o.c + [mpmath.mpf(0)] * (n - len(o.c))
        return Poly([p + q for p, q in zip(a, b)])

    __radd__ = __add__

    def __neg__(self):
        return Poly([-v for v in self.c])

    def __sub__(self, other):
        return self + (-self._lift(other))

    def __rsub__(self, other):
        return self._lift(other) - self

    def __mul__(self, s):
        if isinstance(s, Poly):
            raise TypeError("use @ for the polynomial product")
        if isinstance(s, Fraction):
            s = mpmath.mpf(s.numerator) / s.denominator
        return Poly([v * s for v in self.c])

    __rmul__ = __mul__

    def __truediv__(self, s):
        return Poly([v / s for v in self.c])

    def __matmul__(self, other):
        o = self._lift(other)
        out = [mpmath.mpf(0)] * (len(self.c) + len(o.c) - 1)
        for i, p in enumerate(self.c):
            if p == 0:
                continue
            for j, q in enumerate(o.c):
                out[i + j] += p * q
        return Poly(out)

    def coeff(self, k):
        return self.c[k] if k < len(self.c) else mpmath.mpf(0)

    @property
    def degree(self):
        d = len(self.c) - 1
        while d > 0 and self.c[d] == 0:
            d -= 1
        return d


class CountingMatrix:
    """Wraps a value and counts the products (``@``) made while evaluating a scheme."""

    def __init__(self, counter):
        self.counter = counter

    def __matmul__(self, other):
        self.counter[0] += 1
        return CountingMatrix(self.counter)

    def __add__(self, other):
        return CountingMatrix(self.counter)

    __radd__ = __add__
    __sub__ = __add__
    __rsub__ = __add__

    def __neg__(self):
        return self

    def __mul__(self, s):
        return CountingMatrix(self.counter)

    __rmul__ = __mul__
    __truediv__ = __mul__


# ---------------------------------------------------------------------------
# The schemes.  ``A`` is the (already scaled) argument, ``I`` the identity of
# the same algebra, ``c`` a coefficient dict as returned by coefficients() or
# float_coefficients().  Each returns (cosine approximation, sine approximation).
# ---------------------------------------------------------------------------

def level3(A, I, c=None):
    """k = 3: T^c_4 with two products, T^s_5 with one more (Algorithm3cA/3sA)."""
    A2 = A @ A
    A4 = A2 @ A2
    Tc = I - A2 / 2 + A4 / 24
    Ts = A @ (I - A2 / 6 + A4 / 120)
    return Tc, Ts


def level4(A, I, c=None):
    """k = 4: T^c_8 with three products, T^s_{7,9} with one more (Algorithm4cA/4sA)."""
    A2 = A @ A
    A4 = A2 @ A2
    A8 = A4 @ (-A2 / 720 + A4 / 40320)
    Tc = I - A2 / 2 + A4 / 24 + A8
    Ts = A @ (I - A2 / 6 + A4 / 120 + A8 / 7)     # 6!/7! = 1/7
    return Tc, Ts


def level5(A, I, c=None):
    """k = 5: T^c_8 of Algorithm4cA (three products) and T^s_9 of Algorithm5sA, whose own A_8
    uses 1/7! and 1/9! (one product) before the final product with A."""
    A2 = A @ A
    A4 = A2 @ A2
    A8c = A4 @ (-A2 / 720 + A4 / 40320)
    Tc = I - A2 / 2 + A4 / 24 + A8c
    A8s = A4 @ (-A2 / 5040 + A4 / 362880)
    Ts = A @ (I - A2 / 6 + A4 / 120 + A8s)
    return Tc, Ts


def level6(A, I, c):
    """k = 6: T^c_16 with four products (Algorithm6cA), T^s_{17,25} with two more (Algorithm6sA)."""
    x, z = c["x"], c["z6"]
    A2 = A @ A
    A4 = A2 @ A2
    A8 = A4 @ (x[1] * A2 + x[2] * A4)
    A16 = (x[3] * A4 + A8) @ (x[4] * I + x[5] * A2 + x[6] * A4 + x[7] * A8)
    Tc = I - A2 / 2 + x[8] * A4 + A16
    C24 = (z[5] * I + z[5] * A2 + z[6] * A4 + z[7] * A8 + z[8] * Tc) @ A8
    Ts = A @ (z[0] * I + z[1] * A2 + z[2] * A4 + z[3] * A8 + z[4] * Tc + C24)
    return Tc, Ts


def level7(A, I, c):
    """k = 7: T^c_24 with five products (Algorithm7cA), the sine with two more (Algorithm7sA)."""
    a, z = c["a"], c["z7"]
    A2 = A @ A
    A4 = A2 @ A2
    A6 = A4 @ A2
    Cj = {j: a[(0, j)] * I + a[(1, j)] * A2 + a[(2, j)] * A4 + a[(3, j)] * A6
          for j in (1, 2, 3, 4)}
    A12 = Cj[3] + Cj[4] @ Cj[4]
    A24 = (Cj[2] + A12) @ A12
    Tc = Cj[1] + A24
    C48 = (z[6] * I + z[7] * A2 + z[8] * A4 + z[9] * A6 + z[10] * A12 + z[11] * Tc) @ Tc
    Ts = A @ (z[0] * I + z[1] * A2 + z[2] * A4 + z[3] * A6 + z[4] * A12 + z[5] * Tc + C48)
    return Tc, Ts


SCHEMES = {3: level3, 4: level4, 5: level5, 6: level6, 7: level7}


def scheme_polynomials(level: int, dps: int = 60):
    """The (cosine, sine) scalar polynomials represented by a scheme, mpmath coefficients."""
    with mpmath.workdps(dps):
        c = coefficients(dps)
        return SCHEMES[level](Poly.x(), Poly.one(), c)


def count_products(level: int) -> int:
    """Number of ``@`` products the scheme makes (checks the paper's Pi)."""
    counter = [0]
    SCHEMES[level](CountingMatrix(counter), CountingMatrix(counter),
                   {"x": {i: 1.0 for i in range(1, 9)}, "z6": {i: 1.0 for i in range(9)},
                    "a": {(i, j): 1.0 for i in range(4) for j in range(1, 5)},
                    "z7": {i: 1.0 for i in range(12)}})
    return counter[0]


def evaluate(level: int, X: np.ndarray, dtype=np.float64):
    """Evaluate a scheme on a (scaled) matrix X in ``dtype`` arithmetic."""
    X = np.asarray(X, dtype=dtype)
    I = np.eye(X.shape[0], dtype=dtype)
    fc = float_coefficients()
    if dtype is not np.float64:
        fc = {k: {kk: dtype(v) for kk, v in d.items()} for k, d in fc.items()}
    return SCHEMES[level](X, I, fc)
