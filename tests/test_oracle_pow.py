"""pow() in the oracle's predicates (Sec. 3.1, func), pinned without the GPU.

The paper names pow among the functions of a predicate but fixes no rounding.
The reading both sides follow: for an integral exponent k in 0..64, the
product of k factors formed by binary powering (square, then multiply where
the exponent bit is set, most significant bit first), each step one rounded
multiplication; any other exponent takes the C library's pow.  Pins:
- integer bases: the exact integer power whenever it is below 2^53 (every
  intermediate product is then an exact integer, whatever the order);
- the order of the multiplications, through the predicate language's own
  product for k = 2, 3, 4, 5, 6 and 13 on bases that are not exact (a plain
  left-to-right product gives other roundings on some of them);
- the error bound of binary powering, |r - x^k| <= k u |x^k| (u = 2^-53),
  against the exact rational power;
- exponents outside 0..64 or not integral: the C library's values where they
  are exact (square roots of squares, powers of two).
"""
import math
from fractions import Fraction

import pytest

from oracle import bltlc
import oracle

NAMES = ["X"]


def holds(text, x):
    f = bltlc.parse(text, NAMES)
    return oracle.eval_prefix(f, [[x]], [0.0], None) == 1


@pytest.mark.parametrize("k", range(0, 9))
def test_integer_powers_are_exact(k):
    for x in (0, 1, 2, 3, 7, 10, 31, 60, 999, 4096):
        v = x ** k
        if v >= 2 ** 53:
            continue
        assert holds(f"pow(X,{k}) = {v}", x), (x, k)
        assert not holds(f"pow(X,{k}) = {v + 1}", x), (x, k)


def _square_multiply(k):
    """The binary-powering product as a predicate expression over q = X/7
    (e.g. k = 5: ((q q)(q q)) q), built from k's bits, leading bit first."""
    expr = None
    for bit in bin(k)[2:]:
        if expr is not None:
            expr = f"(({expr})*({expr}))"
        if bit == "1":
            expr = "(X/7)" if expr is None else f"(({expr})*(X/7))"
    return expr


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 13])
def test_multiplication_order_is_binary_powering(k):
    naive = "*".join(["(X/7)"] * k)
    differs = 0
    for x in range(1, 200):
        assert holds(f"pow(X/7,{k}) = {_square_multiply(k)}", x), (x, k)
        differs += not holds(f"pow(X/7,{k}) = {naive}", x)
    if k >= 4:
        assert differs > 0   # the pin separates the two orders


@pytest.mark.parametrize("k", [7, 19, 33, 64])
def test_error_bound_of_binary_powering(k):
    u = Fraction(1, 2 ** 53)
    for x in (3, 11, 41, 100, 173):
        q = Fraction(x / 7.0)               # the double the predicate divides to
        exact = q ** k
        lo, hi = float(exact * (1 - k * u * Fraction(101, 100))), float(exact * (1 + k * u * Fraction(101, 100)))
        assert holds(f"pow(X/7,{k}) >= {lo!r} & pow(X/7,{k}) <= {hi!r}", x), (x, k)


def test_other_exponents_use_the_library_pow():
    assert holds("pow(X,0.5) = 7", 49)
    assert holds("pow(X,65) = 36893488147419103232", 2)      # 2^65, outside 0..64
    assert holds("pow(X,-2) = 0.0625", 4)
    assert holds("pow(X,1.5) = 8", 4)
    assert math.pow(49, 0.5) == 7.0
