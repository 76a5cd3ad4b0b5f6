"""The constants of the GPU's exponential rounded to nearest (the Gaussian
source, csrc/stencil.hpp), checked with exact rational arithmetic: ln 2 split
into three doubles whose sum is within 2^-140 of ln 2 and whose first part has
at most 32 significant bits (so k L1 is exact for |k| <= 2^11), and 1/n! for
n = 2..10 as (high, low) pairs rounded to nearest."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2311_13862_amd", "csrc", "stencil.hpp")


def hexfloats(text):
    return [float.fromhex(t) for t in re.findall(r"-?0x[0-9a-f.]+p[-+]?\d+", text)]


def section():
    s = open(SRC).read()
    i = s.index("__device__ inline double exp_rn")
    return s[i:s.index("const double kd", i)]


def test_ln2_split():
    text = section()
    L1, L2, L3 = hexfloats(re.search(r"constexpr double L1 = .*?;", text).group(0))
    getcontext().prec = 90
    ln2 = Fraction(Decimal(2).ln())
    err = abs(ln2 - Fraction(L1) - Fraction(L2) - Fraction(L3))
    assert err < Fraction(1, 2 ** 140)
    m, e = math.frexp(L1)
    assert (Fraction(m) * 2 ** 32).denominator == 1  # at most 32 significant bits
    assert abs(L2) < 2 ** -33 and abs(L3) < 2 ** -86


def test_inverse_factorials():
    text = section()
    ch = hexfloats(re.search(r"CH\[9\] = \{.*?\};", text, re.S).group(0))
    cl = hexfloats(re.search(r"CL\[9\] = \{.*?\};", text, re.S).group(0).replace("0.0,", "0x0p+0,"))
    assert len(ch) == 9 and len(cl) == 9
    for n in range(2, 11):
        c = Fraction(1, math.factorial(n))
        hi = float(c)
        lo = float(c - Fraction(hi))
        assert ch[n - 2] == hi and cl[n - 2] == lo, n
