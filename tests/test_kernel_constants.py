"""Host checks of constants the GPU kernels carry (CPU only).

The float64 pair sums evaluate 2^f on [-1/2, 1/2] by the Taylor series of
exp(f ln 2) to degree 13; its coefficients, written in the kernel source as
float64 hex literals, must be (ln 2)^k / k! rounded to the nearest double,
and the series must reach 2^f within a few units in the last place."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1305_5179_amd", "csrc", "pairsum.hip")

# ln 2 to 60 digits
LN2 = "0.693147180559945309417232121458176568075500134360255254120680009493393621969694715605863"


def _coefficients():
    text = open(SRC).read()
    m = re.search(r"constexpr double C\[14\] = \{(.*?)\};", text, re.S)
    assert m, "coefficient table not found"
    vals = [float.fromhex(v.strip()) for v in m.group(1).split(",") if v.strip()]
    assert len(vals) == 14
    return vals


def test_exp2_coefficients_are_the_rounded_taylor_terms():
    getcontext().prec = 80
    ln2 = Decimal(LN2)
    c = Decimal(1)
    for k, got in enumerate(_coefficients()):
        if k:
            c = c * ln2 / k
        # nearest double: exact comparison through fractions
        want = float(c)
        assert got == want, (k, got.hex(), want.hex())
        assert abs(Fraction(got) - Fraction(c)) <= Fraction(math.ulp(got)) / 2


def test_exp2_series_accuracy():
    C = _coefficients()
    getcontext().prec = 40
    worst = 0.0
    for i in range(4001):
        f = -0.5 + i / 4000.0
        p = C[13]
        for k in range(12, -1, -1):
            p = p * f + C[k]
        exact = Decimal(2) ** Decimal(f)
        worst = max(worst, float(abs((Decimal(p) - exact) / exact)))
    assert worst < 3 * 2.0 ** -53, worst
