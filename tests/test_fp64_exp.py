"""The FP64 pair exponential of the near-field kernels (exp_pair in
paper_1008_2410_amd/csrc/device_common.h): e = exp(-s) and g = 1 - exp(-s) by Cody-Waite
reduction and a polynomial for expm1.  Its steps are emulated here in double arithmetic with
every fused multiply-add rounded once (exact rational product and sum, then one rounding),
using the constants read from the source, and compared with 50-digit references: both within
1.5 ulp over s in [1e-300, 50], g without cancellation for small s (the kernel of eq.
regB-S2DGau needs 1 - exp(-s) to full relative precision near s = 0)."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction as Fr

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_1008_2410_amd", "csrc", "device_common.h")


def _routine():
    text = open(SRC).read()
    body = text[text.index("void exp_pair(double s, double &e, double &g)"):]
    body = body[:body.index("\n}\n")]
    consts = dict(re.findall(r"(kInvLn2|kLn2Hi|kLn2Lo) = ([0-9.e+-]+)", body))
    first = float(re.search(r"double p = ([0-9.e+-]+);", body).group(1))
    chain = [float(c) for c in re.findall(r"p = fma\(p, x, ([0-9.e+-]+)\);", body)]
    return {k: float(v) for k, v in consts.items()}, [first] + chain


def _fma(a, b, c):
    return float(Fr(a) * Fr(b) + Fr(c))


def _exp_pair(s, consts, coef):
    k = float(round(s * consts["kInvLn2"]))  # round half to even, as rint
    x = -_fma(-k, consts["kLn2Lo"], _fma(-k, consts["kLn2Hi"], s))
    p = coef[0]
    for c in coef[1:]:
        p = _fma(p, x, c)
    em1 = p * x
    t = math.ldexp(1.0, -int(k))
    return _fma(t, em1, t), _fma(-t, em1, 1.0 - t)


def test_fp64_exp_pair_within_an_ulp():
    getcontext().prec = 50
    consts, coef = _routine()
    assert len(consts) == 3 and len(coef) >= 8
    worst_e = worst_g = 0.0
    n = 1500
    for i in range(n):
        s = 10 ** (-300 + 301.7 * i / (n - 1)) if i % 2 == 0 else 50.0 * (i + 0.5) / n
        d = Decimal(s)
        ref_e = (-d).exp()
        ref_g = (d - d * d / 2 + d ** 3 / 6 - d ** 4 / 24) if s < 1e-5 else 1 - ref_e
        e, g = _exp_pair(s, consts, coef)
        worst_e = max(worst_e, float(abs(Decimal(e) - ref_e) / Decimal(math.ulp(float(ref_e)))))
        worst_g = max(worst_g, float(abs(Decimal(g) - ref_g) / Decimal(math.ulp(float(ref_g)))))
    assert worst_e < 1.5, worst_e
    assert worst_g < 1.5, worst_g
