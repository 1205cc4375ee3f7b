"""Host checks of the polynomial coefficients the FP64 kernels evaluate
(paper_2004_06352_amd/csrc/series_coeffs.h): each polynomial, evaluated in
FP64 in the kernels' Horner order, stays within a few units in the last place
of the arctangent or hyperbolic arctangent (mpmath at 40 digits) over its
whole interval, and the intervals are the ones the reductions leave."""
import math
import os
import re

import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2004_06352_amd", "csrc", "series_coeffs.h")


def defines():
    out = {}
    for line in open(HEADER):
        m = re.match(r"#define (LENS_\w+) (.*)$", line.strip())
        if m:
            out[m.group(1)] = m.group(2)
    return out


def hexlist(text):
    return [float.fromhex(t.strip()) for t in text.split(",")]


def horner(x, coeffs):
    """b + b^3 p(b^2) with p in Horner form, FP64 with one rounding per
    operation as the kernels' FMAs do (the FMA's single rounding is taken
    from a 40-digit product and sum)."""
    def fma(a, b, c):
        return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))
    x2 = x * x
    p = coeffs[0]
    for c in coeffs[1:]:
        p = fma(p, x2, c)
    return fma(x * x2, p, x)


D = defines()
CASES = [
    ("atan", "LENS_ATAN_COEFFS", "LENS_ATAN_N", math.tan(math.pi / 16), mp.atan),
    ("atanh", "LENS_ATANH_COEFFS", "LENS_ATANH_N", 3 - 2 * math.sqrt(2), mp.atanh),
    ("atan short", "LENS_ATAN_S_COEFFS", "LENS_ATAN_S_N", math.tan(math.pi / 16) / 5, mp.atan),
    ("atanh short", "LENS_ATANH_S_COEFFS", "LENS_ATANH_S_N", (3 - 2 * math.sqrt(2)) / 5,
     mp.atanh),
]


@pytest.mark.parametrize("name,key,nkey,bound,fn", CASES, ids=[c[0] for c in CASES])
def test_polynomial_within_few_ulp(name, key, nkey, bound, fn):
    mp.mp.dps = 40
    coeffs = hexlist(D[key])
    assert len(coeffs) == int(D[nkey])
    worst = 0.0
    for i in range(1, 2001):
        for x in (bound * i / 2000, -bound * i / 2000):
            got = horner(x, coeffs)
            ref = fn(mp.mpf(x))
            worst = max(worst, float(abs((mp.mpf(got) - ref) / ref)))
    # FP64 evaluation: a few roundings of the last terms on top of the fit
    assert worst < 4 * 2.0 ** -53, f"{name}: {worst:.3g}"


def test_short_interval_bounds():
    assert float.fromhex(D["LENS_ATAN_S_MAX"]) == pytest.approx(math.tan(math.pi / 16) / 5,
                                                                rel=1e-15)
    assert float.fromhex(D["LENS_ATANH_S_MAX"]) == pytest.approx((3 - 2 * math.sqrt(2)) / 5,
                                                                 rel=1e-15)


@pytest.mark.parametrize("name,short", [("atan", False), ("atanh", False), ("atan", True),
                                        ("atanh", True)])
def test_fp32_taylor_tiers(name, short):
    """The FP32 path's Taylor polynomials (to the ninth power on the whole
    reduced interval, to the fifth on its first fifth), evaluated in FP32 in
    the kernels' order, stay within 3 FP32 units of the true function."""
    np = pytest.importorskip("numpy")
    sign = -1.0 if name == "atan" else 1.0
    coeffs = [np.float32(sign ** (4 - i) / (9 - 2 * i)) for i in range(4)]  # 1/9 .. 1/3
    if short:
        coeffs = coeffs[2:]
    full = math.tan(math.pi / 16) if name == "atan" else 3 - 2 * math.sqrt(2)
    bound = full / 5 if short else full
    fn = math.atan if name == "atan" else math.atanh
    worst = 0.0
    for i in range(1, 4001):
        b = np.float32(bound * i / 4000)
        b2 = np.float32(b * b)
        p = coeffs[0]
        for c in coeffs[1:]:
            p = np.float32(p * b2 + c)
        got = np.float32(np.float32(b * b2) * p + b)
        ref = fn(float(b))
        worst = max(worst, abs(float(got) - ref) / ref)
    assert worst < 3 * 2.0 ** -24, f"{name} short={short}: {worst:.3g}"
