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
    ("atanh", "LENS_ATANH_COEFFS", "LENS_ATANH_N", float.fromhex(D["LENS_ATANH_R_MAX"]),
     mp.atanh),
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


def reduction_bound():
    """|s| after the hyperbolic arctangent's reduction: k read from the high
    words is within 1/2 + max(log2(1 + m) - m) + 2^-20 of log2(P/Q)."""
    g = -math.log(math.log(2)) / math.log(2) - 1 / math.log(2) + 1
    r = 2.0 ** (0.5 + g + 2.0 ** -20)
    return (r - 1) / (r + 1)


def test_reduction_interval_bound():
    assert float.fromhex(D["LENS_ATANH_R_MAX"]) == pytest.approx(reduction_bound(), rel=1e-12)
    assert float.fromhex(D["LENS_ATANH_R_MAX"]) > 3 - 2 * math.sqrt(2)


def hi_word(v):
    return int.from_bytes(__import__("struct").pack(">d", v)[:4], "big")


def test_reduction_keeps_the_quotient_inside_the_interval():
    """The kernels' k = (hi(P) - hi(Q) + 2^19) >> 20 for P = D + N, Q = D - N:
    over random pairs, pairs whose mantissas sit where log2(1 + m) - m peaks,
    and exponent gaps up to 60, |(P 2^-k - Q)/(P 2^-k + Q)| stays within the
    bound the polynomial is fitted on, and k is within one of the rounded
    log2(P/Q)."""
    import random
    rng = random.Random(5)
    bound = float.fromhex(D["LENS_ATANH_R_MAX"])
    m_star = 1 / math.log(2) - 1
    cases = []
    for _ in range(20000):
        cases.append((2.0 ** rng.uniform(-40, 40), 2.0 ** rng.uniform(-40, 40)))
    for e in range(-60, 61):
        for mp_, mq in ((m_star, 0.0), (0.0, m_star), (m_star, 0.999999), (0.999999, m_star)):
            for h in (0.49, 0.5, 0.51):
                cases.append(((1 + mp_) * 2.0 ** (e + h), (1 + mq)))
    worst = 0.0
    for P, Q in cases:
        k = (hi_word(P) - hi_word(Q) + (1 << 19)) >> 20
        r = P * 2.0 ** -k / Q
        s = (r - 1) / (r + 1)
        worst = max(worst, abs(s))
        assert abs(k - math.log2(P / Q)) <= 0.5 + 0.0861 + 1e-6
    assert worst <= bound, worst


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
