"""The fitted polynomials the pair kernels evaluate (csrc/hct_poly.inc), checked
on the CPU against the functions they stand for, written out independently of
the fitting script.

For a non-overlapping descreening sphere the HCT integral is H = g(x)/r with
x = S/r and g(x) = (x/(1 - x^2) - atanh x)/2 (the published HCT pair integral
of the GB-OBC model the paper names, Sec. III.D), whose Taylor series is
g(x) = x^3 sum_{k>=1} k x^(2k-2) / (2k + 1); the kernels evaluate P(y) = g(x)/x^3, y = x^2, and the factor
W(y) = (1 - y)^-2 of its derivatives.  Each fit is evaluated here by Horner's
rule in its own precision (products and sums rounded separately, a bound on
the fused form the kernels use) on a fine grid of its stated domain, and must
meet the error its header states; the domain macros must match the headers."""
import os
import re

import mpmath
import numpy as np
import pytest

INC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1803_09652_amd", "csrc", "hct_poly.inc")


def parse():
    """{name: (function letter, degree, ymax, stated error, C type, coefficients
    highest first)} and {macro: value} from the generated header."""
    text = open(INC).read()
    fits = {}
    for m in re.finditer(r"// (\w+): ([PW]), degree (\d+) on y in \[0, ([\d.]+)\]; max relative "
                         r"error ([\d.e+-]+) in (float|double)\.\n(?:#define \w+ [\d.]+f?\n)?"
                         r"__device__ __forceinline__ \w+ \1\(\w+ y\) \{\n(.*?)\n    return p;",
                         text, re.S):
        name, fn, deg, ymax, err, ctype, body = m.groups()
        coef = [float(v.rstrip("f")) for v in
                re.findall(r"([-+]?\d\.\d+e[-+]\d+f?)", body)]
        fits[name] = (fn, int(deg), float(ymax), float(err), ctype, coef)
    macros = {k: float(v.rstrip("f")) for k, v in
              re.findall(r"#define (\w+) ([\d.]+f?)", text)}
    return fits, macros


def exact(fn, y):
    """P from its Taylor series, W in closed form, in 40-digit arithmetic."""
    mpmath.mp.dps = 40
    y = mpmath.mpf(y)
    if fn == "W":
        return 1 / (1 - y) ** 2
    s, term_y, k = mpmath.mpf(0), mpmath.mpf(1), 1
    while True:
        t = k * term_y / (2 * k + 1)
        s += t
        if abs(t) < mpmath.mpf(10) ** -36:
            return s
        term_y *= y
        k += 1


FITS, MACROS = parse()


def test_header_lists_every_fit():
    assert set(FITS) == {"hct_poly", "hct_poly_d", "hct_poly64", "hct_poly_far",
                         "hct_poly64_far", "hct_w_far"}
    for name, (fn, deg, ymax, err, ctype, coef) in FITS.items():
        assert len(coef) == deg + 1, name
    assert MACROS["GBMC_HCT_YMAX"] == FITS["hct_poly"][2]
    assert MACROS["GBMC_HCT_YMAX64"] == FITS["hct_poly64"][2]
    assert MACROS["GBMC_HCT_YFAR"] == FITS["hct_poly_far"][2] == FITS["hct_w_far"][2]


def test_series_and_closed_form_agree():
    # the series against g(x) written with atanh, where it does not cancel
    mpmath.mp.dps = 40
    for y in ("0.05", "0.2", "0.4"):
        x = mpmath.sqrt(mpmath.mpf(y))
        g = (x / (1 - x * x) - mpmath.atanh(x)) / 2
        assert abs(exact("P", y) * x ** 3 / g - 1) < 1e-30
    assert exact("P", 0) == mpmath.mpf(1) / 3


@pytest.mark.parametrize("name", sorted(FITS))
def test_fit_meets_its_stated_error(name):
    fn, deg, ymax, err, ctype, coef = FITS[name]
    dt = np.float32 if ctype == "float" else np.float64
    c = [dt(v) for v in coef]
    worst = 0.0
    for y in np.linspace(0.0, ymax, 1201):
        y = dt(y)
        p = c[0]
        for v in c[1:]:
            p = dt(dt(p * y) + v)
        worst = max(worst, abs(float(p) / float(exact(fn, float(y))) - 1.0))
    # the header rounds the bound to three digits
    assert worst <= err * 1.01 + (1e-18 if ctype == "double" else 0.0), (name, worst, err)
    # and every FP32 fit is about as accurate as the precision allows
    assert err < (2e-6 if name == "hct_poly_d" else 1.5e-7 if ctype == "float" else 3e-16)
