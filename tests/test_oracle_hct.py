"""Pins of the oracle's HCT pair integral H(r; rt, S) and its partials.

H is defined geometrically: the integral of |x|^-4 / (4 pi) over the part of a
ball of radius S centred at distance r that lies outside radius rt around the
origin.  Integrating over spherical shells of radius t, the shell fraction
inside the ball is 1 for t < S - r, (1 - cos theta0)/2 for |r - S| < t < r + S
with cos theta0 = (t^2 + r^2 - S^2)/(2 t r), else 0; so
    H = integral_{rt}^{inf} t^-2 * fraction(t) dt.
These tests integrate that numerically (scipy in FP64, mpmath at 50 digits),
independently of the oracle's closed form.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.integrate import quad


def shell_fraction(t, r, S):
    if t < S - r:
        return 1.0
    if t <= abs(r - S) or t >= r + S:
        return 0.0
    c = (t * t + r * r - S * S) / (2.0 * t * r)
    return 0.5 * (1.0 - c)


def H_quad(r, rt, S):
    lo = rt
    hi = r + S
    if lo >= hi:
        return 0.0
    pts = [p for p in (abs(r - S), S - r) if lo < p < hi]
    val, err = quad(lambda t: shell_fraction(t, r, S) / (t * t), lo, hi, points=pts or None,
                    epsabs=0.0, epsrel=1e-13, limit=400)
    return val


def H_mp(r, rt, S):
    r, rt, S = mpmath.mpf(r), mpmath.mpf(rt), mpmath.mpf(S)
    hi = r + S
    if rt >= hi:
        return mpmath.mpf(0)

    def frac(t):
        if t < S - r:
            return mpmath.mpf(1)
        if t <= abs(r - S) or t >= r + S:
            return mpmath.mpf(0)
        c = (t * t + r * r - S * S) / (2 * t * r)
        return (1 - c) / 2

    pts = sorted({rt, hi} | {p for p in (abs(r - S), S - r) if rt < p < hi})
    return mpmath.quad(lambda t: frac(t) / (t * t), pts)


# geometries covering every branch: (r, rt, S, label)
BRANCH_CASES = [
    (5.0, 1.3, 1.2, "far"),
    (50.0, 1.5, 1.6, "very far"),
    (2.2, 1.4, 1.3, "partial overlap, L = rt"),
    (1.0, 1.1, 1.6, "centre inside ball j, L = rt"),
    (0.3, 0.5, 1.6, "engulfed: rt < S - r"),
    (0.05, 0.2, 1.0, "deep engulfed"),
    (1.0, 3.0, 1.5, "zero: rt >= r + S"),
    (2.5, 1.2, 1.3, "just non-overlapping r - S = rt"),
]


@pytest.mark.parametrize("r,rt,S,label", BRANCH_CASES)
def test_hct_matches_shell_quadrature(orc, r, rt, S, label):
    ref = H_quad(r, rt, S)
    got = orc.hct(r, rt, S)
    if ref == 0.0:
        assert got == 0.0
    else:
        assert abs(got - ref) <= 1e-11 * abs(ref) + 1e-15, label


@pytest.mark.parametrize("r,rt,S,label", BRANCH_CASES[:6])
def test_hct_matches_50_digit_quadrature(orc, r, rt, S, label):
    mpmath.mp.dps = 50
    ref = float(H_mp(r, rt, S))
    assert abs(orc.hct(r, rt, S) - ref) <= 3e-12 * abs(ref), label


def test_hct_random_geometries(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        S = rng.uniform(0.3, 2.0)
        rt = rng.uniform(0.3, 2.0)
        r = rng.uniform(0.02, 12.0)
        ref = H_quad(r, rt, S)
        got = orc.hct(r, rt, S)
        assert abs(got - ref) <= 1e-10 * abs(ref) + 1e-14, (r, rt, S)


def test_hct_far_field_series(orc):
    # Non-overlapping H has the expansion (1/r) sum_k k x^(2k+1)/(2k+1), x = S/r,
    # whose first term is the point-volume value S^3/(3 r^4).
    for r, S in [(20.0, 1.5), (60.0, 1.2), (8.0, 1.0)]:
        x = S / r
        series = sum(k * x ** (2 * k + 1) / (2 * k + 1) for k in range(1, 40)) / r
        assert abs(orc.hct(r, 1.0, S) - series) <= 1e-9 * series
        assert abs(orc.hct(r, 1.0, S) / (S ** 3 / (3 * r ** 4)) - 1.0) < 1.3 * x * x


def test_hct_monotone_and_continuous(orc):
    # continuity across the branch boundaries rt = |r - S| and rt = S - r
    S, rt = 1.5, 1.0
    for r_b in (S - rt, S + rt):
        lo, hi = orc.hct(r_b - 1e-9, rt, S), orc.hct(r_b + 1e-9, rt, S)
        assert abs(lo - hi) < 1e-7
    # H decreases with distance beyond contact
    rs = np.linspace(2.6, 30, 50)
    vals = [orc.hct(r, rt, S) for r in rs]
    assert all(a > b for a, b in zip(vals, vals[1:]))


GRAD_CASES = [c for c in BRANCH_CASES if c[3] != "just non-overlapping r - S = rt"]


@pytest.mark.parametrize("r,rt,S,label", GRAD_CASES)
def test_hct_grad_matches_central_differences(orc, r, rt, S, label):
    g = orc.hct_grad(r, rt, S)
    h = 1e-6
    fd = [
        (orc.hct(r + h, rt, S) - orc.hct(r - h, rt, S)) / (2 * h),
        (orc.hct(r, rt + h, S) - orc.hct(r, rt - h, S)) / (2 * h),
        (orc.hct(r, rt, S + h) - orc.hct(r, rt, S - h)) / (2 * h),
    ]
    scale = max(1e-12, max(abs(v) for v in fd))
    for k in range(3):
        assert abs(g[k] - fd[k]) <= 2e-7 * scale + 1e-10, (label, k, g, fd)


def test_hct_grad_random(orc):
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(300):
        S = rng.uniform(0.3, 2.0)
        rt = rng.uniform(0.3, 2.0)
        r = rng.uniform(0.05, 10.0)
        # stay away from the kinks where a one-sided limit changes
        if min(abs(rt - abs(r - S)), abs(rt - (r + S)), abs(rt - (S - r))) < 1e-3:
            continue
        g = orc.hct_grad(r, rt, S)
        fd = np.array([
            (orc.hct(r + h, rt, S) - orc.hct(r - h, rt, S)),
            (orc.hct(r, rt + h, S) - orc.hct(r, rt - h, S)),
            (orc.hct(r, rt, S + h) - orc.hct(r, rt, S - h)),
        ]) / (2 * h)
        scale = max(1e-12, np.abs(fd).max())
        assert np.all(np.abs(g - fd) <= 3e-7 * scale + 1e-10), (r, rt, S, g, fd)
