"""Pins of the analysis module (CPU): the Hill-form Nernst fit (Eq. 3) and the
standard-potential / pKa relations of section II.D (Eqs. 16-18), checked
against brute-force partition functions of one redox group coupled to
independent pH-active groups, the fits of Eqs. 17 and 18 against exact
curves, and the per-rung reduced fraction against a plain loop over the
records."""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from paper_1803_09652_amd import analysis as an

KB, F, T = 1.98720426e-3, 23.0605478, 300.0


def _weights(E, pH, E0_deprot, pka_red, pka_oxi, v=1):
    """Boltzmann weights of every microstate (redox r in {0 ox, 1 red}, each
    pH group protonated or not): reduction with every group deprotonated costs
    vF(E - E0_deprot); protonating group i costs kT ln10 (pH - pKa_i(r))."""
    out = []
    for r in (0, 1):
        for prot in itertools.product((0, 1), repeat=len(pka_red)):
            G = v * F * (E - E0_deprot) if r else 0.0
            for i, p in enumerate(prot):
                if p:
                    pka = pka_red[i] if r else pka_oxi[i]
                    G += KB * T * math.log(10) * (pH - pka)
            out.append((r, prot, math.exp(-G / (KB * T))))
    return out


def _fred(E, pH, *a):
    w = _weights(E, pH, *a)
    return sum(x for r, _, x in w if r) / sum(x for _, _, x in w)


def test_hill_fit_recovers_parameters():
    E = np.linspace(-0.35, -0.05, 16)
    for E0, n in ((-0.2, 1.0), (-0.17, 0.62), (-0.25, 1.4)):
        f = an.f_red(E, E0, n, T)
        e0, nn, de0, dn = an.fit_hill(E, f, T)
        assert abs(e0 - E0) < 1e-7 and abs(nn - n) < 1e-6
    # noisy fractions: the fit stays within a few standard errors
    rng = np.random.default_rng(4)
    f = np.clip(an.f_red(E, -0.2, 0.8, T) + rng.normal(0, 0.01, E.size), 0, 1)
    e0, nn, de0, dn = an.fit_hill(E, f, T, sigma=np.full(E.size, 0.01))
    assert abs(e0 + 0.2) < 4 * de0 + 1e-4 and abs(nn - 0.8) < 4 * dn + 1e-3


def test_eq3_is_the_nernst_equation_for_n1():
    # Eq. 2: E = E0 + (kT/vF) ln([ox]/[red]) with f_red = [red]/([red]+[ox])
    for E in (-0.3, -0.2, -0.11):
        f = float(an.f_red(E, -0.2, 1.0, T))
        assert math.isclose(E, -0.2 + KB * T / F * math.log((1 - f) / f), rel_tol=0, abs_tol=1e-12)


@pytest.mark.parametrize("pka", [((7.5,), (6.0,)), ((4.2, 9.1), (3.8, 7.7)), ((5.0, 5.0, 6.5), (5.0, 4.1, 6.0))])
def test_eq16_eq17_against_partition_function(pka):
    pka_red, pka_oxi = pka
    E0_deprot = -0.21
    E0_prot = E0_deprot + KB * T * math.log(10) * sum(r - o for r, o in zip(pka_red, pka_oxi)) / F
    assert math.isclose(an.e0_deprot(E0_prot, pka_red, pka_oxi, T), E0_deprot, abs_tol=1e-14)
    for pH in (1.0, 4.0, 6.3, 7.0, 9.5, 13.0):
        brute = brentq(lambda e: _fred(e, pH, E0_deprot, pka_red, pka_oxi) - 0.5, -1.5, 1.0,
                       xtol=1e-14)
        assert abs(float(an.e0_of_ph(pH, E0_prot, pka_red, pka_oxi, T)) - brute) < 1e-10, pH
    # the limits stated with Eq. 17: low pH -> E0_prot, high pH -> E0_deprot
    assert abs(float(an.e0_of_ph(-10.0, E0_prot, pka_red, pka_oxi, T)) - E0_prot) < 1e-9
    assert abs(float(an.e0_of_ph(30.0, E0_prot, pka_red, pka_oxi, T)) - E0_deprot) < 1e-9


def test_eq18_against_partition_function():
    pka_red, pka_oxi = (8.0,), (5.5,)
    E0_deprot = -0.15
    E0_prot = an.e0_deprot(0.0, pka_oxi, pka_red, T) + E0_deprot     # Eq. 16 both ways
    assert E0_prot > E0_deprot
    for E in (-0.5, -0.25, -0.1, 0.0, 0.3):
        def half(pH):
            w = _weights(E, pH, E0_deprot, pka_red, pka_oxi)
            return sum(x for _, p, x in w if p[0]) / sum(x for _, _, x in w) - 0.5
        brute = brentq(half, -5, 20, xtol=1e-13)
        got = float(an.sum_pka_of_e(E, pka_red[0], E0_prot, E0_deprot, T))
        assert abs(got - brute) < 1e-9, (E, got, brute)
    # high E -> pKa_oxi (Eq. 16), low E -> pKa_red
    assert abs(float(an.sum_pka_of_e(3.0, 8.0, E0_prot, E0_deprot, T)) - 5.5) < 1e-9
    assert abs(float(an.sum_pka_of_e(-3.0, 8.0, E0_prot, E0_deprot, T)) - 8.0) < 1e-9


def test_fraction_by_rung_matches_plain_loop():
    rng = np.random.default_rng(9)
    B, K, a = 4, 2, 50
    # per replica: one protonation site (3 states) then K two-state redox sites
    site_system, site_kind, sso, cnt = [], [], [0], []
    for b in range(B):
        site_system.append(b); site_kind.append(0); cnt += [0, 1, 1]; sso.append(sso[-1] + 3)
        for _ in range(K):
            site_system.append(b); site_kind.append(1); cnt += [0, 1]; sso.append(sso[-1] + 2)
    S = len(site_system)
    nst = np.diff(sso)
    state = np.stack([rng.integers(0, nst) for _ in range(a)])
    rep = np.stack([rng.permutation(B) for _ in range(a)])
    f = an.fraction_by_rung(state, rep, site_system, site_kind, sso[:-1] + [sso[-1]], cnt)
    ref = np.zeros((B, K))
    for t in range(a):
        for l in range(B):
            b = rep[t, l]
            redox = [m for m in range(S) if site_system[m] == b and site_kind[m] == 1]
            for k, m in enumerate(redox):
                ref[l, k] += cnt[sso[m] + state[t, m]]
    assert np.allclose(f, ref / a, rtol=0, atol=1e-15)


def test_eq17_fit_recovers_one_group():
    pH = np.linspace(2.0, 10.5, 18)                        # the pH grid of section IV.B
    E0_prot, pr, po = -0.17, 6.1, 4.3
    E0 = an.e0_of_ph(pH, E0_prot, [pr], [po], T)
    e0p, fr, fo, rms = an.fit_e0_of_ph(pH, E0, 1, T)
    assert rms < 1e-10
    assert abs(e0p - E0_prot) < 1e-7 and abs(fr[0] - pr) < 1e-5 and abs(fo[0] - po) < 1e-5


def test_eq17_fit_three_groups_reproduces_the_curve():
    # three pH-active groups (two propionates and a glutamate in the paper's
    # molecule): the parameters need not be unique, the fitted curve must be
    pH = np.linspace(2.0, 10.5, 18)
    E0 = an.e0_of_ph(pH, -0.15, [5.2, 6.0, 4.9], [4.1, 4.8, 4.6], T)
    e0p, fr, fo, rms = an.fit_e0_of_ph(pH, E0, 3, T, guess=(-0.16, [5.0, 5.8, 5.0], [4.3, 4.5, 4.4]))
    # nine parameters, weakly determined: the curve to 0.1 mV (the paper's fits
    # carry errors of mV)
    assert rms < 1e-4
    # Eq. 16: the high-pH limit of the fitted curve is the fitted E0_deprot
    assert abs(float(an.e0_of_ph(40.0, e0p, fr, fo, T)) - an.e0_deprot(e0p, fr, fo, T)) < 1e-9


def test_eq18_fit_recovers_parameters():
    E = np.linspace(-0.353, -0.023, 12)                    # the E grid of section IV.B
    y = an.sum_pka_of_e(E, 13.5, -0.12, -0.21, T)
    s, e0p, e0d, rms = an.fit_pka_of_e(E, y, T)
    assert rms < 1e-10
    assert abs(s - 13.5) < 1e-6 and abs(e0p + 0.12) < 1e-7 and abs(e0d + 0.21) < 1e-7
