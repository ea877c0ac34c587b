"""Pins of the oracle's optional cutoffs (the paper's runs have none):

* the descreening cutoff restricts H to the sphere of radius c around atom i:
  checked against shell quadrature of the truncated integral (the shell
  fraction integrated from rt to min(c, r + S)), including spheres that
  straddle c, lie beyond it, or hold c inside them; its partials against
  central differences;
* a very large cutoff gives the uncut result; a pair beyond the energy cutoff
  contributes nothing; with both cutoffs, forces, dE/dq and dE/drho are the
  derivatives of the cut energy (central differences at a geometry with no
  pair near the energy cutoff); the site Delta E bilinear form still equals
  the brute-force energy difference.
"""
import dataclasses

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from test_oracle_hct import shell_fraction


def H_cut_quad(r, rt, S, c):
    lo, hi = rt, min(c, r + S)
    if lo >= hi:
        return 0.0
    pts = [p for p in (abs(r - S), S - r) if lo < p < hi]
    val, _ = quad(lambda t: shell_fraction(t, r, S) / (t * t), lo, hi, points=pts or None,
                  epsabs=0.0, epsrel=1e-13, limit=400)
    return val


CASES = [
    (10.0, 1.4, 1.5, 12.0, "inside: r + S < c"),
    (10.0, 1.4, 1.5, 10.8, "straddles c"),
    (10.0, 1.4, 1.5, 9.0, "straddles c, centre beyond c"),
    (10.0, 1.4, 1.5, 8.4, "beyond: r - S > c"),
    (2.0, 1.3, 1.6, 2.5, "overlapping pair straddling c"),
    (0.3, 0.5, 1.6, 1.0, "engulfed, c inside ball j"),
    (5.0, 1.5, 1.2, 1.2, "c below rt"),
]


@pytest.mark.parametrize("r,rt,S,c,label", CASES)
def test_hct_cut_matches_truncated_quadrature(orc, r, rt, S, c, label):
    ref = H_cut_quad(r, rt, S, c)
    got = orc.hct_cut(r, rt, S, c)
    assert abs(got - ref) <= 1e-11 * abs(orc.hct(r, rt, S)) + 1e-15, (label, got, ref)


@pytest.mark.parametrize("r,rt,S,c,label", CASES[:6])
def test_hct_cut_partials(orc, r, rt, S, c, label):
    g = orc.hct_cut_grad(r, rt, S, c)
    h = 1e-6
    for k, args in enumerate(((r + h, rt, S), (r, rt + h, S), (r, rt, S + h))):
        am = [r, rt, S]
        am[k] -= h
        fd = (orc.hct_cut(*args, c) - orc.hct_cut(*am, c)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (label, k, fd, g[k])


def test_large_cutoffs_equal_no_cutoff(orc):
    s = synth.make_system(91, 80, 7.0)
    a = orc.energy_forces(s, orc.IGB5)
    b = orc.energy_forces(s, dataclasses.replace(orc.IGB5, rgbmax=1e4, cutoff=1e4))
    for k in ("R", "F", "phi", "dEdrho"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-12), k
    assert abs(a["E"] - b["E"]) <= 1e-10 * abs(a["E"])


def test_pair_beyond_energy_cutoff_contributes_nothing(orc):
    s = synth.System(np.array([0.0, 9.0]), np.zeros(2), np.zeros(2), np.array([0.8, -0.6]),
                     np.array([1.6, 1.9]), np.array([0.8, 0.8]))
    p = dataclasses.replace(orc.IGB5, cutoff=8.0, rgbmax=7.0)
    R = orc.radii(s, p)["R"]
    # nor does it descreen: each radius is the isolated atom's, rho - offset
    assert np.allclose(R, s.rho - 0.09, rtol=1e-15, atol=0)
    e = lambda q: float(orc.energy_fixedR(s, R, p, q=np.asarray(q, float)).sum())
    assert e([0.8, -0.6]) - e([0.8, 0.0]) - e([0.0, -0.6]) == pytest.approx(0.0, abs=1e-13)
    # no force either (beyond both cutoffs the atoms do not interact)
    r = orc.energy_forces(s, p)
    assert np.abs(r["F"]).max() == 0.0


def test_cut_gradients_match_central_differences(orc):
    s = synth.make_system(92, 150, 9.0)
    xyz = s.coords()
    d = np.sqrt(((xyz[:, None] - xyz[None]) ** 2).sum(-1))
    cut = 8.0
    # move the cutoff to the widest gap in the pair distances around 8 A, so
    # that no pair crosses it in the differences
    ds = np.sort(d[np.triu_indices(s.n, 1)])
    near = ds[(ds > 7.0) & (ds < 9.0)]
    k = int(np.argmax(np.diff(near)))
    cut = 0.5 * (near[k] + near[k + 1])
    p = dataclasses.replace(orc.IGB5, rgbmax=6.0, cutoff=cut)
    r = orc.energy_forces(s, p)
    rng = np.random.default_rng(4)
    h = 1e-5
    assert np.diff(near)[k] > 4 * h
    for i in rng.choice(s.n, 8, replace=False):
        for ax, name in enumerate("xyz"):
            sp, sm = s.copy(), s.copy()
            getattr(sp, name)[i] += h
            getattr(sm, name)[i] -= h
            fd = -(orc.energy(sp, p) - orc.energy(sm, p)) / (2 * h)
            assert abs(fd - r["F"][i, ax]) <= 1e-6 * max(1.0, abs(fd)), (i, name)
        for key, attr in (("phi", "q"), ("dEdrho", "rho")):
            sp, sm = s.copy(), s.copy()
            getattr(sp, attr)[i] += h
            getattr(sm, attr)[i] -= h
            fd = (orc.energy(sp, p) - orc.energy(sm, p)) / (2 * h)
            assert abs(fd - r[key][i]) <= 1e-6 * max(1.0, abs(fd)), (i, key)
    # the cutoffs change the result (the test would pass vacuously otherwise)
    assert abs(r["E"] - orc.energy_forces(s, orc.IGB5)["E"]) > 1e-3


def test_cut_bilinear_delta_E(orc):
    p = dataclasses.replace(orc.IGB5, rgbmax=7.0, cutoff=6.0)
    s = synth.make_system(93, 200, 9.0, n_redox=1, n_prot=1, redox_atoms=10, prot_atoms=(6, 8))
    R = orc.radii(s, p)["R"]
    a = orc.site_dE(s, R, p)
    b = orc.site_dE(s, R, p, brute=True)
    assert np.abs(a - b).max() <= 1e-9
