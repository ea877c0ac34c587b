"""Pins of the oracle's salt-screened GB form (kappa > 0): the GB pair and
self terms carry the factor 1/eps_in - exp(-kappa f)/eps_out.

* two distant ions interact by the Debye-Hueckel screened Coulomb law
  k q1 q2 exp(-kappa r) / (eps_out r) (pins the sign and the argument of the
  exponential);
* kappa -> 0 gives the salt-free energy, and a huge kappa leaves the self
  energy -(k/2) q^2 / (eps_in R) (complete screening);
* forces, dE/dq and dE/drho equal central differences of the energy;
* E = q.phi / 2 still holds (E quadratic in q), and the site Delta E bilinear
  form equals the brute-force energy difference.
"""
import dataclasses
import math

import numpy as np
import pytest

import synth

K = 332.0522


def two_ions(r, q1=0.8, q2=-0.6):
    return synth.System(np.array([0.0, r]), np.zeros(2), np.zeros(2), np.array([q1, q2]),
                        np.array([1.6, 1.9]), np.array([0.8, 0.8]))


@pytest.mark.parametrize("kappa", [0.02, 0.08, 0.2])
@pytest.mark.parametrize("r", [25.0, 40.0])
def test_distant_ions_screened_coulomb(orc, kappa, r):
    p = dataclasses.replace(orc.IGB5, kappa=kappa)
    s = two_ions(r)
    R = np.array([1.6 - 0.09, 1.9 - 0.09])
    # interaction = E(q1, q2) - E(q1, 0) - E(0, q2) at fixed radii
    e = lambda q: float(orc.energy_fixedR(s, R, p, q=np.asarray(q, float)).sum())
    inter = e([0.8, -0.6]) - e([0.8, 0.0]) - e([0.0, -0.6])
    dh = K * 0.8 * -0.6 * math.exp(-kappa * r) / (78.5 * r)
    # the three energies are ~100 kcal/mol each: 1e-12 absolute for their cancellation
    assert abs(inter - dh) <= 1e-9 * abs(dh) + 1e-12, (inter, dh)
    assert abs(dh) > 1e-6


def test_kappa_limits(orc):
    s = synth.make_system(71, 40, 6.0)
    E0 = orc.energy_forces(s, orc.IGB5)
    Etiny = orc.energy_forces(s, dataclasses.replace(orc.IGB5, kappa=1e-12))
    assert abs(Etiny["E"] - E0["E"]) <= 1e-9 * abs(E0["E"])
    # complete screening: every exp(-kappa f) vanishes, the GB factor is 1/eps_in
    big = dataclasses.replace(orc.IGB5, kappa=1e4)
    one = synth.System(np.zeros(1), np.zeros(1), np.zeros(1), np.array([0.7]), np.array([1.5]),
                       np.array([0.8]))
    e = orc.energy_forces(one, big)
    a = 1.5 - 0.09
    assert math.isclose(e["Egb"], -0.5 * K * 0.7 ** 2 / a, rel_tol=1e-14)


def test_salt_gradients_match_central_differences(orc):
    p = dataclasses.replace(orc.IGB5, kappa=0.15)
    s = synth.make_system(72, 60, 6.5)
    r = orc.energy_forces(s, p)
    rng = np.random.default_rng(3)
    h = 1e-5
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


def test_salt_quadratic_form_and_bilinear_delta_E(orc):
    p = dataclasses.replace(orc.IGB5, kappa=0.1)
    s = synth.make_system(73, 120, 7.0, n_redox=1, n_prot=1, redox_atoms=8, prot_atoms=(5, 7))
    r = orc.energy_forces(s, p)
    assert abs(r["E"] - 0.5 * float(np.dot(s.q, r["phi"]))) <= 1e-10 * abs(r["E"])
    R = r["R"]
    a = orc.site_dE(s, R, p)
    b = orc.site_dE(s, R, p, brute=True)
    assert np.abs(a - b).max() <= 1e-9
    # salt changes Delta E (the test would pass vacuously otherwise)
    assert np.abs(a - orc.site_dE(s, R, orc.IGB5)).max() > 1e-3
