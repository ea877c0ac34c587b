"""Pins of the oracle's Delta E_elec, Delta G, Metropolis step and E-REMD exchange.

* Delta E: the bilinear form equals the brute-force energy difference E(q') -
  E(q); it is antisymmetric and closes around a three-state cycle.
* Delta G: reduces to the paper's two-state Eq. 8 and Eq. 9.
* MC: an uncoupled redox site follows the Nernst fraction (Eq. 3 with n = 1)
  and an uncoupled protonation site follows Henderson-Hasselbalch; a five-state
  site follows its Boltzmann distribution; the redox attempt sees the charges
  left by an accepted protonation attempt (section II.B and Fig. 1).
* Sweep (section III.A.2): every visit's Delta G is the brute-force energy
  difference at the charges left by the earlier visits, in the visit order;
  a one-site sweep is the single attempt.
* Exchange: the paper's worked numbers (31 % at 30 mV, 59.5 mV per pH unit),
  the pairing pattern of section III.B, and the Eq. 15 rate.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_worked_examples.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def c1():
    return synth.globule_2500()[0]


def small_system(n=60, seed=21, n_redox=1, n_prot=1, prot_states=5, redox_atoms=6,
                 prot_atoms=(4, 6)):
    return synth.make_system(seed, n, 9.0, n_redox=n_redox, n_prot=n_prot,
                             redox_atoms=redox_atoms, prot_atoms=prot_atoms,
                             prot_states=prot_states, random_states=True)


def test_bilinear_equals_brute_globule_256(orc):
    s = synth.globule_256()[0]
    R = orc.radii(s)["R"]
    a = orc.site_dE(s, R)
    b = orc.site_dE(s, R, brute=True)
    assert a.shape == (1,)
    assert np.abs(a - b).max() <= 1e-9


def test_bilinear_equals_brute_globule_2500(orc, c1):
    R = orc.radii(c1)["R"]
    a = orc.site_dE(c1, R)
    b = orc.site_dE(c1, R, brute=True)
    assert a.shape == (4 * 1 + 4 * 4,)
    assert np.abs(a - b).max() <= 1e-9


def _set_state(s, m, t):
    site = s.sites[m]
    site.state = t
    s.q[site.atoms] = site.charges[t]


def test_delta_E_antisymmetric_and_cycle(orc):
    s = small_system(prot_states=3)
    R = orc.radii(s)["R"]
    prot = [m for m, site in enumerate(s.sites) if site.kind == synth.KIND_PROT][0]
    # candidates of a site are its other states in ascending order
    def dE_to(sys_, m, t):
        d = orc.site_dE(sys_, R)
        c0 = sum(x.n_states - 1 for x in sys_.sites[:m])
        cur = sys_.sites[m].state
        return d[c0 + (t if t < cur else t - 1)]
    w = s.copy()
    _set_state(w, prot, 0)
    d01 = dE_to(w, prot, 1)
    _set_state(w, prot, 1)
    d10 = dE_to(w, prot, 0)
    d12 = dE_to(w, prot, 2)
    _set_state(w, prot, 2)
    d20 = dE_to(w, prot, 0)
    assert abs(d01 + d10) <= 1e-10 * max(1, abs(d01))
    assert abs(d01 + d12 + d20) <= 1e-10 * max(1, abs(d01))


def test_delta_G_reduces_to_eq8_and_eq9(orc):
    kB, F = 1.98720426e-3, 23.0605478
    T = 300.0
    dE, dGref_elec = -12.34, -11.5
    # Eq. 8: dG_red = v F (E - E0_ref) + dG_elec - dG_elec,ref  (v = 1)
    E0, E = -0.203, -0.15
    eq8 = F * (E - E0) + dE - dGref_elec
    gref_red_minus_ox = dGref_elec + F * E0
    got = orc.delta_G(1, dE, 1, 0, gref_red_minus_ox, 0.0, 7.0, E, T)
    assert abs(got - eq8) <= 1e-12 * abs(eq8)
    # reverse move has the opposite sign
    back = orc.delta_G(1, -dE, 0, 1, 0.0, gref_red_minus_ox, 7.0, E, T)
    assert abs(back + got) <= 1e-12 * abs(got)
    # Eq. 9: dG_prot = kB T ln10 (pH - pKa_ref) + dG_elec - dG_elec,ref
    pKa, pH = 4.4, 5.2
    eq9 = kB * T * math.log(10) * (pH - pKa) + dE - dGref_elec
    gref_prot_minus_deprot = dGref_elec + kB * T * math.log(10) * pKa
    got = orc.delta_G(0, dE, 1, 0, gref_prot_minus_deprot, 0.0, pH, -0.2, T)
    assert abs(got - eq9) <= 1e-12 * abs(eq9)


def _two_state_chain_sigma(f, a, b, n):
    # asymptotic std of the time average of a 2-state Markov chain
    lam = 1.0 - a - b
    return math.sqrt(f * (1 - f) * (1 + lam) / max(1e-12, 1 - lam) / n)


def _isolated_site_system(kind, seed=31):
    # a small globule with one 2-state site of the given kind and nothing else
    s = synth.make_system(seed, 40, 8.0, n_redox=int(kind == 1), n_prot=int(kind == 0),
                          redox_atoms=5, prot_atoms=(5, 5), prot_states=2)
    return s


@pytest.mark.parametrize("dEv", [-0.06, -0.02, 0.0, 0.03])
def test_mc_nernst_fraction(orc, dEv):
    T, kB, F = 300.0, 1.98720426e-3, 23.0605478
    s = _isolated_site_system(1)
    R = orc.radii(s)["R"]
    E0 = -0.203
    dE_ox_red = orc.site_dE(s, R)[0]         # site starts oxidised (state 0)
    gref = np.array([0.0, dE_ox_red + F * E0])   # dG_elec,ref = dG_elec: Eq. 8 -> F(E - E0)
    tab = orc.SiteTables(s, gref)
    E = E0 + dEv
    n = 200000
    u = synth.uniforms(77, (n, 6))
    occ, acc = orc.mc_run(s, R, tab, 7.0, E, T, u)
    f_red = occ[1] / n
    ref = 1.0 / (1.0 + math.exp(F * (E - E0) / (kB * T)))
    g = F * (E - E0)
    a = min(1.0, math.exp(-g / (kB * T)))      # ox -> red acceptance
    b = min(1.0, math.exp(g / (kB * T)))       # red -> ox
    # exact detailed balance of the 2-state chain gives the Nernst fraction
    assert abs(a / (a + b) - ref) <= 1e-12
    assert abs(f_red - ref) <= 5 * _two_state_chain_sigma(ref, a, b, n)


@pytest.mark.parametrize("pH", [3.4, 4.4, 5.9])
def test_mc_henderson_hasselbalch(orc, pH):
    T, kB = 300.0, 1.98720426e-3
    s = _isolated_site_system(0)
    R = orc.radii(s)["R"]
    pKa = 4.4
    dE = orc.site_dE(s, R)[0]                # deprotonated -> protonated
    gref = np.array([0.0, dE + kB * T * math.log(10) * pKa])
    tab = orc.SiteTables(s, gref)
    n = 200000
    u = synth.uniforms(78, (n, 6))
    occ, _ = orc.mc_run(s, R, tab, pH, -0.2, T, u)
    f_prot = occ[1] / n
    ref = 1.0 / (1.0 + 10 ** (pH - pKa))
    g = kB * T * math.log(10) * (pH - pKa)
    a = min(1.0, math.exp(-g / (kB * T)))
    b = min(1.0, math.exp(g / (kB * T)))
    assert abs(f_prot - ref) <= 5 * _two_state_chain_sigma(ref, a, b, n)


def test_mc_five_state_boltzmann(orc):
    T, kB = 300.0, 1.98720426e-3
    s = synth.make_system(33, 40, 8.0, n_prot=1, prot_atoms=(5, 5), prot_states=5)
    R = orc.radii(s)["R"]
    site = s.sites[0]
    pH = 6.0
    # Uniform proposals among the other states are symmetric, so Metropolis
    # samples p_s ~ exp(-A_s / kB T) with
    # A_s = E_elec(s) + kB T ln10 pH n_H(s) - Gref(s).
    # Gref is chosen so that the A_s are spread over about one kcal/mol.
    drive = np.array([orc.energy_fixedR(_with(s, t), R).sum()
                      + kB * T * math.log(10) * pH * site.counts[t] for t in range(5)])
    target = np.random.default_rng(3).uniform(0.0, 1.0, 5)
    gref = drive - target
    A = np.array([orc.energy_fixedR(_with(s, t), R).sum()
                  + kB * T * math.log(10) * pH * site.counts[t] - gref[t] for t in range(5)])
    p = np.exp(-(A - A.min()) / (kB * T))
    p /= p.sum()
    tab = orc.SiteTables(s, gref)
    n = 200000
    occ, _ = orc.mc_run(s, R, tab, pH, -0.2, T, synth.uniforms(79, (n, 6)))
    emp = occ / n
    assert np.all(p > 0.05)
    # generous bound: 5 sigma with a correlation factor of 10
    sig = np.sqrt(p * (1 - p) * 10 / n)
    assert np.all(np.abs(emp - p) <= 5 * sig), (emp, p)


def _with(s, t):
    w = s.copy()
    _set_state(w, 0, t)
    return w


def test_redox_attempt_sees_accepted_protonation(orc):
    # coupled sites close together: protonation first, then redox on the
    # updated charges (section II.B; Fig. 1 ordering)
    s = small_system(n=60, seed=41, prot_states=2)
    R = orc.radii(s)["R"]
    tab = orc.SiteTables(s)
    prot = [m for m, x in enumerate(s.sites) if x.kind == 0][0]
    redox = [m for m, x in enumerate(s.sites) if x.kind == 1][0]
    u = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.99999])   # protonation accepted (u = 0)
    q_new, out, dG = orc.mc_step(s, R, tab, 7.0, -0.2, 300.0, u)
    assert out[0] == 1
    # redox dG must equal the dG computed on the charges left by the
    # protonation move alone
    w = s.copy()
    _set_state(w, prot, int(tab.current_state[prot]))
    dE = orc.site_dE(w, R)
    c_red = sum(x.n_states - 1 for x in w.sites[:redox])
    site = w.sites[redox]
    t_new = 0 if site.state != 0 else 1
    ref = orc.delta_G(1, dE[c_red], int(site.counts[t_new]), int(site.counts[site.state]),
                      0.0, 0.0, 7.0, -0.2, 300.0)
    assert abs(dG[1] - ref) <= 1e-9
    # and differs from the value on the old charges when the sites interact
    dE_old = orc.site_dE(s, R)
    assert abs(dE_old[c_red] - dE[c_red]) > 1e-6


# ------------------------------------------------------------------ sweep

def _replay_sweep(orc, s, R, u, kinds, acc, pH, E, T):
    """Replays a sweep from its reported decisions with brute-force energies:
    the visit order (protonation first, each kind by ascending u[:, 0]), the
    proposed state of each visit, and dG = E(q') - E(q) + drive - dGref at the
    charges left by the earlier visits."""
    w = s.copy()
    out = {}
    for kind in (0, 1):
        if not kinds & (1 << kind):
            continue
        ms = sorted((m for m, x in enumerate(w.sites) if x.kind == kind), key=lambda m: (u[m, 0], m))
        for m in ms:
            site = w.sites[m]
            cur = site.state
            tp = min(int(math.floor(u[m, 1] * (site.n_states - 1))), site.n_states - 2)
            new = tp if tp < cur else tp + 1
            e0 = orc.energy_fixedR(w, R).sum()
            q_try = w.q.copy()
            q_try[site.atoms] = site.charges[new]
            e1 = orc.energy_fixedR(w, R, q=q_try).sum()
            drive = (orc.KB * T * math.log(10) * pH) if kind == 0 else (orc.FARADAY * E)
            out[m] = (e1 - e0) + drive * (int(site.counts[new]) - int(site.counts[cur]))
            if acc[m] == 1:
                _set_state(w, m, new)
    return out, w


@pytest.mark.parametrize("kinds", [1, 2, 3])
def test_sweep_matches_brute_force_replay(orc, kinds):
    # several interacting sites: every attempt's dG is the brute-force energy
    # difference at the charges left by the earlier attempts of the sweep, in
    # the order the paper's explicit-solvent loop visits them
    s = synth.make_system(51, 80, 7.0, n_redox=2, n_prot=3, redox_atoms=8, prot_atoms=(4, 6),
                          prot_states=3, random_states=True)
    R = orc.radii(s)["R"]
    rng = np.random.default_rng(7)
    u = rng.uniform(size=(len(s.sites), 3))
    u[:, 2] = rng.choice([0.0, 0.999999], size=len(s.sites))   # force a mix of decisions
    tab = orc.SiteTables(s)
    q, acc, dG = orc.mc_sweep(s, R, tab, 7.0, -0.2, 300.0, u, kinds)
    ref, w = _replay_sweep(orc, s, R, u, kinds, acc, 7.0, -0.2, 300.0)
    for m, x in enumerate(s.sites):
        if kinds & (1 << x.kind):
            assert acc[m] in (0, 1)
            assert abs(dG[m] - ref[m]) <= 1e-9, (m, dG[m], ref[m])
            assert acc[m] == int(u[m, 2] < math.exp(-dG[m] / (orc.KB * 300.0)))
        else:
            assert acc[m] == -1
    assert np.array_equal(q, w.q)
    assert [int(v) for v in tab.current_state] == [x.state for x in w.sites]
    # the sites interact: some later attempt saw an accepted earlier one
    assert (acc == 1).any()


def test_sweep_one_redox_site_equals_single_attempt(orc):
    # with one redox site and no protonation site, a redox sweep is the
    # implicit-solvent attempt of that site (same state pick and acceptance)
    s = synth.make_system(52, 50, 6.0, n_redox=1, n_prot=0, redox_atoms=6, random_states=True)
    R = orc.radii(s)["R"]
    for ua in (0.0, 0.3, 0.999999):
        t1, t2 = orc.SiteTables(s), orc.SiteTables(s)
        q1, acc, dG = orc.mc_sweep(s, R, t1, 7.0, -0.25, 300.0, np.array([[0.5, 0.7, ua]]), 2)
        q2, out, dG2 = orc.mc_step(s, R, t2, 7.0, -0.25, 300.0, [0.0, 0.0, 0.0, 0.1, 0.7, ua])
        assert acc[0] == out[1] and abs(dG[0] - dG2[1]) <= 1e-12
        assert np.array_equal(q1, q2)
        assert list(t1.current_state) == list(t2.current_state)


# ------------------------------------------------------------------ exchange

def test_exchange_30mV_worked_example(orc, golden):
    g = golden["exchange_30mV"]
    T, dE, dN = g["T_K"], g["dE_volt"], g["dN_electrons"]
    p_paper = g["acceptance_percent"] / 100.0
    tol = g["printed_precision_percent"] / 100.0
    # replica 0 (rung 0, lower E) has dN more electrons than replica 1?  Use
    # N_i - N_j = dN with i on the lower rung so that Delta > 0.
    E_rung = [-0.2, -0.2 + dE]
    Ne = [dN, 0]
    for u, expect in ((p_paper - tol - 1e-4, 1), (p_paper + tol + 1e-4, 0)):
        rep, acc, _ = orc.remd_exchange(E_rung, Ne, [0, 1], T, 0, False, [u])
        assert acc[0] == expect, (u, acc)


def test_pH_unit_in_mV(orc, golden):
    g = golden["pH_unit_in_mV"]
    T = g["T_K"]
    drive_pH = orc.delta_G(0, 0.0, 1, 0, 0.0, 0.0, 1.0, 0.0, T)
    drive_E = orc.delta_G(1, 0.0, 1, 0, 0.0, 0.0, 0.0, g["mV_per_pH_unit"] / 1000.0, T)
    assert abs(drive_E / drive_pH - 1.0) <= g["printed_precision_mV"] / g["mV_per_pH_unit"]


def test_exchange_pairing_pattern(orc, golden):
    g = golden["exchange_pairing_4_replicas"]
    E_rung = [-0.3, -0.27, -0.24, -0.21]
    Ne = [1, 1, 1, 1]                 # equal electron counts: Delta = 0, always accepted
    rep, acc, Eo = orc.remd_exchange(E_rung, Ne, [0, 1, 2, 3], 300.0, 0, True, [0.5] * 4)
    # (1,2),(3,4) in the paper's 1-based numbering
    assert acc.tolist() == [1, 1] and rep.tolist() == [1, 0, 3, 2]
    assert [[a + 1, b + 1] for a, b in ((0, 1), (2, 3))] == g["first"]
    rep2, acc2, Eo2 = orc.remd_exchange(E_rung, Ne, [0, 1, 2, 3], 300.0, 1, True, [0.5] * 4)
    # (2,3),(1,4): rungs 1<->2 and the wrap pair 3<->0
    assert acc2.tolist() == [1, 1] and rep2.tolist() == [3, 2, 1, 0]
    assert [[1 + 1, 2 + 1], [0 + 1, 3 + 1]] == g["second"]
    assert np.allclose(Eo2[[3, 2, 1, 0]], E_rung)
    # without wrap only the inner pair is attempted
    rep3, acc3, _ = orc.remd_exchange(E_rung, Ne, [0, 1, 2, 3], 300.0, 1, False, [0.5] * 4)
    assert acc3.tolist() == [1] and rep3.tolist() == [0, 2, 1, 3]


def test_exchange_rate_matches_eq15(orc):
    kB, F, T = 1.98720426e-3, 23.0605478, 300.0
    E_rung = [-0.30, -0.28]
    for Ne, expect in (([2, 1], math.exp(-F * 0.02 / (kB * T))), ([1, 2], 1.0), ([1, 1], 1.0)):
        u = synth.uniforms(5, 20000)
        hits = sum(orc.remd_exchange(E_rung, Ne, [0, 1], T, 0, False, [x])[1][0] for x in u)
        rate = hits / u.size
        sig = math.sqrt(max(expect * (1 - expect), 1e-12) / u.size)
        assert abs(rate - expect) <= 5 * sig + 1e-12
