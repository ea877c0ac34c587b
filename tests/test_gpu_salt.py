"""GPU parity with salt (kappa > 0: the Debye-Hueckel factor 1/eps_in -
exp(-kappa f)/eps_out on every GB pair and self term) against the oracle's
salt form:

* radii, energies, forces, dE/dq and dE/drho of a ragged batch, both plans
  (the FP32 energy pass takes its salt instantiation);
* Delta E / Delta G of every candidate (FP64 potential rows, K_SS, self terms);
* the attempt pair and the sequential sweep (cross-site K blocks).
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import TOL, build, compare_system, gpu_eval, params_pair

pytestmark = pytest.mark.gpu

KB, F = 1.98720426e-3, 23.0605478
KAPPA = 0.1      # 1/A, about 0.1 M monovalent salt at 300 K


def _salt_pair(kappa=KAPPA):
    p_gpu, p_or = params_pair()
    return dataclasses.replace(p_gpu, kappa=kappa), dataclasses.replace(p_or, kappa=kappa)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_salt_energy_forces_parity(prec):
    p_gpu, p_or = _salt_pair()
    systems = synth.globule_256() + [synth.make_system(80 + k, n, max(4.0, 18.0 * (n / 2500.0) ** (1 / 3)))
                                 for k, n in enumerate((65, 1, 130, 300))]
    g, batch, plan, atoms = build(systems, prec)
    res = gpu_eval(plan, atoms, p_gpu)
    off = batch.atom_offset
    for b, s in enumerate(systems):
        ref = oracle.energy_forces(s, p_or)
        compare_system(res, b, off, ref, prec)
    # the salt term is really there: the salt-free energy differs
    ref0 = oracle.energy_forces(systems[0], params_pair()[1])
    assert abs(ref0["Egb"] - oracle.energy_forces(systems[0], p_or)["Egb"]) > 1e-3


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_salt_state_dE_parity(prec):
    p_gpu, p_or = _salt_pair()
    systems = synth.eremd_batch(n_rep=3)
    g, batch, plan, atoms = build(systems, prec)
    gref = np.random.default_rng(5).normal(0.0, 20.0, batch.state_count.size)
    sites = g.Sites.from_batch(plan, batch, gref)
    cur = torch.as_tensor(batch.current_state, device=plan.device)
    pH, E, T = np.array([5.0, 7.0, 9.0]), np.array([-0.3, -0.2, -0.1]), 300.0
    g.radii(plan, atoms, p_gpu)
    dE, dG = g.mc_state_dE(plan, sites, atoms, cur, pH, E, T, p_gpu)
    dE, dG = dE.cpu().numpy(), dG.cpu().numpy()
    c, g0 = 0, 0
    for b, s in enumerate(systems):
        n_st = sum(site.n_states for site in s.sites)
        tab = oracle.SiteTables(s, gref[g0:g0 + n_st])
        R = oracle.radii(s, p_or)["R"]
        ref = oracle.site_dE(s, R, p_or, tables=tab)
        refG = oracle.candidate_dG(s, ref, tab, pH[b], E[b], T)
        k = ref.size
        assert np.abs(dE[c:c + k] - ref).max() <= TOL[prec]["dE"], b
        assert np.abs(dG[c:c + k] - refG).max() <= TOL[prec]["dE"], b
        c += k
        g0 += n_st
    assert c == dE.size


def _near_balance_gref(systems, p_or, T, pH, E, seed):
    rng = np.random.default_rng(seed)
    out = []
    for b, s in enumerate(systems):
        R = oracle.radii(s, p_or)["R"]
        dE0 = oracle.site_dE(s, R, p_or)
        c = 0
        for site in s.sites:
            gs = np.zeros(site.n_states)
            for t in range(site.n_states):
                if t == site.state:
                    continue
                drive = (KB * T * math.log(10) * pH if site.kind == 0 else F * E[b]) \
                    * (site.counts[t] - site.counts[site.state])
                gs[t] = dE0[c] + drive + rng.normal(0.0, 0.5)
                c += 1
            out.append(gs)
    return np.concatenate(out)


def test_salt_step_and_sweep_fp64():
    p_gpu, p_or = _salt_pair()
    systems = synth.eremd_batch(n_rep=4)
    T, pH = 300.0, 7.0
    E = np.array(synth.E_LADDER[:4])
    gref = _near_balance_gref(systems, p_or, T, pH, E, 3)
    dev = torch.device("cuda")
    for mode in ("step", "sweep"):
        g, batch, plan, atoms = build(systems, "fp64")
        sites = g.Sites.from_batch(plan, batch, gref)
        cur = torch.as_tensor(batch.current_state, device=dev)
        g.radii(plan, atoms, p_gpu)
        if mode == "step":
            u = synth.uniforms(21, (4, 6))
            dE, dG = g.mc_state_dE(plan, sites, atoms, cur, pH, E, T, p_gpu)
            g.mc_step(plan, sites, atoms, cur, pH, E, dE, dG, torch.as_tensor(u, device=dev), T, p_gpu)
        else:
            u = synth.uniforms(22, (batch.n_sites, 3))
            g.mc_sweep(plan, sites, atoms, cur, pH, E, torch.as_tensor(u, device=dev), T, p_gpu)
        torch.cuda.synchronize()
        q = atoms.q.cpu().numpy()
        st = cur.cpu().numpy()
        m0, g0, n_moves = 0, 0, 0
        for b, s in enumerate(systems):
            ns = len(s.sites)
            n_st = sum(site.n_states for site in s.sites)
            tab = oracle.SiteTables(s, gref[g0:g0 + n_st])
            R = oracle.radii(s, p_or)["R"]
            if mode == "step":
                q_or, _, _ = oracle.mc_step(s, R, tab, pH, E[b], T, u[b], p_or)
            else:
                q_or, _, _ = oracle.mc_sweep(s, R, tab, pH, E[b], T, u[m0:m0 + ns], 3, p_or)
            sl = slice(batch.atom_offset[b], batch.atom_offset[b + 1])
            assert list(st[m0:m0 + ns]) == list(tab.current_state), (mode, b)
            assert np.array_equal(q[sl], q_or), (mode, b)
            n_moves += int(np.sum(np.array(tab.current_state) != batch.current_state[m0:m0 + ns]))
            m0 += ns
            g0 += n_st
        assert n_moves > 0, mode
