"""GPU parity with the optional cutoffs (descreening rgbmax: the HCT integral
restricted to the sphere of that radius around each atom; energy cutoff: pair
terms at or beyond it dropped), against the oracle's cutoff forms:

* a ragged batch (1, 65, 300 and 2,500 atoms), both plans and the
  compact-block order: radii, energies,
  forces, dE/dq, dE/drho (tiles skipped by their bounding spheres, balls
  straddling the descreening sphere, pairs beyond the energy cutoff);
* Delta E / Delta G of every candidate with the pair cutoff (FP64 rows, K_SS);
* a 20,000-atom globule (FP32 plan, rgbmax 12 A, pair cutoff near 6 A): every
  atom.

The energy cutoff is discontinuous, so each test places it in the widest gap
of the pair distances near the nominal value, far from any pair compared with
the rounding of r in either precision.
"""
import dataclasses

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import oracle
import synth
from gpu_common import TOL, build, compare_system, gpu_eval, params_pair

pytestmark = pytest.mark.gpu


def _cutoff_in_gap(systems, lo, hi):
    d = []
    for s in systems:
        xyz = s.coords().astype(np.float64)
        t = cKDTree(xyz)
        pr = t.query_pairs(hi, output_type="ndarray")
        if pr.size:
            r = np.linalg.norm(xyz[pr[:, 0]] - xyz[pr[:, 1]], axis=1)
            d.append(r[(r > lo) & (r < hi)])
    d = np.sort(np.concatenate(d + [np.array([lo, hi])]))
    k = int(np.argmax(np.diff(d)))
    cut = 0.5 * (d[k] + d[k + 1])
    clearance = 0.5 * (d[k + 1] - d[k])
    assert clearance > 1e-5, clearance
    return cut


def _pair(rgbmax, cutoff):
    p_gpu, p_or = params_pair()
    return (dataclasses.replace(p_gpu, rgbmax=rgbmax, cutoff=cutoff),
            dataclasses.replace(p_or, rgbmax=rgbmax, cutoff=cutoff))


@pytest.mark.parametrize("prec,order,kappa", [("fp32", "identity", 0.0), ("fp64", "identity", 0.0),
                                              ("fp32", "blocks", 0.0), ("fp32", "blocks", 0.1)])
def test_cutoff_batch_parity(prec, order, kappa):
    systems = [synth.make_system(120, 1, 2.0), synth.make_system(121, 65, 5.0),
               synth.make_system(122, 300, 8.5)] + synth.globule_2500()
    cut = _cutoff_in_gap(systems, 10.0, 10.5)
    p_gpu, p_or = _pair(12.0, cut)
    p_gpu, p_or = dataclasses.replace(p_gpu, kappa=kappa), dataclasses.replace(p_or, kappa=kappa)
    g, batch, plan, atoms = build(systems, prec)
    if order == "blocks":
        plan.set_order(g.block_order(batch.atom_offset, batch.x, batch.y, batch.z))
    res = gpu_eval(plan, atoms, p_gpu)
    off = batch.atom_offset
    for b, s in enumerate(systems):
        ref = oracle.energy_forces(s, p_or)
        compare_system(res, b, off, ref, prec)
    # the cutoffs matter on the 2,500-atom globule (36 A across)
    full = oracle.energy_forces(systems[3], params_pair()[1])
    ref = oracle.energy_forces(systems[3], p_or)
    assert abs(full["E"] - ref["E"]) > 1e-2 and np.abs(full["R"] - ref["R"]).max() > 1e-3


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_cutoff_state_dE_parity(prec):
    systems = synth.eremd_batch(n_rep=3)
    cut = _cutoff_in_gap(systems, 8.0, 8.5)
    p_gpu, p_or = _pair(10.0, cut)
    g, batch, plan, atoms = build(systems, prec)
    gref = np.random.default_rng(6).normal(0.0, 20.0, batch.state_count.size)
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


def test_cutoff_large_globule_fp32():
    s = synth.make_system(130, 20000, 18.0 * (20000 / 2500.0) ** (1 / 3))
    # 2.5 million pairs per A of distance at 14 A leave no gap wide enough:
    # the pair cutoff goes near 6 A (the descreening cutoff is continuous)
    cut = _cutoff_in_gap([s], 6.0, 6.5)
    p_gpu, p_or = _pair(12.0, cut)
    g, batch, plan, atoms = build([s], "fp32", j_blocks=8)
    res = gpu_eval(plan, atoms, p_gpu)
    ref = oracle.energy_forces(s, p_or)
    compare_system(res, 0, batch.atom_offset, ref, "fp32")


def test_cutoff_sweep_fp64():
    # the sequential sweep with the pair cutoff (potential rows, K_SS and the
    # K dq updates after each accepted visit) against the oracle's sweep
    systems = synth.eremd_batch(n_rep=3)
    cut = _cutoff_in_gap(systems, 9.0, 9.5)
    p_gpu, p_or = _pair(11.0, cut)
    g, batch, plan, atoms = build(systems, "fp64")
    gref = np.random.default_rng(9).normal(0.0, 2.0, batch.state_count.size)
    sites = g.Sites.from_batch(plan, batch, gref)
    dev = plan.device
    cur = torch.as_tensor(batch.current_state, device=dev)
    u = synth.uniforms(31, (batch.n_sites, 3))
    E = np.array([-0.3, -0.25, -0.2])
    g.radii(plan, atoms, p_gpu)
    out = g.mc_sweep(plan, sites, atoms, cur, 7.0, E, torch.as_tensor(u, device=dev), 300.0, p_gpu)
    torch.cuda.synchronize()
    dG = out["dG"].cpu().numpy()
    st = cur.cpu().numpy()
    m0, g0 = 0, 0
    for b, s in enumerate(systems):
        ns = len(s.sites)
        n_st = sum(site.n_states for site in s.sites)
        tab = oracle.SiteTables(s, gref[g0:g0 + n_st])
        R = oracle.radii(s, p_or)["R"]
        q_or, acc_or, dG_or = oracle.mc_sweep(s, R, tab, 7.0, E[b], 300.0, u[m0:m0 + ns], 3, p_or)
        assert np.all(np.abs(dG[m0:m0 + ns] - dG_or) <= 1e-9 * np.maximum(1.0, np.abs(dG_or))), b
        assert list(st[m0:m0 + ns]) == list(tab.current_state), b
        m0 += ns
        g0 += n_st
