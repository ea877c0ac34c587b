"""GPU parity of mc_state_dE / mc_step / remd_exchange (C ABI) against the oracle,
Monte Carlo statistics on the device, and graph capture of a full step."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import TOL, build, params_pair

pytestmark = pytest.mark.gpu

KB, F = 1.98720426e-3, 23.0605478


def _gref(batch, seed):
    return np.random.default_rng(seed).normal(0.0, 20.0, batch.state_count.size)


def _oracle_tables(s, gref_slice):
    return oracle.SiteTables(s, gref_slice)


def _state_slices(systems):
    out, g = [], 0
    for s in systems:
        n = sum(site.n_states for site in s.sites)
        out.append((g, g + n))
        g += n
    return out


def _gpu_dE(g, plan, sites, atoms, batch, pH, E, T, params):
    cur = torch.as_tensor(batch.current_state, device=plan.device)
    g.radii(plan, atoms, params)
    dE, dG = g.mc_state_dE(plan, sites, atoms, cur, pH, E, T, params)
    torch.cuda.synchronize()
    return dE.cpu().numpy(), dG.cpu().numpy(), cur


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("cfg", ["globule_256", "globule_2500", "eremd_batch"])
def test_state_dE_and_dG_parity(prec, cfg):
    p_gpu, p_or = params_pair()
    systems = synth.workload(cfg)
    g, batch, plan, atoms = build(systems, prec)
    seed = ["globule_256", "globule_2500", "eremd_batch"].index(cfg)
    gref = _gref(batch, 5 + seed)
    sites = g.Sites.from_batch(plan, batch, gref)
    rng = np.random.default_rng(seed)
    pH = rng.uniform(3.0, 9.0, len(systems))
    E = rng.uniform(-0.4, -0.1, len(systems))
    T = 300.0
    dE, dG, _ = _gpu_dE(g, plan, sites, atoms, batch, pH, E, T, p_gpu)
    c = 0
    worst = 0.0
    for b, (s, (g0, g1)) in enumerate(zip(systems, _state_slices(systems))):
        R = oracle.radii(s, p_or)["R"]
        tab = _oracle_tables(s, gref[g0:g1])
        ref = oracle.site_dE(s, R, p_or, tables=tab)
        refG = oracle.candidate_dG(s, ref, tab, pH[b], E[b], T)
        k = ref.size
        worst = max(worst, np.abs(dE[c:c + k] - ref).max())
        assert np.abs(dE[c:c + k] - ref).max() <= TOL[prec]["dE"]
        assert np.abs(dG[c:c + k] - refG).max() <= TOL[prec]["dE"]
        c += k
    assert c == dE.size
    print(prec, cfg, "max |dE - ref|", worst)


def _oracle_step(systems, slices, gref, pH, E, T, u, p_or, q_states):
    """Oracle attempt pair on every system; returns (accepted [B,2], states, q, dG)."""
    acc, states, qs, dGs = [], [], [], []
    for b, s in enumerate(systems):
        g0, g1 = slices[b]
        tab = _oracle_tables(s, gref[g0:g1])
        R = oracle.radii(s, p_or)["R"]
        qn, out, dG = oracle.mc_step(s, R, tab, pH[b], E[b], T, u[b], p_or)
        acc.append(out[:2].copy())
        states.append(tab.current_state.copy())
        qs.append(qn)
        dGs.append(dG)
    return np.array(acc), states, qs, dGs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mc_step_parity(prec):
    p_gpu, p_or = params_pair()
    systems = synth.eremd_batch()
    g, batch, plan, atoms = build(systems, prec)
    slices = _state_slices(systems)
    # Gref chosen so that the attempts are neither all accepted nor all rejected:
    # each candidate's dG is roughly centred on zero
    rng = np.random.default_rng(17)
    gref = rng.normal(0.0, 1.0, batch.state_count.size)
    T, pH, E = 300.0, np.full(16, 7.0), np.array(synth.E_LADDER)
    for b, s in enumerate(systems):
        R = oracle.radii(s, p_or)["R"]
        tab = _oracle_tables(s, np.zeros(slices[b][1] - slices[b][0]))
        dE0 = oracle.site_dE(s, R, p_or, tables=tab)
        c = 0
        for m, site in enumerate(s.sites):
            g0 = slices[b][0] + sum(x.n_states for x in s.sites[:m])
            for t in range(site.n_states):
                if t == site.state:
                    continue
                drive = (KB * T * math.log(10) * pH[b] if site.kind == 0 else F * E[b]) \
                    * (site.counts[t] - site.counts[site.state])
                gref[g0 + t] = gref[g0 + site.state] + dE0[c] + drive + rng.normal(0, 0.5)
                c += 1
    sites = g.Sites.from_batch(plan, batch, gref)
    u = synth.uniforms(99, (16, 6))
    dE, dG, cur = _gpu_dE(g, plan, sites, atoms, batch, pH, E, T, p_gpu)
    u_t = torch.as_tensor(u, device=plan.device)
    counters = torch.zeros((batch.n_sites, 2), dtype=torch.int64, device=plan.device)
    out = g.mc_step(plan, sites, atoms, cur, pH, E, torch.as_tensor(dE, device=plan.device),
                    torch.as_tensor(dG, device=plan.device), u_t, T, p_gpu, counters=counters)
    torch.cuda.synchronize()
    acc_ref, states_ref, q_ref, dG_ref = _oracle_step(systems, slices, gref, pH, E, T, u, p_or, None)
    margin = 1e-9 if prec == "fp64" else 1e-3
    acc = out["accepted"].cpu().numpy()
    q = atoms.q.double().cpu().numpy()
    states = cur.cpu().numpy()
    off = batch.atom_offset
    compared = 0
    n_acc = 0
    s0 = 0
    for b, s in enumerate(systems):
        ns = len(s.sites)
        close = any(abs(u[b, 3 * k + 2] - math.exp(min(700, -dG_ref[b][k] / (KB * T)))) < margin
                    for k in range(2))
        if not close:
            assert acc[b].tolist() == acc_ref[b].tolist(), b
            assert states[s0:s0 + ns].tolist() == states_ref[b].tolist(), b
            qr = q_ref[b].astype(np.float32 if prec == "fp32" else np.float64)
            assert np.array_equal(q[off[b]:off[b + 1]], qr.astype(np.float64)), b
            ne_ref = oracle.count_electrons(s, _tables_with_state(s, slices[b], gref, states_ref[b]))
            assert int(out["n_electrons"][b]) == ne_ref
            compared += 1
            n_acc += int(acc[b].sum())
        s0 += ns
    assert compared >= 12
    assert 0 < n_acc < 2 * compared       # both outcomes occur
    cnt = counters.cpu().numpy()
    assert cnt[:, 0].sum() == 2 * 16 and cnt[:, 1].sum() == acc.sum()


def _tables_with_state(s, sl, gref, states):
    t = oracle.SiteTables(s, gref[sl[0]:sl[1]])
    t.current_state[:] = states
    return t


def test_mc_trajectory_matches_oracle_fp64():
    # 25 consecutive attempt pairs on the 2,500-atom globule (fixed coordinates): the state
    # sequence, including protonation -> redox coupling, follows the oracle
    p_gpu, p_or = params_pair()
    systems = synth.globule_2500()
    s = systems[0]
    g, batch, plan, atoms = build(systems, "fp64")
    rng = np.random.default_rng(3)
    R = oracle.radii(s, p_or)["R"]
    tab0 = oracle.SiteTables(s)
    dE0 = oracle.site_dE(s, R, p_or, tables=tab0)
    gref = np.zeros(batch.state_count.size)
    c = 0
    T, pH, E = 300.0, 7.0, -0.25
    for m, site in enumerate(s.sites):
        g0 = sum(x.n_states for x in s.sites[:m])
        for t in range(site.n_states):
            if t == site.state:
                continue
            drive = (KB * T * math.log(10) * pH if site.kind == 0 else F * E) \
                * (site.counts[t] - site.counts[site.state])
            gref[g0 + t] = dE0[c] + drive + rng.normal(0, 0.4)
            c += 1
    sites = g.Sites.from_batch(plan, batch, gref)
    tab = oracle.SiteTables(s, gref)
    q_or = s.q.copy()
    cur = torch.as_tensor(batch.current_state, device=plan.device)
    g.radii(plan, atoms, p_gpu)
    u_all = synth.uniforms(123, (25, 6))
    n_acc = 0
    for it in range(25):
        dE, dG = g.mc_state_dE(plan, sites, atoms, cur, pH, E, T, p_gpu)
        out = g.mc_step(plan, sites, atoms, cur, pH, E, dE, dG,
                        torch.as_tensor(u_all[it:it + 1], device=plan.device), T, p_gpu)
        so = s.copy()
        so.q = q_or
        q_or, o, dG_ref = oracle.mc_step(so, R, tab, pH, E, T, u_all[it], p_or, q=q_or)
        torch.cuda.synchronize()
        for k in range(2):
            p = math.exp(min(700, -dG_ref[k] / (KB * T)))
            assert abs(u_all[it, 3 * k + 2] - p) > 1e-9
        assert out["accepted"].cpu().numpy()[0].tolist() == o[:2].tolist(), it
        assert cur.cpu().numpy().tolist() == tab.current_state.tolist(), it
        n_acc += int(o[:2].sum())
    assert np.array_equal(atoms.q.cpu().numpy(), q_or)
    assert n_acc > 3


def test_nernst_fraction_on_device():
    # many copies of one small globule with one uncoupled 2-state redox site,
    # Gref set so that dG = F (E - E0) (Eq. 8 with dG_elec = dG_elec,ref)
    p_gpu, p_or = params_pair()
    base = synth.make_system(31, 40, 8.0, n_redox=1, redox_atoms=5)
    R = oracle.radii(base, p_or)["R"]
    dE = oracle.site_dE(base, R, p_or)[0]
    E0, T = -0.203, 300.0
    B = 2048
    systems = [base.copy() for _ in range(B)]
    g, batch, plan, atoms = build(systems, "fp64")
    gref = np.tile([0.0, dE + F * E0], B)
    sites = g.Sites.from_batch(plan, batch, gref)
    cur = torch.as_tensor(batch.current_state, device=plan.device)
    E = E0 + 0.02
    g.radii(plan, atoms, p_gpu)
    gen = torch.Generator(device=plan.device)
    gen.manual_seed(7)
    steps, red = 200, 0
    for it in range(steps):
        dEg, dGg = g.mc_state_dE(plan, sites, atoms, cur, 7.0, E, T, p_gpu)
        u = torch.rand((B, 6), dtype=torch.float64, device=plan.device, generator=gen)
        g.mc_step(plan, sites, atoms, cur, 7.0, E, dEg, dGg, u, T, p_gpu)
        red += int(cur.sum())
    f_red = red / (steps * B)
    ref = 1.0 / (1.0 + math.exp(F * (E - E0) / (KB * T)))
    g_ = F * (E - E0)
    a, b = min(1, math.exp(-g_ / (KB * T))), min(1, math.exp(g_ / (KB * T)))
    lam = 1 - a - b
    sig = math.sqrt(ref * (1 - ref) * (1 + lam) / (1 - lam) / (steps * B))
    assert abs(f_red - ref) <= 5 * sig, (f_red, ref, sig)


@pytest.mark.parametrize("M", [2, 3, 4, 16, 17, 600])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("wrap", [True, False])
def test_remd_exchange_parity(M, parity, wrap):
    g = __import__("paper_1803_09652_amd")
    rng = np.random.default_rng(M * 4 + parity * 2 + int(wrap))
    E_rung = np.sort(rng.uniform(-0.45, -0.05, M))
    Ne = rng.integers(0, 4, M).astype(np.int32)
    rep = rng.permutation(M).astype(np.int32)
    u = rng.random(M)
    rep_ref, acc_ref, Eo_ref = oracle.remd_exchange(E_rung, Ne, rep, 300.0, parity, wrap, u)
    dev = torch.device("cuda")
    rep_t = torch.as_tensor(rep, device=dev)
    acc, Eo = g.remd_exchange(torch.as_tensor(E_rung, device=dev), torch.as_tensor(Ne, device=dev),
                              rep_t, parity, torch.as_tensor(u, device=dev), 300.0, wrap)
    torch.cuda.synchronize()
    assert rep_t.cpu().numpy().tolist() == rep_ref.tolist()
    assert acc.cpu().numpy().tolist() == acc_ref.tolist()
    assert np.array_equal(Eo.cpu().numpy(), Eo_ref)


def test_full_step_graph_replay_follows_eager():
    # radii -> energy/forces -> all candidate dE -> MC step, captured once and
    # replayed; the state trajectory equals the eager one step by step
    p_gpu, _ = params_pair()
    systems = synth.eremd_batch(n_rep=4)

    def setup():
        g, batch, plan, atoms = build(systems, "fp32")
        sites = g.Sites.from_batch(plan, batch, np.random.default_rng(2).normal(0, 30, batch.state_count.size))
        cur = torch.as_tensor(batch.current_state, device=plan.device)
        u = torch.zeros((4, 6), dtype=torch.float64, device=plan.device)
        return g, plan, atoms, sites, cur, u

    us = synth.uniforms(8, (6, 4, 6))
    g, plan, atoms, sites, cur, u = setup()
    # device-resident pH / E: nothing is copied from the host inside the capture
    pH = torch.full((4,), 7.0, dtype=torch.float64, device=plan.device)
    E = torch.full((4,), -0.25, dtype=torch.float64, device=plan.device)

    def step():
        g.radii(plan, atoms, p_gpu)
        ef = g.energy_forces(plan, atoms, p_gpu)
        dE, dG = g.mc_state_dE(plan, sites, atoms, cur, pH, E, 300.0, p_gpu)
        g.mc_step(plan, sites, atoms, cur, pH, E, dE, dG, u, 300.0, p_gpu)
        return ef

    traj_eager = []
    for it in range(6):
        u.copy_(torch.as_tensor(us[it]))
        ef = step()
        torch.cuda.synchronize()
        traj_eager.append((cur.cpu().numpy().copy(), atoms.q.cpu().numpy().copy(),
                           ef["force"].cpu().numpy().copy()))
    g, plan, atoms, sites, cur, u = setup()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                              # warm-up (changes state: redo setup)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g, plan, atoms, sites, cur, u = setup()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ef = step()
    # capture does not execute: state is still the initial one
    for it in range(6):
        u.copy_(torch.as_tensor(us[it]))
        graph.replay()
        torch.cuda.synchronize()
        st, q, f = traj_eager[it]
        assert np.array_equal(cur.cpu().numpy(), st), it
        assert np.array_equal(atoms.q.cpu().numpy(), q), it
        assert np.array_equal(ef["force"].cpu().numpy(), f), it
        _ = torch.ones(10, device=plan.device).sum().item()   # eager work between replays
