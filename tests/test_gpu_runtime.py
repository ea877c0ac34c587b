"""GPU tests of the simulation loop (ReplicaMD): Langevin dynamics on the GB
forces with Monte Carlo attempts and E-REMD exchanges on their schedules.

* FP64: the loop equals an oracle-driven loop (oracle Born radii, oracle
  attempt pair, oracle exchange, oracle Langevin step) fed the same noise and
  uniforms, step by step to the end: states, charges, ladder, coordinates and
  velocities;
* E-REMD of an uncoupled redox site at frozen geometry samples the Nernst
  fraction on every rung (Eq. 3 with n = 1), and the Hill fit of the sampled
  fractions returns the site's standard potential;
* FP32: the loop runs the 16-replica E-REMD batch (2,500 atoms each, every
  atom restrained) and keeps the fixed-point accumulators in range.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import build, params_pair

pytestmark = pytest.mark.gpu

KB, F = 1.98720426e-3, 23.0605478
T, PH, DT, GAMMA = 300.0, 7.0, 0.002, 5.0
KR = synth.MD_RESTRAINT


def _replicas(n_rep, n=70, seed=501):
    base = synth.make_system(seed, n, 5.5, n_redox=1, n_prot=1, redox_atoms=6, prot_atoms=(4, 6),
                             min_dist=1.5, prot_states=3)
    return [base] + [synth.perturb(base, seed + 10 + k, sigma=0.2, min_pair=1.5)
                     for k in range(n_rep - 1)]


def test_loop_matches_oracle_driven_loop():
    from paper_1803_09652_amd.runtime import ReplicaMD
    p_gpu, p_or = params_pair()
    B, n_steps, att_every, x_every = 4, 12, 3, 6
    systems = _replicas(B)
    g, batch, plan, atoms = build(systems, "fp64")
    gref = synth.normals(7, batch.state_count.size)          # arbitrary reference energies
    sites = g.Sites.from_batch(plan, batch, gref)
    N = batch.x.shape[0]
    m = synth.masses(8, N)
    v0 = synth.thermal_velocities(9, m, T)
    xref = np.stack([batch.x, batch.y, batch.z])
    E_rung = np.array([-0.30, -0.28, -0.26, -0.24])
    rep0 = np.array([2, 0, 3, 1])
    xi = synth.normals(10, (n_steps, 3, N))
    u_mc = synth.uniforms(11, (n_steps // att_every, B, 6))
    u_x = synth.uniforms(12, (n_steps // x_every, B))
    loop = ReplicaMD(plan, sites, atoms, batch.current_state, 1.0 / m, v0.T, PH, E_rung, rep0,
                     DT, GAMMA, T, att_every, x_every, p_gpu, xref=xref, k_restr=KR)
    dev = plan.device
    rec = loop.run(n_steps, torch.as_tensor(xi, device=dev), torch.as_tensor(u_mc, device=dev),
                   torch.as_tensor(u_x, device=dev))
    torch.cuda.synchronize()

    # the same loop on the oracle
    off, soff = batch.atom_offset, batch.site_state_offset
    sys_ = [s.copy() for s in systems]
    tabs, m0 = [], 0
    for s in systems:
        ns = len(s.sites)
        tabs.append(oracle.SiteTables(s, gref[soff[m0]:soff[m0 + ns]]))
        m0 += ns
    v = [v0[off[b]:off[b + 1]].copy() for b in range(B)]
    rep = rep0.copy()
    E_rep = np.empty(B)
    E_rep[rep] = E_rung
    ne = np.array([oracle.count_electrons(s, t) for s, t in zip(sys_, tabs)], np.int32)
    a_i = x_i = 0
    states = []
    for k in range(n_steps):
        if (k + 1) % att_every == 0:
            for b in range(B):
                R = oracle.radii(sys_[b], p_or)["R"]
                q, _, _ = oracle.mc_step(sys_[b], R, tabs[b], PH, E_rep[b], T, u_mc[a_i, b], p_or)
                sys_[b].q = q
                ne[b] = oracle.count_electrons(sys_[b], tabs[b])
            states.append((np.concatenate([t.current_state for t in tabs]), rep.copy()))
            a_i += 1
        if (k + 1) % x_every == 0:
            rep, _, E_rep = oracle.remd_exchange(E_rung, ne, rep, T, x_i % 2, True, u_x[x_i])
            x_i += 1
        for b in range(B):
            sl = slice(off[b], off[b + 1])
            x, y, z, v[b] = oracle.langevin_step(sys_[b], v[b], 1.0 / m[sl], xi[k][:, sl].T, DT, GAMMA,
                                                 T, p_or, xref=xref[:, sl].T, k_restr=KR)
            sys_[b].x, sys_[b].y, sys_[b].z = x, y, z

    st = rec["state"].cpu().numpy()
    rr = rec["rep_of_rung"].cpu().numpy()
    assert len(states) == st.shape[0] == n_steps // att_every
    for a, (s_ref, r_ref) in enumerate(states):
        assert np.array_equal(st[a], s_ref), a
        assert np.array_equal(rr[a], r_ref), a
    assert np.array_equal(loop.rep_of_rung.cpu().numpy(), rep)
    assert np.allclose(loop.E_rep.cpu().numpy(), E_rep, rtol=0, atol=0)
    q = atoms.q.cpu().numpy()
    pos = torch.stack([atoms.x, atoms.y, atoms.z], 1).cpu().numpy()
    vg = loop.v.cpu().numpy().T
    for b in range(B):
        sl = slice(off[b], off[b + 1])
        assert np.array_equal(q[sl], sys_[b].q), b
        assert np.abs(pos[sl] - sys_[b].coords()).max() <= 1e-9, b
        assert np.abs(vg[sl] - v[b]).max() <= 1e-8 * max(1.0, np.abs(v[b]).max()), b
    # something happened: some attempts were accepted
    assert loop.counters[:, 1].sum().item() > 0


def test_eremd_uncoupled_redox_site_follows_nernst():
    from paper_1803_09652_amd import analysis
    from paper_1803_09652_amd.runtime import ReplicaMD
    p_gpu, p_or = params_pair()
    M, E0 = 16, -0.25
    base = synth.make_system(601, 40, 5.0, n_redox=1, redox_atoms=5, min_dist=1.5)
    systems = [base.copy() for _ in range(M)]
    g, batch, plan, atoms = build(systems, "fp64")
    # reference energies that cancel the site's own electrostatics, so the
    # reduction free energy is F (E - E0) exactly (Eq. 8 with Delta G_elec =
    # Delta G_elec,ref)
    assert base.sites[0].state == 0                           # starts oxidised
    R = oracle.radii(base, p_or)["R"]
    dE = oracle.site_dE(base, R, p_or)[0]                     # oxidised -> reduced
    gref = np.tile([0.0, dE + F * E0], M)
    sites = g.Sites.from_batch(plan, batch, gref)
    state0 = np.zeros(M, np.int32)
    N = batch.x.shape[0]
    E_rung = E0 + 0.02 * (np.arange(M) - (M - 1) / 2)
    loop = ReplicaMD(plan, sites, atoms, state0, np.zeros(N), np.zeros((3, N)), PH, E_rung,
                     dt=DT, gamma=GAMMA, T=T, attempt_every=1, exchange_every=2, params=p_gpu,
                     seed=77)
    rec = loop.run(3000)
    torch.cuda.synchronize()
    f = analysis.fraction_by_rung(rec["state"].cpu().numpy(), rec["rep_of_rung"].cpu().numpy(),
                                  sites.site_system, sites.site_kind, sites.site_state_offset,
                                  sites.state_count)[:, 0]
    exact = analysis.f_red(E_rung, E0, 1.0, T)
    assert np.abs(f - exact).max() < 0.06, np.abs(f - exact).max()
    e0, n, de0, dn = analysis.fit_hill(E_rung, f, T)
    print("E0", e0, "+-", de0, "n", n, "+-", dn, "exchanges accepted",
          loop.exchanges_accepted, "of", loop.n_exchanges)
    assert abs(e0 - E0) < 0.006 and abs(n - 1.0) < 0.15
    # the coordinates never moved (zero inverse mass, zero velocity)
    assert np.array_equal(atoms.x.cpu().numpy(), batch.x)
    assert loop.exchanges_accepted > 0


def test_fp32_eremd_batch_runs_in_range():
    from paper_1803_09652_amd.runtime import ReplicaMD
    p_gpu, _ = params_pair()
    systems = synth.eremd_batch_md(n_rep=16)
    g, batch, plan, atoms = build(systems, "fp32")
    sites = g.Sites.from_batch(plan, batch)
    N = batch.x.shape[0]
    m = synth.masses(3, N)
    xref = np.stack([batch.x, batch.y, batch.z])
    loop = ReplicaMD(plan, sites, atoms, batch.current_state, 1.0 / m,
                     synth.thermal_velocities(4, m, T).T, PH, np.array(synth.E_LADDER), dt=DT,
                     gamma=GAMMA, T=T, attempt_every=5, exchange_every=10, params=p_gpu,
                     xref=xref, k_restr=synth.MD_RESTRAINT, seed=5)
    loop.run(40)
    torch.cuda.synchronize()
    assert not g.check_overflow(plan)
    pos = torch.stack([atoms.x, atoms.y, atoms.z], 1).cpu().numpy()
    assert np.isfinite(pos).all()
    # restrained atoms stay near their centres (thermal rms ~ sqrt(3 kT / k))
    rms = math.sqrt(((pos - xref.T) ** 2).sum(1).mean())
    assert rms < 0.3, rms
    assert loop.n_attempts == 8 and loop.n_exchanges == 4


def test_pure_dynamics_loop_without_sites():
    # CEMD's dynamics alone: no titratable sites, no attempts, no exchanges;
    # a one-atom system beside a 30-atom one (FP64 against the oracle step)
    from paper_1803_09652_amd.runtime import ReplicaMD
    p_gpu, p_or = params_pair()
    systems = [synth.make_system(701, 30, 4.5, min_dist=1.5), synth.make_system(702, 1, 2.0)]
    g, batch, plan, atoms = build(systems, "fp64")
    assert batch.n_sites == 0
    sites = g.Sites.from_batch(plan, batch)
    N = batch.x.shape[0]
    m = synth.masses(12, N)
    v0 = synth.thermal_velocities(13, m, T)
    xref = np.stack([batch.x, batch.y, batch.z])
    xi = synth.normals(14, (8, 3, N))
    loop = ReplicaMD(plan, sites, atoms, np.zeros(0, np.int32), 1.0 / m, v0.T, PH, np.zeros(2),
                     dt=DT, gamma=GAMMA, T=T, attempt_every=0, exchange_every=0, params=p_gpu,
                     xref=xref, k_restr=KR)
    rec = loop.run(8, torch.as_tensor(xi, device=plan.device))
    torch.cuda.synchronize()
    assert rec["state"].shape == (0, 0) and loop.n_attempts == 0 and loop.n_exchanges == 0
    pos = torch.stack([atoms.x, atoms.y, atoms.z], 1).cpu().numpy()
    off = batch.atom_offset
    for b, s in enumerate(systems):
        sl = slice(off[b], off[b + 1])
        sys_, v = s.copy(), v0[sl].copy()
        for k in range(8):
            x, y, z, v = oracle.langevin_step(sys_, v, 1.0 / m[sl], xi[k][:, sl].T, DT, GAMMA, T, p_or,
                                              xref=xref[:, sl].T, k_restr=KR)
            sys_.x, sys_.y, sys_.z = x, y, z
        assert np.abs(pos[sl] - sys_.coords()).max() <= 1e-9, b


def test_two_ph_ladders_exchange_separately():
    # replicas at pH 5 and pH 7 form two ladders; each ladder's exchange
    # attempt sees only its own replicas (FP64, frozen geometry, against the
    # oracle's attempt pair and exchange applied ladder by ladder)
    from paper_1803_09652_amd.runtime import ReplicaMD
    p_gpu, p_or = params_pair()
    systems = _replicas(6)
    g, batch, plan, atoms = build(systems, "fp64")
    gref = synth.normals(17, batch.state_count.size) * 0.5
    sites = g.Sites.from_batch(plan, batch, gref)
    N, B = batch.x.shape[0], 6
    pH = np.array([5.0, 5.0, 5.0, 7.0, 7.0, 7.0])
    E_rung = np.array([-0.30, -0.27, -0.24, -0.30, -0.27, -0.24])
    rep0 = np.array([1, 2, 0, 5, 3, 4])
    ladders = [(0, 3), (3, 6)]
    n_steps = 8
    u_mc = synth.uniforms(18, (n_steps, B, 6))
    u_x = synth.uniforms(19, (n_steps, B))
    loop = ReplicaMD(plan, sites, atoms, batch.current_state, np.zeros(N), np.zeros((3, N)), pH,
                     E_rung, rep0, dt=DT, gamma=GAMMA, T=T, attempt_every=1, exchange_every=1,
                     params=p_gpu, ladders=ladders)
    dev = plan.device
    rec = loop.run(n_steps, u_mc=torch.as_tensor(u_mc, device=dev),
                   u_x=torch.as_tensor(u_x, device=dev))
    torch.cuda.synchronize()

    soff = batch.site_state_offset
    tabs, m0 = [], 0
    for s in systems:
        ns = len(s.sites)
        tabs.append(oracle.SiteTables(s, gref[soff[m0]:soff[m0 + ns]]))
        m0 += ns
    sys_ = [s.copy() for s in systems]
    rep = rep0.copy()
    E_rep = np.empty(B)
    E_rep[rep] = E_rung
    ne = np.array([oracle.count_electrons(s, t) for s, t in zip(sys_, tabs)], np.int32)
    for k in range(n_steps):
        for b in range(B):
            R = oracle.radii(sys_[b], p_or)["R"]
            q, _, _ = oracle.mc_step(sys_[b], R, tabs[b], pH[b], E_rep[b], T, u_mc[k, b], p_or)
            sys_[b].q = q
            ne[b] = oracle.count_electrons(sys_[b], tabs[b])
        assert np.array_equal(rec["state"][k].cpu().numpy(),
                              np.concatenate([t.current_state for t in tabs])), k
        assert np.array_equal(rec["rep_of_rung"][k].cpu().numpy(), rep), k
        for a, e in ladders:
            sys_k = np.sort(rep[a:e])
            local = np.searchsorted(sys_k, rep[a:e])
            loc, _, Eo = oracle.remd_exchange(E_rung[a:e], ne[sys_k], local, T, k % 2, True,
                                              u_x[k, a:e])
            rep[a:e] = sys_k[loc]
            E_rep[sys_k] = Eo
        # replicas never leave their ladder
        assert set(rep[:3]) == {0, 1, 2} and set(rep[3:]) == {3, 4, 5}
    assert np.array_equal(loop.rep_of_rung.cpu().numpy(), rep)
    assert np.array_equal(loop.E_rep.cpu().numpy(), E_rep)
    assert loop.exchanges_accepted > 0
