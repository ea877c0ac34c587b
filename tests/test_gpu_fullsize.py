"""GPU parity at full size, in the launch configuration the benchmark times.

The benchmark's step (``bench.Workload``: its default processing order,
the Monte Carlo branch on a second stream beside the force passes,
double-buffered charges, two exchange-parity hipGraphs captured after two
eager steps and then replayed) is run on

  * the E-REMD batch (16 replicas x 2,500 atoms, every replica compared), and
  * the uneven 64-system batch (500-20,000 atoms; a stratified set of 8
    systems: the smallest, the largest and six at evenly spaced size ranks),

in both plans, and compared step by step with an oracle-driven sequence of
the same steps fed the same uniforms: Born radii, E_C, E_GB, forces, dE/dq and
dE/drho, every candidate's Delta E and Delta G, both Metropolis decisions of
every system, the states, charges and electron counts they leave, and (E-REMD)
the exchange ladder after every step.  Reference free energies are computed by
the oracle (Delta E at the starting geometry plus the reference compound's E0
or pKa term), never taken from the GPU path.

Decisions are compared bitwise away from the acceptance margin |u - p| <=
MARGIN (1e-9 in the FP64 plan, 1e-3 in the FP32 plan, whose Delta G carries up
to 1e-4 kcal/mol).  A system whose decision falls inside the margin is compared
up to that step only (its later states may legitimately differ); in the E-REMD
batch the ladder couples every replica, so the comparison of the whole batch
stops there.  The FP64 plan must reach no margin case.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import TOL, params_pair, rel_inf

pytestmark = pytest.mark.gpu

KB, F = oracle.KB, oracle.FARADAY
T, PH = 300.0, 7.0
MARGIN = {"fp64": 1e-9, "fp32": 1e-3}


def _oracle_gref(systems, p_or, E0_ref, pKa_ref):
    """Reference free energies of every state by the benchmark's recipe, from
    the oracle: Gref(s') - Gref(s0) = Delta E(s0 -> s') at the starting
    geometry and states + (F E0_ref | kB T ln10 pKa_ref) * (count(s') - count(s0))."""
    out = []
    for b, s in enumerate(systems):
        R = oracle.radii(s, p_or)["R"]
        dE0 = oracle.site_dE(s, R, p_or, tables=oracle.SiteTables(s))
        c = 0
        for site in s.sites:
            g = np.zeros(site.n_states)
            ref = F * E0_ref if site.kind == synth.KIND_REDOX else KB * T * math.log(10) * pKa_ref
            for t in range(site.n_states):
                if t == site.state:
                    continue
                g[t] = dE0[c] + ref * (site.counts[t] - site.counts[site.state])
                c += 1
            out.append(g)
    return np.concatenate(out) if out else np.zeros(0)


def _run_workload(prec, systems, exchange, n_steps, gref):
    """The benchmark's step sequence: steps 0 and 1 eager (the capture
    warm-up), then the two parity graphs captured and replayed for steps
    2 .. n_steps - 1.  Returns the workload and one host snapshot per step."""
    import bench
    w = bench.Workload(prec, n_steps, bench.DEFAULT_ORDER, None, True, systems=systems,
                       exchange=exchange, gref=gref)

    def snap(last):
        torch.cuda.synchronize()
        ef = last["force_out"]
        host = lambda t: t.double().cpu().numpy().copy()
        return {"R": host(last["R"]), "Ec": host(ef["e_coul"]), "Egb": host(ef["e_gb"]),
                "force": host(ef["force"]), "dEdq": host(ef["dEdq"]), "dEdrho": host(ef["dEdrho"]),
                "dE": host(last["dE"]), "dG": host(last["dG"]),
                "accepted": last["mc"]["accepted"].cpu().numpy().copy(),
                "n_electrons": last["mc"]["n_electrons"].cpu().numpy().copy(),
                "q": host(last["q_out"]), "state": w.cur.cpu().numpy().copy(),
                "rep": w.rep_of_rung.cpu().numpy().copy(), "E_rep": w.E_rep.cpu().numpy().copy()}

    snaps = []
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for k in range(2):
            w.step(k % 2)
            snaps.append(snap(w.last))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graphs, lasts = [], []
    for parity in (0, 1):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            w.step(parity)
        graphs.append(gr)
        lasts.append(dict(w.last))
    for k in range(2, n_steps):
        graphs[k % 2].replay()
        snaps.append(snap(lasts[k % 2]))
    return w, snaps


def _cand_slices(batch):
    n_cand = np.diff(batch.site_state_offset) - 1
    c_off = np.concatenate([[0], np.cumsum(n_cand)])
    out = []
    for b in range(batch.n_systems):
        m = np.nonzero(batch.site_system == b)[0]
        out.append((int(c_off[m[0]]), int(c_off[m[-1] + 1])) if m.size else (0, 0))
    return out


def _site_slices(batch):
    out = []
    for b in range(batch.n_systems):
        m = np.nonzero(batch.site_system == b)[0]
        out.append((int(m[0]), int(m[-1]) + 1) if m.size else (0, 0))
    return out


def _compare_sequence(prec, w, snaps, pick, force_steps):
    """Replays the workload's steps with the oracle on the systems in pick and
    compares every step.  Returns the number of (system, step) pairs compared
    in full and the worst errors."""
    _, p_or = params_pair()
    tol = TOL[prec]
    batch, systems = w.batch, w.systems
    off = batch.atom_offset
    cand = _cand_slices(batch)
    sites = _site_slices(batch)
    gref = np.asarray(w.gref)
    u_all = w.u_all.cpu().numpy()
    ux_all = w.ux_all.cpu().numpy()
    kT = KB * T
    # oracle state per compared system
    st = {}
    for b in pick:
        s = systems[b].copy()
        g0, g1 = batch.site_state_offset[sites[b][0]], batch.site_state_offset[sites[b][1]]
        st[b] = {"s": s, "tab": oracle.SiteTables(s, gref[g0:g1]),
                 "R": oracle.radii(s, p_or)["R"], "active": True}
    E_rep = (np.array(synth.E_LADDER, dtype=np.float64) if w.exchange
             else np.full(batch.n_systems, w.E_rung.cpu().numpy()[0]))
    rep = np.arange(batch.n_systems, dtype=np.int32)
    worst = {}
    n_full = 0
    ladder_ok = w.exchange

    def err(key, v):
        worst[key] = max(worst.get(key, 0.0), float(v))

    for k, sn in enumerate(snaps):
        if not any(v["active"] for v in st.values()):
            break
        margin_hit = False
        for b in pick:
            o = st[b]
            if not o["active"]:
                continue
            s, tab = o["s"], o["tab"]
            a0, a1 = int(off[b]), int(off[b + 1])
            if k in force_steps:
                ref = oracle.energy_forces(s, p_or)
                e = np.max(np.abs(sn["R"][a0:a1] - ref["R"]) / ref["R"])
                err("R", e)
                assert e <= tol["R"], (k, b, "R", e)
                scale = abs(ref["Ec"]) + abs(ref["Egb"])
                for key in ("Ec", "Egb"):
                    e = abs(sn[key][b] - ref[key]) / scale
                    err(key, e)
                    assert e <= tol["E"], (k, b, key, e)
                for key, rk in (("force", "F"), ("dEdq", "phi"), ("dEdrho", "dEdrho")):
                    e = rel_inf(sn[key][a0:a1], ref[rk])
                    err(key, e)
                    assert e <= tol["grad"], (k, b, key, e)
            c0, c1 = cand[b]
            dE_ref = oracle.site_dE(s, o["R"], p_or, tables=tab)
            dG_ref = oracle.candidate_dG(s, dE_ref, tab, PH, E_rep[b], T)
            if c1 > c0:
                e = np.abs(sn["dE"][c0:c1] - dE_ref).max()
                err("dE", e)
                assert e <= tol["dE"], (k, b, "dE", e)
                e = np.abs(sn["dG"][c0:c1] - dG_ref).max()
                err("dG", e)
                assert e <= tol["dE"], (k, b, "dG", e)
            q_new, out, dG2 = oracle.mc_step(s, o["R"], tab, PH, E_rep[b], T, u_all[k, b], p_or,
                                             q=s.q)
            u = u_all[k, b]
            near = [abs(u[2] - math.exp(min(700.0, -dG2[0] / kT))) <= MARGIN[prec],
                    abs(u[5] - math.exp(min(700.0, -dG2[1] / kT))) <= MARGIN[prec]]
            if any(near):
                assert prec != "fp64", (k, b, "FP64 decision at the margin")
                o["active"] = False
                margin_hit = True
                continue
            assert list(sn["accepted"][b]) == list(out[:2]), (k, b, sn["accepted"][b], out[:2])
            m0, m1 = sites[b]
            assert list(sn["state"][m0:m1]) == list(tab.current_state), (k, b)
            assert np.array_equal(sn["q"][a0:a1], q_new) if prec == "fp64" else \
                np.allclose(sn["q"][a0:a1], q_new, rtol=0, atol=1e-6), (k, b)
            assert sn["n_electrons"][b] == oracle.count_electrons(s, tab), (k, b)
            s.q = q_new
            n_full += 1
        if w.exchange:
            if margin_hit:
                ladder_ok = False
            if not ladder_ok:
                for o in st.values():
                    o["active"] = False
                break
            Ne = np.array([oracle.count_electrons(st[b]["s"], st[b]["tab"]) for b in range(len(systems))],
                          dtype=np.int32)
            rep, _, E_rep = oracle.remd_exchange(synth.E_LADDER, Ne, rep, T, k % 2, True, ux_all[k])
            assert np.array_equal(sn["rep"], rep), (k, sn["rep"], rep)
            assert np.array_equal(sn["E_rep"], E_rep), k
    return n_full, worst


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eremd_step_sequence_matches_oracle(prec):
    import bench
    systems = synth.eremd_batch()
    _, p_or = params_pair()
    gref = _oracle_gref(systems, p_or, bench.E0_REF, bench.PKA_REF)
    n_steps = 8
    w, snaps = _run_workload(prec, systems, True, n_steps, gref)
    assert not bench_overflow(w)
    n_full, worst = _compare_sequence(prec, w, snaps, list(range(len(systems))),
                                      force_steps=set(range(n_steps)))
    print(prec, "E-REMD steps x replicas compared", n_full, worst)
    # at least five whole steps of all 16 replicas (the FP64 plan: all eight)
    assert n_full >= (len(systems) * n_steps if prec == "fp64" else len(systems) * 5)
    # the chain moved: some attempts were accepted
    assert w.counters[:, 1].sum().item() > 0


def bench_overflow(w):
    return bool(w.g.check_overflow(w.plan))


def _stratified(systems, n_pick=8):
    sizes = np.array([s.n for s in systems])
    order = np.argsort(sizes, kind="stable")
    ranks = np.unique(np.round(np.linspace(0, len(systems) - 1, n_pick)).astype(int))
    return [int(order[r]) for r in ranks]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uneven_batch_step_sequence_matches_oracle(prec):
    import bench
    systems = synth.uneven_batch_64()
    _, p_or = params_pair()
    pick = _stratified(systems)
    sizes = [systems[b].n for b in pick]
    assert min(sizes) == min(s.n for s in systems) and max(sizes) == max(s.n for s in systems)
    # every system at E = E0_ref (no ladder); only the compared systems need
    # oracle reference free energies, the others get zeros (their Monte Carlo
    # moves are never compared)
    gref_parts = []
    for b, s in enumerate(systems):
        if b in pick:
            gref_parts.append(_oracle_gref([s], p_or, bench.E0_REF, bench.PKA_REF))
        else:
            gref_parts.append(np.zeros(sum(site.n_states for site in s.sites)))
    gref = np.concatenate(gref_parts)
    n_steps = 4
    w, snaps = _run_workload(prec, systems, False, n_steps, gref)
    assert not bench_overflow(w)
    n_full, worst = _compare_sequence(prec, w, snaps, pick, force_steps={0, n_steps - 1})
    print(prec, "uneven batch systems", list(zip(pick, sizes)), "system-steps", n_full, worst)
    assert n_full >= (len(pick) * n_steps if prec == "fp64" else len(pick) * 2)
