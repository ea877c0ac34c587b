#!/usr/bin/env python3
"""Benchmark of the GB-OBC + Monte Carlo hot path on one MI355X.

The headline workload is the largest single-GPU configuration: the uneven
batch of 64 systems of 500-20,000 atoms (646,341 atoms, 4.25e9 unordered
pairs), each with 2-10 redox and 0-20 protonation sites.  A step is one pass
of the whole hot path over the batch: Born radii, energy + forces + dE/dq +
dE/drho (with the Born radius chain), Delta E / Delta G of every candidate
state change and one protonation + redox Metropolis attempt per system.  The
Monte Carlo branch (it needs only the radii and the current charges) runs on
a second stream beside the energy / force passes and writes its charge update
into the other of two charge buffers; the step is captured in HIP graphs and
replayed.  The E-REMD batch (16 replicas x 2,500 atoms on a redox-potential
ladder, with a replica-exchange attempt every step) is reported beside it.

Prints ONE JSON line.  Pair interactions/s = sum_b N_b (N_b - 1)/2 per step
divided by the step time.
"""
import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GB pair interactions/s (E+forces) & MC dE evals/s, FP32-fixed vs FP64, 1 GPU"
KB, FARADAY = 1.98720426e-3, 23.0605478
E0_REF, PKA_REF = -0.203, 4.4          # reference compound values of section III.C
E_FIXED = E0_REF                        # redox potential of batches without an E ladder

# Algorithmic work per unordered pair of one full evaluation (FMA = 2; add,
# mul, min, max, select = 1; each reciprocal, sqrt, rsqrt, exp, log, tanh = 1),
# the counts fixed before the first measurement from the closed-form
# expressions: descreening pass 53 flops + 7 transcendentals (both H
# directions sharing r), energy/force pass 50 + 4, chain pass 75 + 5 (both
# dH/dr directions and dH/dS).
FLOPS_PER_PAIR = {"radii_pairs": 60, "energy_pairs": 54, "chain_pairs": 80}
# the persistent launches: the energy and chain passes together, and all three
FLOPS_PER_PAIR["force_pairs"] = FLOPS_PER_PAIR["energy_pairs"] + FLOPS_PER_PAIR["chain_pairs"]
FLOPS_PER_PAIR["evaluate_pairs"] = FLOPS_PER_PAIR["radii_pairs"] + FLOPS_PER_PAIR["force_pairs"]
# Peaks (MI355X, 256 CUs at 2.4 GHz): FP32 vector 157.3 TFLOP/s, FP64 vector
# 78.6 TFLOP/s.  The library's device code has packed-FP32 instructions
# disabled, yet the FP32 value is the attainable one: the FP32 pair kernels
# issue up to 1.5 wave-instructions per SIMD per four cycles (SQ_INSTS_VALU
# over GRBM_GUI_ACTIVE on the 64-system batch), more than a 16-lane issue
# model (78.6 TFLOP/s) allows, so the wider published figure is the ceiling.
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}


# Processing order of the pair passes: compact 64-atom blocks by recursive
# bisection.  More tiles then have their two blocks far enough apart for the
# walk without the per-pair overlap test than in a Morton order (90 % against
# 76 % of the off-diagonal tiles of the 64-system batch), which measured
# 1.5-3 % faster per step on both batches.
DEFAULT_ORDER = "blocks"


def set_atom_order(plan, b, order):
    """Sets the plan's processing order: "blocks" (compact 64-atom blocks),
    "spatial" (Morton) or "identity" (the caller's order)."""
    import paper_1803_09652_amd as g
    if order == "spatial":
        plan.set_order(g.spatial_order(b.atom_offset, b.x, b.y, b.z))
    elif order == "blocks":
        plan.set_order(g.block_order(b.atom_offset, b.x, b.y, b.z))
    elif order != "identity":
        raise ValueError(f"unknown atom order {order!r}")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50,
                    help="timed steps of the headline workload (the 64-system batch)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--kernel-steps", type=int, default=10,
                    help="eager steps / force evaluations timed per kernel with HIP events")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the Monte Carlo branch on the main stream after the force passes "
                         "(by default it runs on a second stream beside them, with "
                         "double-buffered charges)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no E-REMD batch, sweep, salt, dynamics loop, "
                         "cutoff or autograd measurements)")
    ap.add_argument("--only", choices=["headline", "eremd", "single"], default=None,
                    help="run one workload's GPU measurement alone and print its JSON object "
                         "(for profiling it)")
    ap.add_argument("--eremd-steps", type=int, default=200,
                    help="timed steps of the E-REMD batch")
    ap.add_argument("--no-cutoff-bench", action="store_true",
                    help="skip the large-globule cutoff measurement")
    ap.add_argument("--md-steps", type=int, default=100,
                    help="steps of the timed simulation loop (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 64 MiB device copy (reference for HBM counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="also time the headline workload with the work shapes the autotuner "
                         "picks for it (the headline itself uses the library defaults, the "
                         "shapes the committed counters were taken with)")
    ap.add_argument("--order", choices=["spatial", "blocks", "identity"], default=DEFAULT_ORDER,
                    help="processing order of the pair passes (results depend on it only "
                         "through FP32 rounding inside tiles)")
    return ap.parse_args()


def reference_gref(g, plan, b, atoms, cur, pH, E_rep, T, params):
    """Reference free energies of every state (Eqs. 8 and 9): Delta G_elec,ref
    is the Delta E of the starting geometry and states (radii() already run),
    plus the reference compound's E0 / pKa term."""
    import numpy as np
    sites0 = g.Sites.from_batch(plan, b)
    dE0, _ = g.mc_state_dE(plan, sites0, atoms, cur, pH, E_rep, T, params)
    dE0 = dE0.cpu().numpy()
    gref = np.zeros(b.state_count.size)
    c = 0
    for m in range(b.n_sites):
        g0, g1 = int(b.site_state_offset[m]), int(b.site_state_offset[m + 1])
        c0 = int(b.current_state[m])
        ref = FARADAY * E0_REF if b.site_kind[m] == 1 else KB * T * math.log(10) * PKA_REF
        for t in range(g1 - g0):
            if t == c0:
                continue
            gref[g0 + t] = dE0[c] + ref * (b.state_count[g0 + t] - b.state_count[g0 + c0])
            c += 1
    return gref


class Workload:
    """A batch resident on the GPU, with static step buffers: by default the
    E-REMD batch (16 replicas x 2,500 atoms on the E ladder, exchanges between
    neighbouring rungs); with `systems` and exchange=False, any batch of
    distinct systems (each at E_FIXED and pH 7, no exchange)."""

    def __init__(self, precision, n_steps, order=DEFAULT_ORDER, tuning=None, overlap=True,
                 systems=None, exchange=True, gref=None):
        import numpy as np
        import torch
        import paper_1803_09652_amd as g
        import synth
        self.g, self.torch = g, torch
        self.systems = systems if systems is not None else synth.eremd_batch()
        self.exchange = exchange
        self.batch = b = synth.make_batch(self.systems)
        self.B = b.n_systems
        jb, wv = tuning if tuning else (None, None)
        self.plan = g.Plan(b.atom_offset, precision, j_blocks_per_item=jb, waves_per_group=wv)
        set_atom_order(self.plan, b, order)
        self.atoms = g.Atoms.from_batch(self.plan, b)
        dev = self.plan.device
        # with overlap, two charge buffers: a step reads one and writes the
        # Monte Carlo update into the other (even steps A -> B, odd steps
        # B -> A), so the Monte Carlo branch can run on a second stream beside
        # the energy / force passes; without, one buffer updated in place
        self.overlap = overlap
        self.atoms_b = g.Atoms(self.plan, self.atoms.x, self.atoms.y, self.atoms.z,
                               self.atoms.q.clone(), self.atoms.rho,
                               self.atoms.screen) if overlap else self.atoms
        self.side = torch.cuda.Stream(device=dev) if overlap else None
        self.params = g.IGB5
        self.T = 300.0
        self.E_rung = (torch.as_tensor(synth.E_LADDER, dtype=torch.float64, device=dev) if exchange
                       else torch.full((self.B,), E_FIXED, dtype=torch.float64, device=dev))
        self.rep_of_rung = torch.arange(self.B, dtype=torch.int32, device=dev)
        self.E_rep = self.E_rung.clone()                   # replica r starts on rung r
        self.pH = torch.full((self.B,), synth.PH_DEFAULT, dtype=torch.float64, device=dev)
        self.cur = torch.as_tensor(b.current_state, device=dev)
        g.radii(self.plan, self.atoms, self.params)
        if gref is None:
            gref = reference_gref(g, self.plan, b, self.atoms, self.cur, self.pH, self.E_rep,
                                  self.T, self.params)
        self.gref = gref
        self.sites = g.Sites.from_batch(self.plan, b, gref)
        rng = torch.Generator(device=dev)
        rng.manual_seed(2024)
        self.u_all = torch.rand((n_steps, self.B, 6), dtype=torch.float64, device=dev, generator=rng)
        self.ux_all = torch.rand((n_steps, self.B), dtype=torch.float64, device=dev, generator=rng)
        self.u = torch.zeros((self.B, 6), dtype=torch.float64, device=dev)
        self.ux = torch.zeros(self.B, dtype=torch.float64, device=dev)
        # device-side step index: every step (eager or graph replay) gathers
        # its uniforms from row k of the tables and advances k itself (modulo
        # the table length, so an index never leaves the tables)
        self.n_rows = n_steps
        self.k_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.pairs = int(sum(s.n * (s.n - 1) // 2 for s in self.systems))
        self.n_cand = self.sites.n_candidates
        # per-site attempt / acceptance counters, accumulated by the MC kernel
        self.counters = torch.zeros((b.n_sites, 2), dtype=torch.int64, device=dev)

    def step(self, parity):
        """One step; parity alternates from step to step (it selects the
        exchange pairs and the charge buffer read)."""
        g, p, torch = self.g, self.params, self.torch
        cur, nxt = (self.atoms, self.atoms_b) if parity == 0 else (self.atoms_b, self.atoms)
        main = torch.cuda.current_stream()
        mc_stream = self.side if self.overlap else main
        # one full evaluation (inputs staged once); with overlap the Monte
        # Carlo stream is released as soon as the radii are final, and the
        # force passes continue on the radii's stream
        ef = g.evaluate(self.plan, cur, p, fork=mc_stream if mc_stream is not main else None)
        R = ef["R"]
        with torch.cuda.stream(mc_stream):
            # Monte Carlo branch: needs the radii and the current charges only
            torch.index_select(self.u_all, 0, self.k_dev, out=self.u.view(1, self.B, 6))
            torch.index_select(self.ux_all, 0, self.k_dev, out=self.ux.view(1, self.B))
            self.k_dev.add_(1).remainder_(self.n_rows)
            if nxt is not cur:
                nxt.q.copy_(cur.q)
            dE, dG = g.mc_state_dE(self.plan, self.sites, cur, self.cur, self.pH, self.E_rep,
                                   self.T, p)
            mc = g.mc_step(self.plan, self.sites, cur, self.cur, self.pH, self.E_rep, dE, dG,
                           self.u, self.T, p, counters=self.counters, q_out=nxt.q)
            # the exchange needs only the electron counts of the attempt
            # (Eq. 14), so it ends the Monte Carlo branch instead of waiting
            # on the main stream for the join
            if self.exchange:
                acc, _ = g.remd_exchange(self.E_rung, mc["n_electrons"], self.rep_of_rung, parity,
                                         self.ux, self.T, True, E_out=self.E_rep)
                self.last_exchange = acc
            else:
                self.last_exchange = None
        if mc_stream is not main:
            main.wait_stream(mc_stream)
        # the step's outputs (static tensors of a captured graph)
        self.last = {"R": R, "force_out": ef, "dE": dE, "dG": dG, "mc": mc, "q_out": nxt.q}
        return ef



def run_gpu(precision, steps, warmup, use_graph, kernel_steps, order=DEFAULT_ORDER, tuning=None,
            overlap=True, systems=None, exchange=True):
    import torch
    n_total = steps + warmup + kernel_steps + 2
    w = Workload(precision, n_total, order, tuning, overlap, systems, exchange)
    torch.cuda.synchronize()
    k = 0       # steps done so far; step k has exchange parity k % 2
    graphs = None
    if use_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for parity in (0, 1):
                w.step(parity)
                k += 1
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graphs = []
        for parity in (0, 1):
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                w.step(parity)
            graphs.append(gr)

    def one():
        nonlocal k
        if graphs is not None:
            graphs[k % 2].replay()
        else:
            w.step(k % 2)
        k += 1

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        one()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / steps
    # run-to-run spread: further steps, each bracketed by its own events
    # (the rate above is the mean over the back-to-back timed region)
    n_spread = min(50, steps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n_spread)]
    for a, b in evs:
        a.record()
        one()
        b.record()
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in evs)
    w.step_spread = ({"reps": n_spread, "median": per[n_spread // 2],
                      "p10": per[n_spread // 10], "p90": per[(9 * n_spread) // 10],
                      "min": per[0], "max": per[-1]} if n_spread else None)
    # per-kernel durations: eager steps on this stream, each hot-path kernel
    # launched with HIP start/stop events bound to its dispatch
    # (back to back, no host synchronisation until the read, like the timed
    # region), read once as the mean per launch
    w.plan.set_timing(True)
    acc = torch.zeros((), dtype=torch.int64, device=w.plan.device)
    for _ in range(kernel_steps):
        w.step(k % 2)
        k += 1
        if w.last_exchange is not None:
            acc += w.last_exchange.sum()
    kernel_ms = w.plan.kernel_ms() if kernel_steps > 0 else {}
    # the Monte Carlo Delta E kernels on their own (no concurrent force passes)
    cur = w.atoms if k % 2 == 0 else w.atoms_b
    w.latest = cur                     # the buffer holding the current charges
    for _ in range(max(1, kernel_steps // 2)):
        w.g.mc_state_dE(w.plan, w.sites, cur, w.cur, w.pH, w.E_rep, w.T, w.params)
    w.mc_alone_ms = w.plan.kernel_ms()
    # the force passes on their own (radii + energy / forces / dE/dq / dE/drho,
    # nothing else on the GPU): each pair kernel's own duration, the one the
    # roofline is quoted on
    for _ in range(kernel_steps):
        w.g.radii(w.plan, cur, w.params)
        w.g.energy_forces(w.plan, cur, w.params)
    w.force_alone_ms = w.plan.kernel_ms() if kernel_steps > 0 else {}
    w.plan.set_timing(False)
    w.exchanges_accepted = int(acc)
    w.exchanges_attempted = (kernel_steps * int(w.last_exchange.numel())
                             if kernel_steps and w.last_exchange is not None else 0)
    return w, ms_step, wall / steps * 1e3, kernel_ms


def time_sweep(w, reps=20):
    """Sequential all-site sweeps (mc_sweep) on the batch: every site of every
    replica attempted once per sweep (potential rows, then one workgroup per
    replica), timed with HIP events over back-to-back calls.  Acceptances are
    counted by the kernel itself (counters), so the timed loop holds nothing
    but the sweeps."""
    import torch
    g, dev = w.g, w.plan.device
    n_sites = w.sites.n_sites
    cur = w.latest
    g.radii(w.plan, cur, w.params)
    state = w.cur.clone()
    counters = torch.zeros((n_sites, 2), dtype=torch.int64, device=dev)
    rng = torch.Generator(device=dev)
    rng.manual_seed(99)
    u = torch.rand((reps + 2, n_sites, 3), dtype=torch.float64, device=dev, generator=rng)
    for k in range(2):
        g.mc_sweep(w.plan, w.sites, cur, state, w.pH, w.E_rep, u[k], w.T, w.params,
                   counters=counters)
    counters.zero_()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(reps):
        g.mc_sweep(w.plan, w.sites, cur, state, w.pH, w.E_rep, u[k + 2], w.T, w.params,
                   counters=counters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tot = counters.sum(0).cpu().tolist()
    return {"ms_per_sweep": ms, "site_attempts_per_s": n_sites / (ms * 1e-3),
            "sites_per_sweep": n_sites, "sweeps": reps,
            "acceptance": tot[1] / max(1, tot[0])}


def time_salt(w, kappa=0.1, steps=20):
    """The force passes with salt (kappa = 0.1 / A, about 0.1 M) beside the
    same passes without: radii and energy / forces of the batch, eager,
    per-kernel means from the timing hook (no Monte Carlo branch sharing the
    GPU, so the means are below those of the full step)."""
    import dataclasses
    g, plan = w.g, w.plan
    atoms = w.latest
    res = {}
    for kap in (0.0, kappa):
        p = dataclasses.replace(w.params, kappa=kap)
        g.radii(plan, atoms, p)
        g.energy_forces(plan, atoms, p)
        w.torch.cuda.synchronize()
        plan.set_timing(True)
        plan.kernel_ms()
        for _ in range(steps):
            g.radii(plan, atoms, p)
            g.energy_forces(plan, atoms, p)
        w.torch.cuda.synchronize()
        ms = plan.kernel_ms()
        plan.set_timing(False)
        res[kap] = {k: v for k, v in ms.items() if k in ("radii_pairs", "energy_pairs", "chain_pairs")}
    salt, base = res[kappa], res[0.0]
    return {"kappa_per_A": kappa, "kernel_ms": salt, "kernel_ms_no_salt": base,
            "energy_pairs_salt_over_no_salt": salt["energy_pairs"] / base["energy_pairs"],
            "pair_interactions_per_s_force_passes": w.pairs / (sum(salt.values()) * 1e-3)}


def time_cutoff(n_atoms=100000, rgbmax=15.0, cutoff=16.0, steps=10):
    """Force evaluations (radii + energy / forces / dE/dq / dE/drho) of one
    large globule with the descreening and pair cutoffs, against the same
    evaluation over all pairs: per-kernel means from the timing hook and the
    whole evaluation from HIP events.  Atoms in compact 64-atom blocks
    (block_order), library default work shapes."""
    import dataclasses
    import torch
    import paper_1803_09652_amd as g
    import synth
    from scipy.spatial import cKDTree
    s = synth.make_system(140, n_atoms, 18.0 * (n_atoms / 2500.0) ** (1 / 3))
    b = synth.make_batch([s])
    plan = g.Plan(b.atom_offset, "fp32")
    plan.set_order(g.block_order(b.atom_offset, b.x, b.y, b.z))
    atoms = g.Atoms.from_batch(plan, b)
    out = {"workload": f"one {n_atoms}-atom globule, FP32 plan, rgbmax {rgbmax} A, pair cutoff "
                       f"{cutoff} A, compact-block order"}
    for name, p, n in (("cutoff", dataclasses.replace(g.IGB5, rgbmax=rgbmax, cutoff=cutoff), steps),
                       ("all_pairs", g.IGB5, 2)):
        g.radii(plan, atoms, p)
        g.energy_forces(plan, atoms, p)
        torch.cuda.synchronize()
        plan.set_timing(True)
        plan.kernel_ms()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            g.radii(plan, atoms, p)
            g.energy_forces(plan, atoms, p)
        e1.record()
        torch.cuda.synchronize()
        kms = plan.kernel_ms()
        plan.set_timing(False)
        out[name] = {"ms_per_evaluation": e0.elapsed_time(e1) / n,
                     "kernel_ms": {k: v for k, v in kms.items()
                                   if k in ("radii_pairs", "energy_pairs", "chain_pairs")}}
    out["overflow"] = bool(g.check_overflow(plan))
    t = cKDTree(s.coords())
    within = (t.count_neighbors(t, cutoff) - s.n) // 2
    out["pairs_within_cutoff"] = int(within)
    out["pairs_all"] = s.n * (s.n - 1) // 2
    out["speedup"] = out["all_pairs"]["ms_per_evaluation"] / out["cutoff"]["ms_per_evaluation"]
    out["pairs_within_cutoff_per_s"] = within / (out["cutoff"]["ms_per_evaluation"] * 1e-3)
    return out


def time_plain_fp64(w, reps=3):
    """The plain FP64 GPU form (gb_plain_fp64: one thread per atom over its
    whole row, closed forms, correctly rounded operations) of one full
    evaluation of the workload's batch, timed with HIP events: the reference
    the metric's FP32-fixed vs FP64 comparison names."""
    import torch
    g, b = w.g, w.batch
    dev = w.plan.device
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    args = (b.atom_offset, d(b.x), d(b.y), d(b.z), d(b.q), d(b.rho), d(b.screen), w.params)
    g.plain_fp64(*args)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.plain_fp64(*args)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_per_evaluation": ms, "value": w.pairs / (ms * 1e-3), "reps": reps,
            "form": "radii + energy + forces + dE/dq + dE/drho, every ordered pair, FP64"}


def time_single_launch(systems, reps=5, precision="fp32", order=DEFAULT_ORDER):
    """One full evaluation (radii, energy, forces, dE/dq, dE/drho) of the
    batch as gb_evaluate's single queued launch (all three pair passes, with
    per-block dependency counters), beside gb_radii + gb_energy_forces (one
    launch per pass), eager, on the same plan and inputs: HIP events around
    each evaluation, and the timing hook's per-kernel means."""
    import torch
    import paper_1803_09652_amd as g
    import synth
    b = synth.make_batch(systems)
    plan = g.Plan(b.atom_offset, precision)
    set_atom_order(plan, b, order)
    atoms = g.Atoms.from_batch(plan, b)
    pairs = pair_count(systems)

    def single():
        plan.set_single_launch(True)
        g.evaluate(plan, atoms, g.IGB5)

    def separate():
        plan.set_single_launch(False)
        g.radii(plan, atoms, g.IGB5)
        g.energy_forces(plan, atoms, g.IGB5)

    out = {"pairs": pairs}
    for name, fn in (("single_launch", single), ("separate_launches", separate)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        plan.set_timing(True)
        plan.kernel_ms()
        for _ in range(reps):
            fn()
        kms = plan.kernel_ms()
        plan.set_timing(False)
        out[name] = {"ms_per_evaluation": ms, "pair_interactions_per_s": pairs / (ms * 1e-3),
                     "kernel_ms": kms, "overflow_or_wait_error": bool(g.check_overflow(plan))}
    ev = out["single_launch"]["kernel_ms"].get("evaluate_pairs")
    if ev:
        ach = FLOPS_PER_PAIR["evaluate_pairs"] * pairs / (ev * 1e-3) / 1e12
        out["single_launch"]["tflops"] = ach
        out["single_launch"]["frac_of_fp32_peak"] = ach / PEAK_TFLOPS["fp32"]
    return out


def copy_calibration():
    """A plain streaming kernel of known size (64 MiB read, 64 MiB written;
    torch's elementwise negation, easy to find by name in the counter output):
    FETCH_SIZE / WRITE_SIZE of these dispatches calibrate the HBM byte
    counters of the pair kernels."""
    import torch
    n = 16 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b
    return {"kernel": "neg", "bytes_read": 4 * n, "bytes_written": 4 * n, "dispatches": 3}


def pair_count(systems):
    return int(sum(s_.n * (s_.n - 1) // 2 for s_ in systems))


def roofline_of(pairs, kernel_ms, traffic=None, traffic_detail=None):
    """FP32 VALU roofline of the dominant pair kernel: algorithmic flops per
    launch (per-pair count x unordered pairs) over its mean duration per
    launch."""
    pair_k = {n: kernel_ms[n] for n in FLOPS_PER_PAIR if n in kernel_ms}
    if not pair_k:
        return None
    dom = max(pair_k, key=pair_k.get)
    ach = FLOPS_PER_PAIR[dom] * pairs / (pair_k[dom] * 1e-3) / 1e12
    return {"bound": "alu", "kernel": dom, "achieved": ach,
            "measured_as": "mean duration per launch of the force passes alone (eager, HIP "
                           "events bound to the dispatches, on the launch stream)",
            "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["fp32"],
            "traffic": traffic, "traffic_detail": traffic_detail,
            "flops_per_pair": FLOPS_PER_PAIR[dom], "pairs_per_launch": pairs,
            "per_kernel_tflops": {n: FLOPS_PER_PAIR[n] * pairs / (v * 1e-3) / 1e12
                                  for n, v in pair_k.items()},
            "per_kernel_frac": {n: FLOPS_PER_PAIR[n] * pairs / (v * 1e-3) / 1e12
                                / PEAK_TFLOPS["fp32"] for n, v in pair_k.items()}}


def measure_workload(systems, exchange, steps, warmup, kernel_steps, use_graph=True,
                     order=DEFAULT_ORDER, tuning=None, overlap=True, precision="fp32"):
    """The step of one workload (captured and replayed), the per-kernel means
    inside the step, the Monte Carlo Delta E kernels alone and the force
    passes alone."""
    import torch
    pairs = pair_count(systems)
    w, ms, wall, kms = run_gpu(precision, steps, warmup, use_graph, kernel_steps, order, tuning,
                               overlap, systems=systems, exchange=exchange)
    g = w.g
    out = {"ms_per_step": ms, "pair_interactions_per_s": pairs / (ms * 1e-3),
           "mc_dE_evals_per_s": w.n_cand / (ms * 1e-3), "steps": steps,
           "wall_ms_per_step": wall, "ms_per_step_spread": w.step_spread,
           "pairs_per_step": pairs, "candidates_per_step": w.n_cand,
           "kernel_ms_in_step": kms, "kernel_ms_force_passes_alone": w.force_alone_ms,
           "overflow": bool(g.check_overflow(w.plan))}
    alone = w.mc_alone_ms
    if "site_rows" in alone or "site_dE" in alone:
        t_mc = alone.get("site_rows", 0.0) + alone.get("site_dE", 0.0)
        out["mc_dE_evals_per_s_standalone"] = w.n_cand / (t_mc * 1e-3)
        out["mc_kernel_ms_standalone"] = {k_: alone[k_] for k_ in ("site_rows", "site_dE")
                                          if k_ in alone}
    if w.exchange:
        out["exchange_attempts_eager"] = w.exchanges_attempted
        out["exchange_accepted_eager"] = w.exchanges_accepted
    cnt = w.counters.sum(0).cpu().tolist()
    out["mc_state_attempts"], out["mc_state_accepted"] = cnt[0], cnt[1]
    torch.cuda.synchronize()
    return out, w


def time_md_loop(steps, warmup, n_rep=16, attempt_every=5, exchange_every=10):
    """The simulation loop (ReplicaMD) on the E-REMD batch for dynamics: 16
    replicas x 2,500 atoms, 2 fs Langevin steps (gamma 5 / ps, every atom
    restrained), a Monte Carlo attempt pair every 5 steps (10 fs, the
    implicit-solvent attempt interval of section III.D) and an exchange
    attempt every 10 steps (20 fs: EAF 50 / ps, the highest of section III.D).  Every
    step is radii + energy / forces + Langevin update; timed with HIP events
    over `steps` eager steps after `warmup`."""
    import numpy as np
    import torch
    import paper_1803_09652_amd as g
    import synth
    from paper_1803_09652_amd.runtime import ReplicaMD
    systems = synth.eremd_batch_md(n_rep)
    b = synth.make_batch(systems)
    plan = g.Plan(b.atom_offset, "fp32")
    set_atom_order(plan, b, DEFAULT_ORDER)
    atoms = g.Atoms.from_batch(plan, b)
    dev, T, params = plan.device, 300.0, g.IGB5
    E_rung = np.array(synth.E_LADDER[:n_rep])
    cur = torch.as_tensor(b.current_state, device=dev)
    pH = torch.full((n_rep,), synth.PH_DEFAULT, dtype=torch.float64, device=dev)
    g.radii(plan, atoms, params)
    gref = reference_gref(g, plan, b, atoms, cur, pH, torch.as_tensor(E_rung, device=dev), T, params)
    sites = g.Sites.from_batch(plan, b, gref)
    m = synth.masses(3, b.n_atoms)
    loop = ReplicaMD(plan, sites, atoms, b.current_state, 1.0 / m,
                     synth.thermal_velocities(4, m, T).T, synth.PH_DEFAULT, E_rung, dt=0.002,
                     gamma=5.0, T=T, attempt_every=attempt_every, exchange_every=exchange_every,
                     params=params, xref=np.stack([b.x, b.y, b.z]), k_restr=synth.MD_RESTRAINT,
                     seed=6)
    loop.run(warmup, record=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    loop.run(steps, record=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    cnt = loop.counters.sum(0).cpu().tolist()
    ns_day = 0.002 * 86400.0 / (ms * 1e-3) / 1000.0     # ns of one replica per day
    return {"workload": f"{n_rep} replicas x {b.n_atoms // n_rep} atoms, dt 2 fs, attempt every "
                        f"{attempt_every} steps, exchange every {exchange_every} steps",
            "ms_per_md_step": ms, "wall_ms_per_md_step": wall / steps * 1e3, "steps": steps,
            "ns_per_day_per_replica": ns_day, "ns_per_day_all_replicas": ns_day * n_rep,
            "pair_interactions_per_s": sum(s.n * (s.n - 1) // 2 for s in systems) / (ms * 1e-3),
            "state_attempts": cnt[0], "state_accepted": cnt[1],
            "exchange_pairs_accepted": loop.exchanges_accepted,
            "overflow": bool(g.check_overflow(plan))}


def host_cpu():
    """CPU model of the host (lscpu, else /proc/cpuinfo), the family / model /
    stepping numbers and clock that identify it where the name is generic (a
    virtual machine's), and its core count."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for l in txt.splitlines():
            if ":" in l:
                k, v = l.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    model = info.get("Model name")
    if not model:
        try:
            with open("/proc/cpuinfo") as f:
                model = next((l.split(":", 1)[1].strip() for l in f
                              if l.startswith("model name")), None)
        except OSError:
            pass
    out = {"cpu_model": model, "nproc": os.cpu_count(),
           "threads_allowed": len(os.sched_getaffinity(0))}
    for key, name in (("CPU family", "cpu_family"), ("Model", "cpu_model_number"),
                      ("Stepping", "cpu_stepping"), ("CPU max MHz", "cpu_max_mhz"),
                      ("BogoMIPS", "bogomips"), ("Hypervisor vendor", "hypervisor")):
        if key in info:
            out[name] = info[key]
    return out


def stratified_sample(systems, n_pick=8):
    """Indices of n_pick systems at evenly spaced size ranks (the smallest and
    the largest included)."""
    import numpy as np
    sizes = np.array([s_.n for s_ in systems])
    order = np.argsort(sizes, kind="stable")
    ranks = np.unique(np.round(np.linspace(0, len(systems) - 1, n_pick)).astype(int))
    return [int(order[r]) for r in ranks]


def cpu_baseline(systems, label):
    """The FP64 oracle as it stands, on the host cores: one full evaluation
    (radii, energy, forces, dE/dq, dE/drho and every candidate Delta E) of each
    system of a bounded sample of the workload, pair interactions per second
    over the whole sample."""
    import oracle
    oracle.lib()
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    pairs = pair_count(systems)
    t0 = time.perf_counter()
    for s_ in systems:
        r = oracle.energy_forces(s_)
        if s_.sites:
            oracle.site_dE(s_, r["R"])
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"{label}: one full evaluation each ({pairs} pairs): radii, energy, forces, "
                      f"dE/dq, dE/drho and every candidate Delta E, FP64, OpenMP on {cores} "
                      f"threads, {dt:.1f} s wall (~{dt * cores:.0f} core-s)",
            **host_cpu()}


def cpu_oracle_detail(reps=3):
    """The oracle on the host at the single-system sizes: one full evaluation
    (radii, energy, forces, dE/dq, dE/drho; plus every candidate Delta E where
    the system has sites) of the 256-, 2,500- and 10,000-atom systems, single
    threaded and with OpenMP on every core, median of `reps` (one rep for the
    10,000-atom system single threaded), with the host's core count and CPU
    model."""
    import ctypes
    import statistics
    import oracle
    import synth
    oracle.lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    n_all = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    out = {"kind": "oracle", "unit": "pair interactions/s", "threads_all": n_all,
           **host_cpu(), "systems": {}}
    for name, sys_ in (("256 atoms", synth.globule_256()[0]), ("2500 atoms", synth.globule_2500()[0]),
                       ("10000 atoms", synth.globule_10000()[0])):
        pairs = sys_.n * (sys_.n - 1) // 2
        res = {}
        for label, nt in (("single_thread", 1), ("all_threads", n_all)):
            gomp.omp_set_num_threads(nt)
            k = 1 if (nt == 1 and sys_.n > 5000) else reps
            ts = []
            for _ in range(k):
                t0 = time.perf_counter()
                r = oracle.energy_forces(sys_)
                if sys_.sites:
                    oracle.site_dE(sys_, r["R"])
                ts.append(time.perf_counter() - t0)
            res[label] = {"value": pairs / statistics.median(ts), "reps": k,
                          "median_s": statistics.median(ts)}
        out["systems"][name] = res
    gomp.omp_set_num_threads(n_all)
    return out


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "hbm_counters_pair_kernels_uneven_64.md")
EREMD_COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "hbm_counters_pair_kernels_ereMD_16x2500.md")


def time_autograd(reps=10):
    """GBEnergy (torch.autograd.Function) on the 10,000-atom globule, FP32
    plan: forward (radii + energy-only pass) and backward (the gradient passes
    on the radius state forward kept) timed separately with HIP events, and
    the pair kernels each phase launched, from the timing hook."""
    import numpy as np
    import torch
    import paper_1803_09652_amd as g
    import synth
    s_ = synth.globule_10000()[0]
    b = synth.make_batch([s_])
    plan = g.Plan(b.atom_offset, "fp32")
    set_atom_order(plan, b, DEFAULT_ORDER)
    dev = plan.device
    t = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float32, device=dev)
    pos = t(np.stack([b.x, b.y, b.z], axis=1)).requires_grad_(True)
    q, rho, scr = t(b.q).requires_grad_(True), t(b.rho).requires_grad_(True), t(b.screen)
    for _ in range(2):
        g.GBEnergy.apply(pos, q, rho, scr, plan, g.IGB5).sum().backward()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1, e2 in ev:
        e0.record()
        E = g.GBEnergy.apply(pos, q, rho, scr, plan, g.IGB5)
        e1.record()
        E.sum().backward()
        e2.record()
    torch.cuda.synchronize()
    fwd = sorted(a.elapsed_time(b_) for a, b_, _ in ev)[reps // 2]
    bwd = sorted(b_.elapsed_time(c) for _, b_, c in ev)[reps // 2]
    plan.set_timing(True)
    E = g.GBEnergy.apply(pos, q, rho, scr, plan, g.IGB5)
    torch.cuda.synchronize()
    k_fwd = plan.kernel_ms()
    E.sum().backward()
    torch.cuda.synchronize()
    k_bwd = plan.kernel_ms()
    plan.set_timing(False)
    return {"workload": "one 10000-atom globule (26 A), FP32 plan, dE/dx, dE/dq, dE/drho",
            "forward_ms": fwd, "backward_ms": bwd, "reps": reps,
            "forward_kernel_ms": k_fwd, "backward_kernel_ms": k_bwd,
            "backward_pair_kernels_ms": sum(v for k_, v in k_bwd.items()
                                            if k_ in ("energy_pairs", "chain_pairs"))}


def kernel_source_hash():
    """SHA-256 over the library sources: the counter summary records it, and
    counters taken from other kernels are not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_09652_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*"))):
        if f.endswith((".hip", ".h", ".inc", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def traffic_from_counters(kernel, path=COUNTER_SUMMARY, order=DEFAULT_ORDER):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, each scaled by
    what the counter reads for a plain copy of known size), from the committed
    rocprofv3 summary; None when absent, taken from other kernel sources or
    taken in another atom order than the one timed."""
    try:
        with open(path) as f:
            lines = [l for l in f if l.startswith("traffic-record: ")]
        rec = json.loads(lines[-1][len("traffic-record: "):])
    except (OSError, IndexError, ValueError):
        return None, "no counter summary"
    if rec.get("source_sha256") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    if rec.get("atom_order") != order:
        return None, f"counters taken in another atom order ({rec.get('atom_order')})"
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None, f"no counters for {kernel}"
    return k["fetch_bytes"] + k["write_bytes"], {
        "fetch_bytes": k["fetch_bytes"], "write_bytes": k["write_bytes"],
        "fetch_factor": rec["fetch_factor"], "write_factor": rec["write_factor"],
        "source": os.path.relpath(path, ROOT)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "the batch shards by system across GPUs in principle, but the benchmark "
              "measures the single-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    torch.cuda.set_device(0)
    use_graph, overlap = not args.no_graph, not args.no_overlap
    run = dict(use_graph=use_graph, order=args.order, overlap=overlap)
    copy_ref = copy_calibration() if args.copy_calibration else None
    if args.only == "headline":
        r, _ = measure_workload(synth.uneven_batch_64(), False, args.steps, args.warmup,
                                args.kernel_steps, **run)
        if copy_ref is not None:
            r["copy_calibration"] = copy_ref
        print(json.dumps(r), flush=True)
        return
    if args.only == "single":
        print(json.dumps({"uneven_batch": time_single_launch(synth.uneven_batch_64(), reps=3,
                                                            order=args.order),
                          "eremd_batch": time_single_launch(synth.eremd_batch(), reps=20,
                                                            order=args.order)}),
              flush=True)
        return
    if args.only == "eremd":
        r, _ = measure_workload(synth.eremd_batch(), True, args.eremd_steps, args.warmup,
                                args.kernel_steps, **run)
        if copy_ref is not None:
            r["copy_calibration"] = copy_ref
        print(json.dumps(r), flush=True)
        return
    # ---- headline: the uneven 64-system batch, FP32-fixed, library default shapes
    systems = synth.uneven_batch_64()
    head, w = measure_workload(systems, False, args.steps, args.warmup, args.kernel_steps, **run)
    pairs, ms_step = head["pairs_per_step"], head["ms_per_step"]
    value = pairs / (ms_step * 1e-3)
    sizes = [s_.n for s_ in systems]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"uneven batch: {len(systems)} protein-like globules of {min(sizes)}-"
                        f"{max(sizes)} atoms ({sum(sizes)} in all), 2-10 redox + 0-20 "
                        "protonation sites each, E = E0_ref, pH 7, T 300 K, igb=5, no cutoff",
            "systems": len(systems), "atoms": sum(sizes), "pairs_per_step": pairs,
            "candidates_per_step": head["candidates_per_step"], "hip_graph": use_graph,
            "atom_order": args.order,
            "mc_branch": "second stream beside the force passes" if overlap
                         else "after the force passes",
            "tuning": "library default",
            "precision": "FP32 pair arithmetic, int64 fixed-point sums, FP64 MC",
        },
        "mc_dE_evals_per_s": head["mc_dE_evals_per_s"],
    }
    for k_ in ("wall_ms_per_step", "ms_per_step_spread", "kernel_ms_in_step",
               "kernel_ms_force_passes_alone", "mc_dE_evals_per_s_standalone",
               "mc_kernel_ms_standalone", "mc_state_attempts", "mc_state_accepted", "overflow"):
        if k_ in head:
            out[k_] = head[k_]
    force_alone = head["kernel_ms_force_passes_alone"]
    dom_rf = roofline_of(pairs, force_alone)
    traffic, detail = (traffic_from_counters(dom_rf["kernel"], order=args.order) if dom_rf
                       else (None, None))
    out["roofline"] = roofline_of(pairs, force_alone, traffic, detail)
    out["fp64_plain"] = time_plain_fp64(w, reps=1)
    out["fp32_over_fp64_plain"] = value / out["fp64_plain"]["value"]
    del w
    torch.cuda.empty_cache()
    out["single_launch"] = time_single_launch(systems, reps=3, order=args.order)
    if not args.no_fp64:
        r64, w64 = measure_workload(systems, False, args.fp64_steps, 2, 1, precision="fp64", **run)
        out["fp64"] = {k_: r64[k_] for k_ in ("ms_per_step", "pair_interactions_per_s",
                                              "mc_dE_evals_per_s", "steps", "kernel_ms_in_step",
                                              "overflow")}
        out["fp64"]["value"] = r64["pair_interactions_per_s"]
        out["fp32_over_fp64"] = value / r64["pair_interactions_per_s"]
        del w64
        torch.cuda.empty_cache()
    if args.autotune:
        from paper_1803_09652_amd import autotune as at
        import paper_1803_09652_amd as g
        b = synth.make_batch(systems)
        ords = {"spatial": g.spatial_order, "blocks": g.block_order}
        tn = at.tune(b, "fp32", order=(ords[args.order](b.atom_offset, b.x, b.y, b.z)
                                       if args.order in ords else None),
                     use_cache=False)
        rt, wt = measure_workload(systems, False, args.steps, args.warmup, 1,
                                  tuning=tn["best"], **run)
        out["fp32_autotuned"] = {"ms_per_step": rt["ms_per_step"],
                                 "pair_interactions_per_s": rt["pair_interactions_per_s"],
                                 "j_blocks_per_item": list(tn["best"][0]),
                                 "waves_per_group": list(tn["best"][1])}
        del wt
        torch.cuda.empty_cache()

    # ---- beside it: the E-REMD batch (16 x 2,500 atoms, exchange every step)
    if not args.no_extras:
        er, we = measure_workload(synth.eremd_batch(), True, args.eremd_steps, args.warmup,
                                  max(args.kernel_steps, 20), **run)
        er["workload"] = ("E-REMD batch: 16 replicas x 2500 atoms (18 A globules), 4 redox + 4 "
                          "protonation sites each, E ladder -0.40..-0.10 V, pH 7, T 300 K, "
                          "exchange attempt every step")
        er_dom = roofline_of(er["pairs_per_step"], er["kernel_ms_force_passes_alone"])
        er_t, er_d = (traffic_from_counters(er_dom["kernel"], EREMD_COUNTER_SUMMARY, args.order)
                      if er_dom
                      else (None, None))
        er["roofline"] = roofline_of(er["pairs_per_step"], er["kernel_ms_force_passes_alone"],
                                     er_t, er_d)
        er["fp64_plain"] = time_plain_fp64(we, reps=2)
        er["fp32_over_fp64_plain"] = er["pair_interactions_per_s"] / er["fp64_plain"]["value"]
        er["single_launch"] = time_single_launch(synth.eremd_batch(), reps=20, order=args.order)
        er["mc_sweep"] = time_sweep(we)
        er["salt"] = time_salt(we)
        del we
        torch.cuda.empty_cache()
        if not args.no_fp64:
            e64, w64 = measure_workload(synth.eremd_batch(), True, 20, 2, 1, precision="fp64",
                                        **run)
            er["fp64"] = {"ms_per_step": e64["ms_per_step"],
                          "value": e64["pair_interactions_per_s"]}
            er["fp32_over_fp64"] = er["pair_interactions_per_s"] / e64["pair_interactions_per_s"]
            del w64
        out["eremd_batch"] = er
        out["autograd"] = time_autograd()
        if args.md_steps > 0:
            out["md_loop"] = time_md_loop(args.md_steps, 10)
        if not args.no_cutoff_bench:
            out["cutoff"] = time_cutoff()
    if copy_ref is not None:
        out["copy_calibration"] = copy_ref
    if not args.no_cpu_baseline:
        pick = stratified_sample(systems)
        out["cpu_baseline"] = cpu_baseline(
            [systems[k_] for k_ in pick],
            f"the {len(pick)} systems of the uneven batch at evenly spaced size ranks "
            f"({', '.join(str(systems[k_].n) for k_ in pick)} atoms)")
        if not args.no_extras:
            out["cpu_oracle_detail"] = cpu_oracle_detail()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
