"""GPU parity of gb_radii / gb_energy_forces (C ABI) against the FP64 oracle.

Sizes span several 64-atom tiles and ragged tails; batches mix uneven and
empty systems; the full-size workloads run in the launch configuration of the
benchmark and are compared on every atom of selected systems.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import TOL, build, compare_system, gpu_eval, oracle_eval, params_pair, rel_inf

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp64"]


def _sys(seed, n, r=None, **kw):
    r = r if r is not None else max(4.0, 18.0 * (n / 2500.0) ** (1 / 3))
    return synth.make_system(seed, n, r, **kw)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("pname", ["IGB5", "IGB2"])
def test_globule_256_parity(prec, pname):
    p_gpu, p_or = params_pair(pname)
    systems = synth.globule_256()
    g, batch, plan, atoms = build(systems, prec)
    res = gpu_eval(plan, atoms, p_gpu)
    ref = oracle_eval(systems[0], p_or, ("c0", pname))
    errs = compare_system(res, 0, batch.atom_offset, ref, prec)
    print(prec, pname, errs)


@pytest.mark.parametrize("prec", PRECS)
def test_globule_2500_parity(prec):
    p_gpu, p_or = params_pair()
    systems = synth.globule_2500()
    g, batch, plan, atoms = build(systems, prec)
    res = gpu_eval(plan, atoms, p_gpu)
    ref = oracle_eval(systems[0], p_or, ("c1", "IGB5"))
    print(prec, compare_system(res, 0, batch.atom_offset, ref, prec))


@pytest.mark.parametrize("prec", PRECS)
def test_ragged_and_degenerate_sizes(prec):
    # 1 atom (Born ion), 2 atoms, one tile minus/plus one, several tiles with a
    # ragged tail, and an empty system in the middle of the batch
    p_gpu, p_or = params_pair()
    sizes = [1, 2, 63, 64, 65, 0, 130, 200]
    systems = [_sys(100 + k, n) if n > 0 else synth.System(*(np.zeros(0),) * 6)
               for k, n in enumerate(sizes)]
    g, batch, plan, atoms = build(systems, prec)
    res = gpu_eval(plan, atoms, p_gpu)
    for b, s in enumerate(systems):
        ref = oracle_eval(s, p_or) if s.n > 0 else None
        compare_system(res, b, batch.atom_offset, ref, prec)


def test_engulfed_and_overlapping_pairs():
    # close contacts (0.3-0.6 A) with large screened radii exercise every branch
    # of the HCT integral and its derivatives in both precisions
    p_gpu, p_or = params_pair()
    s = synth.make_system(7, 150, 6.0, min_dist=0.3)
    s.rho = synth.f32(np.random.default_rng(1).uniform(0.8, 2.6, s.n))
    s.screen = synth.f32(np.random.default_rng(2).uniform(0.6, 0.99, s.n))
    ref = oracle_eval(s, p_or)
    for prec in PRECS:
        g, batch, plan, atoms = build([s], prec)
        res = gpu_eval(plan, atoms, p_gpu)
        print(prec, compare_system(res, 0, batch.atom_offset, ref, prec))


@pytest.mark.parametrize("prec", PRECS)
def test_eremd_batch_all_replicas(prec):
    # the E-REMD batch (16 x 2500) in the benchmark's launch configuration
    p_gpu, p_or = params_pair()
    systems = synth.eremd_batch()
    g, batch, plan, atoms = build(systems, prec)
    res = gpu_eval(plan, atoms, p_gpu)
    worst = {}
    for b, s in enumerate(systems):
        e = compare_system(res, b, batch.atom_offset, oracle_eval(s, p_or, ("c2", b)), prec)
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    print(prec, worst)


def test_fp32_bitwise_deterministic_and_shape_independent():
    p_gpu, _ = params_pair()
    systems = [_sys(11, 700), _sys(12, 333)]
    outs = []
    for jb, wv in ((8, 4), (8, 4), (1, 1), (3, 2), (64, 8), ((1, 8, 2), (2, 1, 4))):
        g, batch, plan, atoms = build(systems, "fp32", j_blocks=jb, waves=wv)
        outs.append(gpu_eval(plan, atoms, p_gpu))
    for o in outs[1:]:
        for k in ("R", "Ec", "Egb", "force", "dEdq", "dEdrho"):
            assert np.array_equal(o[k], outs[0][k]), k


@pytest.mark.parametrize("prec", PRECS)
def test_overlap_heavy_tiles_shape_independent(prec):
    # nearly every pair overlaps (150 atoms within 6 A, large screened radii):
    # the deferred pairs fill several packed rounds per tile, and the result
    # must not depend on the work shape (items of one or many tiles, waves per
    # group) and must match the oracle
    p_gpu, p_or = params_pair()
    s = synth.make_system(7, 150, 6.0, min_dist=0.3)
    s.rho = synth.f32(np.random.default_rng(1).uniform(0.8, 2.6, s.n))
    s.screen = synth.f32(np.random.default_rng(2).uniform(0.6, 0.99, s.n))
    dense = synth.make_system(8, 900, 9.0, min_dist=0.6)
    outs = []
    for jb, wv in ((1, 1), (8, 4), (2, 8)):
        g, batch, plan, atoms = build([s, dense], prec, j_blocks=jb, waves=wv)
        outs.append(gpu_eval(plan, atoms, p_gpu))
    for o in outs[1:]:
        for k in ("R", "Ec", "Egb", "force", "dEdq", "dEdrho"):
            assert np.array_equal(o[k], outs[0][k]), k
    ref = oracle_eval(s, p_or)
    print(prec, compare_system(outs[0], 0, batch.atom_offset, ref, prec))


def test_batch_equals_single_systems_bitwise():
    p_gpu, _ = params_pair()
    systems = [_sys(21, 90), _sys(22, 640), _sys(23, 129), _sys(24, 1)]
    g, batch, plan, atoms = build(systems, "fp32")
    whole = gpu_eval(plan, atoms, p_gpu)
    off = batch.atom_offset
    for b, s in enumerate(systems):
        g, bb, pl, at = build([s], "fp32")
        one = gpu_eval(pl, at, p_gpu)
        assert np.array_equal(one["R"], whole["R"][off[b]:off[b + 1]])
        assert np.array_equal(one["force"], whole["force"][off[b]:off[b + 1]])
        assert np.array_equal(one["dEdrho"], whole["dEdrho"][off[b]:off[b + 1]])
        assert one["Ec"][0] == whole["Ec"][b] and one["Egb"][0] == whole["Egb"][b]


def test_uneven_batch_equals_its_systems_alone_bitwise():
    # the 64-system batch (library default shapes for its size: items of four
    # j blocks in the energy and chain passes) against 8 of its systems at
    # evenly spaced size ranks, each run alone (single-tile items): every
    # result bitwise equal, since every tile and item sum is rounded to fixed
    # point on its own and the integer sums do not depend on the order
    p_gpu, _ = params_pair()
    systems = synth.uneven_batch_64()
    g, batch, plan, atoms = build(systems, "fp32")
    whole = gpu_eval(plan, atoms, p_gpu)
    off = batch.atom_offset
    del plan, atoms
    sizes = np.array([s_.n for s_ in systems])
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[r]) for r in np.unique(np.round(np.linspace(0, len(systems) - 1, 8)).astype(int))]
    assert sizes[pick].min() == sizes.min() and sizes[pick].max() == sizes.max()
    for b in pick:
        g, bb, pl, at = build([systems[b]], "fp32")
        one = gpu_eval(pl, at, p_gpu)
        for k in ("R", "force", "dEdq", "dEdrho"):
            assert np.array_equal(one[k], whole[k][off[b]:off[b + 1]]), (b, k)
        assert one["Ec"][0] == whole["Ec"][b] and one["Egb"][0] == whole["Egb"][b], b


def test_energy_only_mode_matches_full():
    p_gpu, _ = params_pair()
    g, batch, plan, atoms = build([_sys(31, 300)], "fp32")
    full = gpu_eval(plan, atoms, p_gpu)
    eo = gpu_eval(plan, atoms, p_gpu, force=False, dEdq=False, dEdrho=False)
    assert eo["Ec"][0] == full["Ec"][0] and eo["Egb"][0] == full["Egb"][0]
    only_q = gpu_eval(plan, atoms, p_gpu, force=False, dEdq=True, dEdrho=False)
    assert np.array_equal(only_q["dEdq"], full["dEdq"])


def test_overflow_flag_is_raised_and_cleared():
    # charges far outside any physical range overflow the 2^32 energy scale;
    # the flag is reported, not a fault
    g, batch, plan, atoms = build([_sys(41, 100)], "fp32")
    atoms.q.mul_(1.0e6)
    p_gpu, _ = params_pair()
    g.radii(plan, atoms, p_gpu)
    g.energy_forces(plan, atoms, p_gpu)
    assert g.check_overflow(plan) is True
    assert g.check_overflow(plan) is False
    atoms.q.div_(1.0e6)
    g.radii(plan, atoms, p_gpu)
    g.energy_forces(plan, atoms, p_gpu)
    assert g.check_overflow(plan) is False


def test_graph_replay_matches_eager():
    p_gpu, _ = params_pair()
    g, batch, plan, atoms = build([_sys(51, 500), _sys(52, 260)], "fp32")
    eager = gpu_eval(plan, atoms, p_gpu)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # warm-up on the capture stream, then capture
        g.radii(plan, atoms, p_gpu)
        g.energy_forces(plan, atoms, p_gpu)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        R = g.radii(plan, atoms, p_gpu)
        out = g.energy_forces(plan, atoms, p_gpu)
    for rep in range(4):
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(R.double().cpu().numpy(), eager["R"])
        assert np.array_equal(out["force"].double().cpu().numpy(), eager["force"])
        assert np.array_equal(out["e_gb"].cpu().numpy(), eager["Egb"])
        # eager work between replays
        gpu_eval(plan, atoms, p_gpu)


def test_spatial_order_parity_and_determinism():
    # the processing order changes only FP32 rounding inside tiles: results stay
    # within tolerance of the oracle and are bitwise reproducible for one order
    p_gpu, p_or = params_pair()
    systems = [_sys(61, 900), _sys(62, 333), _sys(63, 1)]
    g, batch, plan, atoms = build(systems, "fp32")
    order = g.spatial_order(batch.atom_offset, batch.x, batch.y, batch.z)
    plan.set_order(order)
    a = gpu_eval(plan, atoms, p_gpu)
    b = gpu_eval(plan, atoms, p_gpu)
    for k in ("R", "Ec", "Egb", "force", "dEdq", "dEdrho"):
        assert np.array_equal(a[k], b[k]), k
    for i, s in enumerate(systems):
        compare_system(a, i, batch.atom_offset, oracle_eval(s, p_or), "fp32")
    # FP64: order-independent to 1e-10
    g, batch, plan64, atoms64 = build(systems, "fp64")
    ident = gpu_eval(plan64, atoms64, p_gpu)
    plan64.set_order(order)
    perm = gpu_eval(plan64, atoms64, p_gpu)
    assert rel_inf(perm["force"], ident["force"]) <= 1e-12
    assert np.max(np.abs(perm["R"] - ident["R"]) / ident["R"]) <= 1e-13


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("prec", PRECS)
def test_evaluate_equals_radii_then_energy_forces(prec, single):
    # gb_evaluate (one call; in single-launch mode one kernel launch of the
    # three pair passes with per-block dependency counters) gives the outputs
    # of gb_radii + gb_energy_forces bitwise
    p_gpu, p_or = params_pair()
    systems = [_sys(71, 700), _sys(72, 65), _sys(73, 1), _sys(74, 2500)]
    g, batch, plan, atoms = build(systems, prec)
    two = gpu_eval(plan, atoms, p_gpu)
    plan.set_single_launch(single)
    for _ in range(3):
        one = g.evaluate(plan, atoms, p_gpu)
        torch.cuda.synchronize()
        assert g.check_overflow(plan) is False
        got = {"R": one["R"], "Ec": one["e_coul"], "Egb": one["e_gb"], "force": one["force"],
               "dEdq": one["dEdq"], "dEdrho": one["dEdrho"]}
        for k, v in got.items():
            assert np.array_equal(v.double().cpu().numpy(), two[k]), k
    compare_system(two, 0, batch.atom_offset, oracle_eval(systems[0], p_or), prec)


def test_single_launch_wait_failure_is_reported_never_silent():
    # With a wait bound of 0 polls, an item that finds a block of the preceding
    # pass not yet final gives up at once instead of waiting: the launch still
    # ends normally, and the outcome is either the error flag or results equal
    # to those of a normal run (when every block happened to be ready).  The
    # next call with the default bound is correct again.
    p_gpu, _ = params_pair()
    systems = synth.eremd_batch(n_rep=8)
    g, batch, plan, atoms = build(systems, "fp32")
    ref = g.evaluate(plan, atoms, p_gpu)
    torch.cuda.synchronize()
    ref = {k: v.double().cpu().numpy() for k, v in ref.items() if v is not None}
    assert g.check_overflow(plan) is False
    plan.set_single_launch(True, 0)
    out = g.evaluate(plan, atoms, p_gpu)
    torch.cuda.synchronize()
    flagged = g.check_overflow(plan)
    if not flagged:
        for k, v in out.items():
            if v is not None:
                assert np.array_equal(v.double().cpu().numpy(), ref[k]), k
    print("wait bound 0: error reported" if flagged else "wait bound 0: every block was ready")
    plan.set_single_launch(True, 1 << 22)
    again = g.evaluate(plan, atoms, p_gpu)
    torch.cuda.synchronize()
    assert g.check_overflow(plan) is False
    for k, v in again.items():
        if v is not None:
            assert np.array_equal(v.double().cpu().numpy(), ref[k]), k
