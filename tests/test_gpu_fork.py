"""GPU tests of the full evaluation with one staging of the inputs
(gb_evaluate) and of its forking form (gb_evaluate_fork): their outputs equal
those of gb_radii + gb_energy_forces bitwise, and Monte Carlo work queued on
the fork stream after the call (it needs only the radii) gives the same
Delta E as the same work queued after the whole evaluation on one stream,
eagerly and replayed from a captured hipGraph."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from gpu_common import build, params_pair

pytestmark = pytest.mark.gpu

KEYS = ("R", "e_coul", "e_gb", "force", "dEdq", "dEdrho")


def _systems():
    return [synth.make_system(41, 700, 10.0, n_redox=2, n_prot=3),
            synth.make_system(42, 1300, 13.0, n_redox=1, n_prot=2),
            synth.make_system(43, 65, 5.0, n_prot=1)]


def _host(d):
    return {k: d[k].double().cpu().numpy().copy() for k in KEYS}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_evaluate_and_fork_equal_separate_calls(prec):
    p_gpu, _ = params_pair()
    g, batch, plan, atoms = build(_systems(), prec)
    R = g.radii(plan, atoms, p_gpu)
    ef = g.energy_forces(plan, atoms, p_gpu)
    ref = _host(dict(ef, R=R))
    one = _host(g.evaluate(plan, atoms, p_gpu))
    side = torch.cuda.Stream()
    fk = g.evaluate(plan, atoms, p_gpu, fork=side)
    torch.cuda.current_stream().wait_stream(side)
    fk = _host(fk)
    for k in KEYS:
        assert np.array_equal(one[k], ref[k]), k
        assert np.array_equal(fk[k], ref[k]), k
    # in single-launch mode the fork follows the one queued launch
    plan.set_single_launch(True)
    sq = g.evaluate(plan, atoms, p_gpu, fork=side)
    torch.cuda.current_stream().wait_stream(side)
    assert not g.check_overflow(plan)
    sq = _host(sq)
    plan.set_single_launch(False)
    for k in KEYS:
        assert np.array_equal(sq[k], ref[k]), k


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_monte_carlo_on_the_fork_stream(prec):
    p_gpu, _ = params_pair()
    g, batch, plan, atoms = build(_systems(), prec)
    gref = np.random.default_rng(3).normal(0.0, 20.0, batch.state_count.size)
    sites = g.Sites.from_batch(plan, batch, gref)
    cur = torch.as_tensor(batch.current_state, device=plan.device)
    B = batch.n_systems
    # device tensors: nothing is copied from the host under graph capture
    pH = torch.full((B,), 7.0, dtype=torch.float64, device=plan.device)
    E = torch.linspace(-0.3, -0.1, B, dtype=torch.float64, device=plan.device)
    # serial: the whole evaluation, then the Delta E kernels on the same stream
    g.evaluate(plan, atoms, p_gpu)
    dE0, dG0 = g.mc_state_dE(plan, sites, atoms, cur, pH, E, 300.0, p_gpu)
    dE0, dG0 = dE0.cpu().numpy().copy(), dG0.cpu().numpy().copy()
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()

    def step():
        out = g.evaluate(plan, atoms, p_gpu, fork=side)
        with torch.cuda.stream(side):
            dE, dG = g.mc_state_dE(plan, sites, atoms, cur, pH, E, 300.0, p_gpu)
        main.wait_stream(side)
        return out, dE, dG

    out, dE, dG = step()
    torch.cuda.synchronize()
    assert np.array_equal(dE.cpu().numpy(), dE0)
    assert np.array_equal(dG.cpu().numpy(), dG0)
    # the same step captured in a graph (both streams) and replayed three times,
    # with eager work and synchronisation between the replays
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        main_c = torch.cuda.current_stream()
        out_g = g.evaluate(plan, atoms, p_gpu, fork=side)
        with torch.cuda.stream(side):
            dE_g, dG_g = g.mc_state_dE(plan, sites, atoms, cur, pH, E, 300.0, p_gpu)
        main_c.wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(3):
        gr.replay()
        torch.cuda.synchronize()
        assert np.array_equal(dE_g.cpu().numpy(), dE0)
        assert np.array_equal(dG_g.cpu().numpy(), dG0)
        assert np.array_equal(out_g["force"].double().cpu().numpy(),
                              out["force"].double().cpu().numpy())
        g.radii(plan, atoms, p_gpu)          # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_evaluate_with_cutoffs_and_salt_equals_separate_calls(prec):
    # the cutoff lists are rebuilt by the energy call from the positions the
    # single staging packed; salt takes the other energy kernels
    p_gpu, _ = params_pair()
    p_gpu = dataclasses.replace(p_gpu, rgbmax=10.0, cutoff=12.0, kappa=0.1)
    g, batch, plan, atoms = build(_systems() + synth.globule_2500(), prec)
    plan.set_order(g.block_order(batch.atom_offset, batch.x, batch.y, batch.z))
    R = g.radii(plan, atoms, p_gpu)
    ref = _host(dict(g.energy_forces(plan, atoms, p_gpu), R=R))
    side = torch.cuda.Stream()
    fk = g.evaluate(plan, atoms, p_gpu, fork=side)
    torch.cuda.current_stream().wait_stream(side)
    fk = _host(fk)
    for k in KEYS:
        assert np.array_equal(fk[k], ref[k]), k


def test_fork_on_the_call_stream_is_rejected():
    from paper_1803_09652_amd import _lib as L
    p_gpu, _ = params_pair()
    g, batch, plan, atoms = build(_systems()[:1], "fp32")
    with pytest.raises(L.GbmcError):
        g.evaluate(plan, atoms, p_gpu, fork=torch.cuda.current_stream())
