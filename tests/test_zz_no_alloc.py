"""The no-allocation entry point gb_evaluate_static (C ABI, through the ctypes
binding) against gb_evaluate with a caller workspace: two calls in a row, the
second on a smaller batch, in both plans, bitwise equal (the same kernels on
the same inputs; every sum is integer fixed point, so the workspace address
cannot change a bit).  The static call allocates no device memory: with
preallocated outputs the torch allocator sees no change either.  A plan whose
workspace exceeds the static scratch is refused before any launch."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _case(g, systems, prec):
    batch = synth.make_batch(systems)
    plan = g.Plan(batch.atom_offset, prec)
    plan.set_order(g.spatial_order(batch.atom_offset, batch.x, batch.y, batch.z))
    atoms = g.Atoms.from_batch(plan, batch)
    return plan, atoms


def _host(out):
    return {k: v.double().cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_static_matches_workspace_entry_point_two_calls(prec):
    import paper_1803_09652_amd as g
    g.load()
    big = [synth.make_system(901, 2500, 18.0), synth.make_system(902, 777, 12.0)]
    small = [synth.make_system(903, 300, 8.0)]
    for systems in (big, small):
        print(prec, "systems", [s.n for s in systems], flush=True)
        plan, atoms = _case(g, systems, prec)
        ref = _host(g.evaluate(plan, atoms, g.IGB5))
        from paper_1803_09652_amd.api import _eval_outputs
        out = _eval_outputs(plan, True, True, True)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        g.evaluate_static(plan, atoms, g.IGB5, out=out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        got = _host(out)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (prec, [s.n for s in systems], k)
        assert g.check_overflow(plan, static=True) is False


def test_static_refuses_a_plan_beyond_the_scratch():
    import paper_1803_09652_amd as g
    from paper_1803_09652_amd._lib import GBMC_ERR_UNSUPPORTED, GbmcError
    n = 1_500_000
    plan = g.Plan(np.array([0, n], dtype=np.int32), "fp32")
    z = torch.zeros(n, dtype=torch.float32, device=plan.device)
    atoms = g.Atoms(plan, z, z, z, z, z + 1.5, z)
    with pytest.raises(GbmcError) as e:
        g.evaluate_static(plan, atoms, g.IGB5)
    assert e.value.status == GBMC_ERR_UNSUPPORTED
