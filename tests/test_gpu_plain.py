"""GPU parity of gb_plain_fp64 (C ABI), the plain FP64 GPU form of one full
evaluation that the batched forms' pair rate is compared with: radii,
energies, forces, dE/dq and dE/drho against the oracle at the FP64
tolerances, on a ragged batch with an empty system, and on the E-REMD batch's
first two replicas; salt or cutoffs are refused."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import TOL, compare_system, params_pair

pytestmark = pytest.mark.gpu


def _run(systems, p_gpu):
    import paper_1803_09652_amd as g
    b = synth.make_batch(systems)
    out = g.plain_fp64(b.atom_offset, b.x, b.y, b.z, b.q, b.rho, b.screen, p_gpu)
    torch.cuda.synchronize()
    res = {"R": out["R"].cpu().numpy(), "Ec": out["e_coul"].cpu().numpy(),
           "Egb": out["e_gb"].cpu().numpy(), "force": out["force"].cpu().numpy(),
           "dEdq": out["dEdq"].cpu().numpy(), "dEdrho": out["dEdrho"].cpu().numpy()}
    return b, res


@pytest.mark.parametrize("pname", ["IGB5", "IGB2"])
def test_plain_fp64_ragged_batch(pname):
    p_gpu, p_or = params_pair(pname)
    systems = [synth.make_system(160, 1, 2.0), synth.make_system(161, 2, 2.0),
               synth.make_system(162, 65, 5.0), synth.make_system(163, 300, 8.5)]
    systems.insert(2, synth.System(*(np.zeros(0) for _ in range(6))))
    b, res = _run(systems, p_gpu)
    for k, s in enumerate(systems):
        if s.n == 0:
            assert res["Ec"][k] == 0.0 and res["Egb"][k] == 0.0
            continue
        compare_system(res, k, b.atom_offset, oracle.energy_forces(s, p_or), "fp64")


def test_plain_fp64_ereMD_replicas():
    p_gpu, p_or = params_pair()
    systems = synth.eremd_batch(n_rep=2)
    b, res = _run(systems, p_gpu)
    for k, s in enumerate(systems):
        compare_system(res, k, b.atom_offset, oracle.energy_forces(s, p_or), "fp64")


def test_plain_fp64_refuses_variants():
    import paper_1803_09652_amd as g
    p_gpu, _ = params_pair()
    s = synth.make_system(164, 10, 3.0)
    b = synth.make_batch([s])
    for v in ({"kappa": 0.1}, {"cutoff": 8.0}, {"rgbmax": 8.0}):
        with pytest.raises(g.GbmcError):
            g.plain_fp64(b.atom_offset, b.x, b.y, b.z, b.q, b.rho, b.screen,
                         dataclasses.replace(p_gpu, **v))
