"""Shared helpers of the GPU tests: build a plan from synthetic systems, run
the GPU path through the C ABI, and fetch oracle references.

Tolerances (the method's stated targets where there is one, otherwise derived here):
  FP32-fixed: forces, dE/dq, dE/drho  ||g - g_ref||_inf / ||g_ref||_inf <= 1e-5;
              Born radii   max |R - R_ref| / R_ref <= 2e-6 (pair terms carry
              ~1e-7 relative error; dR/dI amplifies it by at most ~10 here);
              energies     relative <= 1e-6;
              Delta E      absolute <= 1e-4 kcal/mol.
  FP64:       1e-10 for every quantity (relative max-norm; Delta E absolute).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
import synth

TOL = {
    "fp32": dict(R=2e-6, E=1e-6, grad=1e-5, dE=1e-4),
    "fp64": dict(R=1e-10, E=1e-10, grad=1e-10, dE=1e-10),
}


def gb():
    import paper_1803_09652_amd as g
    g.load()
    return g


def params_pair(name="IGB5"):
    g = gb()
    return getattr(g, name), getattr(oracle, name)


def build(systems, precision="fp32", j_blocks=None, waves=None):
    g = gb()
    batch = synth.make_batch(systems)
    plan = g.Plan(batch.atom_offset, precision, j_blocks_per_item=j_blocks, waves_per_group=waves)
    atoms = g.Atoms.from_batch(plan, batch)
    return g, batch, plan, atoms


def gpu_eval(plan, atoms, params, force=True, dEdq=True, dEdrho=True):
    g = gb()
    R = g.radii(plan, atoms, params)
    out = g.energy_forces(plan, atoms, params, force=force, dEdq=dEdq, dEdrho=dEdrho)
    torch.cuda.synchronize()
    res = {"R": R.double().cpu().numpy(), "Ec": out["e_coul"].cpu().numpy(),
           "Egb": out["e_gb"].cpu().numpy()}
    for k in ("force", "dEdq", "dEdrho"):
        res[k] = out[k].double().cpu().numpy() if out[k] is not None else None
    return res


_ORACLE_CACHE = {}


def oracle_eval(system, p_or, key=None):
    if key is not None and key in _ORACLE_CACHE:
        return _ORACLE_CACHE[key]
    r = oracle.energy_forces(system, p_or)
    if key is not None:
        _ORACLE_CACHE[key] = r
    return r


def rel_inf(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def compare_system(res, b, off, ref, prec, check_grads=True):
    """Compare system b of a GPU result against its oracle reference."""
    t = TOL[prec]
    s0, s1 = int(off[b]), int(off[b + 1])
    if s1 == s0:
        assert res["Ec"][b] == 0.0 and res["Egb"][b] == 0.0
        return {}
    errs = {}
    errs["R"] = float(np.max(np.abs(res["R"][s0:s1] - ref["R"]) / ref["R"]))
    # energies relative to |E_C| + |E_GB| (a one-atom system with zero charge has E = 0)
    scale = max(abs(ref["Ec"]) + abs(ref["Egb"]), 1e-12)
    errs["Ec"] = abs(res["Ec"][b] - ref["Ec"]) / scale
    errs["Egb"] = abs(res["Egb"][b] - ref["Egb"]) / scale
    assert errs["R"] <= t["R"], errs
    assert errs["Egb"] <= t["E"], errs
    assert errs["Ec"] <= t["E"], errs
    if check_grads:
        if res["force"] is not None:
            errs["F"] = rel_inf(res["force"][s0:s1], ref["F"])
            assert errs["F"] <= t["grad"], errs
        if res["dEdq"] is not None:
            errs["phi"] = rel_inf(res["dEdq"][s0:s1], ref["phi"])
            assert errs["phi"] <= t["grad"], errs
        if res["dEdrho"] is not None:
            errs["drho"] = rel_inf(res["dEdrho"][s0:s1], ref["dEdrho"])
            assert errs["drho"] <= t["grad"], errs
    return errs
