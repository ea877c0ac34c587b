"""GPU parity of md_langevin_step (C ABI), the leapfrog Langevin step between
Monte Carlo attempts, against the oracle's step (FP64 forces, FP64 update):

* one step of a batch of uneven systems, FP32-fixed and FP64 plans, with
  noise, friction and a harmonic restraint: positions and velocities;
* a 25-step FP64 trajectory, step by step;
* the degenerate cases: a frozen atom (inverse mass 0) and gamma = 0 with no
  noise is plain leapfrog.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import TOL, build, params_pair

pytestmark = pytest.mark.gpu

DT, GAMMA, T, K_RESTR = 0.002, 5.0, 300.0, 25.0


def _systems():
    return [synth.make_system(301, 300, 8.0), synth.make_system(302, 65, 5.0),
            synth.make_system(303, 1, 2.0), synth.make_system(304, 130, 6.0)]


def _state(batch, seed):
    n = batch.x.shape[0]
    m = synth.masses(seed, n)
    v = synth.f32(synth.thermal_velocities(seed + 1, m, T))
    xi = synth.f32(synth.normals(seed + 2, (n, 3)))
    xref = synth.f32(np.stack([batch.x, batch.y, batch.z], 1)
                     + 0.1 * synth.normals(seed + 3, (n, 3)))
    return m, v, xi, xref


def _gpu_steps(g, plan, atoms, p_gpu, inv_m, v, xis, xref, gamma=GAMMA):
    dev, dt_ = plan.device, plan.dtype
    vt = torch.as_tensor(v.T.copy(), dtype=dt_, device=dev)
    im = torch.as_tensor(inv_m, dtype=dt_, device=dev)
    xr = None if xref is None else torch.as_tensor(xref.T.copy(), dtype=dt_, device=dev)
    out = []
    for xi in xis:
        g.radii(plan, atoms, p_gpu)
        f = g.energy_forces(plan, atoms, p_gpu, dEdq=False, dEdrho=False)["force"]
        g.md_step(plan, atoms, vt, f, im, torch.as_tensor(xi.T.copy(), dtype=dt_, device=dev),
                  DT, gamma, T, xref=xr, k_restr=K_RESTR if xr is not None else 0.0)
        torch.cuda.synchronize()
        pos = torch.stack([atoms.x, atoms.y, atoms.z], 1).double().cpu().numpy()
        out.append((pos, vt.double().cpu().numpy().T.copy()))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_one_step_matches_oracle(prec):
    p_gpu, p_or = params_pair()
    systems = _systems()
    g, batch, plan, atoms = build(systems, prec)
    m, v, xi, xref = _state(batch, 11)
    inv_m = 1.0 / m
    inv_m[0] = 0.0                                    # a frozen atom: no inverse mass,
    v[0] = 0.0                                        # no velocity
    (pos, vg), = _gpu_steps(g, plan, atoms, p_gpu, inv_m, v, [xi], xref)
    off = batch.atom_offset
    for b, s in enumerate(systems):
        sl = slice(off[b], off[b + 1])
        x, y, z, vo = oracle.langevin_step(s, v[sl], inv_m[sl], xi[sl], DT, GAMMA, T, p_or,
                                           xref=xref[sl], k_restr=K_RESTR)
        po = np.stack([x, y, z], 1)
        # velocity error: the FP32 force error (relative to the largest force)
        # times the kick dt 418.4 / m, plus storage rounding of v
        kick = DT * oracle.ACC * inv_m[sl].max()
        F = oracle.energy_forces(s, p_or)["F"]
        fmax = max(np.abs(F).max(), 1.0)
        if prec == "fp64":
            tv, tx = 1e-10 * kick * fmax + 1e-12 * np.abs(vo).max(), 1e-12 * (1 + np.abs(po).max())
        else:
            tv = 2 * TOL["fp32"]["grad"] * kick * fmax + 2e-7 * np.abs(vo).max()
            tx = DT * tv + 2e-7 * np.abs(po).max()
        assert np.abs(vg[sl] - vo).max() <= tv, (b, np.abs(vg[sl] - vo).max(), tv)
        assert np.abs(pos[sl] - po).max() <= tx, (b, np.abs(pos[sl] - po).max(), tx)
    # the frozen atom keeps its position and has no velocity after the step
    assert np.array_equal(pos[0], np.array([batch.x[0], batch.y[0], batch.z[0]], dtype=np.float64))
    assert np.all(vg[0] == 0.0)


def test_fp64_trajectory_matches_oracle():
    p_gpu, p_or = params_pair()
    systems = [synth.make_system(305, 90, 6.0, min_dist=1.5), synth.make_system(306, 40, 5.0, min_dist=1.5)]
    g, batch, plan, atoms = build(systems, "fp64")
    m, v, _, xref = _state(batch, 21)
    n = batch.x.shape[0]
    xis = [synth.normals(100 + k, (n, 3)) for k in range(25)]
    traj = _gpu_steps(g, plan, atoms, p_gpu, 1.0 / m, v, xis, xref)
    off = batch.atom_offset
    for b, s in enumerate(systems):
        sl = slice(off[b], off[b + 1])
        sys_ = s.copy()
        vb = v[sl].copy()
        for k in range(25):
            x, y, z, vb = oracle.langevin_step(sys_, vb, 1.0 / m[sl], xis[k][sl], DT, GAMMA, T, p_or,
                                               xref=xref[sl], k_restr=K_RESTR)
            sys_.x, sys_.y, sys_.z = x, y, z
            pos, vg = traj[k]
            assert np.abs(pos[sl] - sys_.coords()).max() <= 1e-9, (b, k)
            assert np.abs(vg[sl] - vb).max() <= 1e-8 * max(1.0, np.abs(vb).max()), (b, k)


def test_no_friction_no_noise_is_leapfrog():
    # gamma = 0: the step is v' = v + dt 418.4 F / m, x' = x + dt v' whatever xi holds
    p_gpu, p_or = params_pair()
    systems = [synth.make_system(307, 64, 5.0, min_dist=1.5)]
    g, batch, plan, atoms = build(systems, "fp64")
    m, v, xi, _ = _state(batch, 31)
    x0 = np.stack([batch.x, batch.y, batch.z], 1)
    (pos, vg), = _gpu_steps(g, plan, atoms, p_gpu, 1.0 / m, v, [xi], None, gamma=0.0)
    F = oracle.energy_forces(systems[0], p_or)["F"]
    v_ref = v + DT * oracle.ACC * F / m[:, None]
    assert np.abs(vg - v_ref).max() <= 1e-10 * max(1.0, np.abs(v_ref).max())
    assert np.abs(pos - (x0 + DT * v_ref)).max() <= 1e-11 * (1 + np.abs(x0).max())
