"""GPU tests of the autograd boundary (GBEnergy): energies per system as a
differentiable function of positions, charges and intrinsic radii.

* the 10,000-atom system (FP32 plan): forward energy and the three input
  gradients against the FP64 oracle's analytic gradients, at the FP32-fixed
  tolerances;
* a batch of uneven systems with a different upstream gradient per system;
* FP64 plan: gradients against the oracle's analytic gradients, against
  central differences of the FP64 GPU energies, and torch.autograd.gradcheck
  on a tiny system.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_common import TOL, gb, oracle_eval, params_pair, rel_inf

pytestmark = pytest.mark.gpu


def _inputs(systems, precision, requires_grad=True):
    g = gb()
    batch = synth.make_batch(systems)
    plan = g.Plan(batch.atom_offset, precision)
    dt = plan.dtype
    dev = plan.device
    pos = torch.as_tensor(np.stack([batch.x, batch.y, batch.z], 1), dtype=dt, device=dev)
    q = torch.as_tensor(batch.q, dtype=dt, device=dev)
    rho = torch.as_tensor(batch.rho, dtype=dt, device=dev)
    scr = torch.as_tensor(batch.screen, dtype=dt, device=dev)
    for t in (pos, q, rho):
        t.requires_grad_(requires_grad)
    return g, batch, plan, pos, q, rho, scr


def test_globule_10000_forward_and_gradients_against_oracle():
    # one 10,000-atom globule, FP32-fixed forward and backward
    p_gpu, p_or = params_pair()
    systems = synth.globule_10000()
    g, batch, plan, pos, q, rho, scr = _inputs(systems, "fp32")
    E = g.GBEnergy.apply(pos, q, rho, scr, plan, p_gpu)
    gE = 0.75
    (E.sum() * gE).backward()
    torch.cuda.synchronize()
    ref = oracle_eval(systems[0], p_or, ("c3", "IGB5"))
    t = TOL["fp32"]
    scale = abs(ref["Ec"]) + abs(ref["Egb"])
    e_err = abs(float(E[0]) - ref["E"]) / scale
    f_err = rel_inf(pos.grad.double().cpu().numpy(), -gE * ref["F"])
    q_err = rel_inf(q.grad.double().cpu().numpy(), gE * ref["phi"])
    r_err = rel_inf(rho.grad.double().cpu().numpy(), gE * ref["dEdrho"])
    print("E", e_err, "dE/dx", f_err, "dE/dq", q_err, "dE/drho", r_err)
    assert e_err <= t["E"]
    assert f_err <= t["grad"] and q_err <= t["grad"] and r_err <= t["grad"]


def test_batch_upstream_gradient_per_system():
    # uneven systems in one plan: each system's gradient is scaled by its own
    # upstream weight, and only the inputs that ask for a gradient get one
    p_gpu, p_or = params_pair()
    systems = [synth.make_system(70 + k, n, max(4.0, 18.0 * (n / 2500.0) ** (1 / 3)))
               for k, n in enumerate((300, 65, 700, 1))]
    g, batch, plan, pos, q, rho, scr = _inputs(systems, "fp32")
    rho.requires_grad_(False)
    E = g.GBEnergy.apply(pos, q, rho, scr, plan, p_gpu)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device=E.device)
    (E * w).sum().backward()
    torch.cuda.synchronize()
    assert rho.grad is None
    off = batch.atom_offset
    gpos = pos.grad.double().cpu().numpy()
    gq = q.grad.double().cpu().numpy()
    for b, s in enumerate(systems):
        ref = oracle_eval(s, p_or)
        s0, s1 = off[b], off[b + 1]
        wb = float(w[b])
        assert abs(float(E[b]) - ref["E"]) <= TOL["fp32"]["E"] * max(abs(ref["Ec"]) + abs(ref["Egb"]), 1e-12)
        if s.n > 1:
            assert rel_inf(gpos[s0:s1], -wb * ref["F"]) <= TOL["fp32"]["grad"]
        assert rel_inf(gq[s0:s1], wb * ref["phi"]) <= TOL["fp32"]["grad"]


def test_fp64_gradients_match_oracle():
    # FP64 plan through the autograd path: the gradients are the oracle's
    # analytic ones (which the CPU tests pin to central differences of the
    # oracle energy) to 1e-10
    p_gpu, p_or = params_pair()
    systems = [synth.make_system(81, 200, 7.0), synth.make_system(82, 70, 5.0)]
    g, batch, plan, pos, q, rho, scr = _inputs(systems, "fp64")
    E = g.GBEnergy.apply(pos, q, rho, scr, plan, p_gpu)
    w = torch.tensor([0.5, -1.5], dtype=torch.float64, device=E.device)
    (E * w).sum().backward()
    off = batch.atom_offset
    t = TOL["fp64"]["grad"]
    for b, s in enumerate(systems):
        ref = oracle_eval(s, p_or)
        s0, s1 = off[b], off[b + 1]
        wb = float(w[b])
        assert rel_inf(pos.grad[s0:s1].cpu().numpy(), -wb * ref["F"]) <= t
        assert rel_inf(q.grad[s0:s1].cpu().numpy(), wb * ref["phi"]) <= t
        assert rel_inf(rho.grad[s0:s1].cpu().numpy(), wb * ref["dEdrho"]) <= t


def test_fp64_gradients_consistent_with_energy_differences():
    # backward is the derivative of forward: four-point central differences of
    # the FP64 GPU energies.  Energies are summed in 2^-32 kcal/mol fixed point
    # per tile partial, so the step is large: h = 2e-3 keeps the rounding noise
    # (~1e-9 x 18 / (12 h)) below 1e-6 and the truncation (h^4 f^(5) / 30) near 1e-7
    p_gpu, _ = params_pair()
    s = synth.make_system(83, 64, 6.0, min_dist=1.4)
    g, batch, plan, pos, q, rho, scr = _inputs([s], "fp64")
    E = g.GBEnergy.apply(pos, q, rho, scr, plan, p_gpu)
    E.sum().backward()
    P0, Q0, R0 = pos.detach().clone(), q.detach().clone(), rho.detach().clone()

    def energy(p_, q_, r_):
        with torch.no_grad():
            return float(g.GBEnergy.apply(p_, q_, r_, scr, plan, p_gpu)[0])

    def d4(f, base, idx, h=2e-3):
        vals = []
        for m in (-2, -1, 1, 2):
            t = base.clone()
            t[idx] += m * h
            vals.append(f(t))
        return (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)

    rng = np.random.default_rng(5)
    for a in rng.choice(s.n, 5, replace=False):
        for c in range(3):
            fd = d4(lambda t: energy(t, Q0, R0), P0, (a, c))
            assert abs(float(pos.grad[a, c]) - fd) <= 2e-5 * max(1.0, abs(fd)), (a, c, fd)
        fd = d4(lambda t: energy(P0, t, R0), Q0, a)
        assert abs(float(q.grad[a]) - fd) <= 2e-5 * max(1.0, abs(fd)), (a, fd)
        fd = d4(lambda t: energy(P0, Q0, t), R0, a)
        assert abs(float(rho.grad[a]) - fd) <= 2e-5 * max(1.0, abs(fd)), (a, fd)


def test_fp64_gradcheck_tiny_system():
    # torch's own check of the backward against its finite differences; eps
    # and tolerances sized for the 2^-32 kcal/mol energy quantum
    p_gpu, _ = params_pair()
    s = synth.make_system(91, 12, 4.0, min_dist=1.5)
    g, batch, plan, pos, q, rho, scr = _inputs([s], "fp64")
    f = lambda p_, q_, r_: g.GBEnergy.apply(p_, q_, r_, scr, plan, p_gpu)
    assert torch.autograd.gradcheck(f, (pos, q, rho), eps=1e-3, atol=1e-3, rtol=1e-3)


def test_fp64_gradients_with_salt_and_cutoffs():
    # the autograd boundary with the GB variants: salt and both cutoffs, the
    # gradients against the oracle's analytic ones (pinned on the CPU by
    # central differences of the cut, salted energy)
    import dataclasses
    p_gpu, p_or = params_pair()
    p_gpu = dataclasses.replace(p_gpu, kappa=0.12, rgbmax=9.0, cutoff=7.3)
    p_or = dataclasses.replace(p_or, kappa=0.12, rgbmax=9.0, cutoff=7.3)
    systems = [synth.make_system(84, 260, 9.0), synth.make_system(85, 90, 6.0)]
    g, batch, plan, pos, q, rho, scr = _inputs(systems, "fp64")
    E = g.GBEnergy.apply(pos, q, rho, scr, plan, p_gpu)
    w = torch.tensor([1.25, -0.5], dtype=torch.float64, device=E.device)
    (E * w).sum().backward()
    off = batch.atom_offset
    t = TOL["fp64"]
    for b, s in enumerate(systems):
        ref = oracle_eval(s, p_or)
        s0, s1 = off[b], off[b + 1]
        wb = float(w[b])
        assert abs(float(E[b]) - ref["E"]) <= t["E"] * (abs(ref["Ec"]) + abs(ref["Egb"]))
        assert rel_inf(pos.grad[s0:s1].cpu().numpy(), -wb * ref["F"]) <= t["grad"]
        assert rel_inf(q.grad[s0:s1].cpu().numpy(), wb * ref["phi"]) <= t["grad"]
        assert rel_inf(rho.grad[s0:s1].cpu().numpy(), wb * ref["dEdrho"]) <= t["grad"]
