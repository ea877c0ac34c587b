"""The simulation loop of CEMD, C(pH,E)MD and E-REMD (section III.A-B, Fig. 1)
on one plan: constant-charge Langevin dynamics on the Coulomb + GB forces,
halted every `attempt_every` steps for a Monte Carlo attempt pair
(protonation, then redox on the updated charges), and every `exchange_every`
steps for a replica-exchange attempt along the redox-potential ladder, the
parity alternating from one exchange attempt to the next (section III.B).

Every step is a fixed sequence of library calls on the current stream:

    gb_radii -> [mc_state_dE -> mc_step] -> [remd_exchange]
             -> gb_energy_forces (forces) -> md_langevin_step

so an attempt is made at the coordinates the dynamics halted at, and the
charges it leaves drive the dynamics from that point on (Fig. 1).  The loop itself
does no arithmetic: it picks the calls and the random inputs (Langevin noise
and Monte Carlo / exchange uniforms, drawn on the device from a seeded torch
generator unless the caller passes them) and records, after every attempt,
the site states and the replica at each rung for the analysis.

The systems of the plan are the replicas.  With exchange_every = 0 each
system keeps its own redox potential (CEMD, C(pH,E)MD); otherwise the systems
are replicas of one molecule on the ladder E_rung (E-REMD).  Replicas at
different pH form separate ladders (only replicas at the same pH exchange
their redox potentials, section III.B): `ladders` lists the rung ranges
[start, stop) of each, and each ladder's exchange attempt is its own call.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import api


class ReplicaMD:
    def __init__(self, plan: api.Plan, sites: api.Sites, atoms: api.Atoms, current_state,
                 inv_mass, v, pH, E_rung, rep_of_rung=None, dt: float = 0.002, gamma: float = 5.0,
                 T: float = 300.0, attempt_every: int = 5, exchange_every: int = 0,
                 params: api.GBParams = api.IGB5, xref=None, k_restr: float = 0.0,
                 wrap: bool = True, seed: int = 0, ladders=None):
        if attempt_every < 0 or exchange_every < 0:
            raise ValueError("attempt_every and exchange_every must be >= 0")
        dev, dt_ = plan.device, plan.dtype
        B, N = plan.n_systems, plan.n_atoms
        self.plan, self.sites, self.atoms, self.params = plan, sites, atoms, params
        self.dt, self.gamma, self.T = float(dt), float(gamma), float(T)
        self.attempt_every, self.exchange_every = int(attempt_every), int(exchange_every)
        self.k_restr, self.wrap = float(k_restr), bool(wrap)
        as_dev = lambda a, dt=dt_: torch.as_tensor(np.asarray(a), dtype=dt, device=dev).contiguous()
        self.inv_mass = as_dev(inv_mass)
        self.v = as_dev(v)
        if tuple(self.v.shape) != (3, N) or tuple(self.inv_mass.shape) != (N,):
            raise ValueError("v must be [3, N] and inv_mass [N]")
        self.xref = None if xref is None else as_dev(xref)
        self.pH = api._dev_f64(pH, B, dev)
        self.E_rung = torch.as_tensor(np.asarray(E_rung, dtype=np.float64), device=dev)
        if self.E_rung.shape != (B,):
            raise ValueError("E_rung must hold one redox potential per system")
        rep = np.arange(B) if rep_of_rung is None else np.asarray(rep_of_rung)
        if sorted(rep.tolist()) != list(range(B)):
            raise ValueError("rep_of_rung must be a permutation of the systems")
        self.rep_of_rung = torch.as_tensor(rep, dtype=torch.int32, device=dev).contiguous()
        # per-replica redox potential: replica rep_of_rung[l] sits at rung l
        E_rep = np.empty(B)
        E_rep[rep] = np.asarray(E_rung, dtype=np.float64)
        self.E_rep = torch.as_tensor(E_rep, device=dev)
        # ladders: rung ranges; each ladder's replicas (fixed set, sorted) and
        # their local indices on its rungs
        lad = [(0, B)] if ladders is None else [(int(a), int(b)) for a, b in ladders]
        if lad and (lad[0][0] != 0 or lad[-1][1] != B
                    or any(l0[1] != l1[0] for l0, l1 in zip(lad, lad[1:]))
                    or any(b <= a for a, b in lad)):
            raise ValueError("ladders must partition the rungs 0..B in order")
        self.ladders = []
        for a, b in lad:
            sys_k = np.sort(rep[a:b])
            local = np.searchsorted(sys_k, rep[a:b]).astype(np.int32)
            self.ladders.append({
                "rungs": (a, b),
                "sys": torch.as_tensor(sys_k, dtype=torch.int64, device=dev),
                "rep": torch.as_tensor(local, device=dev).contiguous(),
                "E_rung": self.E_rung[a:b].contiguous(),
                "E_out": torch.empty(b - a, dtype=torch.float64, device=dev),
            })
        st = np.asarray(current_state, dtype=np.int32)
        if st.shape != (sites.n_sites,):
            raise ValueError("current_state must hold one state per site")
        self.state = torch.as_tensor(st, device=dev).clone()
        # each system's electron count: n_e of its redox sites' current states
        ne = np.zeros(B, dtype=np.int32)
        for m in range(sites.n_sites):
            if sites.site_kind[m] == api.KIND_REDOX:
                ne[sites.site_system[m]] += sites.state_count[sites.site_state_offset[m] + st[m]]
        self.counters = torch.zeros((max(sites.n_sites, 1), 2), dtype=torch.int64, device=dev)
        self.n_electrons = torch.as_tensor(ne, device=dev)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(int(seed))
        self.step_index = 0
        self.n_attempts = 0
        self.n_exchanges = 0
        self._acc_x = torch.zeros((), dtype=torch.int64, device=dev)

    def run(self, n_steps: int, xi: Optional[torch.Tensor] = None,
            u_mc: Optional[torch.Tensor] = None, u_x: Optional[torch.Tensor] = None,
            record: bool = True) -> dict:
        """n_steps MD steps with the attempt and exchange schedules, counted
        from the loop's global step index.  Optional random inputs: xi
        [n_steps, 3, N] (plan dtype) standard normals; u_mc [n_attempts, B, 6]
        and u_x [n_exchanges, B] float64 uniforms, one row per attempt in this
        call.  Returns the records of the attempts made (device tensors): the
        site states [a, S] after each attempt, with the replica at each rung
        [a, B] and each replica's electron count [a, B] at that moment (before
        an exchange attempt of the same step)."""
        plan, dev, B, N = self.plan, self.plan.device, self.plan.n_systems, self.plan.n_atoms
        k0 = self.step_index
        att = [k for k in range(k0, k0 + n_steps)
               if self.attempt_every and (k + 1) % self.attempt_every == 0]
        exch = [k for k in range(k0, k0 + n_steps)
                if self.exchange_every and (k + 1) % self.exchange_every == 0]
        if xi is not None and tuple(xi.shape) != (n_steps, 3, N):
            raise ValueError("xi must be [n_steps, 3, N]")
        if u_mc is not None and tuple(u_mc.shape) != (len(att), B, 6):
            raise ValueError(f"u_mc must be [{len(att)}, {B}, 6]")
        if u_x is not None and tuple(u_x.shape) != (len(exch), B):
            raise ValueError(f"u_x must be [{len(exch)}, {B}]")
        S = self.sites.n_sites
        rec = {"state": torch.empty((len(att), S), dtype=torch.int32, device=dev),
               "rep_of_rung": torch.empty((len(att), B), dtype=torch.int32, device=dev),
               "n_electrons": torch.empty((len(att), B), dtype=torch.int32, device=dev)}
        noise = torch.empty((3, N), dtype=plan.dtype, device=dev)
        a_i = x_i = 0
        for k in range(k0, k0 + n_steps):
            api.radii(plan, self.atoms, self.params)
            if self.attempt_every and (k + 1) % self.attempt_every == 0:
                u = u_mc[a_i] if u_mc is not None else \
                    torch.rand((B, 6), dtype=torch.float64, device=dev, generator=self.gen)
                dE, dG = api.mc_state_dE(plan, self.sites, self.atoms, self.state, self.pH,
                                         self.E_rep, self.T, self.params)
                out = api.mc_step(plan, self.sites, self.atoms, self.state, self.pH, self.E_rep,
                                  dE, dG, u, self.T, self.params, counters=self.counters)
                self.n_electrons.copy_(out["n_electrons"])
                if record:
                    rec["state"][a_i].copy_(self.state[:S])
                    rec["rep_of_rung"][a_i].copy_(self.rep_of_rung)
                    rec["n_electrons"][a_i].copy_(self.n_electrons)
                a_i += 1
                self.n_attempts += 1
            if self.exchange_every and (k + 1) % self.exchange_every == 0:
                u = u_x[x_i] if u_x is not None else \
                    torch.rand(B, dtype=torch.float64, device=dev, generator=self.gen)
                for lad in self.ladders:
                    a, b = lad["rungs"]
                    if len(self.ladders) == 1:
                        # one ladder over every system: replica and local indices agree
                        acc, _ = api.remd_exchange(self.E_rung, self.n_electrons, self.rep_of_rung,
                                                   self.n_exchanges % 2, u, self.T, self.wrap,
                                                   E_out=self.E_rep)
                    else:
                        ne = self.n_electrons.index_select(0, lad["sys"]).contiguous()
                        acc, _ = api.remd_exchange(lad["E_rung"], ne, lad["rep"],
                                                   self.n_exchanges % 2, u[a:b].contiguous(),
                                                   self.T, self.wrap, E_out=lad["E_out"])
                        self.E_rep.index_copy_(0, lad["sys"], lad["E_out"])
                        self.rep_of_rung[a:b] = lad["sys"].index_select(
                            0, lad["rep"].long()).to(torch.int32)
                    self._acc_x += acc.sum()
                x_i += 1
                self.n_exchanges += 1
            f = api.energy_forces(plan, self.atoms, self.params, dEdq=False, dEdrho=False)["force"]
            if xi is not None:
                noise = xi[k - k0]
            else:
                torch.randn((3, N), dtype=plan.dtype, device=dev, generator=self.gen, out=noise)
            api.md_step(plan, self.atoms, self.v, f, self.inv_mass, noise, self.dt, self.gamma,
                        self.T, xref=self.xref, k_restr=self.k_restr)
        self.step_index = k0 + n_steps
        return rec

    @property
    def exchanges_accepted(self) -> int:
        return int(self._acc_x)
