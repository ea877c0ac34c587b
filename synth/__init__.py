"""Seeded synthetic workloads: protein-like globules with titratable sites.

This module only *draws inputs*.  It holds none of the Generalized Born or
Monte Carlo arithmetic, so that both the FP64 oracle (``oracle/``) and the GPU
library (``paper_1803_09652_amd``) can be fed from it without sharing any of the
method's code.

The paper's own test system (NAcMP8 with a histidine peptide, 237 atoms in
implicit solvent, Table 1) and its force-field / state-charge tables (the
supporting-information tables of heme and propionate charges) are not
available, so these globules stand in for them.  Recipe (all values are drawn
in FP64 and rounded to FP32, so that both sides see identical inputs):

* atoms uniform in a sphere of radius ``r_glob`` with rejection closer than
  ``min_dist`` (random sequential addition, in proposal order);
* charges ~ N(0, 0.3) e, shifted to net zero;
* intrinsic GB radii ~ U[1.2, 2.0] A, screening factors ~ U[0.7, 0.9]
  (the heme iron of section III.C, 1.5 A / 0.8, lies inside these ranges);
* a site is the k nearest unassigned atoms to a random centre; sites are
  disjoint;
* redox site: 2 states, state 0 oxidised (n_e = 0), state 1 reduced with charge
  deltas ~ N(0, 0.05) shifted to sum to -1 e (n_e = 1);
* protonation site: 5 states by default (2..5 allowed), state 0 deprotonated
  (n_H = 0); every other state carries one proton (n_H = 1) with its own delta
  pattern summing to +1 e.  Five states is the discrete-state carboxylate model
  (one deprotonated and four protonated tautomers) of the glutamate and
  propionate sites titrated in section III.C.
* dynamics: masses ~ U[12, 16] amu (heavy atoms, hydrogens folded in),
  Maxwell-Boltzmann starting velocities, standard normal Langevin noise.

Generators are ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
from scipy.spatial import cKDTree

KIND_PROT = 0
KIND_REDOX = 1


def f32(a) -> np.ndarray:
    """Round to the nearest FP32 value, returned as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class Site:
    kind: int                 # KIND_PROT or KIND_REDOX
    atoms: np.ndarray         # system-local atom indices, int64, ascending
    charges: np.ndarray       # [n_states, n_atoms] float64 (FP32-representable)
    counts: np.ndarray        # [n_states] int32: n_H (prot) or n_e (redox)
    state: int                # current state

    @property
    def n_states(self) -> int:
        return int(self.charges.shape[0])


@dataclass
class System:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    rho: np.ndarray
    screen: np.ndarray
    sites: List[Site] = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def coords(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def copy(self) -> "System":
        return System(self.x.copy(), self.y.copy(), self.z.copy(), self.q.copy(),
                      self.rho.copy(), self.screen.copy(),
                      [Site(s.kind, s.atoms.copy(), s.charges.copy(), s.counts.copy(), s.state)
                       for s in self.sites])


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def globule_coords(rng: np.random.Generator, n: int, r_glob: float,
                   min_dist: float = 1.0, max_rounds: int = 10000) -> np.ndarray:
    """Random sequential addition of ``n`` points in a ball of radius ``r_glob``.

    Proposals are drawn in batches; a proposal is kept if it lies at least
    ``min_dist`` from every point kept before it (earlier kept points and earlier
    proposals of the same batch), which is exactly sequential addition in
    proposal order.
    """
    kept = np.zeros((0, 3))
    for _ in range(max_rounds):
        need = n - kept.shape[0]
        if need <= 0:
            break
        m = max(64, int(need * 1.5))
        # uniform in the ball: direction x radius^(1/3)
        v = rng.normal(size=(m, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        rad = r_glob * rng.random(m) ** (1.0 / 3.0)
        cand = v * rad[:, None]
        ok = np.ones(m, dtype=bool)
        if kept.shape[0]:
            d, _ = cKDTree(kept).query(cand, k=1, distance_upper_bound=min_dist)
            ok &= ~(d < min_dist)
        idx = np.nonzero(ok)[0]
        sub = cand[idx]
        if idx.size > 1:
            pairs = cKDTree(sub).query_pairs(min_dist, output_type="ndarray")
            if pairs.size:
                # greedy in proposal order: a proposal survives if no earlier
                # *surviving* proposal conflicts with it
                conflicts = [[] for _ in range(idx.size)]
                for a, b in pairs:
                    lo, hi = (a, b) if a < b else (b, a)
                    conflicts[hi].append(lo)
                alive = np.ones(idx.size, dtype=bool)
                for t in range(idx.size):
                    for lo in conflicts[t]:
                        if alive[lo]:
                            alive[t] = False
                            break
                sub = sub[alive]
        kept = np.concatenate([kept, sub[:need]], axis=0)
    if kept.shape[0] < n:
        raise RuntimeError("globule too dense for the minimum distance")
    return kept


def _atom_params(rng: np.random.Generator, n: int):
    q = rng.normal(0.0, 0.3, size=n)
    q -= q.mean()
    rho = rng.uniform(1.2, 2.0, size=n)
    screen = rng.uniform(0.7, 0.9, size=n)
    return f32(q), f32(rho), f32(screen)


def _pick_site_atoms(rng, xyz, taken, k, r_glob):
    free = np.nonzero(~taken)[0]
    if free.size < k:
        raise RuntimeError("not enough free atoms for a site")
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    centre = v * 0.7 * r_glob * rng.random() ** (1.0 / 3.0)
    d = np.linalg.norm(xyz[free] - centre, axis=1)
    sel = np.sort(free[np.argsort(d, kind="stable")[:k]])
    taken[sel] = True
    return sel


def _redox_site(rng, base_q, atoms) -> Site:
    k = atoms.size
    dq = rng.normal(0.0, 0.05, size=k)
    dq += (-1.0 - dq.sum()) / k
    ox = f32(base_q[atoms])
    red = f32(ox + dq)
    return Site(KIND_REDOX, atoms, np.stack([ox, red]), np.array([0, 1], dtype=np.int32), 0)


def _prot_site(rng, base_q, atoms, n_states: int = 5) -> Site:
    k = atoms.size
    ns = int(n_states)
    if not 2 <= ns <= 8:
        raise ValueError("a site has 2..8 states")
    deprot = f32(base_q[atoms])
    rows = [deprot]
    for _ in range(ns - 1):
        dq = rng.normal(0.0, 0.05, size=k)
        # the added proton sits mostly on one atom of the site
        dq[int(rng.integers(0, k))] += 0.5
        dq += (1.0 - dq.sum()) / k
        rows.append(f32(deprot + dq))
    counts = np.array([0] + [1] * (ns - 1), dtype=np.int32)
    return Site(KIND_PROT, atoms, np.stack(rows), counts, 0)


def _apply_states(sys_: System) -> None:
    for s in sys_.sites:
        sys_.q[s.atoms] = s.charges[s.state]


def make_system(seed: int, n: int, r_glob: float, n_redox: int = 0, n_prot: int = 0,
                redox_atoms: int = 74, prot_atoms=(10, 20), random_states: bool = False,
                min_dist: float = 1.0, prot_states: int = 5) -> System:
    rng = rng_for(seed)
    xyz = f32(globule_coords(rng, n, r_glob, min_dist))
    q, rho, screen = _atom_params(rng, n)
    sys_ = System(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), q, rho, screen)
    taken = np.zeros(n, dtype=bool)
    for _ in range(n_redox):
        atoms = _pick_site_atoms(rng, xyz, taken, redox_atoms, r_glob)
        sys_.sites.append(_redox_site(rng, q, atoms))
    for _ in range(n_prot):
        k = int(rng.integers(prot_atoms[0], prot_atoms[1] + 1))
        atoms = _pick_site_atoms(rng, xyz, taken, k, r_glob)
        sys_.sites.append(_prot_site(rng, q, atoms, prot_states))
    if random_states:
        for s in sys_.sites:
            s.state = int(rng.integers(0, s.n_states))
    _apply_states(sys_)
    return sys_


def perturb(base: System, seed: int, sigma: float = 0.5, min_pair: float = 0.5,
            random_states: bool = True) -> System:
    """Replica of ``base``: coordinates + N(0, sigma) per atom.  An atom whose
    perturbation creates a pair closer than ``min_pair`` gets a fresh
    perturbation (higher index of each offending pair, repeated until clear)."""
    rng = rng_for(seed)
    xyz0 = base.coords()
    d = rng.normal(0.0, sigma, size=xyz0.shape)
    xyz = xyz0 + d
    for _ in range(1000):
        pairs = cKDTree(xyz).query_pairs(min_pair, output_type="ndarray")
        if pairs.size == 0:
            break
        bad = np.unique(pairs.max(axis=1))
        xyz[bad] = xyz0[bad] + rng.normal(0.0, sigma, size=(bad.size, 3))
    else:
        raise RuntimeError("could not resolve close pairs")
    xyz = f32(xyz)
    out = base.copy()
    out.x, out.y, out.z = xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy()
    if random_states:
        for s in out.sites:
            s.state = int(rng.integers(0, s.n_states))
        _apply_states(out)
    return out


# --------------------------------------------------------------------------
# The five workloads.  Sizes and distributions follow the workload table of
# the design notes; indices are 0-based.
# --------------------------------------------------------------------------

E_LADDER = tuple(round(-0.40 + 0.02 * k, 10) for k in range(16))   # V
PH_DEFAULT = 7.0
T_DEFAULT = 300.0


def globule_256() -> List[System]:
    return [make_system(0, 256, 12.0, n_redox=1, n_prot=0)]


def globule_2500() -> List[System]:
    return [make_system(1, 2500, 18.0, n_redox=4, n_prot=4)]


def eremd_batch(n_rep: int = 16) -> List[System]:
    base = globule_2500()[0]
    return [perturb(base, 2 + 1000 * r) for r in range(n_rep)]


# Dynamics on the electrostatics alone: the globules carry no bonded or van der
# Waals terms and no exclusions, so every atom is held near its start by a
# harmonic restraint of this stiffness (kcal/mol/A^2), stiff enough that no
# oppositely charged close pair of the 2,500-atom globule can collapse.
MD_RESTRAINT = 2000.0


def eremd_batch_md(n_rep: int = 16) -> List[System]:
    """E-REMD replicas for dynamics: the 2,500-atom globule unperturbed (the
    perturbed replicas hold pairs closer than any restraint can keep apart),
    each replica with its own random site states."""
    base = globule_2500()[0]
    out = []
    for r in range(n_rep):
        rng = rng_for(5 + 1000 * r)
        rep = base.copy()
        for s in rep.sites:
            s.state = int(rng.integers(0, s.n_states))
        _apply_states(rep)
        out.append(rep)
    return out


def globule_10000() -> List[System]:
    return [make_system(3, 10000, 26.0)]


def uneven_batch_sizes(n_sys: int = 64):
    rng = rng_for(4)
    out = []
    for _ in range(n_sys):
        n = int(rng.integers(500, 20001))
        n_redox = int(rng.integers(2, 11))
        n_prot = int(rng.integers(0, 21))
        # site atoms capped at N/2: drop protonation sites first, then redox
        # sites, down to 2 redox sites (74 atoms each; protonation <= 20)
        while n_redox * 74 + n_prot * 20 > n // 2 and n_prot > 0:
            n_prot -= 1
        while n_redox * 74 > n // 2 and n_redox > 2:
            n_redox -= 1
        out.append((n, n_redox, n_prot))
    return out


def uneven_batch_64(n_sys: int = 64) -> List[System]:
    systems = []
    for b, (n, n_redox, n_prot) in enumerate(uneven_batch_sizes(n_sys)):
        r_glob = 18.0 * (n / 2500.0) ** (1.0 / 3.0)
        systems.append(make_system(4 + 1000 * b, n, r_glob, n_redox=n_redox, n_prot=n_prot,
                                   random_states=True))
    return systems


WORKLOADS = {"globule_256": globule_256, "globule_2500": globule_2500, "eremd_batch": eremd_batch,
             "globule_10000": globule_10000, "uneven_batch_64": uneven_batch_64}


def workload(name: str, **kw) -> List[System]:
    return WORKLOADS[name](**kw)


# --------------------------------------------------------------------------
# Flattened batch layout shared by both sides (pure data movement).
# --------------------------------------------------------------------------

@dataclass
class Batch:
    atom_offset: np.ndarray    # [B+1] int32
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    rho: np.ndarray
    screen: np.ndarray
    # site tables (CSR); atom indices are *global* (include atom_offset)
    site_system: np.ndarray        # [S] int32
    site_kind: np.ndarray          # [S] int32
    site_atom_offset: np.ndarray   # [S+1] int32
    site_atoms: np.ndarray         # [sum |A|] int32
    site_state_offset: np.ndarray  # [S+1] int32
    state_charge_offset: np.ndarray  # [n_states_total + 1] int32 into state_charges
    state_charges: np.ndarray      # float64
    state_count: np.ndarray        # [n_states_total] int32
    current_state: np.ndarray      # [S] int32

    @property
    def n_systems(self) -> int:
        return int(self.atom_offset.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.atom_offset[-1])

    @property
    def n_sites(self) -> int:
        return int(self.site_kind.shape[0])

    def n_candidates(self) -> int:
        ns = np.diff(self.site_state_offset)
        return int((ns - 1).sum())


def make_batch(systems: Sequence[System]) -> Batch:
    off = np.zeros(len(systems) + 1, dtype=np.int32)
    for b, s in enumerate(systems):
        off[b + 1] = off[b] + s.n
    cat = lambda name: np.concatenate([getattr(s, name) for s in systems]).astype(np.float64)
    site_system, site_kind, sao, satoms, sso, sco, sch, scount, cur = [], [], [0], [], [0], [0], [], [], []
    for b, s in enumerate(systems):
        for site in s.sites:
            site_system.append(b)
            site_kind.append(site.kind)
            satoms.extend((site.atoms + off[b]).tolist())
            sao.append(len(satoms))
            for t in range(site.n_states):
                sch.extend(site.charges[t].tolist())
                sco.append(len(sch))
                scount.append(int(site.counts[t]))
            sso.append(sso[-1] + site.n_states)
            cur.append(site.state)
    i32 = lambda v: np.asarray(v, dtype=np.int32)
    return Batch(off, cat("x"), cat("y"), cat("z"), cat("q"), cat("rho"), cat("screen"),
                 i32(site_system), i32(site_kind), i32(sao), i32(satoms), i32(sso), i32(sco),
                 np.asarray(sch, dtype=np.float64), i32(scount), i32(cur))


def uniforms(seed: int, shape) -> np.ndarray:
    """FP64 uniforms in [0, 1) for the Monte Carlo decisions (passed as inputs
    to both sides)."""
    return rng_for(seed).random(size=shape)


def normals(seed: int, shape) -> np.ndarray:
    """FP64 standard normal deviates (the Langevin noise; passed as inputs to
    both sides)."""
    return rng_for(seed).standard_normal(size=shape)


def masses(seed: int, n: int) -> np.ndarray:
    """Atomic masses in amu for the dynamics: heavy atoms only, uniform in
    [12, 16] (carbon to oxygen; hydrogens are folded into their heavy atoms, so
    the 2 fs step needs no bond constraints), FP32-representable."""
    return f32(rng_for(seed).uniform(12.0, 16.0, size=n))


def thermal_velocities(seed: int, m: np.ndarray, T: float = 300.0) -> np.ndarray:
    """Maxwell-Boltzmann velocities [n, 3] in A/ps (kB T / m per component,
    with 1 kcal/mol/amu = 418.4 A^2/ps^2)."""
    sd = np.sqrt(1.98720426e-3 * T * 418.4 / np.asarray(m, dtype=np.float64))
    return rng_for(seed).standard_normal(size=(len(m), 3)) * sd[:, None]
