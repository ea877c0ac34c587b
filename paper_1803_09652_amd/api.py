"""Python binding of libgbmc: torch tensors in, libgbmc calls, torch tensors out.

Every computation runs in the HIP kernels behind include/gbmc.h; this module
only checks shapes and dtypes, allocates output tensors and passes device
pointers plus the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

KIND_PROT = 0
KIND_REDOX = 1


@dataclass(frozen=True)
class GBParams:
    """GB-OBC parameters (default: the igb=5 set; see IGB2 for the paper's).
    kappa: inverse Debye length (1/A) of added salt; rgbmax: descreening
    cutoff (A); cutoff: pair cutoff of the energy terms (A); 0 = none."""
    alpha: float = 1.0
    beta: float = 0.8
    gamma: float = 4.85
    offset: float = 0.09
    eps_in: float = 1.0
    eps_out: float = 78.5
    coulomb_k: float = 332.0522
    kappa: float = 0.0
    rgbmax: float = 0.0
    cutoff: float = 0.0

    def c(self) -> L.gbmc_gb_params:
        return L.gbmc_gb_params(self.alpha, self.beta, self.gamma, self.offset, self.eps_in,
                                self.eps_out, self.coulomb_k, self.kappa, self.rgbmax,
                                self.cutoff)


IGB5 = GBParams()
IGB2 = GBParams(alpha=0.8, beta=0.0, gamma=2.909125)


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# the library's default work shapes (radii, energy, chain) per precision
# The library's default shapes for batches below its long-item size (a plan
# created without either knob takes the library's own choice, which for FP32
# batches of at least 2^19 tiles walks four j blocks per item with one wave per
# workgroup in the energy and chain passes); a knob left None when the other
# is given takes the value below.
DEFAULT_SHAPE = {"fp32": {"j_blocks_per_item": (1, 1, 1), "waves_per_group": (2, 4, 4)},
                 "fp64": {"j_blocks_per_item": (1, 1, 1), "waves_per_group": (2, 2, 2)}}


def _per_pass(v, default):
    if v is None:
        return tuple(default)
    if isinstance(v, (int, np.integer)):
        return (int(v),) * L.N_PASSES
    v = tuple(int(x) for x in v)
    if len(v) != L.N_PASSES:
        raise ValueError("give one value, or one per pass (radii, energy, chain)")
    return v


def tuning_struct(j_blocks_per_item=None, waves_per_group=None,
                  precision: str = "fp32") -> L.gbmc_tuning:
    """Work shape per pair pass; each argument is an int (all passes) or a
    (radii, energy, chain) triple; None keeps the library default."""
    jb = _per_pass(j_blocks_per_item, DEFAULT_SHAPE[precision]["j_blocks_per_item"])
    wv = _per_pass(waves_per_group, DEFAULT_SHAPE[precision]["waves_per_group"])
    t = L.gbmc_tuning()
    for k in range(L.N_PASSES):
        t.j_blocks_per_item[k] = jb[k]
        t.waves_per_group[k] = wv[k]
    return t


class Plan:
    """A batch layout (systems back to back) and a precision.

    precision: "fp32" (FP32 pair arithmetic, 64-bit fixed-point sums) or
    "fp64".  Owns the plan's device workspace."""

    def __init__(self, atom_offset: Sequence[int], precision: str = "fp32",
                 j_blocks_per_item=None, waves_per_group=None, device=None):
        lib = L.load()
        self.offset = np.ascontiguousarray(atom_offset, dtype=np.int32)
        if self.offset.ndim != 1 or self.offset.size < 1:
            raise ValueError("atom_offset must be a 1-D array of B+1 offsets")
        if precision not in ("fp32", "fp64"):
            raise ValueError("precision must be 'fp32' or 'fp64'")
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        tun = None
        if j_blocks_per_item is not None or waves_per_group is not None:
            tun = C.byref(tuning_struct(j_blocks_per_item, waves_per_group, precision))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.gbmc_plan_create(C.byref(h), int(self.offset.size - 1), _i32p(self.offset),
                                         L.GBMC_FP32_FIXED if precision == "fp32" else L.GBMC_FP64,
                                         tun))
        self._h = h
        nbytes = int(lib.gbmc_plan_workspace_bytes(h))
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        self.atom_sys = torch.repeat_interleave(
            torch.arange(self.n_systems, device=self.device),
            torch.as_tensor(np.diff(self.offset).astype(np.int64), device=self.device))

    @property
    def handle(self):
        return self._h

    @property
    def n_systems(self) -> int:
        return int(self.offset.size - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.offset[-1])

    def set_order(self, order) -> None:
        """Processing order of the pair passes (a permutation of each system's
        atom range); see spatial_order()."""
        o = np.ascontiguousarray(order, dtype=np.int32)
        if o.shape != (self.n_atoms,):
            raise ValueError("order must have one entry per atom")
        with torch.cuda.device(self.device):
            L.check(L.load().gbmc_plan_set_order(self._h, _i32p(o)))

    def set_single_launch(self, enable: bool = True, wait_polls: int = 1 << 22) -> None:
        """evaluate() as one kernel launch of the three pair passes (with
        bounded dependency waits of wait_polls polls; 0 gives up at once, for
        tests) instead of one launch per pass (the default, faster here)."""
        L.check(L.load().gbmc_plan_set_single_launch(self._h, int(bool(enable)), int(wait_polls)))

    def set_timing(self, enable: bool = True) -> None:
        """Time each hot-path kernel of later eager calls (HIP events bound to
        the dispatch).  Disable before capturing a graph."""
        L.check(L.load().gbmc_plan_set_timing(self._h, int(bool(enable))))

    def kernel_ms(self) -> dict:
        """Duration (ms) of the most recent launch of each timed kernel."""
        ms = (C.c_float * len(L.KERNEL_NAMES))()
        L.check(L.load().gbmc_plan_kernel_ms(self._h, ms))
        return {n: float(v) for n, v in zip(L.KERNEL_NAMES, ms) if v >= 0.0}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().gbmc_plan_destroy(h)
            except Exception:
                pass
            self._h = None


class Atoms:
    """Per-atom SoA device tensors of one plan's dtype."""

    def __init__(self, plan: Plan, x, y, z, q, rho, screen):
        def dev(a):
            t = torch.as_tensor(a, dtype=plan.dtype, device=plan.device)
            t = t.contiguous()
            if t.ndim != 1 or t.shape[0] != plan.n_atoms:
                raise ValueError("atom arrays must be 1-D with one entry per atom")
            return t
        self.x, self.y, self.z = dev(x), dev(y), dev(z)
        self.q, self.rho, self.screen = dev(q), dev(rho), dev(screen)

    @classmethod
    def from_batch(cls, plan: Plan, batch) -> "Atoms":
        return cls(plan, batch.x, batch.y, batch.z, batch.q, batch.rho, batch.screen)

    def c(self, q: Optional[torch.Tensor] = None) -> L.gbmc_atoms:
        return L.gbmc_atoms(self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(),
                            (self.q if q is None else q).data_ptr(), self.rho.data_ptr(),
                            self.screen.data_ptr())


def spatial_order(atom_offset, x, y, z) -> np.ndarray:
    """Morton order of each system's atoms (host computation in libgbmc)."""
    off = np.ascontiguousarray(atom_offset, dtype=np.int32)
    f64 = lambda v: np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    xs, ys, zs = f64(x), f64(y), f64(z)
    out = np.zeros(int(off[-1]), dtype=np.int32)
    L.check(L.load().gbmc_spatial_order(int(off.size - 1), _i32p(off), _f64p(xs), _f64p(ys),
                                        _f64p(zs), _i32p(out)))
    return out


def block_order(atom_offset, x, y, z) -> np.ndarray:
    """Order of each system's atoms in compact 64-atom clusters (recursive
    bisection; host computation in libgbmc), for Plan.set_order."""
    off = np.ascontiguousarray(atom_offset, dtype=np.int32)
    f64 = lambda v: np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    xs, ys, zs = f64(x), f64(y), f64(z)
    out = np.zeros(int(off[-1]), dtype=np.int32)
    L.check(L.load().gbmc_block_order(int(off.size - 1), _i32p(off), _f64p(xs), _f64p(ys),
                                      _f64p(zs), _i32p(out)))
    return out


def _workspace(plan: Plan, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    if workspace is None:
        return plan.workspace
    if (workspace.dtype != torch.uint8 or workspace.numel() < plan.workspace.numel()
            or workspace.device != plan.device or workspace.data_ptr() % 256):
        raise ValueError("workspace must be a 256-byte aligned uint8 tensor of at least "
                         "plan.workspace.numel() bytes on the plan's device")
    return workspace


def radii(plan: Plan, atoms: Atoms, params: GBParams = IGB5,
          workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Effective Born radii R[N] (plan dtype); leaves the per-atom state in the
    workspace (default: the plan's) for energy_forces and mc_state_dE."""
    R = torch.empty(plan.n_atoms, dtype=plan.dtype, device=plan.device)
    a, p = atoms.c(), params.c()
    ws = _workspace(plan, workspace)
    L.check(L.load().gb_radii(plan.handle, C.byref(a), C.byref(p), _ptr(ws), _ptr(R),
                              _stream(plan.device)))
    return R


def energy_forces(plan: Plan, atoms: Atoms, params: GBParams = IGB5, force: bool = True,
                  dEdq: bool = True, dEdrho: bool = True,
                  workspace: Optional[torch.Tensor] = None) -> dict:
    """E_C and E_GB per system (float64 [B]) and the requested gradients.
    Needs a preceding radii() on the same plan, atoms and workspace."""
    dev, dt, n = plan.device, plan.dtype, plan.n_atoms
    out = {
        "e_coul": torch.empty(plan.n_systems, dtype=torch.float64, device=dev),
        "e_gb": torch.empty(plan.n_systems, dtype=torch.float64, device=dev),
        "force": torch.empty((n, 3), dtype=dt, device=dev) if force else None,
        "dEdq": torch.empty(n, dtype=dt, device=dev) if dEdq else None,
        "dEdrho": torch.empty(n, dtype=dt, device=dev) if dEdrho else None,
    }
    a, p = atoms.c(), params.c()
    ws = _workspace(plan, workspace)
    L.check(L.load().gb_energy_forces(plan.handle, C.byref(a), C.byref(p), _ptr(ws),
                                      _ptr(out["e_coul"]), _ptr(out["e_gb"]), _ptr(out["force"]),
                                      _ptr(out["dEdq"]), _ptr(out["dEdrho"]),
                                      _stream(plan.device)))
    return out


def _eval_outputs(plan: Plan, force: bool, dEdq: bool, dEdrho: bool) -> dict:
    dev, dt, n = plan.device, plan.dtype, plan.n_atoms
    return {
        "R": torch.empty(n, dtype=dt, device=dev),
        "e_coul": torch.empty(plan.n_systems, dtype=torch.float64, device=dev),
        "e_gb": torch.empty(plan.n_systems, dtype=torch.float64, device=dev),
        "force": torch.empty((n, 3), dtype=dt, device=dev) if force else None,
        "dEdq": torch.empty(n, dtype=dt, device=dev) if dEdq else None,
        "dEdrho": torch.empty(n, dtype=dt, device=dev) if dEdrho else None,
    }


def evaluate(plan: Plan, atoms: Atoms, params: GBParams = IGB5, force: bool = True,
             dEdq: bool = True, dEdrho: bool = True,
             workspace: Optional[torch.Tensor] = None,
             fork: Optional[torch.cuda.Stream] = None) -> dict:
    """One full evaluation (gb_evaluate): Born radii R, E_C and E_GB per
    system and the requested gradients; leaves the per-atom state in the
    workspace (default: the plan's) for the Monte Carlo calls.  With `fork`
    (another stream; gb_evaluate_fork) that stream waits only until the radii
    are final, so Monte Carlo work queued on it afterwards overlaps the energy
    and force passes; rejoin it (wait_stream) before using the outputs there."""
    out = _eval_outputs(plan, force, dEdq, dEdrho)
    a, p = atoms.c(), params.c()
    ws = _workspace(plan, workspace)
    args = (plan.handle, C.byref(a), C.byref(p), _ptr(ws), _ptr(out["R"]), _ptr(out["e_coul"]),
            _ptr(out["e_gb"]), _ptr(out["force"]), _ptr(out["dEdq"]), _ptr(out["dEdrho"]),
            _stream(plan.device))
    if fork is None:
        L.check(L.load().gb_evaluate(*args))
    else:
        L.check(L.load().gb_evaluate_fork(*args, C.c_void_p(fork.cuda_stream)))
    return out


def evaluate_static(plan: Plan, atoms: Atoms, params: GBParams = IGB5, force: bool = True,
                    dEdq: bool = True, dEdrho: bool = True, out: Optional[dict] = None) -> dict:
    """gb_evaluate_static: the same evaluation in the library's static scratch
    (the call allocates no device memory).  `out` may hold preallocated
    output tensors (keys as returned) so that the call allocates nothing on
    the torch side either."""
    o = out if out is not None else _eval_outputs(plan, force, dEdq, dEdrho)
    a, p = atoms.c(), params.c()
    L.check(L.load().gb_evaluate_static(plan.handle, C.byref(a), C.byref(p), _ptr(o["R"]),
                                        _ptr(o["e_coul"]), _ptr(o["e_gb"]), _ptr(o["force"]),
                                        _ptr(o["dEdq"]), _ptr(o["dEdrho"]),
                                        _stream(plan.device)))
    return o


class Sites:
    """Titratable-site tables of a plan (static), with the site workspace.

    Arrays follow include/gbmc.h (global atom indices); a ``synth.Batch``
    carries them under the same names."""

    def __init__(self, plan: Plan, site_system, site_kind, site_atom_offset, site_atoms,
                 site_state_offset, state_charge_offset, state_charges, state_gref, state_count):
        lib = L.load()
        i32 = lambda v: np.ascontiguousarray(v, dtype=np.int32)
        f64 = lambda v: np.ascontiguousarray(v, dtype=np.float64)
        self.site_system = i32(site_system)
        self.site_kind = i32(site_kind)
        self.site_atom_offset = i32(site_atom_offset)
        self.site_atoms = i32(site_atoms)
        self.site_state_offset = i32(site_state_offset)
        self.state_charge_offset = i32(state_charge_offset)
        self.state_charges = f64(state_charges)
        self.state_gref = f64(state_gref)
        self.state_count = i32(state_count)
        self.plan = plan
        h = C.c_void_p()
        with torch.cuda.device(plan.device):
            L.check(lib.gbmc_sites_create(plan.handle, C.byref(h), int(self.site_kind.size),
                                          _i32p(self.site_system), _i32p(self.site_kind),
                                          _i32p(self.site_atom_offset), _i32p(self.site_atoms),
                                          _i32p(self.site_state_offset),
                                          _i32p(self.state_charge_offset),
                                          _f64p(self.state_charges), _f64p(self.state_gref),
                                          _i32p(self.state_count)))
        self._h = h
        self.n_sites = int(self.site_kind.size)
        self.n_candidates = int(lib.gbmc_sites_n_candidates(h))
        nbytes = int(lib.gbmc_sites_workspace_bytes(h))
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=plan.device)

    @classmethod
    def from_batch(cls, plan: Plan, batch, state_gref=None) -> "Sites":
        gref = np.zeros(batch.state_count.size) if state_gref is None else state_gref
        return cls(plan, batch.site_system, batch.site_kind, batch.site_atom_offset,
                   batch.site_atoms, batch.site_state_offset, batch.state_charge_offset,
                   batch.state_charges, gref, batch.state_count)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().gbmc_sites_destroy(h)
            except Exception:
                pass
            self._h = None


def _dev_f64(v, n, device):
    t = torch.as_tensor(v, dtype=torch.float64, device=device)
    if t.ndim == 0:
        t = t.expand(n)
    return t.contiguous()


def mc_state_dE(plan: Plan, sites: Sites, atoms: Atoms, current_state: torch.Tensor, pH, E_volt,
                T: float = 300.0, params: GBParams = IGB5, with_dG: bool = True):
    """Delta E_elec and Delta G (float64 [n_candidates]) of every candidate
    state change.  Needs a preceding radii() on the same plan and atoms."""
    dev = plan.device
    dE = torch.empty(sites.n_candidates, dtype=torch.float64, device=dev)
    dG = torch.empty(sites.n_candidates, dtype=torch.float64, device=dev) if with_dG else None
    pH_t = _dev_f64(pH, plan.n_systems, dev)
    E_t = _dev_f64(E_volt, plan.n_systems, dev)
    if current_state.dtype != torch.int32 or current_state.device != dev:
        raise ValueError("current_state must be an int32 tensor on the plan's device")
    a, p = atoms.c(), params.c()
    L.check(L.load().mc_state_dE(plan.handle, sites.handle, C.byref(a), C.byref(p),
                                 _ptr(plan.workspace), _ptr(sites.workspace), _ptr(current_state),
                                 _ptr(pH_t), _ptr(E_t), float(T), _ptr(dE), _ptr(dG),
                                 _stream(dev)))
    return dE, dG


def mc_step(plan: Plan, sites: Sites, atoms: Atoms, current_state: torch.Tensor, pH, E_volt,
            dE: torch.Tensor, dG: torch.Tensor, u: torch.Tensor, T: float = 300.0,
            params: GBParams = IGB5, counters: Optional[torch.Tensor] = None,
            q_out: Optional[torch.Tensor] = None) -> dict:
    """One protonation + redox attempt pair per system; updates current_state
    in place and writes the accepted states' site charges into q_out (default
    atoms.q).  Only those charges are written, so a separate q_out must already
    hold the other charges (a copy of atoms.q)."""
    dev = plan.device
    q_dst = atoms.q if q_out is None else q_out
    if q_dst.dtype != plan.dtype or q_dst.shape != (plan.n_atoms,) or not q_dst.is_contiguous():
        raise ValueError("q_out must be a contiguous [N] tensor of the plan dtype")
    if u.dtype != torch.float64 or u.shape != (plan.n_systems, 6):
        raise ValueError("u must be float64 [B, 6]")
    pH_t = _dev_f64(pH, plan.n_systems, dev)
    E_t = _dev_f64(E_volt, plan.n_systems, dev)
    ne = torch.empty(plan.n_systems, dtype=torch.int32, device=dev)
    acc = torch.empty((plan.n_systems, 2), dtype=torch.int32, device=dev)
    a, p = atoms.c(), params.c()
    L.check(L.load().mc_step(plan.handle, sites.handle, C.byref(a), _ptr(q_dst), C.byref(p),
                             _ptr(plan.workspace), _ptr(sites.workspace), _ptr(current_state),
                             _ptr(pH_t), _ptr(E_t), float(T), _ptr(dE), _ptr(dG),
                             _ptr(u.contiguous()), _ptr(ne), _ptr(counters), _ptr(acc),
                             _stream(dev)))
    return {"n_electrons": ne, "accepted": acc}


def mc_sweep(plan: Plan, sites: Sites, atoms: Atoms, current_state: torch.Tensor, pH, E_volt,
             u: torch.Tensor, T: float = 300.0, params: GBParams = IGB5, kinds: int = 3,
             counters: Optional[torch.Tensor] = None,
             q_out: Optional[torch.Tensor] = None) -> dict:
    """One sequential sweep per system: every site of the kinds (bit 0
    protonation, bit 1 redox) attempted once, protonation first, each kind in
    the random order of ascending u[:, 0]; u is float64 [n_sites, 3].
    Updates current_state in place and writes accepted site charges into q_out
    (default atoms.q).  Needs a preceding radii() on the same plan and atoms.
    Returns n_electrons [B], accepted [n_sites] (1/0, -1 for sites of kinds not
    swept) and dG [n_sites] of each attempt."""
    dev = plan.device
    if u.dtype != torch.float64 or u.shape != (sites.n_sites, 3):
        raise ValueError("u must be float64 [n_sites, 3]")
    q_dst = atoms.q if q_out is None else q_out
    if q_dst.dtype != plan.dtype or q_dst.shape != (plan.n_atoms,) or not q_dst.is_contiguous():
        raise ValueError("q_out must be a contiguous [N] tensor of the plan dtype")
    pH_t = _dev_f64(pH, plan.n_systems, dev)
    E_t = _dev_f64(E_volt, plan.n_systems, dev)
    ne = torch.empty(plan.n_systems, dtype=torch.int32, device=dev)
    acc = torch.full((max(sites.n_sites, 1),), -1, dtype=torch.int32, device=dev)
    dG = torch.zeros(max(sites.n_sites, 1), dtype=torch.float64, device=dev)
    a, p = atoms.c(), params.c()
    L.check(L.load().mc_sweep(plan.handle, sites.handle, C.byref(a), _ptr(q_dst), C.byref(p),
                              _ptr(plan.workspace), _ptr(sites.workspace), _ptr(current_state),
                              _ptr(pH_t), _ptr(E_t), float(T), int(kinds), _ptr(u.contiguous()),
                              _ptr(ne), _ptr(counters), _ptr(acc), _ptr(dG), _stream(dev)))
    return {"n_electrons": ne, "accepted": acc[:sites.n_sites], "dG": dG[:sites.n_sites]}


def plain_fp64(atom_offset, x, y, z, q, rho, screen, params: GBParams = IGB5,
               device=None) -> dict:
    """The plain FP64 GPU form of one full evaluation (one thread per atom
    over its whole row, closed forms with correctly rounded operations): the
    reference the batched forms' pair rate is compared with.  Inputs are 1-D
    float64 device tensors (or arrays) in caller order; returns R, e_coul,
    e_gb, force [N, 3], dEdq and dEdrho."""
    off = np.ascontiguousarray(atom_offset, dtype=np.int32)
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    xs, ys, zs, qs, rs, ss = (d(a) for a in (x, y, z, q, rho, screen))
    B, N = int(off.size - 1), int(off[-1])
    lib = L.load()
    ws = torch.empty(max(int(lib.gb_plain_workspace_bytes(N)), 256), dtype=torch.uint8, device=dev)
    off_d = torch.as_tensor(off, device=dev)
    out = {"R": torch.empty(N, dtype=torch.float64, device=dev),
           "e_coul": torch.empty(B, dtype=torch.float64, device=dev),
           "e_gb": torch.empty(B, dtype=torch.float64, device=dev),
           "force": torch.empty((N, 3), dtype=torch.float64, device=dev),
           "dEdq": torch.empty(N, dtype=torch.float64, device=dev),
           "dEdrho": torch.empty(N, dtype=torch.float64, device=dev)}
    a = L.gbmc_atoms(xs.data_ptr(), ys.data_ptr(), zs.data_ptr(), qs.data_ptr(), rs.data_ptr(),
                     ss.data_ptr())
    p = params.c()
    L.check(lib.gb_plain_fp64(B, _i32p(off), _ptr(off_d), C.byref(a), C.byref(p), _ptr(ws),
                              _ptr(out["R"]), _ptr(out["e_coul"]), _ptr(out["e_gb"]),
                              _ptr(out["force"]), _ptr(out["dEdq"]), _ptr(out["dEdrho"]),
                              _stream(dev)))
    out["_keep"] = (xs, ys, zs, qs, rs, ss, ws, off_d)     # inputs live until the call finishes
    return out


def md_step(plan: Plan, atoms: Atoms, v: torch.Tensor, force: torch.Tensor,
            inv_mass: torch.Tensor, xi: torch.Tensor, dt: float, gamma: float, T: float = 300.0,
            xref: Optional[torch.Tensor] = None, k_restr: float = 0.0) -> None:
    """One leapfrog Langevin step (Loncharich, Brooks & Pastor 1992) of every
    atom: atoms.x/y/z and v [3, N] (A/ps) are updated in place from force
    [N, 3] (kcal/mol/A, e.g. energy_forces()["force"]), inv_mass [N] (1/amu),
    standard normals xi [3, N] and an optional harmonic restraint to xref
    [3, N] (k_restr kcal/mol/A^2); dt in ps, gamma in 1/ps."""
    n, dt_ = plan.n_atoms, plan.dtype

    def chk(t, shape, name):
        if t.dtype != dt_ or tuple(t.shape) != shape or not t.is_contiguous() or t.device != plan.device:
            raise ValueError(f"{name} must be a contiguous {dt_} tensor {shape} on the plan's device")
    chk(v, (3, n), "v")
    chk(force, (n, 3), "force")
    chk(inv_mass, (n,), "inv_mass")
    chk(xi, (3, n), "xi")
    if xref is not None:
        chk(xref, (3, n), "xref")
    L.check(L.load().md_langevin_step(plan.handle, _ptr(atoms.x), _ptr(atoms.y), _ptr(atoms.z),
                                      _ptr(v), _ptr(force), _ptr(inv_mass), _ptr(xi), _ptr(xref),
                                      float(k_restr), float(dt), float(gamma), float(T),
                                      _stream(plan.device)))


def remd_exchange(E_rung: torch.Tensor, Ne_of_rep: torch.Tensor, rep_of_rung: torch.Tensor,
                  parity: int, u: torch.Tensor, T: float = 300.0, wrap: bool = True,
                  E_out: Optional[torch.Tensor] = None):
    """E-REMD exchange attempt; rep_of_rung (int32) is updated in place.
    Returns (accepted[n_pairs] int32, E_of_rep[M] float64); E_of_rep is
    written into E_out when given (it may be the caller's per-replica E)."""
    M = int(E_rung.shape[0])
    dev = E_rung.device
    acc = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
    if E_out is not None and (E_out.dtype != torch.float64 or E_out.shape != (M,)
                              or not E_out.is_contiguous()):
        raise ValueError("E_out must be a contiguous float64 [M] tensor")
    Eo = torch.empty(M, dtype=torch.float64, device=dev) if E_out is None else E_out
    L.check(L.load().remd_exchange(M, _ptr(E_rung), _ptr(Ne_of_rep), _ptr(rep_of_rung), float(T),
                                   int(parity), int(bool(wrap)), _ptr(u), _ptr(acc), _ptr(Eo),
                                   _stream(dev)))
    inner = (M - parity) // 2
    n_pairs = inner + (1 if (parity == 1 and wrap and M % 2 == 0 and M > 2) else 0)
    return acc[:n_pairs], Eo


def check_overflow(plan: Plan, workspace: Optional[torch.Tensor] = None,
                   static: bool = False) -> bool:
    """True if, since the last radii() on the workspace (default: the plan's;
    static=True: the static scratch of evaluate_static), a fixed-point
    accumulator overflowed or a dependency wait of a queued launch gave up
    (the results are then not valid); reading clears the flags."""
    flag = C.c_int32(0)
    ws = None if static else _ptr(_workspace(plan, workspace))
    st = L.load().gbmc_check_overflow(plan.handle, ws, _stream(plan.device), C.byref(flag))
    if st != L.GBMC_OK and not flag.value:
        L.check(st)
    return bool(flag.value)


class GBEnergy(torch.autograd.Function):
    """E = E_C + E_GB per system (float64 [B]) as a differentiable function of
    positions [N, 3], charges [N] and intrinsic radii [N] (screens fixed).

    forward runs the radii pass and the energy-only pair pass in a workspace
    of its own, which keeps the per-atom radius state (R, tanh theta,
    dR/dPsi, the descreening sums) for backward; backward runs only the
    hand-written gradient passes on that state (the energy / explicit force
    pair pass giving G = dE/dR and phi = dE/dq, then the Born-radius chain pass
    and dE/drho), never the radii pass again."""

    @staticmethod
    def forward(ctx, pos, q, rho, screen, plan: Plan, params: GBParams = IGB5):
        pos_d, q_d, rho_d, scr_d = (t.detach() for t in (pos, q, rho, screen))
        atoms = Atoms(plan, pos_d[:, 0], pos_d[:, 1], pos_d[:, 2], q_d, rho_d, scr_d)
        ws = torch.empty_like(plan.workspace)
        radii(plan, atoms, params, workspace=ws)
        out = energy_forces(plan, atoms, params, force=False, dEdq=False, dEdrho=False,
                            workspace=ws)
        ctx.plan, ctx.params, ctx.atoms, ctx.ws = plan, params, atoms, ws
        return out["e_coul"] + out["e_gb"]

    @staticmethod
    def backward(ctx, gE):
        plan, params, atoms, ws = ctx.plan, ctx.params, ctx.atoms, ctx.ws
        g = energy_forces(plan, atoms, params, force=ctx.needs_input_grad[0],
                          dEdq=ctx.needs_input_grad[1], dEdrho=ctx.needs_input_grad[2],
                          workspace=ws)
        w = gE.to(plan.dtype)[plan.atom_sys]
        gpos = -g["force"] * w[:, None] if g["force"] is not None else None
        gq = g["dEdq"] * w if g["dEdq"] is not None else None
        grho = g["dEdrho"] * w if g["dEdrho"] is not None else None
        return gpos, gq, grho, None, None, None
