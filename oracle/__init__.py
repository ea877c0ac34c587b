"""FP64 CPU oracle (ctypes binding of ``gb_oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the GPU
library ``paper_1803_09652_amd`` and never imports it.

Every function follows the plain definition in ``gb_oracle.c``: O(N^2) FP64
double loops, closed-form HCT/OBC/Still expressions, Eq. 8/9 for Delta G,
Eq. 14/15 for the replica exchange.  Pins against what the mathematics and the
paper fix live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

KB = 1.98720426e-3        # kcal/(mol K)
FARADAY = 23.0605478      # kcal/(mol V)
ACC = 418.4               # kcal/mol/(amu A) in A/ps^2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


class _Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("alpha", "beta", "gamma", "offset", "eps_in", "eps_out", "coulomb_k", "kappa",
                 "rgbmax", "cutoff")]


@dataclass(frozen=True)
class Params:
    """GB-OBC parameters.  Default: the OBC 'igb=5' set (alpha, beta, gamma =
    1.0, 0.8, 4.85), offset 0.09 A, eps_in 1, eps_out 78.5, k = 332.0522, no
    salt (kappa, the inverse Debye length in 1/A, = 0), no cutoffs (rgbmax: the
    descreening cutoff, cutoff: the pair cutoff of the energy terms, in A; 0 =
    none)."""
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

    def c(self) -> _Params:
        return _Params(self.alpha, self.beta, self.gamma, self.offset, self.eps_in,
                       self.eps_out, self.coulomb_k, self.kappa, self.rgbmax, self.cutoff)


IGB5 = Params()
IGB2 = Params(alpha=0.8, beta=0.0, gamma=2.909125)

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)
_I64 = C.POINTER(C.c_int64)


def _declare(L):
    L.or_hct.restype = C.c_double
    L.or_hct.argtypes = [C.c_double] * 3
    L.or_hct_grad.restype = None
    L.or_hct_grad.argtypes = [C.c_double] * 3 + [_D]
    L.or_hct_cut.restype = C.c_double
    L.or_hct_cut.argtypes = [C.c_double] * 4
    L.or_hct_cut_grad.restype = None
    L.or_hct_cut_grad.argtypes = [C.c_double] * 4 + [_D]
    xyz = [_D, _D, _D]
    L.or_radii.argtypes = [C.c_int] + xyz + [_D, _D, C.POINTER(_Params), _D, _D, _D, _D]
    L.or_energy_fixedR.argtypes = [C.c_int] + xyz + [_D, _D, C.POINTER(_Params), _D]
    L.or_phi_fixedR.argtypes = [C.c_int] + xyz + [_D, _D, C.POINTER(_Params), _D]
    L.or_energy_forces.argtypes = [C.c_int] + xyz + [_D, _D, _D, C.POINTER(_Params),
                                                     _D, _D, _D, _D, _D, _D]
    site_args = [C.c_int, _I, _I, _I, _I, _D, _I, _D]
    L.or_site_dE.argtypes = [C.c_int] + xyz + [_D, _D, C.POINTER(_Params)] + site_args
    L.or_site_dE_brute.argtypes = L.or_site_dE.argtypes
    L.or_delta_G.restype = C.c_double
    L.or_delta_G.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_double]
    L.or_metropolis.restype = C.c_int
    L.or_metropolis.argtypes = [C.c_double, C.c_double, C.c_double]
    mc = [C.c_int] + xyz + [_D, _D, C.POINTER(_Params), C.c_int, _I, _I, _I, _I, _I, _D, _D,
                            _I, _I, C.c_double, C.c_double, C.c_double, _D]
    L.or_mc_step.argtypes = mc + [_I, _D]
    L.or_mc_run.argtypes = [C.c_int] + mc + [_I64, _I64]
    L.or_mc_sweep.argtypes = mc[:-1] + [C.c_int, _D, _I, _D]
    L.or_langevin_step.restype = None
    L.or_langevin_step.argtypes = [C.c_int] + xyz + [_D, _D, _D, C.POINTER(_Params), _D, C.c_double,
                                                     _D, _D, _D, C.c_double, C.c_double, C.c_double]
    L.or_remd_exchange.restype = C.c_int
    L.or_remd_exchange.argtypes = [C.c_int, _D, _I, _I, C.c_double, C.c_int, C.c_int, _D, _I, _D]


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _pi(a):
    return a.ctypes.data_as(_I) if a is not None else None


# ---------------------------------------------------------------- pair terms

def hct(r: float, rt: float, S: float) -> float:
    return lib().or_hct(r, rt, S)


def hct_cut(r: float, rt: float, S: float, c: float) -> float:
    """H restricted to radius c around atom i (descreening cutoff)."""
    return lib().or_hct_cut(r, rt, S, c)


def hct_cut_grad(r: float, rt: float, S: float, c: float) -> np.ndarray:
    out = np.zeros(3)
    lib().or_hct_cut_grad(r, rt, S, c, _pd(out))
    return out


def hct_grad(r: float, rt: float, S: float) -> np.ndarray:
    out = np.zeros(3)
    lib().or_hct_grad(r, rt, S, _pd(out))
    return out


# ------------------------------------------------------------ one system

def _xyz(s):
    return _d(s.x), _d(s.y), _d(s.z)


def radii(s, p: Params = IGB5) -> dict:
    n = s.n
    x, y, z = _xyz(s)
    I, R, T, dR = (np.zeros(n) for _ in range(4))
    pc = p.c()
    lib().or_radii(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.rho)), _pd(_d(s.screen)), C.byref(pc),
                   _pd(I), _pd(R), _pd(T), _pd(dR))
    return dict(I=I, R=R, T=T, dRdPsi=dR)


def energy_forces(s, p: Params = IGB5) -> dict:
    """E_C, E_GB, forces F[n,3] = -dE/dx, phi = dE/dq, dEdrho, G = dE/dR, R."""
    n = s.n
    x, y, z = _xyz(s)
    E = np.zeros(2)
    F = np.zeros(3 * n)
    phi, dEdrho, G, R = (np.zeros(n) for _ in range(4))
    pc = p.c()
    lib().or_energy_forces(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.q)), _pd(_d(s.rho)),
                           _pd(_d(s.screen)), C.byref(pc), _pd(E), _pd(F), _pd(phi),
                           _pd(dEdrho), _pd(G), _pd(R))
    return dict(Ec=E[0], Egb=E[1], E=E[0] + E[1], F=F.reshape(3, n).T.copy(), phi=phi,
                dEdrho=dEdrho, G=G, R=R)


def energy(s, p: Params = IGB5) -> float:
    n = s.n
    x, y, z = _xyz(s)
    E = np.zeros(2)
    pc = p.c()
    lib().or_energy_forces(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.q)), _pd(_d(s.rho)),
                           _pd(_d(s.screen)), C.byref(pc), _pd(E), None, None, None, None, None)
    return float(E[0] + E[1])


def energy_fixedR(s, R, p: Params = IGB5, q=None) -> np.ndarray:
    n = s.n
    x, y, z = _xyz(s)
    E = np.zeros(2)
    pc = p.c()
    lib().or_energy_fixedR(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.q if q is None else q)),
                           _pd(_d(R)), C.byref(pc), _pd(E))
    return E


def phi_fixedR(s, R, p: Params = IGB5) -> np.ndarray:
    n = s.n
    x, y, z = _xyz(s)
    out = np.zeros(n)
    pc = p.c()
    lib().or_phi_fixedR(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.q)), _pd(_d(R)), C.byref(pc),
                        _pd(out))
    return out


class SiteTables:
    """Site CSR tables of one system with system-local atom indices."""

    def __init__(self, s, gref: Optional[np.ndarray] = None):
        sao, atoms, sso, sco, ch, cnt, kind, cur = [0], [], [0], [0], [], [], [], []
        for site in s.sites:
            atoms.extend(int(a) for a in site.atoms)
            sao.append(len(atoms))
            for t in range(site.n_states):
                ch.extend(site.charges[t].tolist())
                sco.append(len(ch))
                cnt.append(int(site.counts[t]))
            sso.append(sso[-1] + site.n_states)
            kind.append(site.kind)
            cur.append(site.state)
        self.n_sites = len(s.sites)
        self.site_atom_offset = _i(sao)
        self.site_atoms = _i(atoms)
        self.site_state_offset = _i(sso)
        self.state_charge_offset = _i(sco)
        self.state_charges = _d(ch)
        self.state_count = _i(cnt)
        self.site_kind = _i(kind)
        self.current_state = _i(cur)
        self.gref = _d(np.zeros(sso[-1]) if gref is None else gref)

    def n_candidates(self) -> int:
        return int((np.diff(self.site_state_offset) - 1).sum())

    def site_args(self):
        return (self.n_sites, _pi(self.site_atom_offset), _pi(self.site_atoms),
                _pi(self.site_state_offset), _pi(self.state_charge_offset),
                _pd(self.state_charges), _pi(self.current_state))


def site_dE(s, R, p: Params = IGB5, brute: bool = False, tables: SiteTables = None) -> np.ndarray:
    t = tables or SiteTables(s)
    n = s.n
    x, y, z = _xyz(s)
    out = np.zeros(t.n_candidates())
    pc = p.c()
    fn = lib().or_site_dE_brute if brute else lib().or_site_dE
    fn(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.q)), _pd(_d(R)), C.byref(pc), *t.site_args(), _pd(out))
    return out


def delta_G(kind: int, dE: float, n_new: int, n_old: int, gref_new: float, gref_old: float,
            pH: float, E_volt: float, T: float) -> float:
    return lib().or_delta_G(kind, dE, n_new, n_old, gref_new, gref_old, pH, E_volt, T)


def candidate_dG(s, dE: np.ndarray, tables: SiteTables, pH: float, E_volt: float,
                 T: float) -> np.ndarray:
    """Delta G for every candidate of one system, from its Delta E_elec."""
    out = np.zeros_like(dE)
    c = 0
    for m in range(tables.n_sites):
        g0 = int(tables.site_state_offset[m])
        ns = int(tables.site_state_offset[m + 1]) - g0
        cur = int(tables.current_state[m])
        for t in range(ns):
            if t == cur:
                continue
            out[c] = delta_G(int(tables.site_kind[m]), float(dE[c]),
                             int(tables.state_count[g0 + t]), int(tables.state_count[g0 + cur]),
                             float(tables.gref[g0 + t]), float(tables.gref[g0 + cur]),
                             pH, E_volt, T)
            c += 1
    return out


def metropolis(dG: float, T: float, u: float) -> bool:
    return bool(lib().or_metropolis(dG, T, u))


def _mc_args(s, R, p, t: SiteTables, q, pH, E_volt, T, u):
    x, y, z = _xyz(s)
    return [s.n, _pd(x), _pd(y), _pd(z), _pd(q), _pd(_d(R)), C.byref(p.c()), t.n_sites,
            _pi(t.site_kind), _pi(t.site_atom_offset), _pi(t.site_atoms),
            _pi(t.site_state_offset), _pi(t.state_charge_offset), _pd(t.state_charges),
            _pd(t.gref), _pi(t.state_count), _pi(t.current_state), pH, E_volt, T, _pd(u)]


def mc_step(s, R, tables: SiteTables, pH: float, E_volt: float, T: float, u,
            p: Params = IGB5, q: Optional[np.ndarray] = None):
    """One protonation + redox attempt pair.  Updates ``tables.current_state``
    and the returned charge vector.  Returns (q, out[4], dG[2])."""
    q = _d(s.q if q is None else q).copy()
    u = _d(u)
    out = np.zeros(4, dtype=np.int32)
    dG = np.zeros(2)
    args = _mc_args(s, R, p, tables, q, pH, E_volt, T, u)
    lib().or_mc_step(*args, _pi(out), _pd(dG))
    return q, out, dG


def mc_run(s, R, tables: SiteTables, pH: float, E_volt: float, T: float, u,
           p: Params = IGB5):
    """len(u) attempt pairs.  Returns (occupancy per state, accepted[2])."""
    u = _d(u)
    n_steps = u.shape[0]
    q = _d(s.q).copy()
    occ = np.zeros(int(tables.site_state_offset[-1]), dtype=np.int64)
    acc = np.zeros(2, dtype=np.int64)
    args = _mc_args(s, R, p, tables, q, pH, E_volt, T, u)
    lib().or_mc_run(n_steps, *args, occ.ctypes.data_as(_I64), acc.ctypes.data_as(_I64))
    return occ, acc


def mc_sweep(s, R, tables: SiteTables, pH: float, E_volt: float, T: float, u, kinds: int = 3,
             p: Params = IGB5, q: Optional[np.ndarray] = None):
    """One sequential sweep (every site of the kinds once; protonation first;
    random order by u[:, 0]); u[n_sites][3].  Updates ``tables.current_state``.
    Returns (q, accepted[n_sites] (1/0, -1 not attempted), dG[n_sites])."""
    q = _d(s.q if q is None else q).copy()
    u = _d(u)
    if u.shape != (tables.n_sites, 3):
        raise ValueError("u must be [n_sites, 3]")
    acc = np.zeros(tables.n_sites, dtype=np.int32)
    dG = np.zeros(tables.n_sites)
    args = _mc_args(s, R, p, tables, q, pH, E_volt, T, u)
    lib().or_mc_sweep(*args[:-1], int(kinds), _pd(u), _pi(acc), _pd(dG))
    return q, acc, dG


def remd_exchange(E_rung, Ne_of_rep, rep_of_rung, T: float, parity: int, wrap: bool, u):
    """Returns (new rep_of_rung, accepted flags per pair, E_of_rep)."""
    E_rung = _d(E_rung)
    M = E_rung.shape[0]
    rep = _i(rep_of_rung).copy()
    acc = np.zeros(M, dtype=np.int32)
    Eo = np.zeros(M)
    u = _d(u)
    if u.shape[0] < M:
        u = np.concatenate([u, np.ones(M - u.shape[0])])
    npairs = lib().or_remd_exchange(M, _pd(E_rung), _pi(_i(Ne_of_rep)), _pi(rep), T,
                                    int(parity), int(bool(wrap)), _pd(u), _pi(acc), _pd(Eo))
    return rep, acc[:npairs], Eo


def count_electrons(s, tables: SiteTables) -> int:
    """N_e of a system: the electron count of every redox site's current state."""
    n = 0
    for m in range(tables.n_sites):
        if tables.site_kind[m] == 1:
            n += int(tables.state_count[int(tables.site_state_offset[m]) + int(tables.current_state[m])])
    return n


def langevin_step(s, v, inv_mass, xi, dt: float, gamma: float, T: float, p: Params = IGB5,
                  xref=None, k_restr: float = 0.0):
    """One leapfrog Langevin step of system s (Loncharich, Brooks & Pastor
    1992) on the Coulomb + GB forces plus an optional harmonic restraint to
    xref [n, 3].  v and xi are [n, 3] (A/ps; standard normals), inv_mass [n]
    in 1/amu, dt in ps, gamma in 1/ps.  Returns (x, y, z, v) after the step;
    s is not modified."""
    n = s.n
    x, y, z = (a.copy() for a in _xyz(s))
    vv = _d(np.asarray(v, dtype=np.float64).T).copy()          # [3, n] component-major
    xr = None if xref is None else _d(np.asarray(xref, dtype=np.float64).T)
    pc = p.c()
    lib().or_langevin_step(n, _pd(x), _pd(y), _pd(z), _pd(_d(s.q)), _pd(_d(s.rho)),
                           _pd(_d(s.screen)), C.byref(pc), _pd(xr), float(k_restr), _pd(vv),
                           _pd(_d(inv_mass)), _pd(_d(np.asarray(xi, dtype=np.float64).T)),
                           float(dt), float(gamma), float(T))
    return x, y, z, vv.T.copy()
