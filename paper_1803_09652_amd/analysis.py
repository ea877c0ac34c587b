"""Post-processing of constant-redox / E-REMD runs (CPU, numpy/scipy): the
fraction of reduced species per redox potential, its fit to the Hill form of
the Nernst equation (Eq. 3), and the thermodynamic-cycle relations between
standard redox potentials and pKa values (Eqs. 16-18, section II.D).

Units: volt, kelvin; pKa and pH dimensionless; v is the number of electrons
of the redox reaction.
"""
from __future__ import annotations

import math

import numpy as np

KB = 1.98720426e-3        # kcal/(mol K)
FARADAY = 23.0605478      # kcal/(mol V)
LN10 = math.log(10.0)


def f_red(E, E0: float, n: float = 1.0, T: float = 300.0, v: int = 1):
    """Eq. 3: fraction reduced at redox potential E for standard potential E0
    and Hill coefficient n."""
    x = n * v * FARADAY * (np.asarray(E, dtype=np.float64) - E0) / (KB * T)
    return 1.0 / (1.0 + np.exp(np.clip(x, -700.0, 700.0)))


def fit_hill(E, fred, T: float = 300.0, v: int = 1, sigma=None):
    """Least-squares fit of Eq. 3 to (E, f_red) points; returns (E0, n, dE0,
    dn), the last two the standard errors of the fit (as the paper reports
    them).  sigma: optional per-point standard deviations of f_red."""
    from scipy.optimize import curve_fit

    E = np.asarray(E, dtype=np.float64)
    fred = np.asarray(fred, dtype=np.float64)
    # start from the logit line through the interior points
    inner = (fred > 1e-3) & (fred < 1 - 1e-3)
    if inner.sum() >= 2:
        lg = np.log(fred[inner] / (1 - fred[inner]))
        slope, icpt = np.polyfit(E[inner], lg, 1)
        n0 = max(abs(slope) * KB * T / (v * FARADAY), 0.05)
        E00 = -icpt / slope if slope != 0 else float(np.mean(E))
    else:
        n0, E00 = 1.0, float(np.mean(E))
    popt, pcov = curve_fit(lambda e, e0, n: f_red(e, e0, n, T, v), E, fred, p0=(E00, n0),
                           sigma=sigma, absolute_sigma=sigma is not None, maxfev=10000)
    err = np.sqrt(np.diag(pcov))
    return float(popt[0]), float(popt[1]), float(err[0]), float(err[1])


def e0_deprot(E0_prot: float, pka_red, pka_oxi, T: float = 300.0, v: int = 1) -> float:
    """Eq. 16 solved for the standard potential with every pH-active group
    deprotonated, from the one with all protonated and the pKa values of
    those groups with the redox group reduced / oxidised."""
    d = np.sum(np.asarray(pka_red, dtype=np.float64) - np.asarray(pka_oxi, dtype=np.float64))
    return E0_prot - KB * T * LN10 * d / (v * FARADAY)


def e0_of_ph(pH, E0_prot: float, pka_red, pka_oxi, T: float = 300.0, v: int = 1):
    """Eq. 17: the pH-dependent standard redox potential."""
    pH = np.asarray(pH, dtype=np.float64)[..., None]
    pr = np.asarray(pka_red, dtype=np.float64)
    po = np.asarray(pka_oxi, dtype=np.float64)
    # ln((10^-pKr + 10^-pH) / (10^-pKo + 10^-pH)) in a form that does not
    # overflow: ln10 * (logaddexp10 terms)
    num = np.logaddexp(-pr * LN10, -pH * LN10)
    den = np.logaddexp(-po * LN10, -pH * LN10)
    return E0_prot + KB * T / (v * FARADAY) * np.sum(num - den, axis=-1)


def sum_pka_of_e(E, sum_pka_red: float, E0_prot: float, E0_deprot: float, T: float = 300.0,
                 v: int = 1):
    """Eq. 18: the sum of the pH-active groups' pKa values at redox potential
    E (log is decimal)."""
    E = np.asarray(E, dtype=np.float64)
    b = 1.0 / (KB * T)
    num = np.logaddexp(-v * FARADAY * E0_prot * b, -FARADAY * E * b)
    den = np.logaddexp(-v * FARADAY * E0_deprot * b, -FARADAY * E * b)
    return sum_pka_red + (num - den) / LN10


def fraction_by_rung(state, rep_of_rung, site_system, site_kind, site_state_offset,
                     state_count, n_e_max=None):
    """Average reduced fraction per rung and per redox site of a replica.

    state [a, S] and rep_of_rung [a, B] are the loop's records (host arrays);
    the replicas are copies of one molecule, so site k of each replica is the
    same residue.  Returns f [B, K] with K redox sites per replica: the mean of
    n_e(state) / n_e_max over the samples of the replica sitting at rung l."""
    state = np.asarray(state)
    rep = np.asarray(rep_of_rung)
    site_system = np.asarray(site_system)
    site_kind = np.asarray(site_kind)
    sso = np.asarray(site_state_offset)
    cnt = np.asarray(state_count)
    B = rep.shape[1]
    redox = [np.flatnonzero((site_system == b) & (site_kind == 1)) for b in range(B)]
    K = len(redox[0])
    if any(len(r) != K for r in redox):
        raise ValueError("replicas must have the same redox sites")
    if K == 0:
        return np.zeros((B, 0))
    sites = np.stack(redox)                                   # [B, K]
    ne = cnt[sso[sites][None, :, :] + state[:, sites]]        # [a, B, K]
    if n_e_max is None:
        n_e_max = max(1, int(cnt.max()))
    # samples of rung l: the replica rep_of_rung[t, l] at time t
    by_rung = np.take_along_axis(ne, rep[:, :, None].astype(np.int64), axis=1)
    return by_rung.mean(axis=0) / n_e_max


def fit_e0_of_ph(pH, E0, n_groups: int = 1, T: float = 300.0, v: int = 1, guess=None):
    """Least-squares fit of Eq. 17 to standard potentials E0 measured at
    several pH (the analysis of Fig. 4).  Returns (E0_prot, pka_red[n],
    pka_oxi[n], residual rms).  guess: optional (E0_prot, pka_red, pka_oxi)."""
    from scipy.optimize import least_squares

    pH = np.asarray(pH, dtype=np.float64)
    E0 = np.asarray(E0, dtype=np.float64)
    n = int(n_groups)
    if guess is None:
        lo, hi = float(np.min(pH)), float(np.max(pH))
        mid = np.linspace(lo, hi, n + 2)[1:-1]
        guess = (float(E0[np.argmin(pH)]), mid + 0.5, mid - 0.5)
    x0 = np.concatenate([[guess[0]], np.atleast_1d(guess[1]), np.atleast_1d(guess[2])])

    def resid(x):
        return e0_of_ph(pH, x[0], x[1:1 + n], x[1 + n:], T, v) - E0

    r = least_squares(resid, x0, xtol=1e-14, ftol=1e-14, gtol=1e-14, max_nfev=20000)
    x = r.x
    return float(x[0]), x[1:1 + n].copy(), x[1 + n:].copy(), float(np.sqrt(np.mean(r.fun ** 2)))


def fit_pka_of_e(E, sum_pka, T: float = 300.0, v: int = 1, guess=None):
    """Least-squares fit of Eq. 18 to the summed pKa values measured at
    several redox potentials.  Returns (sum_pka_red, E0_prot, E0_deprot,
    residual rms)."""
    from scipy.optimize import least_squares

    E = np.asarray(E, dtype=np.float64)
    y = np.asarray(sum_pka, dtype=np.float64)
    if guess is None:
        guess = (float(y[np.argmin(E)]), float(np.mean(E)) + 0.03, float(np.mean(E)) - 0.03)

    def resid(x):
        return sum_pka_of_e(E, x[0], x[1], x[2], T, v) - y

    r = least_squares(resid, np.asarray(guess, dtype=np.float64), xtol=1e-14, ftol=1e-14,
                      gtol=1e-14, max_nfev=20000)
    return float(r.x[0]), float(r.x[1]), float(r.x[2]), float(np.sqrt(np.mean(r.fun ** 2)))
