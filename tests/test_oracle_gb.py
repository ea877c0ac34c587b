"""Pins of the oracle's Born radii, GB+Coulomb energy and gradients.

Each test fixes a value the physics or mathematics determines without the
oracle: the Born energy of a single ion, the far-field and coincident limits of
a pair, invariances, zero net force and torque, and central finite differences
of the oracle's own energy (which is itself pinned by the limits above).
"""
import math

import mpmath
import numpy as np
import pytest

import synth

K = 332.0522


def one_system(xyz, q, rho, screen):
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    return synth.System(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(),
                        np.asarray(q, float), np.asarray(rho, float), np.asarray(screen, float))


@pytest.fixture(scope="module")
def c0():
    return synth.globule_256()[0]


@pytest.mark.parametrize("pname", ["IGB5", "IGB2"])
@pytest.mark.parametrize("q,rho,eps_in", [(1.0, 1.5, 1.0), (-0.7, 2.0, 1.0), (0.4, 1.2, 2.0)])
def test_single_ion_born_energy(orc, pname, q, rho, eps_in):
    p = getattr(orc, pname)
    p = orc.Params(p.alpha, p.beta, p.gamma, p.offset, eps_in, p.eps_out, p.coulomb_k)
    s = one_system([0, 0, 0], [q], [rho], [0.8])
    r = orc.energy_forces(s, p)
    a = rho - 0.09                     # isolated atom: Psi = 0 so R = rho - offset
    born = -0.5 * K * (1.0 / eps_in - 1.0 / 78.5) * q * q / a
    assert r["Ec"] == 0.0
    assert abs(r["Egb"] - born) <= 1e-13 * abs(born)
    assert abs(r["R"][0] - a) <= 1e-15


def test_pair_far_field_limit(orc):
    # at large r, f_GB -> r and the pair energy tends to k q1 q2 / (eps_out r);
    # screens 0 keep the self terms exact (no descreening)
    q1, q2 = 0.8, -0.55
    for r in (30.0, 200.0, 1000.0):
        s = one_system([[0, 0, 0], [r, 0, 0]], [q1, q2], [1.5, 1.7], [0.0, 0.0])
        e = orc.energy_forces(s)
        a1, a2 = 1.5 - 0.09, 1.7 - 0.09
        selfs = -0.5 * K * (1 - 1 / 78.5) * (q1 * q1 / a1 + q2 * q2 / a2)
        pair = e["E"] - selfs
        ref = K * q1 * q2 / (78.5 * r)
        assert abs(pair - ref) <= 1e-13 * abs(selfs)   # rounding of the subtraction


def test_pair_coincident_limit(orc):
    # screens 0 switch descreening off; at r -> 0 with equal radii the GB part
    # tends to the Born energy of one ion carrying q1 + q2
    q1, q2, rho = 0.3, 0.45, 1.6
    s = one_system([[0, 0, 0], [1e-6, 0, 0]], [q1, q2], [rho, rho], [0.0, 0.0])
    e = orc.energy_forces(s)
    a = rho - 0.09
    ref = -0.5 * K * (1 - 1 / 78.5) * (q1 + q2) ** 2 / a
    assert abs(e["Egb"] - ref) <= 1e-10 * abs(ref)


def test_two_atom_energy_against_50_digit_evaluation(orc):
    # Born radii from 50-digit shell quadrature of the descreening integral,
    # then Still's pair function; compared with the FP64 closed-form oracle.
    mpmath.mp.dps = 50
    from test_oracle_hct import H_mp
    r, q1, q2, rho1, rho2, s1, s2 = 3.1, 0.6, -0.4, 1.55, 1.8, 0.79, 0.86
    p = orc.IGB5
    rt1, rt2 = mpmath.mpf(rho1) - mpmath.mpf("0.09"), mpmath.mpf(rho2) - mpmath.mpf("0.09")
    S1, S2 = s1 * rt1, s2 * rt2
    psi1 = rt1 * H_mp(r, rt1, S2)
    psi2 = rt2 * H_mp(r, rt2, S1)

    def R_of(psi, rt, rho):
        th = p.alpha * psi - p.beta * psi ** 2 + p.gamma * psi ** 3
        return 1 / (1 / rt - mpmath.tanh(th) / rho)

    R1, R2 = R_of(psi1, rt1, rho1), R_of(psi2, rt2, rho2)
    f = mpmath.sqrt(r * r + R1 * R2 * mpmath.exp(-r * r / (4 * R1 * R2)))
    tau = 1 - mpmath.mpf(1) / mpmath.mpf("78.5")
    egb = -K * tau / 2 * (q1 * q1 / R1 + q2 * q2 / R2 + 2 * q1 * q2 / f)
    ec = K * q1 * q2 / r
    s = one_system([[0, 0, 0], [r, 0, 0]], [q1, q2], [rho1, rho2], [s1, s2])
    e = orc.energy_forces(s)
    assert abs(e["Egb"] - float(egb)) <= 1e-12 * abs(float(egb))
    assert abs(e["Ec"] - float(ec)) <= 1e-14 * abs(float(ec))


@pytest.mark.parametrize("pname", ["IGB5", "IGB2"])
def test_born_radius_bounds(orc, c0, pname):
    p = getattr(orc, pname)
    r = orc.radii(c0, p)
    rt = c0.rho - 0.09
    assert np.all(r["I"] > 0)
    assert np.all(r["R"] >= rt * (1 - 1e-15))
    assert np.all(r["R"] <= rt * c0.rho / 0.09)


def test_radius_grows_with_burial(orc):
    s1 = one_system([[0, 0, 0]], [0.0], [1.5], [0.8])
    s2 = one_system([[0, 0, 0], [3.0, 0, 0]], [0.0, 0.0], [1.5, 1.5], [0.8, 0.8])
    s3 = one_system([[0, 0, 0], [3.0, 0, 0], [-3.0, 0, 0]], [0.0] * 3, [1.5] * 3, [0.8] * 3)
    R1 = orc.radii(s1)["R"][0]
    R2 = orc.radii(s2)["R"][0]
    R3 = orc.radii(s3)["R"][0]
    assert R1 < R2 < R3


def _rotation(seed):
    rng = np.random.default_rng(seed)
    qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def _moved(s, xyz):
    out = s.copy()
    out.x, out.y, out.z = xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy()
    return out


def test_invariance_translation_rotation_permutation(orc, c0):
    base = orc.energy_forces(c0)
    xyz = c0.coords()
    # translation
    t = orc.energy_forces(_moved(c0, xyz + np.array([13.0, -7.5, 2.25])))
    assert abs(t["E"] - base["E"]) <= 1e-12 * abs(base["E"])
    assert np.abs(t["F"] - base["F"]).max() <= 1e-10 * np.abs(base["F"]).max()
    # rotation: energy invariant, forces rotate
    Q = _rotation(3)
    r = orc.energy_forces(_moved(c0, xyz @ Q.T))
    assert abs(r["E"] - base["E"]) <= 1e-12 * abs(base["E"])
    assert np.abs(r["F"] - base["F"] @ Q.T).max() <= 1e-10 * np.abs(base["F"]).max()
    # permutation: everything permutes
    perm = np.random.default_rng(4).permutation(c0.n)
    sp = synth.System(c0.x[perm], c0.y[perm], c0.z[perm], c0.q[perm], c0.rho[perm],
                      c0.screen[perm])
    pr = orc.energy_forces(sp)
    assert abs(pr["E"] - base["E"]) <= 1e-12 * abs(base["E"])
    for key in ("phi", "dEdrho", "R"):
        assert np.abs(pr[key] - base[key][perm]).max() <= 1e-10 * np.abs(base[key]).max()


def test_charge_sign_symmetry(orc, c0):
    s = c0.copy()
    s.q = -s.q
    assert abs(orc.energy(s) - orc.energy(c0)) <= 1e-12 * abs(orc.energy(c0))


@pytest.mark.parametrize("pname", ["IGB5", "IGB2"])
def test_zero_net_force_and_torque(orc, c0, pname):
    r = orc.energy_forces(c0, getattr(orc, pname))
    F = r["F"]
    xyz = c0.coords()
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() <= 1e-11 * scale * c0.n
    torque = np.cross(xyz, F).sum(0)
    assert np.abs(torque).max() <= 1e-11 * scale * c0.n * 12.0


@pytest.mark.parametrize("pname", ["IGB5", "IGB2"])
def test_gradients_match_central_differences(orc, c0, pname):
    p = getattr(orc, pname)
    r = orc.energy_forces(c0, p)
    rng = np.random.default_rng(9)
    atoms = rng.choice(c0.n, 12, replace=False)
    h = 1e-5
    for i in atoms:
        for ax, name in enumerate("xyz"):
            sp, sm = c0.copy(), c0.copy()
            getattr(sp, name)[i] += h
            getattr(sm, name)[i] -= h
            fd = -(orc.energy(sp, p) - orc.energy(sm, p)) / (2 * h)
            assert abs(fd - r["F"][i, ax]) <= 1e-6 * max(1.0, abs(fd)), (i, name)
        for key, attr in (("phi", "q"), ("dEdrho", "rho")):
            sp, sm = c0.copy(), c0.copy()
            getattr(sp, attr)[i] += h
            getattr(sm, attr)[i] -= h
            fd = (orc.energy(sp, p) - orc.energy(sm, p)) / (2 * h)
            assert abs(fd - r[key][i]) <= 1e-6 * max(1.0, abs(fd)), (i, key)


def test_gradients_engulfed_geometry(orc):
    # a small atom inside the screened sphere of a big neighbour exercises the
    # engulfed branch of H in the chain force and dE/drho
    s = one_system([[0, 0, 0], [0.3, 0.1, 0], [2.5, -0.4, 0.7]], [0.5, -0.3, 0.2],
                   [0.8, 2.4, 1.5], [0.8, 0.95, 0.8])
    rt0, S1 = 0.8 - 0.09, 0.95 * (2.4 - 0.09)
    assert rt0 < S1 - math.hypot(0.3, 0.1)
    r = orc.energy_forces(s)
    h = 1e-6
    for i in range(3):
        for ax, name in enumerate("xyz"):
            sp, sm = s.copy(), s.copy()
            getattr(sp, name)[i] += h
            getattr(sm, name)[i] -= h
            fd = -(orc.energy(sp) - orc.energy(sm)) / (2 * h)
            assert abs(fd - r["F"][i, ax]) <= 1e-6 * max(1.0, abs(fd))
        sp, sm = s.copy(), s.copy()
        sp.rho[i] += h
        sm.rho[i] -= h
        fd = (orc.energy(sp) - orc.energy(sm)) / (2 * h)
        assert abs(fd - r["dEdrho"][i]) <= 1e-6 * max(1.0, abs(fd))


def test_energy_is_half_q_dot_phi(orc, c0):
    # E is a quadratic form in q at fixed radii (radii do not depend on q)
    r = orc.energy_forces(c0)
    assert abs(0.5 * np.dot(c0.q, r["phi"]) - r["E"]) <= 1e-12 * abs(r["E"])
