"""Pins of the oracle's leapfrog Langevin step (Loncharich, Brooks & Pastor
1992), the dynamics between Monte Carlo attempts (section III.D: Langevin
thermostat):

* the unit factor from SI (kcal/mol per amu Angstrom in Angstrom/ps^2);
* a restrained single atom without friction follows the exact discrete
  solution of the leapfrog harmonic oscillator (pins the force sign, the unit
  factor, the restraint and the drift);
* a free atom with friction and no noise decays by the exact factor
  ((1 - a)/(1 + a))^n, its position by the geometric sum (pins the friction);
* free atoms with noise reach the exact variance kB T / m of the scheme from
  rest, step by step (pins the noise amplitude);
* without friction the electrostatic system conserves its total energy to
  second order in dt (pins that the electrostatic forces drive the step).
"""
import math

import numpy as np
import pytest

import oracle
import synth

KB = 1.98720426e-3


def one_atom(x0=(0.3, -0.2, 0.1), q=0.5):
    return synth.System(np.array([x0[0]]), np.array([x0[1]]), np.array([x0[2]]),
                        np.array([q]), np.array([1.7]), np.array([0.8]))


def test_unit_factor_from_si():
    # 1 kcal/mol / (1 g/mol * 1 Angstrom) = 4184 J / (1e-3 kg * 1e-10 m) = 4.184e16 m/s^2
    si = 4184.0 / (1e-3 * 1e-10)
    assert math.isclose(si * 1e10 / 1e24, oracle.ACC, rel_tol=1e-15)


def test_restrained_atom_is_the_discrete_harmonic_oscillator():
    # x'' = -w^2 (x - xref) with w^2 = k ACC / m: the leapfrog recursion
    # x_{n+1} - 2 x_n + x_{n-1} = -w^2 dt^2 x_n has the exact solution
    # A cos(n th) + B sin(n th), cos th = 1 - w^2 dt^2 / 2
    k, m, dt = 250.0, 12.0, 0.002
    xref = np.zeros((1, 3))
    s = one_atom()
    v = np.array([[0.4, 0.0, -0.3]])
    x0 = s.coords()[0].copy()
    w2 = k * oracle.ACC / m
    th = math.acos(1.0 - 0.5 * w2 * dt * dt)
    v_half = v[0] - dt * w2 * x0          # first kick, from x0
    x1 = x0 + dt * v_half
    A, B = x0, (x1 - x0 * math.cos(th)) / math.sin(th)
    zero = np.zeros((1, 3))
    for n in range(1, 301):
        x, y, z, v = oracle.langevin_step(s, v, [1.0 / m], zero, dt, 0.0, 300.0,
                                          xref=xref, k_restr=k)
        s.x, s.y, s.z = x, y, z
        exact = A * math.cos(n * th) + B * math.sin(n * th)
        assert np.allclose(s.coords()[0], exact, rtol=0, atol=1e-12), n


def test_friction_decay_without_noise():
    gamma, dt, m = 5.0, 0.002, 16.0
    a = 0.5 * gamma * dt
    rho = (1 - a) / (1 + a)
    s = one_atom()
    v0 = np.array([[1.5, -0.7, 0.2]])
    x0 = s.coords()[0].copy()
    v = v0.copy()
    zero = np.zeros((1, 3))
    for n in range(1, 101):
        x, y, z, v = oracle.langevin_step(s, v, [1.0 / m], zero, dt, gamma, 300.0)
        s.x, s.y, s.z = x, y, z
        assert np.allclose(v[0], v0[0] * rho ** n, rtol=1e-13, atol=0)
        xs = x0 + dt * v0[0] * rho * (1 - rho ** n) / (1 - rho)
        assert np.allclose(s.coords()[0], xs, rtol=0, atol=1e-12)


def test_noise_reaches_exact_variance_from_rest():
    # uncharged atoms feel no force: each velocity component is the AR(1)
    # process v' = rho v + sig xi / (1 + a), whose variance from rest is
    # (kB T / m)(1 - rho^(2n)) exactly (stationary value kB T / m)
    n_at, gamma, dt, T = 1000, 8.0, 0.002, 300.0
    rng = np.random.default_rng(3)
    s = synth.System(*(rng.uniform(-30, 30, n_at) for _ in range(3)), np.zeros(n_at),
                     rng.uniform(1.2, 2.0, n_at), rng.uniform(0.7, 0.9, n_at))
    inv_m = 1.0 / rng.uniform(1.0, 30.0, n_at)
    v = np.zeros((n_at, 3))
    a = 0.5 * gamma * dt
    rho = (1 - a) / (1 + a)
    for n in range(1, 31):
        xi = rng.standard_normal((n_at, 3))
        x, y, z, v = oracle.langevin_step(s, v, inv_m, xi, dt, gamma, T)
        s.x, s.y, s.z = x, y, z
    var = KB * T * oracle.ACC * inv_m * (1 - rho ** (2 * n))
    chi = (v ** 2 / var[:, None]).mean()
    # 3000 independent unit-variance normals squared: std of the mean sqrt(2/3000)
    assert abs(chi - 1.0) < 4 * math.sqrt(2.0 / v.size), chi


def test_energy_conserved_without_friction():
    s = synth.make_system(41, 40, 6.0, min_dist=2.0)
    n = s.n
    rng = np.random.default_rng(8)
    m = rng.uniform(12.0, 16.0, n)
    k, T, dt = 60.0, 300.0, 0.0005
    xref = s.coords().copy()
    v = rng.standard_normal((n, 3)) * np.sqrt(KB * T * oracle.ACC / m)[:, None]
    zero = np.zeros((n, 3))

    def epot(sys_):
        return oracle.energy(sys_) + 0.5 * k * ((sys_.coords() - xref) ** 2).sum()

    E = []
    v_prev = v
    for step in range(200):
        e_here = epot(s)
        x, y, z, v_new = oracle.langevin_step(s, v_prev, 1.0 / m, zero, dt, 0.0, T,
                                              xref=xref, k_restr=k)
        # kinetic energy at the integer step from the two half-step velocities
        vm = 0.5 * (v_prev + v_new)
        E.append(e_here + 0.5 * (m[:, None] * vm ** 2).sum() / oracle.ACC)
        s.x, s.y, s.z = x, y, z
        v_prev = v_new
    E = np.array(E)
    ke = 1.5 * n * KB * T
    assert np.abs(E - E[0]).max() < 2e-3 * ke, np.abs(E - E[0]).max() / ke
    # a wrong force sign or scale breaks this by orders of magnitude
    assert abs(E[-1] - E[0]) < 1e-3 * ke
