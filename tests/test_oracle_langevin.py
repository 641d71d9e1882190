"""Pins of the oracle's Langevin (OVRVO) integrator and its random numbers.

* Philox4x32-10 reproduces the published known-answer vectors.
* The Box-Muller deviates have the moments of a standard normal and the
  streams of different seeds, steps and half steps are distinct.
* The Ornstein-Uhlenbeck half step relaxes the velocity variance of an
  ensemble started at rest as (kT accel / m)(1 - a^(2k)) after k half
  steps, the closed form of the linear recursion v <- a v + c xi.
* With gamma = 0, OVRVO is the velocity-Verlet step bit for bit.
* A short NVT run of molten NaCl started cold reaches the target kinetic
  temperature (equipartition, 3N/2 kT).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import langevin
from paper_2505_20418_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = np.array([int(x, 16) for x in v["ctr"]], dtype=np.uint64)
        key = [int(x, 16) for x in v["key"]]
        out = langevin.philox4x32_10(ctr, key)
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, size=(50, 4), dtype=np.uint64)
    key = (0x12345678, 0x9abcdef0)
    many = langevin.philox4x32_10(ctr, key)
    for k in range(50):
        assert np.array_equal(many[k], langevin.philox4x32_10(ctr[k], key))


def test_normals_moments_and_distinct_streams():
    n = 200_000
    z = langevin.normals(seed=2024, step=17, half=0, n=n)
    for c in range(3):
        x = z[:, c]
        se = 1.0 / np.sqrt(n)
        assert abs(x.mean()) < 5 * se
        assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0) * se
        kurt = np.mean(x ** 4) / x.var() ** 2
        assert abs(kurt - 3.0) < 5 * np.sqrt(24.0) * se
    # components uncorrelated
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(np.mean(z[:, a] * z[:, b])) < 5 / np.sqrt(n)
    base = langevin.normals(1, 5, 0, 64)
    for other in (langevin.normals(2, 5, 0, 64), langevin.normals(1, 6, 0, 64),
                  langevin.normals(1, 5, 1, 64), langevin.normals(1, 5 + 2 ** 32, 0, 64)):
        assert not np.any(np.isclose(base, other, rtol=0, atol=1e-15))
    assert np.array_equal(base, langevin.normals(1, 5, 0, 64))


def test_ou_variance_relaxation_closed_form():
    n = 100_000
    masses = np.full(n, 22.98977)
    gamma, dt, T = 0.02, 2.0, 1400.0
    kT = inputs.KB_EV_PER_K * T
    a, b2 = langevin.ou_coefficients(gamma, dt, kT, inputs.ACCEL_FACTOR)
    assert a == pytest.approx(np.exp(-gamma * dt / 2), rel=1e-15)
    var_eq = kT * inputs.ACCEL_FACTOR / masses[0]
    vel = np.zeros((n, 3))
    for k in range(1, 41):
        langevin.ou_half_step(vel, masses, a, b2, langevin.normals(9, k, 0, n))
        if k in (1, 5, 20, 40):
            expect = var_eq * (1.0 - a ** (2 * k))
            got = vel.var(axis=0)
            # sampling error of a variance: sqrt(2 / n) relative
            assert np.all(np.abs(got / expect - 1.0) < 5 * np.sqrt(2.0 / n)), (k, got, expect)
            assert np.all(np.abs(vel.mean(axis=0)) < 5 * np.sqrt(expect / n))


def _system():
    s = inputs.molten_nacl(2, seed=1)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-11,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    pos, vel = s.pos.copy(), s.vel.copy()
    F_es = o.step(pos)["forces"]
    F_sr, _ = oracle.bmh(pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    return s, o, pos, vel, F_es, F_sr


def test_gamma_zero_is_velocity_verlet():
    s, o1, p1, v1, fe1, fs1 = _system()
    _, o2, p2, v2, fe2, fs2 = _system()
    w1, w2 = np.zeros(1), np.zeros(1)
    for k in range(3):
        o1.md_step(p1, v1, s.masses, s.species, inputs.BMH_TABLE, inputs.BMH_CUTOFF, 1.0,
                   inputs.ACCEL_FACTOR, fe1, fs1, w1)
        langevin.ovrvo_step(o2, p2, v2, s.masses, s.species, inputs.BMH_TABLE,
                            inputs.BMH_CUTOFF, 1.0, inputs.ACCEL_FACTOR, fe2, fs2, w2,
                            gamma=0.0, kT=0.1, seed=3, step=k)
    assert np.array_equal(p1, p2) and np.array_equal(v1, v2) and np.array_equal(w1, w2)


def test_nvt_reaches_target_temperature():
    """64 ions started at about 250 K, thermostatted to 1500 K with gamma =
    0.05/fs (memory 20 fs): after 100 fs the mean kinetic temperature over
    the next 200 fs matches the target (3N/2 kT per the 3N velocity
    components, Langevin dynamics conserving no momentum)."""
    s, o, pos, vel, F_es, F_sr = _system()
    vel *= np.sqrt(250.0 / 1200.0)
    T = 1500.0
    kT = inputs.KB_EV_PER_K * T
    work = np.zeros(1)
    ke = []
    for k in range(300):
        out = langevin.ovrvo_step(o, pos, vel, s.masses, s.species, inputs.BMH_TABLE,
                                  inputs.BMH_CUTOFF, 1.0, inputs.ACCEL_FACTOR, F_es, F_sr, work,
                                  gamma=0.05, kT=kT, seed=11, step=k)
        ke.append(out["ke"])
    t_kin = 2.0 * np.mean(ke[100:]) / (3 * s.n_ions * inputs.KB_EV_PER_K)
    # one sample's relative spread is sqrt(2 / 3N) = 10%; about ten
    # independent samples in 200 fs
    assert abs(t_kin / T - 1.0) < 0.12, t_kin
