"""Langevin (OVRVO) dynamics and its random numbers, plain numpy (test
infrastructure, like the rest of this package).

The Results section equilibrates molten NaCl in the canonical ensemble with
Langevin dynamics integrated by OVRVO (Sivak, Chodera and Crooks 2013): an
Ornstein-Uhlenbeck half step on the velocities, the velocity-Verlet kick /
drift / kick, and a second Ornstein-Uhlenbeck half step. With friction
gamma = 0 it is velocity Verlet.

The noise is drawn from the counter-based generator Philox4x32-10 (Salmon,
Moraes, Dror and Shaw, SC'11), written here from its published definition,
and turned into normal deviates by the Box-Muller transform. The device
path implements the same generator and transform on its own; for ion i,
step k and half step h (0 before the kick, 1 after) the counter is
(i, h, k mod 2^32, k div 2^32) and the key (seed mod 2^32, seed div 2^32).
"""
from __future__ import annotations

import math

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
TWO_PI = 6.283185307179586


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds. ctr: (..., 4) integers below 2^32; key:
    2 integers below 2^32. Each round multiplies words 0 and 2 by the two
    constants, keeps the high and low halves and mixes in words 1, 3 and the
    key; the key is bumped by the two Weyl constants between rounds."""
    c = np.asarray(ctr, dtype=np.uint64)
    w = [c[..., j].copy() for j in range(4)]
    k0 = np.uint64(key[0]) & _MASK
    k1 = np.uint64(key[1]) & _MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & _MASK
            k1 = (k1 + PHILOX_W1) & _MASK
        p0 = PHILOX_M0 * w[0]
        p1 = PHILOX_M1 * w[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        w = [hi1 ^ w[1] ^ k0, lo1, hi0 ^ w[3] ^ k1, lo0]
    return np.stack(w, axis=-1).astype(np.uint32)


def normals(seed: int, step: int, half: int, n: int) -> np.ndarray:
    """(n, 3) standard normal deviates of ions 0..n-1 for (step, half).
    Box-Muller on the word pairs (0, 1) and (2, 3): u1 = (x + 1) 2^-32 in
    (0, 1], u2 = x' 2^-32 in [0, 1); the pair gives r cos(2 pi u2) and
    r sin(2 pi u2) with r = sqrt(-2 ln u1). Components: x, y from the first
    pair (cos, sin), z from the cosine of the second."""
    i = np.arange(n, dtype=np.uint64)
    ctr = np.stack([i, np.full(n, half, dtype=np.uint64),
                    np.full(n, step & 0xFFFFFFFF, dtype=np.uint64),
                    np.full(n, (step >> 32) & 0xFFFFFFFF, dtype=np.uint64)], axis=-1)
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).astype(np.float64)
    scale = 2.0 ** -32
    u1a, u2a = (x[:, 0] + 1.0) * scale, x[:, 1] * scale
    u1b, u2b = (x[:, 2] + 1.0) * scale, x[:, 3] * scale
    ra = np.sqrt(-2.0 * np.log(u1a))
    rb = np.sqrt(-2.0 * np.log(u1b))
    out = np.empty((n, 3))
    out[:, 0] = ra * np.cos(TWO_PI * u2a)
    out[:, 1] = ra * np.sin(TWO_PI * u2a)
    out[:, 2] = rb * np.cos(TWO_PI * u2b)
    return out


def ou_coefficients(gamma: float, dt: float, kT: float, accel: float):
    """Ornstein-Uhlenbeck half step over dt/2: v <- a v + sqrt(b2 / m) xi with
    a = exp(-gamma dt / 2) and b2 = (1 - a^2) kT accel (kT in eV, m in amu,
    accel converting eV/(A amu) to A/fs^2, so sqrt(b2/m) is in A/fs)."""
    a = math.exp(-gamma * dt / 2.0)
    return a, (1.0 - a * a) * kT * accel


def ou_half_step(vel: np.ndarray, masses: np.ndarray, a: float, b2: float,
                 xi: np.ndarray) -> None:
    """In place: v <- a v + sqrt(b2 / m) xi, per ion and component."""
    c = np.sqrt(b2 / masses)
    vel *= a
    vel += c[:, None] * xi


def ovrvo_step(sess, pos, vel, masses, species, table, cutoff, dt, accel, F_es, F_sr, work,
               gamma: float, kT: float, seed: int, step: int):
    """One OVRVO step through the oracle: O(dt/2), the velocity-Verlet step
    (kick, drift, MaZe forces and short range at the new positions, kick),
    O(dt/2). Returns the velocity-Verlet step's result and the kinetic
    energy [eV] and momentum [amu A/fs] after the second half step."""
    if gamma > 0.0:
        a, b2 = ou_coefficients(gamma, dt, kT, accel)
        ou_half_step(vel, masses, a, b2, normals(seed, step, 0, len(masses)))
    out = sess.md_step(pos, vel, masses, species, table, cutoff, dt, accel, F_es, F_sr, work)
    if gamma > 0.0:
        ou_half_step(vel, masses, a, b2, normals(seed, step, 1, len(masses)))
    out["ke"] = float(0.5 * np.sum(masses[:, None] * vel * vel) / accel)
    out["momentum"] = (masses[:, None] * vel).sum(axis=0)
    return out
