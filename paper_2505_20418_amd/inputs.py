"""Seeded synthetic inputs for the Poisson MaZe hot path.

This module only draws inputs: lattice sites, jitter, velocities, charges,
masses, the short-range force-field table and request streams. It contains
none of the method's arithmetic (no charge assignment, no stencil, no
solver, no force interpolation), so both the CPU oracle and the HIP path can
take their inputs from it without sharing any of the computation.

Workload recipe (molten NaCl, standing in for the private NaCl system of the
paper's Results section):

* rock-salt lattice of ``n**3`` conventional cells with lattice constant
  ``a = 6.375`` A, sites ``(i, j, k) * a/2`` for ``i, j, k in [0, 2n)``,
  charge ``(-1)**(i+j+k)`` (+1 = Na, -1 = Cl); box ``L = n*a``;
* every coordinate jittered by a seeded Gaussian of sigma 0.1 A;
* Maxwell-Boltzmann velocities at temperature ``T`` with the centre-of-mass
  momentum removed;
* grid spacing ``h = a/16 = 0.3984375`` A, so a grid of ``N = 16 n`` points
  per side and undisplaced lattice sites on grid points.

Units: A, fs, amu, eV, elementary charges.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Physical constants of the unit system (CODATA values).
KB_EV_PER_K = 8.617333262e-5          # Boltzmann constant [eV/K]
ACCEL_FACTOR = 9.648533212e-3         # (eV / (A amu)) -> A / fs^2
COULOMB_K_EV_A = 14.3996454784        # e^2 / (4 pi eps0) [eV A]

MASS_NA = 22.98977                    # amu
MASS_CL = 35.453                      # amu
LATTICE_A = 6.375                     # A, conventional rock-salt cell
GRID_PER_CELL = 16                    # grid points per lattice constant

# Tosi-Fumi Born-Huggins-Mayer parameters for NaCl, electrostatics removed:
# V(r) = A exp(B (s - r)) - C / r^6 - D / r^8, one row per pair type in the
# order (Na-Na, Na-Cl, Cl-Cl); columns A [eV], B [1/A], s [A], C [eV A^6],
# D [eV A^8]. These are the commonly tabulated Tosi-Fumi values (b = 0.338e-19
# J with Pauling factors 1.25 / 1 / 0.75, rho = 0.317 A, ionic radii 1.170 /
# 1.585 A, dispersion constants converted from 1e-79 J m^6 and 1e-99 J m^8).
# They are force-field inputs handed to both implementations.
BMH_TABLE = np.array([
    # A         B            s      C        D
    [0.26370, 1.0 / 0.317, 2.340, 1.0486, 0.4993],
    [0.21096, 1.0 / 0.317, 2.755, 6.9906, 8.6760],
    [0.15822, 1.0 / 0.317, 3.170, 72.400, 145.43],
], dtype=np.float64)
BMH_CUTOFF = 6.0


@dataclasses.dataclass
class NaClSystem:
    """One synthetic molten-NaCl configuration."""
    n_cells: int
    box: float                 # L [A]
    grid_spacing: float        # requested h [A]
    pos: np.ndarray            # (Np, 3) float64 [A]
    vel: np.ndarray            # (Np, 3) float64 [A/fs]
    charges: np.ndarray        # (Np,) float64 [e]
    species: np.ndarray        # (Np,) int32, 0 = Na, 1 = Cl
    masses: np.ndarray         # (Np,) float64 [amu]
    temperature: float
    seed: int

    @property
    def n_ions(self) -> int:
        return int(self.charges.shape[0])

    @property
    def grid_n(self) -> int:
        return GRID_PER_CELL * self.n_cells


def rocksalt_sites(n_cells: int, a: float = LATTICE_A):
    """Undisplaced rock-salt sites and their charges (+1 Na, -1 Cl)."""
    m = 2 * n_cells
    i, j, k = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    pos = np.stack([i, j, k], axis=1).astype(np.float64) * (a / 2.0)
    parity = (i + j + k) % 2
    charges = np.where(parity == 0, 1.0, -1.0)
    species = parity.astype(np.int32)
    return pos, charges, species


def maxwell_boltzmann(masses: np.ndarray, temperature: float, rng) -> np.ndarray:
    """Gaussian velocities with variance kT/m per component, zero total momentum."""
    sigma = np.sqrt(KB_EV_PER_K * temperature / masses * ACCEL_FACTOR)
    v = rng.standard_normal((masses.shape[0], 3)) * sigma[:, None]
    p = (masses[:, None] * v).sum(axis=0)
    v -= p / masses.sum()
    return v


def molten_nacl(n_cells: int, seed: int, temperature: float = 1200.0,
                jitter: float = 0.1, a: float = LATTICE_A) -> NaClSystem:
    """Rock-salt NaCl, jittered, with Maxwell-Boltzmann velocities."""
    rng = np.random.default_rng(seed)
    pos, charges, species = rocksalt_sites(n_cells, a)
    if jitter > 0:
        pos = pos + rng.standard_normal(pos.shape) * jitter
    masses = np.where(species == 0, MASS_NA, MASS_CL).astype(np.float64)
    vel = maxwell_boltzmann(masses, temperature, rng)
    return NaClSystem(n_cells=n_cells, box=n_cells * a,
                      grid_spacing=a / GRID_PER_CELL, pos=pos, vel=vel,
                      charges=charges.astype(np.float64), species=species,
                      masses=masses, temperature=temperature, seed=seed)


def bcc_nacl(cells: int = 5, box: float = 20.64, grid_spacing: float = 0.172,
             temperature: float = 1550.0, seed: int = 0) -> NaClSystem:
    """The Results section's molten-salt start: ions on a bcc lattice
    (cells^3 cubic cells, Na on the corners and Cl on the body centres, so
    2 cells^3 ions; 250 ions in 20.64 A for cells = 5) with Maxwell-Boltzmann
    velocities at the target temperature."""
    c = box / cells
    i, j, k = np.meshgrid(np.arange(cells), np.arange(cells), np.arange(cells), indexing="ij")
    corner = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * c
    pos = np.concatenate([corner, corner + 0.5 * c])
    n = corner.shape[0]
    species = np.concatenate([np.zeros(n, np.int32), np.ones(n, np.int32)])
    charges = np.where(species == 0, 1.0, -1.0)
    masses = np.where(species == 0, MASS_NA, MASS_CL).astype(np.float64)
    vel = maxwell_boltzmann(masses, temperature, np.random.default_rng(seed))
    return NaClSystem(n_cells=cells, box=box, grid_spacing=grid_spacing, pos=pos, vel=vel,
                      charges=charges, species=species, masses=masses,
                      temperature=temperature, seed=seed)


# The five workloads (cubic box, h = a/16 throughout).
WORKLOADS = {
    # 64 ions, 32^3 grid, FP64, 100 NVE steps at 1200 K, tol 1e-9
    "nacl64_g32": dict(n_cells=2, seed=1, temperature=1200.0, tol=1e-9, steps=100),
    # 4096 ions, 128^3 grid, FP64, 1000 NVE steps, tol 1e-9
    "nacl4096_g128": dict(n_cells=8, seed=2, temperature=1200.0, tol=1e-9, steps=1000),
    # 32768 ions, 256^3 grid, mixed vs FP64, 500 steps, relative residual 1e-8
    "nacl32768_g256": dict(n_cells=16, seed=3, temperature=1200.0, tol=1e-8, steps=500),
}


def workload(name: str) -> NaClSystem:
    w = WORKLOADS[name]
    return molten_nacl(w["n_cells"], seed=w["seed"], temperature=w["temperature"])


@dataclasses.dataclass
class Replica:
    n_cells: int
    temperature: float
    seed: int


def ensemble_replicas(count: int = 64, master_seed: int = 4,
                      n_choices=(2, 3, 4, 5, 6),
                      t_range=(1100.0, 1400.0)) -> List[Replica]:
    """Uneven replica ensemble: n drawn from n_choices, T uniform in t_range."""
    rng = np.random.default_rng(master_seed)
    ns = rng.choice(np.asarray(n_choices), size=count)
    ts = rng.uniform(t_range[0], t_range[1], size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [Replica(int(n), float(t), int(s)) for n, t, s in zip(ns, ts, seeds)]


@dataclasses.dataclass
class StepRequest:
    arrival_s: float
    session: int
    tol: float
    mixed: bool


def serving_sessions(count: int = 256, seed: int = 5, max_cells: int = 16):
    """Session sizes: n = round(2**U(1, 4)), so 8 n^3 ions are about
    log-uniform over 64..32768; the tolerance class is drawn 50/50."""
    rng = np.random.default_rng(seed)
    ns = np.clip(np.rint(2.0 ** rng.uniform(1.0, math.log2(max_cells), size=count)),
                 2, max_cells).astype(int)
    mixed = rng.random(count) < 0.5
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [dict(n_cells=int(n), mixed=bool(m), tol=(1e-6 if m else 1e-10),
                 seed=int(s)) for n, m, s in zip(ns, mixed, seeds)]


def poisson_arrivals(n_requests: int, n_sessions: int, rate_hz: float = 200.0,
                     seed: int = 5, session_mixed: Optional[List[bool]] = None):
    """Poisson arrival stream of MD-step requests over resident sessions."""
    rng = np.random.default_rng(seed + 1000)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps)
    sess = rng.integers(0, n_sessions, size=n_requests)
    out = []
    for ti, si in zip(t, sess):
        m = bool(session_mixed[si]) if session_mixed is not None else False
        out.append(StepRequest(float(ti), int(si), 1e-6 if m else 1e-10, m))
    return out
