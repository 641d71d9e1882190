"""Device-resident molecular dynamics around the MaZe step.

Velocity Verlet for the ions with MaZe electrostatics and the Tosi-Fumi
short-range term, or its Langevin extension OVRVO for canonical runs (the
Results section's equilibration), all in the library's HIP kernels
(maze_md_prime / maze_md_step). This module only allocates the device
buffers and reads the scalars.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import inputs, maze


class MDRun:
    def __init__(self, system: inputs.NaClSystem, tol: float = 1e-9,
                 precision: int = maze.MAZE_FP64, order: int = 2, dt: float = 1.0,
                 device: str = "cuda", max_iter: int = 100000, stream=None,
                 restore: dict = None, flags: int = 0, gamma: float = 0.0,
                 temperature: float = 0.0, seed: int = 0):
        """restore: a dict from save_state(); the run then continues exactly
        where the saved one stopped (particles, forces, observables and the
        MaZe warm-start history), without the priming step.
        gamma [1/fs], temperature [K], seed: Langevin (OVRVO) thermostat;
        gamma = 0 is velocity Verlet."""
        self.system = system
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        n = system.n_ions
        self.n = n
        src = restore if restore is not None else dict(pos=system.pos, vel=system.vel)
        self.pos = torch.tensor(np.asarray(src["pos"]), **f64).contiguous()
        self.vel = torch.tensor(np.asarray(src["vel"]), **f64).contiguous()
        self.mass = torch.tensor(system.masses, **f64)
        self.species = torch.tensor(system.species, dtype=torch.int32, device=dev)
        self.charges = torch.tensor(system.charges, **f64)
        self.f_es = torch.zeros(n, 3, **f64)
        self.f_sr = torch.zeros(n, 3, **f64)
        nb = (n + 255) // 256
        self.scratch = torch.zeros(6 * n + 8 * nb, **f64)
        self.scalars = torch.zeros(8, **f64)
        self.session = maze.Session(self.charges, self.pos, system.box, system.grid_spacing,
                                    tol=tol, order=order, max_iter=max_iter,
                                    precision=precision, coulomb_k=inputs.COULOMB_K_EV_A,
                                    stream=stream, flags=flags)
        table = (ctypes.c_double * 15)(*inputs.BMH_TABLE.ravel().tolist())
        self.md = maze.maze_md_state(
            n, 0, self.pos.data_ptr(), self.vel.data_ptr(), self.mass.data_ptr(),
            self.species.data_ptr(), self.f_es.data_ptr(), self.f_sr.data_ptr(),
            self.scratch.data_ptr(), self.scalars.data_ptr(), float(dt),
            inputs.ACCEL_FACTOR, inputs.BMH_CUTOFF, table, float(gamma),
            inputs.KB_EV_PER_K * float(temperature), int(seed))
        self.last = None
        if restore is None:
            self.prime_stats = maze.maze_md_prime(self.session.handle, self.md)[1]
        else:
            self.session.load(restore["maze"])
            self.f_es.copy_(torch.as_tensor(np.asarray(restore["f_es"])))
            self.f_sr.copy_(torch.as_tensor(np.asarray(restore["f_sr"])))
            self.scalars.copy_(torch.as_tensor(np.asarray(restore["scalars"])))
            self.prime_stats = None

    def set_thermostat(self, gamma: float, temperature: float = 0.0, seed: int = None):
        """Switch the Langevin friction (0: velocity Verlet, e.g. for the
        microcanonical production after a canonical equilibration)."""
        self.md.gamma = float(gamma)
        self.md.kT = inputs.KB_EV_PER_K * float(temperature)
        if seed is not None:
            self.md.seed = int(seed)

    def step(self, want_stats: bool = False):
        rc, st = maze.maze_md_step(self.session.handle, self.md, want_stats)
        self.last = st
        return rc, st

    def save_state(self) -> dict:
        """Host copy of everything needed to continue this run exactly."""
        return dict(maze=self.session.save(), pos=self.pos.cpu().numpy(),
                    vel=self.vel.cpu().numpy(), f_es=self.f_es.cpu().numpy(),
                    f_sr=self.f_sr.cpu().numpy(), scalars=self.scalars.cpu().numpy())

    def observables(self) -> dict:
        s = self.scalars.cpu().numpy()
        return dict(work=float(s[0]), v_sr=float(s[1]), ke=float(s[2]),
                    momentum=s[3:6].copy(), energy_c=float(s[6]),
                    total=float(s[0] + s[1] + s[2]))

    def close(self):
        self.session.close()


def step_many(runs, want_stats: bool = True):
    """One MD step of several runs together (maze_md_step_batch)."""
    return maze.maze_md_step_batch([r.session.handle for r in runs], [r.md for r in runs],
                                   want_stats)
