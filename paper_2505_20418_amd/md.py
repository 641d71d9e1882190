"""Device-resident molecular dynamics around the MaZe step.

Velocity Verlet for the ions with MaZe electrostatics and the Tosi-Fumi
short-range term, all in the library's HIP kernels (maze_md_prime /
maze_md_step). This module only allocates the device buffers and reads
the scalars.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import inputs, maze


class MDRun:
    def __init__(self, system: inputs.NaClSystem, tol: float = 1e-9,
                 precision: int = maze.MAZE_FP64, order: int = 2, dt: float = 1.0,
                 device: str = "cuda", max_iter: int = 100000, stream=None):
        self.system = system
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        n = system.n_ions
        self.n = n
        self.pos = torch.tensor(system.pos, **f64).contiguous()
        self.vel = torch.tensor(system.vel, **f64).contiguous()
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
                                    stream=stream)
        table = (ctypes.c_double * 15)(*inputs.BMH_TABLE.ravel().tolist())
        self.md = maze.maze_md_state(
            n, 0, self.pos.data_ptr(), self.vel.data_ptr(), self.mass.data_ptr(),
            self.species.data_ptr(), self.f_es.data_ptr(), self.f_sr.data_ptr(),
            self.scratch.data_ptr(), self.scalars.data_ptr(), float(dt),
            inputs.ACCEL_FACTOR, inputs.BMH_CUTOFF, table)
        self.last = None
        self.prime_stats = maze.maze_md_prime(self.session.handle, self.md)[1]

    def step(self, want_stats: bool = False):
        rc, st = maze.maze_md_step(self.session.handle, self.md, want_stats)
        self.last = st
        return rc, st

    def observables(self) -> dict:
        s = self.scalars.cpu().numpy()
        return dict(work=float(s[0]), v_sr=float(s[1]), ke=float(s[2]),
                    momentum=s[3:6].copy(), energy_c=float(s[6]),
                    total=float(s[0] + s[1] + s[2]))

    def close(self):
        self.session.close()
