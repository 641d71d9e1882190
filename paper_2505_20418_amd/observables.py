"""Structural and transport observables on the device (Results section).

Thin wrappers of the library's entry points: pair-distance histograms for
the radial distribution functions g_IJ(r) (maze_rdf_accumulate), and the
velocity autocorrelation functions and mean squared displacements per
species over time origins (maze_tcf_*). The normalisation to g(r) and the
diffusion coefficients are host arithmetic on the accumulated sums.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import maze

ROWS = ("NaNa", "NaCl", "ClCl")


class PairHistogram:
    """Pair counts per species row over frames, bins of width r_max / nbins
    from 0 to r_max (r_max at most half the box)."""

    def __init__(self, species: torch.Tensor, box: float, r_max: float, nbins: int,
                 stream=None):
        self.species = species.to(torch.int32).contiguous()
        self.n = int(self.species.numel())
        self.box = float(box)
        self.nbins = int(nbins)
        self.edges = np.linspace(0.0, float(r_max), self.nbins + 1)
        dev = self.species.device
        self.edges2 = torch.tensor(self.edges ** 2, dtype=torch.float64, device=dev)
        self.hist = torch.zeros(3 * self.nbins, dtype=torch.int64, device=dev)
        self.stream = stream
        self.frames = 0

    def accumulate(self, pos: torch.Tensor):
        rc = maze.lib().maze_rdf_accumulate(pos.data_ptr(), self.species.data_ptr(), self.n,
                                            self.box, self.edges2.data_ptr(), self.nbins,
                                            self.hist.data_ptr(), self.stream)
        maze._check(rc, "maze_rdf_accumulate")
        self.frames += 1

    def counts(self) -> np.ndarray:
        return self.hist.view(3, self.nbins).cpu().numpy()

    def g(self) -> np.ndarray:
        """g_IJ(r) per row: pairs in each shell over the ideal-gas pair count
        of the shell at the same density."""
        s = self.species.cpu().numpy()
        n_na, n_cl = int(np.sum(s == 0)), int(np.sum(s == 1))
        shell = 4.0 / 3.0 * np.pi * (self.edges[1:] ** 3 - self.edges[:-1] ** 3)
        ideal = np.array([n_na * (n_na - 1) / 2.0, n_na * n_cl, n_cl * (n_cl - 1) / 2.0])
        V = self.box ** 3
        return self.counts() / (max(self.frames, 1) * ideal[:, None] * shell[None, :] / V)

    def r_mid(self) -> np.ndarray:
        return 0.5 * (self.edges[1:] + self.edges[:-1])


def g_features(r: np.ndarray, g: np.ndarray, floor: float = 0.0, smooth: int = 5,
               window: float = 3.0) -> dict:
    """The quantities of the paper's g(r) table: onset r_cut (first r where g
    becomes non-null, above `floor`), the first maximum (the highest point
    of a liquid's g: position and height), and the first minimum, the lowest
    point of a `smooth`-bin moving average of g within `window` after the
    maximum (so that counting noise does not end the descent early)."""
    nz = np.nonzero(g > floor)[0]
    if len(nz) == 0:
        return {}
    k0 = int(nz[0])
    kmax = int(np.argmax(g))
    gs = np.convolve(g, np.ones(smooth) / smooth, mode="same")
    dr = float(r[1] - r[0]) if len(r) > 1 else 1.0
    hi = min(len(g) - smooth // 2, kmax + 1 + int(round(window / dr)))
    kmin = kmax + 1 + int(np.argmin(gs[kmax + 1:hi])) if hi > kmax + 1 else kmax
    return dict(r_cut=float(r[k0]), r_max=float(r[kmax]), g_max=float(g[kmax]),
                r_min=float(r[kmin]))


class TimeCorrelations:
    """Per-species VACF and MSD sums over time origins (maze_tcf_*)."""

    def __init__(self, species: torch.Tensor, max_lag: int, origin_every: int, stream=None):
        self.species = species.to(torch.int32).contiguous()
        self.n = int(self.species.numel())
        self.max_lag = int(max_lag)
        h = ctypes.c_void_p()
        rc = maze.lib().maze_tcf_create(self.n, self.species.data_ptr(), self.max_lag,
                                        int(origin_every), stream, ctypes.byref(h))
        maze._check(rc, "maze_tcf_create")
        self.handle = h

    def sample(self, pos: torch.Tensor, vel: torch.Tensor):
        maze._check(maze.lib().maze_tcf_sample(self.handle, pos.data_ptr(), vel.data_ptr()),
                    "maze_tcf_sample")

    def sums(self):
        L = self.max_lag + 1
        s = (ctypes.c_double * (4 * L))()
        c = (ctypes.c_int64 * L)()
        maze._check(maze.lib().maze_tcf_read(self.handle, s, c), "maze_tcf_read")
        return np.array(s).reshape(4, L), np.array(c, dtype=np.int64)

    def averages(self):
        """(vacf, msd): (2, max_lag + 1) per species, per ion and origin."""
        s, c = self.sums()
        sp = self.species.cpu().numpy()
        n_s = np.array([np.sum(sp == 0), np.sum(sp == 1)], dtype=float)
        cc = np.maximum(c, 1)[None, :]
        return s[:2] / (cc * n_s[:, None]), s[2:] / (cc * n_s[:, None])

    def close(self):
        if self.handle:
            maze.lib().maze_tcf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diffusion_vacf(vacf: np.ndarray, dt_sample: float) -> float:
    """Green-Kubo: (1/3) integral of the VACF (trapezoid), A^2/fs."""
    return float(np.trapezoid(vacf, dx=dt_sample) / 3.0)


def diffusion_msd(msd: np.ndarray, dt_sample: float, start: int) -> float:
    """Einstein: least-squares slope of the MSD from lag `start` on, / 6."""
    t = np.arange(len(msd)) * dt_sample
    return float(np.polyfit(t[start:], msd[start:], 1)[0] / 6.0)


A2_PER_FS_TO_CM2_PER_S = 0.1  # 1 A^2/fs = 1e-16 cm^2 / 1e-15 s


def langevin_noise(seed: int, step: int, half: int, n: int, device="cuda") -> torch.Tensor:
    """The (n, 3) deviates of one OVRVO half step (maze_langevin_noise)."""
    out = torch.empty(n, 3, dtype=torch.float64, device=device)
    maze._check(maze.lib().maze_langevin_noise(seed, step, half, n, out.data_ptr(), None),
                "maze_langevin_noise")
    return out
