"""Structural and transport observables of the Results section, plain numpy
(test infrastructure).

* Radial pair distribution functions g_IJ(r) for I, J in {Na, Cl}: pair
  distances under the minimum image in the cubic periodic box, histogrammed
  per species pair and normalised by the ideal-gas pair count of each shell.
* Velocity autocorrelation functions and mean squared displacements per
  species, averaged over time origins; the diffusion coefficient follows
  from either (Green-Kubo integral of the VACF over 3, or the long-time
  slope of the MSD over 6).

The histogram bin of a pair is decided on its squared distance
r2 = dx^2 + dy^2 + dz^2 (each dx = x_j - x_i wrapped by dx - L rint(dx/L),
summed in that order, no fused multiply-add) against squared bin edges
given as input: bin b holds edges2[b] <= r2 < edges2[b+1].
"""
from __future__ import annotations

import numpy as np

ROW_NANA, ROW_NACL, ROW_CLCL = 0, 1, 2


def pair_r2(pos: np.ndarray, box: float):
    """Squared minimum-image distances of all pairs i < j, with the species
    row s_i + s_j left to the caller. Returns (i, j, r2)."""
    n = len(pos)
    i, j = np.triu_indices(n, k=1)
    d = pos[j] - pos[i]
    d = d - box * np.rint(d / box)
    r2 = d[:, 0] * d[:, 0]
    r2 = r2 + d[:, 1] * d[:, 1]
    r2 = r2 + d[:, 2] * d[:, 2]
    return i, j, r2


def rdf_counts(pos: np.ndarray, species: np.ndarray, box: float,
               edges2: np.ndarray) -> np.ndarray:
    """(3, nbins) integer pair counts per species row (Na-Na, Na-Cl, Cl-Cl)."""
    nb = len(edges2) - 1
    i, j, r2 = pair_r2(np.asarray(pos, dtype=np.float64), box)
    row = np.asarray(species)[i] + np.asarray(species)[j]
    b = np.searchsorted(edges2, r2, side="right") - 1
    ok = (b >= 0) & (b < nb)
    out = np.zeros((3, nb), dtype=np.int64)
    np.add.at(out, (row[ok], b[ok]), 1)
    return out


def rdf_normalise(counts: np.ndarray, frames: int, n_na: int, n_cl: int, box: float,
                  edges: np.ndarray) -> np.ndarray:
    """g_IJ(r) per row from counts summed over `frames` configurations: the
    pairs in each shell over the pairs an ideal gas at the same density would
    put there (N_I N_J shell_volume / V for I != J, N_I (N_I - 1) / 2
    shell_volume / V for I = J)."""
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    V = box ** 3
    ideal = np.array([n_na * (n_na - 1) / 2.0, n_na * n_cl, n_cl * (n_cl - 1) / 2.0])
    return counts / (frames * ideal[:, None] * shell[None, :] / V)


def rdf_features(r_mid: np.ndarray, g: np.ndarray, floor: float = 0.0, smooth: int = 5,
                 window: float = 3.0):
    """The comparison quantities of the g(r) table: r_cut (first r where g
    becomes non-null, above `floor`), position and height of the first
    maximum (the highest point of a liquid's g), and the first minimum: the
    lowest point of a `smooth`-bin moving average of g within `window` after
    the maximum."""
    nz = np.nonzero(g > floor)[0]
    if len(nz) == 0:
        return None
    k0 = int(nz[0])
    kmax = int(np.argmax(g))
    gs = np.convolve(g, np.ones(smooth) / smooth, mode="same")
    dr = float(r_mid[1] - r_mid[0])
    hi = min(len(g) - smooth // 2, kmax + 1 + int(round(window / dr)))
    kmin = kmax + 1 + int(np.argmin(gs[kmax + 1:hi])) if hi > kmax + 1 else kmax
    return dict(r_cut=float(r_mid[k0]), r_max=float(r_mid[kmax]), g_max=float(g[kmax]),
                r_min=float(r_mid[kmin]))


class TimeCorrelations:
    """Per-species VACF and MSD sums over time origins. Sample k = 0, 1, ...
    stores an origin when k is a multiple of `origin_every`; every stored
    origin o with lag l = k - k_o <= max_lag adds sum_i v_i(o).v_i(k) and
    sum_i |r_i(k) - r_i(o)|^2 over the ions of each species to the sums of
    lag l (positions unwrapped)."""

    def __init__(self, species: np.ndarray, max_lag: int, origin_every: int):
        self.species = np.asarray(species)
        self.max_lag = max_lag
        self.every = origin_every
        self.k = 0
        self.origins = []  # (k_o, pos, vel)
        self.vacf = np.zeros((2, max_lag + 1))
        self.msd = np.zeros((2, max_lag + 1))
        self.counts = np.zeros(max_lag + 1, dtype=np.int64)

    def sample(self, pos: np.ndarray, vel: np.ndarray):
        if self.k % self.every == 0:
            self.origins.append((self.k, np.array(pos, dtype=np.float64),
                                 np.array(vel, dtype=np.float64)))
        self.origins = [o for o in self.origins if self.k - o[0] <= self.max_lag]
        for k0, p0, v0 in self.origins:
            lag = self.k - k0
            vv = np.sum(v0 * vel, axis=1)
            dr = pos - p0
            rr = np.sum(dr * dr, axis=1)
            for s in (0, 1):
                m = self.species == s
                self.vacf[s, lag] += vv[m].sum()
                self.msd[s, lag] += rr[m].sum()
            self.counts[lag] += 1
        self.k += 1

    def averages(self):
        """(vacf, msd) per species and lag, per ion and origin."""
        n_s = np.array([np.sum(self.species == 0), np.sum(self.species == 1)], dtype=float)
        c = np.maximum(self.counts, 1)[None, :]
        return self.vacf / (c * n_s[:, None]), self.msd / (c * n_s[:, None])


def diffusion_from_vacf(vacf: np.ndarray, dt_sample: float) -> float:
    """Green-Kubo: D = (1/3) integral of <v(0).v(t)> dt (trapezoid rule)."""
    return float(np.trapezoid(vacf, dx=dt_sample) / 3.0)


def diffusion_from_msd(msd: np.ndarray, dt_sample: float, start: int) -> float:
    """Einstein: D = slope of <|r(t) - r(0)|^2> / 6, least squares over the
    lags from `start` on."""
    t = np.arange(len(msd)) * dt_sample
    slope = np.polyfit(t[start:], msd[start:], 1)[0]
    return float(slope / 6.0)
