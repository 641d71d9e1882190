"""Pins of the oracle's structural and transport observables.

* Pair counts of a perfect rock-salt crystal fall in the neighbour shells of
  the structure with their textbook multiplicities, like pairs and unlike
  pairs in the right rows.
* Uniform random points (an ideal gas) give g(r) = 1 within counting noise.
* The first peak, minimum and onset of an analytic curve are located.
* Ballistic motion (constant velocities) gives a constant VACF and an MSD
  growing as |v|^2 t^2, exactly, with the origin bookkeeping counted by
  hand; a Gaussian random walk gives the diffusion coefficient of its step
  variance.
"""
import json
import math
import os

import numpy as np

from oracle import structure
from paper_2505_20418_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_rocksalt_shells():
    shells = json.load(open(os.path.join(GOLDEN, "textbook_values.json")))["rocksalt_shells"]
    a = inputs.LATTICE_A
    pos, _, species = inputs.rocksalt_sites(3)
    pos = np.asarray(pos, dtype=float)
    species = np.asarray(species)
    box = 3 * a
    n_na = int(np.sum(species == 0))
    n_cl = int(np.sum(species == 1))
    assert n_na == n_cl == 108
    dr = a / 41.3                          # no shell radius on a bin edge
    edges = np.arange(0, 61) * dr          # up to 1.45 a < box / 2
    counts = structure.rdf_counts(pos, species, box, edges ** 2)
    expect = np.zeros_like(counts)
    for sh in shells["shells"]:
        r = 0.5 * a * math.sqrt(sh["s"])
        b = int(r // dr)
        assert edges[b] < r < edges[b + 1]
        if sh["like"]:
            expect[0, b] += n_na * sh["count"] // 2
            expect[2, b] += n_cl * sh["count"] // 2
        else:
            expect[1, b] += n_na * sh["count"]
    assert np.array_equal(counts, expect)


def test_ideal_gas_gives_unit_g():
    rng = np.random.default_rng(5)
    n, box = 2000, 30.0
    pos = rng.uniform(0, box, (n, 3))
    species = np.repeat([0, 1], n // 2)
    edges = np.linspace(2.0, 14.0, 25)
    counts = structure.rdf_counts(pos, species, box, edges ** 2)
    g = structure.rdf_normalise(counts, 1, n // 2, n // 2, box, edges)
    for row in range(3):
        sigma = 1.0 / np.sqrt(np.maximum(counts[row], 1))
        assert np.all(np.abs(g[row] - 1.0) < 5 * sigma + 1e-12), (row, g[row])
    # every pair within the range is counted once
    _, _, r2 = structure.pair_r2(pos, box)
    inside = np.sum((r2 >= edges[0] ** 2) & (r2 < edges[-1] ** 2))
    assert counts.sum() == inside


def test_rdf_features_of_analytic_curve():
    r = np.linspace(0.05, 8.0, 160)
    g = np.where(r < 2.0, 0.0, 1.0 + 2.5 * np.exp(-(r - 2.6) ** 2 / 0.1)
                 - 0.6 * np.exp(-(r - 4.2) ** 2 / 0.2))
    # counting noise, including a blip at the onset, must not move them
    g = g + np.where(r < 2.0, 0.0, 0.02 * np.sin(37.0 * r))
    g[np.argmin(np.abs(r - 2.1))] += 0.05
    f = structure.rdf_features(r, g)
    step = r[1] - r[0]
    assert abs(f["r_cut"] - 2.0) <= step
    assert abs(f["r_max"] - 2.6) <= step
    assert abs(f["g_max"] - 3.5) < 0.02
    assert abs(f["r_min"] - 4.2) <= 2 * step


def test_ballistic_correlations_exact():
    rng = np.random.default_rng(2)
    n, tau = 40, 0.25
    species = np.repeat([0, 1], n // 2)
    r0 = rng.uniform(0, 10, (n, 3))
    v = rng.standard_normal((n, 3)) * 0.01
    max_lag, every, K = 12, 3, 40
    tc = structure.TimeCorrelations(species, max_lag, every)
    for k in range(K):
        tc.sample(r0 + (k * tau) * v, v)
    # origins at 0, 3, 6, ...; lag l is seen once per origin k_o <= K-1-l
    for lag in range(max_lag + 1):
        assert tc.counts[lag] == (K - 1 - lag) // every + 1
    vacf, msd = tc.averages()
    v2 = np.sum(v * v, axis=1)
    for s in (0, 1):
        m2 = v2[species == s].mean()
        np.testing.assert_allclose(vacf[s], m2, rtol=1e-13)
        lags = np.arange(max_lag + 1)
        np.testing.assert_allclose(msd[s], m2 * (lags * tau) ** 2, rtol=1e-9, atol=1e-18)


def test_random_walk_diffusion():
    """Steps of variance sigma^2 per component every tau: MSD = 3 sigma^2 l,
    so D = sigma^2 / (2 tau) from the Einstein slope."""
    rng = np.random.default_rng(8)
    n, sigma, tau = 4000, 0.05, 1.0
    species = np.repeat([0, 1], n // 2)
    pos = np.zeros((n, 3))
    tc = structure.TimeCorrelations(species, 20, 5)
    for k in range(200):
        tc.sample(pos, np.zeros((n, 3)))
        pos = pos + sigma * rng.standard_normal((n, 3))
    _, msd = tc.averages()
    D = structure.diffusion_from_msd(msd[0], tau, start=2)
    assert abs(D / (sigma ** 2 / (2 * tau)) - 1.0) < 0.05
