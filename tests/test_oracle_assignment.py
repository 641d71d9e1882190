"""Pins of the oracle's charge assignment and force interpolation against
closed forms and exact invariants (partition of unity, moment
reproduction, translation, momentum conservation, zero self-force, plane
waves, far-field Coulomb)."""
import json
import os

import numpy as np
import pytest

from conftest import fft_poisson

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    return json.load(open(os.path.join(GOLDEN, "textbook_values.json")))


def test_cubic_bspline_weights_textbook(oracle_lib):
    N, box = 16, 16.0  # h = 1
    for e in _golden()["cubic_bspline_weights"]:
        idx, w = oracle_lib.axis_weights(4, 5.0 + e["t"], box, N)
        np.testing.assert_allclose(w, e["w"], rtol=0, atol=1e-15)
        assert list(idx) == [4, 5, 6, 7]


def test_linear_weights_textbook(oracle_lib):
    for e in _golden()["linear_weights"]:
        idx, w = oracle_lib.axis_weights(2, 3.0 + e["t"], 16.0, 16)
        np.testing.assert_allclose(w, e["w"], atol=1e-15)
        assert list(idx) == [3, 4]


@pytest.mark.parametrize("order", [2, 4])
def test_weights_partition_of_unity_and_first_moment(oracle_lib, order):
    rng = np.random.default_rng(order)
    N, box = 12, 5.0
    h = box / N
    for x in rng.uniform(0, box, 50):
        idx, w = oracle_lib.axis_weights(order, x, box, N)
        assert abs(w.sum() - 1.0) < 1e-14
        assert (w >= 0).all()
        # unwrap the support next to x and check sum w_i x_i = x
        xi = idx * h
        xi = xi + box * np.round((x - xi) / box)
        assert abs((w * xi).sum() - x) < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_spread_conserves_charge_and_is_periodic(oracle_lib, order):
    rng = np.random.default_rng(11)
    box, N = 7.3, 14
    pos = rng.uniform(-box, 2 * box, (20, 3))
    Q = rng.standard_normal(20)
    q = oracle_lib.spread_raw(pos, Q, box, N, order)
    assert abs(q.sum() - Q.sum()) < 1e-12
    q2 = oracle_lib.spread_raw(pos + box * rng.integers(-2, 3, (20, 3)), Q, box, N, order)
    np.testing.assert_allclose(q, q2, atol=1e-12)


def test_spread_on_grid_point_is_one_hot(oracle_lib):
    box, N = 8.0, 16
    h = box / N
    q = oracle_lib.spread_raw(np.array([[3 * h, 5 * h, 15 * h]]), np.array([2.5]), box, N, 2)
    assert q[3, 5, 15] == 2.5 and np.count_nonzero(q) == 1
    q4 = oracle_lib.spread_raw(np.array([[3 * h, 5 * h, 15 * h]]), np.array([1.0]), box, N, 4)
    w = np.array([1 / 6, 2 / 3, 1 / 6])
    ref = np.einsum("i,j,k->ijk", w, w, w)
    np.testing.assert_allclose(q4[2:5, 4:7, [14, 15, 0]], ref, atol=1e-15)
    assert abs(q4.sum() - 1) < 1e-14 and np.count_nonzero(q4) == 27


@pytest.mark.parametrize("N", [25, 33])
def test_spread_wraps_on_single_plane_last_tile(oracle_lib, N):
    """N = 8k + 1: an ion in cell N - 2 spreads its cubic B-spline onto
    points N-3, N-2, N-1 and 0 of each axis, with the centred B-spline's
    closed-form weights at t = 0.25 (the GPU spreads by 8^3-point tiles, and
    N - 1 alone is then the last tile)."""
    box = 0.4 * N
    h = box / N
    t = 0.25
    b = lambda s: (2 / 3 - s * s + abs(s) ** 3 / 2) if abs(s) < 1 else \
        ((2 - abs(s)) ** 3 / 6 if abs(s) < 2 else 0.0)
    w = np.array([b(1 + t), b(t), b(1 - t), b(2 - t)])
    q = oracle_lib.spread_raw(np.array([[(N - 2 + t) * h] * 3]), np.array([1.0]), box, N, 4)
    idx = [N - 3, N - 2, N - 1, 0]
    np.testing.assert_allclose(q[np.ix_(idx, idx, idx)], np.einsum("i,j,k->ijk", w, w, w),
                               rtol=0, atol=1e-15)
    assert np.count_nonzero(q) == 64 and abs(q.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("order", [2, 4])
def test_spread_translation_by_one_cell(oracle_lib, order):
    rng = np.random.default_rng(2)
    box, N = 6.4, 16
    h = box / N
    pos = rng.uniform(0, box, (9, 3))
    Q = rng.standard_normal(9)
    q = oracle_lib.spread_raw(pos, Q, box, N, order)
    q2 = oracle_lib.spread_raw(pos + np.array([h, 0, 0]), Q, box, N, order)
    np.testing.assert_allclose(np.roll(q, 1, axis=0), q2, atol=1e-12)
    q3 = oracle_lib.spread_raw(pos + np.array([0, 0, -h]), Q, box, N, order)
    np.testing.assert_allclose(np.roll(q, -1, axis=2), q3, atol=1e-12)


def test_spread_projection_makes_grid_neutral(oracle_lib):
    """A unit charge on a grid point plus a uniform background: 1 - 1/G on
    that point and -1/G everywhere else."""
    box, N = 8.0, 8
    h = box / N
    q = oracle_lib.spread(np.array([[2 * h, 3 * h, 7 * h]]), np.array([1.0]), box, N)
    G = N ** 3
    ref = np.full((N, N, N), -1.0 / G)
    ref[2, 3, 7] = 1.0 - 1.0 / G
    np.testing.assert_allclose(q, ref, atol=1e-16)
    assert abs(q.sum()) < 1e-13


@pytest.mark.parametrize("order", [2, 4])
def test_gather_plane_wave_closed_form(oracle_lib, order):
    """phi_n = cos(2 pi m i / N): the central difference along x is
    -sin(2 pi m i / N) sin(2 pi m / N) / h; an ion on grid point i with linear
    weights sees exactly that, so F_x = k Q sin(th_i) sin(2 pi m / N) / h."""
    box, N, m = 9.0, 18, 2
    h = box / N
    i = np.arange(N)
    phi = np.cos(2 * np.pi * m * i / N)[:, None, None] * np.ones((N, N, N))
    pos = np.array([[5 * h, 2 * h, 7 * h], [11 * h, 0.0, 3 * h]])
    Q = np.array([1.5, -0.5])
    F = oracle_lib.gather(pos, Q, box, phi, order=2, coulomb_k=2.0)
    ref = 2.0 * Q * np.sin(2 * np.pi * m * np.array([5, 11]) / N) * np.sin(2 * np.pi * m / N) / h
    np.testing.assert_allclose(F[:, 0], ref, atol=1e-13)
    np.testing.assert_allclose(F[:, 1:], 0.0, atol=1e-13)
    if order == 4:
        # cubic weights (1/6, 2/3, 1/6) average the derivative over i-1, i, i+1
        F4 = oracle_lib.gather(pos, Q, box, phi, order=4, coulomb_k=2.0)
        s = np.sin(2 * np.pi * m / N)
        g = lambda ii: np.sin(2 * np.pi * m * ii / N) * s / h
        ref4 = 2.0 * Q * np.array([g(5 - 1) / 6 + 2 * g(5) / 3 + g(5 + 1) / 6,
                                   g(11 - 1) / 6 + 2 * g(11) / 3 + g(11 + 1) / 6])
        np.testing.assert_allclose(F4[:, 0], ref4, atol=1e-13)


def _solve_forces(oracle_lib, pos, Q, box, N, order=2):
    h = box / N
    q = oracle_lib.spread(pos, Q, box, N, order)
    phi = fft_poisson(q, h)
    return oracle_lib.gather(pos, Q, box, phi, order=order), phi, q


@pytest.mark.parametrize("order", [2, 4])
def test_total_force_vanishes(oracle_lib, order):
    """Same weights for spreading and interpolation plus central differences
    conserve momentum (Section 2.1, paragraph after equation F_nostra)."""
    rng = np.random.default_rng(4)
    box, N = 10.0, 20
    pos = rng.uniform(0, box, (24, 3))
    Q = np.repeat([1.0, -1.0], 12)
    F, _, _ = _solve_forces(oracle_lib, pos, Q, box, N, order)
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale * len(Q)


@pytest.mark.parametrize("order", [2, 4])
def test_zero_self_force(oracle_lib, order):
    """One charge in a neutralising background feels no force at any offset
    inside the cell (Section 2.1: no self-energy term in the force)."""
    rng = np.random.default_rng(6)
    box, N = 6.0, 12
    for off in rng.uniform(0, box, (4, 3)):
        F, phi, _ = _solve_forces(oracle_lib, off[None, :], np.array([1.0]), box, N, order)
        assert np.abs(F).max() < 1e-12 * np.abs(phi).max()
        # the weight-gradient force of equation F_Benoit does not have this property
    Fb = oracle_lib.gather(np.array([[0.31 * box / N, 0, 0]]), np.array([1.0]), box,
                           _solve_forces(oracle_lib, np.array([[0.31 * box / N, 0, 0]]),
                                         np.array([1.0]), box, N, 2)[1],
                           order=2, weight_gradient=True)
    assert np.abs(Fb).max() > 1e-6


def test_newton_third_law_two_ions(oracle_lib):
    box, N = 8.0, 16
    pos = np.array([[1.1, 2.3, 3.7], [4.9, 2.0, 6.1]])
    F, _, _ = _solve_forces(oracle_lib, pos, np.array([1.0, -1.0]), box, N)
    np.testing.assert_allclose(F[0], -F[1], atol=1e-13 * np.abs(F).max())


def ewald_pair_force(r_vec, box, alpha=None, kmax=12, nmax=3):
    """Periodic Coulomb force on +1 at r_vec from -1 at the origin (Ewald
    sum, Gaussian units). Independent of anything on the grid."""
    from math import erfc, exp, pi, sqrt
    if alpha is None:
        alpha = 5.0 / box
    F = np.zeros(3)
    for nx in range(-nmax, nmax + 1):
        for ny in range(-nmax, nmax + 1):
            for nz in range(-nmax, nmax + 1):
                d = r_vec + box * np.array([nx, ny, nz])
                r = np.linalg.norm(d)
                g = erfc(alpha * r) / r ** 2 + 2 * alpha / sqrt(pi) * exp(-(alpha * r) ** 2) / r
                F += -g * d / r  # attraction: q1 q2 = -1
    V = box ** 3
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kz in range(-kmax, kmax + 1):
                if kx == ky == kz == 0:
                    continue
                k = 2 * pi * np.array([kx, ky, kz]) / box
                k2 = k @ k
                F += -(4 * pi / V) * k / k2 * exp(-k2 / (4 * alpha ** 2)) * np.sin(k @ r_vec)
    return F


def test_far_field_matches_periodic_coulomb(oracle_lib):
    """Two opposite charges at h << r << L: the grid force approaches the
    periodic Coulomb force with O(h^2) error (Appendix A: the MaZe potential
    approaches Coulomb away from the charges)."""
    box, N = 12.0, 96
    r = np.array([3.05, 0.72, 0.31])
    pos = np.array([[2.0, 3.0, 4.0], [2.0, 3.0, 4.0]])
    pos[0] += r
    F, _, _ = _solve_forces(oracle_lib, pos, np.array([1.0, -1.0]), box, N)
    ref = ewald_pair_force(r, box)
    assert np.linalg.norm(F[0] - ref) < 0.02 * np.linalg.norm(ref)
    assert np.dot(F[0], r) < 0  # attraction


@pytest.mark.parametrize("order", [2, 4])
def test_weight_gradient_force_is_energy_gradient(oracle_lib, order):
    """Equation F_Benoit: with phi the exact discrete Poisson solution,
    V = (1/2) phi.q = (1/2) q^T G q with G symmetric, so
    dV/dr_a = phi . dq/dr_a = Q_a sum_n grad W phi_n: the weight-gradient
    force is minus the gradient of the discrete energy (equation
    energy_discr). Checked by a centred difference that stays inside one
    cell, where the weights are polynomials in the position."""
    from conftest import fft_poisson
    box, N = 6.0, 12
    h = box / N
    pos = np.array([[1.13, 2.27, 3.41], [4.02, 1.61, 0.77], [2.55, 4.48, 5.12],
                    [0.64, 3.33, 2.09]])
    Q = np.array([1.0, -1.0, 1.0, -1.0])

    def energy(p):
        q = oracle_lib.spread(p, Q, box, N, order)
        phi = fft_poisson(q, h)
        return oracle_lib.energy(phi, q), phi

    _, phi = energy(pos)
    Fb = oracle_lib.gather(pos, Q, box, phi, order=order, weight_gradient=True)
    d = 1e-4
    for a in range(len(Q)):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, c] += d
            pm[a, c] -= d
            # both sides in the same cell of every axis
            assert np.floor(pp[a, c] / h) == np.floor(pm[a, c] / h)
            g = (energy(pp)[0] - energy(pm)[0]) / (2 * d)
            tol = 1e-7 if order == 2 else 1e-6
            assert abs(-g - Fb[a, c]) <= tol * np.abs(Fb).max() + 1e-12, (a, c, -g, Fb[a, c])
