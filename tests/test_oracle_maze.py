"""Pins of the oracle's MaZe time step, energy and MD driver: the field
reached by the SHAKE update is the Poisson solution (FFT), the residual
identities of the convergence subsection, the Madelung energy of rock salt
under grid refinement, the velocity-Verlet work identity, momentum and
time reversibility."""
import json
import os

import numpy as np
import pytest

from conftest import fft_poisson
from paper_2505_20418_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sys64(seed=1, jitter=0.1):
    return inputs.molten_nacl(2, seed=seed, jitter=jitter)


def _move(s, steps, dt=1.0):
    """Ballistic motion for open-loop tests (no forces needed)."""
    return [s.pos + (k + 1) * dt * s.vel for k in range(steps)]


def test_madelung_energy_converges_under_refinement(oracle_lib):
    """E_grid - Np E_self - Np xi/(2L) -> -Np M / (2 r0) with O(h^2) error
    for ions on a perfect rock-salt lattice (Section 2, equation
    energy_discr; self energy measured with one charge plus background as in
    Appendix A)."""
    tv = json.load(open(os.path.join(GOLDEN, "textbook_values.json")))
    mad = tv["madelung_nacl"]["value"]
    xi = tv["simple_cubic_background_constant"]["value"]
    s0 = _sys64(jitter=0.0)
    L = s0.box
    Np = s0.n_ions
    r0 = L / 4.0
    ref = -Np * mad / (2 * r0)
    errs = []
    for N in (16, 32, 64):
        h = L / N
        sess = oracle_lib.Session(s0.charges, s0.pos, L, h, tol=1e-13)
        e_grid = sess.init_stats["energy"]
        sess.close()
        q1 = oracle_lib.spread(np.zeros((1, 3)), np.ones(1), L, N)
        phi1, _, ok = oracle_lib.pcg(4 * np.pi * q1 / h, thr=1e-13 * np.linalg.norm(4 * np.pi * q1 / h))
        e_self = oracle_lib.energy(phi1, q1)
        errs.append(abs((e_grid - Np * e_self - Np * xi / (2 * L)) - ref) / abs(ref))
    assert errs[-1] < 5e-3
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def test_init_field_is_fft_poisson_solution(oracle_lib):
    s = _sys64()
    N = 32
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13)
    st = sess.state()
    ref = fft_poisson(st["q"], s.box / N)
    assert np.linalg.norm(st["phi_k"] - ref) < 1e-11 * np.linalg.norm(ref)
    assert np.array_equal(st["phi_k"], st["phi_km1"]) and not st["y"].any()


def test_step_reaches_poisson_solution_independent_of_history(oracle_lib):
    """phi^{k+1} = phi_p - (4 pi / h) y* satisfies M phi = -4 pi q / h once the
    SHAKE system is solved (equations SHAKE to SHAKEPhiFinal)."""
    s = _sys64()
    N = 32
    h = s.box / N
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13)
    for pos in _move(s, 4):
        out = sess.step(pos)
        q = oracle_lib.spread(pos, s.charges, s.box, N)
        ref = fft_poisson(q, h)
        assert np.linalg.norm(out["field"] - ref) < 1e-10 * np.linalg.norm(ref)
        assert out["stats"]["rel_residual"] <= 1e-13 * 1.01


def test_step_residual_identity(oracle_lib):
    """The Poisson residual of phi^{k+1} is exactly -(4 pi / h) times the
    MaZe residual M y - sigma_p (convergence subsection, equations res_poisson
    and res_poisson_maze), checked on the oracle's own state with a loose
    tolerance so both residuals are large."""
    s = _sys64()
    N = 32
    h = s.box / N
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-3)
    st0 = sess.state()
    pos = _move(s, 1)[0]
    sess.step(pos)
    st = sess.state()
    phi_p = 2 * st0["phi_k"] - st0["phi_km1"]
    sig = (h / (4 * np.pi)) * oracle_lib.apply_M(phi_p) + st["q"]
    np.testing.assert_allclose(st["sigma_p"], sig, atol=1e-14 * np.abs(sig).max())
    maze_res = oracle_lib.apply_M(st["y"]) - st["sigma_p"]
    pois_res = oracle_lib.apply_M(st["phi_k"]) + 4 * np.pi * st["q"] / h
    assert np.abs(maze_res).max() > 1e-8
    np.testing.assert_allclose(pois_res, -(4 * np.pi / h) * maze_res,
                               atol=1e-9 * np.abs(pois_res).max())


@pytest.mark.parametrize("guess", [0, 1, 2])
def test_direct_solve_guesses_agree_with_maze(oracle_lib, guess):
    s = _sys64()
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12)
    traj = _move(s, 3)
    for p in traj[:2]:
        sess.step(p)
    before = sess.state()
    d = sess.solve(traj[2], guess=guess)
    after = sess.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k  # history untouched
    m = sess.step(traj[2])
    assert np.linalg.norm(d["field"] - m["field"]) < 1e-9 * np.linalg.norm(m["field"])
    np.testing.assert_allclose(d["forces"], m["forces"], atol=1e-8 * np.abs(m["forces"]).max())


def test_maze_needs_fewer_iterations_than_static(oracle_lib):
    """Appendix B: PLCG on the SHAKE system from the previous y converges in
    fewer iterations than the static direct solve (same relative scale)."""
    s = _sys64()
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-9)
    traj = _move(s, 8)
    it_m, it_s, it_t = [], [], []
    for p in traj:
        it_s.append(sess.solve(p, guess=1)["stats"]["iters"])
        it_t.append(sess.solve(p, guess=2)["stats"]["iters"])
        it_m.append(sess.step(p)["stats"]["iters"])
    assert np.mean(it_m[2:]) < np.mean(it_s[2:])
    assert np.mean(it_t[2:]) < np.mean(it_s[2:])


def test_forces_and_energy_gauge_and_momentum(oracle_lib):
    s = _sys64()
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12,
                              coulomb_k=inputs.COULOMB_K_EV_A)
    out = sess.step(_move(s, 1)[0])
    F = out["forces"]
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).max()
    assert abs(out["field"].mean()) < 1e-15 * np.abs(out["field"]).max()


def test_validation_errors(oracle_lib):
    s = _sys64()
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Session(s.charges + 0.01, s.pos, s.box, s.grid_spacing)
    bad = s.pos.copy()
    bad[3, 1] = np.nan
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Session(s.charges, bad, s.box, s.grid_spacing)
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing)
    with pytest.raises(oracle_lib.OracleError):
        sess.step(bad)
    out = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-9, max_iter=1)
    assert out.init_status == oracle_lib.NOT_CONVERGED


def test_bmh_force_is_minus_energy_gradient(oracle_lib):
    s = _sys64()
    F, e = oracle_lib.bmh(s.pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    rng = np.random.default_rng(0)
    for _ in range(5):
        a, c = rng.integers(0, s.n_ions), rng.integers(0, 3)
        d = 1e-5
        p1, p2 = s.pos.copy(), s.pos.copy()
        p1[a, c] += d
        p2[a, c] -= d
        e1 = oracle_lib.bmh(p1, s.species, s.box, inputs.BMH_TABLE)[1]
        e2 = oracle_lib.bmh(p2, s.species, s.box, inputs.BMH_TABLE)[1]
        assert abs(-(e1 - e2) / (2 * d) - F[a, c]) < 1e-6 * max(1.0, abs(F[a, c]))
    assert np.abs(F.sum(axis=0)).max() < 1e-10


def _run_md(oracle_lib, s, steps, tol, dt=1.0):
    sess = oracle_lib.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=tol,
                              coulomb_k=inputs.COULOMB_K_EV_A)
    pos = s.pos.copy()
    vel = s.vel.copy()
    F_es = sess.step(pos)["forces"]  # forces at the start configuration
    F_sr, _ = oracle_lib.bmh(pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    work = np.zeros(1)
    rec = []
    for _ in range(steps):
        x0 = pos.copy()
        f0 = F_es + F_sr
        sess.md_step(pos, vel, s.masses, s.species, inputs.BMH_TABLE, inputs.BMH_CUTOFF,
                     dt, inputs.ACCEL_FACTOR, F_es, F_sr, work)
        rec.append(dict(pos=pos.copy(), vel=vel.copy(), f0=f0, f1=F_es + F_sr, dx=pos - x0))
    return sess, pos, vel, rec


def test_velocity_verlet_work_identity(oracle_lib):
    """KE + W_trap - sum c dt^2 |F|^2 / (8 m) is conserved exactly by velocity
    Verlet for any force (plumbing check of the driver: time index, sign and
    units)."""
    s = _sys64()
    dt = 1.0
    sess, pos, vel, rec = _run_md(oracle_lib, s, 30, 1e-9, dt)
    c = inputs.ACCEL_FACTOR
    m = s.masses[:, None]
    ke0 = 0.5 * (m * s.vel ** 2).sum() / c
    corr0 = (c * dt ** 2 / (8 * m) * rec[0]["f0"] ** 2).sum()
    W = 0.0
    vals = []
    for r in rec:
        W -= 0.5 * ((r["f0"] + r["f1"]) * r["dx"]).sum()
        ke = 0.5 * (m * r["vel"] ** 2).sum() / c
        corr = (c * dt ** 2 / (8 * m) * r["f1"] ** 2).sum()
        vals.append(ke + W - corr)
    base = ke0 - corr0
    assert np.abs(np.array(vals) - base).max() < 1e-9 * ke0


def test_momentum_conserved_at_solver_tolerance(oracle_lib):
    """Total momentum stays at the solver-tolerance level (Results, total
    momentum subsection): looser tolerance, larger drift."""
    s = _sys64()
    drift = {}
    for tol in (1e-5, 1e-11):
        _, _, vel, _ = _run_md(oracle_lib, s, 20, tol)
        drift[tol] = np.linalg.norm((s.masses[:, None] * vel).sum(axis=0))
    assert drift[1e-11] < 1e-7
    assert drift[1e-11] < drift[1e-5]


def test_time_reversibility_short(oracle_lib):
    """Forward 15 steps, flip velocities, 15 back: positions return (time
    reversibility subsection) at a tight tolerance."""
    s = _sys64()
    sess, pos, vel, _ = _run_md(oracle_lib, s, 15, 1e-12)
    s2 = inputs.NaClSystem(**{**s.__dict__, "pos": pos.copy(), "vel": -vel.copy()})
    _, pos_back, _, _ = _run_md(oracle_lib, s2, 15, 1e-12)
    rmsd = np.sqrt(((pos_back - s.pos) ** 2).sum(axis=1)).sum() / (s.n_ions * s.box)
    assert rmsd < 1e-8


def test_generator_masses_reproduce_paper_density():
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["nacl_density"]
    n_pair = g["n_ions"] // 2
    grams = n_pair * (inputs.MASS_NA + inputs.MASS_CL) / 6.02214076e23
    rho = grams / (g["box"] * 1e-8) ** 3
    assert abs(rho - g["density_g_cm3"]) / g["density_g_cm3"] < g["rel_tol"]
