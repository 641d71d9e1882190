"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: FP64 field within 1e-10 relative L2 and forces within 1e-8 relative
of the oracle; integer and index work bit-exact. Sizes span several
segments, x runs and spreading tiles with ragged tails; the full-size
256^3 case is checked through properties computed by the oracle from the
GPU's own outputs.
"""
import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10
FORCE_TOL = 1e-8


@pytest.fixture(scope="module")
def maze():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze as m
    m.lib()
    return m


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def random_system(n_pairs, box, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, box, (2 * n_pairs, 3))
    Q = np.repeat([1.0, -1.0], n_pairs)
    vel = rng.standard_normal(pos.shape) * 0.02
    return pos, Q, vel


def kappa(N):
    """Condition number of -M on mean-zero vectors: 12 / (2 (1 - cos 2pi/N))."""
    return 12.0 / (2.0 * (1.0 - math.cos(2.0 * math.pi / N)))


def c1():
    return inputs.molten_nacl(2, seed=1)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4])
def test_init_and_steps_match_oracle(maze, order):
    s = c1()
    print(f"case: nacl64 32^3 order {order}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-13, order=order,
                     coulomb_k=inputs.COULOMB_K_EV_A)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13, order=order,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    phi0 = g.grid(maze.GRID_PHI)
    assert rel(phi0, o.state()["phi_k"]) <= FIELD_TOL
    assert abs(g.init_stats["iters"] - o.init_stats["iters"]) <= 2
    for k in range(3):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == 0
        assert rel(out["field"], ref["field"]) <= FIELD_TOL
        assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
        assert abs(out["energy"].item() - ref["energy"]) <= 1e-10 * abs(ref["energy"])
        assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 2
        assert out["stats"]["rel_residual"] <= 1e-13 * 1.05
    g.close()


def test_lockstep_cg_iterates(maze):
    """Fixed iteration count (tolerance unreachable): the GPU iterates equal
    the oracle's iterate for iterate, not just the converged answer."""
    s = c1()
    print("case: lockstep nacl64 32^3 max_iter 12", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-300, max_iter=12)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-300, max_iter=12)
    assert g.init_status == maze.MAZE_NOT_CONVERGED and o.init_status == oracle.NOT_CONVERGED
    assert g.init_stats["iters"] == 12
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= 1e-12
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == maze.MAZE_NOT_CONVERGED
        assert out["stats"]["iters"] == 12
        assert rel(g.grid(maze.GRID_Y), o.state()["y"]) <= 1e-12
        assert rel(out["field"], ref["field"]) <= 1e-12
        assert abs(out["stats"]["rel_residual"] - ref["stats"]["rel_residual"]) <= \
            1e-9 * ref["stats"]["rel_residual"]


@pytest.mark.parametrize("N,n_pairs,order", [(4, 3, 2), (4, 2, 4), (20, 17, 2), (36, 40, 4),
                                            (50, 60, 2), (100, 150, 2)])
def test_ragged_grids(maze, N, n_pairs, order):
    """Grid sizes that leave ragged plane segments, x runs and spreading
    tiles (and the smallest grid, where every halo wraps onto itself)."""
    box = 0.4 * N
    pos, Q, vel = random_system(n_pairs, box, seed=N)
    print(f"case: ragged N={N} ions={2 * n_pairs} order={order}", flush=True)
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=1e-13, order=order)
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-13, order=order)
    assert g.N == N == o.N
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    p = pos + vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    g.close()


def test_assigned_charge_and_constraint_match(maze):
    s = c1()
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-13)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13)
    p = s.pos + s.vel
    g.step(dev(p))
    o.step(p)
    st = o.state()
    q = g.grid(maze.GRID_Q).cpu().numpy()
    np.testing.assert_allclose(q - q.mean(), st["q"], rtol=0, atol=1e-14)
    assert rel(g.grid(maze.GRID_SIGMA), st["sigma_p"]) <= 1e-12
    assert rel(g.grid(maze.GRID_Y), st["y"]) <= FIELD_TOL


@pytest.mark.parametrize("guess", [0, 1, 2])
def test_direct_solve_guesses(maze, guess):
    s = c1()
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12)
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        g.step(dev(p))
        o.step(p)
    p = s.pos + 3 * s.vel
    phi_before = g.grid(maze.GRID_PHI).clone()
    out = g.solve(dev(p), guess=guess)
    ref = o.solve(p, guess=guess)
    assert torch.equal(phi_before, g.grid(maze.GRID_PHI))  # history untouched
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 2


def test_absmax_residual_norm(maze):
    s = c1()
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-9,
                     residual_norm=maze.MAZE_NORM_ABSMAX)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-9,
                       residual_norm=oracle.NORM_ABSMAX)
    p = s.pos + s.vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert out["stats"]["max_abs_residual"] <= 1e-9
    assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 2


def test_errors_leave_state_unchanged(maze):
    s = c1()
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-10)
    before = [g.grid(w).clone() for w in (maze.GRID_PHI, maze.GRID_PHI_PREV, maze.GRID_Y)]
    bad = s.pos.copy()
    bad[5, 2] = np.nan
    with pytest.raises(maze.MazeError) as e:
        g.step(dev(bad))
    assert e.value.status == maze.MAZE_E_NONFINITE
    after = [g.grid(w) for w in (maze.GRID_PHI, maze.GRID_PHI_PREV, maze.GRID_Y)]
    for a, b in zip(before, after):
        assert torch.equal(a, b)
    out = g.step(dev(s.pos + s.vel))  # the session still works
    assert out["status"] == 0
    with pytest.raises(maze.MazeError) as e:
        maze.Session(dev(s.charges + 0.01), dev(s.pos), s.box, s.grid_spacing)
    assert e.value.status == maze.MAZE_E_NOT_NEUTRAL
    with pytest.raises(maze.MazeError) as e:
        maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, order=3)
    assert e.value.status == maze.MAZE_E_INVALID
    g1 = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12, max_iter=1)
    assert g1.init_status == maze.MAZE_NOT_CONVERGED
    out = g1.step(dev(s.pos + s.vel))
    assert out["status"] == maze.MAZE_NOT_CONVERGED and out["stats"]["iters"] == 1


def test_bitwise_determinism_and_checkpoint(maze):
    s = c1()
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-10)
    g.step(dev(s.pos + s.vel))
    blob = g.save()
    p = dev(s.pos + 2 * s.vel)
    a = g.step(p, want_field=True)
    a2 = g.step(dev(s.pos + 3 * s.vel), want_field=True)
    g.load(blob)
    b = g.step(p, want_field=True)
    b2 = g.step(dev(s.pos + 3 * s.vel), want_field=True)
    assert torch.equal(a["field"], b["field"]) and torch.equal(a["forces"], b["forces"])
    assert torch.equal(a2["field"], b2["field"]) and torch.equal(a2["forces"], b2["forces"])
    assert a2["stats"]["iters"] == b2["stats"]["iters"]
    with pytest.raises(maze.MazeError):
        g.load(blob[:100])


def test_mixed_precision_error_vs_fp64_oracle(maze):
    """Mixed precision reaches the FP64 residual target; its field error is
    within the rigorous bound kappa * relative residual."""
    s = c1()
    tol = 1e-8
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                     precision=maze.MAZE_MIXED, coulomb_k=inputs.COULOMB_K_EV_A)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    for k in range(4):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        st = out["stats"]
        assert out["status"] == 0 and st["rel_residual"] <= tol
        ef = rel(out["field"], ref["field"])
        eF = rel(out["forces"], ref["forces"])
        eE = abs(out["energy"].item() - ref["energy"]) / abs(ref["energy"])
        print(f"mixed step {k + 1}: iters {st['iters']} refinements {st['refinements']} "
              f"res {st['rel_residual']:.2e} field {ef:.2e} forces {eF:.2e} energy {eE:.2e}")
        assert ef <= kappa(g.N) * st["rel_residual"] * 1.01 + 1e-12
        assert eF <= 1e-4


def test_full_parity_128(maze):
    """4096 ions on 128^3: init and one warm step against the full oracle."""
    s = inputs.molten_nacl(8, seed=2)
    print("case: nacl4096 128^3", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12,
                     coulomb_k=inputs.COULOMB_K_EV_A)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    p = s.pos + s.vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 3


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_256_properties(maze, precision):
    """32768 ions on 256^3 in the benchmark's launch shape: the oracle checks
    the GPU field through the discrete Poisson residual it must satisfy, and
    recomputes the interpolated forces and the energy from that field."""
    s = inputs.molten_nacl(16, seed=3)
    tol = 1e-9 if precision == 0 else 1e-8
    print(f"case: nacl32768 256^3 precision {precision}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                     precision=precision, coulomb_k=inputs.COULOMB_K_EV_A)
    p = s.pos + s.vel
    out = g.step(dev(p), want_field=True)
    N = g.N
    h = s.box / N
    phi = out["field"].cpu().numpy()
    q = oracle.spread(p, s.charges, s.box, N)
    res = oracle.apply_M(phi) + 4 * np.pi * q / h
    r_rel = np.linalg.norm(res) / np.linalg.norm(4 * np.pi * q / h)
    assert r_rel <= tol * 1.001, r_rel
    assert abs(out["stats"]["rel_residual"] - r_rel) <= 1e-3 * r_rel + 1e-15
    F_ref = oracle.gather(p, s.charges, s.box, phi, coulomb_k=inputs.COULOMB_K_EV_A)
    assert rel(out["forces"], F_ref) <= 1e-13
    e_ref = oracle.energy(phi, q, inputs.COULOMB_K_EV_A)
    assert abs(out["energy"].item() - e_ref) <= 1e-11 * abs(e_ref)
    assert abs(phi.mean()) <= 1e-14 * np.abs(phi).max()


def test_md_matches_oracle_md(maze):
    """Ten velocity-Verlet steps with MaZe + short range, GPU vs oracle."""
    from paper_2505_20418_amd.md import MDRun
    s = c1()
    run = MDRun(s, tol=1e-12)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    pos, vel = s.pos.copy(), s.vel.copy()
    F_es = o.step(pos)["forces"]
    F_sr, _ = oracle.bmh(pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    work = np.zeros(1)
    np.testing.assert_allclose(run.f_sr.cpu().numpy(), F_sr, rtol=0, atol=1e-10)
    for _ in range(10):
        run.step()
        o.md_step(pos, vel, s.masses, s.species, inputs.BMH_TABLE, inputs.BMH_CUTOFF, 1.0,
                  inputs.ACCEL_FACTOR, F_es, F_sr, work)
    assert np.abs(run.pos.cpu().numpy() - pos).max() <= 1e-9
    assert np.abs(run.vel.cpu().numpy() - vel).max() <= 1e-10
    obs = run.observables()
    assert abs(obs["work"] - work[0]) <= 1e-8 * max(1.0, abs(work[0]))
    assert np.abs(obs["momentum"]).max() <= 1e-8


@pytest.mark.parametrize("n_cells,grid_n", [(8, 128), (4, 60)])
def test_short_range_tiles_match_oracle(maze, n_cells, grid_n):
    """The short-range term searched over the MaZe tiles (a 5^3 or 7^3 tile
    block) against the oracle's all-pairs sum, including a grid whose last
    tile along each axis is partial."""
    from paper_2505_20418_amd.md import MDRun
    s = inputs.molten_nacl(n_cells, seed=7)
    s.grid_spacing = s.box / grid_n
    print(f"case: short range ions={s.n_ions} N={grid_n}", flush=True)
    run = MDRun(s, tol=1e-6)
    assert run.session.N == grid_n
    F_ref, e_ref = oracle.bmh(s.pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    F = run.f_sr.cpu().numpy()
    assert np.abs(F - F_ref).max() <= 1e-10 * max(1.0, np.abs(F_ref).max())
    assert abs(run.observables()["v_sr"] - e_ref) <= 1e-10 * abs(e_ref)
    run.close()
