"""Edge cases of the assignment and of both PLCG forms, through the C ABI,
against the FP64 oracle.

- Ragged grids whose last spreading tile holds a single plane (N = 8k + 1):
  the cubic B-spline support of an ion in cell N-2 wraps onto point 0 from
  a tile two tiles away.
- Ions exactly on grid points (the unjittered rock-salt lattice, where every
  site is a grid point), on cell faces along single axes, at x = 0 and at
  the largest double below L, and far outside the box (-1.5 L, +2.5 L),
  which must act as their periodic images.
- The two-iteration form at 128^3 against the full oracle, in the launch
  shapes the session's tuner picks there.

Bars: the assigned charge bit-exact where its arithmetic is exact (linear
weights on grid points: every product is +-1 or 0, and every sum is of
integers), else within 1e-14 absolute; FP64 field within 1e-10 relative L2,
forces within 1e-8 relative, energy within 1e-10 relative; mixed precision
within kappa times its relative residual.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

GRID_Q = 3

FIELD_TOL = 1e-10
FORCE_TOL = 1e-8
FORMS = [("sweep", 0), ("sstep", 16)]  # 16 = MAZE_FLAG_SSTEP


@pytest.fixture(scope="module")
def maze():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze as m
    m.lib()
    assert m.MAZE_FLAG_SSTEP == 16 and m.GRID_Q == GRID_Q
    return m


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def kappa(N):
    return 12.0 / (2.0 * (1.0 - math.cos(2.0 * math.pi / N)))


def check_step(g, o, p, order, exact_q=False, tol_iters=3, zero_force=False):
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert out["status"] == 0 and ref["status"] == 0
    q = g.grid(GRID_Q).cpu().numpy()  # the assigned charge before projection
    q_ref = oracle.spread_raw(p, o.charges, o.box, o.N, order)
    if exact_q:
        assert np.array_equal(q, q_ref)
    else:
        np.testing.assert_allclose(q, q_ref, rtol=0, atol=1e-14)
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    F = out["forces"].cpu().numpy()
    if zero_force:
        # forces vanish by symmetry, so a relative bar is meaningless: both
        # sides within 1e-9 of the force scale k / h^2
        scale = o.cfg.coulomb_k / (o.box / o.N) ** 2
        assert np.abs(F - ref["forces"]).max() <= 1e-9 * scale
        assert np.abs(F).max() <= 1e-9 * scale
    else:
        assert rel(F, ref["forces"]) <= FORCE_TOL
    assert abs(out["energy"].item() - ref["energy"]) <= 1e-10 * abs(ref["energy"])
    assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= tol_iters
    return out


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form,flags", FORMS)
@pytest.mark.parametrize("N,order", [(25, 4), (33, 4), (41, 2), (9, 4)])
def test_single_plane_last_tile(maze, form, flags, N, order):
    """N = 8k + 1 leaves a last spreading tile of one plane; ions are placed
    in cells N-2 and N-1 of every axis, whose supports wrap onto point 0."""
    box = 0.4 * N
    h = box / N
    rng = np.random.default_rng(N)
    n_pairs = 3 * N
    pos = rng.uniform(0, box, (2 * n_pairs, 3))
    # a third of the ions in the last two cells along one or more axes
    for i in range(0, 2 * n_pairs, 3):
        ax = i % 3
        pos[i, ax] = (N - 2 + rng.uniform(0, 2)) * h
        if i % 2 == 0:
            pos[i, (ax + 1) % 3] = (N - 2 + rng.uniform(0, 2)) * h
    Q = np.repeat([1.0, -1.0], n_pairs)
    vel = rng.standard_normal(pos.shape) * 0.02
    print(f"case: single-plane last tile {form} N={N} order={order}", flush=True)
    g = maze.Session(dev(Q), dev(pos), box, h, tol=1e-13, order=order, flags=flags)
    o = oracle.Session(Q, pos, box, h, tol=1e-13, order=order)
    assert g.N == N == o.N
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    for k in range(2):
        check_step(g, o, pos + (k + 1) * vel, order)
    g.close()
    o.close()


def lattice_cases(s):
    """Position sets of the reading on ions at cell faces: the unjittered
    lattice (every ion on a grid point); ions on single cell faces; ions at 0
    and just below L; ions far outside the box."""
    L, h = s.box, s.box / round(s.box / s.grid_spacing)
    lat, _, _ = inputs.rocksalt_sites(s.n_cells, inputs.LATTICE_A)
    faces = s.pos.copy()
    faces[0::4, 0] = np.round(faces[0::4, 0] / h) * h  # x on a face, y and z inside
    faces[1::4, 1] = np.round(faces[1::4, 1] / h) * h
    faces[2::4, 2] = np.round(faces[2::4, 2] / h) * h
    faces[3, :] = 0.0
    faces[5, :] = np.nextafter(L, 0.0)
    faces[6, 0] = np.nextafter(L, 0.0)
    faces[6, 1] = 0.0
    images = s.pos.copy()
    images[0] = (-1.5 * L, 2.5 * L, -1.5 * L)
    images[1] = (2.5 * L, -1.5 * L, 2.5 * L)
    images[4::7, 0] -= 2.0 * L
    images[5::7, 1] += 3.0 * L
    images[6::7, 2] -= 5.0 * L
    return {"lattice": lat, "faces": faces, "images": images}


@pytest.mark.parametrize("form,flags", FORMS)
@pytest.mark.parametrize("order", [2, 4])
def test_ions_on_grid_points_faces_and_images(maze, form, flags, order):
    s = inputs.molten_nacl(2, seed=1)
    cases = lattice_cases(s)
    print(f"case: lattice/faces/images {form} order {order}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-13, order=order,
                     flags=flags, coulomb_k=inputs.COULOMB_K_EV_A)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13, order=order,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    for name in ("lattice", "faces", "images", "lattice"):
        print(f"  positions: {name}", flush=True)
        # on the perfect lattice every ion feels zero force by symmetry
        check_step(g, o, cases[name], order, exact_q=(name == "lattice" and order == 2),
                   zero_force=(name == "lattice"))
    g.close()
    o.close()


@pytest.mark.parametrize("form,flags", FORMS)
def test_far_images_equal_wrapped_positions(maze, form, flags):
    """Positions far outside the box give bitwise the result of their images
    in [0, L): the cell decision wraps them before anything else."""
    s = inputs.molten_nacl(2, seed=1)
    images = lattice_cases(s)["images"]
    wrapped = images - s.box * np.floor(images / s.box)
    outs = []
    for p in (images, wrapped):
        g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12,
                         flags=flags)
        outs.append(g.step(dev(p), want_field=True))
        g.close()
    assert torch.equal(outs[0]["field"], outs[1]["field"])
    assert torch.equal(outs[0]["forces"], outs[1]["forces"])


# ---------------------------------------------------------------------------
def test_sstep_full_parity_128_fp64(maze):
    """4096 ions on 128^3, two-iteration form in its tuned shapes: the cold
    solve and two warm steps against the full oracle."""
    s = inputs.molten_nacl(8, seed=2)
    print("case: sstep nacl4096 128^3 fp64", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12,
                     coulomb_k=inputs.COULOMB_K_EV_A, flags=maze.MAZE_FLAG_SSTEP)
    print(f"  update shape {maze.maze_launch_shape(g.handle)} basis "
          f"{maze.maze_basis_shape(g.handle)}", flush=True)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    for k in range(2):
        check_step(g, o, s.pos + (k + 1) * s.vel, 2, tol_iters=4)
    g.close()
    o.close()


def test_sstep_full_parity_128_mixed(maze):
    """The same workload in mixed precision at a 1e-8 relative residual: the
    field within kappa(N) times the residual of the FP64 oracle's converged
    answer, forces and energy stated."""
    s = inputs.molten_nacl(8, seed=2)
    tol = 1e-8
    print("case: sstep nacl4096 128^3 mixed", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                     precision=maze.MAZE_MIXED, coulomb_k=inputs.COULOMB_K_EV_A,
                     flags=maze.MAZE_FLAG_SSTEP)
    print(f"  update shape {maze.maze_launch_shape(g.handle)} basis "
          f"{maze.maze_basis_shape(g.handle)}", flush=True)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        st = out["stats"]
        assert out["status"] == 0 and st["rel_residual"] <= tol
        ef = rel(out["field"], ref["field"])
        eF = rel(out["forces"], ref["forces"])
        eE = abs(out["energy"].item() - ref["energy"]) / abs(ref["energy"])
        print(f"  mixed step {k + 1}: iters {st['iters']} refinements {st['refinements']} "
              f"res {st['rel_residual']:.2e} field {ef:.2e} forces {eF:.2e} energy {eE:.2e}",
              flush=True)
        assert ef <= kappa(g.N) * st["rel_residual"] * 1.01 + 1e-12
        assert eF <= 1e-4 and eE <= 1e-6
    g.close()
    o.close()
