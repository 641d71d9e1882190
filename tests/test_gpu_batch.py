"""Batched stepping (maze_step_batch) through the C ABI.

Sessions of uneven size and mixed precision advance together, one launch
per CG sweep and template class covering all of them. Each session's
result must be bitwise the one it gets stepped alone while the batch stays
below the throughput fill level (same kernels, same geometry, same
fixed-order reductions); a batch swept in the throughput shapes must meet
every tolerance and agree with the step alone within the bound the
tolerance implies; a rejected member must leave only itself unchanged, and
a batch member must agree with the oracle.
"""
import math
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

# (n_cells, grid N, precision, tolerance): uneven grids, both precisions,
# segment/halo classes of ppt 1 and 2, a ragged N that is not a multiple of
# the 8-point tile, and a grid below 48
CASES = [(2, 32, 0, 1e-10), (3, 48, 1, 1e-8), (4, 64, 0, 1e-9), (2, 20, 1, 1e-7),
         (5, 76, 1, 1e-8), (8, 128, 0, 1e-8), (3, 36, 0, 1e-11)]


@pytest.fixture(scope="module")
def maze():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze as m
    m.lib()
    return m


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def make(maze, case, seed):
    n_cells, N, prec, tol = case
    s = inputs.molten_nacl(n_cells, seed=seed)
    s.grid_spacing = s.box / N
    sess = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                        precision=prec, coulomb_k=inputs.COULOMB_K_EV_A)
    assert sess.N == N
    return s, sess


def test_batch_is_bitwise_alone(maze):
    print("case: batch of", CASES, flush=True)
    systems, alone, batch = [], [], []
    for i, c in enumerate(CASES):
        s, a = make(maze, c, seed=100 + i)
        _, b = make(maze, c, seed=100 + i)
        systems.append(s)
        alone.append(a)
        batch.append(b)
    # below one workgroup per CU in the throughput shapes: latency mode
    assert sum(maze.maze_launch_shape(b.handle)["throughput"]["nwg"] for b in batch) < 256
    for k in range(3):
        pos = [dev(s.pos + (k + 1) * s.vel) for s in systems]
        ref = [a.step(p, want_field=True) for a, p in zip(alone, pos)]
        forces = [torch.empty(s.n_ions, 3, dtype=torch.float64, device="cuda") for s in systems]
        energies = torch.empty(len(systems), dtype=torch.float64, device="cuda")
        rc, st = maze.maze_step_batch([b.handle for b in batch], pos, forces, energies)
        assert rc == maze.MAZE_OK
        for i, (r, b) in enumerate(zip(ref, batch)):
            assert st[i]["status"] == maze.MAZE_OK
            assert st[i]["iters"] == r["stats"]["iters"], i
            assert st[i]["refinements"] == r["stats"]["refinements"], i
            assert torch.equal(forces[i], r["forces"]), i
            assert torch.equal(energies[i:i + 1], r["energy"]), i
            assert torch.equal(b.grid(maze.GRID_PHI), r["field"]), i
    for x in alone + batch:
        x.close()


def test_batch_member_matches_oracle(maze):
    c = (3, 48, 0, 1e-12)
    s, g = make(maze, c, seed=5)
    _, other = make(maze, (2, 32, 1, 1e-8), seed=6)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        forces = [torch.empty(s.n_ions, 3, dtype=torch.float64, device="cuda"),
                  torch.empty(64, 3, dtype=torch.float64, device="cuda")]
        rc, st = maze.maze_step_batch([g.handle, other.handle],
                                      [dev(p), dev(inputs.molten_nacl(2, seed=6).pos)], forces)
        ref = o.step(p)
        phi = g.grid(maze.GRID_PHI).cpu().numpy()
        assert np.linalg.norm(phi - ref["field"]) <= 1e-10 * np.linalg.norm(ref["field"])
        F = forces[0].cpu().numpy()
        assert np.linalg.norm(F - ref["forces"]) <= 1e-8 * np.linalg.norm(ref["forces"])
    g.close()
    other.close()


def test_batch_rejected_member_is_unchanged(maze):
    systems, sess = [], []
    for i, c in enumerate(CASES[:3]):
        s, x = make(maze, c, seed=200 + i)
        systems.append(s)
        sess.append(x)
    before = sess[1].grid(maze.GRID_PHI).clone()
    y_before = sess[1].grid(maze.GRID_Y).clone()
    pos = [dev(s.pos + s.vel) for s in systems]
    pos[1][3, 1] = float("nan")
    forces = [torch.zeros(s.n_ions, 3, dtype=torch.float64, device="cuda") for s in systems]
    rc, st = maze.maze_step_batch([x.handle for x in sess], pos, forces)
    assert rc == maze.MAZE_E_NONFINITE
    assert st[1]["status"] == maze.MAZE_E_NONFINITE
    assert st[0]["status"] == maze.MAZE_OK and st[2]["status"] == maze.MAZE_OK
    assert torch.equal(sess[1].grid(maze.GRID_PHI), before)
    assert torch.equal(sess[1].grid(maze.GRID_Y), y_before)
    # the rejected session steps normally afterwards
    out = sess[1].step(dev(systems[1].pos + systems[1].vel))
    assert out["status"] == maze.MAZE_OK
    for x in sess:
        x.close()


def test_throughput_mode_within_tolerance_of_alone(maze, monkeypatch):
    """Throughput shapes change the summation order, so the step differs
    from the step alone by at most the two solves' residuals through the
    inverse operator: for the periodic 7-point M the smallest nonzero
    eigenvalue is 2 (1 - cos(2 pi / N)), and each solve leaves
    ||sigma_p - M y|| <= tol ||q||, so ||phi_a - phi_b|| <= (4 pi / h) *
    2 tol ||q|| / lambda_min."""
    print("case: throughput-mode batch of", CASES, flush=True)
    systems, alone, batch = [], [], []
    for i, c in enumerate(CASES):
        s, a = make(maze, c, seed=300 + i)
        _, b = make(maze, c, seed=300 + i)
        systems.append(s)
        alone.append(a)
        batch.append(b)
    shapes = [maze.maze_launch_shape(b.handle) for b in batch]
    assert any(sh["throughput"] != sh["latency"] for sh in shapes), shapes
    monkeypatch.setenv("MAZE_BATCH_MODE", "throughput")
    pos = [dev(s.pos + s.vel) for s in systems]
    ref = [a.step(p, want_field=True) for a, p in zip(alone, pos)]
    forces = [torch.empty(s.n_ions, 3, dtype=torch.float64, device="cuda") for s in systems]
    rc, st = maze.maze_step_batch([b.handle for b in batch], pos, forces)
    assert rc == maze.MAZE_OK
    for i, (c, r, b) in enumerate(zip(CASES, ref, batch)):
        n_cells, N, prec, tol = c
        assert st[i]["status"] == maze.MAZE_OK and st[i]["converged"] == 1, i
        assert st[i]["rel_residual"] <= tol, i
        h = systems[i].box / N
        qn = torch.linalg.norm(b.grid(maze.GRID_Q)).item()
        lam = 2.0 * (1.0 - math.cos(2.0 * math.pi / N))
        bound = (4.0 * math.pi / h) * 2.0 * tol * qn / lam
        d = torch.linalg.norm(b.grid(maze.GRID_PHI) - r["field"]).item()
        assert d <= bound, (i, d, bound)
    for x in alone + batch:
        x.close()
