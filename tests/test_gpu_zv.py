"""The wavefront-row layout of the two-iteration PLCG's basis kernel through
the C ABI (grids of N = 64, 128 and 256 points a side, where one z row is 64
lanes of N / 64 points and a wavefront holds whole rows).

- Against the FP64 oracle's PLCG at 64^3 and 128^3: workgroups of 8
  wavefronts (segments of 6 rows, so the last segment of every grid is
  ragged), one x run or many, with update kernels in several segment
  shapes, both precisions, both assignment orders. The update kernel has
  no wavefront-row form: a forced one is refused and the tuner's kept.
- In lockstep with the oracle: an unreachable tolerance stops both after the
  same odd iteration count, and the iterates agree to 1e-11.
- At 256^3 (32768 ions) against the segment layout: the same iterates up to
  the rounding order of the Gram sums, and the field satisfies the discrete
  Poisson residual the oracle computes from it.
- Batched (maze_step_batch and maze_batch_*): bitwise the step alone.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10
FORCE_TOL = 1e-8
SSTEP = 16


@pytest.fixture(scope="module")
def maze():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze as m
    m.lib()
    assert m.MAZE_FLAG_SSTEP == SSTEP
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


def random_system(n_pairs, box, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, box, (2 * n_pairs, 3))
    Q = np.repeat([1.0, -1.0], n_pairs)
    vel = rng.standard_normal(pos.shape) * 0.02
    return pos, Q, vel


def force_shapes(monkeypatch, basis, update):
    for var, v in (("MAZE_BASIS_SHAPE", basis), ("MAZE_UPDATE_SHAPE", update)):
        if v:
            monkeypatch.setenv(var, v)
        else:
            monkeypatch.delenv(var, raising=False)


def zv_waves(shape):
    return int(shape.split(":")[1]) if shape and shape.startswith("zv:") else 0


@pytest.mark.parametrize("N,basis,update,precision,order", [
    (64, "zv:8:8", "", 0, 2),
    (64, "zv:8:64", "512:2:16", 1, 4),
    (64, "zv:8:20", "512:2:16", 0, 4),
    (64, "256:1:7", "zv:8:10", 1, 2),
    (128, "zv:8:12", "zv:8:12", 0, 2),
    (128, "zv:8:6", "512:4:8", 1, 2),
])
def test_zv_matches_oracle(maze, monkeypatch, N, basis, update, precision, order):
    force_shapes(monkeypatch, basis, update)
    box = 0.4 * N
    pos, Q, vel = random_system(2 * N, box, seed=11 * N + precision + order)
    print(f"case: zv N={N} basis {basis} update {update} precision {precision} "
          f"order {order}", flush=True)
    tol = 1e-13 if precision == 0 else 1e-9
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=tol, precision=precision, order=order,
                     flags=SSTEP)
    assert g.N == N
    lay = maze.maze_sstep_layout(g.handle)
    assert (lay["basis"], lay["update"]) == (zv_waves(basis), 0)
    if zv_waves(basis):
        bs = maze.maze_basis_shape(g.handle)
        assert (bs["threads"], bs["ppt"], bs["cx"]) == (64 * zv_waves(basis), N // 64,
                                                        int(basis.split(":")[2]))
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-13, order=order)
    if precision == 0:
        assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    for k in range(2):
        p = pos + (k + 1) * vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == 0
        bound = FIELD_TOL if precision == 0 else \
            kappa(N) * out["stats"]["rel_residual"] * 1.01 + 1e-12
        assert rel(out["field"], ref["field"]) <= bound
        if precision == 0:
            assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
            assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 3
    g.close()
    o.close()


@pytest.mark.parametrize("max_iter", [13, 1])
def test_zv_fixed_iteration_count(maze, monkeypatch, max_iter):
    """An unreachable tolerance: exactly max_iter iterations, and the oracle's
    iterate after as many (an odd cap ends after the first of a pair)."""
    force_shapes(monkeypatch, "zv:8:10", "256:1:9")
    N = 64
    box = 0.4 * N
    pos, Q, vel = random_system(150, box, seed=5)
    print(f"case: zv lockstep max_iter {max_iter}", flush=True)
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=1e-300, max_iter=max_iter, flags=SSTEP)
    assert maze.maze_sstep_layout(g.handle) == {"basis": 8, "update": 0}
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-300, max_iter=max_iter)
    assert g.init_status == maze.MAZE_NOT_CONVERGED
    assert g.init_stats["iters"] == max_iter
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= 1e-11
    for k in range(2):
        p = pos + (k + 1) * vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == maze.MAZE_NOT_CONVERGED
        assert out["stats"]["iters"] == max_iter
        assert rel(g.grid(maze.GRID_Y), o.state()["y"]) <= 1e-11
        assert rel(out["field"], ref["field"]) <= 1e-11
    g.close()
    o.close()


@pytest.mark.parametrize("precision,shape", [(0, "zv:8:24"), (1, "zv:8:24"), (1, "zv:16:20")])
def test_zv_full_size_256(maze, monkeypatch, precision, shape):
    """32768 ions on 256^3, the basis kernel in the wavefront-row layout
    against the segment layout (the same update shape): the same iterates up
    to the rounding order of the Gram sums, and the field meets the discrete
    Poisson residual the oracle computes from it."""
    s = inputs.molten_nacl(16, seed=3)
    tol = 1e-9 if precision == 0 else 1e-8
    kw = dict(tol=tol, precision=precision, coulomb_k=inputs.COULOMB_K_EV_A, flags=SSTEP)
    print(f"case: zv nacl32768 256^3 precision {precision} {shape}", flush=True)
    force_shapes(monkeypatch, shape, "512:4:32")
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    assert maze.maze_sstep_layout(g.handle) == {"basis": zv_waves(shape), "update": 0}
    # a segment-layout basis shape valid for the precision (the tuner may
    # pick either layout)
    force_shapes(monkeypatch, "512:2:64" if precision == 0 else "512:4:16", "512:4:32")
    h = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    assert maze.maze_sstep_layout(h.handle) == {"basis": 0, "update": 0}
    p = s.pos + s.vel
    a, b = g.step(dev(p), want_field=True), h.step(dev(p), want_field=True)
    print(f"  iterations: wavefront rows {a['stats']['iters']}, segments {b['stats']['iters']}",
          flush=True)
    assert a["status"] == 0 and b["status"] == 0
    assert abs(a["stats"]["iters"] - b["stats"]["iters"]) <= 2
    assert rel(a["field"], b["field"].cpu().numpy()) <= 1e-6
    N = g.N
    h_ = s.box / N
    phi = a["field"].cpu().numpy()
    q = oracle.spread(p, s.charges, s.box, N)
    res = oracle.apply_M(phi) + 4 * np.pi * q / h_
    r_rel = np.linalg.norm(res) / np.linalg.norm(4 * np.pi * q / h_)
    assert r_rel <= tol * 1.001, r_rel
    g.close()
    h.close()


# (n_cells, N, precision, tol, basis, update)
BATCH = [(4, 64, 0, 1e-10, "zv:8:8", ""), (4, 64, 1, 1e-8, "zv:8:16", "512:2:16"),
         (8, 128, 0, 1e-9, "zv:8:12", ""), (3, 48, 1, 1e-8, "", ""),
         (16, 256, 1, 1e-8, "zv:16:20", "512:4:32")]


def _sessions(maze, monkeypatch, seed):
    systems, alone, batch = [], [], []
    for i, (nc, N, prec, tol, basis, update) in enumerate(BATCH):
        force_shapes(monkeypatch, basis, update)
        s = inputs.molten_nacl(nc, seed=seed + i)
        s.grid_spacing = s.box / N
        kw = dict(tol=tol, precision=prec, coulomb_k=inputs.COULOMB_K_EV_A, flags=SSTEP)
        systems.append(s)
        alone.append(maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw))
        batch.append(maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw))
        assert maze.maze_sstep_layout(batch[-1].handle)["basis"] == zv_waves(basis)
    force_shapes(monkeypatch, "", "")
    return systems, alone, batch


def test_zv_batch_bitwise_alone(maze, monkeypatch):
    monkeypatch.setenv("MAZE_BATCH_MODE", "latency")
    print("case: zv batch", BATCH, flush=True)
    systems, alone, batch = _sessions(maze, monkeypatch, 700)
    for k in range(2):
        pos = [dev(s.pos + (k + 1) * s.vel) for s in systems]
        ref = [a.step(p, want_field=True) for a, p in zip(alone, pos)]
        forces = [torch.empty(s.n_ions, 3, dtype=torch.float64, device="cuda") for s in systems]
        rc, st = maze.maze_step_batch([b.handle for b in batch], pos, forces)
        assert rc == maze.MAZE_OK
        for i, (r, b) in enumerate(zip(ref, batch)):
            assert st[i]["iters"] == r["stats"]["iters"], i
            assert torch.equal(forces[i], r["forces"]), i
            assert torch.equal(b.grid(maze.GRID_PHI), r["field"]), i
    for x in alone + batch:
        x.close()


def test_zv_continuous_batch_bitwise_alone(maze, monkeypatch):
    monkeypatch.setenv("MAZE_BATCH_MODE", "latency")
    print("case: zv continuous batch", BATCH, flush=True)
    systems, alone, mix = _sessions(maze, monkeypatch, 800)
    n = len(BATCH)
    ref = []
    for i in range(n):
        out = alone[i].step(dev(systems[i].pos + systems[i].vel), want_field=True)
        ref.append((out["forces"].clone(), out["field"].clone(), out["stats"]["iters"]))
    batch = maze.Batch(max_sessions=8)
    bufs = {}
    for i in range(n):
        p = dev(systems[i].pos + systems[i].vel)
        F = torch.empty(systems[i].n_ions, 3, dtype=torch.float64, device="cuda")
        E = torch.empty(1, dtype=torch.float64, device="cuda")
        bufs[i] = (p, F, E)
        batch.add(mix[i].handle, p, F, E, tag=i)
        batch.advance()
    got = {}
    rounds = 0
    while len(got) < n:
        rounds += 1
        assert rounds < 100000
        batch.advance()
        for tag, st in batch.take():
            assert st["status"] == maze.MAZE_OK, (tag, st)
            torch.cuda.synchronize()
            got[tag] = (bufs[tag][1], mix[tag].grid(maze.GRID_PHI).clone(), st["iters"])
    for i in range(n):
        assert torch.equal(got[i][0], ref[i][0]), i
        assert torch.equal(got[i][1], ref[i][1]), i
        assert got[i][2] == ref[i][2], i
    batch.close()
    for x in alone + mix:
        x.close()
