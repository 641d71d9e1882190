"""The two-iteration (s = 2) form of the PLCG (MAZE_FLAG_SSTEP) through the
C ABI, against the FP64 oracle's Hestenes-Stiefel PLCG.

Its iterates equal the PLCG's in exact arithmetic, so the bar is the one of
the single-iteration sweep: FP64 field within 1e-10 relative L2 and forces
within 1e-8 of the oracle at convergence, iteration counts within the
two-iteration granularity of the oracle's, and, at a fixed iteration count,
the oracle's iterate within a bound set by the different rounding order.
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


@pytest.fixture(scope="module")
def maze():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze as m
    m.lib()
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


@pytest.mark.parametrize("order", [2, 4])
def test_sstep_steps_match_oracle(maze, order):
    s = inputs.molten_nacl(2, seed=1)
    print(f"case: sstep nacl64 32^3 order {order}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-13, order=order,
                     coulomb_k=inputs.COULOMB_K_EV_A, flags=maze.MAZE_FLAG_SSTEP)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13, order=order,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    assert abs(g.init_stats["iters"] - o.init_stats["iters"]) <= 3
    for k in range(3):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == 0
        assert rel(out["field"], ref["field"]) <= FIELD_TOL
        assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
        assert abs(out["energy"].item() - ref["energy"]) <= 1e-10 * abs(ref["energy"])
        assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 3
        assert out["stats"]["rel_residual"] <= 1e-13 * 1.05
    g.close()


@pytest.mark.parametrize("max_iter", [12, 13, 1])
def test_sstep_fixed_iteration_count(maze, max_iter):
    """Unreachable tolerance: exactly max_iter iterations (an odd cap ends
    after the first of a pair), and the oracle's iterate after as many."""
    s = inputs.molten_nacl(2, seed=1)
    print(f"case: sstep lockstep max_iter {max_iter}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-300,
                     max_iter=max_iter, flags=maze.MAZE_FLAG_SSTEP)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-300, max_iter=max_iter)
    assert g.init_status == maze.MAZE_NOT_CONVERGED
    assert g.init_stats["iters"] == max_iter
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= 1e-11
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == maze.MAZE_NOT_CONVERGED
        assert out["stats"]["iters"] == max_iter
        assert rel(g.grid(maze.GRID_Y), o.state()["y"]) <= 1e-11
        assert rel(out["field"], ref["field"]) <= 1e-11
        assert abs(out["stats"]["rel_residual"] - ref["stats"]["rel_residual"]) <= \
            1e-8 * ref["stats"]["rel_residual"]
    g.close()


@pytest.mark.parametrize("N,n_pairs,order", [(4, 3, 2), (4, 2, 4), (20, 17, 2), (36, 40, 4),
                                            (50, 60, 2), (100, 150, 2)])
def test_sstep_ragged_grids(maze, N, n_pairs, order):
    box = 0.4 * N
    pos, Q, vel = random_system(n_pairs, box, seed=N)
    print(f"case: sstep ragged N={N} ions={2 * n_pairs} order={order}", flush=True)
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=1e-13, order=order,
                     flags=maze.MAZE_FLAG_SSTEP)
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-13, order=order)
    assert g.N == N == o.N
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    p = pos + vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    g.close()


@pytest.mark.parametrize("guess", [0, 1, 2])
def test_sstep_direct_solve_guesses(maze, guess):
    s = inputs.molten_nacl(2, seed=1)
    print(f"case: sstep direct solve guess {guess}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12,
                     flags=maze.MAZE_FLAG_SSTEP)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12)
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        g.step(dev(p))
        o.step(p)
    p = s.pos + 3 * s.vel
    out = g.solve(dev(p), guess=guess)
    ref = o.solve(p, guess=guess)
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 3
    g.close()


def test_sstep_absmax_residual_norm(maze):
    """The max-norm test runs every two iterations: never more than one
    iteration past the single-iteration solve."""
    s = inputs.molten_nacl(2, seed=1)
    print("case: sstep absmax", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-9,
                     residual_norm=maze.MAZE_NORM_ABSMAX, flags=maze.MAZE_FLAG_SSTEP)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-9,
                       residual_norm=oracle.NORM_ABSMAX)
    p = s.pos + s.vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert out["status"] == 0
    assert out["stats"]["max_abs_residual"] <= 1e-9
    assert abs(out["stats"]["iters"] - ref["stats"]["iters"]) <= 3
    g.close()


def test_sstep_mixed_precision(maze):
    """FP32 two-iteration inner solves with the FP64 refinement reach the FP64
    target; the field error is within kappa times the relative residual."""
    s = inputs.molten_nacl(2, seed=1)
    tol = 1e-8
    print("case: sstep mixed 32^3", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                     precision=maze.MAZE_MIXED, coulomb_k=inputs.COULOMB_K_EV_A,
                     flags=maze.MAZE_FLAG_SSTEP)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    for k in range(4):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        st = out["stats"]
        print(f"sstep mixed step {k + 1}: iters {st['iters']} refinements {st['refinements']} "
              f"res {st['rel_residual']:.2e}", flush=True)
        assert out["status"] == 0 and st["rel_residual"] <= tol
        assert rel(out["field"], ref["field"]) <= kappa(g.N) * st["rel_residual"] * 1.01 + 1e-12
        assert rel(out["forces"], ref["forces"]) <= 1e-4
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_sstep_full_size_256(maze, precision):
    """32768 ions on 256^3: the field satisfies the discrete Poisson residual
    the oracle computes from it, forces and energy follow from that field,
    and the iteration count stays within a few percent of the
    single-iteration sweep's on the same step."""
    s = inputs.molten_nacl(16, seed=3)
    tol = 1e-9 if precision == 0 else 1e-8
    print(f"case: sstep nacl32768 256^3 precision {precision}", flush=True)
    kw = dict(tol=tol, precision=precision, coulomb_k=inputs.COULOMB_K_EV_A)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing,
                     flags=maze.MAZE_FLAG_SSTEP, **kw)
    p = s.pos + s.vel
    out = g.step(dev(p), want_field=True)
    N = g.N
    h = s.box / N
    phi = out["field"].cpu().numpy()
    q = oracle.spread(p, s.charges, s.box, N)
    res = oracle.apply_M(phi) + 4 * np.pi * q / h
    r_rel = np.linalg.norm(res) / np.linalg.norm(4 * np.pi * q / h)
    assert r_rel <= tol * 1.001, r_rel
    F_ref = oracle.gather(p, s.charges, s.box, phi, coulomb_k=inputs.COULOMB_K_EV_A)
    assert rel(out["forces"], F_ref) <= 1e-13
    e_ref = oracle.energy(phi, q, inputs.COULOMB_K_EV_A)
    assert abs(out["energy"].item() - e_ref) <= 1e-11 * abs(e_ref)
    g.close()
    one = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    ref = one.step(dev(p))
    a, b = out["stats"]["iters"], ref["stats"]["iters"]
    print(f"iterations: two-iteration form {a}, single-iteration sweep {b}", flush=True)
    assert abs(a - b) <= max(4, 0.05 * b)
    one.close()


def test_sstep_graph_chunks_bitwise(maze):
    """Captured chunks of outer steps give bitwise the results of direct
    launches, over many replays with other work between them."""
    from paper_2505_20418_amd.md import MDRun
    st = torch.cuda.Stream()
    print("case: sstep graph chunks", flush=True)
    with torch.cuda.stream(st):
        s = inputs.molten_nacl(3, seed=23)
        fl = maze.MAZE_FLAG_SSTEP
        a = MDRun(s, tol=1e-10, precision=1, stream=st.cuda_stream, flags=fl)
        b = MDRun(s, tol=1e-10, precision=1, stream=st.cuda_stream,
                  flags=fl | maze.MAZE_FLAG_GRAPH_CHUNKS)
        junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
        for k in range(8):
            ra = a.step(want_stats=True)[1]
            rb = b.step(want_stats=True)[1]
            assert ra["iters"] == rb["iters"] and ra["iters"] > 16
            junk.add_(1.0)
            junk.sum()
        st.synchronize()
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)
        assert torch.equal(a.f_es, b.f_es)
        assert float(junk[0]) == 8.0
        a.close()
        b.close()


BATCH_CASES = [(2, 32, 0, 1e-10), (3, 48, 1, 1e-8), (4, 64, 0, 1e-9), (2, 20, 1, 1e-7),
               (5, 76, 1, 1e-8), (3, 36, 0, 1e-11), (4, 64, 1, 1e-8)]


def _batch_sessions(maze, seed0):
    systems, alone, batch = [], [], []
    for i, (n_cells, N, prec, tol) in enumerate(BATCH_CASES):
        s = inputs.molten_nacl(n_cells, seed=seed0 + i)
        s.grid_spacing = s.box / N
        kw = dict(tol=tol, precision=prec, coulomb_k=inputs.COULOMB_K_EV_A,
                  flags=maze.MAZE_FLAG_SSTEP)
        systems.append(s)
        alone.append(maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw))
        batch.append(maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw))
    return systems, alone, batch


def test_sstep_batch_is_bitwise_alone(maze):
    """Batches of two-iteration sessions (uneven grids, both precisions,
    basis kernels of 256 and 1024 threads) run batched kernels; below the
    fill level each session ends bitwise where the same step alone leaves
    it."""
    print("case: sstep batch", BATCH_CASES, flush=True)
    systems, alone, batch = _batch_sessions(maze, 40)
    assert sum(maze.maze_launch_shape(b.handle)["throughput"]["nwg"] for b in batch) < 256
    print("basis shapes", [maze.maze_basis_shape(b.handle)["threads"] for b in batch], flush=True)
    for k in range(3):
        pos = [dev(s.pos + (k + 1) * s.vel) for s in systems]
        ref = [a.step(p, want_field=True) for a, p in zip(alone, pos)]
        forces = [torch.empty(s.n_ions, 3, dtype=torch.float64, device="cuda") for s in systems]
        rc, st = maze.maze_step_batch([b.handle for b in batch], pos, forces)
        assert rc == maze.MAZE_OK
        for i, (r, b) in enumerate(zip(ref, batch)):
            assert st[i]["iters"] == r["stats"]["iters"], i
            assert st[i]["refinements"] == r["stats"]["refinements"], i
            assert torch.equal(forces[i], r["forces"]), i
            assert torch.equal(b.grid(maze.GRID_PHI), r["field"]), i
    for x in alone + batch:
        x.close()


def test_sstep_batch_throughput_mode(maze, monkeypatch):
    """Forced throughput mode (both kernels in the throughput shape, another
    summation order): every session meets its tolerance, and the field
    differs from the step alone by at most the two solves' residuals through
    the inverse operator, (4 pi / h) 2 tol ||q|| / lambda_min with
    lambda_min = 2 (1 - cos(2 pi / N))."""
    monkeypatch.setenv("MAZE_BATCH_MODE", "throughput")
    print("case: sstep batch throughput mode", flush=True)
    systems, alone, batch = _batch_sessions(maze, 60)
    pos = [dev(s.pos + s.vel) for s in systems]
    ref = [a.step(p, want_field=True) for a, p in zip(alone, pos)]
    rc, st = maze.maze_step_batch([b.handle for b in batch], pos)
    assert rc == maze.MAZE_OK
    for i, (r, b) in enumerate(zip(ref, batch)):
        n_cells, N, prec, tol = BATCH_CASES[i]
        assert st[i]["status"] == maze.MAZE_OK and st[i]["rel_residual"] <= tol, i
        h = systems[i].box / N
        qn = torch.linalg.norm(b.grid(maze.GRID_Q)).item()
        bound = (4 * math.pi / h) * 2 * tol * qn / (2 * (1 - math.cos(2 * math.pi / N)))
        d = torch.linalg.norm(b.grid(maze.GRID_PHI) - r["field"]).item()
        assert d <= bound, (i, d, bound)
    for x in alone + batch:
        x.close()


def test_sstep_profile_counts_outer_steps(maze):
    """Sampled outer steps are timed as a whole and by their update kernel."""
    s = inputs.molten_nacl(4, seed=9)
    print("case: sstep profile", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-9,
                     precision=maze.MAZE_MIXED, flags=maze.MAZE_FLAG_SSTEP)
    maze.maze_profile_enable(g.handle, True)
    maze.maze_trace_enable(g.handle, True)
    out = g.step(dev(s.pos + s.vel))
    pr = maze.maze_profile_read(g.handle)
    n, ms = pr["fp32_sweep"]
    assert pr["fp32_iters"] == out["stats"]["iters"]
    assert 1 <= n <= (out["stats"]["iters"] + 1) // 2
    assert 0 < pr["fp32_update_ms"] < ms
    # exactly the sampled outer steps k = 1, 17, 33, ... that did work: a
    # pass of n iterations works in outer steps 0 .. (n + 1) // 2 - 1 (a
    # refinement pass of two iterations has no sampled step that worked)
    rows = maze.maze_trace_read(g.handle)
    iters = {}
    for p, t, _ in rows:
        if t >= 0:
            iters[p] = max(iters.get(p, 0), t)
    assert len(iters) >= 1
    want = sum(len(range(1, (k + 1) // 2, 16)) for k in iters.values())
    assert n == want, (n, iters)
    g.close()


@pytest.mark.parametrize("N,shape,precision", [(100, "1024:2:8", 0), (64, "1024:4:16", 1),
                                               (36, "1024:1:8", 0), (100, "1024:1:32", 1),
                                               (64, "1024:2:64", 1), (64, "512:4:8", 1),
                                               (100, "512:2:16", 0)])
def test_sstep_basis_shapes(maze, monkeypatch, N, shape, precision):
    """Forced 1024- and 512-thread basis shapes (a segment that is a whole plane, a
    ragged last segment, one x run): the same field as the oracle."""
    monkeypatch.setenv("MAZE_BASIS_SHAPE", shape)
    box = 0.4 * N
    pos, Q, vel = random_system(3 * N, box, seed=N + precision)
    print(f"case: sstep basis shape {shape} N={N} precision {precision}", flush=True)
    tol = 1e-12 if precision == 0 else 1e-9
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=tol, precision=precision,
                     flags=maze.MAZE_FLAG_SSTEP)
    nt, ppt, cx = (int(v) for v in shape.split(":"))
    bs = maze.maze_basis_shape(g.handle)
    assert (bs["threads"], bs["ppt"], bs["cx"]) == (nt, ppt, cx)
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-13)
    p = pos + vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert out["status"] == 0
    bound = FIELD_TOL if precision == 0 else kappa(N) * out["stats"]["rel_residual"] * 1.01 + 1e-12
    assert rel(out["field"], ref["field"]) <= bound
    g.close()


@pytest.mark.parametrize("N,update,basis,precision", [(36, "1:5", "256:1:7", 0),
                                                      (40, "2:6", "1024:1:3", 0),
                                                      (33, "1:4", "256:2:11", 1)])
def test_sstep_march_directions(maze, monkeypatch, N, update, basis, precision):
    """x runs alternate between upward and downward marches. Forced shapes
    give odd and even run counts and a last run of a single plane at either
    end of that alternation (N=36: the update's last run, the 8th, and the
    basis kernel's 6th each hold one plane and march down; N=40: the basis
    kernel's 14th run holds one plane; N=33: nine update runs, the last of
    one plane marching up, and three basis runs with a ragged segment)."""
    monkeypatch.setenv("MAZE_SWEEP_SHAPE", update)
    monkeypatch.setenv("MAZE_BASIS_SHAPE", basis)
    box = 0.4 * N
    pos, Q, vel = random_system(2 * N, box, seed=3 * N + precision)
    print(f"case: sstep march directions N={N} update {update} basis {basis} "
          f"precision {precision}", flush=True)
    tol = 1e-12 if precision == 0 else 1e-9
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=tol, precision=precision,
                     flags=maze.MAZE_FLAG_SSTEP)
    ppt, cx = (int(v) for v in update.split(":"))
    ls = maze.maze_launch_shape(g.handle)["latency"]
    assert (ls["ppt"], ls["cx"]) == (ppt, cx)
    nt, bppt, bcx = (int(v) for v in basis.split(":"))
    bs = maze.maze_basis_shape(g.handle)
    assert (bs["threads"], bs["ppt"], bs["cx"]) == (nt, bppt, bcx)
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-13)
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
    g.close()


@pytest.mark.parametrize("N,update,precision", [(64, "512:4:8", 1), (64, "512:2:16", 0),
                                               (100, "512:2:16", 0), (36, "512:2:5", 1),
                                               (256, "512:4:32", 0)])
def test_sstep_update_shapes_512(maze, monkeypatch, N, update, precision):
    """Forced 512-thread update shapes (row-owning layout where N divides
    512, flat where it does not, a ragged last run, a segment of more than
    half a plane, and the full-size shape): the same field as the oracle,
    or at 256^3 a converged step that matches the 256-thread shape."""
    monkeypatch.setenv("MAZE_UPDATE_SHAPE", update)
    nt, ppt, cx = (int(v) for v in update.split(":"))
    print(f"case: sstep update shape {update} N={N} precision {precision}", flush=True)
    if N == 256:
        s = inputs.molten_nacl(16, seed=3)
        kw = dict(tol=1e-8, precision=precision, coulomb_k=inputs.COULOMB_K_EV_A,
                  flags=maze.MAZE_FLAG_SSTEP)
        g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
        ls = maze.maze_launch_shape(g.handle)["latency"]
        assert (ls["segment"] // ls["ppt"], ls["ppt"], ls["cx"]) == (nt, ppt, cx)
        monkeypatch.setenv("MAZE_UPDATE_SHAPE", "256:4:64")
        h = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
        p = dev(s.pos + s.vel)
        a, b = g.step(p, want_field=True), h.step(p, want_field=True)
        assert a["status"] == 0 and b["status"] == 0
        # the same iterates up to the rounding order of the Gram sums
        assert abs(a["stats"]["iters"] - b["stats"]["iters"]) <= 2
        assert rel(a["field"], b["field"].cpu().numpy()) <= 1e-6
        g.close()
        h.close()
        return
    box = 0.4 * N
    pos, Q, vel = random_system(2 * N, box, seed=7 * N + precision)
    tol = 1e-12 if precision == 0 else 1e-9
    g = maze.Session(dev(Q), dev(pos), box, 0.4, tol=tol, precision=precision,
                     flags=maze.MAZE_FLAG_SSTEP)
    ls = maze.maze_launch_shape(g.handle)["latency"]
    assert (ls["segment"] // ls["ppt"], ls["ppt"], ls["cx"]) == (nt, ppt, cx)
    o = oracle.Session(Q, pos, box, 0.4, tol=1e-13)
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
    g.close()


def test_sstep_tuned_shapes_are_cached(maze):
    s = inputs.molten_nacl(8, seed=4)
    print("case: sstep tuned basis shape 128^3", flush=True)
    kw = dict(tol=1e-8, precision=maze.MAZE_MIXED, flags=maze.MAZE_FLAG_SSTEP)
    a = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    b = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    sa, sb = maze.maze_basis_shape(a.handle), maze.maze_basis_shape(b.handle)
    ua = maze.maze_launch_shape(a.handle)["latency"]
    ub = maze.maze_launch_shape(b.handle)["latency"]
    print("basis shape", sa, "update shape", ua, flush=True)
    # the basis and update shapes are tuned and cached as a pair
    assert sa == sb and sa["threads"] in (256, 512, 1024) and sa["nwg"] >= 1
    assert ua == ub and ua["segment"] // ua["ppt"] in (256, 512)
    ra, rb = a.step(dev(s.pos + s.vel)), b.step(dev(s.pos + s.vel))
    assert ra["status"] == 0 and torch.equal(ra["forces"], rb["forces"])
    a.close()
    b.close()


@pytest.mark.parametrize("tol", [1e-9, 0.5])
def test_first_pass_on_device_matches_host_decided(maze, tol):
    """A mixed step sets its first FP32 pass up on the device; a session that
    records a residual trace decides it on the host. Both take the same test
    and inner tolerance, so the steps agree bit for bit. At tol 0.5 the
    right-hand side's residual already meets the threshold (no pass)."""
    s = inputs.molten_nacl(4, seed=13)
    print(f"case: first pass on device against host, nacl 512 ions tol {tol}", flush=True)
    kw = dict(tol=tol, precision=maze.MAZE_MIXED, flags=maze.MAZE_FLAG_SSTEP)
    a = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    b = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, **kw)
    maze.maze_trace_enable(b.handle, True)
    passes = []
    for k in range(3):
        p = dev(s.pos + (k + 1) * s.vel)
        x, y = a.step(p, want_field=True), b.step(p, want_field=True)
        assert x["status"] == maze.MAZE_OK and y["status"] == maze.MAZE_OK, k
        assert x["stats"]["iters"] == y["stats"]["iters"], k
        assert x["stats"]["refinements"] == y["stats"]["refinements"], k
        assert torch.equal(x["field"], y["field"]), k
        assert torch.equal(x["forces"], y["forces"]), k
        passes.append(x["stats"]["refinements"])
    print(f"  passes per step {passes}", flush=True)
    if tol == 0.5:
        assert passes == [0, 0, 0]
    else:
        assert min(passes) >= 1
    a.close()
    b.close()
