"""Launch shapes of the fused CG sweep through the C ABI.

A launch shape (points per thread, x planes per workgroup) sets how the grid
is cut into workgroups: segment length, run length, halo width and the order
of the per-workgroup partial sums. It must never change the arithmetic, so
every shape, forced or picked by the autotuner, has to meet the FP64 parity
bar against the oracle, including shapes whose runs do not divide N and
segments longer than a plane.
"""
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
    a = a.cpu().numpy()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def system(n_cells, N, seed):
    s = inputs.molten_nacl(n_cells, seed=seed)
    s.grid_spacing = s.box / N
    return s


def check_shape(sh, N):
    """Segment, run and workgroup count consistent with the grid."""
    P = N * N
    nseg = -(-P // sh["segment"])
    cx = min(sh["cx"], N)
    assert sh["segment"] == 256 * sh["ppt"]
    assert sh["nwg"] == nseg * (-(-N // cx))


# (n_cells, N, forced "ppt:cx"): runs that do not divide N, a run longer
# than N (clamped), segments longer than the whole plane (N = 20: 1024 > 400)
SHAPES = [(2, 20, "4:3"), (2, 20, "1:64"), (3, 36, "2:5"), (3, 36, "4:16"),
          (3, 48, "1:4"), (3, 48, "2:7"), (4, 64, "4:64")]


@pytest.mark.parametrize("n_cells,N,shape", SHAPES)
def test_forced_shape_matches_oracle(maze, monkeypatch, n_cells, N, shape):
    print(f"case: N {N} forced shape {shape}", flush=True)
    s = system(n_cells, N, seed=40 + N)
    monkeypatch.setenv("MAZE_SWEEP_SHAPE", shape)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-13,
                     coulomb_k=inputs.COULOMB_K_EV_A)
    monkeypatch.delenv("MAZE_SWEEP_SHAPE")
    sh = maze.maze_launch_shape(g.handle)
    ppt, cx = (int(v) for v in shape.split(":"))
    for k in ("latency", "throughput"):
        assert (sh[k]["ppt"], sh[k]["cx"]) == (ppt, min(cx, N)), sh
        check_shape(sh[k], N)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    for k in range(2):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == 0
        assert rel(out["field"], ref["field"]) <= FIELD_TOL
        assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    g.close()


@pytest.mark.parametrize("N,prec", [(32, 0), (32, 1), (48, 0), (96, 1)])
def test_tuned_shapes_are_valid_and_cached(maze, N, prec):
    """The tuned shape is a valid candidate, the throughput shape has runs of
    at most 16 planes, and a second session of the same size and precision
    reuses the cached choice."""
    s = system(N // 16, N, seed=7)
    a = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-8,
                     precision=prec, coulomb_k=inputs.COULOMB_K_EV_A)
    b = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-8,
                     precision=prec, coulomb_k=inputs.COULOMB_K_EV_A)
    sa = maze.maze_launch_shape(a.handle)
    sb = maze.maze_launch_shape(b.handle)
    print(f"case: N {N} precision {prec} shapes {sa}", flush=True)
    assert sa == sb
    for k in ("latency", "throughput"):
        assert sa[k]["ppt"] in (1, 2, 4)
        check_shape(sa[k], N)
    assert sa["throughput"]["cx"] <= 16
    # sessions with one shape step bitwise alike
    p = dev(s.pos + s.vel)
    ra = a.step(p, want_field=True)
    rb = b.step(p, want_field=True)
    assert torch.equal(ra["field"], rb["field"])
    assert torch.equal(ra["forces"], rb["forces"])
    a.close()
    b.close()


def test_forced_shape_beyond_partials_is_refused(maze, monkeypatch):
    """A forced shape with more workgroups than the session's partials
    buffer has rows (1:1 at 128^3: 8192 workgroups against at most 4096
    rows there) is not taken; the session falls back to its tuned shape, so
    it steps bitwise like a session created without the forced shape."""
    s = system(8, 128, seed=9)
    ref = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-10,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    monkeypatch.setenv("MAZE_SWEEP_SHAPE", "1:1")
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-10,
                     coulomb_k=inputs.COULOMB_K_EV_A)
    monkeypatch.delenv("MAZE_SWEEP_SHAPE")
    sh = maze.maze_launch_shape(g.handle)
    print(f"case: oversized forced shape at 128^3 -> {sh}", flush=True)
    assert (sh["latency"]["ppt"], sh["latency"]["cx"]) != (1, 1)
    assert (sh["throughput"]["ppt"], sh["throughput"]["cx"]) != (1, 1)
    assert sh == maze.maze_launch_shape(ref.handle)
    p = dev(s.pos + s.vel)
    out, want = g.step(p, want_field=True), ref.step(p, want_field=True)
    assert out["status"] == 0
    assert torch.equal(out["field"], want["field"])
    g.close()
    ref.close()
