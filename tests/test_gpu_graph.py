"""CG iterations replayed from captured HIP graphs (MAZE_FLAG_GRAPH_CHUNKS).

The graphs hold the same sweep kernels with the same arguments as the
direct launches, so MD runs with and without the flag must agree bit for
bit over many replays (each step replays the chunk graphs several times),
with unrelated eager work on the same stream in between, in both
precisions. A session asking for graphs on the null stream is refused.
Batched solves whose sessions all ask for graphs replay their poll groups
from graphs captured per launch structure, on the same bar.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze
    maze.lib()
    return maze


@pytest.mark.parametrize("n_cells,precision,tol", [(2, 0, 1e-11), (4, 1, 1e-9), (3, 0, 1e-10)])
def test_graph_chunks_bitwise_equal(gpu, n_cells, precision, tol):
    from paper_2505_20418_amd.md import MDRun
    maze = gpu
    st = torch.cuda.Stream()
    print(f"case: graph chunks n_cells {n_cells} precision {precision}", flush=True)
    with torch.cuda.stream(st):
        s = inputs.molten_nacl(n_cells, seed=20 + n_cells)
        a = MDRun(s, tol=tol, precision=precision, stream=st.cuda_stream)
        b = MDRun(s, tol=tol, precision=precision, stream=st.cuda_stream,
                  flags=maze.MAZE_FLAG_GRAPH_CHUNKS)
        junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
        for k in range(12):
            ra = a.step(want_stats=True)[1]
            rb = b.step(want_stats=True)[1]
            assert ra["iters"] == rb["iters"] and ra["iters"] > 16
            junk.add_(1.0)                      # eager work between replays
            junk.sum()
        st.synchronize()
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)
        assert torch.equal(a.f_es, b.f_es) and torch.equal(a.scalars, b.scalars)
        assert torch.equal(a.session.grid(maze.GRID_Y), b.session.grid(maze.GRID_Y))
        assert float(junk[0]) == 12.0
        a.close()
        b.close()


def test_graph_chunks_need_a_stream(gpu):
    maze = gpu
    s = inputs.molten_nacl(2, seed=1)
    q = torch.tensor(s.charges, dtype=torch.float64, device="cuda")
    p = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    with pytest.raises(maze.MazeError) as e:
        maze.Session(q, p, s.box, s.grid_spacing, flags=maze.MAZE_FLAG_GRAPH_CHUNKS,
                     stream=0)
    assert e.value.status == maze.MAZE_E_INVALID


def test_graph_chunks_follow_the_solution_vector(gpu):
    """Direct Poisson solves (their own solution buffer) interleaved with
    MaZe steps (y): each replay must update the vector of its solve."""
    maze = gpu
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = inputs.molten_nacl(3, seed=31)
        q = torch.tensor(s.charges, dtype=torch.float64, device="cuda")
        p0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
        kw = dict(tol=1e-10, coulomb_k=inputs.COULOMB_K_EV_A, stream=st.cuda_stream)
        a = maze.Session(q, p0, s.box, s.grid_spacing, **kw)
        b = maze.Session(q, p0, s.box, s.grid_spacing, flags=maze.MAZE_FLAG_GRAPH_CHUNKS, **kw)
        for k in range(6):
            p = torch.tensor(s.pos + (k + 1) * s.vel, dtype=torch.float64, device="cuda")
            guess = (maze.MAZE_GUESS_STATIC, maze.MAZE_GUESS_TIMEPROP, maze.MAZE_GUESS_ZERO)[k % 3]
            sa, sb = a.solve(p, guess=guess), b.solve(p, guess=guess)
            assert torch.equal(sa["field"], sb["field"]), k
            ra, rb = a.step(p, want_field=True), b.step(p, want_field=True)
            assert ra["stats"]["iters"] == rb["stats"]["iters"], k
            assert torch.equal(ra["field"], rb["field"]), k
            assert torch.equal(ra["forces"], rb["forces"]), k
        a.close()
        b.close()


# seven sessions of uneven size, both precisions: (n_cells, grid N, precision, tolerance)
BATCH_GRAPH_CASES = [(2, 32, 0, 1e-10), (3, 48, 1, 1e-8), (4, 64, 0, 1e-9), (2, 20, 1, 1e-7),
                     (5, 76, 1, 1e-8), (3, 36, 0, 1e-11), (4, 64, 1, 1e-8)]


@pytest.mark.parametrize("sstep,mode", [(True, "latency"), (False, "latency"),
                                        (True, "throughput")])
def test_batch_graph_groups_bitwise(gpu, monkeypatch, sstep, mode):
    """Batched poll groups replayed from captured graphs (every session with
    MAZE_FLAG_GRAPH_CHUNKS) give bitwise the results of direct launches, over
    several calls with other work on the stream between them."""
    maze = gpu
    monkeypatch.setenv("MAZE_BATCH_MODE", mode)
    st = torch.cuda.Stream()
    base = maze.MAZE_FLAG_SSTEP if sstep else 0
    print(f"case: batch graph groups sstep={sstep} mode={mode}", flush=True)
    with torch.cuda.stream(st):
        systems, direct, graph = [], [], []
        for i, (n_cells, N, prec, tol) in enumerate(BATCH_GRAPH_CASES):
            s = inputs.molten_nacl(n_cells, seed=900 + i)
            s.grid_spacing = s.box / N
            Q = torch.tensor(s.charges, dtype=torch.float64, device="cuda")
            P = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
            kw = dict(tol=tol, precision=prec, coulomb_k=inputs.COULOMB_K_EV_A,
                      stream=st.cuda_stream)
            systems.append(s)
            direct.append(maze.Session(Q, P, s.box, s.grid_spacing, flags=base, **kw))
            graph.append(maze.Session(Q, P, s.box, s.grid_spacing,
                                      flags=base | maze.MAZE_FLAG_GRAPH_CHUNKS, **kw))
        junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
        for k in range(4):
            pos = [torch.tensor(np.ascontiguousarray(s.pos + (k + 1) * s.vel),
                                dtype=torch.float64, device="cuda") for s in systems]
            outs = []
            for sess in (direct, graph):
                F = [torch.empty(s.n_ions, 3, dtype=torch.float64, device="cuda")
                     for s in systems]
                E = torch.empty(len(systems), dtype=torch.float64, device="cuda")
                rc, stats = maze.maze_step_batch([x.handle for x in sess], pos, F, E)
                assert rc == maze.MAZE_OK
                outs.append((F, E, stats))
                junk.add_(1.0)
                junk.sum()
            (Fa, Ea, sa), (Fb, Eb, sb) = outs
            st.synchronize()
            assert torch.equal(Ea, Eb), k
            for i in range(len(systems)):
                assert sa[i]["iters"] == sb[i]["iters"] and sa[i]["iters"] > 8, (k, i)
                assert torch.equal(Fa[i], Fb[i]), (k, i)
                assert torch.equal(direct[i].grid(maze.GRID_PHI), graph[i].grid(maze.GRID_PHI))
        assert float(junk[0]) == 8.0
        for x in direct + graph:
            x.close()
