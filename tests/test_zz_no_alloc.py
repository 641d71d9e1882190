"""maze_step_batch_noalloc (the batch step that allocates nothing, its batch
table a fixed device array of the library) against maze_step_batch on
identical sessions: statuses, iteration counts, forces, energies and fields
bitwise equal, over two calls in a row, the second with fewer sessions;
and the capacity limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

SSTEP = 16
# (n_cells, grid N, precision, tolerance, flags): both precisions, both CG
# forms (a batch splits into one-iteration and two-iteration sub-batches),
# uneven and ragged grids
CASES = [(2, 32, 0, 1e-10, 0), (3, 48, 1, 1e-8, SSTEP), (4, 64, 0, 1e-9, SSTEP),
         (2, 20, 1, 1e-7, 0), (3, 36, 0, 1e-11, 0)]


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


def make(maze, case, seed):
    n_cells, N, prec, tol, flags = case
    s = inputs.molten_nacl(n_cells, seed=seed)
    s.grid_spacing = s.box / N
    sess = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                        precision=prec, coulomb_k=inputs.COULOMB_K_EV_A, flags=flags)
    assert sess.N == N
    return s, sess


def test_noalloc_batch_equals_batch(maze):
    systems, ref_sess, fix_sess = [], [], []
    for i, c in enumerate(CASES):
        s, a = make(maze, c, seed=300 + i)
        _, b = make(maze, c, seed=300 + i)
        systems.append(s)
        ref_sess.append(a)
        fix_sess.append(b)
    # two calls in a row, the second with a smaller batch
    for call, members in enumerate((list(range(len(CASES))), [0, 2, 3])):
        print(f"case: no-alloc batch call {call + 1}, sessions {members}", flush=True)
        pos = [dev(systems[i].pos + (call + 1) * systems[i].vel) for i in members]
        outs = []
        for fn, sess in ((maze.maze_step_batch, ref_sess),
                         (maze.maze_step_batch_noalloc, fix_sess)):
            forces = [torch.empty(systems[i].n_ions, 3, dtype=torch.float64, device="cuda")
                      for i in members]
            energies = torch.empty(len(members), dtype=torch.float64, device="cuda")
            rc, st = fn([sess[i].handle for i in members], pos, forces, energies)
            assert rc == maze.MAZE_OK
            outs.append((st, forces, energies))
        (st_a, f_a, e_a), (st_b, f_b, e_b) = outs
        assert torch.equal(e_a, e_b)
        for q, i in enumerate(members):
            assert st_b[q]["status"] == st_a[q]["status"] == maze.MAZE_OK
            assert st_b[q]["iters"] == st_a[q]["iters"], i
            assert st_b[q]["refinements"] == st_a[q]["refinements"], i
            assert st_b[q]["rel_residual"] == st_a[q]["rel_residual"], i
            assert torch.equal(f_a[q], f_b[q]), i
            assert torch.equal(ref_sess[i].grid(maze.GRID_PHI), fix_sess[i].grid(maze.GRID_PHI))
    for x in ref_sess + fix_sess:
        x.close()


def test_noalloc_batch_capacity(maze):
    s, a = make(maze, CASES[0], seed=400)
    handles = [a.handle] * 257
    pos = [dev(s.pos)] * 257
    with pytest.raises(maze.MazeError) as e:
        maze.maze_step_batch_noalloc(handles, pos)
    assert e.value.status == maze.MAZE_E_CAPACITY
    # a valid call still works after the refused one
    rc, st = maze.maze_step_batch_noalloc([a.handle], [dev(s.pos + s.vel)])
    assert rc == maze.MAZE_OK and st[0]["status"] == maze.MAZE_OK
    a.close()
