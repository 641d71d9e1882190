"""The streaming copy the benchmark's ceiling is measured with
(maze_stream_copy): bytes arrive intact for sizes that leave ragged last
chunks, and bad arguments are refused."""
import ctypes

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def maze():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze as m
    m.lib()
    return m


@pytest.mark.parametrize("nbytes", [16, 16 * 16385, (64 << 20) + 48, (1 << 30) + 16 * 777])
def test_stream_copy_moves_every_byte(maze, nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes % 1000)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    maze.maze_stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_stream_copy_refuses_bad_arguments(maze):
    L = maze.lib()
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    vp = ctypes.c_void_p
    assert L.maze_stream_copy(vp(a.data_ptr()), vp(b.data_ptr()), 40, None) == maze.MAZE_E_INVALID
    assert L.maze_stream_copy(vp(a.data_ptr() + 8), vp(b.data_ptr()), 32, None) == \
        maze.MAZE_E_INVALID
    assert L.maze_stream_copy(None, vp(b.data_ptr()), 32, None) == maze.MAZE_E_INVALID
    assert L.maze_stream_copy(vp(a.data_ptr()), vp(b.data_ptr()), 0, None) == maze.MAZE_OK
