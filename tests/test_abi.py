"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point that include/maze.h declares, and the ctypes structures
match the C layout (checked with a small program compiled by gcc)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maze.h")
LIB = os.path.join(ROOT, "paper_2505_20418_amd", "libmaze.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(maze_[a-z_0-9]+)\s*\(", src)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libmaze.so not built")


@needs_lib
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@needs_lib
def test_binding_covers_header():
    from paper_2505_20418_amd import maze
    assert set(maze.EXPORTED) == set(declared_functions())


@needs_lib
def test_host_only_entry_points():
    L = ctypes.CDLL(LIB)
    L.maze_abi_version.restype = ctypes.c_int
    assert L.maze_abi_version() == 2
    L.maze_strerror.restype = ctypes.c_char_p
    assert b"neutral" in L.maze_strerror(-2)
    L.maze_grid_n.restype = ctypes.c_int
    L.maze_grid_n.argtypes = [ctypes.c_void_p]
    assert L.maze_grid_n(None) == 0
    L.maze_destroy.argtypes = [ctypes.c_void_p]
    L.maze_destroy(None)  # no-op
    from paper_2505_20418_amd import maze
    cfg = maze.maze_config(4096, 2, 51.0, 0.3984375, 1e-9, 1000, 0, 0, 0, 1.0, None)
    L.maze_device_bytes.restype = ctypes.c_size_t
    L.maze_device_bytes.argtypes = [ctypes.POINTER(maze.maze_config)]
    nbytes = L.maze_device_bytes(ctypes.byref(cfg))
    G = 128 ** 3
    assert 9 * 8 * G <= nbytes <= 10 * 8 * G + (64 << 20)
    bad = maze.maze_config(4096, 3, 51.0, 0.3984375, 1e-9, 1000, 0, 0, 0, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(bad)) == 0
    tiny = maze.maze_config(4, 2, 1.0, 0.5, 1e-9, 10, 0, 0, 0, 1.0, None)  # N = 2 < 4
    assert L.maze_device_bytes(ctypes.byref(tiny)) == 0
    # multigrid: a grid that halves to <= 12^3 is accepted, an odd 101^3 is not;
    # an unknown flag bit is rejected
    ok = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0, 0, 1.0, None)
    mg = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0, maze.MAZE_FLAG_MULTIGRID, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(mg)) > L.maze_device_bytes(ctypes.byref(ok))
    odd = maze.maze_config(4, 2, 40.4, 0.4, 1e-9, 10, 0, 0, maze.MAZE_FLAG_MULTIGRID, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(odd)) == 0
    badflag = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0, 32, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(badflag)) == 0
    # the two-iteration CG is accepted alone, not with the multigrid preconditioner
    ss = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0, maze.MAZE_FLAG_SSTEP, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(ss)) == L.maze_device_bytes(ctypes.byref(ok))
    ssmg = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0,
                            maze.MAZE_FLAG_SSTEP | maze.MAZE_FLAG_MULTIGRID, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(ssmg)) == 0
    # graph chunks need a stream that can be captured (not the null stream)
    nostream = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0, maze.MAZE_FLAG_GRAPH_CHUNKS,
                                1.0, None)
    assert L.maze_device_bytes(ctypes.byref(nostream)) == 0
    withstream = maze.maze_config(4, 2, 25.6, 0.4, 1e-9, 10, 0, 0, maze.MAZE_FLAG_GRAPH_CHUNKS,
                                  1.0, ctypes.c_void_p(0x1000))
    assert L.maze_device_bytes(ctypes.byref(withstream)) > 0


def test_struct_layout_matches_c(tmp_path):
    from paper_2505_20418_amd import maze
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "maze.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("maze_config %zu\nmaze_stats %zu\nmaze_md_state %zu\n", sizeof(maze_config),
         sizeof(maze_stats), sizeof(maze_md_state));
  F(maze_config, tol); F(maze_config, coulomb_k); F(maze_config, stream);
  F(maze_stats, h); F(maze_stats, energy); F(maze_stats, status);
  F(maze_md_state, scalars_dev); F(maze_md_state, dt); F(maze_md_state, bmh_table);
  F(maze_md_state, gamma); F(maze_md_state, kT); F(maze_md_state, seed);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog),
                           "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().split("\n") if line)
    assert int(out["maze_config"]) == ctypes.sizeof(maze.maze_config)
    assert int(out["maze_stats"]) == ctypes.sizeof(maze.maze_stats)
    assert int(out["maze_md_state"]) == ctypes.sizeof(maze.maze_md_state)
    for key, val in out.items():
        if "." in key:
            t, m = key.split(".")
            assert getattr(getattr(maze, t), m).offset == int(val), key


@needs_lib
def test_empty_and_degenerate_inputs_on_host():
    """Cases the entry points settle before any device work: no ions is
    refused at admission; zero or one ion gives no pairs to histogram and no
    noise to draw; malformed observable arguments are refused."""
    from paper_2505_20418_amd import maze
    L = maze.lib()
    empty = maze.maze_config(0, 2, 25.6, 0.4, 1e-9, 10, 0, 0, 0, 1.0, None)
    assert L.maze_device_bytes(ctypes.byref(empty)) == 0
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced on these paths
    assert L.maze_rdf_accumulate(None, None, 0, 10.0, dummy, 10, dummy, None) == maze.MAZE_OK
    assert L.maze_rdf_accumulate(dummy, dummy, 1, 10.0, dummy, 10, dummy, None) == maze.MAZE_OK
    assert L.maze_rdf_accumulate(dummy, dummy, 5, 10.0, dummy, 0, dummy, None) == maze.MAZE_E_INVALID
    assert L.maze_rdf_accumulate(dummy, dummy, 5, 10.0, dummy, 5000, dummy, None) == maze.MAZE_E_INVALID
    assert L.maze_rdf_accumulate(dummy, dummy, 5, -1.0, dummy, 10, dummy, None) == maze.MAZE_E_INVALID
    assert L.maze_langevin_noise(1, 0, 0, 0, None, None) == maze.MAZE_OK
    assert L.maze_langevin_noise(1, 0, 2, 4, dummy, None) == maze.MAZE_E_INVALID
    assert L.maze_langevin_noise(1, -1, 0, 4, dummy, None) == maze.MAZE_E_INVALID
    h = ctypes.c_void_p()
    assert L.maze_tcf_create(0, dummy, 10, 1, None, ctypes.byref(h)) == maze.MAZE_E_INVALID
    assert L.maze_tcf_create(4, dummy, 10, 0, None, ctypes.byref(h)) == maze.MAZE_E_INVALID
    assert not h.value
    assert L.maze_tcf_sample(None, dummy, dummy) == maze.MAZE_E_INVALID
    L.maze_tcf_destroy(None)
