"""The oracle's OpenMP timing build (its order-independent loops threaded,
every reduction sequential) returns bitwise the plain build's results, so
the CPU baseline timed with it times the same computation."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, %r)
import oracle
from paper_2505_20418_amd import inputs
omp = sys.argv[1] == "1"
out = {}
for n_cells, N, order in ((2, 32, 2), (2, 36, 4)):
    s = inputs.molten_nacl(n_cells, seed=11)
    h = s.box / N
    o = oracle.Session(s.charges, s.pos, s.box, h, tol=1e-11, order=order,
                       coulomb_k=inputs.COULOMB_K_EV_A, omp=omp)
    for k in range(3):
        r = o.step(s.pos + (k + 1) * s.vel)
        out[f"{N}_{k}_field"] = r["field"]
        out[f"{N}_{k}_forces"] = r["forces"]
        out[f"{N}_{k}_energy"] = np.array([r["energy"], r["stats"]["iters"],
                                            r["stats"]["rel_residual"]])
    r = o.solve(s.pos + 4 * s.vel, guess=oracle.GUESS_TIMEPROP)
    out[f"{N}_solve"] = r["field"]
    pos, vel = s.pos.copy(), s.vel.copy()
    F_es = o.step(pos)["forces"]
    F_sr, _ = oracle.bmh(pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    work = np.zeros(1)
    for _ in range(2):
        o.md_step(pos, vel, s.masses, s.species, inputs.BMH_TABLE, inputs.BMH_CUTOFF, 1.0,
                  inputs.ACCEL_FACTOR, F_es, F_sr, work)
    out[f"{N}_md"] = np.concatenate([pos.ravel(), vel.ravel(), work])
    o.close()
np.savez(sys.argv[2], **out)
""" % ROOT


def _run(tmp_path, omp, threads):
    import oracle
    oracle.build(force=False)
    script = tmp_path / "run.py"
    script.write_text(_SCRIPT)
    out = tmp_path / f"out_{omp}_{threads}.npz"
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    subprocess.check_call([sys.executable, str(script), "1" if omp else "0", str(out)], env=env)
    return np.load(out)


def test_openmp_build_is_bitwise_the_plain_build(tmp_path):
    plain = _run(tmp_path, False, 1)
    for threads in (1, 4):
        par = _run(tmp_path, True, threads)
        assert set(par.files) == set(plain.files)
        for k in plain.files:
            assert np.array_equal(par[k], plain[k]), (threads, k)
