"""Multigrid-preconditioned PLCG (MAZE_FLAG_MULTIGRID) against the oracle.

The V-cycle preconditioner changes how fast the solve converges, not what
it converges to: the field, forces and energy must match the oracle's
Jacobi-PCG solution to the FP64 bar, with both the FP64 and the FP32
V-cycle (the outer CG is FP64 in both), on grids whose hierarchies end on
odd or single-level coarse grids, and the iteration count must be small.
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
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n_cells,N", [(2, 32), (3, 48), (2, 40), (1, 12), (1, 9)])
def test_multigrid_matches_oracle(maze, precision, n_cells, N):
    s = inputs.molten_nacl(n_cells, seed=40 + N)
    s.grid_spacing = s.box / N
    print(f"case: multigrid N={N} ions={s.n_ions} precision={precision}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-13,
                     precision=precision, flags=maze.MAZE_FLAG_MULTIGRID,
                     coulomb_k=inputs.COULOMB_K_EV_A)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-13,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    assert g.N == N
    assert rel(g.grid(maze.GRID_PHI), o.state()["phi_k"]) <= FIELD_TOL
    for k in range(3):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        ref = o.step(p)
        assert out["status"] == 0
        assert rel(out["field"], ref["field"]) <= FIELD_TOL
        assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
        assert abs(out["energy"].item() - ref["energy"]) <= 1e-10 * abs(ref["energy"])
        assert out["stats"]["rel_residual"] <= 1e-13 * 1.05
        assert out["stats"]["iters"] <= 40, out["stats"]
    g.close()


def test_multigrid_full_parity_128(maze):
    s = inputs.molten_nacl(8, seed=2)
    print("case: multigrid 128^3 full parity", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=1e-12,
                     flags=maze.MAZE_FLAG_MULTIGRID, coulomb_k=inputs.COULOMB_K_EV_A)
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=1e-12,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    p = s.pos + s.vel
    out = g.step(dev(p), want_field=True)
    ref = o.step(p)
    assert rel(out["field"], ref["field"]) <= FIELD_TOL
    assert rel(out["forces"], ref["forces"]) <= FORCE_TOL
    assert out["stats"]["iters"] <= 30
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_multigrid_256_iterations_and_residual(maze, precision):
    """Full size: the oracle checks the GPU field through the discrete
    Poisson residual it must satisfy and recomputes the interpolated forces
    from it; a warm step needs few outer iterations (Jacobi PLCG needs about
    240 at this size and tolerance)."""
    s = inputs.workload("nacl32768_g256")
    tol = 1e-8
    print(f"case: multigrid 256^3 precision {precision}", flush=True)
    g = maze.Session(dev(s.charges), dev(s.pos), s.box, s.grid_spacing, tol=tol,
                     precision=precision, flags=maze.MAZE_FLAG_MULTIGRID)
    for k in range(3):
        p = s.pos + (k + 1) * s.vel
        out = g.step(dev(p), want_field=True)
        assert out["status"] == 0
    assert out["stats"]["iters"] <= 15, out["stats"]
    N = g.N
    h = s.box / N
    phi = out["field"].cpu().numpy()
    q = oracle.spread(p, s.charges, s.box, N)
    res = oracle.apply_M(phi) + 4 * np.pi * q / h
    r_rel = np.linalg.norm(res) / np.linalg.norm(4 * np.pi * q / h)
    assert r_rel <= tol * 1.001, r_rel
    assert abs(out["stats"]["rel_residual"] - r_rel) <= 1e-3 * r_rel + 1e-15
    F_ref = oracle.gather(p, s.charges, s.box, phi)
    assert rel(out["forces"], F_ref) <= 1e-13
    g.close()
