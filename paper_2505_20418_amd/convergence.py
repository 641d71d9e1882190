"""Convergence study: MaZe against direct Poisson solves (Appendix B).

Appendix B compares the Jacobi PLCG solve of the MaZe constraint system
(equation "SHAKEy", warm-started from the previous step's y*) with PLCG
solves of the Poisson equation itself (equation "linearproblem") started
from the previous potential ("static") or from its Verlet extrapolation
2 phi^k - phi^{k-1} ("time-propagated"), as in the convergence subsection of
the Results section. Every solve here goes through the library (maze_step,
maze_solve) on the same relative residual scale, ||M phi + 4 pi q / h|| /
||4 pi q / h|| = ||sigma_p - M y|| / ||q||, with per-iteration residual
histories from the library's trace.

The configurations replay a trajectory through a session: at each step the
static and time-propagated solves see the same history as the MaZe step,
and maze_solve leaves that history untouched.
"""
from __future__ import annotations

import argparse
import json
import math
from typing import Dict, List, Sequence

import numpy as np
import torch

from . import inputs, maze


def ballistic_trajectory(system: inputs.NaClSystem, n_steps: int, dt: float = 1.0):
    """Positions r_k = r_0 + k dt v (ions moving freely): the sequence of
    configurations a step-to-step warm start sees, without the force field."""
    return [system.pos + (k + 1) * dt * system.vel for k in range(n_steps)]


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def replay_compare(charges: np.ndarray, traj: Sequence[np.ndarray], box: float,
                   grid_spacing: float, tol: float, precision: int = maze.MAZE_FP64,
                   trace_steps: Sequence[int] = (), order: int = 2) -> Dict:
    """Replays positions through one session; per step, the static and
    time-propagated Poisson solves and then the MaZe step. Returns per-step
    iteration counts, final relative residuals, the largest difference of
    the three fields relative to the MaZe field, and residual histories for
    the steps in trace_steps."""
    sess = maze.Session(_dev(charges), _dev(traj[0]), box, grid_spacing, tol=tol,
                        precision=precision, order=order)
    h = sess.handle
    maze.maze_trace_enable(h, True)
    out = {"static": [], "timeprop": [], "maze": [], "res_static": [], "res_timeprop": [],
           "res_maze": [], "field_diff": [], "traces": {}}
    for k, p in enumerate(traj):
        pd = _dev(p)
        rs = sess.solve(pd, guess=maze.MAZE_GUESS_STATIC)
        ts = maze.maze_trace_read(h)
        rt = sess.solve(pd, guess=maze.MAZE_GUESS_TIMEPROP)
        tt = maze.maze_trace_read(h)
        rm = sess.step(pd, want_field=True)
        tm = maze.maze_trace_read(h)
        out["static"].append(rs["stats"]["iters"])
        out["timeprop"].append(rt["stats"]["iters"])
        out["maze"].append(rm["stats"]["iters"])
        out["res_static"].append(rs["stats"]["rel_residual"])
        out["res_timeprop"].append(rt["stats"]["rel_residual"])
        out["res_maze"].append(rm["stats"]["rel_residual"])
        nf = torch.linalg.norm(rm["field"]).item()
        d = max(torch.linalg.norm(rs["field"] - rm["field"]).item(),
                torch.linalg.norm(rt["field"] - rm["field"]).item()) / nf
        out["field_diff"].append(d)
        if k in trace_steps:
            out["traces"][k] = {"static": ts, "timeprop": tt, "maze": tm}
    sess.close()
    return out


def summarize(r: Dict, skip: int) -> Dict:
    s = {}
    for key in ("maze", "timeprop", "static"):
        v = np.array(r[key][skip:], dtype=float)
        s[key] = {"mean_iters": float(v.mean()), "min": int(v.min()), "max": int(v.max())}
    s["ratio_timeprop_over_maze"] = s["timeprop"]["mean_iters"] / s["maze"]["mean_iters"]
    s["ratio_static_over_maze"] = s["static"]["mean_iters"] / s["maze"]["mean_iters"]
    s["max_rel_residual"] = float(max(max(r["res_maze"][skip:]), max(r["res_static"][skip:]),
                                      max(r["res_timeprop"][skip:])))
    s["max_field_diff"] = float(max(r["field_diff"][skip:]))
    return s


LEVELS = (1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9)


def iterations_to_levels(rows, levels=LEVELS) -> Dict[str, int]:
    """First iteration at which a traced residual history is at or below
    each level (None if never)."""
    hist = [(it, r) for _, it, r in rows if it >= 0]
    out = {}
    for lv in levels:
        out[f"{lv:.0e}"] = next((it for it, r in hist if r <= lv), None)
    return out


def level_study(system: inputs.NaClSystem, n_steps: int, tol: float, order: int,
                dt: float, skip: int = 3) -> Dict:
    """Iterations each solve needs to reach a ladder of relative residuals,
    averaged over the replayed steps after `skip`."""
    traj = ballistic_trajectory(system, n_steps, dt)
    r = replay_compare(system.charges, traj, system.box, system.grid_spacing, tol,
                       trace_steps=tuple(range(skip, n_steps)), order=order)
    out = {"order": order, "dt_fs": dt, **summarize(r, skip)}
    lv = {}
    for key in ("maze", "timeprop", "static"):
        per = [iterations_to_levels(r["traces"][k][key]) for k in range(skip, n_steps)]
        lv[key] = {L: (float(np.mean([p[L] for p in per])) if all(p[L] is not None for p in per)
                       else None) for L in per[0]}
    out["iters_to_level"] = lv
    out["first_residual"] = {key: float(np.mean([[x for x in r["traces"][k][key] if x[1] == 0][0][2]
                                                 for k in range(skip, n_steps)]))
                             for key in ("maze", "timeprop", "static")}
    return out


def iterations_vs_grid(n_cells: int, grids: Sequence[int], n_steps: int, tol: float,
                       seed: int = 21, skip: int = 3) -> List[Dict]:
    """One system (n_cells^3 rock-salt cells, molten), refined grids N:
    mean iterations per step of the three solves."""
    s = inputs.molten_nacl(n_cells, seed=seed)
    traj = ballistic_trajectory(s, n_steps)
    rows = []
    for N in grids:
        r = replay_compare(s.charges, traj, s.box, s.box / N, tol)
        rows.append({"N": N, "ions": s.n_ions, **summarize(r, skip)})
    return rows


def iterations_vs_ions(box: float, N: int, counts: Sequence[int], n_steps: int, tol: float,
                       seed: int = 22, temperature: float = 1200.0,
                       skip: int = 3) -> List[Dict]:
    """Fixed box and grid, a varying number of ions (random neutral NaCl at
    uniform positions with Maxwell-Boltzmann velocities): mean iterations
    per step of the three solves."""
    rows = []
    for n in counts:
        rng = np.random.default_rng(seed + n)
        half = n // 2
        pos = rng.uniform(0.0, box, size=(2 * half, 3))
        q = np.concatenate([np.ones(half), -np.ones(half)])
        m = np.concatenate([np.full(half, inputs.MASS_NA), np.full(half, inputs.MASS_CL)])
        vel = inputs.maxwell_boltzmann(m, temperature, rng)
        traj = [pos + (k + 1) * vel for k in range(n_steps)]
        r = replay_compare(q, traj, box, box / N, tol)
        rows.append({"ions": 2 * half, "N": N, **summarize(r, skip)})
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description="MaZe vs direct Poisson PLCG convergence study")
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--out", default=None, help="write the JSON result here")
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the convergence study runs on the GPU"
    res = {"tol": args.tol, "scale": "||M phi + 4 pi q/h|| / ||4 pi q/h||"}
    s = inputs.molten_nacl(8, seed=2)
    traj = ballistic_trajectory(s, args.steps)
    r = replay_compare(s.charges, traj, s.box, s.grid_spacing, args.tol,
                       trace_steps=(args.steps - 1,))
    res["nacl4096_g128"] = summarize(r, 3)
    tr = r["traces"][args.steps - 1]
    res["trace_nacl4096_g128"] = {k: [[it, rr] for _, it, rr in v if it >= 0]
                                  for k, v in tr.items()}
    res["levels"] = [level_study(s, args.steps, args.tol, order, dt)
                     for order in (2, 4) for dt in (1.0, 0.25)]
    res["vs_grid"] = iterations_vs_grid(4, (32, 48, 64, 96, 128), args.steps, args.tol)
    res["vs_ions"] = iterations_vs_ions(37.15, 96, (128, 256, 512, 1024, 1458), args.steps,
                                        args.tol)
    txt = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt)
    print(json.dumps({k: v for k, v in res.items() if not k.startswith("trace")}, indent=1))
    return res


if __name__ == "__main__":
    main()
