"""Force and energy estimators (Section 2.1; two-particle appendix).

Two measurements through the library:

* one unit charge in a uniform neutralising background, moved across a grid
  cell: the discrete energy of equation "energy_discr" (which contains the
  self-energy and oscillates with the sub-cell position), the force of
  equation "F_nostra" (zero at every offset) and the weight-gradient force
  of equation "F_Benoit" (which follows the self-energy oscillation);
* molten NaCl in NVE with either force: total momentum and the drift of
  KE + V_sr + V_work over the run.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import inputs, maze, md


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def self_energy_scan(order: int, box: float = 6.0, N: int = 12, points: int = 21,
                     y_off: float = 0.0, z_off: float = 0.0):
    """Energy and both forces of one unit charge at x = (3 + t) h, t in
    [0, 1], with a uniform neutralising background."""
    h = box / N
    rows = []
    Q = _dev(np.array([1.0]))
    flags = maze.MAZE_FLAG_ALLOW_NET_CHARGE
    for t in np.linspace(0.0, 1.0, points):
        pos = _dev(np.array([[(3.0 + t) * h, (2.0 + y_off) * h, (5.0 + z_off) * h]]))
        a = maze.Session(Q, pos, box, h, tol=1e-13, order=order, flags=flags)
        b = maze.Session(Q, pos, box, h, tol=1e-13, order=order,
                         flags=flags | maze.MAZE_FLAG_WEIGHT_GRADIENT_FORCE)
        ra = a.solve(pos, want_field=False)
        rb = b.solve(pos, want_field=False)
        rows.append({"t": float(t), "energy": ra["energy"].item(),
                     "force_nostra_x": ra["forces"][0, 0].item(),
                     "force_benoit_x": rb["forces"][0, 0].item()})
        a.close()
        b.close()
    e = np.array([r["energy"] for r in rows])
    fb = np.array([r["force_benoit_x"] for r in rows])
    fn = np.array([r["force_nostra_x"] for r in rows])
    return {"order": order, "N": N, "h": h, "rows": rows,
            "energy_spread": float(e.max() - e.min()), "energy_mean": float(e.mean()),
            "max_abs_force_nostra": float(np.abs(fn).max()),
            "max_abs_force_benoit": float(np.abs(fb).max())}


def nve_run(flags: int, order: int, steps: int, tol: float = 1e-10, n_cells: int = 2,
            seed: int = 1, dt: float = 1.0):
    """NVE molten NaCl: momentum and conserved-energy drift per force."""
    s = inputs.molten_nacl(n_cells, seed=seed)
    run = md.MDRun(s, tol=tol, order=order, dt=dt, flags=flags)
    o0 = run.observables()
    p_max = 0.0
    for _ in range(steps):
        run.step()
        p_max = max(p_max, float(np.abs(run.observables()["momentum"]).max()))
    o1 = run.observables()
    run.close()
    return {"flags": flags, "order": order, "steps": steps, "tol": tol,
            "max_abs_momentum_amu_A_per_fs": p_max,
            "total_energy_drift_eV": o1["total"] - o0["total"],
            "kinetic_eV": o1["ke"]}


def main(argv=None):
    ap = argparse.ArgumentParser(description="force and energy estimator study")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the estimator study runs on the GPU"
    res = {"self_energy": [self_energy_scan(o) for o in (2, 4)], "nve": []}
    for order in (2, 4):
        for flags in (0, maze.MAZE_FLAG_WEIGHT_GRADIENT_FORCE):
            res["nve"].append(nve_run(flags, order, args.steps))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    brief = {"self_energy": [{k: v for k, v in r.items() if k != "rows"}
                             for r in res["self_energy"]], "nve": res["nve"]}
    print(json.dumps(brief, indent=1))
    return res


if __name__ == "__main__":
    main()
