"""Molten-NaCl structure and transport through the library (Results
section): a canonical equilibration with the OVRVO Langevin integrator from
a bcc start, a microcanonical production run, and from it the radial pair
distribution functions g_IJ(r) (onset, first maximum, first minimum) and the
diffusion coefficients of Na+ and Cl- from the integral of the velocity
autocorrelation function and from the slope of the mean squared
displacement. Every step and every observable runs in the library's
kernels; this module drives them and does the final host arithmetic.

Defaults follow the paper's protocol: 250 ions in L = 20.64 A, T = 1550 K,
friction 1e-3 /fs, time step 0.25 fs, 2.5 ps canonical, 25 ps
microcanonical, h = 0.172 A (120^3).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import inputs, maze, md, observables

# Values the paper prints for this system (its g(r) table and diffusion
# coefficients), for comparison only: a different code and trajectory.
PAPER = {
    "g": {"NaCl": dict(r_cut=1.9, r_max=2.6, g_max=3.5, r_min=4.2),
          "NaNa": dict(r_cut=2.3, r_max=4.2, g_max=1.6, r_min=6.1),
          "ClCl": dict(r_cut=2.6, r_max=4.1, g_max=1.7, r_min=6.1)},
    "D_cm2_s": {"Na": 0.16e-3, "Cl": 0.14e-3},
}


def run_study(nvt_ps=2.5, nve_ps=25.0, dt=0.25, gamma=1e-3, temperature=1550.0, tol=1e-8,
              precision=maze.MAZE_MIXED, seed=1, rdf_every=20, tcf_every=4, max_lag_fs=1000.0,
              origin_fs=20.0, r_max=10.0, dr=0.05, progress_every=4000, log=print):
    s = inputs.bcc_nacl(temperature=temperature, seed=seed)
    run = md.MDRun(s, tol=tol, precision=precision, dt=dt, gamma=gamma,
                   temperature=temperature, seed=seed)
    n_nvt = int(round(nvt_ps * 1000.0 / dt))
    n_nve = int(round(nve_ps * 1000.0 / dt))
    kb3n = 3 * s.n_ions * inputs.KB_EV_PER_K
    out = {"ions": s.n_ions, "box_A": s.box, "grid": run.session.N, "dt_fs": dt,
           "gamma_per_fs": gamma, "temperature_K": temperature, "tol": tol,
           "precision": "mixed" if precision == maze.MAZE_MIXED else "fp64",
           "nvt_steps": n_nvt, "nve_steps": n_nve}
    t0 = time.perf_counter()
    ke = []
    for k in range(n_nvt):
        run.step()
        if k >= n_nvt // 2 and k % 10 == 0:
            ke.append(run.observables()["ke"])
        if progress_every and (k + 1) % progress_every == 0:
            log(f"nvt step {k + 1}/{n_nvt}: T_kin {2 * run.observables()['ke'] / kb3n:.0f} K")
    torch.cuda.synchronize()
    out["nvt_wall_s"] = time.perf_counter() - t0
    out["nvt_mean_T_K"] = float(2.0 * np.mean(ke) / kb3n) if ke else None

    run.set_thermostat(0.0)
    nbins = int(round(r_max / dr))
    rdf = observables.PairHistogram(run.species, s.box, r_max, nbins)
    dt_sample = tcf_every * dt
    max_lag = int(round(max_lag_fs / dt_sample))
    every = max(1, int(round(origin_fs / dt_sample)))
    tcf = observables.TimeCorrelations(run.species, max_lag, every)
    o0 = run.observables()
    totals, temps = [], []
    t0 = time.perf_counter()
    for k in range(n_nve):
        run.step()
        if k % rdf_every == 0:
            rdf.accumulate(run.pos)
        if k % tcf_every == 0:
            tcf.sample(run.pos, run.vel)
        if k % 200 == 0:
            o = run.observables()
            totals.append(o["total"])
            temps.append(2 * o["ke"] / kb3n)
        if progress_every and (k + 1) % progress_every == 0:
            log(f"nve step {k + 1}/{n_nve}: total {run.observables()['total']:.6f} eV")
    torch.cuda.synchronize()
    out["nve_wall_s"] = time.perf_counter() - t0
    out["md_steps_per_s"] = (n_nvt + n_nve) / (out["nvt_wall_s"] + out["nve_wall_s"])
    o1 = run.observables()
    out["nve_momentum_start"] = o0["momentum"].tolist()
    out["nve_momentum_end"] = o1["momentum"].tolist()
    out["nve_mean_T_K"] = float(np.mean(temps))
    out["nve_total_energy_drift_eV"] = o1["total"] - o0["total"]
    out["nve_total_energy_rms_eV"] = float(np.std(totals))
    out["nve_max_abs_momentum"] = float(np.abs(o1["momentum"]).max())

    r = rdf.r_mid()
    g = rdf.g()
    out["g_features"] = {name: observables.g_features(r, g[k])
                         for k, name in enumerate(observables.ROWS)}
    out["g_r"] = {"r": r.tolist(), **{name: g[k].tolist()
                                      for k, name in enumerate(observables.ROWS)}}
    vacf, msd = tcf.averages()
    D = {}
    for k, name in enumerate(("Na", "Cl")):
        D[name] = {"vacf_cm2_s": observables.diffusion_vacf(vacf[k], dt_sample)
                   * observables.A2_PER_FS_TO_CM2_PER_S,
                   "msd_cm2_s": observables.diffusion_msd(msd[k], dt_sample, start=max_lag // 2)
                   * observables.A2_PER_FS_TO_CM2_PER_S}
    out["diffusion"] = D
    out["vacf_normalised"] = {name: (vacf[k] / vacf[k][0]).tolist()
                              for k, name in enumerate(("Na", "Cl"))}
    out["paper"] = PAPER
    tcf.close()
    run.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="molten-NaCl structure and transport study")
    ap.add_argument("--nvt-ps", type=float, default=2.5)
    ap.add_argument("--nve-ps", type=float, default=25.0)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the study runs on the GPU"
    res = run_study(nvt_ps=args.nvt_ps, nve_ps=args.nve_ps, tol=args.tol,
                    precision=maze.MAZE_FP64 if args.fp64 else maze.MAZE_MIXED,
                    log=lambda m: print(m, flush=True))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    brief = {k: v for k, v in res.items() if k not in ("g_r", "vacf_normalised")}
    print(json.dumps(brief, indent=1))
    return res


if __name__ == "__main__":
    main()
