#!/usr/bin/env python3
"""Benchmark of the Poisson MaZe MD step on one MI355X.

Workload (default): molten NaCl, 32768 ions (16^3 rock-salt cells, seeded
jitter, Maxwell-Boltzmann velocities at 1200 K), L = 102 A, 256^3 grid,
dt = 1 fs, PLCG relative residual 1e-8. Each step is a full device-resident
MD step: velocity-Verlet kick/drift, charge assignment, the warm-started
MaZe PLCG solve, field update, force interpolation and the Tosi-Fumi short
range. The mixed-precision path (FP32 stencil and vectors, FP64 dots and
refinement) is the headline value; the FP64 path runs side by side, and the
mixed path's field, force and energy error against FP64 is reported on a
replay of the FP64 trajectory.

The PLCG runs in its two-iteration (s-step, s = 2) form by default
(`--cg sstep`): a basis kernel and an update kernel per two iterations.
`--cg sweep` runs the one-iteration fused sweep instead; the default run
also times that form on the same workload (`one_iteration_sweep`).

Prints ONE JSON line. `roofline` describes the dominant kernel, the update
kernel of the two-iteration CG in the mixed path's FP32 inner solves (the
FP64 one is in `roofline_fp64`; each carries its basis kernel under
`basis_kernel`), timed with HIP events that the library records around
sampled outer steps on the stream they run on. `cpu_baseline` times the
plain FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2505_20418_amd", "csrc")
# committed counter summaries: HBM bytes per launch, with the hash of the
# kernel source they were taken with
TRAFFIC = {"sweep": (os.path.join(ROOT, "profiles", "traffic_cg_sweep_nacl32768_g256.json"),
                     os.path.join(CSRC, "k_cg.hip")),
           "sstep": (os.path.join(ROOT, "profiles", "traffic_sstep_nacl32768_g256.json"),
                     os.path.join(CSRC, "k_sstep.hip"))}
# algorithmic HBM bytes per grid point of one fused CG sweep, and of the
# update kernel of the two-iteration form: read x, r, p and write x, r, p
# once (FP64: 8 B each, FP32: 4 B each); the basis kernel reads r and p
SWEEP_BYTES = {"fp64": 48, "fp32": 24}
BASIS_BYTES = {"fp64": 16, "fp32": 8}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


# Launch shapes the benchmark pins for the 256^3 headline sessions of the
# two-iteration CG (threads:points per thread:x planes, or zv:wavefronts:x
# planes for the wavefront-row layout of the basis kernel), so that every
# run times the shapes the committed counter summaries were taken in: the
# fastest shapes in whole-MD-step timings of the tuner's candidates, which
# the tuner's own short timings do not rank reliably between boxes. Basis
# kernel, FP32: zv:16:20 41.7 us, zv:8:24 42.8 us, zv:16:22 43.8 us, zv:8:52
# 49.0 us; FP64: zv:8:52 71.5 us, zv:8:64 83.0 us, 512:2:64 86.5 us. Update
# kernel, FP32: 512:4:32 77.8 us, 512:4:16 82.7 us, 512:2:32 86.4 us.
PINNED_SHAPES = {
    ("nacl32768_g256", "fp32"): {"MAZE_BASIS_SHAPE": "zv:16:20", "MAZE_UPDATE_SHAPE": "512:4:32"},
    ("nacl32768_g256", "fp64"): {"MAZE_BASIS_SHAPE": "zv:8:52", "MAZE_UPDATE_SHAPE": "512:4:32"},
}
# and of the one-iteration sweep (points per thread:x planes)
PINNED_SWEEP = {
    ("nacl32768_g256", "fp32"): {"MAZE_SWEEP_SHAPE": "4:22"},
    ("nacl32768_g256", "fp64"): {"MAZE_SWEEP_SHAPE": "4:64"},
}


def run_md(system, tol, precision, steps, warmup, record_positions=False, order=2, flags=0,
           gamma=0.0, pin=None):
    """pin: environment settings that force launch shapes while the session
    is created (read by the library's tuner at maze_init)."""
    import torch
    from paper_2505_20418_amd import maze, md

    saved = {k: os.environ.get(k) for k in (pin or {})}
    os.environ.update(pin or {})
    try:
        run = md.MDRun(system, tol=tol, precision=precision, order=order, flags=flags,
                       gamma=gamma, temperature=system.temperature, seed=7)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    h = run.session.handle
    for _ in range(warmup):
        run.step()
    maze.maze_profile_enable(h, True)
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    traj = None
    if record_positions:
        traj = torch.empty((steps,) + tuple(run.pos.shape), dtype=run.pos.dtype,
                           device=run.pos.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k].record(stream)
        run.step()
        if traj is not None:
            traj[k].copy_(run.pos)
    evs[steps].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = maze.maze_profile_read(h)
    maze.maze_profile_enable(h, False)
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    obs = run.observables()
    shape = maze.maze_launch_shape(h)["latency"]
    shape["basis"] = maze.maze_basis_shape(h)
    shape["basis"]["layout"] = maze.maze_sstep_layout(h)["basis"]
    out = dict(steps_per_s=steps / (t1 - t0), wall_s=t1 - t0, lat_ms=lat, prof=prof,
               obs=obs, grid_n=run.session.N, traj=traj, shape=shape)
    run.close()
    return out


def replay_errors(system, traj, tol, n_replay, every=1, flags=0):
    """Drive a fresh mixed session and a fresh FP64 session through the same
    recorded positions (both advance every step, so the warm starts match
    the run); errors of mixed against FP64 at every `every`-th step."""
    import torch
    from paper_2505_20418_amd import inputs, maze

    dev = torch.device("cuda")
    Q = torch.tensor(system.charges, dtype=torch.float64, device=dev)
    p0 = torch.tensor(system.pos, dtype=torch.float64, device=dev)
    s64 = maze.Session(Q, p0, system.box, system.grid_spacing, tol=tol,
                       precision=maze.MAZE_FP64, coulomb_k=inputs.COULOMB_K_EV_A, flags=flags)
    s32 = maze.Session(Q, p0, system.box, system.grid_spacing, tol=tol,
                       precision=maze.MAZE_MIXED, coulomb_k=inputs.COULOMB_K_EV_A, flags=flags)
    ef, eF, eE, at = [], [], [], []
    for k in range(min(n_replay, traj.shape[0])):
        want = (k + 1) % every == 0
        a = s64.step(traj[k], want_field=want)
        b = s32.step(traj[k], want_field=want)
        if not want:
            continue
        at.append(k + 1)
        ef.append((torch.linalg.norm(b["field"] - a["field"]) / torch.linalg.norm(a["field"])).item())
        eF.append((torch.linalg.norm(b["forces"] - a["forces"]) / torch.linalg.norm(a["forces"])).item())
        eE.append(abs((b["energy"] - a["energy"]).item()) / abs(a["energy"].item()))
    s64.close()
    s32.close()
    out = dict(field_rel_l2_max=max(ef), forces_rel_l2_max=max(eF), energy_rel_max=max(eE),
               steps_compared=len(ef))
    if every > 1:
        out.update(steps=at, field_rel_l2=ef, forces_rel_l2=eF, energy_rel=eE)
    return out


def roofline(prof_key, prof, G, dtype_key, shape=None, sstep=False):
    """Roofline of the dominant CG kernel from the library's event timings:
    the fused sweep, or (sstep) the update kernel of the two-iteration form
    with its basis kernel alongside."""
    n, ms = prof[prof_key]
    if n == 0:
        return None
    upd_ms = prof[f"{dtype_key}_update_ms"] if sstep else ms
    avg_s = upd_ms / n / 1e3
    bpl = SWEEP_BYTES[dtype_key] * G
    achieved = bpl / avg_s / 1e9
    kernel = f"k_sstep update ({dtype_key})" if sstep else f"k_cg_sweep ({dtype_key})"
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
         "kernel": kernel, "avg_launch_us": round(avg_s * 1e6, 2),
         "launches_timed": n, "algorithmic_bytes_per_launch": bpl}
    if sstep:
        b_s = (ms - upd_ms) / n / 1e3
        bb = BASIS_BYTES[dtype_key] * G
        r["basis_kernel"] = {"kernel": f"k_sstep basis ({dtype_key})",
                             "avg_launch_us": round(b_s * 1e6, 2),
                             "algorithmic_bytes_per_launch": bb,
                             "achieved": round(bb / b_s / 1e9, 1),
                             "frac": round(bb / b_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None}
        r["outer_step_us"] = round(ms / n * 1e3, 2)
        r["iterations_per_outer_step"] = 2
        ob = bpl + bb
        r["outer_step"] = {"kernels": "basis + update", "algorithmic_bytes": ob,
                           "avg_us": round(ms / n * 1e3, 2),
                           "achieved": round(ob / (ms / n / 1e3) / 1e9, 1),
                           "frac": round(ob / (ms / n / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        if shape is not None and "basis" in shape:
            bs = shape["basis"]
            # layout: wavefronts per workgroup of the wavefront-row layout, 0
            # for the segment layout
            r["basis_kernel"]["launch_shape"] = {
                "threads": bs["threads"], "ppt": bs["ppt"], "cx": bs["cx"],
                "workgroups": bs["nwg"], "grid_threads": bs["nwg"] * bs["threads"],
                "layout": bs.get("layout", 0)}
    if shape is not None:
        # the launch shape the session swept in; a kernel trace of this run
        # also holds the autotuner's timing sweeps in other shapes, which
        # this grid size (workgroups x threads) tells apart
        threads = shape["segment"] // shape["ppt"] if "segment" in shape else 256
        r["launch_shape"] = {"threads": threads, "ppt": shape["ppt"], "cx": shape["cx"],
                             "workgroups": shape["nwg"], "grid_threads": shape["nwg"] * threads}
    return r


def attach_ceilings(r, copy_gbps):
    """The sweep's rate against the measured copy rate, and the counter-
    measured rate (HBM bytes from the counters over the same launch time)
    against both ceilings."""
    if r is None:
        return
    r["copy_GBps"] = round(copy_gbps, 1)
    r["frac_of_copy"] = round(r["achieved"] / copy_gbps, 4)
    if r.get("traffic"):
        g = r["traffic"] / (r["avg_launch_us"] * 1e-6) / 1e9
        r["counter_GBps"] = round(g, 1)
        r["counter_frac"] = round(g / HBM_PEAK_GBS, 4)
        r["counter_frac_of_copy"] = round(g / copy_gbps, 4)


def attach_outer(r, copy_gbps):
    """The outer step (basis and update kernel, two iterations) against the
    ceilings, on algorithmic bytes and, where both kernels' counter traffic
    is known, on counted HBM bytes."""
    o = r.get("outer_step")
    if o is None:
        return
    o["copy_GBps"] = round(copy_gbps, 1)
    o["frac_of_copy"] = round(o["achieved"] / copy_gbps, 4)
    tb = (r.get("basis_kernel") or {}).get("traffic")
    if r.get("traffic") and tb:
        o["traffic"] = r["traffic"] + tb
        g = o["traffic"] / (o["avg_us"] * 1e-6) / 1e9
        o["counter_GBps"] = round(g, 1)
        o["counter_frac"] = round(g / HBM_PEAK_GBS, 4)
    else:
        o["traffic"] = None


def attach_traffic(r, key, form="sweep"):
    """HBM bytes per launch from the committed counter summary, if it was
    taken with the current kernel source and in the launch shape this run
    swept in (for the two-iteration form: key_update and key_basis)."""
    path, src = TRAFFIC[form]
    if r is None or not os.path.exists(path):
        return
    try:
        t = json.load(open(path))
    except Exception:
        return
    if t.get("stencil_sha") != source_hash(src):
        return
    targets = [(r, key)] if form == "sweep" else [(r, f"{key}_update"),
                                                  (r.get("basis_kernel"), f"{key}_basis")]
    for obj, k in targets:
        if obj is None or k not in t:
            continue
        want = t[k].get("launch_shape")
        have = obj.get("launch_shape", r.get("launch_shape"))
        if want is None or have is None:
            continue
        shape_key = lambda x: (x.get("threads", 256), x["ppt"], x["cx"],  # noqa: E731
                               x.get("layout", 0))
        if shape_key(want) != shape_key(have):
            continue
        obj["traffic"] = t[k]["hbm_bytes_per_launch"]


def cpu_worker(mode: str, workload: str, omp: bool, iters_per_step: float = 0.0,
               steps: int = 5) -> dict:
    """One CPU-oracle measurement, run in a process of its own (no torch; the
    OpenMP build takes its threads from OMP_NUM_THREADS):
      sample  the headline workload: one MD step with the solve capped at 0
              iterations plus 60 PLCG iterations, extrapolated to
              iters_per_step iterations per step;
      run     the workload's cold solve, then `steps` warm MD steps, timed."""
    import oracle
    from paper_2505_20418_amd import inputs

    wl = inputs.WORKLOADS[workload]
    system = inputs.workload(workload)
    tol = wl["tol"]
    common = dict(coulomb_k=inputs.COULOMB_K_EV_A, omp=omp)
    pos, vel = system.pos.copy(), system.vel.copy()
    F_sr, _ = oracle.bmh(pos, system.species, system.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    work = np.zeros(1)
    args = (system.masses, system.species, inputs.BMH_TABLE, inputs.BMH_CUTOFF, 1.0,
            inputs.ACCEL_FACTOR)
    if mode == "sample":
        n_cg = 60
        sess = oracle.Session(system.charges, pos, system.box, system.grid_spacing, tol=tol,
                              max_iter=0, **common)
        F_es = np.zeros_like(pos)
        t0 = time.perf_counter()
        sess.md_step(pos, vel, *args, F_es, F_sr, work)
        t_other = time.perf_counter() - t0
        N = sess.N
        b = 4 * np.pi * sess.state()["q"] / (system.box / N)
        L = oracle.lib_omp() if omp else oracle.lib()
        x = np.zeros_like(b)
        it = oracle.ctypes.c_int(0)
        t0 = time.perf_counter()
        L.oracle_pcg(N, oracle._d(b.ravel()), oracle._d(x.ravel()), 0.0, oracle.NORM_REL2, n_cg,
                     oracle.ctypes.byref(it))
        t_iter = (time.perf_counter() - t0) / n_cg
        sess.close()
        per_step = t_other + iters_per_step * t_iter
        return {"steps_per_s": 1.0 / per_step, "s_non_cg_per_step": t_other,
                "s_per_cg_iteration": t_iter, "iters_per_step": iters_per_step, "grid": N}
    tag = f"cpu oracle {workload} ({'OpenMP' if omp else 'plain'}, " \
          f"{os.environ.get('OMP_NUM_THREADS', '1') if omp else 1} threads)"
    t0 = time.perf_counter()
    sess = oracle.Session(system.charges, pos, system.box, system.grid_spacing, tol=tol,
                          **common)
    t_init = time.perf_counter() - t0
    print(f"bench: {tag}: cold solve {t_init:.1f} s", file=sys.stderr, flush=True)
    F_es = sess.step(pos)["forces"]  # forces at the start, as the MD prime step
    iters = 0
    t0 = time.perf_counter()
    for k in range(steps):
        st = sess.md_step(pos, vel, *args, F_es, F_sr, work)
        iters += st["stats"]["iters"]
        if steps <= 10:
            print(f"bench: {tag}: step {k + 1}/{steps}, {st['stats']['iters']} iterations, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    sess.close()
    return {"steps_per_s": steps / dt, "steps": steps, "s_per_step": dt / steps,
            "cg_iterations_per_step": iters / steps,
            "s_per_cg_iteration": dt / max(iters, 1), "s_cold_solve": t_init,
            "grid": inputs.GRID_PER_CELL * wl["n_cells"]}


def _cpu_run(mode, workload, omp, threads, iters_per_step=0.0, steps=5):
    """cpu_worker in a child process with `threads` OpenMP threads."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker",
           json.dumps({"mode": mode, "workload": workload, "omp": omp,
                       "iters_per_step": iters_per_step, "steps": steps})]
    # the worker's progress lines go straight to this process's stderr
    out = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, text=True, check=True).stdout
    return json.loads(out.strip().splitlines()[-1])


def cpu_baseline(workload, iters_per_step, full=False):
    """The plain FP64 oracle on the host's cores: the plain build on one
    thread and its OpenMP build (order-independent loops threaded, bitwise
    the same results) on every core this process may use. Default: the
    headline workload's step from a one-step sample plus 60 PLCG iterations
    (extrapolated to the GPU FP64 path's iterations per step), and the
    64-ion workload's 100 NVE steps measured in full. full: also 5 measured
    warm steps of the 4096-ion and 32768-ion workloads after their cold
    solves."""
    from paper_2505_20418_amd import inputs

    import oracle
    oracle.build(force=False)
    threads = len(os.sched_getaffinity(0))
    t_start = time.perf_counter()
    legs = [(1, False), (threads, True)]
    sample = {t: _cpu_run("sample", workload, omp, t, iters_per_step) for t, omp in legs}
    c1 = {t: _cpu_run("run", "nacl64_g32", omp, t, steps=inputs.WORKLOADS["nacl64_g32"]["steps"])
          for t, omp in legs}
    out = {"value": round(sample[threads]["steps_per_s"], 6), "unit": "MD steps/s",
           "cores": threads, "kind": "oracle", **host_description()}
    out["single_thread"] = {"value": round(sample[1]["steps_per_s"], 6), "cores": 1}
    for t in sample:
        sample[t] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in sample[t].items()}
    out["headline_sample"] = {"1": sample[1], str(threads): sample[threads]}
    out["nacl64_g32_100_steps"] = {
        str(t): {k: (round(v, 5) if isinstance(v, float) else v) for k, v in c1[t].items()}
        for t in c1}
    if full:
        # the 256^3 cold solve alone takes minutes on one thread: there the
        # one-thread figure is the headline sample's
        for wl, wl_legs in (("nacl4096_g128", legs), ("nacl32768_g256", legs[1:])):
            out[f"{wl}_warm_steps"] = {
                str(t): {k: (round(v, 4) if isinstance(v, float) else v)
                         for k, v in _cpu_run("run", wl, omp, t, steps=5).items()}
                for t, omp in wl_legs}
    total = time.perf_counter() - t_start
    out["sample"] = (f"{workload}: one oracle MD step with the solve capped at 0 iterations plus "
                     f"60 oracle PLCG iterations, extrapolated to {iters_per_step:.1f} iterations "
                     f"per step (GPU FP64 path), on {threads} threads (OpenMP build: stencil, "
                     f"AXPY and elementwise loops threaded, reductions sequential) and on 1 "
                     f"thread; plus nacl64_g32's 100 NVE steps measured on both"
                     + ("; plus 5 measured warm steps of nacl4096_g128 (both) and "
                        "nacl32768_g256 (all threads)" if full else "")
                     + f"; {total:.1f} s of CPU work; plain C, -O2 -ffp-contract=off")
    return out


def copy_bandwidth(gib: float = 4.0, reps: int = 10) -> float:
    """Rate (bytes read + written per second, GB/s) of the library's
    streaming copy kernel (maze_stream_copy) between two 4 GiB buffers, an
    8 GiB footprint far beyond the L2 and Infinity Cache: the practical HBM
    ceiling for kernels that read and write every byte once."""
    import torch
    from paper_2505_20418_amd import maze
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    maze.maze_stream_copy(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        maze.maze_stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    assert torch.equal(a[:1024], b[:1024]) and torch.equal(a[-1024:], b[-1024:])
    del a, b
    return 2.0 * n * 8 / t / 1e9


def host_description():
    """CPU model and thread count of the host, and a numpy triad rate
    (a = b + s c over 3 x 800 MB; 24 bytes per element) as the oracle's own
    bandwidth roofline."""
    model = None
    ident = {}
    keys = {"vendor_id": "vendor", "cpu family": "family", "model": "model_number",
            "stepping": "stepping", "cpu MHz": "mhz", "cache size": "cache"}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if ident:
                    break  # the first processor's block is enough
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k == "model name" and model is None:
                model = v
            elif k in keys and keys[k] not in ident:
                ident[keys[k]] = v
            elif k == "flags" and "vector_isa" not in ident:
                have = set(v.split())
                ident["vector_isa"] = [f for f in ("avx2", "fma", "avx512f", "avx512_bf16")
                                       if f in have]
    except OSError:
        pass
    n = 100_000_000
    b = np.ones(n)
    c = np.ones(n)
    a = np.empty(n)
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        np.multiply(c, 3.0, out=a)
        np.add(a, b, out=a)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    # multiply reads c, writes a; add reads a and b, writes a: 40 B/element
    # the model name is what the host reports (virtual machines often give
    # a generic one); the identification fields below pin it down further
    return {"cpu_model": model, "cpu_id": ident, "host_threads": os.cpu_count(),
            "host_triad_GBps": round(40.0 * n / best / 1e9, 1)}


def copy_calibration(gib: float = 2.0, reps: int = 5):
    """The library's streaming copy (k_stream_copy) of known size, for
    scaling the HBM counters."""
    import torch
    from paper_2505_20418_amd import maze
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        maze.maze_stream_copy(b, a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8,
                      "launches": reps}))


def bench_c2(steps: int, warmup: int, flags: int, copy_gbps: float):
    """4096 ions (8^3 rock-salt cells), L = 51 A, 128^3 grid, FP64 MaZe at a
    1e-9 relative residual with warm starts: MD steps/s and the roofline of
    its CG kernels."""
    from paper_2505_20418_amd import inputs, maze

    name = "nacl4096_g128"
    wl = inputs.WORKLOADS[name]
    system = inputs.workload(name)
    N = inputs.GRID_PER_CELL * wl["n_cells"]
    ss = bool(flags & maze.MAZE_FLAG_SSTEP)
    r = run_md(system, wl["tol"], maze.MAZE_FP64, steps, warmup, flags=flags)
    rl = roofline("fp64_sweep", r["prof"], N ** 3, "fp64", r["shape"], sstep=ss)
    attach_ceilings(rl, copy_gbps)
    if ss and rl is not None:
        attach_ceilings(rl.get("basis_kernel"), copy_gbps)
        attach_outer(rl, copy_gbps)
    return {"value": round(r["steps_per_s"], 4), "unit": "MD steps/s", "steps": steps,
            "config": {"workload": name, "ions": system.n_ions, "grid": N, "box_A": system.box,
                       "tol_rel_residual": wl["tol"], "precision": "fp64", "dt_fs": 1.0,
                       "temperature_K": system.temperature},
            "cg_iterations_per_step": round(r["prof"]["fp64_iters"] / steps, 1),
            "latency_ms": {"p50": round(float(np.percentile(r["lat_ms"], 50)), 3),
                           "p99": round(float(np.percentile(r["lat_ms"], 99)), 3)},
            "roofline": rl}


def bench_ensemble(steps: int, warmup: int, tol: float = 1e-8, flags: int = 0):
    """64 molten-NaCl replicas of uneven size (2..6 cells per side, 32^3 to
    96^3 grids, 1100-1400 K), mixed precision, advanced together with one
    batched MD step per round, with the batched poll groups launched
    directly and replayed from captured HIP graphs (MAZE_FLAG_GRAPH_CHUNKS);
    the same replicas stepped one by one for comparison."""
    import torch
    from paper_2505_20418_amd import inputs, maze, md

    reps = inputs.ensemble_replicas(64, master_seed=4)
    stream = torch.cuda.Stream()  # graphs need a stream that can be captured

    def timed(fl):
        with torch.cuda.stream(stream):
            runs = [md.MDRun(inputs.molten_nacl(r.n_cells, seed=r.seed,
                                                temperature=r.temperature),
                             tol=tol, precision=maze.MAZE_MIXED, flags=fl,
                             stream=stream.cuda_stream) for r in reps]
            for _ in range(warmup):
                md.step_many(runs, want_stats=False)
            stream.synchronize()
            lat = []
            t0 = time.perf_counter()
            for _ in range(steps):
                a = time.perf_counter()
                md.step_many(runs, want_stats=False)
                stream.synchronize()
                lat.append(time.perf_counter() - a)
            return runs, time.perf_counter() - t0, np.array(lat) * 1e3

    runs, t_batch, lat_ms = timed(flags)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        for _ in range(steps):
            for r in runs:
                r.step()
        stream.synchronize()
        t_serial = time.perf_counter() - t0
    for r in runs:
        r.close()
    runs_g, t_graph, lat_g = timed(flags | maze.MAZE_FLAG_GRAPH_CHUNKS)
    for r in runs_g:
        r.close()
    pts = sum((inputs.GRID_PER_CELL * r.n_cells) ** 3 for r in reps)
    ions = sum(8 * r.n_cells ** 3 for r in reps)
    pct = lambda a, q: round(float(np.percentile(a, q)), 3)  # noqa: E731
    return {"replicas": len(reps), "ions_total": ions, "grid_points_total": pts,
            "tol_rel_residual": tol, "precision": "mixed", "steps": steps,
            "cg_form": "two-iteration" if flags & maze.MAZE_FLAG_SSTEP else "one-iteration",
            "replica_steps_per_s": round(len(reps) * steps / t_batch, 1),
            "ensemble_steps_per_s": round(steps / t_batch, 3),
            "step_ms": {"p50": pct(lat_ms, 50), "p99": pct(lat_ms, 99)},
            "graph_replica_steps_per_s": round(len(reps) * steps / t_graph, 1),
            "graph_step_ms": {"p50": pct(lat_g, 50), "p99": pct(lat_g, 99)},
            "serial_replica_steps_per_s": round(len(reps) * steps / t_serial, 1),
            "batching_speedup": round(t_serial / t_batch, 3)}


def bench_observables(system, tol, steps, warmup, flags=0):
    """The Results section's canonical dynamics and observables at the
    headline size: OVRVO MD steps/s (mixed, gamma 1e-3 /fs) beside velocity
    Verlet, the pair histogram of all 32768 ions (pairs/s), and one VACF /
    MSD sample over 51 time origins."""
    import torch
    from paper_2505_20418_amd import maze, observables

    out = {}
    for name, g in (("velocity_verlet", 0.0), ("ovrvo", 1e-3)):
        r = run_md(system, tol, maze.MAZE_MIXED, steps, warmup, gamma=g, flags=flags)
        out[f"{name}_mixed_md_steps_per_s"] = round(r["steps_per_s"], 4)
        out[f"{name}_cg_iterations_per_step"] = round(r["prof"]["fp32_iters"] / steps, 1)
    dev = torch.device("cuda")
    pos = torch.tensor(system.pos, dtype=torch.float64, device=dev)
    vel = torch.tensor(system.vel, dtype=torch.float64, device=dev)
    species = torch.tensor(system.species, dtype=torch.int32, device=dev)
    n = system.n_ions
    h = observables.PairHistogram(species, system.box, 12.0, 240)
    h.accumulate(pos)
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        h.accumulate(pos)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    out["pair_histogram"] = {"ions": n, "pairs": n * (n - 1) // 2, "ms": round(t * 1e3, 3),
                             "pairs_per_s": round(n * (n - 1) / 2 / t, 1), "bins": 240,
                             "r_max_A": 12.0}
    tc = observables.TimeCorrelations(species, 1000, 20)
    for _ in range(60):
        tc.sample(pos, vel)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        tc.sample(pos, vel)
    e1.record()
    torch.cuda.synchronize()
    out["time_correlations"] = {"ions": n, "origins": 51, "max_lag_samples": 1000,
                                "ms_per_sample": round(e0.elapsed_time(e1) / reps, 4)}
    tc.close()
    return out


def bench_serving(full: bool, rate_hz: float = 200.0, flags: int = 0, continuous: bool = True):
    """Poisson stream (mean 200 requests/s) of MD-step requests over molten-
    NaCl sessions of log-uniform size, half mixed at 1e-6, half FP64 at
    1e-10, admitted by HBM budget. continuous: steps in flight join and
    leave the running batched CG launches (maze_batch); else rounds of
    batched MD steps grouped by cost class."""
    from paper_2505_20418_amd import serve

    if full:
        n_sess, max_cells, n_req, budget = 256, 16, 2000, 64 << 30
    else:
        n_sess, max_cells, n_req, budget = 64, 8, 400, 16 << 30
    specs = serve.specs_from_inputs(count=n_sess, seed=5, max_cells=max_cells)
    srv = serve.Server(serve.GpuBackend(flags=flags, continuous=continuous), specs, budget,
                       max_batch=64)
    t0 = time.perf_counter()
    resident = srv.prefill()
    t_prefill = time.perf_counter() - t0
    reqs = serve.poisson_requests(n_req, n_sess, rate_hz=rate_hz, seed=5)
    rep = srv.serve(reqs)
    srv.close()
    rep = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
    for key in ("latency_ms", "service_ms"):
        rep[key] = {k: (round(v, 3) if v is not None else None) for k, v in rep[key].items()}
    rep.update({"sessions": n_sess, "max_ions": 8 * max_cells ** 3,
                "max_grid": inputs_grid(max_cells), "arrival_rate_hz": rate_hz,
                "prefilled_resident": resident, "prefill_s": round(t_prefill, 2),
                "mix": "full (256 sessions, 64-32768 ions, 32^3-256^3)" if full
                else "reduced (sessions up to 4096 ions, 128^3)",
                "cg_form": "two-iteration" if flags else "one-iteration"})
    if continuous:
        rep["mean_in_flight"] = rep.pop("mean_batch")
        rep["max_in_flight"] = rep.pop("max_batch")
        rep["poll_groups"] = rep.pop("rounds")
    return rep


def inputs_grid(n_cells):
    from paper_2505_20418_amd import inputs
    return inputs.GRID_PER_CELL * n_cells


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="nacl32768_g256")
    ap.add_argument("--cg", choices=("sstep", "sweep"), default="sstep",
                    help="PLCG form of the headline: two-iteration (s-step) or one-iteration "
                         "fused sweep")
    ap.add_argument("--no-sweep-compare", action="store_true",
                    help="skip timing the one-iteration sweep beside the two-iteration form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pin", action="store_true",
                    help="let the session tuner pick the headline sessions' launch shapes")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the 4096-ion, 128^3 FP64 leg")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="also time 5 warm oracle steps of the 4096- and 32768-ion workloads "
                         "after their cold solves (minutes of CPU work)")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--mixed-only", action="store_true",
                    help="skip the FP64 side-by-side run (for profiling)")
    ap.add_argument("--replay", type=int, default=6, help="steps replayed for the error report")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-order4", action="store_true")
    ap.add_argument("--no-multigrid", action="store_true")
    ap.add_argument("--no-observables", action="store_true")
    ap.add_argument("--serving-rate", type=float, default=200.0,
                    help="mean Poisson arrival rate of the serving leg [requests/s]")
    ap.add_argument("--error-trajectory", type=int, default=500,
                    help="record an FP64 trajectory of this many steps and compare the mixed "
                         "path with it every 50 steps (0: off)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-reduced", action="store_true",
                    help="serve a reduced mix (64 sessions up to 4096 ions, 128^3) instead of "
                         "the full one (256 sessions, 64-32768 ions, 32^3-256^3)")
    ap.add_argument("--serving-rounds", action="store_true",
                    help="also serve the stream in rounds of batched MD steps (cost classes)")
    args = ap.parse_args()
    if args.cpu_worker:
        spec = json.loads(args.cpu_worker)
        print(json.dumps(cpu_worker(spec["mode"], spec["workload"], spec["omp"],
                                    spec["iters_per_step"], spec["steps"])))
        return

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(slab decomposition across GPUs is designed, not implemented).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    from paper_2505_20418_amd import inputs, maze

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = inputs.WORKLOADS[args.workload]
    system = inputs.workload(args.workload)
    tol = wl["tol"]
    G = (inputs.GRID_PER_CELL * wl["n_cells"]) ** 3

    ss = args.cg == "sstep"
    cg_flags = maze.MAZE_FLAG_SSTEP if ss else 0
    log(f"bench: {args.workload} ions={system.n_ions} grid={inputs.GRID_PER_CELL * wl['n_cells']}^3 "
        f"tol={tol} cg={args.cg} mixed: warmup {args.warmup}, {args.steps} timed steps")
    pins = PINNED_SHAPES if ss else PINNED_SWEEP
    pin32 = None if args.no_pin else pins.get((args.workload, "fp32"))
    pin64 = None if args.no_pin else pins.get((args.workload, "fp64"))
    mixed = run_md(system, tol, maze.MAZE_MIXED, args.steps, args.warmup, flags=cg_flags,
                   pin=pin32)
    log(f"bench: mixed {mixed['steps_per_s']:.3f} steps/s")
    fp64 = None
    errors = None
    if not args.mixed_only:
        fp64 = run_md(system, tol, maze.MAZE_FP64, args.steps, args.warmup,
                      record_positions=True, flags=cg_flags, pin=pin64)
        log(f"bench: fp64 {fp64['steps_per_s']:.3f} steps/s")
        if args.replay > 0:
            errors = replay_errors(system, fp64["traj"], tol, args.replay, flags=cg_flags)
            log(f"bench: mixed vs fp64 errors {errors}")

    r_mixed = roofline("fp32_sweep", mixed["prof"], G, "fp32", mixed["shape"], sstep=ss)
    r_fp64 = (roofline("fp64_sweep", fp64["prof"], G, "fp64", fp64["shape"], sstep=ss)
              if fp64 else None)
    if ss:
        attach_traffic(r_mixed, "fp32", "sstep")
        attach_traffic(r_fp64, "fp64", "sstep")
    else:
        attach_traffic(r_mixed, "fp32_sweep")
        attach_traffic(r_fp64, "fp64_sweep")
    copy_gbps = copy_bandwidth()
    attach_ceilings(r_mixed, copy_gbps)
    attach_ceilings(r_fp64, copy_gbps)
    if ss:
        for r in (r_mixed, r_fp64):
            if r is None:
                continue
            attach_ceilings(r.get("basis_kernel"), copy_gbps)
            attach_outer(r, copy_gbps)
            r["shapes_pinned"] = bool(pin32)

    it_mixed = mixed["prof"]["fp32_iters"] / args.steps
    it_fp64 = fp64["prof"]["fp64_iters"] / args.steps if fp64 else None
    cpu = None
    if not args.no_cpu_baseline and it_fp64:
        log("bench: timing the CPU oracle sample")
        cpu = cpu_baseline(args.workload, it_fp64, full=args.cpu_baseline_full)

    value = mixed["steps_per_s"]
    line = {
        "metric": "MD steps/s + stencil-CG HBM GB/s (NaCl 32k ions, 256^3); mixed vs FP64; p99",
        "value": round(value, 4),
        "unit": "MD steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 / value, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "ions": system.n_ions,
                   "grid": inputs.GRID_PER_CELL * wl["n_cells"], "box_A": system.box,
                   "tol_rel_residual": tol, "dt_fs": 1.0, "temperature_K": system.temperature,
                   "assignment_order": 2, "precision": "mixed (fp32 stencil/vectors, fp64 dots "
                   "and refinement)", "cg_form": ("two-iteration s-step PLCG (s=2)" if ss else
                                                 "one-iteration fused PLCG sweep"),
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(mixed["lat_ms"], 50)), 3),
                       "p99": round(float(np.percentile(mixed["lat_ms"], 99)), 3)},
        "cg_iterations_per_step": {"mixed_fp32_inner": round(it_mixed, 1)},
        "roofline": r_mixed,
    }
    if fp64:
        line["fp64"] = {"value": round(fp64["steps_per_s"], 4), "unit": "MD steps/s",
                        "latency_ms": {"p50": round(float(np.percentile(fp64["lat_ms"], 50)), 3),
                                       "p99": round(float(np.percentile(fp64["lat_ms"], 99)), 3)}}
        line["speedup_mixed_vs_fp64"] = round(value / fp64["steps_per_s"], 3)
        line["cg_iterations_per_step"]["fp64"] = round(it_fp64, 1)
        line["roofline_fp64"] = r_fp64
        line["mixed_error_vs_fp64"] = errors
    if ss and not args.no_sweep_compare:
        # the same workload with the one-iteration fused sweep
        log("bench: one-iteration sweep")
        one = {}
        for name, prec, key, dk in (("mixed", maze.MAZE_MIXED, "fp32_sweep", "fp32"),
                                    ("fp64", maze.MAZE_FP64, "fp64_sweep", "fp64")):
            if name == "fp64" and args.mixed_only:
                continue
            r = run_md(system, tol, prec, args.steps, args.warmup,
                       pin=None if args.no_pin else PINNED_SWEEP.get((args.workload, dk)))
            rl = roofline(key, r["prof"], G, dk, r["shape"])
            attach_traffic(rl, key)
            attach_ceilings(rl, copy_gbps)
            one[name] = {"value": round(r["steps_per_s"], 4), "unit": "MD steps/s",
                         "cg_iterations_per_step": round(r["prof"][f"{dk}_iters"] / args.steps, 1),
                         "latency_ms": {"p50": round(float(np.percentile(r["lat_ms"], 50)), 3),
                                        "p99": round(float(np.percentile(r["lat_ms"], 99)), 3)},
                         "roofline": rl}
        line["one_iteration_sweep"] = one
        line["speedup_two_iteration_vs_sweep"] = round(value / one["mixed"]["value"], 3)
        log(f"bench: one-iteration sweep {one}")
    if not args.no_order4:
        # the same workload with the cubic B-spline assignment the paper names
        # (64 points per ion): smoother charge motion, far fewer iterations
        log("bench: order-4 assignment")
        o4 = {}
        for name, prec in (("mixed", maze.MAZE_MIXED), ("fp64", maze.MAZE_FP64)):
            r = run_md(system, tol, prec, args.steps, args.warmup, order=4, flags=cg_flags)
            key = "fp32_iters" if prec == maze.MAZE_MIXED else "fp64_iters"
            o4[name] = {"value": round(r["steps_per_s"], 4), "unit": "MD steps/s",
                        "cg_iterations_per_step": round(r["prof"][key] / args.steps, 1),
                        "latency_ms": {"p50": round(float(np.percentile(r["lat_ms"], 50)), 3),
                                       "p99": round(float(np.percentile(r["lat_ms"], 99)), 3)}}
        o4["speedup_mixed_vs_fp64"] = round(o4["mixed"]["value"] / o4["fp64"]["value"], 3)
        line["order4"] = o4
        log(f"bench: order4 {o4}")
    if not args.no_multigrid:
        # the same workload with the multigrid-preconditioned PLCG (FP64
        # outer CG; FP64 or FP32 V-cycle), for both assignment orders
        log("bench: multigrid preconditioner")
        mgl = {}
        for order in (2, 4):
            for name, prec in (("mixed", maze.MAZE_MIXED), ("fp64", maze.MAZE_FP64)):
                r = run_md(system, tol, prec, args.steps, args.warmup, order=order,
                           flags=maze.MAZE_FLAG_MULTIGRID)
                mgl[f"order{order}_{name}"] = {
                    "value": round(r["steps_per_s"], 4), "unit": "MD steps/s",
                    "latency_ms": {"p50": round(float(np.percentile(r["lat_ms"], 50)), 3),
                                   "p99": round(float(np.percentile(r["lat_ms"], 99)), 3)}}
        line["multigrid"] = mgl
        log(f"bench: multigrid {mgl}")
    if args.error_trajectory > 0:
        log(f"bench: mixed vs FP64 over {args.error_trajectory} steps")
        tr = run_md(system, tol, maze.MAZE_FP64, args.error_trajectory, 0, record_positions=True,
                    flags=cg_flags)
        line["mixed_error_trajectory"] = replay_errors(system, tr["traj"], tol,
                                                       args.error_trajectory, every=50,
                                                       flags=cg_flags)
        log(f"bench: trajectory errors {line['mixed_error_trajectory']}")
    if not args.no_c2 and args.workload != "nacl4096_g128":
        log("bench: nacl4096_g128 (FP64, tol 1e-9)")
        line["nacl4096_g128"] = bench_c2(args.steps, args.warmup, cg_flags, copy_gbps)
        log(f"bench: nacl4096_g128 {line['nacl4096_g128']['value']} MD steps/s")
    if not args.no_observables:
        log("bench: Langevin dynamics and observables")
        line["observables"] = bench_observables(system, tol, args.steps, args.warmup, cg_flags)
        log(f"bench: observables {line['observables']}")
    if not args.no_ensemble:
        log("bench: ensemble of 64 replicas")
        line["ensemble"] = bench_ensemble(max(3, args.steps // 3), 4, flags=cg_flags)
        log(f"bench: ensemble {line['ensemble']}")
    if not args.no_serving:
        log("bench: serving")
        line["serving"] = bench_serving(not args.serving_reduced, args.serving_rate,
                                        flags=cg_flags)
        log(f"bench: serving {line['serving']}")
        if args.serving_rounds:
            line["serving_rounds"] = bench_serving(not args.serving_reduced, args.serving_rate,
                                                   flags=cg_flags, continuous=False)
            log(f"bench: serving in rounds {line['serving_rounds']}")
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
