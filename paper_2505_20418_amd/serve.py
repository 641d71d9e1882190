"""Continuous-batching service of MD-step requests over resident MaZe sessions.

Requests ask to advance one session by one MD step and arrive over time.
With a backend that keeps steps in flight (the GPU backend's default, the
library's maze_batch), scheduling works at CG-iteration granularity:

* a request whose session is resident (or can be admitted) and has no step
  in flight is added to the running batch at once: its step joins the
  batched CG launches already on the device at their next poll group, and
  leaves them when its solve ends, so a cheap step does not wait for an
  expensive one and arrivals overlap with the work in flight. At most
  ``max_batch`` steps are in flight, and at most one per session (a
  session's steps depend on each other);
* a session stays resident on the device between its steps, so its MaZe
  warm start (phi^k, phi^{k-1}, y*) and its particles persist;
* a session that is not resident is admitted when its device bytes fit in
  the HBM budget; otherwise resident sessions with no step in flight are
  parked least-recently-used first (their state copied to the host with the
  library's checkpoint and restored exactly on their next admission).

A backend without steps in flight is served in rounds, each one batched MD
step of the sessions it holds; requests that arrive while a round runs join
the next. With the default ``cost_class`` policy a round serves one class
of sessions of similar step cost (powers of four of N^4, doubled for FP64),
the cheapest with a waiting request unless one has waited longer than
``max_wait_s``; ``fifo`` takes every ready session, oldest first.

Per request the server records latency (completion minus arrival) and
service time (completion minus the moment its step started). The backend
does the device work; the GPU backend calls the library (maze_batch_* or
maze_md_step_batch). The clock and the sleep function are injectable so the
scheduling logic can be exercised with a simulated clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class SessionSpec:
    """One served MD session of synthetic molten NaCl."""
    n_cells: int
    seed: int
    mixed: bool
    tol: float
    temperature: float = 1200.0


@dataclasses.dataclass
class Request:
    arrival_s: float      # seconds after the start of the stream
    session: int


@dataclasses.dataclass
class Completion:
    session: int
    arrival_s: float
    done_s: float
    service_s: float
    batch_size: int
    status: int
    iters: int

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class GpuBackend:
    """Sessions as device-resident MD runs of the library (flags: MAZE_FLAG_*
    for every session, e.g. MAZE_FLAG_SSTEP for the two-iteration CG).
    continuous=True keeps steps in flight in a maze_batch; False serves
    rounds of maze_md_step_batch."""

    def __init__(self, device: str = "cuda", dt: float = 1.0, flags: int = 0,
                 continuous: bool = True):
        from . import inputs, maze, md  # noqa: F401  (fails loudly without the library)
        self.device = device
        self.dt = dt
        self.flags = flags
        self.continuous = bool(continuous)
        maze.lib()

    # ---- steps in flight (continuous mode) ----
    def open_batch(self, max_steps: int):
        from . import maze
        return maze.Batch(max_sessions=max_steps)

    def add(self, batch, run, tag: int):
        batch.add_md(run.session.handle, run.md, tag)

    def advance(self, batch):
        batch.advance()

    def take(self, batch):
        return batch.take()

    def close_batch(self, batch):
        batch.close()

    def _system(self, spec: SessionSpec):
        from . import inputs
        return inputs.molten_nacl(spec.n_cells, seed=spec.seed, temperature=spec.temperature)

    def bytes_needed(self, spec: SessionSpec) -> int:
        from . import inputs, maze
        s = self._system(spec)
        cfg = maze.maze_config(s.n_ions, 2, s.box, s.grid_spacing, spec.tol, 100000,
                               maze.MAZE_MIXED if spec.mixed else maze.MAZE_FP64, 0, self.flags,
                               inputs.COULOMB_K_EV_A, None)
        n = s.n_ions
        particles = 8 * (3 * 5 + 2) * n + 8 * (6 * n + 8 * ((n + 255) // 256) + 8) + 4 * n
        return int(maze.maze_device_bytes(cfg)) + particles

    def create(self, spec: SessionSpec):
        from . import maze, md
        return md.MDRun(self._system(spec), tol=spec.tol,
                        precision=maze.MAZE_MIXED if spec.mixed else maze.MAZE_FP64,
                        dt=self.dt, device=self.device, flags=self.flags)

    def park(self, run) -> dict:
        state = run.save_state()
        run.close()
        return state

    def restore(self, spec: SessionSpec, state: dict):
        from . import maze, md
        return md.MDRun(self._system(spec), tol=spec.tol,
                        precision=maze.MAZE_MIXED if spec.mixed else maze.MAZE_FP64,
                        dt=self.dt, device=self.device, restore=state, flags=self.flags)

    def step(self, runs: Sequence) -> List[dict]:
        from . import md
        _, stats = md.step_many(list(runs), want_stats=True)
        return stats

    def destroy(self, run):
        run.close()


@dataclasses.dataclass
class _Slot:
    spec: SessionSpec
    obj: object = None            # resident backend object
    parked: Optional[dict] = None  # host checkpoint while not resident
    nbytes: int = 0
    last_used: float = -1.0
    steps: int = 0


def step_cost(spec: SessionSpec) -> float:
    """Relative cost of one MD step of a session: grid points times CG
    iterations (which grow about as the grid side N), so N^4, doubled for
    FP64 vectors."""
    N = 16 * spec.n_cells
    return float(N) ** 4 * (1.0 if spec.mixed else 2.0)


def cost_class(spec: SessionSpec) -> int:
    """Sessions within a factor of four of estimated cost share a class."""
    return int(np.floor(np.log(step_cost(spec)) / np.log(4.0)))


class Server:
    """Continuous-batching scheduler over a backend (see module docstring)."""

    def __init__(self, backend, specs: Sequence[SessionSpec], hbm_budget: int,
                 max_batch: int = 64, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, policy: str = "cost_class",
                 max_wait_s: float = 0.25):
        if policy not in ("cost_class", "fifo"):
            raise ValueError(f"unknown policy {policy}")
        self.backend = backend
        self.slots = [_Slot(spec=s) for s in specs]
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.policy = policy
        self.max_wait_s = float(max_wait_s)
        self.klass = [cost_class(s) for s in specs]
        self.clock = clock
        self.sleep = sleep
        self.used = 0
        self.peak_used = 0
        self.admitted = 0
        self.parked = 0
        self.restored = 0
        self.refused: List[Request] = []
        self.completions: List[Completion] = []
        self.rounds: List[int] = []

    # ---- residency -----------------------------------------------------------
    def _bytes(self, sid: int) -> int:
        sl = self.slots[sid]
        if sl.nbytes == 0:
            sl.nbytes = int(self.backend.bytes_needed(sl.spec))
        return sl.nbytes

    def resident(self, sid: int) -> bool:
        return self.slots[sid].obj is not None

    def _evict_one(self, protect: set, queued: set) -> bool:
        cands = [i for i, s in enumerate(self.slots) if s.obj is not None and i not in protect]
        if not cands:
            return False
        # idle sessions (nothing queued) first, then least recently used
        cands.sort(key=lambda i: (i in queued, self.slots[i].last_used))
        victim = cands[0]
        sl = self.slots[victim]
        sl.parked = self.backend.park(sl.obj)
        sl.obj = None
        self.used -= sl.nbytes
        self.parked += 1
        return True

    def admit(self, sid: int, protect: set = frozenset(), queued: set = frozenset()) -> bool:
        """Makes session sid resident if the budget allows (parking others
        outside `protect` as needed). False if it cannot fit now."""
        if self.resident(sid):
            return True
        need = self._bytes(sid)
        if need > self.budget:
            return False
        while self.used + need > self.budget:
            if not self._evict_one(protect | {sid}, queued):
                return False
        sl = self.slots[sid]
        if sl.parked is not None:
            sl.obj = self.backend.restore(sl.spec, sl.parked)
            sl.parked = None
            self.restored += 1
        else:
            sl.obj = self.backend.create(sl.spec)
            self.admitted += 1
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return True

    def prefill(self, sids: Optional[Sequence[int]] = None) -> int:
        """Creates sessions up front while they fit in the budget; returns
        the number made resident."""
        n = 0
        for sid in (range(len(self.slots)) if sids is None else sids):
            if self.used + self._bytes(sid) > self.budget:
                break
            if self.admit(sid):
                n += 1
        return n

    # ---- serving loop ----------------------------------------------------------
    def serve(self, requests: Sequence[Request]) -> dict:
        if getattr(self.backend, "continuous", False):
            return self._serve_continuous(requests)
        return self._serve_rounds(requests)

    def _serve_continuous(self, requests: Sequence[Request]) -> dict:
        """Steps in flight: arrivals join the running batch at once (see the
        module docstring)."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        pending = collections.deque(reqs)
        queues: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        in_flight: Dict[int, tuple] = {}  # sid -> (request, start time, steps in flight at add)
        batch = self.backend.open_batch(self.max_batch)
        self.mid_flight_joins = 0
        t0 = self.clock()
        n_queued = 0
        try:
            while pending or n_queued or in_flight:
                now = self.clock() - t0
                while pending and pending[0].arrival_s <= now:
                    r = pending.popleft()
                    if self._bytes(r.session) > self.budget:
                        self.refused.append(r)
                        continue
                    queues[r.session].append(r)
                    n_queued += 1
                ready = sorted((q[0].arrival_s, sid) for sid, q in queues.items()
                               if q and sid not in in_flight)
                queued = {sid for sid, q in queues.items() if q}
                for _, sid in ready:
                    if len(in_flight) >= self.max_batch:
                        break
                    if not self.admit(sid, protect=set(in_flight), queued=queued):
                        continue
                    r = queues[sid].popleft()
                    n_queued -= 1
                    if in_flight:
                        self.mid_flight_joins += 1
                    t_add = self.clock() - t0
                    self.backend.add(batch, self.slots[sid].obj, sid)
                    in_flight[sid] = (r, t_add, len(in_flight) + 1)
                if not in_flight:
                    if n_queued:
                        raise RuntimeError("no queued session fits in the HBM budget with the "
                                           "resident sessions it cannot park")
                    if pending:
                        self.sleep(max(0.0, pending[0].arrival_s - (self.clock() - t0)))
                    continue
                self.rounds.append(len(in_flight))
                self.backend.advance(batch)
                for sid, st in self.backend.take(batch):
                    r, t_add, width = in_flight.pop(sid)
                    t_end = self.clock() - t0
                    sl = self.slots[sid]
                    sl.last_used = t_end
                    sl.steps += 1
                    self.completions.append(Completion(
                        session=sid, arrival_s=r.arrival_s, done_s=t_end,
                        service_s=t_end - t_add, batch_size=width,
                        status=int(st.get("status", 0)), iters=int(st.get("iters", 0))))
        finally:
            self.backend.close_batch(batch)
        rep = self.report(self.clock() - t0)
        rep["mode"] = "continuous"
        rep["mid_flight_joins"] = self.mid_flight_joins
        return rep

    def _serve_rounds(self, requests: Sequence[Request]) -> dict:
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        pending = collections.deque(reqs)
        queues: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        t0 = self.clock()
        n_queued = 0
        while pending or n_queued:
            now = self.clock() - t0
            while pending and pending[0].arrival_s <= now:
                r = pending.popleft()
                if self._bytes(r.session) > self.budget:
                    self.refused.append(r)
                    continue
                queues[r.session].append(r)
                n_queued += 1
            ready = sorted((q[0].arrival_s, sid) for sid, q in queues.items() if q)
            if not ready:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival_s - (self.clock() - t0)))
                continue
            queued = {sid for _, sid in ready}
            if self.policy == "cost_class":
                oldest_arrival, oldest = ready[0]
                if now - oldest_arrival > self.max_wait_s:
                    k = self.klass[oldest]
                else:
                    k = min(self.klass[sid] for _, sid in ready)
                ready = [(a, sid) for a, sid in ready if self.klass[sid] == k]
            batch: List[int] = []
            for _, sid in ready:
                if len(batch) >= self.max_batch:
                    break
                if self.admit(sid, protect=set(batch), queued=queued):
                    batch.append(sid)
            if not batch:
                raise RuntimeError("no queued session fits in the HBM budget with the "
                                   "resident sessions it cannot park")
            t_start = self.clock()
            stats = self.backend.step([self.slots[sid].obj for sid in batch])
            t_end = self.clock()
            self.rounds.append(len(batch))
            for sid, st in zip(batch, stats):
                r = queues[sid].popleft()
                n_queued -= 1
                sl = self.slots[sid]
                sl.last_used = t_end
                sl.steps += 1
                self.completions.append(Completion(
                    session=sid, arrival_s=r.arrival_s, done_s=t_end - t0,
                    service_s=t_end - t_start, batch_size=len(batch),
                    status=int(st.get("status", 0)), iters=int(st.get("iters", 0))))
        rep = self.report(self.clock() - t0)
        rep["mode"] = "rounds"
        return rep

    def report(self, wall_s: float) -> dict:
        lat = np.array([c.latency_s for c in self.completions]) * 1e3
        svc = np.array([c.service_s for c in self.completions]) * 1e3
        pct = lambda a, q: float(np.percentile(a, q)) if a.size else None  # noqa: E731
        return {
            "requests_completed": len(self.completions),
            "requests_refused": len(self.refused),
            "wall_s": wall_s,
            "steps_per_s": len(self.completions) / wall_s if wall_s > 0 else None,
            "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                           "mean": float(lat.mean()) if lat.size else None},
            "service_ms": {"p50": pct(svc, 50), "p99": pct(svc, 99)},
            "rounds": len(self.rounds),
            "mean_batch": float(np.mean(self.rounds)) if self.rounds else 0.0,
            "max_batch": int(max(self.rounds)) if self.rounds else 0,
            "admitted": self.admitted, "parked": self.parked, "restored": self.restored,
            "hbm_budget": self.budget, "hbm_peak_used": self.peak_used,
            "statuses": dict(collections.Counter(c.status for c in self.completions)),
        }

    def close(self):
        for sl in self.slots:
            if sl.obj is not None:
                self.backend.destroy(sl.obj)
                sl.obj = None
                self.used -= sl.nbytes


def specs_from_inputs(count: int = 256, seed: int = 5, max_cells: int = 16) -> List[SessionSpec]:
    """Session mix of the serving workload (sizes log-uniform over 64..32768
    ions, tolerance class 50/50: 1e-6 mixed or 1e-10 FP64)."""
    from . import inputs
    out = []
    for d in inputs.serving_sessions(count=count, seed=seed, max_cells=max_cells):
        out.append(SessionSpec(n_cells=d["n_cells"], seed=d["seed"], mixed=d["mixed"],
                               tol=d["tol"]))
    return out


def poisson_requests(n_requests: int, n_sessions: int, rate_hz: float = 200.0,
                     seed: int = 5) -> List[Request]:
    from . import inputs
    return [Request(r.arrival_s, r.session)
            for r in inputs.poisson_arrivals(n_requests, n_sessions, rate_hz=rate_hz, seed=seed)]
