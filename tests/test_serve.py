"""Scheduling logic of the continuous-batching server, on the CPU.

A fake backend stands in for the device: it keeps a step counter per
session and advances a simulated clock by a cost that grows with the batch,
so admission by budget, parking, continuous batching and the latency
accounting can be checked exactly without a GPU.
"""
import pytest

from paper_2505_20418_amd.serve import Request, Server, SessionSpec


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-9)


class FakeBackend:
    def __init__(self, clock, sizes, step_cost=0.010, per_session=0.002):
        self.clock = clock
        self.sizes = sizes
        self.step_cost = step_cost
        self.per_session = per_session
        self.live = {}
        self.batches = []
        self.created = 0

    def bytes_needed(self, spec):
        return self.sizes[spec.seed]

    def create(self, spec):
        self.created += 1
        obj = {"sid": spec.seed, "steps": 0}
        self.live[id(obj)] = obj
        return obj

    def park(self, obj):
        del self.live[id(obj)]
        return {"steps": obj["steps"], "sid": obj["sid"]}

    def restore(self, spec, state):
        obj = {"sid": state["sid"], "steps": state["steps"]}
        self.live[id(obj)] = obj
        return obj

    def step(self, objs):
        self.batches.append([o["sid"] for o in objs])
        self.clock.t += self.step_cost + self.per_session * len(objs)
        for o in objs:
            o["steps"] += 1
        return [{"status": 0, "iters": 10} for _ in objs]

    def destroy(self, obj):
        self.live.pop(id(obj), None)


def make(n=4, sizes=None, budget=10**9, max_batch=64):
    clock = FakeClock()
    sizes = sizes or {i: 100 for i in range(n)}
    be = FakeBackend(clock, sizes)
    specs = [SessionSpec(n_cells=2, seed=i, mixed=False, tol=1e-9) for i in range(n)]
    return Server(be, specs, budget, max_batch=max_batch, clock=clock, sleep=clock.sleep), be, clock


def test_requests_arriving_during_a_round_join_the_next():
    srv, be, clock = make()
    reqs = [Request(0.0, 0), Request(0.0, 1), Request(0.005, 2), Request(0.006, 3)]
    rep = srv.serve(reqs)
    # the first scheduling round holds what arrived at t=0; the two later
    # arrivals form the second
    assert be.batches == [[0, 1], [2, 3]]
    assert rep["requests_completed"] == 4
    c = {x.session: x for x in srv.completions}
    assert c[0].done_s == pytest.approx(0.014)
    assert c[2].done_s == pytest.approx(0.014 + 0.014)
    assert c[2].latency_s == pytest.approx(0.028 - 0.005)
    assert c[0].service_s == pytest.approx(0.014)


def test_one_request_per_session_per_round_in_arrival_order():
    srv, be, clock = make(n=2)
    reqs = [Request(0.0, 0), Request(0.0, 0), Request(0.0, 1), Request(0.0, 0)]
    srv.serve(reqs)
    assert be.batches == [[0, 1], [0], [0]]
    assert [x.session for x in srv.completions] == [0, 1, 0, 0]
    assert srv.slots[0].steps == 3 and srv.slots[1].steps == 1


def test_budget_parks_least_recently_used_and_restores_state():
    sizes = {0: 60, 1: 60, 2: 60}
    srv, be, clock = make(n=3, sizes=sizes, budget=130)
    reqs = [Request(0.0, 0), Request(0.0, 1), Request(0.1, 2), Request(0.2, 0)]
    srv.serve(reqs)
    # two fit; session 2 parks the least recently used idle one, and session 0
    # comes back with its step count intact
    assert srv.peak_used <= 130
    assert srv.parked >= 1 and srv.restored >= 1
    assert srv.slots[0].steps == 2
    obj0 = srv.slots[0].obj if srv.slots[0].obj is not None else srv.slots[0].parked
    assert obj0["steps"] == 2


def test_max_batch_and_refusal():
    sizes = {0: 10, 1: 10, 2: 10, 3: 10**6}
    srv, be, clock = make(n=4, sizes=sizes, budget=1000, max_batch=2)
    reqs = [Request(0.0, i) for i in range(4)]
    rep = srv.serve(reqs)
    assert rep["requests_refused"] == 1            # session 3 can never fit
    assert all(len(b) <= 2 for b in be.batches)
    assert rep["requests_completed"] == 3


def test_prefill_stops_at_budget():
    sizes = {i: 40 for i in range(5)}
    srv, be, clock = make(n=5, sizes=sizes, budget=100)
    assert srv.prefill() == 2
    assert srv.used == 80


def make_mixed_sizes(policy, max_wait_s=0.25):
    clock = FakeClock()
    specs = [SessionSpec(n_cells=2, seed=0, mixed=True, tol=1e-6),
             SessionSpec(n_cells=16, seed=1, mixed=False, tol=1e-10),
             SessionSpec(n_cells=2, seed=2, mixed=True, tol=1e-6)]
    sizes = {0: 10, 1: 10, 2: 10}

    class CostBackend(FakeBackend):
        """A round lasts as long as its most expensive member."""
        def step(self, objs):
            self.batches.append([o["sid"] for o in objs])
            self.clock.t += max(0.001 if o["sid"] != 1 else 0.060 for o in objs)
            for o in objs:
                o["steps"] += 1
            return [{"status": 0, "iters": 10} for _ in objs]

    be = CostBackend(clock, sizes)
    srv = Server(be, specs, 10 ** 9, clock=clock, sleep=clock.sleep, policy=policy,
                 max_wait_s=max_wait_s)
    return srv, be


def test_cost_classes_keep_small_sessions_off_big_rounds():
    srv, be = make_mixed_sizes("cost_class")
    srv.serve([Request(0.0, 0), Request(0.0, 1), Request(0.0, 2)])
    # the two 32^3 sessions go first, in their own round; the 256^3 one after
    assert be.batches == [[0, 2], [1]]
    c = {x.session: x for x in srv.completions}
    assert c[0].latency_s == pytest.approx(0.001) and c[2].latency_s == pytest.approx(0.001)
    assert c[1].latency_s == pytest.approx(0.061)
    # the fifo policy puts all three in one 60 ms round
    srv2, be2 = make_mixed_sizes("fifo")
    srv2.serve([Request(0.0, 0), Request(0.0, 1), Request(0.0, 2)])
    assert be2.batches == [[0, 1, 2]]
    assert all(x.latency_s == pytest.approx(0.060) for x in srv2.completions)


def test_cost_classes_do_not_starve_the_expensive_class():
    """A steady stream of small requests would always win the cheapest-class
    rule; once the big request has waited max_wait_s its class goes next."""
    srv, be = make_mixed_sizes("cost_class", max_wait_s=0.01)
    reqs = [Request(0.0, 1)] + [Request(0.0005 * k, 0 if k % 2 else 2) for k in range(60)]
    srv.serve(reqs)
    big = [x for x in srv.completions if x.session == 1][0]
    assert big.latency_s <= 0.01 + 0.002 + 0.060 + 1e-9
    assert srv.report(1.0)["requests_completed"] == len(reqs)


# ---- steps in flight (continuous mode) ------------------------------------
class FakeContinuous:
    """A device that keeps steps in flight: each advance is one poll group of
    `group` seconds, and a step of session s finishes after units[s] groups."""
    continuous = True

    def __init__(self, clock, sizes, units, group=0.001):
        self.clock = clock
        self.sizes = sizes
        self.units = units
        self.group = group
        self.live = {}
        self.flight = {}
        self.ready = []
        self.adds = []
        self.max_flight = 0

    def bytes_needed(self, spec):
        return self.sizes[spec.seed]

    def create(self, spec):
        obj = {"sid": spec.seed, "steps": 0}
        self.live[id(obj)] = obj
        return obj

    def park(self, obj):
        assert obj["sid"] not in self.flight, "a session with a step in flight was parked"
        del self.live[id(obj)]
        return {"steps": obj["steps"], "sid": obj["sid"]}

    def restore(self, spec, state):
        obj = {"sid": state["sid"], "steps": state["steps"]}
        self.live[id(obj)] = obj
        return obj

    def destroy(self, obj):
        self.live.pop(id(obj), None)

    def open_batch(self, n):
        self.cap = n
        return self

    def add(self, batch, obj, tag):
        assert tag not in self.flight
        self.flight[tag] = [self.units[obj["sid"]], obj]
        self.adds.append((self.clock.t, tag, len(self.flight)))
        self.max_flight = max(self.max_flight, len(self.flight))
        assert len(self.flight) <= self.cap

    def advance(self, batch):
        self.clock.t += self.group
        for k in list(self.flight):
            self.flight[k][0] -= 1
            if self.flight[k][0] == 0:
                self.flight[k][1]["steps"] += 1
                self.ready.append(k)
                del self.flight[k]

    def take(self, batch):
        out = [(k, {"status": 0, "iters": 10}) for k in self.ready]
        self.ready = []
        return out

    def close_batch(self, batch):
        pass


def make_cont(n=3, units=None, sizes=None, budget=10**9, max_batch=64):
    clock = FakeClock()
    units = units or {i: 5 for i in range(n)}
    sizes = sizes or {i: 100 for i in range(n)}
    be = FakeContinuous(clock, sizes, units)
    specs = [SessionSpec(n_cells=2, seed=i, mixed=False, tol=1e-9) for i in range(n)]
    return Server(be, specs, budget, max_batch=max_batch, clock=clock, sleep=clock.sleep), be, clock


def test_cheap_step_joins_and_leaves_before_an_expensive_one():
    srv, be, clock = make_cont(n=2, units={0: 100, 1: 2})
    rep = srv.serve([Request(0.0, 0), Request(0.005, 1)])
    c = {x.session: x for x in srv.completions}
    # session 1 was added while session 0's step was in flight and finished
    # after its own two poll groups, long before session 0
    assert rep["mode"] == "continuous" and rep["mid_flight_joins"] == 1
    assert be.adds[1][1] == 1 and be.adds[1][2] == 2
    assert c[1].done_s == pytest.approx(0.007)
    assert c[1].service_s == pytest.approx(0.002)
    assert c[0].done_s == pytest.approx(0.100)
    assert c[1].done_s < c[0].done_s


def test_one_step_per_session_in_flight():
    srv, be, clock = make_cont(n=1, units={0: 3})
    rep = srv.serve([Request(0.0, 0), Request(0.0, 0), Request(0.0, 0)])
    assert rep["requests_completed"] == 3
    assert [a[2] for a in be.adds] == [1, 1, 1]
    done = sorted(x.done_s for x in srv.completions)
    assert done == pytest.approx([0.003, 0.006, 0.009])
    # latency counts from arrival, service from the step's start
    assert sorted(x.latency_s for x in srv.completions) == pytest.approx([0.003, 0.006, 0.009])
    assert all(x.service_s == pytest.approx(0.003) for x in srv.completions)


def test_in_flight_cap_and_order():
    srv, be, clock = make_cont(n=5, units={i: 4 for i in range(5)}, max_batch=2)
    rep = srv.serve([Request(0.0, i) for i in range(5)])
    assert rep["requests_completed"] == 5
    assert be.max_flight == 2
    assert [a[1] for a in be.adds] == [0, 1, 2, 3, 4]


def test_parking_never_takes_a_session_in_flight():
    sizes = {0: 60, 1: 60, 2: 60}
    srv, be, clock = make_cont(n=3, units={0: 30, 1: 2, 2: 2}, sizes=sizes, budget=130)
    reqs = [Request(0.0, 0), Request(0.001, 1), Request(0.002, 2), Request(0.010, 1)]
    rep = srv.serve(reqs)
    assert rep["requests_completed"] == 4
    assert rep["parked"] >= 1 and rep["hbm_peak_used"] <= 130
    assert srv.slots[0].steps == 1 and srv.slots[1].steps == 2 and srv.slots[2].steps == 1
