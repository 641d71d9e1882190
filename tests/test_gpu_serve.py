"""Served MD steps through the continuous-batching server on the device.

Sessions of uneven size and both precisions are served from a Poisson
request stream under an HBM budget small enough to force parking and
restoring. Each session must end exactly where the same number of steps
taken alone leaves it: batching shares launches but not arithmetic, and the
checkpoint restores the warm-start history bit for bit.
"""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze
    maze.lib()


def test_served_sessions_equal_alone(gpu):
    from paper_2505_20418_amd import md, serve
    specs = [serve.SessionSpec(2, 11, False, 1e-10), serve.SessionSpec(3, 12, True, 1e-6),
             serve.SessionSpec(4, 13, False, 1e-10), serve.SessionSpec(2, 14, True, 1e-6),
             serve.SessionSpec(3, 15, False, 1e-10)]
    be = serve.GpuBackend(continuous=False)
    sizes = [be.bytes_needed(s) for s in specs]
    budget = int(sum(sorted(sizes)[-3:]) * 1.01)     # at most ~3 resident at once
    # arrival-order batching: with this budget and stream it parks and
    # restores sessions (the cost-class order is tested below)
    srv = serve.Server(be, specs, budget, max_batch=4, policy="fifo")
    reqs = serve.poisson_requests(24, len(specs), rate_hz=400.0, seed=3)
    print(f"case: serve {len(specs)} sessions, {len(reqs)} requests, budget {budget}", flush=True)
    rep = srv.serve(reqs)
    assert rep["requests_completed"] == len(reqs)
    assert rep["parked"] >= 1 and rep["restored"] >= 1, rep
    assert rep["hbm_peak_used"] <= budget
    assert set(rep["statuses"]) <= {0}
    for sid, spec in enumerate(specs):
        sl = srv.slots[sid]
        if sl.steps == 0:
            continue
        run = sl.obj if sl.obj is not None else be.restore(spec, sl.parked)
        alone = be.create(spec)
        for _ in range(sl.steps):
            alone.step()
        assert torch.equal(run.pos, alone.pos), sid
        assert torch.equal(run.vel, alone.vel), sid
        assert torch.equal(run.scalars, alone.scalars), sid
        alone.close()
        if sl.obj is None:
            run.close()
    srv.close()


def test_cost_class_served_sessions_equal_alone(gpu):
    """Rounds of one cost class at a time: each session still ends exactly
    where the same number of steps alone leaves it."""
    from paper_2505_20418_amd import serve
    specs = [serve.SessionSpec(2, 21, True, 1e-6), serve.SessionSpec(4, 22, False, 1e-10),
             serve.SessionSpec(2, 23, False, 1e-10), serve.SessionSpec(3, 24, True, 1e-6)]
    be = serve.GpuBackend(continuous=False)
    srv = serve.Server(be, specs, 1 << 34, max_batch=8)
    reqs = serve.poisson_requests(30, len(specs), rate_hz=500.0, seed=4)
    print(f"case: cost-class serve {len(specs)} sessions, {len(reqs)} requests", flush=True)
    rep = srv.serve(reqs)
    assert rep["requests_completed"] == len(reqs)
    assert set(rep["statuses"]) <= {0}
    for sid, spec in enumerate(specs):
        sl = srv.slots[sid]
        if sl.steps == 0:
            continue
        alone = be.create(spec)
        for _ in range(sl.steps):
            alone.step()
        assert torch.equal(sl.obj.pos, alone.pos), sid
        assert torch.equal(sl.obj.vel, alone.vel), sid
        alone.close()
    srv.close()


def test_continuous_served_sessions_equal_alone(gpu):
    """Steps in flight (maze_batch): arrivals join the running batch, and
    sessions are parked and restored under a tight budget; each session
    still ends exactly where the same number of steps alone leaves it."""
    from paper_2505_20418_amd import serve
    specs = [serve.SessionSpec(2, 31, False, 1e-10), serve.SessionSpec(3, 32, True, 1e-6),
             serve.SessionSpec(4, 33, False, 1e-10), serve.SessionSpec(2, 34, True, 1e-6),
             serve.SessionSpec(3, 35, False, 1e-10)]
    be = serve.GpuBackend()
    assert be.continuous
    sizes = [be.bytes_needed(s) for s in specs]
    budget = int(sum(sorted(sizes)[-3:]) * 1.01)
    srv = serve.Server(be, specs, budget, max_batch=4)
    reqs = serve.poisson_requests(30, len(specs), rate_hz=800.0, seed=6)
    print(f"case: continuous serve {len(specs)} sessions, {len(reqs)} requests", flush=True)
    rep = srv.serve(reqs)
    assert rep["mode"] == "continuous"
    assert rep["requests_completed"] == len(reqs)
    assert rep["mid_flight_joins"] >= 1, rep
    assert rep["parked"] >= 1 and rep["restored"] >= 1, rep
    assert rep["hbm_peak_used"] <= budget
    assert set(rep["statuses"]) <= {0}
    for sid, spec in enumerate(specs):
        sl = srv.slots[sid]
        if sl.steps == 0:
            continue
        run = sl.obj if sl.obj is not None else be.restore(spec, sl.parked)
        alone = be.create(spec)
        for _ in range(sl.steps):
            alone.step()
        assert torch.equal(run.pos, alone.pos), sid
        assert torch.equal(run.vel, alone.vel), sid
        assert torch.equal(run.scalars, alone.scalars), sid
        alone.close()
        if sl.obj is None:
            run.close()
    srv.close()


def test_continuous_serving_large_sessions_all_converge(gpu):
    """Sessions of 64^3 to 192^3 (throughput-mode batched kernels, many
    workgroups per session) served with steps in flight: every step
    converges and every session's positions stay finite. A solve's leader
    sets its done flag while other workgroups of the same launch start, so
    every workgroup must take one decision for all its threads: a workgroup
    split by that flag once wrote a finished solve's vectors from partial
    Gram sums."""
    from paper_2505_20418_amd import serve
    specs = [serve.SessionSpec(4 + 2 * (i % 5), 900 + i, i % 2 == 0, 1e-6 if i % 2 == 0 else 1e-10)
             for i in range(20)]
    be = serve.GpuBackend()
    srv = serve.Server(be, specs, 64 << 30, max_batch=32)
    srv.prefill()
    reqs = serve.poisson_requests(300, len(specs), rate_hz=2000.0, seed=7)
    print(f"case: continuous serve {len(specs)} sessions up to 192^3, {len(reqs)} requests",
          flush=True)
    rep = srv.serve(reqs)
    assert rep["requests_completed"] == len(reqs)
    assert set(rep["statuses"]) <= {0}, rep["statuses"]
    for sl in srv.slots:
        if sl.obj is not None:
            assert torch.isfinite(sl.obj.pos).all()
    srv.close()
