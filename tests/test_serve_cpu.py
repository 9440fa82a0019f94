"""Scheduler of the serving loop, on the CPU with a fake executor whose results
come from the FP64 oracle (tiny lattices)."""
import math

import numpy as np
import pytest

import oracle
from paper_1501_04741_amd import inputs
from paper_1501_04741_amd.serve import DONE, FAILED, FakeExecutor, Job, Server, summarize


def _oracle_eval(job):
    w = np.asarray(job.design, dtype=np.float64)
    r = oracle.adjoint(job.params, w, job.steps)
    return r["J"], r["grad"]


def _job(rid, nx, ny, nz=1, flow=9, steps=12, arrival=0.0, design=None, **kw):
    p = dict(flow=flow, scalar=0, nx=nx, ny=ny, nz=nz, tau=0.8, u_in=0.02, switch_fn="ramp", switch_param=0.01,
             c_dp=1.0)
    p.update(kw)
    w = inputs.porosity(nx, ny, nz, rid, 3) if design is None else design
    return Job(rid=rid, params=p, steps=steps, design=w, precision="fp64", arrival=arrival)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def test_every_request_gets_its_own_result():
    ex = FakeExecutor(_oracle_eval)
    srv = Server(ex, hbm_budget_bytes=10 ** 9, quantum=5)
    jobs = [_job(0, 16, 8), _job(1, 20, 6), _job(2, 8, 6, 5, flow=19), _job(3, 12, 10)]
    for j in jobs:
        srv.submit(j)
    srv.drain()
    assert all(j.state == DONE for j in jobs)
    for j in jobs:
        J, g = _oracle_eval(j)
        assert j.J == J and np.array_equal(j.grad, g)
    assert ex.open_handles == 0 and srv.used == 0


def test_batches_never_mix_kinds_and_respect_max_batch():
    ex = FakeExecutor(lambda j: (1.0, None), max_batch=2)
    srv = Server(ex, hbm_budget_bytes=10 ** 9, quantum=4)
    jobs = [_job(i, 16, 8) for i in range(5)] + [_job(10 + i, 8, 6, 5, flow=19) for i in range(3)]
    for j in jobs:
        srv.submit(j)
    srv.drain()
    assert all(j.state == DONE for j in jobs)
    assert max(len(rids) for _, rids, _ in ex.log) == 2          # FakeExecutor asserts one kind per launch
    d2 = {j.rid for j in jobs if j.params["flow"] == 9}
    for _, rids, _ in ex.log:
        assert set(rids) <= d2 or not (set(rids) & d2)


def test_admission_by_footprint():
    ex = FakeExecutor(lambda j: (1.0, None))
    one = ex.footprint(_job(0, 32, 32))
    srv = Server(ex, hbm_budget_bytes=int(2.5 * one), quantum=3)
    jobs = [_job(i, 32, 32) for i in range(6)]
    for j in jobs:
        srv.submit(j)
    concurrent = []
    while not srv.idle():
        srv.tick()
        concurrent.append(sum(1 for j in srv.active))
        assert srv.used <= srv.budget
    assert max(concurrent) == 2
    assert all(j.state == DONE for j in jobs)
    # FIFO admission: admission times are non-decreasing in submission order
    adm = [j.admitted for j in jobs]
    assert adm == sorted(adm)


def test_oversized_request_is_rejected_alone():
    ex = FakeExecutor(lambda j: (1.0, None))
    small = ex.footprint(_job(0, 16, 8))
    srv = Server(ex, hbm_budget_bytes=4 * small, quantum=5)
    big = _job(1, 256, 256)
    ok = _job(2, 16, 8)
    srv.submit(big)
    srv.submit(ok)
    srv.drain()
    assert big.state == FAILED and "exceeds the budget" in big.error
    assert ok.state == DONE


def test_failures_are_isolated():
    def ev(job):
        if job.rid == 1:
            return float("nan"), None
        return _oracle_eval(job)
    ex = FakeExecutor(ev, fail_on_open={2})
    srv = Server(ex, hbm_budget_bytes=10 ** 9, quantum=5)
    jobs = [_job(0, 16, 8), _job(1, 16, 8), _job(2, 16, 8), _job(3, 16, 8)]
    for j in jobs:
        srv.submit(j)
    srv.drain()
    assert jobs[1].state == FAILED and "not finite" in jobs[1].error
    assert jobs[2].state == FAILED and "open" in jobs[2].error
    for j in (jobs[0], jobs[3]):
        J, g = _oracle_eval(j)
        assert j.state == DONE and j.J == J and np.array_equal(j.grad, g)
    assert ex.open_handles == 0 and srv.used == 0


def test_late_arrivals_join_running_batches():
    """Continuous batching: a request submitted while another is mid-primal
    shares launches with it from the next tick on."""
    ex = FakeExecutor(lambda j: (1.0, None))
    clock = FakeClock()
    srv = Server(ex, hbm_budget_bytes=10 ** 9, quantum=4, clock=clock)
    a = _job(0, 16, 8, steps=40)
    b = _job(1, 16, 8, steps=40)
    srv.submit(a)
    srv.tick()
    srv.tick()
    assert a.t == 8
    srv.submit(b)
    srv.tick()
    shared = [rids for kind, rids, _ in ex.log if kind == "primal" and set(rids) == {0, 1}]
    assert shared, ex.log
    srv.drain()
    assert a.state == DONE and b.state == DONE


def test_latency_accounting_with_fake_clock():
    ex = FakeExecutor(lambda j: (2.0, None))
    clock = FakeClock()
    srv = Server(ex, hbm_budget_bytes=10 ** 9, quantum=10, clock=clock)
    jobs = [_job(i, 16, 8, steps=20, arrival=0.5 * i) for i in range(4)]
    pending = list(jobs)
    while pending or not srv.idle():
        while pending and pending[0].arrival <= clock.t:
            srv.submit(pending.pop(0))
        srv.tick()
        clock.t += 0.25
    for j in jobs:
        assert j.finished >= j.arrival and math.isfinite(j.latency)
    s = summarize(jobs)
    assert s["completed"] == 4 and s["p99_ms"] >= s["p50_ms"] > 0


def test_replay_submits_in_arrival_order():
    ex = FakeExecutor(lambda j: (1.0, None))
    srv = Server(ex, hbm_budget_bytes=10 ** 9, quantum=8)
    trace = inputs.poisson_trace(12, rate_per_s=1000.0, seed=1, steps=16)
    jobs = []
    for r in trace:
        p = dict(r.params, nx=16, ny=8, nz=1 if r.params["flow"] == 9 else 6)
        jobs.append(Job(rid=r.rid, params=p, steps=r.steps, design=inputs.porosity(p["nx"], p["ny"], p["nz"], r.seed, 3),
                        arrival=r.arrival_s, precision="fp64"))
    done = srv.replay(jobs, realtime=False)
    assert len(done) == 12 and all(j.state == DONE for j in done)
    arr = [r.arrival_s for r in trace]
    assert arr == sorted(arr) and arr[0] == 0.0


def test_sjf_admits_short_requests_first_and_fifo_keeps_order():
    ex = FakeExecutor(lambda j: (1.0, None), seconds_per_node_step=1e-9)
    big = _job(0, 64, 64, steps=20)
    small = [_job(i, 16, 8, steps=20) for i in (1, 2)]
    budget = ex.footprint(big)
    for policy in ("sjf", "fifo"):
        srv = Server(FakeExecutor(lambda j: (1.0, None), seconds_per_node_step=1e-9), hbm_budget_bytes=budget,
                     quantum=5, policy=policy, clock=FakeClock())
        jobs = [_job(0, 64, 64, steps=20)] + [_job(i, 16, 8, steps=20) for i in (1, 2)]
        for j in jobs:
            srv.submit(j)
        order = []
        while not srv.idle():
            srv.tick()
            for j in srv.finished:
                if j.rid not in order:
                    order.append(j.rid)
        if policy == "sjf":
            assert order.index(1) < order.index(0) and order.index(2) < order.index(0)
        else:
            assert order[0] == 0


def test_active_state_cap_and_aging():
    ex = FakeExecutor(lambda j: (1.0, None), seconds_per_node_step=1e-6)
    one = ex.step_bytes(_job(0, 32, 32))
    clock = FakeClock()
    srv = Server(ex, hbm_budget_bytes=10 ** 12, quantum=5, policy="sjf", max_active_state_bytes=2 * one,
                 aging=1.0, clock=clock)
    for i in range(5):
        srv.submit(_job(i, 32, 32, steps=20))
    while not srv.idle():
        srv.tick()
        assert srv.active_state <= 2 * one
        assert sum(1 for j in srv.active) <= 2
    # aging: an old large request overtakes newer short ones once it has waited longer
    # than the difference of their estimated times
    srv = Server(FakeExecutor(lambda j: (1.0, None), seconds_per_node_step=1e-6), hbm_budget_bytes=10 ** 12,
                 quantum=5, policy="sjf", max_active_state_bytes=1, clock=clock)
    clock.t = 0.0
    srv.t0 = 0.0
    big = _job(0, 64, 64, steps=20, arrival=0.0)     # estimate 64*64*20*1e-6 = 0.082 s
    srv.submit(big)
    clock.t = 1.0
    late = _job(1, 16, 8, steps=20, arrival=1.0)     # estimate 0.00256 s, waited 0
    srv.submit(late)
    assert srv._next() is big


def test_time_quantum_lets_small_requests_take_more_steps_per_tick():
    ex = FakeExecutor(lambda j: (1.0, None), seconds_per_node_step=1e-8)
    srv = Server(ex, hbm_budget_bytes=10 ** 12, quantum_ms=1.0)
    big = _job(0, 128, 128, steps=400)
    small = _job(1, 16, 8, steps=400)
    srv.submit(big)
    srv.submit(small)
    srv.tick()
    steps = {rids: k for kind, rids, k in ex.log if kind == "primal"}
    assert steps[(1,)] > steps[(0,)]           # separate cost classes, more steps for the small one
    srv.drain()
    assert small.finished <= big.finished


def test_deferred_admission_keeps_request_queued():
    from paper_1501_04741_amd.serve import DeferAdmission

    class Tight(FakeExecutor):
        def __init__(self):
            super().__init__(lambda j: (1.0, None))
            self.busy = False

        def open(self, job):
            if self.busy:
                raise DeferAdmission("device memory")
            self.busy = True
            return super().open(job)

        def close(self, handle):
            self.busy = False
            super().close(handle)

    ex = Tight()
    srv = Server(ex, hbm_budget_bytes=10 ** 12, quantum=5)
    jobs = [_job(i, 16, 8, steps=10) for i in range(3)]
    for j in jobs:
        srv.submit(j)
    srv.drain()
    assert all(j.state == DONE for j in jobs)
    assert srv.stats["deferred"] >= 2


def test_arena_first_fit_and_coalescing():
    import torch

    from paper_1501_04741_amd.serve import Arena
    a = Arena(10 * 256, "cpu")
    blocks = [a.alloc(256) for _ in range(10)]
    assert all(b is not None for b in blocks) and a.alloc(1) is None
    offs = [b[0] for b in blocks]
    assert offs == [256 * i for i in range(10)]
    for i in (1, 2, 5):
        a.release(offs[i], 256)
    assert a.free == [(256, 512), (1280, 256)]
    b = a.alloc(300)                       # rounds to 512, first fit at 256
    assert b[0] == 256 and b[1].numel() == 512
    a.release(256, 300)
    for i in (0, 3, 4, 6, 7, 8, 9):
        a.release(offs[i], 256)
    assert a.free == [(0, 2560)] and a.free_bytes() == 2560
    assert a.buf.dtype == torch.uint8


def test_cancel_queued_and_mid_flight_requests():
    """A queued request leaves the queue; admitted ones are closed at the next tick
    whether in their primal or adjoint phase; memory and handles return, and the
    other requests still get their own results."""
    from paper_1501_04741_amd.serve import ADJOINT, CANCELLED, PRIMAL
    ex = FakeExecutor(_oracle_eval)
    jobs = [_job(i, 16, 8, steps=20) for i in range(4)]
    srv = Server(ex, hbm_budget_bytes=2 * ex.footprint(jobs[0]), quantum=5, policy="fifo")
    for j in jobs:
        srv.submit(j)
    srv.tick()                        # jobs 0 and 1 admitted (budget holds two), 2 and 3 queued
    assert [j.state for j in jobs] == [PRIMAL, PRIMAL, "queued", "queued"]
    assert srv.cancel(3) and jobs[3].state == CANCELLED
    for _ in range(5):                # job 0 reaches its adjoint
        srv.tick()
    assert jobs[0].state == ADJOINT
    assert srv.cancel(0)              # mid-adjoint
    assert srv.cancel(99) is False
    srv.drain()
    assert jobs[0].state == CANCELLED and jobs[3].state == CANCELLED
    assert jobs[1].state == DONE and jobs[2].state == DONE
    for j in (jobs[1], jobs[2]):
        J, g = _oracle_eval(j)
        assert j.J == J and np.array_equal(j.grad, g)
    assert ex.open_handles == 0 and srv.used == 0 and srv.active_state == 0
    assert srv.stats["cancelled"] == 2
