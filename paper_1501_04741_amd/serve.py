"""Continuous-batching server for design evaluations (w -> J, dJ/dw).

Requests of different lattice sizes arrive over time.  The scheduler:

* admits queued requests, oldest first, while the sum of their workspace
  footprints (lattice, checkpoints, ring, adjoint states) fits the HBM budget;
  a request that alone exceeds the budget is rejected;
* keeps every admitted request's context resident on the device until its
  gradient is ready;
* on each tick advances, per lattice kind (flow, scalar, precision), all
  requests in their primal phase by one quantum of steps with ONE batched
  launch per step, then all requests in their adjoint phase likewise (the
  adjoint call seeds newcomers and recomputes trajectory segments as needed);
* finishes requests whose adjoint reached t = 0 (objective and gradient are
  read back after a stream event), frees their memory and admits more.

Requests that arrive while others run join at the next tick: their steps
share launches with the running ones.  Each request's arithmetic is the same
device code as a one-request run, so results do not depend on the mix.

The scheduler talks to an executor.  ``GpuExecutor`` uses the library's
batched C ABI; ``FakeExecutor`` runs on the CPU (for scheduler tests).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, Dict, List, Optional

import numpy as np

QUEUED, PRIMAL, ADJOINT, FINISHING, DONE, FAILED = "queued", "primal", "adjoint", "finishing", "done", "failed"


@dataclasses.dataclass
class Job:
    rid: int
    params: dict
    steps: int
    design: Any                  # numpy array or tensor, flat, N values
    precision: str = "fp32"
    arrival: float = 0.0         # seconds on the server clock
    state: str = QUEUED
    footprint: int = 0
    handle: Any = None
    t: int = 0                   # primal steps done
    t_adj: int = 0               # adjoint steps remaining
    token: Any = None
    admitted: float = math.nan
    finished: float = math.nan
    J: float = math.nan
    grad: Any = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Executor:
    """What the scheduler needs from a device back end."""

    max_batch = 32

    def footprint(self, job: Job) -> int: ...
    def kind(self, job: Job): ...
    def open(self, job: Job) -> Any: ...
    def primal(self, handles: List[Any], k: int) -> None: ...
    def adjoint(self, handles: List[Any], k: int) -> None: ...
    def finish(self, handle) -> Any: ...            # enqueue readback, return a token
    def ready(self, token) -> bool: ...
    def result(self, handle, token): ...            # (J, grad)
    def close(self, handle) -> None: ...
    def mark(self) -> Any: ...                      # a point in the device work queue
    def wait(self, mark) -> None: ...


class Server:
    def __init__(self, executor: Executor, hbm_budget_bytes: int, quantum: int = 50,
                 clock: Callable[[], float] = time.perf_counter, max_inflight_ticks: int = 2):
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.quantum = int(quantum)
        self.clock = clock
        self.t0 = clock()
        self.queue: collections.deque = collections.deque()
        self.active: List[Job] = []
        self.finished: List[Job] = []
        self.used = 0
        self.max_inflight = max_inflight_ticks
        self.marks: collections.deque = collections.deque()
        self.stats = collections.Counter()

    def now(self) -> float:
        return self.clock() - self.t0

    # --------------------------------------------------------------- intake
    def submit(self, job: Job) -> Job:
        job.footprint = self.ex.footprint(job)
        if job.footprint > self.budget:
            job.state = FAILED
            job.error = "footprint %d B exceeds the budget %d B" % (job.footprint, self.budget)
            job.finished = job.arrival
            self.finished.append(job)
            self.stats["rejected"] += 1
            return job
        self.queue.append(job)
        self.stats["submitted"] += 1
        return job

    def _admit(self):
        while self.queue and self.used + self.queue[0].footprint <= self.budget:
            job = self.queue.popleft()
            try:
                job.handle = self.ex.open(job)
            except Exception as e:  # allocation or validation failure: fail this request only
                job.state = FAILED
                job.error = "open: %s" % e
                job.finished = self.now()
                self.finished.append(job)
                self.stats["failed"] += 1
                continue
            self.used += job.footprint
            job.state = PRIMAL
            job.t = 0
            job.admitted = self.now()
            self.active.append(job)
            self.stats["admitted"] += 1

    # ----------------------------------------------------------------- tick
    def _groups(self, state):
        groups: Dict[Any, List[Job]] = collections.OrderedDict()
        for j in self.active:
            if j.state == state:
                groups.setdefault(self.ex.kind(j), []).append(j)
        for key, jobs in groups.items():
            for i in range(0, len(jobs), self.ex.max_batch):
                yield jobs[i:i + self.ex.max_batch]

    def tick(self) -> bool:
        """One scheduling round; returns True if any device work was issued."""
        self._poll()
        self._admit()
        issued = False
        for jobs in self._groups(PRIMAL):
            k = min(self.quantum, min(j.steps - j.t for j in jobs))
            if k > 0:
                self.ex.primal([j.handle for j in jobs], k)
                issued = True
                self.stats["primal_launch_steps"] += k
            for j in jobs:
                j.t += k
                if j.t >= j.steps:
                    j.state = ADJOINT
                    j.t_adj = j.steps
        for jobs in self._groups(ADJOINT):
            k = min(self.quantum, min(j.t_adj for j in jobs))
            self.ex.adjoint([j.handle for j in jobs], k)
            issued = True
            self.stats["adjoint_launch_steps"] += k
            for j in jobs:
                j.t_adj -= k
                if j.t_adj == 0:
                    j.token = self.ex.finish(j.handle)
                    j.state = FINISHING
        if issued:
            self.marks.append(self.ex.mark())
            while len(self.marks) > self.max_inflight:
                self.ex.wait(self.marks.popleft())
        return issued

    def _poll(self):
        still = []
        for j in self.active:
            if j.state == FINISHING and self.ex.ready(j.token):
                try:
                    J, grad = self.ex.result(j.handle, j.token)
                    if not np.isfinite(J):
                        raise FloatingPointError("objective is not finite")
                    if grad is not None and not np.all(np.isfinite(grad)):
                        raise FloatingPointError("gradient is not finite")
                    j.J, j.grad, j.state = J, grad, DONE
                    self.stats["done"] += 1
                except Exception as e:
                    j.state, j.error = FAILED, str(e)
                    self.stats["failed"] += 1
                j.finished = self.now()
                self.ex.close(j.handle)
                j.handle = None
                self.used -= j.footprint
                self.finished.append(j)
            else:
                still.append(j)
        self.active = still

    def idle(self) -> bool:
        return not self.queue and not self.active

    def drain(self, max_ticks: int = 10 ** 9):
        n = 0
        while not self.idle() and n < max_ticks:
            if not self.tick() and self.active:
                # only finishing work left: wait for the device
                if self.marks:
                    self.ex.wait(self.marks.popleft())
                else:
                    time.sleep(1e-4)
            n += 1

    # ------------------------------------------------------------ replay
    def replay(self, jobs: List[Job], realtime: bool = True):
        """Submit jobs at their arrival times (server clock) and run to completion."""
        pending = sorted(jobs, key=lambda j: j.arrival)
        i = 0
        self.t0 = self.clock()
        while i < len(pending) or not self.idle():
            now = self.now()
            while i < len(pending) and (pending[i].arrival <= now or not realtime):
                self.submit(pending[i])
                i += 1
            issued = self.tick()
            if not issued:
                if self.active and self.marks:
                    self.ex.wait(self.marks.popleft())
                elif i < len(pending) and realtime:
                    time.sleep(max(0.0, min(1e-3, pending[i].arrival - self.now())))
        return self.finished


def summarize(jobs: List[Job], t_first_arrival: float = 0.0) -> dict:
    done = [j for j in jobs if j.state == DONE]
    lat = np.array([j.latency for j in done]) * 1e3
    if not done:
        return {"completed": 0, "failed": len(jobs)}
    span = max(j.finished for j in done) - min(t_first_arrival, min(j.arrival for j in done))
    return {
        "completed": len(done),
        "failed": sum(1 for j in jobs if j.state == FAILED),
        "gradients_per_s": len(done) / span if span > 0 else float("inf"),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "span_s": span,
    }


# ------------------------------------------------------------------ GPU
class GpuExecutor(Executor):
    """Device back end: one library context per request, batched launches."""

    max_batch = 32

    def __init__(self, device=None, per_request_cap_bytes: int = 4 << 30):
        import torch

        from . import lbm as _lbm
        self.torch = torch
        self.lbm = _lbm
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = torch.cuda.current_stream(self.device)
        self.cap = int(per_request_cap_bytes)

    def _plan_bytes(self, job: Job) -> int:
        """Workspace for the request: store-all (no recompute) when it fits the
        per-request cap, otherwise the largest checkpoint interval that fits,
        never less than the sqrt(N) plan."""
        L = self.lbm
        sqrt_b = L.lbm_required_bytes(L.make_config(job.params, job.steps, job.precision))
        all_b = L.lbm_required_bytes(L.make_config(job.params, job.steps, job.precision,
                                                   checkpoint_interval=max(job.steps, 1)))
        return max(sqrt_b, min(all_b, self.cap))

    def footprint(self, job: Job) -> int:
        job._budget = self._plan_bytes(job)
        L = self.lbm
        return L.lbm_required_bytes(L.make_config(job.params, job.steps, job.precision,
                                                  hbm_budget_bytes=job._budget))

    def kind(self, job: Job):
        p = job.params
        return (p["flow"], p.get("scalar", 0), job.precision)

    def open(self, job: Job):
        L = self.lbm.Lbm(job.params, nsteps=job.steps, precision=job.precision, hbm_budget_bytes=job._budget,
                         device=self.device, stream=self.stream)
        L.set_design(job.design)
        L.reset()
        L._J = self.torch.empty(1, dtype=self.torch.float64, device=self.device)
        return L

    def primal(self, handles, k):
        self.lbm.lbm_primal_steps_batch([h.ctx for h in handles], k, record=True)
        for h in handles:
            t, rec, _ = h.times()
            if rec == h.nsteps:
                self.lbm.lbm_objective_async(h.ctx, h._J)

    def adjoint(self, handles, k):
        self.lbm.lbm_adjoint_steps_batch([h.ctx for h in handles], k)

    def finish(self, handle):
        g = handle.gradient()
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        handle._grad = g
        return ev

    def ready(self, token) -> bool:
        return token.query()

    def result(self, handle, token):
        token.synchronize()
        return float(handle._J.item()), handle._grad.detach().cpu().numpy()

    def close(self, handle):
        handle.close()

    def mark(self):
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, mark):
        mark.synchronize()


def run_one_at_a_time(jobs: List[Job], device=None, clock=time.perf_counter):
    """Baseline: the same trace on the same GPU, one request at a time in
    arrival order (FIFO), no overlap: each request is created, runs its full
    primal, objective, adjoint and gradient with single-context launches,
    and is read back before the next one starts."""
    import torch

    from .lbm import Lbm
    ex = GpuExecutor(device)
    t0 = clock()
    out = []
    for job in sorted(jobs, key=lambda j: j.arrival):
        while clock() - t0 < job.arrival:
            time.sleep(min(1e-3, job.arrival - (clock() - t0)))
        budget = ex._plan_bytes(job)
        L = Lbm(job.params, nsteps=job.steps, precision=job.precision, hbm_budget_bytes=budget, device=ex.device)
        J, g = L.value_and_grad(job.design)
        job.J = J
        job.grad = g.cpu().numpy()
        torch.cuda.synchronize()
        job.finished = clock() - t0
        job.state = DONE if np.isfinite(J) else FAILED
        L.close()
        out.append(job)
    return out


# ------------------------------------------------------------------ CPU
class FakeExecutor(Executor):
    """CPU back end for scheduler tests.  Each request is evaluated by a
    supplied function (e.g. the FP64 oracle on a tiny lattice) when its
    adjoint completes; device time is simulated as proportional to
    nodes x steps so that ordering and latency accounting can be checked."""

    def __init__(self, evaluate: Callable[[Job], Any], bytes_per_node_step: int = 64, max_batch: int = 32,
                 seconds_per_node_step: float = 0.0, fail_on_open: Optional[set] = None):
        self.evaluate = evaluate
        self.bpn = bytes_per_node_step
        self.max_batch = max_batch
        self.sec = seconds_per_node_step
        self.fail_on_open = fail_on_open or set()
        self.log: List[tuple] = []
        self.open_handles = 0

    def footprint(self, job):
        p = job.params
        n = p["nx"] * p["ny"] * p["nz"]
        return n * self.bpn * (int(math.isqrt(max(job.steps, 1))) + 4)

    def kind(self, job):
        return (job.params["flow"], job.params.get("scalar", 0), job.precision)

    def open(self, job):
        if job.rid in self.fail_on_open:
            raise MemoryError("simulated allocation failure")
        self.open_handles += 1
        return {"job": job, "primal": 0, "adjoint": 0}

    def _cost(self, handles, k):
        if self.sec:
            time.sleep(self.sec * k * sum(h["job"].params["nx"] * h["job"].params["ny"] * h["job"].params["nz"]
                                          for h in handles))

    def primal(self, handles, k):
        assert len(handles) <= self.max_batch
        assert len({self.kind(h["job"]) for h in handles}) == 1
        self.log.append(("primal", tuple(h["job"].rid for h in handles), k))
        for h in handles:
            h["primal"] += k
        self._cost(handles, k)

    def adjoint(self, handles, k):
        assert len({self.kind(h["job"]) for h in handles}) == 1
        self.log.append(("adjoint", tuple(h["job"].rid for h in handles), k))
        for h in handles:
            assert h["primal"] == h["job"].steps
            h["adjoint"] += k
        self._cost(handles, k)

    def finish(self, handle):
        assert handle["adjoint"] == handle["job"].steps
        return self.evaluate(handle["job"])

    def ready(self, token):
        return True

    def result(self, handle, token):
        return token

    def close(self, handle):
        self.open_handles -= 1

    def mark(self):
        return None

    def wait(self, mark):
        pass
