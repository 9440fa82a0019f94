"""Continuous-batching server for design evaluations (w -> J, dJ/dw).

Requests of different lattice sizes arrive over time.  The scheduler:

* admits queued requests while the sum of their workspace footprints
  (lattice, checkpoints, ring, adjoint states) fits the HBM budget and the
  active set's per-step state bytes stay under a cap (enough parallel work to
  fill the GPU without time-slicing every large request at once); the next
  request is the one with the shortest estimated device time minus its
  waiting time ("sjf" with linear aging, so large requests cannot starve) or
  the oldest ("fifo"); a request that alone exceeds the budget is rejected;
* keeps every admitted request's context resident on the device until its
  gradient is ready;
* on each tick advances, per lattice kind (flow, scalar, precision) and
  per-step cost class (power-of-two state size), all requests in their
  primal phase by one quantum with ONE batched launch per step, then all
  requests in their adjoint phase likewise (the adjoint call seeds newcomers
  and recomputes trajectory segments as needed).  With a time quantum, each
  class advances by the number of steps that takes about that much device
  time, so small requests are not held to the pace of large ones;
* finishes requests whose adjoint reached t = 0 (objective and gradient are
  read back after a stream event), frees their memory and admits more;
* cancels a request on demand: a queued one leaves the queue, an admitted one
  (in its primal, adjoint or read-back phase) is closed at the next tick and
  its memory returns to the budget.  Every request's launches go to one
  stream, so work still queued for a cancelled request runs before any later
  request's work that reuses its memory.

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

QUEUED, PRIMAL, ADJOINT, FINISHING, DONE, FAILED, CANCELLED = (
    "queued", "primal", "adjoint", "finishing", "done", "failed", "cancelled")


class DeferAdmission(Exception):
    """Raised by an executor's open() when the request cannot be placed now
    (e.g. transient device-memory exhaustion); the request stays queued."""


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
    estimate: float = 0.0        # estimated device seconds
    step_bytes: int = 0          # state bytes the request adds to every step
    handle: Any = None
    t: int = 0                   # primal steps done
    t_adj: int = 0               # adjoint steps remaining
    token: Any = None
    admitted: float = math.nan
    finished: float = math.nan
    cancel_requested: bool = False
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
    def estimate(self, job: Job) -> float: ...      # device seconds for the whole evaluation
    def step_bytes(self, job: Job) -> int: ...      # bytes of one state of the request
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
                 clock: Callable[[], float] = time.perf_counter, max_inflight_ticks: int = 2,
                 policy: str = "sjf", max_active_state_bytes: Optional[int] = None, aging: float = 1.0,
                 quantum_ms: Optional[float] = None):
        if policy not in ("sjf", "fifo"):
            raise ValueError("policy must be 'sjf' or 'fifo'")
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.quantum = int(quantum)
        self.policy = policy
        self.max_active_state = max_active_state_bytes
        self.aging = float(aging)
        self.quantum_s = None if quantum_ms is None else float(quantum_ms) * 1e-3
        self.active_state = 0
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
        job.estimate = self.ex.estimate(job)
        job.step_bytes = self.ex.step_bytes(job)
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

    def _fits(self, job: Job) -> bool:
        if self.used + job.footprint > self.budget:
            return False
        if self.max_active_state is not None and self.active and \
                self.active_state + job.step_bytes > self.max_active_state:
            return False
        return True

    def _next(self) -> Optional[Job]:
        if not self.queue:
            return None
        if self.policy == "fifo":
            head = self.queue[0]
            return head if self._fits(head) else None
        now = self.now()
        for job in sorted(self.queue, key=lambda j: (j.estimate - self.aging * (now - j.arrival), j.arrival)):
            if self._fits(job):
                return job
        return None

    def _admit(self):
        while True:
            job = self._next()
            if job is None:
                return
            self.queue.remove(job)
            try:
                job.handle = self.ex.open(job)
            except DeferAdmission as e:
                if self.active:  # memory will come back when running requests finish
                    self.queue.appendleft(job)
                    self.stats["deferred"] += 1
                    return
                job.state = FAILED
                job.error = "open: %s" % e
                job.finished = self.now()
                self.finished.append(job)
                self.stats["failed"] += 1
                continue
            except Exception as e:  # allocation or validation failure: fail this request only
                job.state = FAILED
                job.error = "open: %s" % e
                job.finished = self.now()
                self.finished.append(job)
                self.stats["failed"] += 1
                continue
            self.used += job.footprint
            self.active_state += job.step_bytes
            job.state = PRIMAL
            job.t = 0
            job.admitted = self.now()
            self.active.append(job)
            self.stats["admitted"] += 1

    def cancel(self, rid: int) -> bool:
        """Cancel request rid: dropped from the queue now, or closed at the next
        tick if admitted.  Returns False if no such request is queued or active."""
        for j in list(self.queue):
            if j.rid == rid:
                self.queue.remove(j)
                j.state = CANCELLED
                j.finished = self.now()
                self.finished.append(j)
                self.stats["cancelled"] += 1
                return True
        for j in self.active:
            if j.rid == rid:
                j.cancel_requested = True
                return True
        return False

    def _reap_cancelled(self):
        still = []
        for j in self.active:
            if j.cancel_requested:
                self.ex.close(j.handle)
                j.handle = None
                j.token = None
                self.used -= j.footprint
                self.active_state -= j.step_bytes
                j.state = CANCELLED
                j.finished = self.now()
                self.finished.append(j)
                self.stats["cancelled"] += 1
            else:
                still.append(j)
        self.active = still

    # ----------------------------------------------------------------- tick
    def _groups(self, state):
        groups: Dict[Any, List[Job]] = collections.OrderedDict()
        for j in self.active:
            if j.state == state:
                cls = int(math.log2(max(j.step_bytes, 1))) if self.quantum_s is not None else 0
                groups.setdefault((self.ex.kind(j), cls), []).append(j)
        for key, jobs in groups.items():
            for i in range(0, len(jobs), self.ex.max_batch):
                yield jobs[i:i + self.ex.max_batch]

    def _steps(self, jobs: List[Job], remaining: int) -> int:
        if self.quantum_s is None:
            k = self.quantum
        else:
            per_step = max(j.estimate / (2.0 * max(j.steps, 1)) for j in jobs)  # primal or adjoint step
            k = max(1, int(self.quantum_s / max(per_step, 1e-9)))
        return min(k, remaining)

    def tick(self) -> bool:
        """One scheduling round; returns True if any device work was issued."""
        self._reap_cancelled()
        self._poll()
        self._admit()
        issued = False
        for jobs in self._groups(PRIMAL):
            k = self._steps(jobs, min(j.steps - j.t for j in jobs))
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
            k = self._steps(jobs, min(j.t_adj for j in jobs))
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
                self.active_state -= j.step_bytes
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
    errors = collections.Counter(j.error.split(":")[0] for j in jobs if j.state == FAILED)
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
        "failure_reasons": dict(errors),
    }


# ------------------------------------------------------------------ GPU
class Arena:
    """First-fit sub-allocator over one device buffer reserved up front
    (address-ordered free list, neighbours merged on release), so that serving
    makes no device allocation or free calls.  Blocks are 256-byte aligned."""

    ALIGN = 256

    def __init__(self, nbytes: int, device):
        import torch
        self.size = int(nbytes) // self.ALIGN * self.ALIGN
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]

    def _round(self, n):
        return (int(n) + self.ALIGN - 1) // self.ALIGN * self.ALIGN

    def alloc(self, nbytes: int):
        n = self._round(nbytes)
        for i, (off, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, sz - n)
                return off, self.buf[off:off + n]
        return None

    def release(self, off: int, nbytes: int):
        n = self._round(nbytes)
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, (off, n))
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            self.free[i] = (off, n + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def free_bytes(self) -> int:
        return sum(sz for _, sz in self.free)


class GpuExecutor(Executor):
    """Device back end: one library context per request, batched launches.

    Workspaces come from an ``Arena`` when ``arena_bytes`` is given (no device
    allocation while serving); designs are uploaded and results read back
    through pinned host buffers with asynchronous copies, so the host never
    waits for queued device work except when it chooses to (tick pacing)."""

    max_batch = 32

    def __init__(self, device=None, per_request_cap_bytes: int = 64 << 30, arena_bytes: Optional[int] = None,
                 inplace_min_state_bytes: Optional[int] = 32 << 20):
        """inplace_min_state_bytes: requests whose state is at least this large stream in
        place (one primal and one adjoint buffer instead of two each; the in-place
        kernels also move their bytes faster), the others use ping-pong buffers.
        Requests of one kind share batched launches either way (in-place and
        ping-pong requests are different kinds).  None: never in place.  On the
        400-request Poisson trace at 20/s: in place from 32 MB 14.2 gradients/s,
        p50 1.34 s, p99 9.4 s; every request in place 14.0 / 1.49 s / 9.5 s; none
        13.7 / 0.80 s / 10.0 s."""
        import torch

        from . import lbm as _lbm
        self.torch = torch
        self.lbm = _lbm
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = torch.cuda.current_stream(self.device)
        self.cap = int(per_request_cap_bytes)
        self.inplace_min = inplace_min_state_bytes
        self.arena = Arena(arena_bytes, self.device) if arena_bytes else None

    def _plan_bytes(self, job: Job) -> int:
        """Workspace budget for the request: store-all (every step's moments held, no
        recompute) when it fits the per-request cap, otherwise the largest
        checkpoint interval that fits, never less than the plan of a checkpoint
        every ~sqrt(N) steps (ping-pong: the smallest-workspace plan).  Sets
        job._store_all and job._inplace."""
        L = self.lbm
        ip = bool(self.inplace_min is not None and job.steps > 0 and self.step_bytes(job) >= self.inplace_min)
        cfg = lambda **kw: L.make_config(job.params, job.steps, job.precision, inplace=ip, **kw)
        all_b = L.lbm_required_bytes(cfg(checkpoint_interval=max(job.steps, 1)))
        job._store_all = all_b <= self.cap
        job._inplace = ip
        if ip:
            floor_b = L.lbm_required_bytes(cfg(checkpoint_interval=max(1, math.ceil(math.sqrt(job.steps)))))
        else:
            floor_b = L.lbm_required_bytes(cfg())
        return max(floor_b, min(all_b, self.cap))

    def footprint(self, job: Job) -> int:
        job._budget = self._plan_bytes(job)
        L = self.lbm
        return L.lbm_required_bytes(L.make_config(job.params, job.steps, job.precision,
                                                  hbm_budget_bytes=job._budget, inplace=job._inplace))

    def kind(self, job: Job):
        p = job.params
        return (p["flow"], p.get("scalar", 0), job.precision, bool(getattr(job, "_inplace", False)))

    def step_bytes(self, job: Job) -> int:
        p = job.params
        s = 4 if job.precision == "fp32" else 8
        return (p["flow"] + p.get("scalar", 0)) * p["nx"] * p["ny"] * p["nz"] * s

    def estimate(self, job: Job) -> float:
        # forward (2 states/step) + adjoint (2) + recorded moments and design (~1), plus a recompute
        # (2) unless every step's moments are held, at ~5.5 TB/s, plus launch overhead
        if not hasattr(job, "_store_all"):
            self._plan_bytes(job)
        passes = 5.0 if job._store_all else 7.0
        return job.steps * (passes * self.step_bytes(job) / 5.5e12 + 3 * 6e-6)

    def open(self, job: Job):
        torch = self.torch
        block = None
        ws = None
        if self.arena is not None:
            block = self.arena.alloc(job.footprint)
            if block is None:
                raise DeferAdmission("arena: no free block of %d B" % job.footprint)
            ws = block[1]
        make = lambda: self.lbm.Lbm(job.params, nsteps=job.steps, precision=job.precision,
                                    hbm_budget_bytes=job._budget, device=self.device, stream=self.stream,
                                    workspace=ws, inplace=job._inplace)
        try:
            try:
                L = make()
            except torch.cuda.OutOfMemoryError:
                torch.cuda.empty_cache()
                try:
                    L = make()
                except torch.cuda.OutOfMemoryError as e:
                    raise DeferAdmission("device memory: %s" % str(e).splitlines()[0])
        except Exception:
            if block is not None:
                self.arena.release(block[0], job.footprint)
            raise
        L._block = block
        L._footprint = job.footprint
        L._inplace = job._inplace
        dt = torch.float32 if job.precision == "fp32" else torch.float64
        host = torch.as_tensor(np.ascontiguousarray(np.asarray(job.design).reshape(-1)), dtype=dt).pin_memory()
        L._w_host = host
        L._w_dev = host.to(self.device, non_blocking=True)
        L.set_design(L._w_dev)
        L.reset()
        L._J = torch.empty(1, dtype=torch.float64, device=self.device)
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
        torch = self.torch
        g = handle.gradient()
        host_g = torch.empty(g.shape, dtype=g.dtype, pin_memory=True)
        host_J = torch.empty(1, dtype=torch.float64, pin_memory=True)
        host_g.copy_(g, non_blocking=True)
        host_J.copy_(handle._J, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return (ev, host_g, host_J, g)

    def ready(self, token) -> bool:
        return token[0].query()

    def result(self, handle, token):
        ev, host_g, host_J, _ = token
        ev.synchronize()
        return float(host_J[0]), host_g.numpy().copy()

    def close(self, handle):
        handle.close()
        if getattr(handle, "_block", None) is not None:
            self.arena.release(handle._block[0], handle._footprint)
            handle._block = None

    def mark(self):
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, mark):
        mark.synchronize()


def run_one_at_a_time(jobs: List[Job], device=None, clock=time.perf_counter,
                      per_request_cap_bytes: int = 64 << 30, inplace_min_state_bytes: Optional[int] = 32 << 20):
    """Baseline: the same trace on the same GPU, one request at a time in
    arrival order (FIFO), no overlap: each request is created, runs its full
    primal, objective, adjoint and gradient with single-context launches,
    and is read back before the next one starts.  Each request gets the same
    checkpoint plan and streaming as in the server (same per-request cap and
    in-place threshold)."""
    import torch

    from .lbm import Lbm
    ex = GpuExecutor(device, per_request_cap_bytes=per_request_cap_bytes,
                     inplace_min_state_bytes=inplace_min_state_bytes)
    t0 = clock()
    out = []
    for job in sorted(jobs, key=lambda j: j.arrival):
        while clock() - t0 < job.arrival:
            time.sleep(min(1e-3, job.arrival - (clock() - t0)))
        budget = ex._plan_bytes(job)
        L = Lbm(job.params, nsteps=job.steps, precision=job.precision, hbm_budget_bytes=budget, device=ex.device,
                inplace=job._inplace)
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

    def step_bytes(self, job):
        p = job.params
        return (p["flow"] + p.get("scalar", 0)) * p["nx"] * p["ny"] * p["nz"] * 8

    def estimate(self, job):
        p = job.params
        return max(self.sec, 1e-9) * p["nx"] * p["ny"] * p["nz"] * job.steps

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
