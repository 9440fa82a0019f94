"""Batched launches and the serving loop on the GPU: every request's result is
bitwise the same alone (single-context kernels) and in the mix (batched
kernels, other requests admitted mid-flight)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1501_04741_amd import inputs
from paper_1501_04741_amd import lbm as L
from paper_1501_04741_amd.lbm import Lbm
from paper_1501_04741_amd.serve import DONE, FAILED, GpuExecutor, Job, Server

pytestmark = pytest.mark.gpu


def _p(flow, scalar, nx, ny, nz, **kw):
    p = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, tau=0.8, tau_s=0.6, u_in=0.02, switch_fn="ramp",
             switch_param=0.01, c_dp=1.0)
    if scalar:
        p.update(c_var=1.0, c_dp=0.1, s_in_lo=0.0, s_in_hi=1.0, s_split_axis=1)
    p.update(kw)
    return p


def _alone(p, w, steps, prec, interval=0):
    ctx = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=interval)
    J, g = ctx.value_and_grad(torch.from_numpy(w))
    out = (J, g.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("kind", ["d2q9", "d3q19_d3q7"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_abi_bitwise_equals_single(kind, prec):
    if kind == "d2q9":
        ps = [_p(9, 0, 40, 12, 1), _p(9, 0, 70, 9, 1), _p(9, 0, 300, 6, 1), _p(9, 0, 130, 17, 1)]
    else:
        ps = [_p(19, 7, 18, 8, 7), _p(19, 7, 33, 6, 5), _p(19, 7, 70, 9, 6)]
    steps = 37
    intervals = [0, 5, 37, 1, 9][: len(ps)]
    dt = np.float32 if prec == "fp32" else np.float64
    ws = [inputs.porosity(p["nx"], p["ny"], p["nz"], i, 3, dt) for i, p in enumerate(ps)]
    ref = [_alone(p, w, steps, prec, c) for p, w, c in zip(ps, ws, intervals)]
    ctxs = [Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=c) for p, c in zip(ps, intervals)]
    for c, w in zip(ctxs, ws):
        c.set_design(torch.from_numpy(w))
        c.reset()
    handles = [c.ctx for c in ctxs]
    for k in (7, 13, steps - 20):
        L.lbm_primal_steps_batch(handles, k, record=True)
    Js = [c.objective()[0] for c in ctxs]
    for k in (5, 11, steps - 16):
        L.lbm_adjoint_steps_batch(handles, k)
    for c, (J, g), Jb in zip(ctxs, ref, Js):
        assert Jb == J
        assert np.array_equal(c.gradient().cpu().numpy(), g)


@pytest.mark.parametrize("widths", [(256, 512, 1024), (256, 192, 300), (384, 192, 576), (128, 130)],
                         ids=["4_waves", "mixed_1", "3_waves", "2_vs_3"])
def test_batched_block_widths_bitwise_equal_single(widths):
    """Batched launches take blocks of up to four waves when every member's row
    splits into them (256/512/1024-wide rows: four; 384/192/576: three; otherwise
    fewer): results stay bitwise those of the single-context kernels, including
    recomputed segments batched with members of other widths."""
    ps = [_p(9, 0, nx, 7, 1) for nx in widths]
    steps = 21
    intervals = [4, 21, 6, 5][: len(ps)]
    ws = [inputs.porosity(p["nx"], p["ny"], p["nz"], 10 + i, 3) for i, p in enumerate(ps)]
    ref = [_alone(p, w, steps, "fp64", c) for p, w, c in zip(ps, ws, intervals)]
    ctxs = [Lbm(p, nsteps=steps, precision="fp64", checkpoint_interval=c) for p, c in zip(ps, intervals)]
    for c, w in zip(ctxs, ws):
        c.set_design(torch.from_numpy(w))
        c.reset()
    handles = [c.ctx for c in ctxs]
    L.lbm_primal_steps_batch(handles, steps, record=True)
    Js = [c.objective()[0] for c in ctxs]
    for k in (3, steps - 3):
        L.lbm_adjoint_steps_batch(handles, k)
    for c, (J, g), Jb in zip(ctxs, ref, Js):
        assert Jb == J
        assert np.array_equal(c.gradient().cpu().numpy(), g)


def _alone_inplace(p, w, steps, prec, interval=0):
    ctx = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=interval, inplace=True)
    J, g = ctx.value_and_grad(torch.from_numpy(w))
    out = (J, g.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("kind", ["d2q9", "d3q19_d3q7"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_inplace_batched_bitwise_equals_single_inplace(kind, prec):
    """In-place members (store-all and checkpointed plans, whose segments are
    recomputed in place) batched together, with members one step apart so that
    every batched step and every batched adjoint step runs two launches (one
    per phase): J and the gradient equal the single-context in-place run
    bitwise, which in turn equals the ping-pong run."""
    if kind == "d2q9":
        ps = [_p(9, 0, 40, 12, 1), _p(9, 0, 70, 9, 1), _p(9, 0, 300, 6, 1), _p(9, 0, 128, 17, 1)]
    else:
        ps = [_p(19, 7, 18, 8, 7), _p(19, 7, 33, 6, 5), _p(19, 7, 64, 9, 6)]
    steps = 31
    intervals = [0, 5, 9, 4][: len(ps)]
    dt = np.float32 if prec == "fp32" else np.float64
    ws = [inputs.porosity(p["nx"], p["ny"], p["nz"], 20 + i, 3, dt) for i, p in enumerate(ps)]
    ref = [_alone_inplace(p, w, steps, prec, c) for p, w, c in zip(ps, ws, intervals)]
    pp = _alone(ps[1], ws[1], steps, prec, intervals[1])
    assert pp[0] == ref[1][0] and np.array_equal(pp[1], ref[1][1])
    ctxs = [Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=c, inplace=True) for p, c in zip(ps, intervals)]
    for c, w in zip(ctxs, ws):
        c.set_design(torch.from_numpy(w))
        c.reset()
    handles = [c.ctx for c in ctxs]
    ctxs[0].primal_steps(1, record=True)  # member 0 runs one step ahead: mixed phases
    for k in (6, 13):
        L.lbm_primal_steps_batch(handles, k, record=True)
    ctxs[0].primal_steps(steps - 20, record=True)
    L.lbm_primal_steps_batch(handles[1:], steps - 19, record=True)
    Js = [c.objective()[0] for c in ctxs]
    ctxs[-1].adjoint_steps(1)  # the last member one adjoint step ahead: mixed patterns
    for k in (4, 12):
        L.lbm_adjoint_steps_batch(handles, k)
    ctxs[-1].adjoint_steps(steps - 17)
    L.lbm_adjoint_steps_batch(handles[:-1], steps - 16)
    for c, (J, g), Jb in zip(ctxs, ref, Js):
        assert Jb == J
        assert np.array_equal(c.gradient().cpu().numpy(), g)


def test_inplace_batched_unrecorded_steps_bitwise_equal_single():
    ps = [_p(19, 7, 18, 8, 7), _p(19, 7, 33, 6, 5), _p(19, 7, 128, 9, 6)]
    ws = [inputs.porosity(p["nx"], p["ny"], p["nz"], 30 + i, 3, np.float64) for i, p in enumerate(ps)]
    single = [Lbm(p, nsteps=0, precision="fp64", inplace=True) for p in ps]
    batch = [Lbm(p, nsteps=0, precision="fp64", inplace=True) for p in ps]
    for a, b, w in zip(single, batch, ws):
        a.set_design(torch.from_numpy(w))
        b.set_design(torch.from_numpy(w))
        a.reset()
        b.reset()
    batch[1].primal_steps(1)  # one step ahead: mixed phases
    L.lbm_primal_steps_batch([b.ctx for b in batch], 24, record=False)
    L.lbm_primal_steps_batch([batch[0].ctx, batch[2].ctx], 1, record=False)
    for a in single:
        a.primal_steps(25)
    for a, b in zip(single, batch):
        fa, ga = a.get_state()
        fb, gb = b.get_state()
        assert torch.equal(fa, fb) and torch.equal(ga, gb)
        assert a.objective()[0] == b.objective()[0]


def test_batched_abi_rejects_mixed_kinds_and_bad_state():
    a = Lbm(_p(9, 0, 20, 8, 1), nsteps=4, precision="fp32")
    b = Lbm(_p(19, 0, 8, 6, 5), nsteps=4, precision="fp32")
    c = Lbm(_p(9, 0, 20, 8, 1), nsteps=4, precision="fp64")
    for x in (a, b, c):
        x.set_design(torch.full((x.N,), 0.8, dtype=x.dtype))
    with pytest.raises(L.LbmError):
        L.lbm_primal_steps_batch([a.ctx, b.ctx], 1, record=True)
    with pytest.raises(L.LbmError):
        L.lbm_primal_steps_batch([a.ctx, c.ctx], 1, record=True)
    with pytest.raises(L.LbmError):
        L.lbm_primal_steps_batch([a.ctx, a.ctx], 1, record=True)
    with pytest.raises(L.LbmError):
        L.lbm_adjoint_steps_batch([a.ctx], 1)  # nothing recorded
    with pytest.raises(L.LbmError):
        L.lbm_primal_steps_batch([a.ctx], 5, record=True)  # beyond the horizon
    # nothing ran: a full single run still works
    J, g = a.value_and_grad(torch.full((a.N,), 0.8, dtype=a.dtype))
    assert np.isfinite(J)


def _jobs(n_each=3, steps=60, prec="fp32"):
    sizes = [_p(9, 0, 96, 20, 1), _p(9, 0, 256, 12, 1), _p(19, 0, 24, 10, 8), _p(19, 0, 40, 12, 10)]
    jobs = []
    rid = 0
    dt = np.float32 if prec == "fp32" else np.float64
    for rep in range(n_each):
        for p in sizes:
            w = inputs.porosity(p["nx"], p["ny"], p["nz"], rid, 3, dt)
            jobs.append(Job(rid=rid, params=p, steps=steps + 7 * (rid % 3), design=w, precision=prec,
                            arrival=0.001 * rid))
            rid += 1
    return jobs


def test_served_results_equal_alone_bitwise():
    jobs = _jobs()
    ex = GpuExecutor()
    srv = Server(ex, hbm_budget_bytes=8 << 30, quantum=17)
    # stagger: half submitted now, the rest after a few ticks (joining running batches)
    for j in jobs[:6]:
        srv.submit(j)
    for _ in range(3):
        srv.tick()
    for j in jobs[6:]:
        srv.submit(j)
    srv.drain()
    assert all(j.state == DONE for j in jobs), [(j.rid, j.state, j.error) for j in jobs]
    for j in jobs:
        ctx = Lbm(j.params, nsteps=j.steps, precision=j.precision, hbm_budget_bytes=ex._plan_bytes(j),
                  inplace=j._inplace)
        J, g = ctx.value_and_grad(torch.from_numpy(j.design))
        assert j.J == J, (j.rid, j.J, J)
        assert np.array_equal(j.grad, g.cpu().numpy()), j.rid
        ctx.close()


def test_served_fp32_results_match_oracle():
    jobs = _jobs(n_each=1, steps=40)
    srv = Server(GpuExecutor(), hbm_budget_bytes=8 << 30, quantum=9)
    srv.replay(jobs, realtime=False)
    for j in jobs:
        assert j.state == DONE
        ref = oracle.adjoint(j.params, j.design.astype(np.float64), j.steps)
        assert abs(j.J - ref["J"]) <= 1e-4 * abs(ref["J"])
        assert np.linalg.norm(j.grad - ref["grad"]) <= 1e-3 * np.linalg.norm(ref["grad"])


def test_serving_failure_isolation():
    jobs = _jobs(n_each=1, steps=30)
    bad = jobs[1]
    bad.design = bad.design.copy()
    bp = bad.params
    bad.design[bp["nx"] // 2 + bp["nx"] * (bp["ny"] // 2 + bp["ny"] * (bp["nz"] // 2))] = np.nan  # interior node
    ex = GpuExecutor()
    srv = Server(ex, hbm_budget_bytes=8 << 30, quantum=11)
    srv.replay(jobs, realtime=False)
    assert bad.state == FAILED and "finite" in bad.error
    for j in jobs:
        if j is bad:
            continue
        assert j.state == DONE
        ctx = Lbm(j.params, nsteps=j.steps, precision=j.precision, hbm_budget_bytes=ex._plan_bytes(j),
                  inplace=j._inplace)
        J, g = ctx.value_and_grad(torch.from_numpy(j.design))
        assert j.J == J and np.array_equal(j.grad, g.cpu().numpy())
        ctx.close()
    assert srv.used == 0


def test_arena_backed_server_results_equal_alone():
    jobs = _jobs(n_each=2, steps=45)
    ex = GpuExecutor(arena_bytes=2 << 30)
    srv = Server(ex, hbm_budget_bytes=2 << 30, quantum_ms=2.0, max_active_state_bytes=8 << 20)
    srv.replay(jobs, realtime=False)
    assert all(j.state == DONE for j in jobs), [(j.rid, j.state, j.error) for j in jobs]
    assert ex.arena.free_bytes() == ex.arena.size
    for j in jobs:
        ctx = Lbm(j.params, nsteps=j.steps, precision=j.precision, hbm_budget_bytes=ex._plan_bytes(j),
                  inplace=j._inplace)
        J, g = ctx.value_and_grad(torch.from_numpy(j.design))
        assert j.J == J and np.array_equal(j.grad, g.cpu().numpy()), j.rid
        ctx.close()


def test_inplace_requests_served_equal_alone_bitwise():
    """Requests above the in-place threshold (here every request of the 40x12x10 size)
    stream in place, batched among themselves beside the batched ping-pong ones;
    every result equals the request run alone (ping-pong, every step's moments held)."""
    jobs = _jobs(n_each=2, steps=33)
    big = 19 * 40 * 12 * 10 * 4
    ex = GpuExecutor(inplace_min_state_bytes=big)
    srv = Server(ex, hbm_budget_bytes=4 << 30, quantum=10)
    for j in jobs[:4]:
        srv.submit(j)
    for _ in range(2):
        srv.tick()
    for j in jobs[4:]:
        srv.submit(j)
    srv.drain()
    assert all(j.state == DONE for j in jobs), [(j.rid, j.state, j.error) for j in jobs]
    inplace = [j for j in jobs if j._inplace]
    assert len(inplace) == 2 and all(j.params["nx"] == 40 for j in inplace)
    for j in jobs:
        J, g = _alone(j.params, j.design, j.steps, j.precision, interval=j.steps)
        assert j.J == J, (j.rid, j.J, J)
        assert np.array_equal(j.grad, g), j.rid


def test_cancelled_requests_free_their_memory_and_leave_the_rest_exact():
    """Cancel one request while queued and two mid-flight (primal and adjoint
    phase, one of them streamed in place); the others still equal their runs
    alone bitwise and the arena is whole again."""
    from paper_1501_04741_amd.serve import ADJOINT, CANCELLED, PRIMAL
    jobs = _jobs(n_each=2, steps=40)
    ex = GpuExecutor(arena_bytes=2 << 30, inplace_min_state_bytes=19 * 40 * 12 * 10 * 4)
    srv = Server(ex, hbm_budget_bytes=2 << 30, quantum=10, policy="fifo")
    for j in jobs:
        srv.submit(j)
    srv.tick()
    queued = next(j for j in jobs if j.state == "queued") if any(j.state == "queued" for j in jobs) else None
    for _ in range(4):
        srv.tick()
    in_adj = next(j for j in jobs if j.state == ADJOINT)
    in_primal = next((j for j in jobs if j.state == PRIMAL), None)
    victims = [in_adj] + ([in_primal] if in_primal else []) + ([queued] if queued and queued.state == "queued" else [])
    for v in victims:
        assert srv.cancel(v.rid)
    srv.drain()
    for v in victims:
        assert v.state == CANCELLED
    assert ex.arena.free_bytes() == ex.arena.size and srv.used == 0
    for j in jobs:
        if j in victims:
            continue
        assert j.state == DONE, (j.rid, j.state, j.error)
        J, g = _alone(j.params, j.design, j.steps, j.precision, interval=j.steps)
        assert j.J == J and np.array_equal(j.grad, g), j.rid


def test_served_requests_at_full_size_match_oracle_golden():
    """One request of each serving size (the first of its size in the benchmark's
    400-request trace, seed 1), served together in FP32 at its real size and
    horizon (2000 + 2000 steps; 200 + 200 for D3Q19 192x96x96), against the
    oracle's J and gradient stored by tests/golden/make_oracle_goldens.py:
    J within 1e-4, the gradient at 4096 seeded interior nodes within 1e-3
    relative L2 and its norm within 1e-3."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_serving_requests.npz")
    if not os.path.exists(path):
        pytest.skip("oracle golden oracle_serving_requests.npz not generated")
    ref = np.load(path, allow_pickle=False)
    trace = inputs.poisson_trace(400, 20.0, seed=1)
    jobs = []
    for i in range(len(ref["rid"])):
        req = trace[int(ref["rid"][i])]
        jobs.append(Job(rid=req.rid, params=req.params, steps=int(ref["steps"][i]),
                        design=inputs.request_design(req), precision="fp32", arrival=0.0))
    srv = Server(GpuExecutor(), hbm_budget_bytes=200 << 30, quantum=50)
    srv.replay(jobs, realtime=False)
    for i, j in enumerate(jobs):
        assert j.state == DONE, (j.rid, j.state, j.error)
        Jr = float(ref["J"][i])
        idx = ref["sample_idx"][i]
        gs = ref["grad_sample"][i]
        err = np.linalg.norm(j.grad[idx] - gs) / np.linalg.norm(gs)
        nerr = abs(np.linalg.norm(j.grad) / float(ref["grad_norm"][i]) - 1)
        print("request %d (%s): J %.10g oracle %.10g, sampled gradient rel-L2 %.2e, norm %.2e" % (
            j.rid, "x".join(str(j.params[k]) for k in ("nx", "ny", "nz")), j.J, Jr, err, nerr))
        assert abs(j.J - Jr) <= 1e-4 * abs(Jr)
        assert err <= 1e-3 and nerr <= 1e-3
