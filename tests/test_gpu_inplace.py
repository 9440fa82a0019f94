"""In-place streaming (one buffer per state, alternating even/odd access
patterns) against the ping-pong path, bitwise: unrecorded primal runs of odd
and even length, the one-shot iteration in chunks, state import/export in both
phases; and the calls an in-place context refuses."""
import numpy as np
import pytest
import torch

import oracle
from paper_1501_04741_amd import inputs
from paper_1501_04741_amd import lbm as L
from paper_1501_04741_amd.lbm import Lbm, LbmError

pytestmark = pytest.mark.gpu


def _np(t):
    return None if t is None else t.detach().cpu().numpy()


def _p(flow, scalar, nx, ny, nz, **kw):
    p = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, tau=0.8, tau_s=0.6, u_in=0.02, switch_fn="ramp",
             switch_param=0.05, c_dp=1.0)
    if scalar:
        p.update(c_hf=0.5, c_var=1.0, s_in_lo=0.0, s_in_hi=1.0, s_split_axis=1)
    p.update(kw)
    return p


CASES = [
    ("d2q9_ragged", _p(9, 0, 70, 9, 1)),
    ("d2q9_d2q5_dirichlet_blended", _p(9, 5, 40, 11, 1, scalar_wall="dirichlet", s_wall=1.0, tau_s_solid=3.0)),
    ("d3q19", _p(19, 0, 21, 7, 6)),
    ("d3q19_d3q7_mrt_pressure_mix", _p(19, 7, 24, 6, 5, collision="mrt", inlet="pressure", rho_in=1.02,
                                       u_cap=0.012, c_mix=1.0, s_in_lo=-1.0)),
    ("d3q19_d3q7_periodic", _p(19, 7, 9, 6, 5, periodic=1, c_dp=0.0, c_hf=0.0, c_var=0.0)),
]


def _pair(p, prec, seed=0):
    dt = np.float32 if prec == "fp32" else np.float64
    w = torch.from_numpy(inputs.porosity(p["nx"], p["ny"], p["nz"], seed, 3, dt))
    a = Lbm(p, nsteps=0, precision=prec)
    b = Lbm(p, nsteps=0, precision=prec, inplace=True)
    for c in (a, b):
        c.set_design(w)
        c.reset()
    return a, b


def _same_state(a, b):
    fa, ga = a.get_state()
    fb, gb = b.get_state()
    assert np.array_equal(_np(fa), _np(fb))
    if ga is not None:
        assert np.array_equal(_np(ga), _np(gb))
    for x, y in zip(a.fields(), b.fields()):
        if x is not None:
            assert np.array_equal(_np(x), _np(y))
    assert a.objective() == b.objective()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_inplace_primal_bitwise_equals_pingpong(name, p, prec):
    a, b = _pair(p, prec)
    done = 0
    for k in (0, 1, 1, 5, 16):          # ends on both phases along the way
        a.primal_steps(k)
        b.primal_steps(k)
        done += k
        _same_state(a, b)
    assert done == 23


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name,p", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_inplace_oneshot_bitwise_equals_pingpong(name, p, prec):
    a, b = _pair(p, prec, seed=1)
    for c in (a, b):
        c.primal_steps(3)                # start the one-shot from an odd phase
    for k in (1, 4, 7, 2):
        a.oneshot_steps(k, 0.5, -0.001)
        b.oneshot_steps(k, 0.5, -0.001)
        assert np.array_equal(_np(a.design()), _np(b.design()))
        assert np.array_equal(_np(a.gradient()), _np(b.gradient()))
        la, lga = a.get_adjoint()
        lb, lgb = b.get_adjoint()
        assert np.array_equal(_np(la), _np(lb))
        if lga is not None:
            assert np.array_equal(_np(lga), _np(lgb))
        _same_state(a, b)


def test_inplace_oneshot_matches_oracle():
    p = CASES[3][1]
    iters, zeta, pen = 45, 2.0, -0.002
    w0 = inputs.porosity(p["nx"], p["ny"], p["nz"], 1, 3)
    ctx = Lbm(p, nsteps=0, precision="fp64", inplace=True)
    ctx.set_design(torch.from_numpy(w0))
    ctx.reset()
    for k in (1, 25, iters - 26):
        ctx.oneshot_steps(k, zeta, pen)
    ref = oracle.oneshot(p, w0, iters, zeta, pen)
    f, g = ctx.get_state()
    lf, lg = ctx.get_adjoint()
    assert np.max(np.abs(_np(ctx.design()) - ref["w"])) <= 1e-12
    assert np.max(np.abs(_np(f) - ref["f"])) <= 1e-13
    scale = max(np.abs(ref["lam_f"]).max(), np.abs(ref["lam_g"]).max())
    assert np.max(np.abs(_np(lf) - ref["lam_f"])) <= 1e-10 * scale
    assert np.max(np.abs(_np(lg) - ref["lam_g"])) <= 1e-10 * scale


def test_inplace_set_state_round_trip():
    p = CASES[1][1]
    n = p["nx"] * p["ny"]
    rng = np.random.default_rng(5)
    e, wt, _, _ = oracle.lattice(9)
    f0 = torch.from_numpy(wt[:, None] * (1 + 0.05 * rng.standard_normal((9, n)))).cuda()
    g0 = torch.from_numpy(0.3 * rng.random((5, n))).cuda()
    a, b = _pair(p, "fp64")
    for c in (a, b):
        c.set_state(f0, g0)
    fb, gb = b.get_state()
    assert torch.equal(fb, f0) and torch.equal(gb, g0)
    for k in (1, 2):
        a.primal_steps(k)
        b.primal_steps(k)
        _same_state(a, b)


def test_inplace_refuses_recording_adjoint_and_mixed_batches():
    p = CASES[0][1]
    a, b = _pair(p, "fp32")
    with pytest.raises(LbmError):
        b.primal_steps(1, record=True)
    with pytest.raises(LbmError):
        b.adjoint_steps(1)
    with pytest.raises(LbmError):  # a batch is all in place or all ping-pong
        L.lbm_primal_steps_batch([b.ctx, a.ctx], 1, record=False)
    b.primal_steps(2)                    # still usable
    a.primal_steps(2)
    _same_state(a, b)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_inplace_recorded_run_and_adjoint_bitwise_equal_pingpong(name, p, prec):
    """A recorded in-place run (moments of every step, one primal buffer, the
    adjoint streamed in place too) against the ping-pong store-all plan: states after
    every forward chunk, J, the adjoint state after every backward chunk and
    the gradient are bitwise equal."""
    steps = 23
    dt = np.float32 if prec == "fp32" else np.float64
    w = torch.from_numpy(inputs.porosity(p["nx"], p["ny"], p["nz"], 2, 3, dt))
    a = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=steps)
    b = Lbm(p, nsteps=steps, precision=prec, inplace=True)
    assert b.workspace_bytes < a.workspace_bytes
    for c in (a, b):
        c.set_design(w)
        c.reset()
    for k in (7, 1, 15):
        a.primal_steps(k, record=True)
        b.primal_steps(k, record=True)
        _same_state(a, b)
    for k in (1, 4, 11, 7):
        a.adjoint_steps(k)
        b.adjoint_steps(k)
        la, lga = a.get_adjoint()
        lb, lgb = b.get_adjoint()
        assert np.array_equal(_np(la), _np(lb))
        if lga is not None:
            assert np.array_equal(_np(lga), _np(lgb))
    assert np.array_equal(_np(a.gradient()), _np(b.gradient()))


def test_inplace_recorded_value_and_grad_matches_oracle():
    p = CASES[1][1]
    steps = 40
    w = inputs.porosity(p["nx"], p["ny"], p["nz"], 0, 3)
    ctx = Lbm(p, nsteps=steps, precision="fp64", inplace=True)
    J, g = ctx.value_and_grad(torch.from_numpy(w))
    ref = oracle.adjoint(p, w, steps)
    assert abs(J - ref["J"]) <= 1e-10 * abs(ref["J"])
    assert np.linalg.norm(_np(g) - ref["grad"]) <= 1e-10 * np.linalg.norm(ref["grad"])


def test_inplace_streaming_hint_variants_bitwise_equal_pingpong_fp64_256x128x128():
    """The benchmark channel in FP64 (638 MB states, beyond twice the 256 MB
    last-level cache) takes the in-place kernels' streaming-hint variants in both
    phases: a recorded run with its adjoint, and an unrecorded run, against the
    ping-pong path, bitwise, after chunks ending in both phases."""
    wl = inputs.workload("d3q19_channel_256x128x128")
    p = inputs.model_params(wl)
    steps = 5
    w = torch.from_numpy(inputs.design_for(wl, np.float64)).cuda()
    a = Lbm(p, nsteps=steps, precision="fp64", checkpoint_interval=steps)
    b = Lbm(p, nsteps=steps, precision="fp64", inplace=True)
    assert b.plan()["state_bytes"] > 2 * 256 * 2**20
    for c in (a, b):
        c.set_design(w)
        c.reset()

    def same_state():
        fa, _ = a.get_state()
        fb, _ = b.get_state()
        assert torch.equal(fa, fb)
        del fa, fb

    for k in (2, 3):
        a.primal_steps(k, record=True)
        b.primal_steps(k, record=True)
        same_state()
    assert a.objective() == b.objective()
    for k in (1, 2, 2):
        a.adjoint_steps(k)
        b.adjoint_steps(k)
        la, _ = a.get_adjoint()
        lb, _ = b.get_adjoint()
        assert torch.equal(la, lb)
        del la, lb
    assert torch.equal(a.gradient(), b.gradient())
    a.close()
    b.close()
    # unrecorded: the unrecorded in-place variants beyond twice the cache
    a = Lbm(p, nsteps=0, precision="fp64")
    b = Lbm(p, nsteps=0, precision="fp64", inplace=True)
    for c in (a, b):
        c.set_design(w)
        c.reset()
    for k in (3, 2):
        a.primal_steps(k)
        b.primal_steps(k)
        same_state()
    a.close()
    b.close()



def test_unrecorded_inplace_between_one_and_two_caches_bitwise_equal_pingpong():
    """Unrecorded in-place steps on states between one and two last-level caches
    take streaming stores in the odd phase only: the benchmark channel in FP32
    (319 MB) alone, and four 128x96x96 channels (0.36 GB together) in one batched
    launch per phase, against the ping-pong path and the single-context kernels,
    bitwise, after chunks ending in both phases."""
    wl = inputs.workload("d3q19_channel_256x128x128")
    p = inputs.model_params(wl)
    w = torch.from_numpy(inputs.design_for(wl, np.float32)).cuda()
    a = Lbm(p, nsteps=0, precision="fp32")
    b = Lbm(p, nsteps=0, precision="fp32", inplace=True)
    assert 256 * 2**20 < b.plan()["state_bytes"] <= 2 * 256 * 2**20
    for c in (a, b):
        c.set_design(w)
        c.reset()
    for k in (3, 2):
        a.primal_steps(k)
        b.primal_steps(k)
        fa, _ = a.get_state()
        fb, _ = b.get_state()
        assert torch.equal(fa, fb)
        del fa, fb
    assert a.objective() == b.objective()
    a.close()
    b.close()
    q = dict(p, nx=128, ny=96, nz=96)
    ws = [torch.from_numpy(inputs.porosity(128, 96, 96, 40 + k, 5, np.float32)).cuda() for k in range(4)]
    single = [Lbm(q, nsteps=0, precision="fp32", inplace=True) for _ in range(4)]
    batch = [Lbm(q, nsteps=0, precision="fp32", inplace=True) for _ in range(4)]
    total = sum(c.plan()["state_bytes"] for c in batch)
    assert 256 * 2**20 < total <= 2 * 256 * 2**20
    for x, y, wk in zip(single, batch, ws):
        for c in (x, y):
            c.set_design(wk)
            c.reset()
    for k in (3, 2):
        for x in single:
            x.primal_steps(k)
        L.lbm_primal_steps_batch([c.ctx for c in batch], k, record=False)
        for x, y in zip(single, batch):
            fx, _ = x.get_state()
            fy, _ = y.get_state()
            assert torch.equal(fx, fy)
            del fx, fy
    for c in single + batch:
        c.close()

def test_set_design_after_adjoint_refuses_state_reads_until_reset():
    """Once an adjoint has run (and recomputed segments have overwritten the
    primal buffers), a new design invalidates the primal state: calls that read it
    are refused until lbm_reset or lbm_set_state."""
    p = CASES[2][1]
    w = torch.from_numpy(inputs.porosity(p["nx"], p["ny"], p["nz"], 0, 3))
    c = Lbm(p, nsteps=12, precision="fp64", checkpoint_interval=4)
    c.set_design(w)
    c.reset()
    c.primal_steps(12, record=True)
    c.adjoint_steps(12)
    c.gradient()
    c.set_design(w * 0.5)
    for call in (c.objective, c.fields, c.get_state, lambda: c.primal_steps(1),
                 lambda: c.oneshot_steps(1, 0.0)):
        with pytest.raises(LbmError) as e:
            call()
        assert e.value.status == L.LBM_ESTATE
    c.reset()
    c.primal_steps(3)
    J, _ = c.objective()
    ref = oracle.primal(p, _np(w * 0.5).astype(np.float64), 3)
    assert abs(J - ref["J"]) <= 1e-10 * abs(ref["J"])


@pytest.mark.parametrize("C", [4, 5, 1, 23])
@pytest.mark.parametrize("name,p", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_inplace_checkpointed_run_bitwise_equal_pingpong(name, p, C):
    """An in-place recorded run with a checkpoint every C steps (states copied out in
    their phase's layout, segments recomputed in place inside their checkpoint)
    against the ping-pong plan with the same C and the in-place store-all plan:
    J, the adjoint state after every backward chunk and the gradient bitwise."""
    steps = 23
    prec = "fp64" if C in (4, 23) else "fp32"
    dt = np.float32 if prec == "fp32" else np.float64
    w = torch.from_numpy(inputs.porosity(p["nx"], p["ny"], p["nz"], 6, 3, dt))
    a = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=C)
    b = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=C, inplace=True)
    c = Lbm(p, nsteps=steps, precision=prec, inplace=True)
    assert b.plan()["interval"] == min(C, steps) and c.plan()["interval"] == steps
    for x in (a, b, c):
        x.set_design(w)
        x.reset()
    for k in (6, 17):
        for x in (a, b, c):
            x.primal_steps(k, record=True)
        _same_state(a, b)
    assert a.objective() == c.objective()
    for k in (1, 3, 9, 10):
        for x in (a, b, c):
            x.adjoint_steps(k)
        la = _np(a.get_adjoint()[0])
        assert np.array_equal(la, _np(b.get_adjoint()[0]))
        assert np.array_equal(la, _np(c.get_adjoint()[0]))
    g = _np(a.gradient())
    assert np.array_equal(g, _np(b.gradient()))
    assert np.array_equal(g, _np(c.gradient()))
    if prec == "fp64" and name != "d3q19_d3q7_mrt_pressure_mix":  # its 23-step gradient is ~1e-8: rounding-level
        ref = oracle.adjoint(p, w.numpy(), steps)
        assert np.linalg.norm(g - ref["grad"]) <= 1e-10 * np.linalg.norm(ref["grad"])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name,p", [CASES[1], CASES[3]], ids=[CASES[1][0], CASES[3][0]])
def test_checkpointed_run_ending_before_the_last_segment(name, p, prec):
    """A checkpointed forward keeps the moments of the horizon's last segment only.
    A recorded run that stops earlier (13 of 23 steps, a checkpoint every 4, so
    inside segment 3 of 6) therefore holds none: the backward recomputes that
    segment as well.  J, the adjoint state after each chunk and the gradient
    bitwise equal to the store-all plan stopped at the same step, ping-pong and
    in place, and (FP64) within 1e-10 of the oracle's 13-step run."""
    steps, stop = 23, 13
    dt = np.float32 if prec == "fp32" else np.float64
    w = torch.from_numpy(inputs.porosity(p["nx"], p["ny"], p["nz"], 8, 3, dt))
    xs = [Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=4),
          Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=4, inplace=True),
          Lbm(p, nsteps=steps, precision=prec, inplace=True),
          Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=steps)]
    assert [x.plan()["interval"] for x in xs] == [4, 4, steps, steps]
    for x in xs:
        x.set_design(w)
        x.reset()
        x.primal_steps(5, record=True)
        x.primal_steps(stop - 5, record=True)
    J = xs[0].objective()
    assert all(x.objective() == J for x in xs[1:])
    for k in (2, 6, 5):
        for x in xs:
            x.adjoint_steps(k)
        la = _np(xs[0].get_adjoint()[0])
        for x in xs[1:]:
            assert np.array_equal(la, _np(x.get_adjoint()[0]))
    g = _np(xs[0].gradient())
    for x in xs[1:]:
        assert np.array_equal(g, _np(x.gradient()))
    if prec == "fp64" and name != "d3q19_d3q7_mrt_pressure_mix":
        ref = oracle.adjoint(p, w.numpy(), stop)
        assert abs(J[0] - ref["J"]) <= 1e-10 * abs(ref["J"])
        assert np.linalg.norm(g - ref["grad"]) <= 1e-10 * np.linalg.norm(ref["grad"])
    for x in xs:
        x.close()
