"""Pressure inlet with its velocity limit and the mixing objective on the GPU:
parity with the FP64 oracle (primal, adjoint, one-shot, batched), and the
paper's empty mixing duct (Section 4) reproduced against its printed values."""
import numpy as np
import pytest
import torch

import oracle
from paper_1501_04741_amd import inputs
from paper_1501_04741_amd import lbm as L
from paper_1501_04741_amd.lbm import Lbm

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _case(flow, scalar, nx, ny, nz, steps, frac=0.5, **kw):
    """A pressure-driven channel whose velocity limit sits at `frac` of the range
    of inlet velocities the oracle reaches after `steps` (so both inlet forms run;
    frac = None: no limit)."""
    p = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, tau=0.8, tau_s=0.6, inlet="pressure", rho_in=1.02,
             rho_out=1.0, switch_fn="ramp", switch_param=0.05, c_dp=1.0)
    if scalar:
        p.update(c_mix=1.0, c_hf=0.3, s_in_lo=-1.0, s_in_hi=1.0, s_split_axis=1, scalar_wall="adiabatic")
    p.update(kw)
    w = 0.5 + 0.5 * inputs.porosity(nx, ny, nz, 0, 3)
    if frac is not None:
        r = oracle.primal(p, w, steps)
        _, u, _ = oracle.fields(p, r["f"], r["g"] if scalar else None)
        uin = u[0][oracle.mask(p) == 2]
        p["u_cap"] = float(uin.min() + frac * (uin.max() - uin.min()))
    return p, w


CASES = [
    ("d2q9_capped", (9, 0, 70, 9, 1), {}),
    ("d2q9_d2q5_mix_capped", (9, 5, 40, 11, 1), {}),
    ("d2q9_d2q5_mix_free", (9, 5, 33, 8, 1), dict(frac=None)),
    ("d3q19_d3q7_mix_capped", (19, 7, 18, 8, 7), {}),
    ("d3q19_capped_ragged", (19, 0, 66, 5, 4), dict(frac=0.3)),
]


@pytest.mark.parametrize("name,shape,kw", CASES, ids=[c[0] for c in CASES])
def test_pressure_inlet_fp64_matches_oracle(name, shape, kw):
    steps = 60
    p, w = _case(*shape, steps, **kw)
    for interval in (0, 7):
        ctx = Lbm(p, nsteps=steps, precision="fp64", checkpoint_interval=interval)
        ctx.set_design(torch.from_numpy(w))
        ctx.primal_steps(steps, record=True)
        f, g = ctx.get_state()
        rho, u, s = ctx.fields()
        J, G = ctx.objective()
        ref = oracle.primal(p, w, steps)
        rr, ur, sr = oracle.fields(p, ref["f"], ref["g"] if p["scalar"] else None)
        assert np.max(np.abs(_np(f) - ref["f"])) < 1e-13
        assert np.max(np.abs(_np(rho) - rr)) < 1e-12
        assert np.max(np.abs(_np(u) - ur)) < 1e-13
        if p["scalar"]:
            assert np.max(np.abs(_np(g) - ref["g"])) < 1e-13
            assert np.max(np.abs(_np(s) - sr)) < 1e-12
        assert np.allclose(G, ref["globals"], rtol=1e-12, atol=1e-13)
        assert abs(J - ref["J"]) <= 1e-10 * abs(ref["J"])
        ctx.adjoint_steps(steps)
        lf, lg = ctx.get_adjoint()
        grad = _np(ctx.gradient())
        a = oracle.adjoint(p, w, steps)
        assert np.linalg.norm(grad - a["grad"]) <= 1e-10 * np.linalg.norm(a["grad"])
        scale = max(np.abs(a["lam_f"]).max(), np.abs(a["lam_g"]).max() if p["scalar"] else 0.0)
        assert np.max(np.abs(_np(lf) - a["lam_f"])) <= 1e-10 * scale
        if p["scalar"]:
            assert np.max(np.abs(_np(lg) - a["lam_g"])) <= 1e-10 * scale
        ctx.close()


def test_pressure_inlet_fp32_matches_oracle():
    steps = 200
    p, w = _case(19, 7, 40, 12, 10, steps)
    w32 = w.astype(np.float32)
    ctx = Lbm(p, nsteps=steps, precision="fp32")
    ctx.set_design(torch.from_numpy(w32))
    ctx.primal_steps(steps, record=True)
    J, _ = ctx.objective()
    _, u, _ = ctx.fields()
    ctx.adjoint_steps(steps)
    grad = _np(ctx.gradient()).astype(np.float64)
    w64 = w32.astype(np.float64)
    ref = oracle.adjoint(p, w64, steps)
    r = oracle.primal(p, w64, steps)
    _, ur, _ = oracle.fields(p, r["f"], r["g"])
    assert np.max(np.abs(_np(u) - ur)) <= 1e-4 * np.max(np.abs(ur))
    assert abs(J - ref["J"]) <= 1e-4 * abs(ref["J"])
    assert np.linalg.norm(grad - ref["grad"]) <= 1e-3 * np.linalg.norm(ref["grad"])


def test_pressure_inlet_oneshot_fp64_matches_oracle():
    iters, zeta, pen = 60, 2.0, -0.002
    p, _ = _case(9, 5, 40, 11, 1, iters)
    w0 = inputs.porosity(p["nx"], p["ny"], p["nz"], 1, 3)
    ctx = Lbm(p, nsteps=0, precision="fp64")
    ctx.set_design(torch.from_numpy(w0))
    ctx.reset()
    for k in (1, 25, iters - 26):
        ctx.oneshot_steps(k, zeta, pen)
    ref = oracle.oneshot(p, w0, iters, zeta, pen)
    w = _np(ctx.design())
    f, g = ctx.get_state()
    lf, lg = ctx.get_adjoint()
    assert np.max(np.abs(w - ref["w"])) <= 1e-12
    assert np.max(np.abs(_np(f) - ref["f"])) <= 1e-13
    assert np.max(np.abs(_np(g) - ref["g"])) <= 1e-13
    scale = max(np.abs(ref["lam_f"]).max(), np.abs(ref["lam_g"]).max())
    assert np.max(np.abs(_np(lf) - ref["lam_f"])) <= 1e-10 * scale
    assert np.max(np.abs(_np(lg) - ref["lam_g"])) <= 1e-10 * scale
    assert np.linalg.norm(_np(ctx.gradient()) - ref["grad"]) <= 1e-10 * np.linalg.norm(ref["grad"])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_pressure_inlet_batched_bitwise_equals_single(prec):
    steps = 31
    dt = np.float32 if prec == "fp32" else np.float64
    cases = [_case(19, 7, 18, 8, 7, steps), _case(19, 7, 33, 6, 5, steps, frac=0.2)]
    ref, ctxs = [], []
    for (p, w), c in zip(cases, (0, 5)):
        a = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=c)
        J, g = a.value_and_grad(torch.from_numpy(w.astype(dt)))
        ref.append((J, _np(g)))
        b = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=c)
        b.set_design(torch.from_numpy(w.astype(dt)))
        b.reset()
        ctxs.append(b)
    h = [c.ctx for c in ctxs]
    L.lbm_primal_steps_batch(h, 13, record=True)
    L.lbm_primal_steps_batch(h, steps - 13, record=True)
    Js = [c.objective()[0] for c in ctxs]
    L.lbm_adjoint_steps_batch(h, 20)
    L.lbm_adjoint_steps_batch(h, steps - 20)
    for c, (J, g), Jb in zip(ctxs, ref, Js):
        assert Jb == J
        assert np.array_equal(_np(c.gradient()), g)


def test_empty_mixer_reproduces_the_papers_printed_values():
    """The mixing duct of Section 4 without obstacles, run to steady state in FP32,
    against the 'Empty' row of the paper's results table: objective 49.266, outlet
    velocity mean 0.051 and SD 0.031, outlet temperature mean 0.000 and SD 0.763.
    The temperature statistics are weighted by the outlet flux u_x, the weighting
    of the objective itself (Mix = sum u_x (1 - T^2), so the weighted SD is
    sqrt(1 - Mix / sum u_x)); unweighted, the SD is 0.806."""
    wl = inputs.workload("d3q19_d3q7_mixer_empty_450x50x50")
    p = inputs.model_params(wl)
    ctx = Lbm(p, nsteps=0, precision="fp32")
    ctx.set_design(torch.from_numpy(inputs.design_for(wl)))
    ctx.reset()
    mask, _ = ctx.export_maps()
    outlet = _np(mask) == 3
    ctx.primal_steps(80000)
    J, G = ctx.objective()
    _, u, s = ctx.fields()
    ux = _np(u)[0][outlet]
    T = _np(s)[outlet]
    mix = float(np.sum(ux * (1 - T) * (1 + T)))
    assert abs(J - mix) <= 1e-6 * abs(mix)
    t_mean = float(np.sum(ux * T) / np.sum(ux))
    t_sd = float(np.sqrt(np.sum(ux * T * T) / np.sum(ux) - t_mean ** 2))
    print("empty mixer: J %.4f u mean %.5f sd %.5f T mean %.5f sd %.5f" % (J, ux.mean(), ux.std(), t_mean, t_sd))
    assert abs(J / 49.266 - 1) < 1e-2          # measured -0.14%
    assert abs(ux.mean() - 0.051) < 1e-3       # measured 0.0511
    assert abs(ux.std() - 0.031) < 1e-3        # measured 0.0311
    assert abs(t_mean - 0.000) < 5e-3
    assert abs(t_sd - 0.763) < 3e-3            # measured 0.7630
