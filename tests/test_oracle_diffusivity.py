"""Pins of the oracle's design-dependent scalar diffusivity: Section 3.2 gives
material properties as the linear blend beta = w beta_fluid + (1-w) beta_solid,
so the scalar relaxation time is tau_s(w) = w tau_s + (1-w) tau_s_solid
(alpha = c^2 (tau_s - 1/2) is linear in tau_s).

Checked: the per-node relaxation factor, the diffusion rate of a Fourier mode in
a uniform design (closed form alpha(w) k^2), the reduction to a constant
diffusivity, and derivatives through the new w-dependence (complex step along
a direction, per-step dot product, central differences at every node).
"""
import numpy as np
import pytest

import oracle
from paper_1501_04741_amd import inputs


@pytest.mark.parametrize("flow,scalar", [(9, 5), (19, 7)])
@pytest.mark.parametrize("w", [1.0, 0.6, 0.0])
def test_interior_scalar_relaxes_at_the_blended_rate(flow, scalar, w):
    """g' - E^s(T, G u) = (1 - omega(w)) (g - E^s(T, G u)) with omega(w) = 1/(w tau_s + (1-w) tau_ss)."""
    rng = np.random.default_rng(3)
    nz = 4 if flow == 19 else 1
    e, wt, _, cs2 = oracle.lattice(flow)
    es, wts, _, c2 = oracle.lattice(scalar)
    cfg = dict(flow=flow, scalar=scalar, nx=4, ny=4, nz=nz, periodic=1, tau=0.9, tau_s=0.56, tau_s_solid=3.5,
               switch_fn="power", switch_param=3.0)
    f = wt * (1 + 0.05 * rng.standard_normal(flow))
    g = wts * (0.5 + 0.1 * rng.standard_normal(scalar))
    _, gp = oracle.node_op(cfg, 1, 1, 1 if flow == 19 else 0, f, g, w)
    u = (f @ e) / f.sum() * w ** 3
    T = g.sum()
    Es = wts * T * (1 + es @ u / c2)
    om = 1 / (w * 0.56 + (1 - w) * 3.5)
    assert np.allclose(gp - Es, (1 - om) * (g - Es), atol=1e-16)


@pytest.mark.parametrize("flow,scalar", [(9, 5), (19, 7)])
@pytest.mark.parametrize("w", [1.0, 0.7, 0.0])
def test_fourier_mode_diffuses_at_the_blended_diffusivity(flow, scalar, w):
    """T = A sin(k x) in a periodic box at rest with uniform w decays as
    exp(-alpha(w) k^2 t), alpha(w) = w alpha_fluid + (1-w) alpha_solid."""
    nx, ny, nz = 64, 3, (3 if flow == 19 else 1)
    tau_s, tau_ss = 0.6, 1.4
    cfg = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, periodic=1, tau=0.8, tau_s=tau_s, tau_s_solid=tau_ss,
               switch_fn="power", switch_param=3.0)
    n = nx * ny * nz
    x = np.arange(n) % nx
    k = 2 * np.pi / nx
    e, wt, _, _ = oracle.lattice(flow)
    es, wts, _, c2 = oracle.lattice(scalar)
    f0 = np.repeat(wt[:, None], n, axis=1)
    g0 = wts[:, None] * (1e-3 * np.sin(k * x))[None, :]
    t1, t2 = 100, 400
    r1 = oracle.primal(cfg, np.full(n, w), t1, f0=f0, g0=g0)
    r2 = oracle.primal(cfg, np.full(n, w), t2 - t1, f0=r1["f"], g0=r1["g"])
    amp = lambda g: abs(2 * np.mean(g.sum(axis=0) * np.exp(-1j * k * x)))
    rate = -np.log(amp(r2["g"]) / amp(r1["g"])) / (t2 - t1)
    alpha = w * c2 * (tau_s - 0.5) + (1 - w) * c2 * (tau_ss - 0.5)
    assert abs(rate / (alpha * k * k) - 1) < 5e-3


def test_equal_solid_and_fluid_rates_change_nothing():
    p = dict(flow=9, scalar=5, nx=16, ny=8, nz=1, tau=0.8, tau_s=0.7, u_in=0.02, c_dp=1.0, c_hf=1.0, c_var=0.5,
             s_in_lo=0.0, s_in_hi=1.0, s_split_axis=1, switch_fn="power", switch_param=3.0)
    w = inputs.porosity(16, 8, 1, 0, 3)
    a = oracle.adjoint(p, w, 60)
    b = oracle.adjoint(dict(p, tau_s_solid=0.7), w, 60)
    assert abs(a["J"] - b["J"]) <= 1e-14 * abs(a["J"])
    assert np.linalg.norm(a["grad"] - b["grad"]) <= 1e-12 * np.linalg.norm(a["grad"])


def _vd(flow, scalar, **kw):
    nz = 6 if flow == 19 else 1
    nx, ny = (16, 8) if flow == 9 else (8, 6)
    p = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, tau=0.8, tau_s=0.56, tau_s_solid=4.5, u_in=0.02,
             rho_out=1.0, switch_fn="ramp", switch_param=0.1, c_dp=-0.1, c_hf=1.0, scalar_wall="dirichlet",
             s_wall=1.0, s_in_lo=0.0, s_in_hi=0.0)
    p.update(kw)
    return p, inputs.porosity(nx, ny, nz, 0, 3)


@pytest.mark.parametrize("flow,scalar,steps", [(9, 5, 200), (19, 7, 40)])
def test_blended_diffusivity_adjoint_vs_complex_step(flow, scalar, steps):
    p, w = _vd(flow, scalar)
    rng = np.random.default_rng(9)
    dw = rng.standard_normal(w.size)
    a = oracle.adjoint(p, w, steps)
    J, dJ = oracle.directional(p, w, dw, steps)
    assert abs(a["J"] - J) <= 1e-14 * abs(J)
    assert abs(a["grad"] @ dw - dJ) <= 1e-12 * abs(dJ)


def test_blended_diffusivity_adjoint_vs_central_differences():
    p, w = _vd(9, 5)
    steps = 150
    g = oracle.adjoint(p, w, steps)["grad"]
    eps = 1e-5
    fd = np.zeros_like(w)
    for k in np.nonzero(oracle.mask(p) == 0)[0]:
        wp = w.copy(); wp[k] += eps
        wm = w.copy(); wm[k] -= eps
        fd[k] = (oracle.primal(p, wp, steps)["J"] - oracle.primal(p, wm, steps)["J"]) / (2 * eps)
    assert np.max(np.abs(fd - g)) < 1e-6 * np.abs(g).max()


def test_blended_diffusivity_step_dot_product():
    p, w = _vd(19, 7)
    n = p["nx"] * p["ny"] * p["nz"]
    r = oracle.primal(p, w, 10)
    f, g = r["f"], r["g"]
    rng = np.random.default_rng(4)
    df, dg, dw = rng.standard_normal(f.shape), rng.standard_normal(g.shape), rng.standard_normal(n)
    lf, lg = rng.standard_normal(f.shape), rng.standard_normal(g.shape)
    tf, tg = oracle.step_tangent(p, w, f, g, df, dg, dw)
    af, ag, gw = oracle.step_adjoint(p, w, f, g, lf, lg)
    lhs = np.sum(tf * lf) + np.sum(tg * lg)
    rhs = np.sum(df * af) + np.sum(dg * ag) + np.sum(dw * gw)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
