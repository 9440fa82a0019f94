"""Pins of the oracle's pressure inlet (with its velocity limit) and of the mixing
objective of Section 4 (eq. mixing:obj).

The setup of Section 4 drives the channel by Zou-He pressure conditions at both
ends and limits the inlet velocity; the oracle reads the limit per inlet node: a
node whose pressure-form velocity would exceed u_cap takes the velocity form at
u_cap.  These tests fix that reading from outside the oracle: imposed mass and
momentum of the rebuilt state (closed forms from the known populations), Zou-He
exactness on equilibria, continuity at the limit, pressure-driven Poiseuille flow,
the mixing flux on a known outlet state, and derivatives through both branches
(complex step, finite differences, dot-product transposition).
"""
import numpy as np
import pytest

import oracle
from paper_1501_04741_amd import inputs


def _z(flow):
    return (5, 2) if flow == 19 else (1, 0)


def _known_P(f, e):
    """P = sum_{e_x=0} f + 2 sum_{e_x=-1} f: what reached x = 0 from inside."""
    return f[e[:, 0] == 0].sum() + 2.0 * f[e[:, 0] == -1].sum()


def _equilibrium(flow, rho, ux):
    e, wt, _, cs2 = oracle.lattice(flow)
    eu = e[:, 0] * ux
    return wt * rho * (1 + eu / cs2 + eu ** 2 / (2 * cs2 ** 2) - ux ** 2 / (2 * cs2))


@pytest.mark.parametrize("flow,scalar", [(9, 5), (19, 7)])
def test_pressure_inlet_imposes_density_and_normal_flow(flow, scalar):
    """Uncapped: the rebuilt and relaxed inlet state has mass rho_in and momentum
    rho_in (1 - P/rho_in, 0, 0); the scalar keeps T_in."""
    rng = np.random.default_rng(3)
    nz, z = _z(flow)
    e, wt, _, _ = oracle.lattice(flow)
    es, wts, _, _ = oracle.lattice(scalar)
    cfg = dict(flow=flow, scalar=scalar, nx=6, ny=5, nz=nz, tau=0.9, tau_s=0.7, inlet="pressure", rho_in=1.03,
               u_cap=0.0, s_in_lo=0.25, s_in_hi=0.75, s_split_axis=1)
    for _ in range(5):
        f = wt * 1.01 * (1 + 0.05 * rng.standard_normal(flow))
        g = wts * (0.4 + 0.1 * rng.standard_normal(scalar))
        up = 1.0 - _known_P(f, e) / 1.03
        for y, tin in ((1, 0.25), (3, 0.75)):
            h, gp = oracle.node_op(cfg, 0, y, z, f, g, 0.5)
            assert abs(h.sum() - 1.03) < 1e-15
            assert np.allclose(h @ e, 1.03 * np.array([up, 0, 0]), atol=1e-16)
            assert abs(gp.sum() - tin) < 1e-15


@pytest.mark.parametrize("flow", [9, 19])
def test_capped_inlet_is_the_velocity_inlet_at_the_cap(flow):
    """Where the pressure form would exceed u_cap the node is the velocity inlet at
    u_cap: mass P/(1-u_cap), momentum rho u_cap, and the same output as the velocity
    form with u_in = u_cap; below the cap it stays the pressure form."""
    rng = np.random.default_rng(5)
    nz, z = _z(flow)
    e, wt, _, _ = oracle.lattice(flow)
    base = dict(flow=flow, scalar=0, nx=6, ny=5, nz=nz, tau=0.8)
    for _ in range(5):
        f = wt * (1 + 0.05 * rng.standard_normal(flow))
        P = _known_P(f, e)
        rho_in = P / (1 - 0.08)            # pressure-form velocity 0.08
        capped = dict(base, inlet="pressure", rho_in=rho_in, u_cap=0.05)
        h, _ = oracle.node_op(capped, 0, 2, z, f, None, 0.5)
        assert abs(h.sum() - P / (1 - 0.05)) < 1e-15
        assert np.allclose(h @ e, h.sum() * np.array([0.05, 0, 0]), atol=1e-16)
        hv, _ = oracle.node_op(dict(base, u_in=0.05), 0, 2, z, f, None, 0.5)
        assert np.array_equal(h, hv)
        free = dict(capped, u_cap=0.1)
        h, _ = oracle.node_op(free, 0, 2, z, f, None, 0.5)
        assert abs(h.sum() - rho_in) < 1e-15
        assert abs((h @ e)[0] - rho_in * 0.08) < 1e-15


@pytest.mark.parametrize("flow", [9, 19])
def test_pressure_inlet_is_exact_on_equilibria(flow):
    """E(rho_in, (u,0,0)) passes the uncapped pressure inlet unchanged for any tau
    (Zou-He reconstruction is exact on equilibria)."""
    nz, z = _z(flow)
    for tau in (0.8, 1.3):
        for u in (0.0, 0.03, -0.01):
            E = _equilibrium(flow, 1.04, u)
            cfg = dict(flow=flow, nx=6, ny=5, nz=nz, tau=tau, inlet="pressure", rho_in=1.04, u_cap=0.0)
            h, _ = oracle.node_op(cfg, 0, 2, z, E, None, 0.3)
            assert np.allclose(h, E, atol=1e-16)


@pytest.mark.parametrize("flow", [9, 19])
def test_inlet_is_continuous_at_the_cap(flow):
    """The two forms agree where the pressure-form velocity equals u_cap, so the
    operator is continuous (Lipschitz) across the limit."""
    nz, z = _z(flow)
    e, wt, _, _ = oracle.lattice(flow)
    rng = np.random.default_rng(6)
    f = wt * (1 + 0.05 * rng.standard_normal(flow))
    P = _known_P(f, e)
    cfg = dict(flow=flow, nx=6, ny=5, nz=nz, tau=0.8, inlet="pressure", u_cap=0.05)
    outs = []
    for d in (-1e-9, 1e-9):
        h, _ = oracle.node_op(dict(cfg, rho_in=P / (1 - 0.05 - d)), 0, 2, z, f, None, 0.5)
        outs.append(h)
    assert np.max(np.abs(outs[1] - outs[0])) < 1e-8


def test_pressure_driven_poiseuille_channel():
    """Zou-He pressure at both ends of a bounce-back channel at w = 1: constant mass
    flux along x, a parabolic profile between walls half-way to the first fluid
    rows (tau = 1/2 + sqrt(3/16)), and mean velocity H^2/(12 nu rho) |dp/dx| with
    dp/dx = c_s^2 (rho_out - rho_in)/(nx - 1) set by the two imposed densities."""
    nx, ny = 60, 18
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    rho_in = 1.006
    cfg = dict(flow=9, nx=nx, ny=ny, nz=1, tau=tau, inlet="pressure", rho_in=rho_in, u_cap=0.0, rho_out=1.0,
               switch_fn="power", switch_param=3.0)
    n = nx * ny
    r = oracle.primal(cfg, np.ones(n), 8000)
    rho, u, _ = oracle.fields(cfg, r["f"])
    ux = u[0].reshape(ny, nx)
    rho = rho.reshape(ny, nx)
    assert np.allclose(rho[1:-1, 0], rho_in, atol=1e-15)
    flux = (rho * ux)[1:-1, :].sum(axis=0)
    assert np.allclose(flux, flux[nx // 2], rtol=1e-5)
    H = ny - 2
    yy = np.arange(1, ny - 1)
    xm = nx // 2
    ubar = ux[1:-1, xm].mean()
    prof = 6 * ubar * (yy - 0.5) * (ny - 1.5 - yy) / H ** 2
    assert np.max(np.abs(ux[1:-1, xm] - prof)) < 3e-3 * np.max(prof)   # measured 2.0e-3
    nu = (tau - 0.5) / 3
    dpdx = (1.0 - rho_in) / 3 / (nx - 1)
    expect = H ** 2 / (12 * nu * rho[1:-1, xm].mean()) * (-dpdx)
    assert abs(ubar / expect - 1) < 5e-3                                # measured 1.9e-3


@pytest.mark.parametrize("flow,scalar", [(9, 5), (19, 7)])
def test_mixing_flux_on_known_outlet_state(flow, scalar):
    """Outlet carrying E(1, (u0,0,0)) and E^s(T(y), u0): the mixing objective is
    sum u0 (1 - T)(1 + T) over the outlet nodes (eq. mixing:obj)."""
    nx, ny = 6, 5
    nz = 5 if flow == 19 else 1
    n = nx * ny * nz
    es, wts, _, c2 = oracle.lattice(scalar)
    base = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, u_in=0.0, rho_out=1.0, c_dp=0.0, c_mix=1.0)
    msk = oracle.mask(base)
    yy = (np.arange(n) // nx) % ny
    Tn = -0.9 + 0.45 * yy
    u0 = 0.02
    f = np.repeat(_equilibrium(flow, 1.0, u0)[:, None], n, axis=1)
    g = wts[:, None] * Tn[None, :] * (1 + (es[:, 0:1] * u0) / c2)
    r = oracle.primal(base, np.ones(n), 0, f0=f, g0=g)
    outl = msk == 3
    assert abs(r["J"] - np.sum(u0 * (1 - Tn[outl]) * (1 + Tn[outl]))) < 1e-15


def _pressure_case(flow, scalar, steps, frac=0.5):
    """A small pressure-driven channel whose cap sits inside the range of the
    inlet velocities it reaches, so both inlet forms occur."""
    nz = 6 if flow == 19 else 1
    nx, ny = (16, 8) if flow == 9 else (8, 6)
    p = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, tau=0.8, tau_s=0.6, inlet="pressure", rho_in=1.02,
             rho_out=1.0, switch_fn="power", switch_param=3.0, c_dp=1.0)
    if scalar:
        p.update(c_mix=1.0, c_hf=0.3, s_in_lo=-1.0, s_in_hi=1.0, s_split_axis=1, scalar_wall="adiabatic")
    w = 0.5 + 0.5 * inputs.porosity(nx, ny, nz, 0, 3)
    r = oracle.primal(p, w, steps)
    _, u, _ = oracle.fields(p, r["f"], r["g"] if scalar else None)
    inl = oracle.mask(p) == 2
    lo, hi = u[0][inl].min(), u[0][inl].max()
    assert hi > lo > 0
    p["u_cap"] = lo + frac * (hi - lo)
    return p, w


@pytest.mark.parametrize("flow,scalar,steps", [(9, 0, 300), (9, 5, 200), (19, 7, 40)])
def test_pressure_inlet_adjoint_vs_complex_step(flow, scalar, steps):
    """<dJ/dw, dw> from the adjoint equals the complex-step derivative of J along dw
    through a run in which inlet nodes switch between the two forms."""
    p, w = _pressure_case(flow, scalar, steps)
    rng = np.random.default_rng(9)
    dw = rng.standard_normal(w.size)
    a = oracle.adjoint(p, w, steps)
    J, dJ = oracle.directional(p, w, dw, steps)
    assert abs(a["J"] - J) <= 1e-14 * abs(J)
    assert abs(a["grad"] @ dw - dJ) <= 1e-12 * abs(dJ)


def test_pressure_inlet_adjoint_vs_central_differences():
    """Central differences of the real run (eps = 1e-5) at every interior node of
    16x8 with both inlet forms present."""
    p, w = _pressure_case(9, 5, 150)
    steps = 150
    g = oracle.adjoint(p, w, steps)["grad"]
    eps = 1e-5
    fd = np.zeros_like(w)
    inner = np.nonzero(oracle.mask(p) == 0)[0]
    for k in inner:
        wp = w.copy(); wp[k] += eps
        wm = w.copy(); wm[k] -= eps
        fd[k] = (oracle.primal(p, wp, steps)["J"] - oracle.primal(p, wm, steps)["J"]) / (2 * eps)
    assert np.max(np.abs(fd - g)) < 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("flow,scalar", [(9, 5), (19, 7)])
def test_pressure_inlet_step_adjoint_dot_product(flow, scalar):
    """One step: the adjoint step is the transpose of the tangent step with both
    inlet forms present."""
    p, w = _pressure_case(flow, scalar, 60 if flow == 9 else 20)
    n = p["nx"] * p["ny"] * p["nz"]
    r = oracle.primal(p, w, 60 if flow == 9 else 20)
    f, g = r["f"], r["g"]
    rng = np.random.default_rng(4)
    df = rng.standard_normal(f.shape)
    dg = rng.standard_normal(g.shape)
    dw = rng.standard_normal(n)
    lf = rng.standard_normal(f.shape)
    lg = rng.standard_normal(g.shape)
    tf, tg = oracle.step_tangent(p, w, f, g, df, dg, dw)
    af, ag, gw = oracle.step_adjoint(p, w, f, g, lf, lg)
    lhs = np.sum(tf * lf) + np.sum(tg * lg)
    rhs = np.sum(df * af) + np.sum(dg * ag) + np.sum(dw * gw)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_mixing_objective_seed_vs_finite_differences():
    p, w = _pressure_case(9, 5, 100)
    r = oracle.primal(p, w, 100)
    J, lf, lg = oracle.objective_seed(p, r["f"], r["g"])
    assert abs(J - r["J"]) < 1e-14 * abs(J)
    rng = np.random.default_rng(1)
    df = rng.standard_normal(r["f"].shape)
    dg = rng.standard_normal(r["g"].shape)
    eps = 1e-7
    Jp = oracle.objective_seed(p, r["f"] + eps * df, r["g"] + eps * dg)[0]
    Jm = oracle.objective_seed(p, r["f"] - eps * df, r["g"] - eps * dg)[0]
    fd = (Jp - Jm) / (2 * eps)
    assert abs(fd - (np.sum(lf * df) + np.sum(lg * dg))) < 1e-7 * abs(fd)
