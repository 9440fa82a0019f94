"""Pins of the oracle's heating plate (Section 4, heat exchanger).

The exchanger duct has a D x D heating plate at the bottom, in the middle of the
channel, held at T = 1 while the other walls are adiabatic; the oracle reads it
as the stretch plate_x0 <= x < plate_x1 of the y = 0 wall across the whole width.
These tests fix that node class from outside the oracle: the plate nodes emit the
scalar equilibrium at rest at the plate value and still bounce the flow back,
every other wall node keeps its configured scalar condition, the field export
reports the plate value, and derivatives through runs with a plate agree with
complex step, central differences and the transposed tangent step.  The printed
values of the empty exchanger (Table tab:results) are checked on the GPU path.
"""
import numpy as np
import pytest

import oracle
from paper_1501_04741_amd import inputs


def _case(flow, **kw):
    nz = 6 if flow == 19 else 1
    nx, ny = (16, 8) if flow == 9 else (10, 6)
    scalar = 7 if flow == 19 else 5
    p = dict(flow=flow, scalar=scalar, nx=nx, ny=ny, nz=nz, tau=0.8, tau_s=0.6, u_in=0.03, rho_out=1.0,
             switch_fn="power", switch_param=3.0, c_dp=-0.1, c_hf=1.0, scalar_wall="adiabatic",
             s_in_lo=0.0, plate_x0=nx // 2 - 3, plate_x1=nx // 2 + 3, s_plate=1.0)
    p.update(kw)
    return p


@pytest.mark.parametrize("flow", [9, 19])
@pytest.mark.parametrize("wall", ["adiabatic", "dirichlet"])
def test_plate_nodes_hold_the_plate_value_and_bounce_the_flow(flow, wall):
    p = _case(flow, scalar_wall=wall, s_wall=0.3, s_plate=1.7)
    e, wt, opp, _ = oracle.lattice(flow)
    es, wts, opps, _ = oracle.lattice(p["scalar"])
    rng = np.random.default_rng(5)
    zs = (0, 2, p["nz"] - 1) if flow == 19 else (0,)
    for x in range(p["nx"]):
        for y in (0, p["ny"] - 1):
            for z in zs:
                f = wt * (1.0 + 0.05 * rng.standard_normal(flow))
                g = wts * (0.4 + 0.1 * rng.standard_normal(p["scalar"]))
                h, gp = oracle.node_op(p, x, y, z, f, g, 0.5)
                assert np.array_equal(h, f[opp])
                if y == 0 and p["plate_x0"] <= x < p["plate_x1"]:
                    assert np.allclose(gp, 1.7 * wts, rtol=0, atol=1e-16)
                elif wall == "dirichlet":
                    assert np.allclose(gp, 0.3 * wts, rtol=0, atol=1e-16)
                else:
                    assert np.array_equal(gp, g[opps])
    # side walls (3D): the plate is the bottom row only
    if flow == 19:
        f = wt.copy()
        g = wts * 0.2
        _, gp = oracle.node_op(p, p["plate_x0"], 2, 0, f, g, 0.5)
        assert np.array_equal(gp, g[opps]) if wall == "adiabatic" else np.allclose(gp, 0.3 * wts)


def test_no_plate_when_the_range_is_empty():
    p = _case(9, plate_x0=5, plate_x1=5)
    e, wt, opp, _ = oracle.lattice(9)
    es, wts, opps, _ = oracle.lattice(5)
    g = wts * 0.3
    _, gp = oracle.node_op(p, 5, 0, 0, wt, g, 0.5)
    assert np.array_equal(gp, g[opps])


def test_fields_report_the_plate_value():
    p = _case(19, s_plate=0.8)
    n = p["nx"] * p["ny"] * p["nz"]
    w = inputs.porosity(p["nx"], p["ny"], p["nz"], 0, 3)
    r = oracle.primal(p, w, 7)
    _, _, T = oracle.fields(p, r["f"], r["g"])
    idx = np.arange(n)
    x, y = idx % p["nx"], (idx // p["nx"]) % p["ny"]
    plate = (y == 0) & (x >= p["plate_x0"]) & (x < p["plate_x1"])
    assert np.all(T[plate] == 0.8)
    # the plate heats the fluid next to it: after 7 steps the rows above it are warm
    above = (y == 1) & (x >= p["plate_x0"]) & (x < p["plate_x1"]) & (oracle.mask(p) == 0)
    assert T[above].min() > 0.05


@pytest.mark.parametrize("flow,steps", [(9, 200), (19, 40)])
@pytest.mark.parametrize("inlet", ["velocity", "pressure"])
def test_plate_adjoint_vs_complex_step(flow, steps, inlet):
    """<dJ/dw, dw> from the adjoint equals the complex-step derivative of J along
    dw through a run with a plate, blended diffusivity (solid 1 against fluid
    0.003 in the exchanger; here tau_s_solid = 2) and the heat-flux objective."""
    kw = dict(tau_s_solid=2.0)
    if inlet == "pressure":
        kw.update(inlet="pressure", rho_in=1.03, u_cap=0.02)
    p = _case(flow, **kw)
    w = 0.5 + 0.5 * inputs.porosity(p["nx"], p["ny"], p["nz"], 1, 3)
    rng = np.random.default_rng(13)
    dw = rng.standard_normal(w.size)
    a = oracle.adjoint(p, w, steps)
    J, dJ = oracle.directional(p, w, dw, steps)
    assert abs(a["J"] - J) <= 1e-14 * abs(J)
    assert abs(a["grad"] @ dw - dJ) <= 1e-12 * abs(dJ)


def test_plate_adjoint_vs_central_differences():
    """Central differences of the real run (eps = 1e-5) at every interior node of
    16x8 with the plate."""
    p = _case(9)
    steps = 150
    w = 0.5 + 0.5 * inputs.porosity(16, 8, 1, 2, 3)
    g = oracle.adjoint(p, w, steps)["grad"]
    eps = 1e-5
    fd = np.zeros_like(w)
    for k in np.nonzero(oracle.mask(p) == 0)[0]:
        wp = w.copy(); wp[k] += eps
        wm = w.copy(); wm[k] -= eps
        fd[k] = (oracle.primal(p, wp, steps)["J"] - oracle.primal(p, wm, steps)["J"]) / (2 * eps)
    assert np.max(np.abs(fd - g)) < 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("flow", [9, 19])
def test_plate_step_adjoint_dot_product(flow):
    """One step with plate nodes: the adjoint step is the transpose of the tangent step."""
    p = _case(flow)
    n = p["nx"] * p["ny"] * p["nz"]
    w = inputs.porosity(p["nx"], p["ny"], p["nz"], 0, 3)
    r = oracle.primal(p, w, 20)
    rng = np.random.default_rng(8)
    df, dg = rng.standard_normal(r["f"].shape), rng.standard_normal(r["g"].shape)
    lf, lg = rng.standard_normal(r["f"].shape), rng.standard_normal(r["g"].shape)
    dw = rng.standard_normal(n)
    tf, tg = oracle.step_tangent(p, w, r["f"], r["g"], df, dg, dw)
    af, ag, gw = oracle.step_adjoint(p, w, r["f"], r["g"], lf, lg)
    lhs = np.sum(tf * lf) + np.sum(tg * lg)
    rhs = np.sum(df * af) + np.sum(dg * ag) + np.sum(dw * gw)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
