"""Pins of the oracle's time-averaged objective (n_avg): J is the mean of the
node-sum objective (eq. objective:function) over the last n_avg states of the
run, so its adjoint adds (1/n_avg) dPhi/df^n at every step of that window.

Fixed from outside the oracle's windowed code: the windowed J equals the mean of
separate single-state runs of N - k steps; the windowed gradient equals the mean
of the single-state gradients of those runs (the adjoint is linear in its
sources); and complex-step directional derivatives and central differences of
the whole windowed run."""
import numpy as np
import pytest

import oracle
from paper_1501_04741_amd import inputs


def _case(flow, scalar, **kw):
    if flow == 19:
        p = dict(flow=19, scalar=scalar, nx=10, ny=6, nz=5)
    else:
        p = dict(flow=9, scalar=scalar, nx=16, ny=8, nz=1)
    p.update(tau=0.8, tau_s=0.6, u_in=0.02, switch_fn="power", switch_param=3.0, c_dp=0.1)
    if scalar:
        p.update(c_var=1.0, c_hf=0.4, s_in_lo=0.0, s_in_hi=1.0, s_split_axis=1)
    p.update(kw)
    return p


CASES = [_case(9, 0), _case(9, 5), _case(19, 7, inlet="pressure", rho_in=1.02, u_cap=0.012, c_mix=1.0,
                                             s_in_lo=-1.0)]


@pytest.mark.parametrize("p", CASES, ids=["d2q9", "d2q9_d2q5_var", "d3q19_d3q7_pressure_mix"])
def test_window_objective_and_gradient_are_means_of_single_state_runs(p):
    N, W = 40, 7
    w = inputs.porosity(p["nx"], p["ny"], p["nz"], 2, 3)
    pw = dict(p, n_avg=W)
    single = [oracle.adjoint(p, w, N - k) for k in range(W)]
    J_mean = np.mean([r["J"] for r in single])
    g_mean = np.mean([r["grad"] for r in single], axis=0)
    assert abs(oracle.primal(pw, w, N)["J"] - J_mean) <= 1e-14 * abs(J_mean)
    a = oracle.adjoint(pw, w, N)
    assert abs(a["J"] - J_mean) <= 1e-14 * abs(J_mean)
    assert np.linalg.norm(a["grad"] - g_mean) <= 1e-12 * np.linalg.norm(g_mean)
    # n_avg = 1 (and 0) is the final state alone, bitwise
    for n1 in (0, 1):
        b = oracle.adjoint(dict(p, n_avg=n1), w, N)
        assert b["J"] == single[0]["J"] and np.array_equal(b["grad"], single[0]["grad"])


@pytest.mark.parametrize("p", CASES[1:], ids=["d2q9_d2q5_var", "d3q19_d3q7_pressure_mix"])
def test_window_adjoint_vs_complex_step(p):
    N, W = 50, 12
    pw = dict(p, n_avg=W)
    w = inputs.porosity(p["nx"], p["ny"], p["nz"], 3, 3)
    dw = np.random.default_rng(5).standard_normal(w.size)
    a = oracle.adjoint(pw, w, N)
    J, dJ = oracle.directional(pw, w, dw, N)
    assert abs(a["J"] - J) <= 1e-14 * abs(J)
    assert abs(a["grad"] @ dw - dJ) <= 1e-12 * abs(dJ)


def test_window_adjoint_vs_central_differences():
    p = dict(CASES[1], n_avg=9)
    N = 60
    w = inputs.porosity(16, 8, 1, 4, 3)
    g = oracle.adjoint(p, w, N)["grad"]
    eps = 1e-5
    for k in np.nonzero(oracle.mask(p) == 0)[0][::5]:
        wp = w.copy(); wp[k] += eps
        wm = w.copy(); wm[k] -= eps
        fd = (oracle.primal(p, wp, N)["J"] - oracle.primal(p, wm, N)["J"]) / (2 * eps)
        assert abs(fd - g[k]) < 1e-6 * np.abs(g).max()


def test_window_longer_than_the_run_is_rejected():
    p = dict(CASES[0], n_avg=11)
    w = np.full(128, 0.7)
    with pytest.raises(ValueError):
        oracle.primal(p, w, 10)
    with pytest.raises(ValueError):
        oracle.adjoint(p, w, 10)
    assert np.isfinite(oracle.primal(p, w, 11)["J"])
