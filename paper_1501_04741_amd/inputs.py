"""Seeded synthetic inputs: design fields, workload presets, request traces.

This module holds no arithmetic of the method itself.  It produces inputs that
both the GPU path and the CPU oracle consume: porosity/design fields ``w``
(uniform random in [0, 1), smoothed by a periodic box filter), the parameter
dicts of the named workloads, and Poisson request traces for the serving loop.

A design field is shaped ``(nz, ny, nx)`` and flattened with x fastest,
matching the node index ``n = x + nx*(y + ny*z)`` both implementations use.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import product

import numpy as np


def porosity(nx: int, ny: int, nz: int, seed: int, k: int, dtype=np.float64) -> np.ndarray:
    """Random design field in [0, 1): uniform draws smoothed by a k-wide box.

    Draws ``rng.random((nz, ny, nx))`` from PCG64(seed), then averages over the
    k x k (2D, over y and x) or k x k x k (3D) neighbourhood with periodic wrap,
    adding the offsets in the fixed order -k//2 .. k//2 per axis, and finally
    casts to ``dtype``.  Returned flat, x fastest.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w0 = rng.random((nz, ny, nx))
    r = k // 2
    axes = (1, 2) if nz == 1 else (0, 1, 2)
    acc = np.zeros_like(w0)
    for off in product(range(-r, r + 1), repeat=len(axes)):
        acc += np.roll(w0, shift=tuple(-o for o in off), axis=axes)
    w = acc / float(k ** len(axes))
    return np.ascontiguousarray(w.reshape(-1).astype(dtype))


# --------------------------------------------------------------------------
# Workload presets.  Keys are the configuration keys shared by the GPU binding
# and the oracle wrapper; "steps", "precision", "filter", "seed" and
# "checkpoint_interval" describe the run, not the model.
_CHANNEL = dict(tau=0.8, rho_out=1.0, switch_fn="ramp", switch_param=0.01, periodic=0)

WORKLOADS = {
    # D2Q9 BGK + Brinkman, 64x32 channel, pressure drop, FP64
    "d2q9_channel_64x32": dict(
        _CHANNEL, flow=9, scalar=0, nx=64, ny=32, nz=1, u_in=0.01, c_dp=1.0, c_hf=0.0, c_var=0.0,
        steps=1000, precision="fp64", filter=3, seed=0, checkpoint_interval=0),
    # D2Q9 flow + D2Q5 temperature, 512x256 heat-exchanger channel:
    # hot walls T=1, inlet T=0, J = outlet heat flux - 0.1 x pressure drop
    "d2q9_d2q5_exchanger_512x256": dict(
        _CHANNEL, flow=9, scalar=5, nx=512, ny=256, nz=1, u_in=0.01, tau_s=0.6,
        scalar_wall="dirichlet", s_wall=1.0, s_in_lo=0.0, s_in_hi=0.0, s_split_axis=0,
        c_dp=-0.1, c_hf=1.0, c_var=0.0, steps=20000, precision="fp32", filter=3, seed=0,
        checkpoint_interval=500),
    # D3Q19 flow + D3Q7 scalar mixer, 128x64x64 duct: inlet split on y
    # (0 below ny/2, 1 at and above), J = outlet variance + 0.1 x pressure drop
    "d3q19_d3q7_mixer_128x64x64": dict(
        _CHANNEL, flow=19, scalar=7, nx=128, ny=64, nz=64, u_in=0.02, tau_s=0.6,
        scalar_wall="adiabatic", s_in_lo=0.0, s_in_hi=1.0, s_split_axis=1,
        c_dp=0.1, c_hf=0.0, c_var=1.0, steps=5000, precision="fp32", filter=5, seed=0,
        checkpoint_interval=0),
    # D3Q19 Brinkman channel 256x128x128 (4.19M nodes), J = pressure drop; the
    # 160 GB budget holds the moments of all 2000 steps (no recompute)
    "d3q19_channel_256x128x128": dict(
        _CHANNEL, flow=19, scalar=0, nx=256, ny=128, nz=128, u_in=0.02, c_dp=1.0, c_hf=0.0, c_var=0.0,
        steps=2000, precision="fp32", filter=5, seed=0, checkpoint_interval=0, hbm_budget_gb=160),
    # The paper's mixing duct without obstacles (Section 4, table of settings):
    # 450x50x50, pressure drop 0.016666 (rho_in = 1 + 3 dp) with the inlet velocity
    # limited to 0.05, nu = 0.02 (tau = 3 nu + 1/2), scalar diffusivity 0.003
    # (D3Q7, c^2 = 1/4: tau_s = 0.003/0.25 + 1/2), inlet scalar -1 below y = 25
    # and 1 from there on, adiabatic walls, J = outlet mixing flux; w = 1 (all fluid).
    "d3q19_d3q7_mixer_empty_450x50x50": dict(
        _CHANNEL, flow=19, scalar=7, nx=450, ny=50, nz=50, tau=0.56, tau_s=0.512, inlet="pressure",
        rho_in=1.0 + 3 * 0.016666, u_cap=0.05, u_in=0.0, scalar_wall="adiabatic", s_in_lo=-1.0, s_in_hi=1.0,
        s_split_axis=1, c_dp=0.0, c_hf=0.0, c_var=0.0, c_mix=1.0, steps=40000, precision="fp32", design="fluid",
        seed=0, checkpoint_interval=0),
    # The paper's heat-exchanger duct without obstacles (Section 4): 352x50x50,
    # pressure drop 0.03 (rho_in = 1 + 3 dp) with the inlet velocity limited to 0.05,
    # scalar diffusivity 0.003 in the fluid and 1 in the solid (D3Q7, c^2 = 1/4:
    # tau_s = alpha/c^2 + 1/2), inlet T = 0, adiabatic walls but for the D x D
    # heating plate at T = 1 in the middle of the bottom wall (x = 151 .. 200,
    # centred on the 352-node duct), J = outlet heat flux sum u_x T (eq.
    # exchanger:obj); w = 1 (all fluid); 3e4 iterations as printed.  The viscosity
    # is the mixer's nu = 0.02 (tau = 0.56): at the exchanger's nu = 0.01
    # (tau = 0.53) the Zou-He inlet and outlet nodes diverge within a few thousand
    # steps (with BGK or MRT interiors, in FP32 and FP64).
    "d3q19_d3q7_exchanger_empty_352x50x50": dict(
        _CHANNEL, flow=19, scalar=7, nx=352, ny=50, nz=50, tau=0.56, tau_s=0.512, tau_s_solid=4.5,
        inlet="pressure", rho_in=1.0 + 3 * 0.03, u_cap=0.05, u_in=0.0, scalar_wall="adiabatic", s_in_lo=0.0,
        s_in_hi=0.0, s_split_axis=0, plate_x0=151, plate_x1=201, s_plate=1.0, c_dp=0.0, c_hf=1.0, c_var=0.0,
        c_mix=0.0, steps=30000, precision="fp32", design="fluid", seed=0, checkpoint_interval=0),
}

# Request sizes of the serving stream (drawn uniformly).
SERVE_SIZES = (
    dict(_CHANNEL, flow=9, scalar=0, nx=256, ny=128, nz=1, u_in=0.01, filter=3),
    dict(_CHANNEL, flow=9, scalar=0, nx=1024, ny=512, nz=1, u_in=0.01, filter=3),
    dict(_CHANNEL, flow=19, scalar=0, nx=96, ny=48, nz=48, u_in=0.02, filter=5),
    dict(_CHANNEL, flow=19, scalar=0, nx=192, ny=96, nz=96, u_in=0.02, filter=5),
)

RUN_KEYS = ("steps", "precision", "filter", "seed", "checkpoint_interval", "hbm_budget_gb", "design")


def model_params(workload: dict) -> dict:
    """The model keys of a workload (drops the run-description keys)."""
    return {k: v for k, v in workload.items() if k not in RUN_KEYS}


def workload(name: str, **overrides) -> dict:
    w = dict(WORKLOADS[name])
    w.update(overrides)
    return w


def design_for(wl: dict, dtype=None) -> np.ndarray:
    """The seeded design field of a workload, in its run precision ("design":
    "fluid" is the empty channel, w = 1 everywhere)."""
    if dtype is None:
        dtype = np.float32 if wl.get("precision", "fp64") == "fp32" else np.float64
    if wl.get("design") == "fluid":
        return np.ones(wl["nx"] * wl["ny"] * wl["nz"], dtype)
    return porosity(wl["nx"], wl["ny"], wl["nz"], wl.get("seed", 0), wl.get("filter", 3), dtype)


@dataclass
class Request:
    rid: int
    arrival_s: float
    params: dict       # model keys
    steps: int
    seed: int


def poisson_trace(n_requests: int, rate_per_s: float, seed: int = 1, steps: int = 2000,
                  sizes=SERVE_SIZES) -> list:
    """Poisson arrivals (exponential gaps, mean 1/rate) with uniformly drawn sizes.

    Request r carries design seed r; its field is ``porosity(..., seed=r)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    kinds = rng.integers(0, len(sizes), size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        p = dict(sizes[int(kinds[r])])
        p.pop("filter")
        out.append(Request(rid=r, arrival_s=float(t[r]), params=dict(p, c_dp=1.0, c_hf=0.0, c_var=0.0),
                           steps=steps, seed=r))
    return out


def request_design(req: Request, dtype=np.float32) -> np.ndarray:
    p = req.params
    k = 3 if p["flow"] == 9 else 5
    return porosity(p["nx"], p["ny"], p["nz"], req.seed, k, dtype)
