"""Writes the oracle's whole-run results for the FP32 workloads to tests/golden/.

Calls only the FP64 CPU oracle (``oracle``) and the seeded input generators
(``paper_1501_04741_amd.inputs``, which hold none of the method's arithmetic);
nothing here touches the GPU library.  Each file holds the objective J and the
gradient dJ/dw of the unsteady discrete adjoint (Section 2.2, eq.
adjoint:derivative, summed over every step) for the workload's own seeded
design field, rounded to FP32 as the GPU run receives it.

  exchanger  D2Q9+D2Q5 512x256, 20000 steps: J and the full gradient
  mixer      D3Q19+D3Q7 128x64x64, 5000 steps: J and the full gradient
  channel    D3Q19 256x128x128 at 200 steps (the full 2000-step horizon needs
             more host memory than the oracle's square-root checkpointing can
             spare): J, the gradient at 8192 interior nodes drawn with
             PCG64(0), and the L2 norm of the full gradient

With "fields" before the case, it stores instead the oracle's macroscopic
fields after the workload's full forward horizon (no adjoint; for the channel
the whole 2000 steps): the velocity and the scalar at 16384 nodes drawn with
PCG64(1) from all nodes, their largest magnitudes over the whole lattice, and
J.  These pin the FP32 velocity over the full horizon (relative to the largest
velocity, bar 1e-4).

With "serving" it stores J and the gradient (its norm and 4096 sampled interior
nodes) of the first request of each size in the benchmark's serving trace.

With "directional" it stores J and the complex-step directional derivative
dJ/dw . v of the benchmark channel over its full 2000 steps (v: standard normal
values from PCG64(2)).

Usage: python tests/golden/make_oracle_goldens.py [fields] {exchanger|mixer|channel|serving|directional} [threads]
Run time on 8 host cores: about 50 min, 2-3 h and 35 min; fields about 10,
15 and 30 min.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1501_04741_amd import inputs  # noqa: E402

CASES = {
    "exchanger": dict(workload="d2q9_d2q5_exchanger_512x256", steps=None, sample=0),
    "mixer": dict(workload="d3q19_d3q7_mixer_128x64x64", steps=None, sample=0),
    "channel": dict(workload="d3q19_channel_256x128x128", steps=200, sample=8192),
}


def golden_path(case: str) -> str:
    return os.path.join(HERE, "oracle_%s.npz" % CASES[case]["workload"])


def fields_path(case: str) -> str:
    return os.path.join(HERE, "oracle_fields_%s.npz" % CASES[case]["workload"])


def make_fields(case: str) -> str:
    """Macroscopic fields of the oracle's forward run over the workload's horizon."""
    spec = CASES[case]
    wl = inputs.workload(spec["workload"])
    p = inputs.model_params(wl)
    steps = int(wl["steps"])
    w = inputs.design_for(wl).astype(np.float64)
    t0 = time.time()
    r = oracle.primal(p, w, steps)
    secs = time.time() - t0
    rho, u, T = oracle.fields(p, r["f"], r["g"])
    n = rho.size
    idx = np.sort(np.random.Generator(np.random.PCG64(1)).choice(n, size=16384, replace=False)).astype(np.int64)
    out = dict(workload=np.array(spec["workload"]), steps=np.int64(steps), J=np.float64(r["J"]), idx=idx,
               u=u[:, idx], T=T[idx], rho=rho[idx], u_max=np.float64(np.abs(u).max()),
               T_max=np.float64(np.abs(T).max()), seconds=np.float64(secs), threads=np.int64(oracle.threads()))
    path = fields_path(case)
    np.savez_compressed(path, **out)
    print("fields %s: %s, %d steps, J = %.12g, max|u| = %.6g, %.0f s on %d threads" % (
        case, spec["workload"], steps, r["J"], out["u_max"], secs, out["threads"]), flush=True)
    return path


def directional_path() -> str:
    return os.path.join(HERE, "oracle_directional_d3q19_channel_256x128x128.npz")


def direction(n: int) -> np.ndarray:
    """The seeded direction of the whole-horizon directional derivative."""
    return np.random.Generator(np.random.PCG64(2)).standard_normal(n)


def make_directional() -> str:
    """J and dJ/dw . v of the benchmark channel over its full 2000 steps, by complex
    step through the whole run (exact up to rounding), for the seeded direction v:
    the gradient's projection at the horizon the adjoint golden cannot reach."""
    wl = inputs.workload("d3q19_channel_256x128x128")
    p = inputs.model_params(wl)
    steps = int(wl["steps"])
    w = inputs.design_for(wl).astype(np.float64)
    v = direction(w.size)
    t0 = time.time()
    J, dJ = oracle.directional(p, w, v, steps)
    secs = time.time() - t0
    path = directional_path()
    np.savez_compressed(path, workload=np.array("d3q19_channel_256x128x128"), steps=np.int64(steps), J=np.float64(J),
                        dJ_v=np.float64(dJ), direction_seed=np.int64(2), seconds=np.float64(secs),
                        threads=np.int64(oracle.threads()))
    print("directional: %d steps, J = %.12g, dJ.v = %.12g, %.0f s" % (steps, J, dJ, secs), flush=True)
    return path


def serving_path() -> str:
    return os.path.join(HERE, "oracle_serving_requests.npz")


# Horizon of the serving golden per request size: the trace's 2000 steps, but
# 200 for D3Q19 192x96x96, whose 2000-step oracle adjoint would take hours.
SERVING_STEPS = (2000, 2000, 2000, 200)


def serving_requests():
    """The first request of each size in the benchmark's 400-request trace
    (Poisson 20/s, seed 1), with the horizon the golden holds for it."""
    trace = inputs.poisson_trace(400, 20.0, seed=1)
    out = []
    for kind, size in enumerate(inputs.SERVE_SIZES):
        req = next(r for r in trace if (r.params["flow"], r.params["nx"]) == (size["flow"], size["nx"]))
        out.append((kind, req, SERVING_STEPS[kind]))
    return out


def make_serving() -> str:
    """J and dJ/dw of the oracle for one request of each serving size: the
    gradient's norm and its values at 4096 interior nodes drawn with PCG64(0)."""
    rows = dict(rid=[], kind=[], steps=[], J=[], grad_norm=[], sample_idx=[], grad_sample=[], seconds=[])
    for kind, req, steps in serving_requests():
        p = req.params
        w = inputs.request_design(req).astype(np.float64)  # the FP32 field the GPU receives
        t0 = time.time()
        r = oracle.adjoint(p, w, steps)
        secs = time.time() - t0
        idx = sample_nodes(p, 4096)
        for k, v in (("rid", req.rid), ("kind", kind), ("steps", steps), ("J", r["J"]),
                     ("grad_norm", np.linalg.norm(r["grad"])), ("sample_idx", idx), ("grad_sample", r["grad"][idx]),
                     ("seconds", secs)):
            rows[k].append(v)
        print("serving request %d (size %d, %s %dx%dx%d): %d steps, J = %.12g, %.0f s" % (
            req.rid, kind, "D3Q19" if p["flow"] == 19 else "D2Q9", p["nx"], p["ny"], p["nz"], steps, r["J"], secs),
            flush=True)
    path = serving_path()
    np.savez_compressed(path, threads=np.int64(oracle.threads()), **{k: np.array(v) for k, v in rows.items()})
    return path


def sample_nodes(params: dict, count: int) -> np.ndarray:
    """Sorted indices of `count` distinct interior nodes, drawn with PCG64(0)."""
    interior = np.flatnonzero(oracle.mask(params) == 0)
    rng = np.random.Generator(np.random.PCG64(0))
    return np.sort(rng.choice(interior, size=count, replace=False)).astype(np.int64)


def make(case: str) -> str:
    spec = CASES[case]
    wl = inputs.workload(spec["workload"])
    p = inputs.model_params(wl)
    steps = spec["steps"] or wl["steps"]
    w = inputs.design_for(wl).astype(np.float64)  # the FP32-rounded field the GPU run receives
    t0 = time.time()
    r = oracle.adjoint(p, w, steps)
    secs = time.time() - t0
    grad = r["grad"]
    out = dict(workload=np.array(spec["workload"]), steps=np.int64(steps), J=np.float64(r["J"]),
               grad_norm=np.float64(np.linalg.norm(grad)), seconds=np.float64(secs),
               threads=np.int64(oracle.threads()))
    if spec["sample"]:
        idx = sample_nodes(p, spec["sample"])
        out.update(sample_idx=idx, grad_sample=grad[idx])
    else:
        out.update(grad=grad)
    path = golden_path(case)
    np.savez_compressed(path, **out)
    print("%s: %s, %d steps, J = %.12g, |grad| = %.6g, %.0f s on %d threads" % (
        case, spec["workload"], steps, r["J"], out["grad_norm"], secs, out["threads"]), flush=True)
    return path


if __name__ == "__main__":
    args = sys.argv[1:]
    fields = bool(args) and args[0] == "fields"
    if fields:
        args = args[1:]
    if len(args) > 1:
        oracle.threads(int(args[1]))
    if args[0] == "serving":
        make_serving()
    elif args[0] == "directional":
        make_directional()
    else:
        (make_fields if fields else make)(args[0])
