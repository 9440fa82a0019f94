"""Benchmark: one design evaluation (J and dJ/dw) of the adjoint LBM hot path.

A bench step is the whole hot path over one design field: set the design,
reset, N recorded primal steps, objective, N adjoint steps and the gradient
export.  Default workload: the D3Q19 Brinkman channel 256x128x128 (4.19M
nodes), N = 2000, FP32, in the plan the 160 GB budget allows: every step's
moments held (store-all), so the timed backward recomputes nothing.  The
fixed-interval checkpoint plan, whose backward recomputes every trajectory
segment, is timed in the ``recompute`` leg.

Prints ONE JSON line.  ``value`` is the gradient-evaluation throughput in
MLUPS: lattice nodes x primal steps differentiated per second (forward and
adjoint inside the timed region).  Kernel-level figures come from HIP events
recorded on the library's stream inside the timed steps: the primal kernel
over the N forward launches, the adjoint kernel over the launches of the last
trajectory segment (which needs no recompute).  The same line carries the
serving measurement (a Poisson trace of design-evaluation requests through
the continuous-batching server and, on the same GPU, one request at a time)
and the CPU oracle timed on bounded samples of the configured workloads.

Only one GPU is supported: ``--gpus N`` with N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "primal/adjoint MLUPS + HBM roofline frac; served gradients/s, p50/p99 ms"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE, each scaled by what the
# counter reads for a 1 GiB device copy in the same run, per workload and kernel.  The figures hold
# for the kernel sources, host dispatch and compile flags whose SHA-256 prefix is given and are
# reported only while those files still match.
COUNTER_TRAFFIC = {
    "sources_sha256_16": "0c1888759bfd6b07",
    "bytes_per_launch": {
        "d3q19_batch_8x128x96x96": {
            "k_adjoint_batch<19,0,float,in place>": 1687919265,
            "k_adjoint_batch<19,0,float,ping-pong>": 1687932075,
            "k_primal_batch<19,0,float,in place,recorded>": 1615575058,
            "k_primal_batch<19,0,float,ping-pong,recorded>": 1615607431
        },
        "d3q19_channel_256x128x128": {
            "k_adjoint<19,0,float>": 751457705,
            "k_adjoint_inplace<19,0,double>": 1502780745,
            "k_adjoint_inplace<19,0,float,MRT>": 751799323,
            "k_adjoint_inplace<19,0,float>": 751456539,
            "k_oneshot_inplace<19,0,float>": 1324587485,
            "k_primal<19,0,float,recorded>": 718939932,
            "k_primal<19,0,float,unrecorded>": 653906601,
            "k_primal_inplace<19,0,double,recorded>": 1437787838,
            "k_primal_inplace<19,0,float,MRT,recorded>": 719388548,
            "k_primal_inplace<19,0,float,recorded>": 718947258,
            "k_primal_inplace<19,0,float,unrecorded>": 653902865
        },
        "d3q19_d3q7_mixer_empty_450x50x50": {
            "k_oneshot<19,7,float>": 515547366,
            "k_oneshot_inplace<19,7,float>": 512695024,
            "k_primal<19,7,float,unrecorded>": 255639950,
            "k_primal_inplace<19,7,float,unrecorded>": 253450985
        }
    }
}
_COUNTER_SOURCES = ("paper_1501_04741_amd/csrc/kernels.hpp", "paper_1501_04741_amd/csrc/lattice.hpp",
                    "paper_1501_04741_amd/csrc/lbm_adj.hip", "paper_1501_04741_amd/build.py")


def sources_sha():
    """Hash of the code (comments and blank space dropped) that decides what the
    profiled kernels do: the kernels, the host dispatch and the build flags."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in _COUNTER_SOURCES:
        text = open(os.path.join(ROOT, rel)).read()
        if rel.endswith(".py"):
            text = re.sub(r"(?m)^\s*#.*$", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()[:16]


def _measured_traffic(workload, kernel):
    if sources_sha() != COUNTER_TRAFFIC["sources_sha256_16"]:
        return None
    return COUNTER_TRAFFIC["bytes_per_launch"].get(workload, {}).get(kernel)


def klabel(family, p, prec, mode=""):
    """Label of a kernel variant in the bench line, and the key of its counter
    traffic: the kernel family with lattice, precision, collision and mode
    ("recorded" / "unrecorded" for the primal kernels, "in place" / "ping-pong"
    for the batched ones), e.g. k_primal_inplace<19,0,float,recorded>."""
    parts = [str(p["flow"]), str(p.get("scalar", 0)), "float" if prec == "fp32" else "double"]
    if p.get("collision") == "mrt":
        parts.append("MRT")
    if p.get("tau_s_solid"):
        parts.append("VD")
    if mode:
        parts.append(mode)
    return "%s<%s>" % (family, ",".join(parts))


def _class_counts(p):
    """Node counts per class for a channel (interior, wall, inlet, outlet)."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    if p.get("periodic"):
        return nx * ny * nz, 0, 0, 0
    rows_fluid = (ny - 2) * (nz - 2 if p["flow"] == 19 else 1)
    rows_total = ny * nz
    wall = (rows_total - rows_fluid) * nx
    return rows_fluid * (nx - 2), wall, rows_fluid, rows_fluid


def moment_values(p):
    """Values per node the recorded primal keeps for the adjoint: rho, u and the
    scalar sum, or all scalar populations when the diffusivity is blended."""
    qs = p.get("scalar", 0)
    blended = qs and p.get("tau_s_solid", 0.0) not in (0.0, p.get("tau_s", 0.6))
    return (3 if p["flow"] == 19 else 2) + 1 + ((qs if blended else 1) if qs else 0)


def primal_bytes(p, precision, recorded=True):
    """Bytes one primal launch must move, by node class: interior 2*Qt*s + s (pull Qt,
    store Qt, read w), other classes 2*Qt*s; a recorded launch also writes the M
    moments the adjoint needs at interior, outlet and pressure-inlet nodes."""
    s = 4 if precision == "fp32" else 8
    qt = p["flow"] + p.get("scalar", 0)
    m = moment_values(p) if recorded else 0
    m_in = m if p.get("inlet") == "pressure" else 0
    ni, nw, nin, nout = _class_counts(p)
    return ni * (2 * qt * s + s + m * s) + nout * (2 * qt * s + m * s) + nin * (2 * qt * s + m_in * s) + nw * 2 * qt * s


def algorithmic_bytes(p, precision):
    """Bytes one recorded primal launch and one adjoint launch must move, by node class.

    primal (recorded): see primal_bytes.
    adjoint: interior 2*Qt*s + M*s + 3s (cotangent pull, store, moments, w, grad
             read+write); outlet and pressure inlet 2*Qt*s + M*s; velocity inlet and
             wall 2*Qt*s (their transposed Jacobians do not depend on the primal state)."""
    s = 4 if precision == "fp32" else 8
    qt = p["flow"] + p.get("scalar", 0)
    m = moment_values(p)
    m_in = m if p.get("inlet") == "pressure" else 0
    ni, nw, nin, nout = _class_counts(p)
    adjoint = ni * (2 * qt * s + m * s + 3 * s) + nout * (2 * qt * s + m * s) + nin * (2 * qt * s + m_in * s) + \
        nw * 2 * qt * s
    return primal_bytes(p, precision, True), adjoint


def oneshot_bytes(p, precision):
    """Bytes one fused one-shot launch must move: every node pulls and stores its
    state and adjoint state (4*Qt*s) and writes its gradient estimate (s);
    interior nodes also read and write the design value (2s)."""
    s = 4 if precision == "fp32" else 8
    qt = p["flow"] + p.get("scalar", 0)
    ni, nw, nin, nout = _class_counts(p)
    return ni * (4 * qt * s + 3 * s) + (nw + nin + nout) * (4 * qt * s + s)


def mixer_leg(dev, steps=4000, os_iters=400):
    """Forward steps and one-shot iterations on the paper's mixing duct (450x50x50
    D3Q19 + D3Q7, pressure inlet with velocity limit, mixing objective), FP32:
    ping-pong and in place; the one-shot iteration streams in place (one primal
    and one adjoint buffer), the ping-pong one-shot is reported beside it."""
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.lbm import Lbm

    wl = inputs.workload("d3q19_d3q7_mixer_empty_450x50x50")
    p = inputs.model_params(wl)
    w = torch.from_numpy(inputs.design_for(wl)).to(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    P = Lbm(p, nsteps=0, precision="fp32", device=dev)
    P.set_design(w)
    P.reset()
    P.primal_steps(200)
    ev[0].record()
    P.primal_steps(steps)
    ev[1].record()
    torch.cuda.synchronize()
    P.close()
    O = Lbm(p, nsteps=0, precision="fp32", device=dev)
    O.set_design(w)
    O.reset()
    O.oneshot_steps(20, 0.0, 0.0)
    ev[2].record()
    O.oneshot_steps(os_iters, 0.0, 0.0)
    ev[3].record()
    torch.cuda.synchronize()
    O.close()
    I = Lbm(p, nsteps=0, precision="fp32", device=dev, inplace=True)
    I.set_design(w)
    I.reset()
    I.primal_steps(200)
    ei = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ei[2].record()
    I.primal_steps(steps)
    ei[3].record()
    I.reset()
    I.oneshot_steps(20, 0.0, 0.0)
    ei[0].record()
    I.oneshot_steps(os_iters, 0.0, 0.0)
    ei[1].record()
    torch.cuda.synchronize()
    I.close()
    nodes = p["nx"] * p["ny"] * p["nz"]
    prim_us = ev[0].elapsed_time(ev[1]) * 1e3 / steps
    os_us = ev[2].elapsed_time(ev[3]) * 1e3 / os_iters
    osi_us = ei[0].elapsed_time(ei[1]) * 1e3 / os_iters
    pi_us = ei[2].elapsed_time(ei[3]) * 1e3 / steps
    pb, ob = primal_bytes(p, "fp32", recorded=False), oneshot_bytes(p, "fp32")
    wk = "d3q19_d3q7_mixer_empty_450x50x50"
    roof = lambda b, us, k: {"bound": "hbm", "achieved": b / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": b,
                             "avg_launch_us": us, "traffic": _measured_traffic(wk, k)}
    kp = klabel("k_primal", p, "fp32", "unrecorded")
    kpi = klabel("k_primal_inplace", p, "fp32", "unrecorded")
    ko = klabel("k_oneshot", p, "fp32")
    koi = klabel("k_oneshot_inplace", p, "fp32")
    return {"workload": wk, "nodes": nodes,
            "primal": {"kernel": kp, "steps_timed": steps, "mlups": nodes / prim_us, "roofline": roof(pb, prim_us, kp)},
            "oneshot": {"kernel": koi, "iterations_timed": os_iters,
                        "mlups": nodes / osi_us, "roofline": roof(ob, osi_us, koi)},
            "primal_inplace": {"kernel": kpi, "steps_timed": steps, "mlups": nodes / pi_us,
                               "roofline": roof(pb, pi_us, kpi)},
            "oneshot_ping_pong": {"kernel": ko, "iterations_timed": os_iters,
                                  "mlups": nodes / os_us, "roofline": roof(ob, os_us, ko)},
            "note": "two primal states (234 MB) fit the 256 MB last-level cache; the ping-pong one-shot's four "
                    "do not, the in-place one-shot's two do"}


def mrt_leg(dev, steps=200, collision="mrt", inplace=True, prec="fp32"):
    """Recorded primal and adjoint launches of the 256x128x128 D3Q19 channel,
    all moments held: with the forced MRT interior collision (d'Humieres
    rates), or with BGK and ping-pong buffers, or in FP64, for comparison."""
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.lbm import Lbm

    wl = inputs.workload("d3q19_channel_256x128x128")
    p = dict(inputs.model_params(wl), collision=collision)
    w = torch.from_numpy(inputs.design_for(wl)).to(dev)
    if prec == "fp64":
        w = w.double()
    if inplace:
        L = Lbm(p, nsteps=steps, precision=prec, device=dev, inplace=True)
    else:
        L = Lbm(p, nsteps=steps, precision=prec, checkpoint_interval=steps, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for rep_ in range(2):  # the second pass is timed
        L.set_design(w)
        L.reset()
        ev[0].record()
        L.primal_steps(steps, record=True)
        ev[1].record()
        L.adjoint_steps(1)
        ev[2].record()
        L.adjoint_steps(steps - 1)
        ev[3].record()
    torch.cuda.synchronize()
    L.close()
    prim_us = ev[0].elapsed_time(ev[1]) * 1e3 / steps
    adj_us = ev[2].elapsed_time(ev[3]) * 1e3 / (steps - 1)
    pb, ab = algorithmic_bytes(p, prec)
    nodes = p["nx"] * p["ny"] * p["nz"]
    roof = lambda b, us: {"bound": "hbm", "achieved": b / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": b, "avg_launch_us": us}
    sfx = "_inplace" if inplace else ""
    wk = "d3q19_channel_256x128x128"
    kp = klabel("k_primal" + sfx, p, prec, "recorded")
    ka = klabel("k_adjoint" + sfx, p, prec)
    return {"workload": "%s, %s collision, %s, %s" % (
                wk, collision.upper(), "in place" if inplace else "ping-pong", prec.upper()),
            "steps_timed": steps,
            "primal": {"kernel": kp, "mlups": nodes / prim_us,
                       "roofline": dict(roof(pb, prim_us), traffic=_measured_traffic(wk, kp))},
            "adjoint": {"kernel": ka, "mlups": nodes / adj_us,
                        "roofline": dict(roof(ab, adj_us), traffic=_measured_traffic(wk, ka))}}


def recompute_leg(dev, workload="d3q19_channel_256x128x128", inplace=True):
    """The fixed-interval checkpoint plan of the 256x128x128 channel (N = 2000,
    FP32): the checkpoint interval C that minimises the workspace.  The recorded
    forward keeps a full state every C steps and the moments of the last
    segment; the backward recomputes every other segment from its checkpoint
    before reversing it.  In place: one working buffer (copied to a checkpoint
    every C steps) and one adjoint buffer, segments recomputed in place inside
    their checkpoint; ping-pong: two of each.  One warm-up evaluation, one timed."""
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.lbm import Lbm

    wl = inputs.workload(workload)
    p = inputs.model_params(wl)
    N = int(wl["steps"])
    prec = wl["precision"]
    w = torch.from_numpy(inputs.design_for(wl)).to(dev)
    L = Lbm(p, nsteps=N, precision=prec, device=dev)  # the smallest ping-pong workspace
    plan = L.plan()
    C = plan["interval"]
    if inplace:  # the same interval, streamed in place
        L.close()
        L = Lbm(p, nsteps=N, precision=prec, checkpoint_interval=C, device=dev, inplace=True)
        plan = L.plan()
    k_last = N - ((N - 1) // C) * C
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    grad = torch.empty(L.N, dtype=L.dtype, device=dev)
    for rep_ in range(2):  # the second pass is timed
        L.set_design(w)
        L.reset()
        ev[0].record()
        L.primal_steps(N, record=True)
        ev[1].record()
        L.adjoint_steps(1)
        ev[2].record()
        L.adjoint_steps(k_last - 1)
        ev[3].record()
        L.adjoint_steps(N - k_last)
        ev[4].record()
        L.gradient(out=grad)
    torch.cuda.synchronize()
    ws = L.workspace_bytes
    L.close()
    nodes = L.N
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[1].elapsed_time(ev[4])
    prim_us = fwd_ms * 1e3 / N
    adj_us = ev[2].elapsed_time(ev[3]) * 1e3 / (k_last - 1)
    pb, ab = algorithmic_bytes(p, prec)
    recomputed = N - k_last  # every segment but the last is recomputed once
    bwd_bytes = N * ab + recomputed * pb
    roof = lambda b, us: {"bound": "hbm", "achieved": b / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": b, "avg_launch_us": us}
    sfx = "_inplace" if inplace else ""
    kp = klabel("k_primal" + sfx, p, prec, "recorded")
    ka = klabel("k_adjoint" + sfx, p, prec)
    return {"workload": "%s, checkpoint every %d steps (%d checkpoints, %d moment sets), %s" % (
                workload, C, plan["checkpoints"], plan["moment_sets"], "in place" if inplace else "ping-pong"),
            "lbm_steps": N, "checkpoint_interval": C, "workspace_gb": round(ws / 1e9, 3),
            "recomputed_steps": recomputed,
            "evaluation_mlups": nodes * N / ((fwd_ms + bwd_ms) * 1e-3) / 1e6,
            "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "forward_mlups": nodes * N / (fwd_ms * 1e-3) / 1e6,
            "backward_mlups": nodes * N / (bwd_ms * 1e-3) / 1e6,
            "backward_roofline": {"bound": "hbm", "achieved": bwd_bytes / (bwd_ms * 1e-3) / 1e9,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": bwd_bytes / (bwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "bytes": bwd_bytes,
                                  "note": "N adjoint launches + the recorded primal launches of the recompute"},
            "primal": {"kernel": kp, "mlups": nodes / prim_us,
                       "roofline": dict(roof(pb, prim_us), traffic=_measured_traffic(workload, kp))},
            "adjoint": {"kernel": ka, "mlups": nodes / adj_us,
                        "roofline": dict(roof(ab, adj_us), traffic=_measured_traffic(workload, ka))}}


def batched_leg(dev, n_ctx=8, steps=100):
    """Batched launches at HBM scale: n_ctx D3Q19 FP32 channels of 128x96x96 (90 MB
    state each, 0.7 GB per in-place step over eight of them), every step's
    moments held, advanced by one k_primal_batch / k_adjoint_batch launch per
    step, streamed in place (the serving form) and with ping-pong buffers; the
    same contexts one at a time with the single-context kernels for comparison."""
    import numpy as np
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd import lbm as L
    from paper_1501_04741_amd.lbm import Lbm

    p = dict(inputs.SERVE_SIZES[3], nx=128, ny=96, nz=96)
    p.pop("filter")
    p.update(c_dp=1.0, c_hf=0.0, c_var=0.0)
    ws = [torch.from_numpy(inputs.porosity(128, 96, 96, 100 + k, 5, np.float32)).to(dev) for k in range(n_ctx)]
    pb, ab = algorithmic_bytes(p, "fp32")
    roof = lambda b, us: {"bound": "hbm", "achieved": b / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": b, "avg_launch_us": us}
    key = "d3q19_batch_%dx128x96x96" % n_ctx
    out = {"workload": "%d x D3Q19 128x96x96 FP32 channels, %d recorded steps, every step's moments held" % (
        n_ctx, steps)}
    for inplace in (True, False):
        ctxs = [Lbm(p, nsteps=steps, precision="fp32", checkpoint_interval=steps, device=dev, inplace=inplace)
                for _ in range(n_ctx)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        h = [c.ctx for c in ctxs]
        for rep_ in range(2):  # the second pass is timed
            for c, w in zip(ctxs, ws):
                c.set_design(w)
                c.reset()
            ev[0].record()
            L.lbm_primal_steps_batch(h, steps, record=True)
            ev[1].record()
            L.lbm_adjoint_steps_batch(h, 1)
            ev[2].record()
            L.lbm_adjoint_steps_batch(h, steps - 1)
            ev[3].record()
        # the same work one context at a time (single-context kernels)
        for c, w in zip(ctxs, ws):
            c.set_design(w)
            c.reset()
        ev[4].record()
        for c in ctxs:
            c.primal_steps(steps, record=True)
        ev[5].record()
        torch.cuda.synchronize()
        for c in ctxs:
            c.close()
        prim_us = ev[0].elapsed_time(ev[1]) * 1e3 / steps
        adj_us = ev[2].elapsed_time(ev[3]) * 1e3 / (steps - 1)
        single_us = ev[4].elapsed_time(ev[5]) * 1e3 / (steps * n_ctx)
        mode = "in place" if inplace else "ping-pong"
        kp = klabel("k_primal_batch", p, "fp32", mode + ",recorded")
        ka = klabel("k_adjoint_batch", p, "fp32", mode)
        r = {"primal": {"kernel": kp, "roofline": dict(roof(n_ctx * pb, prim_us), traffic=_measured_traffic(key, kp))},
             "adjoint": {"kernel": ka, "roofline": dict(roof(n_ctx * ab, adj_us), traffic=_measured_traffic(key, ka))},
             "primal_single_context": {
                 "kernel": klabel("k_primal_inplace" if inplace else "k_primal", p, "fp32", "recorded"),
                 "roofline": roof(pb, single_us)}}
        if inplace:
            out.update(r)
        else:
            out["ping_pong"] = r
    return out


def inplace_leg(dev, steps=200):
    """The 256x128x128 channel streamed in place (one buffer per state): an
    unrecorded forward and the one-shot iteration, FP32, with the workspace of
    the in-place and the ping-pong one-shot contexts."""
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.lbm import Lbm

    wl = inputs.workload("d3q19_channel_256x128x128")
    p = inputs.model_params(wl)
    w = torch.from_numpy(inputs.design_for(wl)).to(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    c = Lbm(p, nsteps=0, precision="fp32", device=dev, inplace=True)
    c.set_design(w)
    c.reset()
    c.primal_steps(20)
    ev[0].record()
    c.primal_steps(steps)
    ev[1].record()
    c.reset()
    c.oneshot_steps(20, 0.0, 0.0)
    ev[2].record()
    c.oneshot_steps(steps, 0.0, 0.0)
    ev[3].record()
    torch.cuda.synchronize()
    ws_inplace = c.workspace_bytes
    c.close()
    ws_pp = Lbm(p, nsteps=0, precision="fp32", device=dev).workspace_bytes
    prim_us = ev[0].elapsed_time(ev[1]) * 1e3 / steps
    os_us = ev[2].elapsed_time(ev[3]) * 1e3 / steps
    pb, ob = primal_bytes(p, "fp32", recorded=False), oneshot_bytes(p, "fp32")
    nodes = p["nx"] * p["ny"] * p["nz"]
    roof = lambda b, us: {"bound": "hbm", "achieved": b / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": b, "avg_launch_us": us}
    wk = "d3q19_channel_256x128x128"
    kp = klabel("k_primal_inplace", p, "fp32", "unrecorded")
    ko = klabel("k_oneshot_inplace", p, "fp32")
    return {"workload": wk + " streamed in place", "steps_timed": steps,
            "primal": {"kernel": kp, "mlups": nodes / prim_us,
                       "roofline": dict(roof(pb, prim_us), traffic=_measured_traffic(wk, kp))},
            "oneshot": {"kernel": ko, "mlups": nodes / os_us,
                        "roofline": dict(roof(ob, os_us), traffic=_measured_traffic(wk, ko))},
            "workspace_gb": {"inplace": round(ws_inplace / 1e9, 3), "ping_pong": round(ws_pp / 1e9, 3)}}


# Bounded oracle samples: (workload, steps).  The 64x32 channel runs its full
# horizon; the others a few steps, since the per-step cost is constant.
CPU_SAMPLES = (("d2q9_channel_64x32", 1000), ("d2q9_d2q5_exchanger_512x256", 20),
               ("d3q19_d3q7_mixer_128x64x64", 4), ("d3q19_channel_256x128x128", 4))


def _cpu_sample(name, steps):
    import numpy as np

    import oracle
    from paper_1501_04741_amd import inputs
    wl = inputs.workload(name)
    p = inputs.model_params(wl)
    w64 = inputs.design_for(wl).astype(np.float64)
    t0 = time.perf_counter()
    oracle.adjoint(p, w64, steps)
    dt = time.perf_counter() - t0
    n = p["nx"] * p["ny"] * p["nz"]
    return {"workload": name, "steps": steps, "seconds": dt, "mlups": n * steps / dt / 1e6}


def cpu_baseline(workload, samples=CPU_SAMPLES):
    """The FP64 oracle (primal + unsteady adjoint, local Jacobians by complex step)
    on the host's cores: bounded samples of every configured workload; ``value``
    is the benchmark workload's, in the unit of the GPU figure (nodes x steps
    differentiated per second)."""
    import oracle
    cores = oracle.threads()
    runs = [_cpu_sample(name, steps) for name, steps in samples]
    main = next((r for r in runs if r["workload"] == workload), runs[-1])
    return {"value": main["mlups"], "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "nproc": os.cpu_count(),
            "sample": "%s: %d primal + %d adjoint steps of the FP64 oracle (adjoint by complex-step local "
                      "Jacobians), %.1f s; other workloads in 'samples'" % (
                          main["workload"], main["steps"], main["steps"], main["seconds"]),
            "samples": runs}


def _request_designs(trace):
    """Seeded design fields of the trace's requests, drawn in parallel host threads
    (numpy's rolls and sums release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_1501_04741_amd import inputs
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        return list(pool.map(inputs.request_design, trace))


def serving_leg(args):
    """Replays a Poisson trace through the continuous-batching server and, on the
    same GPU, one request at a time (FIFO, no overlap).  Returns a dict: served
    and one-at-a-time gradients/s with p50/p99 latency, their ratio, and the
    largest difference between a served result and the same request run alone."""
    import gc

    import numpy as np
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.serve import GpuExecutor, Job, Server, run_one_at_a_time, summarize

    trace = inputs.poisson_trace(args.requests, args.rate, seed=1, steps=args.serve_steps)
    designs = _request_designs(trace)

    def jobs():
        return [Job(rid=r.rid, params=r.params, steps=r.steps, design=d, precision="fp32", arrival=r.arrival_s)
                for r, d in zip(trace, designs)]

    torch.cuda.set_device(0)
    # warm-up: one small request through both paths (kernel loading, allocator)
    warm = jobs()[:2]
    for j in warm:
        j.arrival = 0.0
    cap = int(args.max_active_gb * 2**30) if args.max_active_gb > 0 else None
    budget = int(args.budget_gb * 2**30)
    req_cap = int(args.request_cap_gb * 2**30)
    inpl_min = int(args.inplace_min_mb * 2**20) if args.inplace_min_mb >= 0 else None
    # workspaces come from one arena
    ex = GpuExecutor(arena_bytes=budget, per_request_cap_bytes=req_cap, inplace_min_state_bytes=inpl_min)
    Server(ex, budget, quantum=args.quantum).replay(warm, realtime=False)
    torch.cuda.synchronize()
    print("[bench] serving %d requests at %.1f/s" % (args.requests, args.rate), file=sys.stderr, flush=True)
    qms = args.quantum_ms if args.quantum_ms > 0 else None
    srv = Server(ex, budget, quantum=args.quantum, policy=args.policy, max_active_state_bytes=cap,
                 quantum_ms=qms)
    served = srv.replay(jobs(), realtime=True)
    s_batched = summarize(served)
    rec = {
        "config": {"workload": "poisson_trace", "requests": args.requests, "rate_per_s": args.rate,
                   "sizes": ["D2Q9 256x128", "D2Q9 1024x512", "D3Q19 96x48x48", "D3Q19 192x96x96"],
                   "steps": args.serve_steps, "precision": "fp32", "objective": "pressure drop",
                   "quantum": args.quantum, "budget_gb": args.budget_gb,
                   "policy": args.policy, "max_active_gb": args.max_active_gb, "quantum_ms": args.quantum_ms,
                   "request_cap_gb": args.request_cap_gb, "inplace_min_mb": args.inplace_min_mb,
                   "trace_seed": 1},
        "served": s_batched,
        "scheduler": dict(srv.stats),
    }
    results = [(j.rid, j.J, j.grad) for j in served if j.state == "done"]
    del srv, ex, served
    gc.collect()
    torch.cuda.empty_cache()
    if not args.no_baseline:
        print("[bench] one-at-a-time replay", file=sys.stderr, flush=True)
        base = run_one_at_a_time(jobs(), per_request_cap_bytes=req_cap, inplace_min_state_bytes=inpl_min)
        one = summarize(base)
        rec["one_at_a_time"] = one
        bg = one.get("gradients_per_s")
        rec["speedup_vs_one_at_a_time"] = (s_batched["gradients_per_s"] / bg) if bg else None
        rec["p50_vs_one_at_a_time"] = (one["p50_ms"] / s_batched["p50_ms"]) if bg else None
        rec["p99_vs_one_at_a_time"] = (one["p99_ms"] / s_batched["p99_ms"]) if bg else None
        alone = {j.rid: j for j in base}
        dj = [abs(J - alone[r].J) / max(abs(alone[r].J), 1e-300) for r, J, _ in results if r in alone]
        dg = [np.linalg.norm(g - alone[r].grad) / max(np.linalg.norm(alone[r].grad), 1e-300)
              for r, _, g in results if r in alone and g is not None]
        rec["served_vs_alone"] = {"compared": len(dj), "max_rel_J": float(max(dj)) if dj else None,
                                  "max_rel_l2_grad": float(max(dg)) if dg else None}
    return rec


def serve_main(args):
    """The serving measurement alone, as its own JSON line."""
    leg = serving_leg(args)
    rec = {
        "metric": "served gradients/s, p50/p99 ms",
        "value": leg["served"].get("gradients_per_s"),
        "unit": "gradients/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": leg.pop("config"),
    }
    rec.update(leg)
    print(json.dumps(rec), flush=True)
    return 0


def legs_main(names, copy_probe_mb=0):
    """Runs only the named legs (no headline evaluation) and prints their results;
    copy_probe_mb > 0 adds one device copy of that size (counter calibration)."""
    import torch
    dev = torch.device("cuda:0")
    legs = {
        "mixer": lambda: mixer_leg(dev),
        "mrt": lambda: mrt_leg(dev),
        "inplace": lambda: inplace_leg(dev),
        "ping_pong": lambda: mrt_leg(dev, collision="bgk", inplace=False),
        "fp64": lambda: mrt_leg(dev, collision="bgk", inplace=True, prec="fp64"),
        "batched": lambda: batched_leg(dev),
        "recompute": lambda: recompute_leg(dev, inplace=True),
        "recompute_ping_pong": lambda: recompute_leg(dev, inplace=False),
    }
    unknown = [n for n in names if n not in legs]
    if unknown:
        print("unknown legs: %s" % ", ".join(unknown), file=sys.stderr)
        return 2
    torch.cuda.set_device(dev)
    out = {}
    for n in names:
        print("[bench] %s leg" % n, file=sys.stderr, flush=True)
        out[n] = legs[n]()
    if copy_probe_mb:
        a = torch.empty(copy_probe_mb * 2**20 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="d3q19_channel_256x128x128")
    ap.add_argument("--lbm-steps", type=int, default=None, help="override the primal horizon N")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixer", action="store_true", help="skip the mixing-duct, MRT, in-place, ping-pong and FP64 legs")
    ap.add_argument("--ping-pong", action="store_true", help="run the main evaluation with ping-pong buffers")
    ap.add_argument("--no-recompute", action="store_true", help="skip the checkpoint + recompute leg")
    ap.add_argument("--only", default="", metavar="LEGS",
                    help="run only these comma-separated legs (mixer, mrt, inplace, ping_pong, fp64, batched, "
                         "recompute, recompute_ping_pong) and print them as one JSON object (for profiling)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="also run one device copy of MB megabytes (counter calibration for profiles)")
    ap.add_argument("--serve", action="store_true",
                    help="measure the serving loop on a Poisson request trace instead (own JSON line)")
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--serve-steps", type=int, default=2000, help="primal (= adjoint) steps per request")
    ap.add_argument("--budget-gb", type=float, default=240.0, help="HBM budget for admitted requests")
    ap.add_argument("--inplace-min-mb", type=float, default=32.0,
                    help="served requests whose state is at least this large stream in place (negative: never)")
    ap.add_argument("--request-cap-gb", type=float, default=64.0,
                    help="workspace cap per served request: every step's moments are held (no recompute) "
                         "when they fit, else the largest checkpoint interval that does")
    ap.add_argument("--quantum", type=int, default=50, help="steps per request per scheduling tick")
    ap.add_argument("--quantum-ms", type=float, default=10.0,
                    help="device time per cost class per tick (0 = fixed --quantum steps)")
    ap.add_argument("--no-baseline", action="store_true", help="skip the one-at-a-time replay")
    ap.add_argument("--policy", default="sjf", choices=["sjf", "fifo"])
    ap.add_argument("--max-active-gb", type=float, default=0.3,
                    help="cap on the summed state size of admitted requests (0 = none)")
    args = ap.parse_args(argv)
    if args.serve and args.gpus == 1:
        return serve_main(args)

    if args.gpus != 1:
        print("bench.py measures one GPU only (the hot path runs on a single MI355X; no multi-GPU path is "
              "built): run with --gpus 1", file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    if args.only:
        return legs_main(args.only.split(","), args.copy_probe)

    import numpy as np
    import torch

    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.lbm import Lbm, lbm_objective_async

    wl = inputs.workload(args.workload)
    if args.lbm_steps:
        wl["steps"] = args.lbm_steps
    p = inputs.model_params(wl)
    N = int(wl["steps"])
    prec = wl["precision"]
    print("[bench] workload %s, N=%d, %s; building context" % (args.workload, N, prec), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    budget = int(wl.get("hbm_budget_gb", 0) * 2**30)
    # in place (one primal and one adjoint buffer, both streamed in place, every step's moments
    # held) when that fits the budget and the workload asks for no checkpoints; else the
    # ping-pong plan
    inplace = not args.ping_pong and wl.get("checkpoint_interval", 0) in (0, N)
    if inplace:
        try:
            L = Lbm(p, nsteps=N, precision=prec, hbm_budget_bytes=budget, device=dev, inplace=True)
        except Exception:
            inplace = False
    if not inplace:
        L = Lbm(p, nsteps=N, precision=prec, checkpoint_interval=wl.get("checkpoint_interval", 0),
                hbm_budget_bytes=budget, device=dev)
    plan = L.plan()
    C = plan["interval"]
    k_last = N - ((N - 1) // C) * C  # adjoint steps of the last segment (moments held, no recompute)
    w_np = inputs.design_for(wl)
    w = torch.from_numpy(w_np).to(dev)
    grad = torch.empty(L.N, dtype=L.dtype, device=dev)
    J_dev = torch.zeros(1, dtype=torch.float64, device=dev)

    def one(ev):
        L.set_design(w)
        L.reset()
        ev[0].record()
        L.primal_steps(N, record=True)
        ev[1].record()
        lbm_objective_async(L.ctx, J_dev)
        L.adjoint_steps(1)  # seeds lambda^N, zeroes the gradient, first reverse step
        ev[2].record()
        if k_last > 1:
            L.adjoint_steps(k_last - 1)
        ev[3].record()
        L.adjoint_steps(N - k_last)
        ev[4].record()
        L.gradient(out=grad)

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    for i in range(args.warmup):
        one(mk())
    torch.cuda.synchronize()
    print("[bench] warmup done; timing %d steps" % args.steps, file=sys.stderr, flush=True)
    evs = [mk() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    adj_seg_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs])) if k_last > 1 else float("nan")
    bwd_ms = float(np.mean([e[1].elapsed_time(e[4]) for e in evs]))
    primal_launch_ms = fwd_ms / N
    adjoint_launch_ms = adj_seg_ms / (k_last - 1) if k_last > 1 else float("nan")
    J = float(J_dev.item())
    if args.copy_probe:
        a = torch.empty(args.copy_probe * 2**20 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # one-shot descent iterations (fused primal + stationary adjoint + update), zeta = 0, streamed
    # like the evaluation above
    os_iters = 200
    L.close()
    O = Lbm(p, nsteps=0, precision=prec, device=dev, inplace=inplace)
    O.set_design(w)
    O.reset()
    O.oneshot_steps(20, 0.0, 0.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    O.oneshot_steps(os_iters, 0.0, 0.0)
    e1.record()
    torch.cuda.synchronize()
    os_launch_ms = e0.elapsed_time(e1) / os_iters
    O.close()

    nodes = L.N
    pb, ab = algorithmic_bytes(p, prec)
    sfx = "_inplace" if inplace else ""
    kp, ka, ko = (klabel("k_primal" + sfx, p, prec, "recorded"), klabel("k_adjoint" + sfx, p, prec),
                  klabel("k_oneshot" + sfx, p, prec))
    ob = oneshot_bytes(p, prec)
    os_gbs = ob / (os_launch_ms * 1e-3) / 1e9
    prim_gbs = pb / (primal_launch_ms * 1e-3) / 1e9
    adj_gbs = ab / (adjoint_launch_ms * 1e-3) / 1e9 if k_last > 1 else None
    rec = {
        "metric": METRIC,
        "value": nodes * N / (ms_per_step * 1e-3) / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": "D3Q19" if p["flow"] == 19 else "D2Q9",
                   "scalar": p.get("scalar", 0), "grid": [p["nx"], p["ny"], p["nz"]], "nodes": nodes,
                   "lbm_steps": N, "precision": prec, "checkpoint_interval": C,
                   "streaming": "in place" if inplace else "ping-pong",
                   "checkpoints": plan["checkpoints"], "moment_sets": plan["moment_sets"],
                   "workspace_gb": round(L.workspace_bytes / 1e9, 3), "switch": "%s(%g)" % (p["switch_fn"],
                                                                                          p["switch_param"])},
        "value_definition": "nodes x primal steps differentiated per second: one step = design set, "
                            "recorded forward, objective, adjoint, gradient; %s" % (
                                "store-all plan: every step's moments held, nothing recomputed" if C >= N else
                                "checkpoint every %d steps: the backward recomputes each segment" % C),
        "J": J,
        "gradients_per_s": 1e3 / ms_per_step,
        "primal_mlups": nodes / (primal_launch_ms * 1e-3) / 1e6,
        "adjoint_kernel_mlups": (nodes / (adjoint_launch_ms * 1e-3) / 1e6) if k_last > 1 else None,
        "backward_mlups": nodes * N / (bwd_ms * 1e-3) / 1e6,
        "forward_ms": fwd_ms,
        "backward_ms": bwd_ms,
        "roofline": None,  # the dominant kernel's, filled in below
        "roofline_primal": {"bound": "hbm", "kernel": kp, "achieved": prim_gbs,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": prim_gbs / HBM_PEAK_GBS,
                            "traffic": _measured_traffic(args.workload, kp),
                            "bytes_per_launch": pb, "avg_launch_us": primal_launch_ms * 1e3},
        "roofline_adjoint": {"bound": "hbm", "kernel": ka, "achieved": adj_gbs,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": (adj_gbs / HBM_PEAK_GBS) if adj_gbs else None,
                             "traffic": _measured_traffic(args.workload, ka),
                             "bytes_per_launch": ab,
                             "avg_launch_us": adjoint_launch_ms * 1e3 if k_last > 1 else None},
        "oneshot": {"kernel": ko, "iterations_timed": os_iters,
                    "mlups": nodes / (os_launch_ms * 1e-3) / 1e6,
                    "roofline": {"bound": "hbm", "achieved": os_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": os_gbs / HBM_PEAK_GBS,
                                 "traffic": _measured_traffic(args.workload, ko),
                                 "bytes_per_launch": ob,
                                 "avg_launch_us": os_launch_ms * 1e3}},
    }
    # the dominant kernel is the one with more time in an evaluation: N primal launches against
    # N adjoint launches
    adj_dominant = k_last > 1 and adjoint_launch_ms > primal_launch_ms
    rec["roofline"] = dict(rec["roofline_adjoint" if adj_dominant else "roofline_primal"])
    if not args.no_mixer:
        print("[bench] mixing duct leg", file=sys.stderr, flush=True)
        rec["mixer"] = mixer_leg(dev)
        print("[bench] MRT leg", file=sys.stderr, flush=True)
        rec["mrt"] = mrt_leg(dev)
        print("[bench] in-place leg", file=sys.stderr, flush=True)
        rec["inplace"] = inplace_leg(dev)
        print("[bench] ping-pong leg", file=sys.stderr, flush=True)
        rec["ping_pong"] = mrt_leg(dev, collision="bgk", inplace=False)
        print("[bench] FP64 leg", file=sys.stderr, flush=True)
        rec["fp64"] = mrt_leg(dev, collision="bgk", inplace=True, prec="fp64")
        print("[bench] batched leg", file=sys.stderr, flush=True)
        rec["batched"] = batched_leg(dev)
    if not args.no_recompute:
        print("[bench] checkpoint + recompute leg", file=sys.stderr, flush=True)
        rec["recompute"] = recompute_leg(dev, inplace=True)
        rec["recompute_ping_pong"] = recompute_leg(dev, inplace=False)
    if not args.no_serve:
        import gc
        del L, O, grad
        gc.collect()
        torch.cuda.empty_cache()
        rec["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        print("[bench] GPU timing done; timing the CPU oracle samples", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(args.workload)
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
