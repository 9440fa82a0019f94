"""Python handle on the plain FP64 CPU oracle (``oracle/lbm_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.

The shared object is built with g++ (OpenMP, no fast-math) on first use, or
whenever the source is newer than the built file.  ``build()`` forces it.

Configurations are plain dicts with the keys of ``CONFIG_KEYS`` (missing keys
take the defaults below); the workload presets that produce them live with the
seeded input generators, not here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbmoracle.so")
_lock = threading.Lock()
_lib = None


class Config(ctypes.Structure):
    """Field-for-field mirror of ``struct lbmo_cfg``."""

    _fields_ = [
        ("flow_q", ctypes.c_int32),
        ("scalar_q", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("tau_s", ctypes.c_double),
        ("u_in", ctypes.c_double),
        ("rho_out", ctypes.c_double),
        ("scalar_wall", ctypes.c_int32),
        ("s_split_axis", ctypes.c_int32),
        ("s_wall", ctypes.c_double),
        ("s_in_lo", ctypes.c_double),
        ("s_in_hi", ctypes.c_double),
        ("switch_fn", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("switch_param", ctypes.c_double),
        ("c_dp", ctypes.c_double),
        ("c_hf", ctypes.c_double),
        ("c_var", ctypes.c_double),
        ("inlet_mode", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
        ("rho_in", ctypes.c_double),
        ("u_cap", ctypes.c_double),
        ("c_mix", ctypes.c_double),
        ("collision", ctypes.c_int32),
        ("reserved3", ctypes.c_int32),
        ("mrt_s", ctypes.c_double * 5),
        ("tau_s_solid", ctypes.c_double),
        ("plate_x0", ctypes.c_int32),
        ("plate_x1", ctypes.c_int32),
        ("s_plate", ctypes.c_double),
        ("n_avg", ctypes.c_int32),
        ("reserved4", ctypes.c_int32),
    ]

NG = 9  # boundary sums ("globals") the objective is built from


DEFAULTS = dict(
    flow=9, scalar=0, nx=16, ny=8, nz=1, periodic=0, tau=0.8, tau_s=0.6, u_in=0.01, rho_out=1.0,
    scalar_wall="adiabatic", s_split_axis=0, s_wall=1.0, s_in_lo=0.0, s_in_hi=0.0,
    switch_fn="power", switch_param=3.0, c_dp=1.0, c_hf=0.0, c_var=0.0,
    inlet="velocity", rho_in=1.0, u_cap=0.0, c_mix=0.0,
    collision="bgk", mrt_rates=(1.19, 1.4, 1.2, 1.4, 1.98), tau_s_solid=0.0,
    plate_x0=0, plate_x1=0, s_plate=1.0, n_avg=1,
)
CONFIG_KEYS = tuple(DEFAULTS)


def build(force: bool = True) -> str:
    """Compile the oracle shared object in place; returns its path."""
    with _lock:
        stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
        if force or stale:
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                   "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    d = P(ctypes.c_double)
    c = P(Config)
    sig = {
        "lbmo_threads": (ctypes.c_int, [ctypes.c_int]),
        "lbmo_lattice": (ctypes.c_int, [ctypes.c_int, P(ctypes.c_int32), d, P(ctypes.c_int32), d]),
        "lbmo_mrt": (ctypes.c_int, [c, d, d, d]),
        "lbmo_mask": (ctypes.c_int, [c, P(ctypes.c_uint8)]),
        "lbmo_src_map": (ctypes.c_int, [c, P(ctypes.c_int64)]),
        "lbmo_node_op": (ctypes.c_int, [c, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, ctypes.c_double, d, d]),
        "lbmo_primal": (ctypes.c_int, [c, d, d, d, ctypes.c_int64, d, d, d, d]),
        "lbmo_directional": (ctypes.c_int, [c, d, d, ctypes.c_int64, d, d]),
        "lbmo_adjoint": (ctypes.c_int, [c, d, d, d, ctypes.c_int64, d, d, d, d]),
        "lbmo_fields": (ctypes.c_int, [c, d, d, d, d, d]),
        "lbmo_step": (ctypes.c_int, [c, d, d, d, d, d]),
        "lbmo_step_tangent": (ctypes.c_int, [c, d, d, d, d, d, d, d, d]),
        "lbmo_step_adjoint": (ctypes.c_int, [c, d, d, d, d, d, d, d, d]),
        "lbmo_objective_seed": (ctypes.c_int, [c, d, d, d, d, d]),
        "lbmo_oneshot": (ctypes.c_int, [c, d, d, d, ctypes.c_int64, ctypes.c_double, ctypes.c_double, d, d, d, d,
                                        d, d]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return int(_load().lbmo_threads(int(n)))


def make_config(params: dict) -> Config:
    p = dict(DEFAULTS)
    unknown = set(params) - set(DEFAULTS)
    if unknown:
        raise KeyError("unknown config keys: %s" % sorted(unknown))
    p.update(params)
    sw = {"adiabatic": 0, "dirichlet": 1}[p["scalar_wall"]] if isinstance(p["scalar_wall"], str) else int(p["scalar_wall"])
    fn = {"power": 0, "ramp": 1}[p["switch_fn"]] if isinstance(p["switch_fn"], str) else int(p["switch_fn"])
    im = {"velocity": 0, "pressure": 1}[p["inlet"]] if isinstance(p["inlet"], str) else int(p["inlet"])
    co = {"bgk": 0, "mrt": 1}[p["collision"]] if isinstance(p["collision"], str) else int(p["collision"])
    return Config(
        flow_q=int(p["flow"]), scalar_q=int(p["scalar"]), nx=int(p["nx"]), ny=int(p["ny"]), nz=int(p["nz"]),
        periodic=int(p["periodic"]), tau=float(p["tau"]), tau_s=float(p["tau_s"]), u_in=float(p["u_in"]),
        rho_out=float(p["rho_out"]), scalar_wall=sw, s_split_axis=int(p["s_split_axis"]),
        s_wall=float(p["s_wall"]), s_in_lo=float(p["s_in_lo"]), s_in_hi=float(p["s_in_hi"]),
        switch_fn=fn, reserved=0, switch_param=float(p["switch_param"]), c_dp=float(p["c_dp"]),
        c_hf=float(p["c_hf"]), c_var=float(p["c_var"]), inlet_mode=im, reserved2=0, rho_in=float(p["rho_in"]),
        u_cap=float(p["u_cap"]), c_mix=float(p["c_mix"]), collision=co, reserved3=0,
        mrt_s=(ctypes.c_double * 5)(*[float(v) for v in p["mrt_rates"]]), tau_s_solid=float(p["tau_s_solid"]),
        plate_x0=int(p["plate_x0"]), plate_x1=int(p["plate_x1"]), s_plate=float(p["s_plate"]),
        n_avg=int(p["n_avg"]), reserved4=0,
    )


def _sizes(cfg: Config):
    n = cfg.nx * cfg.ny * cfg.nz
    return n, cfg.flow_q, cfg.scalar_q


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, size):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != size:
        raise ValueError("expected %d values, got %d" % (size, a.size))
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected the configuration" % what)


def _cfg(params):
    return params if isinstance(params, Config) else make_config(params)


def lattice(q: int):
    """(e[q,3] int, weights[q], opp[q], c^2) of D2Q5, D3Q7, D2Q9 or D3Q19."""
    lib = _load()
    e = np.zeros(3 * q, np.int32)
    wt = np.zeros(q)
    opp = np.zeros(q, np.int32)
    cs2 = ctypes.c_double()
    _check(lib.lbmo_lattice(q, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(wt),
                            opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cs2)), "lattice")
    return e.reshape(q, 3), wt, opp, cs2.value


def mrt(params):
    """(U[19,19], rates[19], K[19,19]) of the D3Q19 MRT collision of a configuration."""
    cfg = _cfg(dict(params, collision="mrt"))
    U = np.zeros(361)
    r = np.zeros(19)
    K = np.zeros(361)
    _check(_load().lbmo_mrt(ctypes.byref(cfg), _dp(U), _dp(r), _dp(K)), "mrt")
    return U.reshape(19, 19), r, K.reshape(19, 19)


def mask(params):
    cfg = _cfg(params)
    n, _, _ = _sizes(cfg)
    out = np.zeros(n, np.uint8)
    _check(_load().lbmo_mask(ctypes.byref(cfg), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "mask")
    return out


def src_map(params):
    cfg = _cfg(params)
    n, q, _ = _sizes(cfg)
    out = np.zeros(q * n, np.int64)
    _check(_load().lbmo_src_map(ctypes.byref(cfg), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "src_map")
    return out.reshape(q, n)


def node_op(params, x, y, z, f, g=None, w=1.0):
    cfg = _cfg(params)
    _, q, qs = _sizes(cfg)
    f = _f64(f, q)
    g = _f64(g if g is not None else np.zeros(max(qs, 1)), max(qs, 1) if g is None else qs)
    h = np.zeros(q)
    gp = np.zeros(max(qs, 1))
    _check(_load().lbmo_node_op(ctypes.byref(cfg), int(x), int(y), int(z), _dp(f), _dp(g), float(w), _dp(h), _dp(gp)),
           "node_op")
    return h, gp[:qs]


def _state_args(cfg, f0, g0):
    n, q, qs = _sizes(cfg)
    fa = _f64(f0, q * n) if f0 is not None else None
    ga = _f64(g0, qs * n) if (g0 is not None and qs) else None
    return fa, ga


def _opt(a):
    return _dp(a) if a is not None else None


def primal(params, w, nsteps, f0=None, g0=None):
    """Run nsteps of the primal scheme; returns dict(f, g, globals, J).

    f, g are the pre-collision state after nsteps (shape (Q, N), (Qs, N))."""
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    w = _f64(w, n)
    fa, ga = _state_args(cfg, f0, g0)
    fN = np.zeros(q * n)
    gN = np.zeros(max(qs, 1) * n)
    G = np.zeros(NG)
    J = ctypes.c_double()
    _check(_load().lbmo_primal(ctypes.byref(cfg), _dp(w), _opt(fa), _opt(ga), int(nsteps), _dp(fN), _dp(gN), _dp(G),
                               ctypes.byref(J)), "primal")
    return dict(f=fN.reshape(q, n), g=gN[: qs * n].reshape(qs, n), globals=G, J=J.value)


def directional(params, w, dw, nsteps):
    """(J, dJ/dw . dw) by complex step through the whole run."""
    cfg = _cfg(params)
    n, _, _ = _sizes(cfg)
    w = _f64(w, n)
    dw = _f64(dw, n)
    J = ctypes.c_double()
    dJ = ctypes.c_double()
    _check(_load().lbmo_directional(ctypes.byref(cfg), _dp(w), _dp(dw), int(nsteps), ctypes.byref(J), ctypes.byref(dJ)),
           "directional")
    return J.value, dJ.value


def adjoint(params, w, nsteps, f0=None, g0=None):
    """Unsteady discrete adjoint; returns dict(J, grad, lam_f, lam_g)."""
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    w = _f64(w, n)
    fa, ga = _state_args(cfg, f0, g0)
    grad = np.zeros(n)
    lf = np.zeros(q * n)
    lg = np.zeros(max(qs, 1) * n)
    J = ctypes.c_double()
    _check(_load().lbmo_adjoint(ctypes.byref(cfg), _dp(w), _opt(fa), _opt(ga), int(nsteps), ctypes.byref(J), _dp(grad),
                                _dp(lf), _dp(lg)), "adjoint")
    return dict(J=J.value, grad=grad, lam_f=lf.reshape(q, n), lam_g=lg[: qs * n].reshape(qs, n))


def fields(params, f, g=None):
    """(rho[N], u[3,N], T[N]) of a pre-collision state."""
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    fa = _f64(f, q * n)
    ga = _f64(g, qs * n) if qs else np.zeros(1)
    rho = np.zeros(n)
    u = np.zeros(3 * n)
    T = np.zeros(n)
    _check(_load().lbmo_fields(ctypes.byref(cfg), _dp(fa), _dp(ga), _dp(rho), _dp(u), _dp(T)), "fields")
    return rho, u.reshape(3, n), T


def step(params, w, f, g=None):
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    fa = _f64(f, q * n)
    ga = _f64(g, qs * n) if qs else np.zeros(1)
    fn = np.zeros(q * n)
    gn = np.zeros(max(qs, 1) * n)
    _check(_load().lbmo_step(ctypes.byref(cfg), _dp(_f64(w, n)), _dp(fa), _dp(ga), _dp(fn), _dp(gn)), "step")
    return fn.reshape(q, n), gn[: qs * n].reshape(qs, n)


def step_tangent(params, w, f, g, df, dg, dw):
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    z1 = np.zeros(1)
    args = [_f64(w, n), _f64(f, q * n), _f64(g, qs * n) if qs else z1, _f64(df, q * n),
            _f64(dg, qs * n) if qs else z1, _f64(dw, n)]
    dfn = np.zeros(q * n)
    dgn = np.zeros(max(qs, 1) * n)
    _check(_load().lbmo_step_tangent(ctypes.byref(cfg), *[_dp(a) for a in args], _dp(dfn), _dp(dgn)), "step_tangent")
    return dfn.reshape(q, n), dgn[: qs * n].reshape(qs, n)


def step_adjoint(params, w, f, g, lf, lg):
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    z1 = np.zeros(1)
    args = [_f64(w, n), _f64(f, q * n), _f64(g, qs * n) if qs else z1, _f64(lf, q * n), _f64(lg, qs * n) if qs else z1]
    lfo = np.zeros(q * n)
    lgo = np.zeros(max(qs, 1) * n)
    gw = np.zeros(n)
    _check(_load().lbmo_step_adjoint(ctypes.byref(cfg), *[_dp(a) for a in args], _dp(lfo), _dp(lgo), _dp(gw)),
           "step_adjoint")
    return lfo.reshape(q, n), lgo[: qs * n].reshape(qs, n), gw


def objective_seed(params, f, g=None):
    """(J, dJ/df, dJ/dg) of a pre-collision state."""
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    fa = _f64(f, q * n)
    ga = _f64(g, qs * n) if qs else np.zeros(1)
    J = ctypes.c_double()
    lf = np.zeros(q * n)
    lg = np.zeros(max(qs, 1) * n)
    _check(_load().lbmo_objective_seed(ctypes.byref(cfg), _dp(fa), _dp(ga), ctypes.byref(J), _dp(lf), _dp(lg)),
           "objective_seed")
    return J.value, lf.reshape(q, n), lg[: qs * n].reshape(qs, n)


def oneshot(params, w, iters, zeta, c_pen=0.0, f0=None, g0=None):
    """One-shot descent iterations (primal step, stationary-adjoint step with
    the objective source, gradient estimate, clipped design update).
    Returns dict(w, f, g, lam_f, lam_g, grad, J) after ``iters`` iterations;
    grad and J belong to the last iteration's state."""
    cfg = _cfg(params)
    n, q, qs = _sizes(cfg)
    wa = _f64(w, n).copy()
    fa, ga = _state_args(cfg, f0, g0)
    fN = np.zeros(q * n)
    gN = np.zeros(max(qs, 1) * n)
    lf = np.zeros(q * n)
    lg = np.zeros(max(qs, 1) * n)
    gr = np.zeros(n)
    J = ctypes.c_double()
    _check(_load().lbmo_oneshot(ctypes.byref(cfg), _dp(wa), _opt(fa), _opt(ga), int(iters), float(zeta), float(c_pen),
                                _dp(fN), _dp(gN), _dp(lf), _dp(lg), _dp(gr), ctypes.byref(J)), "oneshot")
    return dict(w=wa, f=fN.reshape(q, n), g=gN[: qs * n].reshape(qs, n), lam_f=lf.reshape(q, n),
                lam_g=lg[: qs * n].reshape(qs, n), grad=gr, J=J.value)


def penalty(params, w):
    """P(w) = sum over interior nodes of w (1 - w) (eq. P): zero at w in {0, 1}."""
    w = _f64(w, _sizes(_cfg(params))[0])
    return float(np.sum((w * (1.0 - w))[mask(params) == 0]))


def penalty_gradient(params, w, c_pen):
    """c_pen * dP/dw = c_pen (1 - 2w) at interior nodes, 0 elsewhere (eq. P); the
    term the optimiser adds to dJ/dw for the penalised objective J + c_pen P."""
    w = _f64(w, _sizes(_cfg(params))[0])
    return np.where(mask(params) == 0, c_pen * (1.0 - 2.0 * w), 0.0)
