"""ctypes binding of ``liblbmadj.so`` (the C ABI in ``include/lbm_adj.h``).

The ``lbm_*`` functions below carry the C names and only marshal arguments;
every step of the method runs in the library's HIP kernels.  PyTorch provides
device memory (the workspace and the caller-owned tensors) and the stream.

The library is loaded on first use; if it has not been built this raises
``LbmLibraryMissing`` -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmadj.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_ENONFINITE = 0, -1, -2, -3, -4, -5
LBM_FP32, LBM_FP64 = 4, 8
_WALL = {"adiabatic": 0, "dirichlet": 1}
_SWITCH = {"power": 0, "ramp": 1}
_PREC = {"fp32": LBM_FP32, "fp64": LBM_FP64}


class LbmLibraryMissing(RuntimeError):
    pass


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str = ""):
        self.status = status
        super().__init__("%s failed with status %d (%s)%s" % (
            where, status, _STATUS_NAMES.get(status, "?"), (": " + message) if message else ""))


_STATUS_NAMES = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "HIP error", -4: "invalid state",
                 -5: "non-finite objective"}


class LbmConfig(ctypes.Structure):
    """Field-for-field mirror of ``lbm_config``."""

    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("flow", ctypes.c_int32),
        ("scalar", ctypes.c_int32),
        ("precision", ctypes.c_int32),
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
        ("reserved0", ctypes.c_int32),
        ("switch_param", ctypes.c_double),
        ("c_dp", ctypes.c_double),
        ("c_hf", ctypes.c_double),
        ("c_var", ctypes.c_double),
        ("nsteps", ctypes.c_int64),
        ("checkpoint_interval", ctypes.c_int64),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("inlet", ctypes.c_int32),
        ("n_avg", ctypes.c_int32),
        ("rho_in", ctypes.c_double),
        ("u_cap", ctypes.c_double),
        ("c_mix", ctypes.c_double),
        ("collision", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
        ("mrt_rates", ctypes.c_double * 5),
        ("tau_s_solid", ctypes.c_double),
        ("inplace", ctypes.c_int32),
        ("reserved3", ctypes.c_int32),
        ("plate_x0", ctypes.c_int32),
        ("plate_x1", ctypes.c_int32),
        ("s_plate", ctypes.c_double),
    ]

NG = 9  # boundary sums ("globals") lbm_objective returns
_INLET = {"velocity": 0, "pressure": 1}
_COLL = {"bgk": 0, "mrt": 1}


MODEL_DEFAULTS = dict(
    flow=9, scalar=0, nx=16, ny=8, nz=1, periodic=0, tau=0.8, tau_s=0.6, u_in=0.01, rho_out=1.0,
    scalar_wall="adiabatic", s_split_axis=0, s_wall=1.0, s_in_lo=0.0, s_in_hi=0.0,
    switch_fn="power", switch_param=3.0, c_dp=1.0, c_hf=0.0, c_var=0.0,
    inlet="velocity", rho_in=1.0, u_cap=0.0, c_mix=0.0,
    collision="bgk", mrt_rates=(1.19, 1.4, 1.2, 1.4, 1.98), tau_s_solid=0.0,
    plate_x0=0, plate_x1=0, s_plate=1.0, n_avg=1,
)


def make_config(params: dict, nsteps: int, precision: str = "fp32", checkpoint_interval: int = 0,
                hbm_budget_bytes: int = 0, inplace: bool = False) -> LbmConfig:
    p = dict(MODEL_DEFAULTS)
    unknown = set(params) - set(MODEL_DEFAULTS)
    if unknown:
        raise KeyError("unknown model keys: %s" % sorted(unknown))
    p.update(params)
    sw = _WALL[p["scalar_wall"]] if isinstance(p["scalar_wall"], str) else int(p["scalar_wall"])
    fn = _SWITCH[p["switch_fn"]] if isinstance(p["switch_fn"], str) else int(p["switch_fn"])
    im = _INLET[p["inlet"]] if isinstance(p["inlet"], str) else int(p["inlet"])
    co = _COLL[p["collision"]] if isinstance(p["collision"], str) else int(p["collision"])
    return LbmConfig(
        struct_size=ctypes.sizeof(LbmConfig), flow=int(p["flow"]), scalar=int(p["scalar"]),
        precision=_PREC[precision], nx=int(p["nx"]), ny=int(p["ny"]), nz=int(p["nz"]),
        periodic=int(p["periodic"]), tau=float(p["tau"]), tau_s=float(p["tau_s"]), u_in=float(p["u_in"]),
        rho_out=float(p["rho_out"]), scalar_wall=sw, s_split_axis=int(p["s_split_axis"]),
        s_wall=float(p["s_wall"]), s_in_lo=float(p["s_in_lo"]), s_in_hi=float(p["s_in_hi"]),
        switch_fn=fn, reserved0=0, switch_param=float(p["switch_param"]), c_dp=float(p["c_dp"]),
        c_hf=float(p["c_hf"]), c_var=float(p["c_var"]), nsteps=int(nsteps),
        checkpoint_interval=int(checkpoint_interval), hbm_budget_bytes=int(hbm_budget_bytes), inlet=im,
        n_avg=int(p["n_avg"]), rho_in=float(p["rho_in"]), u_cap=float(p["u_cap"]), c_mix=float(p["c_mix"]), collision=co,
        reserved2=0, mrt_rates=(ctypes.c_double * 5)(*[float(v) for v in p["mrt_rates"]]),
        tau_s_solid=float(p["tau_s_solid"]), inplace=1 if inplace else 0, reserved3=0,
        plate_x0=int(p["plate_x0"]), plate_x1=int(p["plate_x1"]), s_plate=float(p["s_plate"]))


_lock = threading.Lock()
_lib = None


def library():
    """The loaded ``liblbmadj.so`` (raises LbmLibraryMissing if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise LbmLibraryMissing(
                "%s is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                "(or python paper_1501_04741_amd/build.py) first" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i32, i64, u64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        cfgp = P(LbmConfig)
        sig = {
            "lbm_required_bytes": [cfgp, P(u64)],
            "lbm_create": [cfgp, vp, vp, u64, P(vp)],
            "lbm_create_static": [cfgp, vp, P(vp)],
            "lbm_destroy": [vp],
            "lbm_set_design": [vp, vp],
            "lbm_reset": [vp],
            "lbm_set_state": [vp, vp, vp],
            "lbm_primal_steps": [vp, i64, i32],
            "lbm_objective": [vp, P(d), P(d)],
            "lbm_objective_async": [vp, vp],
            "lbm_adjoint_steps": [vp, i64],
            "lbm_gradient": [vp, vp],
            "lbm_gradient_penalty": [vp, d, vp],
            "lbm_fields": [vp, vp, vp, vp],
            "lbm_get_state": [vp, vp, vp],
            "lbm_get_adjoint": [vp, vp, vp],
            "lbm_export_maps": [vp, vp, vp],
            "lbm_times": [vp, P(i64), P(i64), P(i64)],
            "lbm_oneshot_steps": [vp, i64, d, d],
            "lbm_get_design": [vp, vp],
            "lbm_plan": [vp, P(i64), P(i64), P(i64), P(u64)],
            "lbm_primal_steps_batch": [P(vp), i32, i64, i32],
            "lbm_adjoint_steps_batch": [P(vp), i32, i64],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.lbm_static_workspace_bytes.argtypes = []
        lib.lbm_static_workspace_bytes.restype = ctypes.c_uint64
        lib.lbm_last_error.argtypes = [vp]
        lib.lbm_last_error.restype = ctypes.c_char_p
        lib.lbm_status_string.argtypes = [ctypes.c_int]
        lib.lbm_status_string.restype = ctypes.c_char_p
        _lib = lib
        return lib


def _chk(status: int, where: str, ctx=None):
    if status != LBM_OK:
        msg = ""
        if ctx is not None:
            msg = (library().lbm_last_error(ctx) or b"").decode()
        raise LbmError(status, where, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------ C-named thin wrappers
def lbm_required_bytes(cfg: LbmConfig) -> int:
    out = ctypes.c_uint64()
    _chk(library().lbm_required_bytes(ctypes.byref(cfg), ctypes.byref(out)), "lbm_required_bytes")
    return out.value


def lbm_create(cfg: LbmConfig, stream_handle: int, workspace_ptr: int, workspace_bytes: int):
    ctx = ctypes.c_void_p()
    _chk(library().lbm_create(ctypes.byref(cfg), ctypes.c_void_p(stream_handle), ctypes.c_void_p(workspace_ptr),
                              workspace_bytes, ctypes.byref(ctx)), "lbm_create")
    return ctx


def lbm_create_static(cfg: LbmConfig, stream_handle: int):
    ctx = ctypes.c_void_p()
    _chk(library().lbm_create_static(ctypes.byref(cfg), ctypes.c_void_p(stream_handle), ctypes.byref(ctx)),
         "lbm_create_static")
    return ctx


def lbm_static_workspace_bytes() -> int:
    return int(library().lbm_static_workspace_bytes())


def lbm_destroy(ctx):
    _chk(library().lbm_destroy(ctx), "lbm_destroy")


def lbm_set_design(ctx, w):
    _chk(library().lbm_set_design(ctx, _ptr(w)), "lbm_set_design", ctx)


def lbm_reset(ctx):
    _chk(library().lbm_reset(ctx), "lbm_reset", ctx)


def lbm_set_state(ctx, f, g=None):
    _chk(library().lbm_set_state(ctx, _ptr(f), _ptr(g)), "lbm_set_state", ctx)


def lbm_primal_steps(ctx, nsteps: int, record: bool = False):
    _chk(library().lbm_primal_steps(ctx, int(nsteps), 1 if record else 0), "lbm_primal_steps", ctx)


def lbm_objective(ctx):
    J = ctypes.c_double()
    G = (ctypes.c_double * NG)()
    st = library().lbm_objective(ctx, ctypes.byref(J), G)
    if st == LBM_ENONFINITE:
        raise LbmError(st, "lbm_objective", "non-finite objective")
    _chk(st, "lbm_objective", ctx)
    return J.value, list(G)


def lbm_objective_async(ctx, J_dev):
    _chk(library().lbm_objective_async(ctx, _ptr(J_dev)), "lbm_objective_async", ctx)


def lbm_adjoint_steps(ctx, nsteps: int):
    _chk(library().lbm_adjoint_steps(ctx, int(nsteps)), "lbm_adjoint_steps", ctx)


def lbm_gradient(ctx, grad):
    _chk(library().lbm_gradient(ctx, _ptr(grad)), "lbm_gradient", ctx)


def lbm_gradient_penalty(ctx, penalty: float, grad):
    _chk(library().lbm_gradient_penalty(ctx, float(penalty), _ptr(grad)), "lbm_gradient_penalty", ctx)


def lbm_fields(ctx, rho, u, s=None):
    _chk(library().lbm_fields(ctx, _ptr(rho), _ptr(u), _ptr(s)), "lbm_fields", ctx)


def lbm_get_state(ctx, f, g=None):
    _chk(library().lbm_get_state(ctx, _ptr(f), _ptr(g)), "lbm_get_state", ctx)


def lbm_get_adjoint(ctx, lf, lg=None):
    _chk(library().lbm_get_adjoint(ctx, _ptr(lf), _ptr(lg)), "lbm_get_adjoint", ctx)


def lbm_export_maps(ctx, mask=None, src=None):
    _chk(library().lbm_export_maps(ctx, _ptr(mask), _ptr(src)), "lbm_export_maps", ctx)


def lbm_oneshot_steps(ctx, nsteps: int, zeta: float, penalty: float = 0.0):
    _chk(library().lbm_oneshot_steps(ctx, int(nsteps), float(zeta), float(penalty)), "lbm_oneshot_steps", ctx)


def lbm_get_design(ctx, w):
    _chk(library().lbm_get_design(ctx, _ptr(w)), "lbm_get_design", ctx)


def lbm_times(ctx):
    t, r, a = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _chk(library().lbm_times(ctx, ctypes.byref(t), ctypes.byref(r), ctypes.byref(a)), "lbm_times", ctx)
    return t.value, r.value, a.value


def lbm_plan(ctx):
    c, s, r, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
    _chk(library().lbm_plan(ctx, ctypes.byref(c), ctypes.byref(s), ctypes.byref(r), ctypes.byref(b)), "lbm_plan",
         ctx)
    return dict(interval=c.value, checkpoints=s.value, moment_sets=r.value, state_bytes=b.value)


def lbm_primal_steps_batch(ctxs, nsteps: int, record: bool = False):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    _chk(library().lbm_primal_steps_batch(arr, len(ctxs), int(nsteps), 1 if record else 0),
         "lbm_primal_steps_batch", ctxs[0] if ctxs else None)


def lbm_adjoint_steps_batch(ctxs, nsteps: int):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    _chk(library().lbm_adjoint_steps_batch(arr, len(ctxs), int(nsteps)), "lbm_adjoint_steps_batch",
         ctxs[0] if ctxs else None)


# ------------------------------------------------------------ object form
class Lbm:
    """One lattice (flow + optional scalar) with its workspace on one GPU.

    ``params`` holds the model keys of ``MODEL_DEFAULTS``; ``nsteps`` is the
    horizon a recorded run may reach.  Device memory comes from torch."""

    def __init__(self, params: dict, nsteps: int, precision: str = "fp32", checkpoint_interval: int = 0,
                 hbm_budget_bytes: int = 0, device=None, stream=None, workspace=None, inplace: bool = False):
        """workspace: optional caller-owned uint8 device tensor (256-byte aligned) of at
        least lbm_required_bytes; by default one is allocated with torch.empty;
        "static": the library's static device workspace (lbm_create_static, no
        allocation; one such context per device at a time).
        inplace: stream in place (one primal and one adjoint buffer, each read and
        rewritten by every step).  With nsteps = 0 the context runs unrecorded steps
        and the one-shot iteration; with nsteps > 0 a recorded run keeps the moments
        of every step unless checkpoint_interval (1 <= C < nsteps) or the budget asks
        for checkpoints, whose segments the adjoint then recomputes in place; the
        adjoint streams in place too."""
        library()
        self.device = torch.device(device if device is not None else "cuda")
        self.params = dict(params)
        self.precision = precision
        self.cfg = make_config(params, nsteps, precision, checkpoint_interval, hbm_budget_bytes, inplace)
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.nx, self.ny, self.nz = self.cfg.nx, self.cfg.ny, self.cfg.nz
        self.N = self.nx * self.ny * self.nz
        self.Q, self.QS = self.cfg.flow, self.cfg.scalar
        self.nsteps = nsteps
        self.workspace_bytes = lbm_required_bytes(self.cfg)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if isinstance(workspace, str) and workspace == "static":
            # the library's static device workspace: nothing is allocated
            self.workspace = None
            with torch.cuda.device(self.device):
                self.ctx = lbm_create_static(self.cfg, self.stream.cuda_stream)
            self._design = None
            return
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        elif workspace.numel() < self.workspace_bytes or workspace.data_ptr() % 256:
            raise ValueError("workspace must be 256-byte aligned and hold %d bytes" % self.workspace_bytes)
        self.workspace = workspace
        self.ctx = lbm_create(self.cfg, self.stream.cuda_stream, self.workspace.data_ptr(), self.workspace_bytes)
        self._design = None

    # lifecycle
    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_destroy(self.ctx)
            self.ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t, dtype):
        t = torch.as_tensor(t)
        return t.to(device=self.device, dtype=dtype).contiguous()

    def set_design(self, w):
        w = self._dev(w, self.dtype).reshape(-1)
        if w.numel() != self.N:
            raise ValueError("design field has %d values, lattice has %d nodes" % (w.numel(), self.N))
        self._design = w  # keep alive until the stream-ordered copy has run
        lbm_set_design(self.ctx, w)

    def reset(self):
        lbm_reset(self.ctx)

    def set_state(self, f, g=None):
        f = self._dev(f, torch.float64).reshape(self.Q, self.N)
        g = None if (g is None or self.QS == 0) else self._dev(g, torch.float64).reshape(self.QS, self.N)
        self._state_in = (f, g)
        lbm_set_state(self.ctx, f, g)

    def primal_steps(self, nsteps: int, record: bool = False):
        lbm_primal_steps(self.ctx, nsteps, record)

    def objective(self):
        """(J, globals) of the current state; synchronises the stream."""
        return lbm_objective(self.ctx)

    def adjoint_steps(self, nsteps: int):
        lbm_adjoint_steps(self.ctx, nsteps)

    def gradient(self, out=None, penalty: float = 0.0):
        """dJ/dw; with penalty != 0 the gradient of J + penalty * sum w (1 - w)."""
        if out is None:
            out = torch.empty(self.N, dtype=self.dtype, device=self.device)
        if penalty:
            lbm_gradient_penalty(self.ctx, penalty, out)
        else:
            lbm_gradient(self.ctx, out)
        return out

    def fields(self):
        rho = torch.empty(self.N, dtype=torch.float64, device=self.device)
        u = torch.empty(3, self.N, dtype=torch.float64, device=self.device)
        s = torch.empty(self.N, dtype=torch.float64, device=self.device)
        lbm_fields(self.ctx, rho, u, s)
        return rho, u, s

    def get_state(self):
        f = torch.empty(self.Q, self.N, dtype=torch.float64, device=self.device)
        g = torch.empty(self.QS, self.N, dtype=torch.float64, device=self.device) if self.QS else None
        lbm_get_state(self.ctx, f, g)
        return f, g

    def get_adjoint(self):
        lf = torch.empty(self.Q, self.N, dtype=torch.float64, device=self.device)
        lg = torch.empty(self.QS, self.N, dtype=torch.float64, device=self.device) if self.QS else None
        lbm_get_adjoint(self.ctx, lf, lg)
        return lf, lg

    def export_maps(self):
        mask = torch.empty(self.N, dtype=torch.uint8, device=self.device)
        src = torch.empty(self.Q, self.N, dtype=torch.int64, device=self.device)
        lbm_export_maps(self.ctx, mask, src)
        return mask, src

    def oneshot_steps(self, nsteps: int, zeta: float, penalty: float = 0.0):
        lbm_oneshot_steps(self.ctx, nsteps, zeta, penalty)

    def design(self):
        out = torch.empty(self.N, dtype=self.dtype, device=self.device)
        lbm_get_design(self.ctx, out)
        return out

    def times(self):
        return lbm_times(self.ctx)

    def plan(self):
        return lbm_plan(self.ctx)

    # one full design evaluation: J and dJ/dw
    def value_and_grad(self, w, nsteps: int = None):
        n = self.nsteps if nsteps is None else nsteps
        self.set_design(w)
        self.reset()
        self.primal_steps(n, record=True)
        J, _ = self.objective()
        self.adjoint_steps(n)
        return J, self.gradient()
