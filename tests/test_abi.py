"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, and validates configurations (no GPU work is issued)."""
import ctypes
import os
import re

import pytest

from paper_1501_04741_amd import build as hipbuild
from paper_1501_04741_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=False)
    return lbm.library()


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm_adj.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "lbm_primal_steps" in names and "lbm_adjoint_steps" in names and "lbm_gradient" in names
    for n in names:
        assert hasattr(lib, n), n


def test_config_struct_size_matches(lib):
    cfg = lbm.make_config(dict(flow=9, nx=16, ny=8), 10)
    assert cfg.struct_size == ctypes.sizeof(lbm.LbmConfig) == 272
    bad = lbm.make_config(dict(flow=9, nx=16, ny=8), 10)
    bad.struct_size = 150
    out = ctypes.c_uint64()
    assert lib.lbm_required_bytes(ctypes.byref(bad), ctypes.byref(out)) == lbm.LBM_EINVAL


@pytest.mark.parametrize("params,ok", [
    (dict(flow=9, nx=16, ny=8), True),
    (dict(flow=9, nx=16, ny=8, nz=2), False),          # 2D needs nz = 1
    (dict(flow=19, nx=16, ny=8, nz=2), False),         # 3D needs nz >= 3
    (dict(flow=19, scalar=5, nx=16, ny=8, nz=4), False),
    (dict(flow=9, scalar=7, nx=16, ny=8), False),
    (dict(flow=9, nx=2, ny=8), False),
    (dict(flow=9, nx=16, ny=8, tau=0.5), False),
    (dict(flow=9, nx=16, ny=8, switch_fn="ramp", switch_param=0.0), False),
    (dict(flow=9, nx=16, ny=8, u_in=1.0), False),
    (dict(flow=19, scalar=7, nx=16, ny=8, nz=6), True),
    (dict(flow=9, nx=16, ny=8, inlet="pressure", rho_in=1.05, u_cap=0.05), True),
    (dict(flow=9, nx=16, ny=8, inlet="pressure", rho_in=1.05), True),        # no limit
    (dict(flow=9, nx=16, ny=8, inlet="pressure", rho_in=0.0), False),
    (dict(flow=9, nx=16, ny=8, inlet="pressure", rho_in=1.05, u_cap=1.0), False),
    (dict(flow=9, nx=16, ny=8, inlet="pressure", rho_in=1.05, u_cap=-0.1), False),
    (dict(flow=9, nx=16, ny=8, inlet=2), False),
    (dict(flow=19, scalar=7, nx=16, ny=8, nz=6, plate_x0=4, plate_x1=12), True),
    (dict(flow=19, scalar=7, nx=16, ny=8, nz=6, plate_x0=4, plate_x1=17), False),   # beyond nx
    (dict(flow=19, scalar=7, nx=16, ny=8, nz=6, plate_x0=9, plate_x1=8), False),    # reversed
    (dict(flow=19, scalar=7, nx=16, ny=8, nz=6, plate_x0=-1, plate_x1=8), False),
    (dict(flow=19, nx=16, ny=8, nz=6, collision="mrt"), True),
    (dict(flow=9, nx=16, ny=8, collision="mrt"), False),                     # MRT is D3Q19 only
    (dict(flow=19, nx=16, ny=8, nz=6, collision="mrt", mrt_rates=(1.19, 1.4, 1.2, 1.4, 2.0)), False),
    (dict(flow=19, nx=16, ny=8, nz=6, collision=2), False),
    (dict(flow=9, scalar=5, nx=16, ny=8, tau_s_solid=4.5), True),
    (dict(flow=9, scalar=5, nx=16, ny=8, tau_s_solid=0.4), False),
])
def test_config_validation(lib, params, ok):
    cfg = lbm.make_config(params, 10)
    out = ctypes.c_uint64()
    st = lib.lbm_required_bytes(ctypes.byref(cfg), ctypes.byref(out))
    assert (st == lbm.LBM_OK) == ok


def _bytes(params, nsteps, **kw):
    return lbm.lbm_required_bytes(lbm.make_config(params, nsteps, **kw))


def test_checkpoint_plan_sizes(lib):
    """Workspace = 4 states (2 adjoint, 2 primal ping-pong) + S checkpoints + C
    moment sets (rho, u[, scalar]: 3-5 values per node) + small node arrays."""
    MB = 2 ** 20
    p = dict(flow=19, nx=256, ny=128, nz=128)
    n = 256 * 128 * 128
    state, mom = 19 * n * 4, 4 * n * 4
    total = lambda C, S: (4 + S) * state + C * mom
    # default: the smallest workspace over all intervals
    best = min(total(C, -(-2000 // C)) for C in range(1, 2001))
    assert abs(_bytes(p, 2000) - best) < 64 * MB
    # a budget that holds every step's moments stores all (C = N: no recompute)
    assert abs(_bytes(p, 2000, hbm_budget_bytes=10 ** 15) - total(2000, 1)) < 64 * MB
    # a budget in between picks the largest interval that fits
    budget = 40 * 2 ** 30
    got = _bytes(p, 2000, hbm_budget_bytes=budget)
    assert got <= budget
    C_fit = max(C for C in range(1, 2001) if total(C, -(-2000 // C)) + 64 * MB <= budget)
    assert abs(got - total(C_fit, -(-2000 // C_fit))) < 64 * MB
    # a budget below the smallest plan is refused
    cfg = lbm.make_config(p, 2000, hbm_budget_bytes=best // 2)
    out = ctypes.c_uint64()
    assert lib.lbm_required_bytes(ctypes.byref(cfg), ctypes.byref(out)) == lbm.LBM_ENOMEM
    # explicit interval, 2D flow + scalar (4 moment values per node)
    n2 = 512 * 256
    c500 = _bytes(dict(flow=9, scalar=5, nx=512, ny=256), 20000, checkpoint_interval=500)
    assert abs(c500 - ((4 + 40) * 14 * n2 * 4 + 500 * 4 * n2 * 4)) < 4 * MB


def test_inplace_workspace_holds_two_states(lib):
    """An in-place context keeps one primal and one adjoint buffer: two states
    fewer than the smallest ping-pong plan of the same lattice, no moments; a
    recorded in-place plan keeps every step's moments, or checkpoints every C
    steps plus a working buffer."""
    p = dict(flow=19, nx=256, ny=128, nz=128)
    state = 19 * 256 * 128 * 128 * 4
    small = lbm.lbm_required_bytes(lbm.make_config(p, 0))
    inpl = lbm.lbm_required_bytes(lbm.make_config(p, 0, inplace=True))
    assert inpl < 2.2 * state + 64 * 2 ** 20
    assert small - inpl >= 3 * state      # ping-pong: 4 states + checkpoint + moment set
    # a recorded in-place run adds the moments of every step and no checkpoints (its
    # adjoint streams in place too)
    rec = lbm.lbm_required_bytes(lbm.make_config(p, 10, inplace=True))
    mom = 4 * 256 * 128 * 128 * 4
    assert rec == inpl + 10 * mom
    # with a checkpoint interval C < N: the working buffer, one adjoint buffer, a
    # state every C steps and the moments of one segment
    st = lbm.lbm_required_bytes(lbm.make_config(p, 0, inplace=True)) // 2
    c3 = lbm.lbm_required_bytes(lbm.make_config(p, 10, checkpoint_interval=3, inplace=True))
    assert abs(c3 - (inpl + 4 * state + 3 * mom)) < 4 * 2 ** 20
    # a budget that cannot hold every step's moments picks the largest C that fits
    all100 = lbm.lbm_required_bytes(lbm.make_config(p, 100, inplace=True))
    assert all100 == inpl + 100 * mom
    budget = 5 * 10 ** 9
    assert all100 > budget
    b = lbm.lbm_required_bytes(lbm.make_config(p, 100, hbm_budget_bytes=budget, inplace=True))
    assert b <= budget
    need = {C: lbm.lbm_required_bytes(lbm.make_config(p, 100, checkpoint_interval=C, inplace=True))
            for C in range(1, 101)}
    best = max(C for C in need if need[C] <= budget)   # the largest C whose plan fits
    assert best < 100 and b == need[best]
    S = -(-100 // best)
    assert abs(b - (inpl + S * state + best * mom)) < 4 * 2 ** 20
    with pytest.raises(lbm.LbmError):   # not even the smallest plan fits
        lbm.lbm_required_bytes(lbm.make_config(p, 100, hbm_budget_bytes=inpl + mom, inplace=True))


def test_solver_default_interval_minimises_the_in_place_workspace(lib):
    """LbmSolver's default in-place plan: the checkpoint interval with the smallest
    workspace, which is below the ping-pong default's on the benchmark channel."""
    from paper_1501_04741_amd import inputs
    from paper_1501_04741_amd.autograd import smallest_inplace_interval
    from paper_1501_04741_amd.lbm import lbm_required_bytes, make_config
    p = inputs.model_params(inputs.workload("d3q19_channel_256x128x128"))
    C = smallest_inplace_interval(p, 2000, "fp32")
    size = lambda c: lbm_required_bytes(make_config(p, 2000, "fp32", checkpoint_interval=c, inplace=True))
    assert 1 < C < 2000
    assert all(size(C) <= size(c) for c in (1, C // 2, C - 1, C + 1, 2 * C, 2000))
    assert size(C) < lbm_required_bytes(make_config(p, 2000, "fp32"))
