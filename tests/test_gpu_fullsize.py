"""The benchmark workload at full size (D3Q19 256x128x128, FP32) in the launch
configuration the benchmark times (forward streamed in place with streaming
stores, moments of every step held, adjoint streamed in place): from a developed
flow, every primal step, the objective, every adjoint step and the gradient of
a short recorded run against the FP64 oracle's single-step operators applied
to the GPU's own states, node by node over the whole lattice."""
import numpy as np
import pytest
import torch

import oracle
from paper_1501_04741_amd import inputs
from paper_1501_04741_amd.lbm import Lbm

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_full_size_steps_match_oracle_operators():
    wl = inputs.workload("d3q19_channel_256x128x128")
    p = inputs.model_params(wl)
    N = 3
    w32 = inputs.design_for(wl)
    w64 = w32.astype(np.float64)
    # a developed flow first (300 unrecorded steps), so every node class is active
    warm = Lbm(p, nsteps=0, precision="fp32", inplace=True)
    warm.set_design(torch.from_numpy(w32))
    warm.reset()
    warm.primal_steps(300)
    f0, _ = warm.get_state()
    warm.close()
    ctx = Lbm(p, nsteps=N, precision="fp32", hbm_budget_bytes=int(wl["hbm_budget_gb"] * 2**30), inplace=True)
    assert ctx.plan()["moment_sets"] == N
    ctx.set_design(torch.from_numpy(w32))
    ctx.set_state(f0)
    states = [_np(ctx.get_state()[0])]
    assert np.max(np.abs(states[0] - _np(f0))) < 1e-7
    for n in range(N):
        ctx.primal_steps(1, record=True)
        states.append(_np(ctx.get_state()[0]))
    J, _ = ctx.objective()
    # primal: f^{n+1} = oracle step of the GPU's f^n (FP32 storage: ~1e-7 absolute on O(0.3) populations)
    for n in range(N):
        ref, _ = oracle.step(p, w64, states[n])
        assert np.max(np.abs(states[n + 1] - ref)) < 2e-6, n
    Jr, lam, _ = oracle.objective_seed(p, states[N])
    assert abs(J - Jr) <= 1e-4 * abs(Jr)
    # adjoint: lambda^n = oracle adjoint step of the GPU's lambda^{n+1}; gradient = sum of the steps' dW/dw terms
    gsum = np.zeros(w64.size)
    lam_gpu = lam
    for n in reversed(range(N)):
        ctx.adjoint_steps(1)
        lam_n = _np(ctx.get_adjoint()[0])
        ref_lam, _, gw = oracle.step_adjoint(p, w64, states[n], None, lam_gpu, None)
        scale = np.max(np.abs(ref_lam))
        assert np.max(np.abs(lam_n - ref_lam)) <= 1e-4 * scale, n
        gsum += gw
        lam_gpu = lam_n
    grad = _np(ctx.gradient())
    assert np.linalg.norm(grad - gsum) <= 1e-3 * np.linalg.norm(gsum)
    ctx.close()


def _state(ctx):
    f, g = ctx.get_state()
    return _np(f), (None if g is None else _np(g))


@pytest.mark.parametrize("name", ["d2q9_d2q5_exchanger_512x256", "d3q19_d3q7_mixer_128x64x64"])
def test_full_length_run_matches_oracle_operators_and_fp64(name):
    """The heat-exchanger (512x256 D2Q9+D2Q5, 20000 steps, checkpoint every 500)
    and mixer (128x64x64 D3Q19+D3Q7, 5000 steps) workloads at full size and full
    length in FP32, with their own checkpoint plans: the last two primal steps,
    the objective and the first two adjoint steps against the oracle's single-step
    operators applied to the GPU's own states and cotangents; then the whole
    adjoint sweep (segments recomputed from checkpoints) against the same run in
    FP64, whose arithmetic the small-lattice tests tie to the oracle at 1e-10."""
    wl = inputs.workload(name)
    p = inputs.model_params(wl)
    N, C, tail = wl["steps"], wl["checkpoint_interval"], 2
    w32 = inputs.design_for(wl)
    w64 = w32.astype(np.float64)
    ctx = Lbm(p, nsteps=N, precision="fp32", checkpoint_interval=C)
    ctx.set_design(torch.from_numpy(w32))
    ctx.reset()
    ctx.primal_steps(N - tail, record=True)
    states = [_state(ctx)]
    for _ in range(tail):
        ctx.primal_steps(1, record=True)
        states.append(_state(ctx))
    J, _ = ctx.objective()
    for n in range(tail):
        rf, rg = oracle.step(p, w64, *states[n])
        assert np.max(np.abs(states[n + 1][0] - rf)) < 2e-6, n
        assert np.max(np.abs(states[n + 1][1] - rg)) < 2e-6, n
    Jr, lf, lg = oracle.objective_seed(p, *states[tail])
    assert abs(J - Jr) <= 1e-4 * abs(Jr)
    lam = (lf, lg)
    for n in reversed(range(tail)):
        ctx.adjoint_steps(1)
        gf, gg = ctx.get_adjoint()
        rf, rg, _ = oracle.step_adjoint(p, w64, *states[n], *lam)
        scale = max(np.abs(rf).max(), np.abs(rg).max())
        assert np.max(np.abs(_np(gf) - rf)) <= 1e-4 * scale, n
        assert np.max(np.abs(_np(gg) - rg)) <= 1e-4 * scale, n
        lam = (_np(gf), _np(gg))
    ctx.adjoint_steps(N - tail)
    grad = _np(ctx.gradient()).astype(np.float64)
    ctx.close()
    ref = Lbm(p, nsteps=N, precision="fp64", checkpoint_interval=C)
    J64, g64 = ref.value_and_grad(torch.from_numpy(w64))
    g64 = _np(g64)
    ref.close()
    err = np.linalg.norm(grad - g64) / np.linalg.norm(g64)
    print("%s: J %.8g (fp64 %.8g), gradient rel L2 %.3g" % (name, J, J64, err))
    assert abs(J - J64) <= 1e-4 * abs(J64)
    assert err <= 1e-3
