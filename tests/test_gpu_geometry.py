"""Row widths whose wave count is not a multiple of four (5, 6 and 7 waves per x
row: 64-, 192- and 64-thread blocks) against the FP64 oracle: recorded primal,
objective, adjoint and gradient, with ping-pong and in-place streaming, D2Q9 and
D3Q19 with their scalar lattices."""
import numpy as np
import pytest
import torch

import oracle
from paper_1501_04741_amd import inputs
from paper_1501_04741_amd.lbm import Lbm

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


CASES = [
    ("d2q9_d2q5_300", dict(flow=9, scalar=5, nx=300, ny=6, nz=1)),      # 5 waves: 5 x 64
    ("d3q19_350", dict(flow=19, scalar=0, nx=350, ny=4, nz=4)),         # 6 waves: 2 x 192
    ("d3q19_d3q7_448", dict(flow=19, scalar=7, nx=448, ny=4, nz=3)),    # 7 waves, no ragged lanes
]


@pytest.mark.parametrize("inplace", [False, True], ids=["ping_pong", "in_place"])
@pytest.mark.parametrize("name,shape", CASES, ids=[c[0] for c in CASES])
def test_row_widths_match_oracle(name, shape, inplace):
    steps = 24
    p = dict(shape, tau=0.8, tau_s=0.6, u_in=0.02, rho_out=1.0, switch_fn="ramp", switch_param=0.05, c_dp=1.0)
    if p["scalar"]:
        p.update(c_hf=0.5, c_var=1.0, s_in_lo=0.0, s_in_hi=1.0, s_split_axis=1)
    w = inputs.porosity(p["nx"], p["ny"], p["nz"], 2, 3)
    ctx = Lbm(p, nsteps=steps, precision="fp64", inplace=inplace)
    ctx.set_design(torch.from_numpy(w))
    ctx.primal_steps(steps, record=True)
    f, g = ctx.get_state()
    J, _ = ctx.objective()
    ctx.adjoint_steps(steps)
    grad = _np(ctx.gradient())
    ctx.close()
    ref = oracle.adjoint(p, w, steps)
    r = oracle.primal(p, w, steps)
    assert np.max(np.abs(_np(f) - r["f"])) < 1e-13
    if p["scalar"]:
        assert np.max(np.abs(_np(g) - r["g"])) < 1e-13
    assert abs(J - ref["J"]) <= 1e-10 * abs(ref["J"])
    assert np.linalg.norm(grad - ref["grad"]) <= 1e-10 * np.linalg.norm(ref["grad"])
