"""Karman vortex street (Sec. 4.3) in 3-D at reduced size 256 x 64 x 16,
D3Q27 TRT with equilibrium inflow/outflow cells and a bounce-back cylinder:
the FP64 GPU path against the FP64 reference's momentum-exchange force time
series (tests/golden/karman_reduced_forces.txt, written by the committed
reference script), and FP32/FP16C storage against FP64 on the time-averaged
drag."""
import os

import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
NX, NY, NZ, R, CX, CY, U0, TAU, EVERY = 256, 64, 16, 4.0, 64.0, 32.0, 0.05, 0.548, 250


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def golden():
    rows = []
    with open(os.path.join(HERE, "golden", "karman_reduced_forces.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                rows.append([float(v) for v in line])
    return np.array(rows)


def run(lbm, storage, steps):
    flags = wl.karman_flags(NX, NY, NZ, R, CX, CY)
    rho, u = wl.karman_fields(NX, NY, NZ, U0)
    arith = "fp64" if storage == "fp64" else "fp32"
    p = lbm.make_params(NX, NY, NZ, q=27, collision="trt", storage=storage, arith=arith, tau=TAU,
                        eq_rho=1.0, eq_u=(U0, 0.0, 0.0))
    out = []
    with lbm.Lattices(p) as g:
        g.set_boundaries(0, flags)
        g.set_rho_u(0, rho, u)
        for step in range(0, steps + 1, EVERY):
            if step:
                g.step(EVERY)
            d = g.diagnostics(0)
            out.append([step, *d["force_on_solid"]])
            assert d["nonfinite_cells"] == 0
    return np.array(out)


def test_fp64_forces_match_reference(lbm):
    """The FP64 force series over 2500 steps to 1e-12 of the largest force
    (the FP64 path's relative bar)."""
    ref = golden()
    say("karman fp64")
    got = run(lbm, "fp64", int(ref[-1, 0]))
    assert np.array_equal(got[:, 0], ref[:, 0])
    scale = np.abs(ref[:, 1:3]).max()
    err = np.abs(got[:, 1:] - ref[:, 1:]).max()
    say("  max force difference", err, "scale", scale)
    assert err <= 1e-12 * scale          # measured 5.4e-14 (relative 7.5e-15)


def test_fp16c_mean_drag_within_one_percent(lbm):
    ref = golden()
    say("karman fp16c")
    got = run(lbm, "fp16c", int(ref[-1, 0]))
    late = ref[:, 0] >= ref[-1, 0] / 2
    drag_ref = ref[late, 1].mean()
    drag = got[late, 1].mean()
    say("  mean drag fp16c", drag, "fp64", drag_ref)
    assert abs(drag / drag_ref - 1) < 1e-2
