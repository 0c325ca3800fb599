"""lbm_diagnostics_noalloc, the diagnostics entry point for callers that
cannot allocate (its reduction scratch is a static device array of the
library), against lbm_diagnostics on the same states: two calls in a row,
the second on a smaller lattice, each bit-identical to the allocating entry
point with the same reference field (given on the device here, on the host
there), and the non-finite count reported the same way."""
import ctypes

import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import one_step_inputs, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def _same(a, b):
    for k in ("mass", "kinetic_energy", "u_max", "l2_error", "nonfinite_cells", "step", "nonfinite_updates"):
        assert getattr(a, k) == getattr(b, k), k
    assert list(a.momentum) == list(b.momentum)
    assert list(a.force_on_solid) == list(b.force_on_solid)


@pytest.mark.parametrize("storage", ["fp16c", "fp64"])
def test_noalloc_diagnostics_match_allocating_entry_point(lbm, storage):
    import torch
    dims = [(600, 40, 30), (37, 9, 5)]                 # the second call on the smaller lattice
    arith = "fp64" if storage == "fp64" else "fp32"
    params, inputs = [], []
    for k, (nx, ny, nz) in enumerate(dims):
        flags, rho, u = one_step_inputs(nx, ny, nz, 19, seed=91 + k)
        params.append(lbm.make_params(nx, ny, nz, q=19, collision="trt", storage=storage, arith=arith, tau=0.7,
                                      force=(1e-5, 0.0, 0.0), wall_u=(0.0, 0.05, 0.0)))
        inputs.append((flags, rho, u))
    with lbm.Lattices(params) as g:
        for k, (flags, rho, u) in enumerate(inputs):
            g.set_boundaries(k, flags)
            g.set_rho_u(k, rho, u)
        g.step(3)
        for rep in range(2):                           # the static scratch keeps the last call's contents
            for k, (flags, rho, u) in enumerate(inputs):
                u_ref = 0.5 * u
                ref_dev = torch.from_numpy(np.ascontiguousarray(u_ref)).to("cuda")
                torch.cuda.synchronize()
                a = lbm.lbm_diagnostics(g.h, k, flags.size, u_ref)
                b = lbm.lbm_diagnostics_noalloc(g.h, k, ref_dev.data_ptr())
                say("noalloc", storage, k, rep, b.mass, b.kinetic_energy, b.l2_error)
                _same(a, b)
                a0 = lbm.lbm_diagnostics(g.h, k, flags.size)
                b0 = lbm.lbm_diagnostics_noalloc(g.h, k, None)
                _same(a0, b0)
                assert b0.l2_error == -1.0 and b0.mass > 0


def test_noalloc_diagnostics_report_nonfinite_updates(lbm, orc):
    """A cell of zero density (f_0 = -1): after one step both entry points
    report the counted update and return LBM_ENONFINITE."""
    nx, ny, nz = 40, 6, 5
    N = nx * ny * nz
    codes = orc.encode("fp16c", np.zeros((19, N), np.float32))
    codes[0, 100] = orc.encode("fp16c", np.array([-1.0], np.float32))[0]
    with lbm.Lattices(lbm.make_params(nx, ny, nz, q=19, storage="fp16c")) as g:
        g.set_ddf(0, codes)
        g.step(1)
        d = lbm.LbmDiag()
        rc = lbm.library().lbm_diagnostics_noalloc(g.h, 0, None, ctypes.byref(d))
        a = lbm.lbm_diagnostics(g.h, 0, N)
    assert rc == -5 and d.nonfinite_updates == 1
    _same(a, d)


def test_noalloc_diagnostics_refuse_lattices_past_the_scratch(lbm):
    """A lattice of rows of one cell has one reduction tile per cell: 600 x 600
    of them need more than the 32 MiB static array, so the call is refused
    with LBM_EINVAL (and nothing else happens), while lbm_diagnostics
    serves it."""
    with lbm.Lattices(lbm.make_params(1, 600, 600, q=19, storage="fp16s")) as g:
        d = lbm.LbmDiag()
        rc = lbm.library().lbm_diagnostics_noalloc(g.h, 0, None, ctypes.byref(d))
        assert rc == -1 and "static array" in lbm.lbm_last_error()
        a = lbm.lbm_diagnostics(g.h, 0, 360000)
        assert a.mass == pytest.approx(360000.0, rel=1e-12)
