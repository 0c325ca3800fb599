"""The FP64 reductions (lbm_diagnostics) against the reference's
diagnostics of the same stored state, in every storage format, on lattices
with walls, a moving lid and EQ cells: mass, momentum and kinetic energy
(Sec. 4.2's discrete sum), max |u|, the L2 error norm (Sec. 4.1) against a
reference field and the momentum-exchange force.  The GPU takes the moments
in the step's arithmetic (FP32 except the FP64 path) and sums in FP64; the
reference is FP64 throughout, so FP32 moments bound the agreement (a few
1e-7 relative), FP64 agrees to 1e-12.  Repeated calls are bit-identical
(fixed reduction order)."""
import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import decode_codes, one_step_inputs, ref_codes, say

pytestmark = pytest.mark.gpu

FORMATS = ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


@pytest.mark.parametrize("q,collision", [(19, "trt"), (27, "srt")])
@pytest.mark.parametrize("storage", FORMATS)
def test_diagnostics_of_a_stored_state(lbm, orc, storage, q, collision):
    """600 x 40 x 30 cells: rows of two 512-cell segments (the second
    ragged), 2400 row tiles, more than the 512 workgroups of the second
    reduction pass, so each of those sums five tiles."""
    nx, ny, nz = 600, 40, 30
    N = nx * ny * nz
    say("diagnostics", storage, q, collision)
    flags, rho, u = one_step_inputs(nx, ny, nz, q, seed=71 + q)
    force, wall_u, eq_u = (2e-5, -1e-5, 0.0), (0.0, 0.07, 0.02), (0.03, 0.0, 0.0)
    eq = (flags & wl.EQ) != 0
    rho[eq] = 1.01
    u[:, eq] = np.array(eq_u)[:, None]
    ref = orc.Lattice(nx, ny, nz, q=q, tau=0.7, collision=collision, storage=storage, force=force,
                      wall_u=wall_u, flags=flags).init(rho, u)
    ref.f = orc.store(storage, ref.f + wl.random_noise(q, N, seed=9) * (flags == 0))
    codes = ref_codes(orc, storage, ref.f)
    u_ref = 0.9 * u
    arith = "fp64" if storage == "fp64" else "fp32"
    p = lbm.make_params(nx, ny, nz, q=q, collision=collision, storage=storage, arith=arith, tau=0.7,
                        force=force, wall_u=wall_u, eq_rho=1.01, eq_u=eq_u)
    with lbm.Lattices(p) as g:
        g.set_boundaries(0, flags)
        g.set_ddf(0, codes)
        d = g.diagnostics(0, u_ref)
        d2 = g.diagnostics(0, u_ref)
    ref.f = decode_codes(orc, storage, codes)
    dr = ref.diagnostics(u_ref)
    for k in ("mass", "kinetic_energy", "u_max", "l2_error"):
        assert d[k] == d2[k], k                                    # fixed order: identical bits
    assert np.array_equal(d["force_on_solid"], d2["force_on_solid"])
    rel = 1e-12 if storage == "fp64" else 2e-6
    assert d["mass"] == pytest.approx(dr["mass"], rel=1e-12 if storage == "fp64" else 1e-7)
    for k in ("kinetic_energy", "u_max", "l2_error"):
        assert d[k] == pytest.approx(dr[k], rel=rel), (k, d[k], dr[k])
    mscale = np.abs(dr["momentum"]).max()
    assert np.allclose(d["momentum"], dr["momentum"], rtol=rel, atol=rel * mscale)
    fscale = np.abs(dr["force_on_solid"]).max()
    assert fscale > 0
    assert np.allclose(d["force_on_solid"], dr["force_on_solid"], rtol=rel, atol=rel * fscale)
    assert d["nonfinite_cells"] == 0 and d["nonfinite_updates"] == 0
