"""A blow-up made visible in every storage format, and the velocity clamp
reached on both sides.

FP16C and the posits have no NaN or Inf and their encoders saturate
(Sec. 3.1.4 and the encoders of the conversion listing), so a cell whose
update goes non-finite would be stored as finite garbage.  The step counts,
before encoding, the cell updates whose density or velocity before the
velocity clamp is not finite; lbm_diagnostics reports them as
nonfinite_updates and returns LBM_ENONFINITE.  The reference counts the same
cells (oracle: non-finite density or velocity before the clamp).

The clamp is the kernel listing's OpenCL clamp(u, -c, c) = fmin(fmax(u, -c), c):
cells whose pulled velocity exceeds c = 1/sqrt(3) are stepped by the GPU and
by the reference from the same stored codes and compared to the one-step bar."""
import ctypes

import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import StepBar, assert_step_parity, ref_codes, say

pytestmark = pytest.mark.gpu

FORMATS = ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]
CASES = [(19, "srt"), (19, "trt"), (19, "mrt"), (27, "srt"), (27, "trt")]


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def _arith(storage):
    return "fp64" if storage == "fp64" else "fp32"


def _diag_status(lbm, g, k=0):
    d = lbm.LbmDiag()
    rc = lbm.library().lbm_diagnostics(g.h, k, None, ctypes.byref(d))
    return rc, d


@pytest.mark.parametrize("q,collision", CASES)
@pytest.mark.parametrize("storage", FORMATS)
def test_zero_density_cell_is_counted(lbm, orc, storage, q, collision):
    """One cell of a lattice at rest holds f_0 = -1 (shifted), so its pulled
    density is 0 and its momentum 0: the velocity 0/0 is not finite.  One
    step: the GPU counts exactly that update (LBM_ENONFINITE), the stored
    result is finite (the clamp maps NaN into [-c, c] and the equilibrium at
    rho = 0 does not depend on u) and equals the reference's to the one-step
    bar; the reference counts the same cell.  Before the step the
    diagnostics already see the 0/0 velocity in the stored state; after it
    the state is finite.  Counters reset on set_ddf."""
    nx, ny, nz = 70, 5, 4
    N = nx * ny * nz
    n0 = 3 + nx * (2 + ny * 1)
    say("zero density", storage, q, collision)
    ref = orc.Lattice(nx, ny, nz, q=q, tau=0.6, collision=collision, storage=storage)
    f = np.zeros((q, N))
    f[0, n0] = -1.0
    ref.f = f
    codes = ref_codes(orc, storage, f)
    p = lbm.make_params(nx, ny, nz, q=q, collision=collision, storage=storage, arith=_arith(storage), tau=0.6)
    with lbm.Lattices(p) as g:
        g.set_ddf(0, codes)
        rc, d = _diag_status(lbm, g)
        # the stored state already has a cell whose velocity is 0/0
        assert rc == -5 and d.nonfinite_cells == 1 and d.nonfinite_updates == 0
        g.step(1)
        rc, d = _diag_status(lbm, g)
        out = g.get_ddf(0)
        g.set_ddf(0, out)                       # re-initialising clears the count
        rc2, d2 = _diag_status(lbm, g)
    ref.step(1)
    assert ref.nonfinite_updates == 1
    assert rc == -5 and d.nonfinite_updates == 1, (rc, d.nonfinite_updates)
    assert d.nonfinite_cells == 0               # the stored state itself is finite
    assert rc2 == 0 and d2.nonfinite_updates == 0
    assert_step_parity(orc, storage, out, ref.f, f"zero density {storage} Q{q} {collision}",
                       bar=StepBar(orc, q, 0.6, collision, f))


@pytest.mark.parametrize("storage", ["fp32", "fp16", "fp16s"])
def test_nan_ddf_is_counted(lbm, orc, storage):
    """A cell holding NaN in every direction (only FP32, FP16 and FP16S have
    NaN codes): the cells x + c_i pull direction i from it, so q updates
    see a NaN density.  The diagnostics count those q cells in the decoded
    state before the step; the step counts the q updates."""
    nx, ny, nz = 40, 6, 5
    N = nx * ny * nz
    n0 = 7 + nx * (3 + ny * 2)
    q = 19
    codes = ref_codes(orc, storage, np.zeros((q, N)))
    codes[:, n0] = ref_codes(orc, storage, np.full((q, 1), np.nan))[:, 0]
    p = lbm.make_params(nx, ny, nz, q=q, collision="trt", storage=storage, tau=0.6)
    with lbm.Lattices(p) as g:
        g.set_ddf(0, codes)
        rc, d = _diag_status(lbm, g)
        assert rc == -5 and d.nonfinite_cells == q and d.nonfinite_updates == 0
        g.step(1)
        rc, d = _diag_status(lbm, g)
    ref = orc.Lattice(nx, ny, nz, q=q, tau=0.6, collision="trt", storage=storage)
    ref.f = np.where(np.isnan(orc.decode(storage, codes)) if storage != "fp32" else np.isnan(codes),
                     np.nan, 0.0)
    ref.step(1)
    assert ref.nonfinite_updates == q
    assert rc == -5 and d.nonfinite_updates == q, d.nonfinite_updates


def _clamp_inputs(nx, ny, nz, q, seed):
    """Random near-equilibrium fields with walls, a moving lid and an EQ
    plane, plus fast 3x3x3 blocks around ~0.05 % of the cells (about 1 % of
    the cells in all) whose velocity has |u_x| = 0.75 > c: the block centres
    pull a velocity above the clamp's limit."""
    from lbm_testlib import one_step_inputs
    flags, rho, u = one_step_inputs(nx, ny, nz, q, seed=seed)
    rng = np.random.default_rng(seed + 1)
    N = nx * ny * nz
    centres = rng.choice(N, size=max(2, N // 2000), replace=False)
    u3 = u.reshape(3, nz, ny, nx)
    fast = np.zeros((nz, ny, nx), bool)
    for c in centres:
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        xs, ys, zs = [(x + d) % nx for d in (-1, 0, 1)], [(y + d) % ny for d in (-1, 0, 1)], [(z + d) % nz for d in (-1, 0, 1)]
        sign = 1.0 if rng.random() < 0.5 else -1.0
        for zz in zs:
            for yy in ys:
                for xx in xs:
                    u3[0, zz, yy, xx] = 0.75 * sign
                    u3[1, zz, yy, xx] = 0.1
                    fast[zz, yy, xx] = True
    return flags, rho, u, centres, fast.reshape(-1)


@pytest.mark.parametrize("q,collision", CASES)
@pytest.mark.parametrize("storage", FORMATS)
def test_one_step_with_clamped_cells(lbm, orc, storage, q, collision):
    """One GPU step from the same stored codes as the reference on a lattice
    where about 1 % of the cells move faster than c: every fluid cell, the
    clamped ones included, within the one-step bar."""
    nx, ny, nz = 300, 6, 5
    say("clamp", storage, q, collision)
    flags, rho, u, centres, fast = _clamp_inputs(nx, ny, nz, q, seed=61 + q)
    force, wall_u = (1e-5, 0.0, 0.0), (0.0, 0.08, 0.0)
    ref = orc.Lattice(nx, ny, nz, q=q, tau=0.6, collision=collision, storage=storage, force=force, wall_u=wall_u,
                      flags=flags)
    eq = (flags & wl.EQ) != 0
    rho[eq] = 1.0
    u[:, eq] = 0.0
    ref.init(rho, u)
    codes = ref_codes(orc, storage, ref.f)
    bar = StepBar(orc, q, 0.6, collision, ref.f)
    # the reference's pulled velocity at the block centres exceeds c
    rp, up = ref.moments()
    fluid_centres = [c for c in centres if flags[c] == 0]
    assert fluid_centres and np.abs(up[0, fluid_centres]).max() > 1 / np.sqrt(3)
    p = lbm.make_params(nx, ny, nz, q=q, collision=collision, storage=storage, arith=_arith(storage), tau=0.6,
                        force=force, wall_u=wall_u)
    with lbm.Lattices(p) as g:
        g.set_boundaries(0, flags)
        g.set_ddf(0, codes)
        g.step(1)
        out = g.get_ddf(0)
        d = g.diagnostics(0)
    ref.step(1)
    assert d["nonfinite_updates"] == 0 and ref.nonfinite_updates == 0
    assert_step_parity(orc, storage, out, ref.f, f"clamp {storage} Q{q} {collision}", bar=bar)
