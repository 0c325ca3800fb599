"""lbm_step_diagnostics, one step fused with the diagnostics of the state it
reads (the cadence of the paper's kinetic-energy samples, Sec. 4.2, and
drag/lift series, Sec. 4.3), against lbm_diagnostics followed by lbm_step on
a second handle with the same state: the diagnostics bit for bit and the
stepped DDF codes bit for bit, in every storage format, on a 600 x 40 x 30
lattice (rows of two 512-cell segments, the second ragged) with walls, a
moving lid, EQ cells and a body force; the reference field given on the
device; the step counters; and handles of several lattices refused."""
import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import one_step_inputs, ref_codes, say

pytestmark = pytest.mark.gpu

FORMATS = ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]
FIELDS = ("mass", "kinetic_energy", "u_max", "l2_error", "nonfinite_cells", "nonfinite_updates")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2112_08926_amd as lbm
    return torch, lbm, oracle


def _pair(lbm, orc, storage, q, collision, nx=600, ny=40, nz=30, seed=3):
    N = nx * ny * nz
    flags, rho, u = one_step_inputs(nx, ny, nz, q, seed=seed + q, with_moving=nz > 1)
    force, wall_u, eq_u = (2e-5, -1e-5, 0.0), (0.0, 0.07, 0.02), (0.03, 0.0, 0.0)
    eq = (flags & wl.EQ) != 0
    rho[eq] = 1.01
    u[:, eq] = np.array(eq_u)[:, None]
    ref = orc.Lattice(nx, ny, nz, q=q, tau=0.7, collision=collision, storage=storage, force=force,
                      wall_u=wall_u, flags=flags).init(rho, u)
    ref.f = orc.store(storage, ref.f + wl.random_noise(q, N, seed=9) * (flags == 0))
    codes = ref_codes(orc, storage, ref.f)
    arith = "fp64" if storage == "fp64" else "fp32"
    p = lbm.make_params(nx, ny, nz, q=q, collision=collision, storage=storage, arith=arith, tau=0.7,
                        force=force, wall_u=wall_u, eq_rho=1.01, eq_u=eq_u)
    gs = [lbm.Lattices(p), lbm.Lattices(p)]
    for g in gs:
        g.set_boundaries(0, flags)
        g.set_ddf(0, codes)
    return gs, u, N


@pytest.mark.parametrize("q,collision", [(19, "trt"), (27, "srt"), (19, "mrt")])
@pytest.mark.parametrize("storage", FORMATS)
def test_fused_step_matches_diagnostics_then_step(env, storage, q, collision):
    torch, lbm, orc = env
    say("step_diagnostics", storage, q, collision)
    (a, b), u, N = _pair(lbm, orc, storage, q, collision)
    try:
        u_ref = np.ascontiguousarray(0.9 * u)
        u_dev = torch.from_numpy(u_ref).cuda()
        da = a.diagnostics(0, u_ref)
        a.step(1)
        db = b.step_diagnostics(u_dev.data_ptr())
        torch.cuda.synchronize()
        for k in FIELDS:
            assert da[k] == db[k], (k, da[k], db[k])
        assert np.array_equal(da["momentum"], db["momentum"])
        assert np.array_equal(da["force_on_solid"], db["force_on_solid"])
        assert da["step"] == db["step"] == 0
        assert np.array_equal(a.get_ddf(0), b.get_ddf(0))
        assert a.info()["step"] == b.info()["step"] == 1
        # and the handles stay in step afterwards (the fused call flipped the buffers)
        a.step(5)
        b.step(5)
        assert np.array_equal(a.get_ddf(0), b.get_ddf(0))
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("q,collision,dims", [(9, "srt", (600, 40, 1)), (15, "trt", (600, 20, 12))])
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s", "fp16c", "p16_2c"])
def test_fused_step_other_velocity_sets(env, storage, q, collision, dims):
    """D2Q9 (one z-plane, no lid) and D3Q15: the same bit-identities."""
    torch, lbm, orc = env
    say("step_diagnostics", storage, q, collision, dims)
    (a, b), u, N = _pair(lbm, orc, storage, q, collision, *dims)
    try:
        da = a.diagnostics(0)
        a.step(1)
        db = b.step_diagnostics()
        for k in FIELDS:
            assert da[k] == db[k], (k, da[k], db[k])
        assert np.array_equal(da["momentum"], db["momentum"])
        assert np.array_equal(da["force_on_solid"], db["force_on_solid"])
        assert np.array_equal(a.get_ddf(0), b.get_ddf(0))
    finally:
        a.close()
        b.close()


def test_fused_steps_between_graph_steps(env):
    """A diagnostic step in the middle of graph-captured steps: the state
    after 1 + 1 + 10 steps equals that of 12 plain steps."""
    torch, lbm, orc = env
    (a, b), _, _ = _pair(lbm, orc, "fp16s", 19, "trt", nx=64, ny=32, nz=16)
    try:
        for g in (a, b):
            g.set_launch(graph_steps=4)
        a.step(12)
        b.step(1)
        d = b.step_diagnostics()
        assert d["step"] == 1
        b.step(10)
        assert np.array_equal(a.get_ddf(0), b.get_ddf(0))
        assert a.info()["step"] == b.info()["step"] == 12
    finally:
        a.close()
        b.close()


def test_fused_step_refuses_ensembles(env):
    torch, lbm, orc = env
    p = lbm.make_params(16, 8, 8, q=19, storage="fp16s")
    with lbm.Lattices([p, p]) as g:
        with pytest.raises(lbm.LbmError) as ei:
            g.step_diagnostics()
        assert ei.value.code == -4


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 3, 2), (70, 2, 3)])
@pytest.mark.parametrize("storage", ["fp32", "fp16s", "p16_1s"])
def test_fused_step_on_tiny_and_ragged_lattices(env, storage, dims):
    """Lattices smaller than a wavefront, and a row of 70 cells (one full and
    one nearly empty wavefront): the lanes past the row's end take part in
    the reduction without adding to it or storing."""
    torch, lbm, orc = env
    nx, ny, nz = dims
    (a, b), u, N = _pair(lbm, orc, storage, 19, "trt", nx=nx, ny=ny, nz=nz, seed=11)
    try:
        da = a.diagnostics(0)
        a.step(1)
        db = b.step_diagnostics()
        for k in FIELDS:
            assert da[k] == db[k], (k, da[k], db[k])
        assert np.array_equal(da["momentum"], db["momentum"])
        assert np.array_equal(da["force_on_solid"], db["force_on_solid"])
        assert np.array_equal(a.get_ddf(0), b.get_ddf(0))
    finally:
        a.close()
        b.close()
