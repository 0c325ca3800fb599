"""A device allocation that fails inside the library leaves the handle in a
state that never launches on a missing or stale tile table: setting a
batched launch whose tile table cannot be allocated returns LBM_ENOMEM,
lbm_step then refuses to launch (LBM_EINVAL) instead of reading a freed or
null table, and once allocation works again a launch set anew steps exactly
like a handle that never saw the failure.  The device memory the handle
reports (lbm_info) is what it holds: it comes back to its value after
creation once the tile tables are rebuilt, also after the autotuner."""
import numpy as np
import pytest

import lbm_workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def _failing_allocator(lbm, stream):
    from paper_2112_08926_amd import _lib

    class Failing(_lib._TorchAllocator):
        fail = False

        def _alloc(self, nbytes, ctx):
            if self.fail:
                return None
            return super()._alloc(nbytes, ctx)
    return Failing(stream)


def test_failed_tile_table_blocks_steps_until_set_again(lbm):
    import torch
    specs = wl.ensemble_specs(count=3, seed=5, lo=16, hi=30)
    params = [lbm.make_params(s["nx"], s["ny"], s["nz"], storage="fp16s", tau=s["tau"], force=s["force"])
              for s in specs]
    inputs = [wl.ensemble_member_inputs(s) for s in specs]
    stream = torch.cuda.Stream()
    alloc = _failing_allocator(lbm, stream)
    h = lbm.lbm_create(params, stream, alloc)
    try:
        for k, (flags, rho, u) in enumerate(inputs):
            lbm.lbm_set_boundaries(h, k, flags, flags.size)
            lbm.lbm_set_rho_u(h, k, flags.size, rho, u)
        cfg = lbm.lbm_get_launch(h)
        assert cfg.mode == lbm.LAUNCH_BATCHED
        lbm.lbm_step(h, 2)
        alloc.fail = True
        cfg.mode = 2                                   # cell-contiguous tiles: a new table
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_launch(h, cfg)
        assert ei.value.code == -2                     # LBM_ENOMEM
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_step(h, 1)                         # no table: refused, nothing launched
        assert ei.value.code == -1
        alloc.fail = False
        lbm.lbm_set_launch(h, cfg)
        lbm.lbm_step(h, 3)
        got = [lbm.lbm_get_ddf(h, k, np.empty((19, f.size), np.uint16), f.size, 19) for k, (f, _, _) in enumerate(inputs)]
    finally:
        lbm.lbm_destroy(h)
    with lbm.Lattices(params) as g:
        for k, (flags, rho, u) in enumerate(inputs):
            g.set_boundaries(k, flags)
            g.set_rho_u(k, rho, u)
        g.step(2)
        g.set_launch(mode=2)
        g.step(3)
        for k in range(len(inputs)):
            assert np.array_equal(g.get_ddf(k), got[k]), k


def test_device_bytes_track_what_is_held(lbm):
    n = 48
    p = lbm.make_params(n, n, n, collision="trt", storage="fp16s", tau=0.6, wall_u=(0, 0.1, 0))
    with lbm.Lattices(p) as g:
        g.set_boundaries(0, wl.cavity_flags(n, n, n))
        held = g.info()["device_bytes"]
        g.autotune(1)
        g.set_launch(mode=0, block=256, cells_per_lane=1, persistent=0)
        g.get_rho_u(0)
        g.diagnostics(0, np.zeros(3 * n ** 3))
        g.set_rho_u(0, np.ones(n ** 3), np.zeros(3 * n ** 3))
        g.set_launch(mode=2, block=128)
        g.set_launch(mode=0, block=256)
        assert g.info()["device_bytes"] == held
