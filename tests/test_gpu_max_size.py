"""Lattices at the largest sizes the interface accepts (N < 2^31 cells and
N * bytes per DDF < 2^32, the limits of 32-bit in-plane offsets): an FP32
cavity of 1024 x 1024 x 1023 (4.29 GB per direction plane) and an FP16S
cavity of 2048 x 1024 x 1023 (2.15e9 cells), each about 170 GB of HBM for
both DDF buffers.

One step from rest with a moving lid changes only the layer under the lid,
and every cell's update depends on its 3x3x3 neighbourhood only, so a small
reference cavity gives the exact expectation for any cell of the big one:
each coordinate maps to the small cavity's cell at the same distance from
the nearer wall, or to its middle when far from both.  Sampled cells (every
combination of near-wall and middle coordinates, including the last cells of
the lattice) are compared to the one-step bar, in the row launch and in the
cell-contiguous launch (whose per-lane offsets span the whole plane)."""
import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import StepBar, assert_step_parity, ref_codes, say

pytestmark = pytest.mark.gpu

SMALL = 12                      # reference cavity edge; middle cell 6
LID = (0.0, 0.1, 0.0)


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def coords(n):
    """Near-wall coordinates on both sides and the middle."""
    return np.array(sorted({0, 1, 2, 3, n // 2, n - 4, n - 3, n - 2, n - 1}), dtype=np.int64)


def to_small(c, n):
    return np.where(c < SMALL // 2, c, np.where(c >= n - SMALL // 2, c - (n - SMALL), SMALL // 2))


def expected(orc, storage, pts, dims):
    """Reference codes after one step from rest of the small cavity, at the
    cells the sampled big-lattice cells map to."""
    ref = orc.Lattice(SMALL, SMALL, SMALL, q=19, tau=0.6, collision="trt", storage=storage, wall_u=LID,
                      flags=wl.cavity_flags(SMALL, SMALL, SMALL)).init()
    ref.step(1)
    sx, sy, sz = (to_small(pts[:, a], dims[a]) for a in range(3))
    return ref.f[:, sx + SMALL * (sy + SMALL * sz)]


@pytest.mark.parametrize("storage,dims", [("fp32", (1024, 1024, 1023)), ("fp16s", (2048, 1024, 1023))])
def test_largest_lattice_one_step(lbm, orc, storage, dims):
    import torch
    torch.cuda.empty_cache()
    nx, ny, nz = dims
    N = nx * ny * nz
    b = 4 if storage == "fp32" else 2
    assert N < 2 ** 31 and N * b < 2 ** 32
    pts = np.stack(np.meshgrid(coords(nx), coords(ny), coords(nz), indexing="ij"), axis=-1).reshape(-1, 3)
    n_big = pts[:, 0] + nx * (pts[:, 1] + ny * pts[:, 2])
    exp = expected(orc, storage, pts, dims)
    say(f"max size {storage} {dims}: building flags ({N} cells)")
    flags = wl.cavity_flags(nx, ny, nz)
    p = lbm.make_params(nx, ny, nz, q=19, collision="trt", storage=storage, tau=0.6, wall_u=LID)
    with lbm.Lattices(p, torch_alloc=False) as g:
        for cfg in (dict(mode=0, block=256), dict(mode=2, block=256)):
            g.set_boundaries(0, flags)                    # also resets every cell to rest
            g.set_launch(**cfg)
            g.step(1)
            say(f"  {cfg}: stepped, copying {N * 19 * b / 1e9:.0f} GB out")
            got = g.get_ddf(0)[:, n_big]
            lid_layer = pts[:, 2] == nz - 2
            moved = np.abs(exp[:, lid_layer & (pts[:, 0] > 0) & (pts[:, 0] < nx - 1)
                               & (pts[:, 1] > 0) & (pts[:, 1] < ny - 1)]).max()
            assert moved > 1e-3                           # the lid has moved something
            assert_step_parity(orc, storage, got, exp, f"{storage} {cfg}",
                               bar=StepBar(orc, 19, 0.6, "trt", np.zeros((19, 1))))
            same = float(np.mean(got == ref_codes(orc, storage, exp)))
            say(f"  {cfg}: {len(n_big)} sampled cells, identical codes {same:.4f}")
            del got
