"""The sampled one-step check used at full size (each sampled cell stepped by
the reference from its 3x3x3 neighbourhood, the neighbourhoods side by side
in one small periodic lattice) against one reference step of the whole
lattice: on every cell of small walled lattices the two agree exactly, and a
neighbourhood gathered with a wrong index is caught."""
import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import check_samples, decode_codes, ref_codes, sample_points, synthetic_codes


def _full_step(orc, storage, q, collision, tau, dims, flags, codes, force=(0, 0, 0), wall_u=(0, 0, 0)):
    nx, ny, nz = dims
    ref = orc.Lattice(nx, ny, nz, q=q, tau=tau, collision=collision, storage=storage, force=force,
                      wall_u=wall_u, flags=flags)
    ref.f = decode_codes(orc, storage, codes)
    ref.step(1)
    return ref_codes(orc, storage, ref.f)


def _all_points(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], axis=1)


@pytest.mark.parametrize("storage,q,collision", [("fp16s", 19, "trt"), ("fp32", 19, "srt"),
                                                  ("p16_1s", 27, "trt"), ("fp16c", 19, "mrt")])
def test_sampled_step_equals_full_step(orc, storage, q, collision):
    dims = (13, 7, 6)
    N = 13 * 7 * 6
    flags = wl.cavity_flags(*dims)
    f3 = flags.reshape(6, 7, 13)
    f3[2, 3, 5] = wl.SOLID                          # an obstacle inside
    f3[1:5, 1:6, 10] = wl.EQ                        # an EQ plane
    codes = synthetic_codes(orc, storage, q, N, seed=3)
    kw = dict(force=(1e-4, 0, -2e-5), wall_u=(0, 0.1, 0))
    out = _full_step(orc, storage, q, collision, 0.57, dims, flags, codes, **kw)
    same, m = check_samples(orc, storage, q, collision, 0.57, dims, flags, codes, out, _all_points(dims),
                            "all cells", **kw)
    assert same == 1.0 and m == int(np.count_nonzero((flags & wl.SOLID) == 0))


def test_sampled_step_periodic_wrap(orc):
    """Cells on the faces of a periodic box pull across the wrap."""
    dims = (9, 5, 4)
    flags = np.zeros(9 * 5 * 4, dtype=np.uint8)
    codes = synthetic_codes(orc, "fp32", 19, flags.size, seed=4)
    out = _full_step(orc, "fp32", 19, "trt", 0.8, dims, flags, codes)
    pts = sample_points(dims, np.random.default_rng(0), n_random=10)
    same, _ = check_samples(orc, "fp32", 19, "trt", 0.8, dims, flags, codes, out, pts, "wrap")
    assert same == 1.0


def test_sampled_step_catches_a_wrong_neighbourhood(orc):
    """Output of a lattice whose x and y neighbours were swapped (a transposed
    index) fails the sampled check."""
    dims = (8, 8, 5)
    flags = wl.cavity_flags(*dims)
    codes = synthetic_codes(orc, "fp32", 19, flags.size, seed=6)
    # step the transposed lattice, then transpose its output back
    t = lambda a: a.reshape(a.shape[:-1] + (5, 8, 8)).swapaxes(-1, -2).reshape(a.shape)
    wrong = t(_full_step(orc, "fp32", 19, "trt", 0.6, dims, t(flags), t(codes), wall_u=(0, 0.1, 0)))
    with pytest.raises(AssertionError):
        check_samples(orc, "fp32", 19, "trt", 0.6, dims, flags, codes, wrong, _all_points(dims), "wrong",
                      wall_u=(0, 0.1, 0))
