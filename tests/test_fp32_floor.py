"""How far FP32 arithmetic with FP32 storage carries the Taylor-Green run of
the FP32 parity test (D3Q19 SRT, periodic 32^3, tau 0.6, u0 0.05, 1000
steps) from the FP64 reference: the float32 emulation of the kernel
listing's operation order (tests/fp32_emulation.py) ends 2.0e-5 (relative
L2 of u) away from FP64.  That floor is set by rounding every stored DDF to
float32 each step, so the 1e-5 stated for FP32/FP32 cannot be met by this
operation order; the GPU test's bar is derived from it.  CPU only."""
import numpy as np
import pytest

import lbm_workloads as wl
from fp32_emulation import srt_run

N3, TAU, U0, STEPS = 32, 0.6, 0.05, 1000


def fp32_floor(orc, steps=STEPS):
    c, w, _ = orc.velset(19)
    rho, u = wl.taylor_green_fields(N3, N3, N3, U0)
    ref = orc.Lattice(N3, N3, N3, q=19, tau=TAU).init(rho, u)
    ref.step(steps)
    _, u_r = ref.moments()
    u_e = srt_run(c.tolist(), w, rho, u, (N3, N3, N3), TAU, steps)
    return float(np.linalg.norm(u_e - u_r) / np.linalg.norm(u_r))


@pytest.mark.slow
def test_fp32_floor_of_the_taylor_green_run(orc):
    err = fp32_floor(orc)
    print("float32 emulation vs FP64, relative L2 of u:", err)
    assert 1.5e-5 < err < 2.5e-5


def test_emulation_matches_reference_after_one_step(orc):
    """The emulation is the reference's step rounded to float32: after one
    step of a random periodic lattice the two differ by float32 rounding
    only.  The velocity of a cell is a sum of 19 stored float32 values (each
    rounded by at most 2^-24 of |f| <= 0.03) over a density rounded near 1,
    so they differ by a few 1e-8 absolute, far below what a wrong or
    missing term would change (1e-4 and more)."""
    c, w, _ = orc.velset(19)
    n = 6
    rho, u = wl.random_fields(n ** 3, seed=3)
    ref = orc.Lattice(n, n, n, q=19, tau=TAU).init(rho, u)
    ref.step(1)
    _, u_r = ref.moments()
    u_e = srt_run(c.tolist(), w, rho, u, (n, n, n), TAU, 1)
    assert np.abs(u_e - u_r).max() <= 1e-7
