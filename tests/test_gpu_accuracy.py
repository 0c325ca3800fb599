"""Accuracy of each storage format on the Poiseuille channel of Sec. 4.1
(256 x 64 x 64, R = 31, periodic along x, D3Q19 SRT, tau 0.8, Guo force
1e-6, 50 000 steps from rest): L2 error E against the parabola, compared with
the FP64 reference run with the same storage emulated
(tests/golden/poiseuille_r31_errors.txt)."""
import os

import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
R, TAU, F, STEPS, NX, NY = 31, 0.8, 1e-6, 50000, 256, 64


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def golden():
    out = {}
    with open(os.path.join(HERE, "golden", "poiseuille_r31_errors.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                out[line[0]] = (float(line[1]), float(line[2]))
    return out


@pytest.fixture(scope="module")
def gpu_errors(lbm):
    nu = (TAU - 0.5) / 3.0
    flags = wl.poiseuille_flags(NX, NY, NY, R)
    u_ref = wl.poiseuille_profile(NX, NY, NY, R, F, nu)
    errs = {}
    for fmt in ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]:
        say("poiseuille", fmt)
        arith = "fp64" if fmt == "fp64" else "fp32"
        with lbm.Lattices(lbm.make_params(NX, NY, NY, storage=fmt, arith=arith, tau=TAU,
                                          force=(F, 0, 0))) as g:
            g.set_boundaries(0, flags)
            g.step(STEPS)
            d = g.diagnostics(0, u_ref)
            rho, u = g.get_rho_u(0)
        # every x slice carries the same flow
        ux = u[0].reshape(NY, NY, NX)
        slice_spread = float(np.abs(ux - ux[:, :, :1]).max())
        errs[fmt] = (d["l2_error"], d["u_max"], slice_spread)
        if fmt in ("fp64", "fp32"):
            errs[fmt + "_u"] = u
        say("  E=%.4e umax=%.4e slice spread %.2e" % errs[fmt][:3])
    return errs


def test_fp64_and_fp32_match_reference(gpu_errors):
    """FP64 agrees with the reference to the 7 significant digits the golden
    file stores (one unit of the last digit is < 1.4e-7 relative here)."""
    g = golden()
    assert gpu_errors["fp64"][0] == pytest.approx(g["fp64"][0], rel=1.4e-7)
    assert gpu_errors["fp32"][0] == pytest.approx(g["fp64"][0], rel=1e-2)
    assert gpu_errors["fp64"][2] == 0.0 and gpu_errors["fp32"][2] == 0.0


def test_fp16c_within_twice_fp32_error(gpu_errors):
    """The 16-bit criterion E(16-bit) <= 2 E(FP32) holds for FP16C at this
    low velocity (u_max 2.4e-3); the other formats exceed it, as the
    reference with emulated storage also shows (Sec. 4.1: 16-bit errors grow
    at low velocity)."""
    assert gpu_errors["fp16c"][0] <= 2.0 * gpu_errors["fp32"][0]


@pytest.mark.parametrize("fmt", ["fp16", "fp16s", "fp16c", "p16_1s", "p16_2c"])
def test_16bit_error_tracks_reference(gpu_errors, fmt):
    """FP32 arithmetic with 16-bit storage ends within a factor 2 of the FP64
    reference with the same storage emulated."""
    e_ref = golden()[fmt][0]
    assert 0.5 * e_ref <= gpu_errors[fmt][0] <= 2.0 * e_ref, (fmt, gpu_errors[fmt][0], e_ref)


def test_p16_0s_stalls_like_reference(gpu_errors):
    """P16_0S resolves nothing below ~5e-7 near zero, so the force increments
    of this case are rounded away and the flow does not develop, on the GPU
    as in the reference."""
    g = golden()["p16_0s"]
    assert g[1] < 1e-5 and gpu_errors["p16_0s"][1] < 1e-5


@pytest.mark.parametrize("fmt", ["fp32", "fp16s", "fp16c"])
def test_without_ddf_shifting(lbm, gpu_errors, fmt):
    """Sec. 2.2 ablation (Sec. 4.1: without shifting the 16-bit formats become
    unfeasible, and FP32 benefits from shifting at low velocities).  The
    16-bit formats cannot represent the small changes of f_i ~ w_i at this
    velocity and the flow never develops (E ~ 1), as in the reference with
    the storage emulated.  FP32 arithmetic without shifting loses digits in
    rho = sum f_i ~ 1 and f_i - f_i^eq: its velocity field ends more than 3x
    further from the FP64 run's than the shifted FP32 field.  (The reference's
    fp32_unshifted line emulates only the storage, in FP64 arithmetic, and
    shows the storage part of this alone: E 7.50e-3 vs 7.39e-3.)"""
    nu = (TAU - 0.5) / 3.0
    flags = wl.poiseuille_flags(NX, NY, NY, R)
    u_ref = wl.poiseuille_profile(NX, NY, NY, R, F, nu)
    with lbm.Lattices(lbm.make_params(NX, NY, NY, storage=fmt, tau=TAU, force=(F, 0, 0),
                                      unshifted=True)) as g:
        g.set_boundaries(0, flags)
        g.step(STEPS)
        d = g.diagnostics(0, u_ref)
        _, u = g.get_rho_u(0)
    e_ref = golden()[fmt + "_unshifted"][0]
    say("unshifted", fmt, "E=%.4e ref %.4e" % (d["l2_error"], e_ref))
    if fmt == "fp32":
        u64 = gpu_errors["fp64_u"]
        dev_plain = np.linalg.norm(u - u64) / np.linalg.norm(u64)
        dev_shift = np.linalg.norm(gpu_errors["fp32_u"] - u64) / np.linalg.norm(u64)
        say("  FP32 field vs FP64: shifted %.3e, unshifted %.3e" % (dev_shift, dev_plain))
        assert dev_plain > 3 * dev_shift
    else:
        assert d["l2_error"] > 0.9 and e_ref > 0.9
