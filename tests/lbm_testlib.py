"""Helpers shared by the GPU parity tests: building matching GPU and reference
lattices from the same seeded inputs, and comparing their states.

Tolerances (derived from the arithmetic):
  FP64 storage + FP64 arithmetic: relative 1e-12 after many steps (the two
    sides differ only in FMA contraction and summation rounding, ~1e-16 per op);
  FP32 arithmetic: one step differs from the FP64 reference by the FP32
    rounding of terms of size <= ~0.5, i.e. a few 1e-8 absolute; we allow
    ARITH32_ABS = 5e-7;
  16-bit storage: the GPU code must decode to within half a code spacing
    (the storage rounding) plus ARITH32_ABS of the reference's exact value.
"""
from __future__ import annotations

import sys

import numpy as np

import lbm_workloads as wl

ARITH32_ABS = 5e-7


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def gpu_params(nx, ny, nz, **kw):
    import paper_2112_08926_amd as lbm
    return lbm.make_params(nx, ny, nz, **kw)


def ordinal(codes: np.ndarray) -> np.ndarray:
    """Sign-magnitude 16-bit code -> integer in value order (+0 and -0 equal)."""
    c = codes.astype(np.int64)
    mag = c & 0x7FFF
    return np.where(c & 0x8000, -mag, mag)


def ref_codes(orc, storage: str, f: np.ndarray) -> np.ndarray:
    """Stored representation of reference DDFs f (values already representable)."""
    if storage == "fp64":
        return f.copy()
    if storage == "fp32":
        return f.astype(np.float32)
    return orc.encode(storage, f.astype(np.float32))


def decode_codes(orc, storage: str, codes: np.ndarray) -> np.ndarray:
    if storage in ("fp64", "fp32"):
        return codes.astype(np.float64)
    return orc.decode(storage, codes)


def half_spacing(orc, storage: str, values: np.ndarray) -> np.ndarray:
    """Half the distance to the neighbouring codes of each representable value."""
    codes = orc.encode(storage, values.astype(np.float32))
    mag = codes.astype(np.int64) & 0x7FFF
    up = orc.decode(storage, np.minimum(mag + 1, 0x7FFF).astype(np.uint16))
    down = orc.decode(storage, np.maximum(mag - 1, 0).astype(np.uint16))
    here = np.abs(orc.decode(storage, mag.astype(np.uint16)))
    return 0.5 * np.maximum(np.abs(up - here), np.abs(here - down))


def assert_step_parity(orc, storage: str, gpu_codes: np.ndarray, ref_f: np.ndarray, label: str = ""):
    """One-step comparison of GPU stored codes with reference FP64 values
    computed from the same inputs (reference stored through the format)."""
    if storage == "fp64":
        scale = np.abs(ref_f).max()
        err = np.abs(gpu_codes - ref_f).max()
        assert err <= 1e-13 * scale, (label, err, scale)
        return 1.0
    if storage == "fp32":
        err = np.abs(gpu_codes.astype(np.float64) - ref_f).max()
        assert err <= ARITH32_ABS, (label, err)
        return float(np.mean(gpu_codes == ref_f.astype(np.float32)))
    got = orc.decode(storage, gpu_codes)
    # |got - ref| <= (GPU rounding: half spacing at got) + (reference rounding:
    # half spacing at ref) + (FP32 arithmetic error before the rounding)
    bound = half_spacing(orc, storage, got) + half_spacing(orc, storage, ref_f) + ARITH32_ABS
    err = np.abs(got - ref_f)
    bad = err > bound * (1 + 1e-12)
    assert not bad.any(), (label, int(bad.sum()), float(err[bad].max()) if bad.any() else 0.0)
    same = float(np.mean(gpu_codes == ref_codes(orc, storage, ref_f)))
    return same


def one_step_inputs(nx, ny, nz, q, seed, solid_frac=0.05, with_eq=True, with_moving=True):
    """Flags with random walls, a moving lid plane and an EQ plane, plus random
    near-equilibrium fields."""
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    flags = np.where(rng.random(N) < solid_frac, wl.SOLID, 0).astype(np.uint8)
    f3 = flags.reshape(nz, ny, nx)
    if with_moving:
        f3[-1, :, :] = wl.SOLID | wl.MOVING
    if with_eq:
        f3[:, 0, :] = np.where(f3[:, 0, :] & wl.SOLID, f3[:, 0, :], wl.EQ)
    rho, u = wl.random_fields(N, seed)
    return flags, rho, u
