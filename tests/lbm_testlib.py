"""Helpers shared by the GPU parity tests: building matching GPU and reference
lattices from the same seeded inputs, and comparing their states.

Tolerances (derived from the arithmetic):
  FP64 storage + FP64 arithmetic: relative 1e-12 after many steps (the two
    sides differ only in FMA contraction and summation rounding, ~1e-16 per op);
  FP32 arithmetic, one step: a stored value f'_i = f_i - omega (f_i - feq_i)
    (+ the Guo source) carries the rounding of the final operations, a few
    eps |f_i| and eps |f'_i|, and the rounding of the density and velocity
    it is computed from: the density is a sum of the q pulled DDFs plus 1
    (error ~ eps (1 + sum |f_j|)), the velocity j / rho likewise, and feq_i
    depends on both with weight ~ w_i, scaled by the relaxation rate.  So
        E_i = K eps (omega_max w_i (1 + S) + |f'_i| + M),
    eps = 2^-24, S = q max |f_in| bounds the sum of the pulled |f_j|, M =
    max |f_in|; K = 4 for SRT and TRT (a float32 emulation of the SRT step
    stays below 1.6 eps omega w_i (1 + S)), 16 for MRT, whose moment
    transforms sum 19 terms with integer coefficients up to 24;
  the GPU's float result is within E_i of the exact value and its code the
    nearest to that float, the reference's code the nearest to the exact
    value, so |decoded GPU - reference| <= half spacing at the GPU code +
    half spacing at the reference code + E_i (float32: half an ulp each);
  16-bit formats: at least 99.8 % of the codes are identical on the
    near-equilibrium one-step states (the measured floor, 99.84 % for FP16C,
    is set by the values whose exact result lies within E_i of a rounding
    boundary between two codes: near zero the codes of FP16C and FP16S are
    closer together than E_i), at least 98 % on the white-noise full-size
    states (measured floor 98.6 %), which put more values near zero.
"""
from __future__ import annotations

import sys

import numpy as np

import lbm_workloads as wl

EPS32 = 2.0 ** -24
MIN_SAME_16BIT = 0.998
# The full-size sampled states are white noise around rest (each DDF one of
# 4096 values w_i a, a uniform in +-0.05), so about 1 % of the values lie
# closer to zero than where FP16C and FP16S codes are E_i apart; measured
# floor 98.6 % (an ensemble lattice in FP16S), 98.7 % for the FP16C cavity.
MIN_SAME_SYNTHETIC = 0.98


class StepBar:
    """E_i of the one-step FP32 comparison (see the module docstring) for
    velocity set q, relaxation time tau, collision and the pre-step DDFs."""

    def __init__(self, orc, q, tau, collision, f_in, trt_magic=0.25):
        _, w, _ = orc.velset(q)
        wp, wm = orc.relaxation_rates(tau, trt_magic)
        om = max(wp, wm) if collision == "trt" else (max(wp, 1.98) if collision == "mrt" else wp)
        M = float(np.abs(np.asarray(f_in, dtype=np.float64)).max()) if np.size(f_in) else 0.0
        K = 16.0 if collision == "mrt" else 4.0
        self.base = K * EPS32 * (om * w * (1.0 + q * M) + M)       # per direction i
        self.K = K

    def bound(self, ref_f):
        return self.base[:, None] + self.K * EPS32 * np.abs(ref_f)


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
        return np.ascontiguousarray(codes, dtype=np.float64)
    return orc.decode(storage, codes)


def half_spacing(orc, storage: str, values: np.ndarray) -> np.ndarray:
    """Half the distance to the neighbouring codes of each representable value."""
    codes = orc.encode(storage, values.astype(np.float32))
    mag = codes.astype(np.int64) & 0x7FFF
    up = orc.decode(storage, np.minimum(mag + 1, 0x7FFF).astype(np.uint16))
    down = orc.decode(storage, np.maximum(mag - 1, 0).astype(np.uint16))
    here = np.abs(orc.decode(storage, mag.astype(np.uint16)))
    return 0.5 * np.maximum(np.abs(up - here), np.abs(here - down))


def half_ulp32(values: np.ndarray) -> np.ndarray:
    v = np.abs(values.astype(np.float32))
    return 0.5 * (np.nextafter(v, np.float32(np.inf)).astype(np.float64) - v.astype(np.float64))


def assert_step_parity(orc, storage: str, gpu_codes: np.ndarray, ref_f: np.ndarray, label: str = "",
                       bar: StepBar | None = None, min_same: float | None = None):
    """One-step comparison of GPU stored codes with reference FP64 values
    computed from the same inputs (reference stored through the format).
    bar: the FP32 arithmetic bound (required for FP32 arithmetic); min_same:
    least fraction of identical codes (default MIN_SAME_16BIT for 16-bit
    formats).  Returns the fraction of identical codes."""
    if storage == "fp64":
        scale = np.abs(ref_f).max()
        err = np.abs(gpu_codes - ref_f).max()
        assert err <= 1e-13 * scale, (label, err, scale)
        return 1.0
    assert bar is not None, "FP32 arithmetic needs a StepBar"
    E = bar.bound(ref_f)
    if storage == "fp32":
        got = gpu_codes.astype(np.float64)
        bound = half_ulp32(got) + half_ulp32(ref_f) + E
        same = float(np.mean(gpu_codes == ref_f.astype(np.float32)))
    else:
        got = orc.decode(storage, gpu_codes)
        bound = half_spacing(orc, storage, got) + half_spacing(orc, storage, ref_f) + E
        same = float(np.mean(gpu_codes == ref_codes(orc, storage, ref_f)))
    err = np.abs(got - ref_f)
    bad = err > bound * (1 + 1e-12)
    assert not bad.any(), (label, int(bad.sum()), float(err[bad].max()) if bad.any() else 0.0,
                           float(bound[bad].min()) if bad.any() else 0.0)
    if storage != "fp32":
        floor = MIN_SAME_16BIT if min_same is None else min_same
        assert same >= floor, (label, "identical codes", same)
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


# ------------------------------------------------------------ sampled parity at full size
AMP, TABLE = 0.05, 4096


def synthetic_codes(orc, storage, q, N, seed, indices=None):
    """Stored codes [q, N]: direction i draws from the codes of w_i * a over
    a seeded table of a values (uniform in +-AMP), plane by plane."""
    _, w, _ = orc.velset(q)
    a = wl.uniform_table(TABLE, AMP, seed)
    table = ref_codes(orc, storage, w[:, None] * a[None, :])
    out = np.empty((q, N), dtype=table.dtype)
    for i in range(q):
        idx = indices[i] if indices is not None else wl.table_indices(N, seed, i, TABLE)
        np.take(table[i], idx, out=out[i])
    return out


def sample_points(dims, rng, n_random=1200, extra=None):
    """Distinct (x, y, z): the product of special coordinates per axis (both
    ends, their neighbours, the ends of 256-cell segments), random cells and
    `extra`."""
    axes = []
    for n in dims:
        s = {0, 1, 2, n - 3, n - 2, n - 1, n // 2}
        s |= {v for v in (255, 256, 257, 511, 512) if v < n}
        axes.append(sorted(v for v in s if 0 <= v < n))
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    r = np.stack([rng.integers(0, n, n_random) for n in dims], axis=1)
    parts = [g, r] + ([np.asarray(extra).reshape(-1, 3)] if extra is not None else [])
    pts = np.concatenate(parts).astype(np.int64)
    nx, ny = dims[0], dims[1]
    _, keep = np.unique(pts[:, 0] + nx * (pts[:, 1] + ny * pts[:, 2]), return_index=True)
    return pts[np.sort(keep)]


def check_samples(orc, storage, q, collision, tau, dims, flags, codes_in, codes_out, pts, label,
                  force=(0.0, 0.0, 0.0), wall_u=(0.0, 0.0, 0.0), min_same=MIN_SAME_SYNTHETIC):
    """Reference step of each sampled cell from its 3x3x3 neighbourhood;
    returns the fraction of identical codes and the number of compared
    non-wall cells.  Wall cells must keep their codes exactly; EQ cells are
    compared like fluid cells (the reference keeps the input's equilibrium
    codes, the device writes its own, which may round differently)."""
    nx, ny, nz = dims
    S = len(pts)
    off = np.arange(3) - 1
    X = (pts[:, 0][:, None] + off) % nx                   # [S, 3]: x - 1, x, x + 1
    Y = (pts[:, 1][:, None] + off) % ny
    Z = (pts[:, 2][:, None] + off) % nz
    # small lattice (3S, 3, 3): cell a + 3k + 3S (b + 3c) holds (X[k,a], Y[k,b], Z[k,c])
    big = (X[None, None, :, :] + nx * (Y.T[None, :, :, None] + ny * Z.T[:, None, :, None])).reshape(-1)
    centre_big = pts[:, 0] + nx * (pts[:, 1] + ny * pts[:, 2])
    centre_small = 3 * np.arange(S) + 1 + 12 * S
    fl3 = flags[big]
    ref = orc.Lattice(3 * S, 3, 3, q=q, tau=tau, collision=collision, storage=storage, force=force,
                      wall_u=wall_u, flags=fl3)
    ref.f = decode_codes(orc, storage, codes_in[:, big])
    bar = StepBar(orc, q, tau, collision, ref.f)
    ref.step(1)
    exp = ref.f[:, centre_small]
    got = codes_out[:, centre_big]
    solid = (flags[centre_big] & wl.SOLID) != 0
    assert np.array_equal(got[:, solid], codes_in[:, centre_big][:, solid]), label
    same = assert_step_parity(orc, storage, got[:, ~solid], exp[:, ~solid], label, bar=bar, min_same=min_same)
    return same, int((~solid).sum())


def model_walls(orc, storage, q, codes, flags, eq_rho=1.0, eq_u=(0.0, 0.0, 0.0)):
    """Put into SOLID cells the code of 0 and into EQ cells the stored
    equilibrium of (eq_rho, eq_u): what the model holds there (and what a
    step writes there), in place."""
    zero = ref_codes(orc, storage, np.zeros(q))
    eq = ref_codes(orc, storage, orc.equilibrium(q, eq_rho, np.asarray(eq_u, dtype=np.float64)))
    solid = np.flatnonzero(flags & wl.SOLID)
    eqm = np.flatnonzero((flags & (wl.EQ | wl.SOLID)) == wl.EQ)
    for i in range(q):
        codes[i][solid] = zero[i]
        codes[i][eqm] = eq[i]
    return codes
