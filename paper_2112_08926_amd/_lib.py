"""ctypes binding of liblbm.so (include/lbm.h).  Argument marshalling only:
every step of the lattice Boltzmann path runs in the library's HIP kernels.

The functions ``lbm_*`` below carry the names of the C functions and take the
same arguments in Python form; ``Lattices`` wraps a handle.
"""
from __future__ import annotations

import ctypes
import hashlib
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library shares with torch)

from . import tuning

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm.so")

STORAGE = {"fp64": 0, "fp32": 1, "fp16": 2, "fp16s": 3, "fp16c": 4,
           "p16_0s": 5, "p16_1s": 6, "p16_2c": 7}
COLLISION = {"srt": 0, "trt": 1, "mrt": 2}
ARITH = {"fp32": 0, "fp64": 1}
FLAG_SOLID, FLAG_EQ, FLAG_MOVING = 1, 2, 4
LAUNCH_PER_LATTICE, LAUNCH_BATCHED = 0, 1
_DTYPE = {0: np.float64, 1: np.float32}          # 16-bit formats: uint16 codes

_STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
           -4: "LBM_EUNSUPPORTED", -5: "LBM_ENONFINITE"}


class LbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_STATUS.get(code, code)}: {message}")
        self.code = code


class LbmParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("q", ctypes.c_int32), ("collision", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("arith", ctypes.c_int32), ("unshifted", ctypes.c_int32),
                ("tau", ctypes.c_double), ("trt_magic", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("wall_u", ctypes.c_double * 3),
                ("eq_rho", ctypes.c_double), ("eq_u", ctypes.c_double * 3)]


class LbmDiag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("kinetic_energy", ctypes.c_double), ("u_max", ctypes.c_double),
                ("l2_error", ctypes.c_double), ("force_on_solid", ctypes.c_double * 3),
                ("nonfinite_cells", ctypes.c_int64), ("step", ctypes.c_int64),
                ("nonfinite_updates", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"mass": self.mass, "momentum": np.array(self.momentum[:]),
                "kinetic_energy": self.kinetic_energy, "u_max": self.u_max,
                "l2_error": self.l2_error, "force_on_solid": np.array(self.force_on_solid[:]),
                "nonfinite_cells": int(self.nonfinite_cells), "step": int(self.step),
                "nonfinite_updates": int(self.nonfinite_updates)}


class LbmLaunch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("block", ctypes.c_int32),
                ("cells_per_lane", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LbmInfo(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("n_lattices", ctypes.c_int32), ("bytes_per_ddf", ctypes.c_int32),
                ("step", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_P = ctypes.c_void_p

_lib = None


def library_path() -> str:
    return _LIB_PATH


def library():
    """Load liblbm.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2112_08926_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(_LIB_PATH)
    S = ctypes.c_int
    sig = {
        "lbm_create": (S, [ctypes.POINTER(LbmParams), ctypes.c_int32, _P, _ALLOC_FN, _FREE_FN, _P,
                           ctypes.POINTER(_P)]),
        "lbm_set_boundaries": (S, [_P, ctypes.c_int32, _P]),
        "lbm_set_rho_u": (S, [_P, ctypes.c_int32, _P, _P]),
        "lbm_step": (S, [_P, ctypes.c_int64]),
        "lbm_get_rho_u": (S, [_P, ctypes.c_int32, _P, _P]),
        "lbm_set_ddf": (S, [_P, ctypes.c_int32, _P]),
        "lbm_get_ddf": (S, [_P, ctypes.c_int32, _P]),
        "lbm_diagnostics": (S, [_P, ctypes.c_int32, _P, ctypes.POINTER(LbmDiag)]),
        "lbm_step_diagnostics": (S, [_P, _P, ctypes.POINTER(LbmDiag)]),
        "lbm_diagnostics_noalloc": (S, [_P, ctypes.c_int32, _P, ctypes.POINTER(LbmDiag)]),
        "lbm_set_launch": (S, [_P, ctypes.POINTER(LbmLaunch)]),
        "lbm_get_launch": (S, [_P, ctypes.POINTER(LbmLaunch)]),
        "lbm_autotune": (S, [_P, ctypes.c_int32, ctypes.POINTER(LbmLaunch)]),
        "lbm_info_get": (S, [_P, ctypes.POINTER(LbmInfo)]),
        "lbm_synchronize": (S, [_P]),
        "lbm_destroy": (None, [_P]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_encode": (S, [ctypes.c_int32, _P, _P, ctypes.c_int64, _P]),
        "lbm_decode": (S, [ctypes.c_int32, _P, _P, ctypes.c_int64, _P]),
        "lbm_copy_probe": (S, [_P, _P, ctypes.c_size_t, _P]),
        "lbm_memory_probe": (S, [ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


_LIB_ID = None


def library_id() -> str:
    """SHA-256 of liblbm.so: names the build in the autotuning cache."""
    global _LIB_ID
    if _LIB_ID is None:
        h = hashlib.sha256()
        with open(_LIB_PATH, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 20), b""):
                h.update(chunk)
        _LIB_ID = h.hexdigest()
    return _LIB_ID


def lbm_last_error() -> str:
    msg = library().lbm_last_error()
    return msg.decode() if msg else ""


def _check(rc: int):
    if rc != 0:
        raise LbmError(rc, lbm_last_error())


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _host_ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(_P)


def make_params(nx, ny, nz, q=19, collision="srt", storage="fp32", arith="fp32", tau=0.6,
                trt_magic=0.25, force=(0.0, 0.0, 0.0), wall_u=(0.0, 0.0, 0.0), eq_rho=1.0,
                eq_u=(0.0, 0.0, 0.0), unshifted=False) -> LbmParams:
    return LbmParams(int(nx), int(ny), int(nz), int(q), COLLISION.get(collision, collision),
                     STORAGE.get(storage, storage), ARITH.get(arith, arith), int(bool(unshifted)), float(tau),
                     float(trt_magic), (ctypes.c_double * 3)(*force), (ctypes.c_double * 3)(*wall_u),
                     float(eq_rho), (ctypes.c_double * 3)(*eq_u))


# ----------------------------------------------------------------- same-name wrappers
class _TorchAllocator:
    """Device allocator hooks backed by torch's caching allocator."""

    def __init__(self, stream):
        self.stream = stream
        self.alloc = _ALLOC_FN(self._alloc)
        self.free = _FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), self.stream)

    def _free(self, ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)


def lbm_create(params, stream=None, allocator: _TorchAllocator | None = None):
    """Returns the handle (a c_void_p)."""
    plist = [params] if isinstance(params, LbmParams) else list(params)
    arr = (LbmParams * len(plist))(*plist)
    h = _P()
    alloc = allocator.alloc if allocator else _ALLOC_FN(0)
    free = allocator.free if allocator else _FREE_FN(0)
    _check(library().lbm_create(arr, len(plist), _stream_ptr(stream), alloc, free, None, ctypes.byref(h)))
    return h


def _check_host(a, n: int, dtype, what: str) -> np.ndarray:
    """The library reads or writes exactly n elements of `dtype` at a host
    pointer; refuse anything else instead of letting it run past the array."""
    c = np.ascontiguousarray(a, dtype=dtype)
    if c.size != n:
        raise ValueError(f"{what}: {c.size} elements, the lattice needs {n}")
    return c


def lbm_set_boundaries(h, lattice: int, flags: np.ndarray, N: int):
    fl = _check_host(flags, N, np.uint8, "flags")
    _check(library().lbm_set_boundaries(h, lattice, _host_ptr(fl)))


def lbm_set_rho_u(h, lattice: int, N: int, rho: np.ndarray | None = None, u: np.ndarray | None = None):
    r = None if rho is None else _check_host(rho, N, np.float64, "rho")
    v = None if u is None else _check_host(u, 3 * N, np.float64, "u")
    _check(library().lbm_set_rho_u(h, lattice, _host_ptr(r), _host_ptr(v)))


def lbm_step(h, n_steps: int):
    _check(library().lbm_step(h, int(n_steps)))


def lbm_get_rho_u(h, lattice: int, N: int):
    rho = np.empty(N, dtype=np.float64)
    u = np.empty((3, N), dtype=np.float64)
    _check(library().lbm_get_rho_u(h, lattice, _host_ptr(rho), _host_ptr(u)))
    return rho, u


def _ddf_dtype(bytes_per_ddf: int):
    return {8: np.float64, 4: np.float32, 2: np.uint16}[bytes_per_ddf]


def lbm_set_ddf(h, lattice: int, codes: np.ndarray, N: int, q: int):
    """codes: q*N stored DDFs in the handle's storage type (float64, float32
    or uint16 codes)."""
    c = np.asarray(codes)
    if c.size != q * N:
        raise ValueError(f"codes: {c.size} elements, the lattice needs {q * N}")
    dt = _ddf_dtype(lbm_info_get(h).bytes_per_ddf)
    if c.dtype != dt:
        raise ValueError(f"codes must be {np.dtype(dt).name} for this storage")
    c = np.ascontiguousarray(c)
    _check(library().lbm_set_ddf(h, lattice, _host_ptr(c)))


def lbm_get_ddf(h, lattice: int, out: np.ndarray, N: int, q: int):
    if not out.flags.c_contiguous or out.size != q * N:
        raise ValueError(f"out must be a C-contiguous array of {q * N} elements")
    dt = _ddf_dtype(lbm_info_get(h).bytes_per_ddf)
    if out.dtype != dt:
        raise ValueError(f"out must be {np.dtype(dt).name} for this storage")
    _check(library().lbm_get_ddf(h, lattice, _host_ptr(out)))
    return out


def lbm_diagnostics(h, lattice: int, N: int, u_ref: np.ndarray | None = None) -> LbmDiag:
    """Returns the LbmDiag; raises LbmError on failure other than
    LBM_ENONFINITE (then the returned record has nonfinite_cells > 0 or
    nonfinite_updates > 0)."""
    d = LbmDiag()
    ref = None if u_ref is None else _check_host(u_ref, 3 * N, np.float64, "u_ref")
    rc = library().lbm_diagnostics(h, lattice, _host_ptr(ref), ctypes.byref(d))
    if rc not in (0, -5):
        _check(rc)
    return d


def lbm_step_diagnostics(h, u_ref_dev: int | None = None) -> LbmDiag:
    """One step fused with the diagnostics of the state it reads (a handle
    of one lattice); u_ref_dev: None or the device address of 3*N doubles.
    Raises like lbm_diagnostics."""
    d = LbmDiag()
    rc = library().lbm_step_diagnostics(h, u_ref_dev, ctypes.byref(d))
    if rc not in (0, -5):
        _check(rc)
    return d


def lbm_diagnostics_noalloc(h, lattice: int, u_ref_dev: int | None = None) -> LbmDiag:
    """lbm_diagnostics without allocation; u_ref_dev: None or the device
    address of 3*N doubles (e.g. a torch tensor's data_ptr()).  Raises like
    lbm_diagnostics."""
    d = LbmDiag()
    rc = library().lbm_diagnostics_noalloc(h, lattice, u_ref_dev, ctypes.byref(d))
    if rc not in (0, -5):
        _check(rc)
    return d


def lbm_set_launch(h, cfg: LbmLaunch):
    _check(library().lbm_set_launch(h, ctypes.byref(cfg)))


def lbm_get_launch(h) -> LbmLaunch:
    c = LbmLaunch()
    _check(library().lbm_get_launch(h, ctypes.byref(c)))
    return c


def lbm_autotune(h, trial_steps: int) -> LbmLaunch:
    c = LbmLaunch()
    _check(library().lbm_autotune(h, int(trial_steps), ctypes.byref(c)))
    return c


def lbm_info_get(h) -> LbmInfo:
    i = LbmInfo()
    _check(library().lbm_info_get(h, ctypes.byref(i)))
    return i


def lbm_synchronize(h):
    _check(library().lbm_synchronize(h))


def lbm_destroy(h):
    library().lbm_destroy(h)


def lbm_encode(storage, d_in: int, d_out: int, n: int, stream=None):
    _check(library().lbm_encode(STORAGE.get(storage, storage), d_in, d_out, int(n), _stream_ptr(stream)))


def lbm_decode(storage, d_in: int, d_out: int, n: int, stream=None):
    _check(library().lbm_decode(STORAGE.get(storage, storage), d_in, d_out, int(n), _stream_ptr(stream)))


def lbm_copy_probe(d_src: int, d_dst: int, nbytes: int, stream=None):
    _check(library().lbm_copy_probe(d_src, d_dst, int(nbytes), _stream_ptr(stream)))


PROBE = {"copy": 0, "read": 1, "read_misaligned": 2, "write": 3, "write_misaligned": 4}


def lbm_memory_probe(kind, d_src: int | None, d_dst: int, nbytes: int, stream=None):
    _check(library().lbm_memory_probe(PROBE.get(kind, kind), d_src, d_dst, int(nbytes), _stream_ptr(stream)))


# ----------------------------------------------------------------- convenience wrapper
class Lattices:
    """One handle: n lattices sharing velocity set, collision, storage and
    arithmetic.  `stream` defaults to a new torch stream of default priority
    (HIP graphs cannot be captured on the null stream); device memory comes
    from torch's caching allocator unless torch_alloc=False."""

    def __init__(self, params, stream=None, torch_alloc: bool = True):
        self.params = [params] if isinstance(params, LbmParams) else list(params)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self._alloc = _TorchAllocator(self.stream) if torch_alloc else None
        self.device = torch.cuda.current_device()
        self.h = lbm_create(self.params, self.stream, self._alloc)
        self.q = self.params[0].q
        self.storage = self.params[0].storage

    def N(self, k: int = 0) -> int:
        p = self.params[k]
        return p.nx * p.ny * p.nz

    def ddf_dtype(self):
        return _DTYPE.get(self.storage, np.uint16)

    def set_boundaries(self, k: int, flags):
        lbm_set_boundaries(self.h, k, flags, self.N(k))

    def set_rho_u(self, k: int, rho=None, u=None):
        lbm_set_rho_u(self.h, k, self.N(k), rho, u)

    def step(self, n: int = 1):
        lbm_step(self.h, n)

    def get_rho_u(self, k: int = 0):
        return lbm_get_rho_u(self.h, k, self.N(k))

    def get_ddf(self, k: int = 0) -> np.ndarray:
        out = np.empty((self.q, self.N(k)), dtype=self.ddf_dtype())
        return lbm_get_ddf(self.h, k, out, self.N(k), self.q)

    def set_ddf(self, k: int, codes):
        lbm_set_ddf(self.h, k, np.asarray(codes).astype(self.ddf_dtype(), copy=False), self.N(k), self.q)

    def diagnostics(self, k: int = 0, u_ref=None) -> dict:
        return lbm_diagnostics(self.h, k, self.N(k), u_ref).as_dict()

    def step_diagnostics(self, u_ref_dev: int | None = None) -> dict:
        """One step, returning the diagnostics of the state it read."""
        return lbm_step_diagnostics(self.h, u_ref_dev).as_dict()

    def set_launch(self, mode=None, block=None, cells_per_lane=None, persistent=None, graph_steps=None):
        c = lbm_get_launch(self.h)
        for name, v in (("mode", mode), ("block", block), ("cells_per_lane", cells_per_lane),
                        ("persistent", persistent), ("graph_steps", graph_steps)):
            if v is not None:
                setattr(c, name, int(v))
        lbm_set_launch(self.h, c)

    def launch(self) -> dict:
        return lbm_get_launch(self.h).as_dict()

    def autotune(self, trial_steps: int = 5, cache: str | None = None) -> dict:
        """Autotune the launch (lbm_autotune) and return it.  With `cache` (a
        JSON file path), a configuration cached for this ensemble, device and
        library build is applied instead of timing, and a new result is
        added to the file.  A cached entry the library rejects is tuned
        again and replaced."""
        if cache is None:
            return lbm_autotune(self.h, trial_steps).as_dict()
        props = torch.cuda.get_device_properties(self.device)
        key = tuning.ensemble_key(self.params, f"{props.name}|{props.gcnArchName}", library_id())
        hit = tuning.load(cache, key)
        if hit is not None:
            try:
                self.set_launch(**hit)
                return self.launch()
            except LbmError:
                pass
        best = lbm_autotune(self.h, trial_steps).as_dict()
        p = self.params[0]
        tuning.store(cache, key, best, note=f"q={p.q} storage={p.storage} lattices={len(self.params)}")
        return best

    def info(self) -> dict:
        i = lbm_info_get(self.h)
        return {k: int(getattr(i, k)) for k, _ in i._fields_}

    def synchronize(self):
        lbm_synchronize(self.h)

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
