"""FP64 CPU reference ("oracle") of the lattice Boltzmann hot path of
Lehmann et al., arXiv 2112.08926.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product package
``paper_2112_08926_amd`` never imports it, and the two share no code: the
arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, built with gcc), this
module only marshals numpy arrays into it.

Parity status per function (each is pinned by ``tests/test_oracle_*.py``):
  decode / encode (all six 16-bit formats)   pinned: Table 2, Fig. 2, IEEE via numpy
  velset / equilibrium                       pinned: moment identities, Table 1
  step (pull, bounce-back, SRT, TRT, Guo)    pinned: streaming, conservation, closed forms
  velocity clamp (incl. NaN)                 pinned: clamped moments at omega = 1, rho = 0 cell
  moving-wall bounce-back                    pinned: plane Couette closed form (exact)
  Guo source                                 pinned: its zeroth, first and second moments
  non-finite count before the clamp          pinned: rho = 0 and NaN cells
  moments / diagnostics                      pinned: closed forms, brute-force sums
``tests/test_oracle_mutations.py`` plants one plausible mistake at a time in
a copy of lbm_oracle.c and checks that these pins catch every one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# The mutation test (tests/test_oracle_mutations.py) points this at a build of
# a deliberately broken copy of lbm_oracle.c to show that the pins catch it.
_SO = os.environ.get("LBM_ORACLE_SO", _SO)

FORMATS = {"fp64": 0, "fp32": 1, "fp16": 2, "fp16s": 3, "fp16c": 4,
           "p16_0s": 5, "p16_1s": 6, "p16_2c": 7}
SIXTEEN_BIT = ("fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c")

SOLID, EQ, MOVING = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile lbm_oracle.c into liboracle.so with gcc (ISO C, no FMA
    contraction, OpenMP for the outer loop only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.oracle_decode.restype = ctypes.c_double
        L.oracle_decode.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.oracle_encode.restype = ctypes.c_uint32
        L.oracle_encode.argtypes = [ctypes.c_int, ctypes.c_float]
        L.oracle_step.restype = ctypes.c_int64
        _lib = L
    return _lib


class _Lattice(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("q", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("shifted", ctypes.c_int32),
                ("nthreads", ctypes.c_int32),
                ("omega", ctypes.c_double), ("omega_minus", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("wall_u", ctypes.c_double * 3),
                ("mrt_rates", ctypes.c_double * 19)]


def _ptr(a, ctype):
    """Pointer to the data of an array laid out as the C side reads it:
    C-contiguous, elements of the C type's size (an F-ordered view, which
    numpy returns e.g. for a[:, index_array], would be read scrambled)."""
    if not a.flags.c_contiguous or a.dtype.itemsize != ctypes.sizeof(ctype):
        raise ValueError(f"array passed to the reference must be C-contiguous {ctype.__name__}")
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _fmt(fmt) -> int:
    return FORMATS[fmt] if isinstance(fmt, str) else int(fmt)


# --------------------------------------------------------------------------
# number formats (Sec. 3, Table 2)
# --------------------------------------------------------------------------
def decode(fmt, codes) -> np.ndarray:
    """FP64 value of each 16-bit code of format ``fmt``."""
    c = np.ascontiguousarray(codes, dtype=np.uint16)
    out = np.empty(c.shape, dtype=np.float64)
    lib().oracle_decode_array(_fmt(fmt), _ptr(c, ctypes.c_uint16), _ptr(out, ctypes.c_double),
                              ctypes.c_int64(c.size))
    return out


def encode(fmt, x) -> np.ndarray:
    """16-bit code of each float32 ``x`` in format ``fmt``."""
    xf = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(xf.shape, dtype=np.uint16)
    lib().oracle_encode_array(_fmt(fmt), _ptr(xf, ctypes.c_float), _ptr(out, ctypes.c_uint16),
                              ctypes.c_int64(xf.size))
    return out


def store(fmt, values) -> np.ndarray:
    """Value each FP64 number holds after storage in ``fmt`` (FP64: itself;
    FP32: rounded to float; 16-bit: rounded to float, then to a code)."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = np.empty(v.shape, dtype=np.float64)
    lib().oracle_store_array(_fmt(fmt), _ptr(v, ctypes.c_double), _ptr(out, ctypes.c_double),
                             ctypes.c_int64(v.size))
    return out


# --------------------------------------------------------------------------
# velocity sets and equilibrium (Sec. 2.2)
# --------------------------------------------------------------------------
def velset(q: int):
    """(c[q,3] int, w[q] float64, opp[q] int) of D3Q7, D2Q9 (q = 9, c_z = 0),
    D3Q13, D3Q15, D3Q19 or D3Q27 (Table 1)."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    opp = np.zeros(q, dtype=np.int32)
    if lib().oracle_velset(q, _ptr(c, ctypes.c_int32), _ptr(w, ctypes.c_double),
                           _ptr(opp, ctypes.c_int32)) != 0:
        raise ValueError(f"unsupported velocity set with {q} directions")
    return c, w, opp


def equilibrium(q: int, rho: float, u, shifted: bool = True) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(q, dtype=np.float64)
    lib().oracle_equilibrium(q, int(shifted), ctypes.c_double(rho), _ptr(uu, ctypes.c_double),
                             _ptr(out, ctypes.c_double))
    return out


def relaxation_rates(tau: float, trt_magic: float = 0.25):
    """omega+ = 1/tau; TRT omega- from the magic parameter
    Lambda = (tau+ - 1/2)(tau- - 1/2)."""
    wp = 1.0 / tau
    wm = 1.0 / (0.5 + trt_magic / (tau - 0.5))
    return wp, wm


# The D3Q19 MRT moments in the order of the basis (rho, e, eps, j_x, q_x,
# j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y,
# m_z).  READING (the paper only names MRT): the rates d'Humieres et al.
# (2002) use, with the shear moments at omega = 1/tau; the conserved moments
# carry rate 0.
MRT_SHEAR = (9, 11, 13, 14, 15)


def mrt_rates(omega: float):
    s = [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, omega, 1.4, omega, 1.4, omega, omega, omega,
         1.98, 1.98, 1.98]
    return np.array(s)


def mrt_basis():
    """(M[19, 19], |row|^2[19]) of the D3Q19 MRT moment basis."""
    M = np.empty((19, 19))
    n2 = np.empty(19)
    lib().oracle_mrt_basis(_ptr(M, ctypes.c_double), _ptr(n2, ctypes.c_double))
    return M, n2


# --------------------------------------------------------------------------
# lattice
# --------------------------------------------------------------------------
class Lattice:
    """One lattice of the FP64 reference: DDFs f[q, N] (shifted by default),
    cell index n = x + (y + z ny) nx, flags uint8[N] with SOLID/EQ/MOVING."""

    def __init__(self, nx, ny, nz, q=19, tau=0.6, collision="srt", storage="fp64",
                 force=(0.0, 0.0, 0.0), wall_u=(0.0, 0.0, 0.0), trt_magic=0.25,
                 shifted=True, flags=None, omega=None, omega_minus=None, nthreads=0, rates=None):
        self.nx, self.ny, self.nz, self.q = int(nx), int(ny), int(nz), int(q)
        self.N = self.nx * self.ny * self.nz
        wp, wm = relaxation_rates(tau, trt_magic)
        if omega is not None:
            wp = omega
        if omega_minus is not None:
            wm = omega_minus
        s = mrt_rates(wp) if rates is None else np.asarray(rates, dtype=np.float64)
        self.p = _Lattice(self.nx, self.ny, self.nz, self.q,
                          {"srt": 0, "trt": 1, "mrt": 2}[collision], _fmt(storage), int(shifted),
                          int(nthreads), wp, wm,
                          (ctypes.c_double * 3)(*force), (ctypes.c_double * 3)(*wall_u),
                          (ctypes.c_double * 19)(*s))
        self.flags = (np.zeros(self.N, dtype=np.uint8) if flags is None
                      else np.ascontiguousarray(flags, dtype=np.uint8).reshape(self.N))
        self.f = np.zeros((self.q, self.N), dtype=np.float64)
        self.t = 0
        self.nonfinite_updates = 0

    @property
    def f(self) -> np.ndarray:
        """DDFs [q, N] in FP64; any array assigned is copied to C order."""
        return self._f

    @f.setter
    def f(self, value):
        v = np.ascontiguousarray(value, dtype=np.float64)
        if v.shape != (self.q, self.N):
            raise ValueError(f"DDF array of shape {v.shape}, expected {(self.q, self.N)}")
        self._f = v

    def init(self, rho=None, u=None):
        """DDFs = stored equilibrium of rho[N] and u[3, N] (rest state if None)."""
        rho = np.ones(self.N) if rho is None else np.ascontiguousarray(rho, np.float64).reshape(self.N)
        u = (np.zeros((3, self.N)) if u is None
             else np.ascontiguousarray(u, np.float64).reshape(3, self.N))
        lib().oracle_init(ctypes.byref(self.p), _ptr(rho, ctypes.c_double),
                          _ptr(u, ctypes.c_double), _ptr(self.flags, ctypes.c_uint8),
                          _ptr(self.f, ctypes.c_double))
        self.t = 0
        self.nonfinite_updates = 0
        return self

    def step(self, n=1):
        """n time steps; ``nonfinite_updates`` accumulates the fluid cells
        whose density or velocity before the clamp was not finite."""
        out = np.empty_like(self.f)
        for _ in range(int(n)):
            rc = lib().oracle_step(ctypes.byref(self.p), _ptr(self.f, ctypes.c_double),
                                   _ptr(out, ctypes.c_double), _ptr(self.flags, ctypes.c_uint8))
            if rc < 0:
                raise RuntimeError("oracle_step failed")
            self.nonfinite_updates += int(rc)
            self.f, out = out, self.f
            self.t += 1
        return self

    def moments(self):
        rho = np.empty(self.N)
        u = np.empty((3, self.N))
        lib().oracle_moments(ctypes.byref(self.p), _ptr(self.f, ctypes.c_double),
                             _ptr(self.flags, ctypes.c_uint8), _ptr(rho, ctypes.c_double),
                             _ptr(u, ctypes.c_double))
        return rho, u

    def diagnostics(self, u_ref=None) -> dict:
        out = np.zeros(11)
        ref = None
        if u_ref is not None:
            ref = np.ascontiguousarray(u_ref, np.float64).reshape(3, self.N)
        lib().oracle_diagnostics(ctypes.byref(self.p), _ptr(self.f, ctypes.c_double),
                                 _ptr(self.flags, ctypes.c_uint8),
                                 _ptr(ref, ctypes.c_double) if ref is not None else None,
                                 _ptr(out, ctypes.c_double))
        return {"mass": out[0], "momentum": out[1:4].copy(), "kinetic_energy": out[4],
                "u_max": out[5], "l2_error": out[6], "force_on_solid": out[7:10].copy(),
                "nonfinite_cells": int(out[10])}
