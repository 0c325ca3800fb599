"""A numpy float32 emulation of the D3Q19 SRT step in the operation order of
the paper's kernel listing with DDF shifting (Sec. 2.2): the sums of the
pulled DDFs for the density (the 1 last) and, by alternating pair sums, the
momentum; u = j / rho with IEEE division; the shifted equilibrium in its
three-FMA form; the collision as one FMA.  Every operation rounds to float32
(an FMA is the exact float64 product plus the addend, rounded to float32).
Periodic lattices, no walls, no force.

Test infrastructure: it measures how far FP32 arithmetic with FP32 storage
itself carries a run from FP64 (the floor any FP32 implementation of this
order meets), which sets the tolerance of the GPU's FP32 Taylor-Green
parity test.  It shares nothing with the GPU library."""
from __future__ import annotations

import numpy as np

F32 = np.float32


def fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def _cdot(ci, x, y, z):
    """c_i . (x, y, z) for components in {-1, 0, 1}, additions only, in x, y, z order."""
    s = None
    for comp, v in zip(ci, (x, y, z)):
        if comp == 0:
            continue
        term = v if comp > 0 else -v
        s = term if s is None else (s + term if comp > 0 else s - v)
    return s if s is not None else np.zeros_like(x)


def equilibrium32(c, w, rho, ux, uy, uz):
    """Stored (shifted) equilibrium codes of float32 rho, u, as the
    initialisation computes them: C = -3 (ux ux + uy uy + uz uz) without
    fusion, B = 3 (c.u), w rho (1/2 (B B + C) + B) + w (rho - 1) in FMAs."""
    C = F32(-3) * (ux * ux + uy * uy + uz * uz)
    rhom1 = rho - F32(1)
    out = np.empty((len(w),) + rho.shape, F32)
    for i in range(len(w)):
        wi = F32(w[i])
        B = F32(3) * _cdot(c[i], ux, uy, uz)
        out[i] = fma32(wi * rho, fma32(np.full_like(B, 0.5), fma32(B, B, C), B), wi * rhom1)
    return out


def moments32(c, f):
    """rho = f0 + f1 + ... + 1 and u = j / rho with j the alternating pair sums, in float32."""
    r = f[0].copy()
    for i in range(1, len(f)):
        r = r + f[i]
    rho = r + F32(1)
    j = []
    for a in range(3):
        s = np.zeros_like(rho)
        for i in range(1, len(f), 2):
            comp = c[i][a]
            if comp > 0:
                s = s + f[i]
                s = s - f[i + 1]
            elif comp < 0:
                s = s + f[i + 1]
                s = s - f[i]
        j.append(s)
    return rho, [ja / rho for ja in j]


def srt_run(c, w, rho0, u0, dims, tau, steps):
    """`steps` SRT steps of a periodic lattice of dims (nx, ny, nz) from the
    equilibrium of rho0[N], u0[3, N]; returns the float32 velocity the
    moments of the final state give (after streaming, as the next step
    sees them), as float64 [3, N]."""
    nx, ny, nz = dims
    q = len(w)
    cs = F32(0.57735026918962576451)
    f = equilibrium32(c, w, rho0.astype(F32), *[u0[a].astype(F32) for a in range(3)])
    f = f.reshape(q, nz, ny, nx)
    om = F32(1.0 / tau)
    omw = F32(1) - om
    w32 = [F32(wi) for wi in w]

    def pull(g):
        return np.stack([np.roll(g[i], shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2)) for i in range(q)])

    for _ in range(steps):
        fp = pull(f)
        rho, (vx, vy, vz) = moments32(c, fp)
        ux, uy, uz = [np.minimum(np.maximum(v, -cs), cs) for v in (vx, vy, vz)]
        C = F32(-3) * fma32(ux, ux, fma32(uy, uy, uz * uz))
        rhom1 = rho - F32(1)
        u3x, u3y, u3z = F32(3) * ux, F32(3) * uy, F32(3) * uz
        half = np.full_like(rho, 0.5)
        w0 = w32[0]
        feq0 = fma32(w0 * rho, F32(0.5) * C, w0 * rhom1)
        out = np.empty_like(fp)
        out[0] = fma32(np.full_like(rho, omw), fp[0], om * feq0)
        for i in range(1, q, 2):
            wi = w32[i]
            B = _cdot(c[i], u3x, u3y, u3z)
            t = fma32(B, B, C)
            ei = fma32(wi * rho, fma32(half, t, B), wi * rhom1)
            ej = fma32(wi * rho, fma32(half, t, -B), wi * rhom1)
            out[i] = fma32(np.full_like(rho, omw), fp[i], om * ei)
            out[i + 1] = fma32(np.full_like(rho, omw), fp[i + 1], om * ej)
        f = out
    rho, u = moments32(c, pull(f))
    return np.stack([ua.reshape(-1).astype(np.float64) for ua in u])
