"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and by the
FP64 reference: geometry flags, initial density/velocity fields, analytic
reference fields and a counter-based random generator.

This module holds none of the lattice Boltzmann arithmetic (no equilibrium, no
streaming, no collision, no codec); it only describes the workloads of
Lehmann et al., arXiv 2112.08926, Sec. 4 and 5, at the sizes the tests and
the benchmark use.

Flag bits (one byte per cell): SOLID = 1 (bounce-back wall), EQ = 2 (cell held
at a fixed equilibrium), MOVING = 4 (together with SOLID: a wall moving with
the lattice's wall velocity).
"""
from __future__ import annotations

import math

import numpy as np

SOLID, EQ, MOVING = 1, 2, 4

_MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# splitmix64: the published counter-based generator (Steele, Lea, Flood 2014)
# --------------------------------------------------------------------------
def splitmix64(state: int):
    """Return (next_state, output) of one splitmix64 draw."""
    state = (state + 0x9E3779B97F4A7C15) & _MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return state, z ^ (z >> 31)


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state, out = splitmix64(self.state)
        return out

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        span = hi - lo + 1
        return lo + int(self.uniform() * span)


def cell_coords(nx, ny, nz):
    """x, y, z arrays of shape (N,) for n = x + (y + z ny) nx."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


# --------------------------------------------------------------------------
# Taylor-Green vortex (Sec. 4.2), extruded along z
# --------------------------------------------------------------------------
def taylor_green_fields(nx, ny, nz, u0=0.05, t=0.0, nu=0.0):
    """Density and velocity of the 2-D Taylor-Green vortex (Sec. 4.2) with one
    vortex period per box, k_x = 2 pi/nx, k_y = 2 pi/ny, uniform along z with
    u_z = 0, at time t:
      u_x =  u0 cos(k_x x) sin(k_y y) e^{-nu (k_x^2 + k_y^2) t}
      u_y = -u0 (k_x/k_y) sin(k_x x) cos(k_y y) e^{-nu (k_x^2 + k_y^2) t}
      rho = 1 - 3 u0^2/4 (cos(2 k_x x) + (k_x/k_y)^2 cos(2 k_y y)) e^{-2 nu (k_x^2 + k_y^2) t}
    which for a square box is the paper's solution (decay exp(-2 nu k^2 t)).
    Returns rho[N], u[3, N]."""
    x, y, _ = cell_coords(nx, ny, nz)
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    decay = math.exp(-nu * (kx * kx + ky * ky) * t)
    u = np.zeros((3, x.size))
    u[0] = u0 * np.cos(kx * x) * np.sin(ky * y) * decay
    u[1] = -u0 * (kx / ky) * np.sin(kx * x) * np.cos(ky * y) * decay
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * kx * x) + (kx / ky) ** 2 * np.cos(2 * ky * y)) * decay * decay
    return rho, u


# --------------------------------------------------------------------------
# Poiseuille flow through a cylinder (Sec. 4.1)
# --------------------------------------------------------------------------
def poiseuille_radius(ny, nz):
    """Cell-centred distance from the channel axis (centre of the y-z box)."""
    y = np.arange(ny) + 0.5 - ny / 2.0
    z = np.arange(nz) + 0.5 - nz / 2.0
    return np.sqrt(y[None, :] ** 2 + z[:, None] ** 2)          # [nz, ny]


def poiseuille_flags(nx, ny, nz, R):
    """Channel along x (periodic), cells with distance > R from the axis are
    bounce-back walls."""
    r = poiseuille_radius(ny, nz)
    plane = np.where(r > R, SOLID, 0).astype(np.uint8)          # [nz, ny]
    return np.broadcast_to(plane[:, :, None], (nz, ny, nx)).reshape(-1).copy()


def poiseuille_profile(nx, ny, nz, R, force, nu, rho=1.0):
    """Analytic velocity u_x(r) = f/(4 rho nu) (R^2 - r^2) inside the channel,
    0 in the walls.  Returns u[3, N]."""
    r = poiseuille_radius(ny, nz)
    ux = np.where(r > R, 0.0, force / (4.0 * rho * nu) * (R * R - r * r))
    u = np.zeros((3, nx * ny * nz))
    u[0] = np.broadcast_to(ux[:, :, None], (nz, ny, nx)).reshape(-1)
    return u


# --------------------------------------------------------------------------
# Lid-driven cavity (Sec. 4.4)
# --------------------------------------------------------------------------
def cavity_flags(nx, ny, nz):
    """One-cell walls on all six faces; the top z plane moves (MOVING|SOLID),
    with the lid velocity parallel to y given as the lattice's wall velocity."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[:, :, 0] = f[:, :, -1] = SOLID
    f[:, 0, :] = f[:, -1, :] = SOLID
    f[0, :, :] = SOLID
    f[-1, :, :] = SOLID | MOVING
    return f.reshape(-1)


# --------------------------------------------------------------------------
# Karman vortex street (Sec. 4.3), 3-D: flow along +x, cylinder along z
# --------------------------------------------------------------------------
def karman_flags(nx, ny, nz, radius, cx, cy):
    """Cylinder (axis along z) of the given radius as bounce-back wall;
    equilibrium cells on the x = 0, x = nx-1, y = 0 and y = ny-1 planes."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    inside = (x[None, :] - cx) ** 2 + (y[:, None] - cy) ** 2 <= radius * radius
    f[:, inside] = SOLID
    f[:, :, 0] = f[:, :, -1] = EQ
    f[:, 0, :] = f[:, -1, :] = EQ
    return f.reshape(-1)


def karman_fields(nx, ny, nz, u0):
    """Inflow velocity u0 along x on the half y < ny/2 (and on the EQ cells),
    rest elsewhere: the asymmetric start that triggers the instability."""
    x, y, _ = cell_coords(nx, ny, nz)
    rho = np.ones(x.size)
    u = np.zeros((3, x.size))
    u[0] = np.where(y < ny // 2, u0, 0.0)
    return rho, u


def karman_eq_mask(nx, ny, nz):
    x, y, _ = cell_coords(nx, ny, nz)
    return (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1)


# --------------------------------------------------------------------------
# Ensemble of uneven lattices
# --------------------------------------------------------------------------
def ensemble_specs(count=256, seed=2112, lo=32, hi=96, tau_lo=0.55, tau_hi=1.0):
    """Per-lattice dicts: sizes uniform in [lo, hi] per axis, tau uniform in
    [tau_lo, tau_hi]; even index -> Taylor-Green vortex, odd -> Poiseuille
    channel along x with R = min(ny, nz)//2 - 1 and force 1e-6."""
    g = SplitMix64(seed)
    specs = []
    for k in range(count):
        nx, ny, nz = g.randint(lo, hi), g.randint(lo, hi), g.randint(lo, hi)
        tau = tau_lo + (tau_hi - tau_lo) * g.uniform()
        kind = "tgv" if k % 2 == 0 else "poiseuille"
        spec = {"nx": nx, "ny": ny, "nz": nz, "tau": tau, "kind": kind}
        if kind == "poiseuille":
            spec["R"] = min(ny, nz) // 2 - 1
            spec["force"] = (1e-6, 0.0, 0.0)
        else:
            spec["u0"] = 0.05
            spec["force"] = (0.0, 0.0, 0.0)
        specs.append(spec)
    return specs


def ensemble_member_inputs(spec):
    """flags, rho, u for one ensemble member."""
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    if spec["kind"] == "tgv":
        rho, u = taylor_green_fields(nx, ny, nz, spec["u0"])
        return np.zeros(nx * ny * nz, dtype=np.uint8), rho, u
    flags = poiseuille_flags(nx, ny, nz, spec["R"])
    return flags, np.ones(nx * ny * nz), np.zeros((3, nx * ny * nz))


# --------------------------------------------------------------------------
# Random near-equilibrium states for one-step comparisons
# --------------------------------------------------------------------------
def random_fields(N, seed, u_amp=0.08, rho_amp=0.02):
    """rho[N] in 1 +- rho_amp, u[3, N] with components in +- u_amp."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_amp * (2.0 * rng.random(N) - 1.0)
    u = u_amp * (2.0 * rng.random((3, N)) - 1.0)
    return rho, u


def random_noise(q, N, seed, amp=1e-3):
    """Non-equilibrium perturbation of the DDFs, uniform in +- amp."""
    rng = np.random.default_rng(seed + 7919)
    return amp * (2.0 * rng.random((q, N)) - 1.0)


# --------------------------------------------------------------------------
# Full-size synthetic states, drawn plane by plane
# --------------------------------------------------------------------------
def uniform_table(size, amp, seed):
    """`size` values uniform in +- amp (sorted), the entries a full-size
    state draws from."""
    rng = np.random.default_rng(seed)
    return np.sort(amp * (2.0 * rng.random(size) - 1.0))


def table_indices(N, seed, plane, size):
    """N seeded indices uniform in [0, size) for one direction plane of a
    full-size state (numpy PCG64 seeded with (seed, plane))."""
    return np.random.default_rng([seed, plane]).integers(0, size, N, dtype=np.uint16)


# --------------------------------------------------------------------------
# Karman vortex street in two dimensions (Sec. 4.3 as the paper runs it)
# --------------------------------------------------------------------------
def karman2d_fields(nx, ny, u0):
    """Velocity u0 along +y on the left half x < nx/2 (the perimeter's EQ
    cells take u0 from the lattice's EQ state), rest elsewhere: the
    asymmetric start that triggers the instability at once."""
    x, y, _ = cell_coords(nx, ny, 1)
    rho = np.ones(x.size)
    u = np.zeros((3, x.size))
    u[1] = np.where(x < nx // 2, u0, 0.0)
    return rho, u
