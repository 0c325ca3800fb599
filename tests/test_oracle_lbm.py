"""Pins of the FP64 reference lattice Boltzmann step against what the paper
and the mathematics fix: velocity-set isotropy and Table 1, moments of the
(shifted) equilibrium, pure streaming and bounce-back, exact conservation,
Guo forcing's momentum input, the rest state, the Taylor-Green closed form
and the Poiseuille profile."""
import math
import os

import numpy as np
import pytest

import lbm_workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))

# Listing 2 neighbour list: direction i in the order of its comments.
D3Q19_LISTING = ["000", "+00", "-00", "0+0", "0-0", "00+", "00-", "++0", "--0", "+0+", "-0-",
                 "0++", "0--", "+-0", "-+0", "+0-", "-0+", "0+-", "0-+"]


def _vec(s):
    return [{"+": 1, "-": -1, "0": 0}[ch] for ch in s]


def test_d3q19_order_matches_listing(orc):
    c, w, opp = orc.velset(19)
    assert c.tolist() == [_vec(s) for s in D3Q19_LISTING]
    # Sec. 2.2: u_x sums f1 f2 f7 f8 f9 f10 f13 f14 f15 f16 -- exactly the c_x != 0
    assert sorted(np.nonzero(c[:, 0])[0].tolist()) == [1, 2, 7, 8, 9, 10, 13, 14, 15, 16]
    assert set(np.round(w * 36).astype(int).tolist()) == {12, 2, 1}     # 1/3, 1/18, 1/36


@pytest.mark.parametrize("q", [9, 15, 19, 27])
def test_velocity_set_isotropy(orc, q):
    """Weights sum to one, odd moments vanish, and the second and fourth
    moments are those of an isotropic lattice with c_s^2 = 1/3 (in the xy
    plane for D2Q9, whose directions have c_z = 0)."""
    c, w, opp = orc.velset(q)
    dim = 2 if q == 9 else 3
    if q == 9:
        assert not c[:, 2].any()
    cf = c[:, :dim].astype(np.float64)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ cf, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, cf, cf), np.eye(dim) / 3.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, cf, cf, cf), 0.0, atol=1e-16)
    d = np.eye(dim)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, cf, cf, cf, cf), iso4, atol=1e-15)
    assert np.array_equal(c[opp], -c)
    assert len({tuple(v) for v in c.tolist()}) == q


def test_d3q7_and_d3q13_are_not_hydrodynamic_with_this_equilibrium(orc):
    """Why the step offers neither: D3Q7's second moment is c_s^2 = 1/4, so the
    equilibrium of Sec. 2.2 carries 3/4 of the momentum; D3Q13's fourth
    moment is not isotropic (the viscous stress would depend on direction)."""
    c, w, _ = orc.velset(7)
    cf = c.astype(np.float64)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, cf, cf), np.eye(3) / 4.0, atol=1e-15)
    feq = orc.equilibrium(7, 1.0, np.array([0.01, 0.0, 0.0]), shifted=True)
    assert (cf.T @ feq)[0] == pytest.approx(0.75 * 0.01, rel=1e-12)
    c, w, _ = orc.velset(13)
    cf = c.astype(np.float64)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, cf, cf), np.eye(3) / 3.0, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, cf, cf, cf, cf)
    assert m4[0, 0, 0, 0] != pytest.approx(3 * m4[0, 0, 1, 1], rel=1e-6)


def _table1():
    rows = {}
    with open(os.path.join(HERE, "golden", "table1_delta.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                name, d, ds = line.split()
                rows[int(name[3:])] = (float(d), float(ds))
    return rows


@pytest.mark.parametrize("q", [7, 9, 13, 15, 19, 27])
def test_table1_delta(orc, q):
    """Sec. 2.3: max_i |f_i^eq|/rho over u = c c_j/|c_j| (and u = 0), rounded up
    to two decimals, for the plain and the shifted equilibrium."""
    c, w, _ = orc.velset(q)
    cs = 1.0 / math.sqrt(3.0)
    dmax = dsmax = 0.0
    for j in range(q):
        u = np.zeros(3) if j == 0 else cs * c[j] / np.linalg.norm(c[j])
        dmax = max(dmax, np.abs(orc.equilibrium(q, 1.0, u, shifted=False)).max())
        dsmax = max(dsmax, np.abs(orc.equilibrium(q, 1.0, u, shifted=True)).max())
    d, ds = _table1()[q]
    assert math.ceil(dmax * 100 - 1e-9) / 100 == d
    assert math.ceil(dsmax * 100 - 1e-9) / 100 == ds


@pytest.mark.parametrize("q", [9, 15, 19, 27])
@pytest.mark.parametrize("shifted", [True, False])
def test_equilibrium_moments(orc, q, shifted):
    """Zeroth, first and second moments of f^eq (Sec. 2.2, shifted by the
    weights when shifting): rho (or rho-1), rho u, rho u u + p I (in the xy
    plane, with u_z = 0, for D2Q9)."""
    c, w, _ = orc.velset(q)
    dim = 2 if q == 9 else 3
    cf = c[:, :dim].astype(np.float64)
    rng = np.random.default_rng(q)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(3)
        u[dim:] = 0.0
        feq = orc.equilibrium(q, rho, u, shifted=shifted)
        shift = 1.0 if shifted else 0.0
        assert feq.sum() == pytest.approx(rho - shift, abs=1e-14)
        assert np.allclose(cf.T @ feq, rho * u[:dim], atol=1e-15)
        second = np.einsum("ia,ib,i->ab", cf, cf, feq)
        expect = rho * np.outer(u[:dim], u[:dim]) + (rho - shift) / 3.0 * np.eye(dim)
        assert np.allclose(second, expect, atol=1e-14)
    assert np.array_equal(orc.equilibrium(q, 1.0, np.zeros(3), shifted=True), np.zeros(q))
    assert np.allclose(orc.equilibrium(q, 1.0, np.zeros(3), shifted=False), w, atol=0)


@pytest.mark.parametrize("q", [7, 9, 13, 15, 19, 27])
def test_pure_streaming_moves_each_direction_by_c(orc, q):
    """With omega = 0 collision is the identity: one step moves the DDF of
    direction i from x to x + c_i, wrapping periodically (Listing 2 pull)."""
    nx, ny, nz = 5, 4, 3
    c, _, _ = orc.velset(q)
    lat = orc.Lattice(nx, ny, nz, q=q, omega=0.0, omega_minus=0.0)
    x0, y0, z0 = 0, 3, 2                                    # a corner: every c_i wraps somewhere
    n0 = x0 + nx * (y0 + ny * z0)
    lat.f[:, n0] = 1.0 + np.arange(q)
    lat.step()
    for i in range(q):
        xs, ys, zs = (x0 + c[i, 0]) % nx, (y0 + c[i, 1]) % ny, (z0 + c[i, 2]) % nz
        n1 = xs + nx * (ys + ny * zs)
        assert lat.f[i, n1] == 1.0 + i
        assert np.count_nonzero(lat.f[i]) == 1


@pytest.mark.parametrize("q", [9, 15, 19, 27])
def test_bounce_back_and_moving_wall(orc, q):
    """A DDF heading into a wall comes back reversed one step later at the same
    cell (mid-grid bounce-back); off a moving wall it gains 6 w rho_w c.u_w."""
    c, w, opp = orc.velset(q)
    nx = ny = nz = 5
    flags = np.zeros(nx * ny * nz, np.uint8)
    wall_u = (0.01, 0.02, -0.03)
    for moving in (False, True):
        for i in range(1, q):
            p = np.array([2, 2, 2])
            s = p + c[i]                                  # the wall cell DDF i runs into
            fl = flags.copy()
            ns = s[0] + nx * (s[1] + ny * s[2])
            fl[ns] = wl.SOLID | (wl.MOVING if moving else 0)
            lat = orc.Lattice(nx, ny, nz, q=q, omega=0.0, omega_minus=0.0, flags=fl, wall_u=wall_u)
            np0 = p[0] + nx * (p[1] + ny * p[2])
            lat.f[i, np0] = 0.25
            lat.step()
            o = opp[i]
            extra = 6.0 * w[o] * float(np.dot(c[o], wall_u)) if moving else 0.0
            assert lat.f[o, np0] == pytest.approx(0.25 + extra, abs=1e-17)


def _random_periodic(orc, q, collision, tau, force=(0, 0, 0), shape=(6, 5, 4), seed=5):
    nx, ny, nz = shape
    N = nx * ny * nz
    rho, u = wl.random_fields(N, seed)
    lat = orc.Lattice(nx, ny, nz, q=q, tau=tau, collision=collision, force=force).init(rho, u)
    lat.f += wl.random_noise(q, N, seed)
    return lat


@pytest.mark.parametrize("q", [9, 15, 19, 27])
@pytest.mark.parametrize("collision", ["srt", "trt"])
def test_mass_and_momentum_conservation(orc, q, collision):
    c, w, _ = orc.velset(q)
    lat = _random_periodic(orc, q, collision, 0.57)
    m0 = lat.f.sum()
    p0 = c.T.astype(float) @ lat.f.sum(axis=1)
    lat.step(50)
    assert lat.f.sum() == pytest.approx(m0, abs=1e-12)
    assert np.allclose(c.T.astype(float) @ lat.f.sum(axis=1), p0, atol=1e-13)


@pytest.mark.parametrize("q", [9, 15, 19, 27])
@pytest.mark.parametrize("collision", ["srt", "trt"])
def test_guo_force_adds_F_per_cell_per_step(orc, q, collision):
    """With the Guo force the total momentum of a periodic box grows by
    exactly F per cell and step, and mass stays conserved (F in the plane
    for D2Q9)."""
    c, _, _ = orc.velset(q)
    F = np.array([2e-5, -1e-5, 0.0 if q == 9 else 3e-5])
    lat = _random_periodic(orc, q, collision, 0.8, force=F)
    m0 = lat.f.sum()
    p0 = c.T.astype(float) @ lat.f.sum(axis=1)
    lat.step(10)
    p1 = c.T.astype(float) @ lat.f.sum(axis=1)
    assert np.allclose(p1 - p0, 10 * lat.N * F, rtol=1e-9, atol=1e-14)
    assert lat.f.sum() == pytest.approx(m0, abs=1e-12)


@pytest.mark.parametrize("q", [9, 15, 19, 27])
def test_trt_equals_srt_when_rates_match(orc, q):
    a = _random_periodic(orc, q, "srt", 0.7, force=(1e-5, 0, 0))
    b = _random_periodic(orc, q, "trt", 0.7, force=(1e-5, 0, 0))
    b.p.omega_minus = a.p.omega
    a.step(3)
    b.step(3)
    assert np.allclose(a.f, b.f, atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", [9, 15, 19, 27])
def test_srt_omega_one_gives_equilibrium(orc, q):
    lat = _random_periodic(orc, q, "srt", 1.0)
    lat.step()
    rho, u = lat.moments()
    # the stored DDFs at each cell are the equilibrium of the moments they had
    # after streaming; their own moments (without pulling) are those
    f = lat.f
    c, _, _ = orc.velset(q)
    r_own = f.sum(axis=0) + 1.0
    u_own = (c.T.astype(float) @ f) / r_own
    for n in range(0, lat.N, 7):
        feq = orc.equilibrium(q, r_own[n], u_own[:, n])
        assert np.allclose(f[:, n], feq, atol=1e-15)
    assert np.all(np.isfinite(rho)) and np.all(np.isfinite(u))


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"])
def test_rest_state_is_exactly_zero_and_stays_zero(orc, storage):
    """Sec. 2.2: with shifting the rest state is f^s = 0 exactly, in every
    storage format, also next to (moving-free) walls."""
    n = 8
    flags = wl.cavity_flags(n, n, n) & wl.SOLID
    lat = orc.Lattice(n, n, n, q=19, tau=0.6, collision="trt", storage=storage, flags=flags).init()
    assert not lat.f.any()
    lat.step(5)
    assert not lat.f.any()


@pytest.mark.parametrize("storage", ["fp32", "fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"])
def test_stored_values_are_representable(orc, storage):
    lat = _random_periodic(orc, 19, "srt", 0.6)
    lat.p.storage = orc.FORMATS[storage]
    lat.step()
    assert np.array_equal(orc.store(storage, lat.f), lat.f)


def test_taylor_green_decay_closed_form(orc):
    """Sec. 4.2: velocity decays as exp(-2 nu k^2 t) and energy as
    exp(-4 nu k^2 t); D3Q19 SRT, 32^3 periodic, tau 0.6, u0 0.05, 1000 steps.
    The lattice solution carries an O(k^2) correction: 0.5 % on the rate."""
    n, tau, u0, steps = 32, 0.6, 0.05, 1000
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / n
    rho, u = wl.taylor_green_fields(n, n, n, u0)
    lat = orc.Lattice(n, n, n, q=19, tau=tau).init(rho, u)
    e0 = lat.diagnostics()["kinetic_energy"]
    lat.step(steps)
    d = lat.diagnostics()
    rate_e = -math.log(d["kinetic_energy"] / e0) / steps
    assert rate_e / (4 * nu * k * k) == pytest.approx(1.0, abs=5e-3)
    _, u_t = lat.moments()
    _, u_ref = wl.taylor_green_fields(n, n, n, u0, t=steps, nu=nu)
    err = np.linalg.norm(u_t - u_ref) / np.linalg.norm(u_ref)
    assert err < 1.5e-2
    # exact mass conservation on the periodic box (FP64)
    assert d["mass"] == pytest.approx(rho.sum(), rel=1e-13)


def test_taylor_green_decay_closed_form_d2q9(orc):
    """The paper's Taylor-Green runs use D2Q9 SRT (Sec. 4.2): on a 64^2
    periodic box (tau 0.6, u0 0.05) the energy decays at 4 nu k^2 and the
    velocity field follows the closed form."""
    n, tau, u0, steps = 64, 0.6, 0.05, 2000
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / n
    rho, u = wl.taylor_green_fields(n, n, 1, u0)
    lat = orc.Lattice(n, n, 1, q=9, tau=tau).init(rho, u)
    e0 = lat.diagnostics()["kinetic_energy"]
    lat.step(steps)
    d = lat.diagnostics()
    rate_e = -math.log(d["kinetic_energy"] / e0) / steps
    assert rate_e / (4 * nu * k * k) == pytest.approx(1.0, abs=3e-3)
    _, u_t = lat.moments()
    _, u_ref = wl.taylor_green_fields(n, n, 1, u0, t=steps, nu=nu)
    assert np.linalg.norm(u_t - u_ref) / np.linalg.norm(u_ref) < 5e-3
    assert not u_t[2].any()


def test_poiseuille_profile_and_wall_force(orc):
    """Sec. 4.1: steady Poiseuille flow through a cylinder (Lx = 1), D3Q19 SRT,
    mid-grid bounce-back, Guo force; L2 error against the parabola small, and
    at steady state the walls take up the whole body force (momentum
    exchange)."""
    R, tau, F = 7, 0.8, 1e-5
    ny = nz = 2 * (R + 1)
    nu = (tau - 0.5) / 3.0
    flags = wl.poiseuille_flags(1, ny, nz, R)
    lat = orc.Lattice(1, ny, nz, q=19, tau=tau, force=(F, 0, 0), flags=flags).init()
    lat.step(6000)
    u_ref = wl.poiseuille_profile(1, ny, nz, R, F, nu)
    d = lat.diagnostics(u_ref)
    assert d["l2_error"] < 0.05
    n_fluid = int(np.count_nonzero(flags == 0))
    assert d["force_on_solid"][0] == pytest.approx(F * n_fluid, rel=2e-3)
    assert abs(d["force_on_solid"][1]) < 1e-9 and abs(d["force_on_solid"][2]) < 1e-9
    # the same run with 4 x-slices gives the same slice in every x
    lat4 = orc.Lattice(4, ny, nz, q=19, tau=tau, force=(F, 0, 0),
                       flags=wl.poiseuille_flags(4, ny, nz, R)).init()
    lat4.step(50)
    f4 = lat4.f.reshape(19, nz, ny, 4)
    assert all(np.array_equal(f4[..., 0], f4[..., x]) for x in range(1, 4))


def test_moments_and_diagnostics_consistent(orc):
    n = 6
    lat = _random_periodic(orc, 19, "srt", 0.7, shape=(n, n, n))
    rho, u = lat.moments()
    d = lat.diagnostics(u_ref=0.5 * u)
    assert d["mass"] == pytest.approx(rho.sum(), rel=1e-14)
    assert np.allclose(d["momentum"], (rho * u).sum(axis=1), rtol=1e-13)
    assert d["kinetic_energy"] == pytest.approx(0.5 * (rho * (u * u).sum(0)).sum(), rel=1e-13)
    assert d["u_max"] == pytest.approx(np.sqrt((u * u).sum(0)).max(), rel=1e-15)
    assert d["l2_error"] == pytest.approx(1.0, rel=1e-13)      # |u - u/2| / |u/2|
    assert d["nonfinite_cells"] == 0
    lat.f[3, 10] = np.nan
    assert lat.diagnostics()["nonfinite_cells"] >= 1


def test_trt_rates_and_viscosity(orc):
    """TRT: the symmetric rate 1/tau sets the viscosity nu = (tau - 1/2)/3
    (nomenclature table), the antisymmetric one follows from the magic
    parameter Lambda = (tau+ - 1/2)(tau- - 1/2) = 1/4."""
    for tau, tau_minus in ((0.6, 3.0), (0.51, 25.5), (0.548, 0.5 + 0.25 / 0.048)):
        wp, wm = orc.relaxation_rates(tau, 0.25)
        assert wp == pytest.approx(1.0 / tau) and 1.0 / wm == pytest.approx(tau_minus)
    n, tau, u0, steps = 32, 0.6, 0.02, 300
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / n
    rho, u = wl.taylor_green_fields(n, n, 4, u0)
    lat = orc.Lattice(n, n, 4, q=19, tau=tau, collision="trt").init(rho, u)
    e0 = lat.diagnostics()["kinetic_energy"]
    lat.step(steps)
    rate = -math.log(lat.diagnostics()["kinetic_energy"] / e0) / steps
    assert rate / (4 * nu * k * k) == pytest.approx(1.0, abs=1e-2)


# ---------------------------------------------------------------- MRT (D3Q19)
def test_mrt_basis_rows_are_the_polynomials_and_orthogonal(orc):
    """Rows of the moment basis are the stated polynomials of c_i (spot
    checks written out per direction class), mutually orthogonal, with the
    conserved moments rho, j as rows 0, 3, 5, 7."""
    M, n2 = orc.mrt_basis()
    c, _, _ = orc.velset(19)
    cf = c.astype(float)
    assert np.array_equal(M[0], np.ones(19))
    assert np.array_equal(M[3], cf[:, 0]) and np.array_equal(M[5], cf[:, 1]) and np.array_equal(M[7], cf[:, 2])
    # e: rest -30, faces -11, edges 8; eps: rest 12, faces -4, edges 1
    assert M[1, 0] == -30 and M[1, 1] == -11 and M[1, 7] == 8
    assert M[2, 0] == 12 and M[2, 1] == -4 and M[2, 7] == 1
    # q_x: faces -4 c_x, edges c_x
    assert M[4, 1] == -4 and M[4, 2] == 4 and M[4, 7] == 1 and M[4, 3] == 0
    # m_x on the edge ++0 is (cy^2 - cz^2) cx = 1
    assert M[16, 7] == 1 and M[16, 9] == -1
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.array_equal(np.diag(G), n2)


def test_mrt_with_equal_rates_is_srt(orc):
    """Every rate equal to omega: M^-1 (omega I) M = omega I, so MRT is the SRT
    step (with the Guo force as well)."""
    a = _random_periodic(orc, 19, "srt", 0.7, force=(1e-5, -2e-5, 3e-6))
    b = orc.Lattice(a.nx, a.ny, a.nz, q=19, tau=0.7, collision="mrt", force=(1e-5, -2e-5, 3e-6),
                    rates=np.full(19, 1 / 0.7))
    b.f = a.f.copy()
    a.step(3)
    b.step(3)
    assert np.allclose(a.f, b.f, atol=2e-16, rtol=0)


@pytest.mark.parametrize("forced", [False, True])
def test_mrt_conserves_mass_and_momentum(orc, forced):
    F = np.array([2e-5, -1e-5, 3e-5]) if forced else np.zeros(3)
    a = _random_periodic(orc, 19, "srt", 0.57)
    lat = orc.Lattice(a.nx, a.ny, a.nz, q=19, tau=0.57, collision="mrt", force=F)
    lat.f = a.f.copy()
    c, _, _ = orc.velset(19)
    m0 = lat.f.sum()
    p0 = c.T.astype(float) @ lat.f.sum(axis=1)
    lat.step(20)
    assert lat.f.sum() == pytest.approx(m0, abs=1e-12)
    assert np.allclose(c.T.astype(float) @ lat.f.sum(axis=1), p0 + 20 * lat.N * F, atol=1e-13)


def test_mrt_shear_viscosity_from_taylor_green_decay(orc):
    """The shear moments alone set the viscosity: the Taylor-Green energy
    decays at 4 nu k^2 with nu = (1/s_nu - 1/2)/3, whatever the other rates
    (two different sets of them give the same decay)."""
    n, tau, u0, steps = 24, 0.7, 0.03, 600
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / n
    rho, u = wl.taylor_green_fields(n, n, 1, u0)
    rates = []
    for alt in (False, True):
        r = orc.mrt_rates(1 / tau)
        if alt:
            r[[1, 2, 4, 6, 8, 10, 12, 16, 17, 18]] = [1.5, 1.1, 1.6, 1.6, 1.6, 1.2, 1.2, 1.7, 1.7, 1.7]
        lat = orc.Lattice(n, n, 1, q=19, tau=tau, collision="mrt", rates=r).init(rho, u)
        e0 = lat.diagnostics()["kinetic_energy"]
        lat.step(steps)
        rate = -math.log(lat.diagnostics()["kinetic_energy"] / e0) / steps
        rates.append(rate)
        assert rate / (4 * nu * k * k) == pytest.approx(1.0, abs=1e-2)
    assert rates[0] == pytest.approx(rates[1], rel=2e-3)


# ---------------------------------------------------------------- clamp, moving wall, Guo
def _cell_moments(c, f, shifted=True):
    """rho and u of stored DDFs f[q] of one cell, from their sums."""
    rho = f.sum() + (1.0 if shifted else 0.0)
    return rho, (c.T.astype(float) @ f) / rho


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("collision", ["srt", "trt"])
def test_clamp_limits_velocity_to_speed_of_sound(orc, q, collision):
    """The kernel listing clamps each velocity component to [-c, c],
    c = 1/sqrt(3).  A single periodic cell (every neighbour is itself) whose
    DDFs carry rho = 1 and j = (0.9, -0.9, 0.9): at omega = 1 the stored DDFs
    are the equilibrium of the clamped velocity, so their own moments give
    rho = 1 and u = (c, -c, c), although the pulled velocity was 0.9."""
    c, _, _ = orc.velset(q)
    cs = 1.0 / math.sqrt(3.0)
    lat = orc.Lattice(1, 1, 1, q=q, omega=1.0, omega_minus=1.0, collision=collision)
    f = np.zeros(q)
    f[1], f[2] = 0.45, -0.45                 # +x / -x: j_x = 0.9, sum 0
    f[3], f[4] = -0.45, 0.45                 # +y / -y: j_y = -0.9
    f[5], f[6] = 0.45, -0.45                 # +z / -z: j_z = 0.9
    lat.f = f[:, None]
    rho_in, u_in = _cell_moments(c, f)
    assert rho_in == 1.0 and np.allclose(u_in, [0.9, -0.9, 0.9], rtol=1e-15)
    lat.step()
    rho, u = _cell_moments(c, lat.f[:, 0])
    assert rho == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(u, [cs, -cs, cs], rtol=0, atol=1e-15)
    assert lat.nonfinite_updates == 0
    # below the limit the clamp does nothing: the same cell with j/4
    lat.f = (f / 4.0)[:, None]
    lat.step()
    assert np.allclose(_cell_moments(c, lat.f[:, 0])[1], [0.225, -0.225, 0.225], rtol=0, atol=1e-15)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("collision", ["srt", "trt", "mrt"])
def test_zero_density_is_counted_and_stays_finite(orc, q, collision):
    """A cell whose pulled DDFs give rho = 0 and j = 0 has the velocity 0/0,
    not finite before the clamp: the step counts it.  The listing's OpenCL
    clamp is fmin(fmax(u, -c), c), which maps NaN to a finite value, and
    the equilibrium at rho = 0 is -w_i whatever that value is, so at
    omega = 1 the cell stores -w_i exactly and stays finite (a blow-up the
    stored state alone would not show)."""
    if collision == "mrt" and q != 19:
        pytest.skip("MRT is D3Q19 only")
    _, w, _ = orc.velset(q)
    lat = orc.Lattice(1, 1, 1, q=q, omega=1.0, omega_minus=1.0, collision=collision,
                      rates=np.ones(19) if collision == "mrt" else None)
    f = np.zeros(q)
    f[0] = -1.0                              # shifted: rho = sum f + 1 = 0, j = 0
    lat.f = f[:, None]
    lat.step()
    assert lat.nonfinite_updates == 1
    assert np.all(np.isfinite(lat.f))
    assert np.allclose(lat.f[:, 0], -w, rtol=0, atol=1e-15)
    # the same with a non-finite DDF: counted, and the stored values are NaN
    lat.f = np.full((q, 1), np.nan)
    lat.step()
    assert lat.nonfinite_updates == 2 and np.isnan(lat.f).all()


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("collision", ["srt", "trt"])
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_couette_between_resting_and_moving_wall(orc, q, collision, tau):
    """Plane Couette flow: a resting wall at z = 0 and a wall moving with
    U along x at z = nz-1 (bounce-back with the 6 w_i c_i.u_w term off the
    moving wall, rho_w = 1), periodic in x and y.  The steady solution is
    the linear profile u_x = U (z - 1/2) / (nz - 2) with the walls half a
    cell outside the fluid, which mid-grid bounce-back reproduces exactly
    for any tau; u_y = u_z = 0 and rho = 1.  A wrong sign or factor of the
    moving-wall term changes the slope."""
    nz, U = 10, 0.01
    flags = np.zeros(nz, np.uint8)
    flags[0] = wl.SOLID
    flags[nz - 1] = wl.SOLID | wl.MOVING
    lat = orc.Lattice(1, 1, nz, q=q, tau=tau, collision=collision, wall_u=(U, 0.0, 0.0), flags=flags).init()
    lat.step(20000)
    rho, u = lat.moments()
    z = np.arange(1, nz - 1)
    assert np.abs(u[0, 1:-1] - U * (z - 0.5) / (nz - 2)).max() <= 1e-10 * U
    assert np.abs(u[1:, 1:-1]).max() <= 1e-14 * U
    assert np.abs(rho[1:-1] - 1.0).max() <= 1e-14


@pytest.mark.parametrize("q", [9, 15, 19, 27])
def test_guo_source_moments(orc, q):
    """The Guo source S_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i].F has zeroth
    moment 0, first moment F and second moment u F + F u (the moments that
    make the forcing second-order accurate).  At omega = 1 the SRT step
    stores feq(rho, u) + S_i / 2 with u = (j + F/2)/rho, so S is recovered
    from one step of a single periodic cell and its three moments are
    checked against these identities (a wrong coefficient in either part
    of S changes one of them)."""
    c, _, _ = orc.velset(q)
    cf = c.astype(np.float64)
    F = np.array([3e-4, -2e-4, 0.0 if q == 9 else 1e-4])
    rng = np.random.default_rng(123 + q)
    rho0, u0 = 1.01, np.array([0.03, -0.02, 0.0 if q == 9 else 0.04])
    f = orc.equilibrium(q, rho0, u0) + 1e-3 * rng.standard_normal(q)
    if q == 9:
        # keep the D2Q9 cell in the plane: no z component to leave
        f = f.copy()
    lat = orc.Lattice(1, 1, 1, q=q, omega=1.0, collision="srt", force=tuple(F))
    lat.f = f[:, None]
    rho = f.sum() + 1.0
    u = (cf.T @ f + 0.5 * F) / rho
    lat.step()
    S = 2.0 * (lat.f[:, 0] - orc.equilibrium(q, rho, u))
    assert abs(S.sum()) <= 1e-15
    assert np.allclose(cf.T @ S, F, rtol=1e-12, atol=1e-18)
    second = np.einsum("i,ia,ib->ab", S, cf, cf)
    expect = np.outer(u, F) + np.outer(F, u)
    if q == 9:
        second, expect = second[:2, :2], expect[:2, :2]
    assert np.allclose(second, expect, rtol=1e-10, atol=1e-17)
