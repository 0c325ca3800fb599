"""Poiseuille error against the centre velocity at constant Reynolds number
(Sec. 4.1, its figure of E against u_max at constant Re and R, panels
R = 31 and R = 63): D3Q19 SRT, Guo force, mid-grid bounce-back, a periodic
slab 4 cells long, run for 3 R^2 / nu steps.  At fixed Re and R,
u_max = Re nu / (2 R), so the sweep runs over tau (nu = (tau - 1/2) / 3) and
tau = 1 marks u_max = Re / (12 R).  Both radii run Re = 1, 10, 100 (at
Re = 0.1, the paper's fourth curve, FP16C has failed up to tau = 1.5 and the
comparisons below do not apply; the paper states the FP16C advantage for the
higher Reynolds numbers).  Each radius is swept the first time a test asks
for it.  The paper states, and the bars below check with margins:

* the error minimum stays close to tau = 1 (here, for both radii: FP64's
  minimum lies at tau in [0.9, 1.6], i.e. u_max within a factor 2 of its
  tau = 1 value, and the smallest tau and, where u_max < 1 there, tau = 2.5
  are at least 1.3x worse);
* at u_max >= u_max(tau = 1), FP16C is almost always better than FP16S (here:
  at every such point with u_max < 1, for both radii);
* the better a format resolves small numbers, the lower u_max can go before
  the error becomes large (here: at R = 31, Re = 1, tau = 0.55,
  u_max = 2.7e-4, FP16S stays within 10 % of FP64 while FP16C has failed,
  E > 0.5);
* without DDF shifting the 16-bit formats become very inaccurate (here: for
  Re <= 10 every unshifted point has failed, E > 0.5, or is at least 3x
  worse than shifted, and failed for tau <= 1; at Re = 100 the
  unshifted/shifted error ratio has a geometric mean over the sweep of at
  least 2, though single points come close to 1); FP32 benefits from
  shifting at low velocities (unshifted FP32 has failed at R = 31, Re = 1,
  tau = 0.55, and at R = 63, Re = 1, tau = 0.6, and is over 10x worse than
  shifted at R = 63, Re = 10, tau = 0.6) and FP64 does not notice it
  (within 1 % everywhere); shifted FP32 matches FP64 within 8 % at every
  point of R = 31 and within 25 % at R = 63, where 358 000 steps at
  tau = 0.6 leave it up to 20 % off (below FP64's error there, not above)."""
import math

import pytest

import lbm_workloads as wl
from lbm_testlib import say

pytestmark = pytest.mark.gpu

NX = 4
SWEEPS = {31: ((1.0, 10.0, 100.0), (0.55, 0.6, 0.75, 0.93, 1.0, 1.25, 1.5, 2.5)),
          63: ((1.0, 10.0, 100.0), (0.6, 0.75, 1.0, 1.25, 1.5, 2.5))}
POINTS = [(R, Re) for R, (res, _) in SWEEPS.items() for Re in res]
FP32_BAR = {31: 0.08, 63: 0.25}
FORMATS = ("fp64", "fp32", "fp16s", "fp16c")


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def u_max(R, Re, tau):
    return Re * (tau - 0.5) / 3.0 / (2 * R)


def run_panel(lbm, R, out):
    ny = nz = 2 * (R + 1)
    flags = wl.poiseuille_flags(NX, ny, nz, R)
    for Re in SWEEPS[R][0]:
        for tau in SWEEPS[R][1]:
            nu = (tau - 0.5) / 3.0
            u = u_max(R, Re, tau)
            force = 4 * nu * u / R ** 2                     # u_max = F R^2 / (4 nu)
            steps = int(3 * R * R / nu) // 1000 * 1000 + 1000
            u_ref = wl.poiseuille_profile(NX, ny, nz, R, force, nu)
            for fmt in FORMATS:
                for unshifted in (False, True):
                    arith = "fp64" if fmt == "fp64" else "fp32"
                    p = lbm.make_params(NX, ny, nz, q=19, collision="srt", storage=fmt, arith=arith, tau=tau,
                                        force=(force, 0, 0), unshifted=unshifted)
                    with lbm.Lattices(p) as g:
                        g.set_boundaries(0, flags)
                        g.set_launch(mode=2, block=256, graph_steps=1000)
                        g.step(steps)
                        out[(R, Re, tau, fmt, unshifted)] = g.diagnostics(0, u_ref)["l2_error"]
            say(f"R={R} Re={Re} tau={tau} u_max={u:.2e}: " +
                " ".join(f"{f}{'*' if s else ''}={out[(R, Re, tau, f, s)]:.2e}" for f in FORMATS for s in (False, True)))


class Panels(dict):
    """Errors keyed by (R, Re, tau, format, unshifted); a radius is swept on
    its first lookup."""

    def __init__(self, lbm):
        super().__init__()
        self.lbm = lbm

    def __missing__(self, key):
        if any(k[0] == key[0] for k in self):
            raise KeyError(key)
        run_panel(self.lbm, key[0], self)
        return self[key]


@pytest.fixture(scope="module")
def sweep(lbm):
    return Panels(lbm)


@pytest.mark.parametrize("R,Re", POINTS)
def test_error_minimum_near_tau_one(sweep, R, Re):
    taus = [t for t in SWEEPS[R][1] if u_max(R, Re, t) < 1.0]
    e = {t: sweep[(R, Re, t, "fp64", False)] for t in taus}
    best = min(e, key=e.get)
    assert 0.9 <= best <= 1.6, (R, Re, best, e)
    assert e[taus[0]] > 1.3 * e[best], (R, Re, e)
    if 2.5 in e:
        assert e[2.5] > 1.3 * e[best], (R, Re, e)


@pytest.mark.parametrize("R,Re", POINTS)
def test_fp16c_better_than_fp16s_at_high_velocity(sweep, R, Re):
    for t in SWEEPS[R][1]:
        if t >= 1.0 and u_max(R, Re, t) < 1.0:
            assert sweep[(R, Re, t, "fp16c", False)] < sweep[(R, Re, t, "fp16s", False)], (R, Re, t)


def test_small_numbers_allow_low_velocity(sweep):
    e64 = sweep[(31, 1.0, 0.55, "fp64", False)]
    assert abs(sweep[(31, 1.0, 0.55, "fp16s", False)] / e64 - 1) < 0.10
    assert sweep[(31, 1.0, 0.55, "fp16c", False)] > 0.5


@pytest.mark.parametrize("R,Re", POINTS)
def test_shifting(sweep, R, Re):
    log_ratio = {"fp16s": [], "fp16c": []}
    for t in SWEEPS[R][1]:
        if u_max(R, Re, t) >= 1.0:
            continue
        e64 = sweep[(R, Re, t, "fp64", False)]
        assert abs(sweep[(R, Re, t, "fp64", True)] / e64 - 1) < 0.01, (R, Re, t)
        assert abs(sweep[(R, Re, t, "fp32", False)] / e64 - 1) < FP32_BAR[R], (R, Re, t)
        for fmt in ("fp16s", "fp16c"):
            ratio = sweep[(R, Re, t, fmt, True)] / sweep[(R, Re, t, fmt, False)]
            log_ratio[fmt].append(math.log(ratio))
            if Re <= 10:
                assert ratio > 3.0 or sweep[(R, Re, t, fmt, True)] > 0.5, (R, Re, t, fmt, ratio)
                if t <= 1.0:
                    assert sweep[(R, Re, t, fmt, True)] > 0.5, (R, Re, t, fmt)
    for fmt, lr in log_ratio.items():
        assert math.exp(sum(lr) / len(lr)) > 2.0, (R, Re, fmt, lr)


def test_unshifted_fp32_worse_at_low_velocity(sweep):
    assert sweep[(31, 1.0, 0.55, "fp32", True)] > 0.5
    assert sweep[(63, 1.0, 0.6, "fp32", True)] > 0.5
    assert sweep[(63, 10.0, 0.6, "fp32", True)] > 10 * sweep[(63, 10.0, 0.6, "fp32", False)]
