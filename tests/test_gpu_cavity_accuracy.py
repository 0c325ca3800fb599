"""The paper's lid-driven cavity (its Sec. 4 cavity and the DDF range section
with Table 1): 128^3, D3Q19 SRT, lid velocity 0.1 along y by moving
bounce-back, Re = L u0 / nu = 1000, 100 000 steps; u_y along the vertical
line and u_z along the horizontal line through the box centre, against the
GPU FP64 run (equal to the reference to 1e-12 in the parity tests).  The
paper states, and the bars below check with margins:

* with DDF shifting the formats deviate from FP64 only in the 4th digit of
  the relative velocity (here: max deviation along both lines below
  5e-4 u0 for every 16-bit format, below 1e-4 u0 for FP32), smallest for
  FP16C (here: below FP16 and FP16S; P16_1S also below FP16S; P16_2C is
  not the smallest in this run and is not asserted);
* without shifting the deviations grow to the 2nd digit (here: at least 5x
  the shifted deviation for FP16, FP16S and FP16C, above 1e-3 u0; FP32 also
  above 1e-3 u0, FP64 unchanged within 1e-9 u0);
* the DDFs accumulate around the weights w_i, the shifted ones around 0, and
  stay within 2 rho delta (Table 1, D3Q19: delta 0.34, shifted 0.17) (here,
  FP32 storage after 100 000 steps: per-direction medians within 10 % of
  w_i, respectively within 0.1 w_i of 0, and all fluid DDFs within the
  bounds with rho the largest density)."""
import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import say

pytestmark = pytest.mark.gpu

N, U0, RE, STEPS = 128, 0.1, 1000.0, 100000
TAU = 3 * N * U0 / RE + 0.5
RUNS = [("fp64", False), ("fp32", False), ("fp16", False), ("fp16s", False), ("fp16c", False), ("p16_1s", False),
        ("p16_2c", False), ("fp64", True), ("fp32", True), ("fp16", True), ("fp16s", True), ("fp16c", True)]
DELTA, DELTA_SHIFTED = 0.34, 0.17


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


@pytest.fixture(scope="module")
def runs(lbm, orc):
    flags = wl.cavity_flags(N, N, N)
    fluid = flags == 0
    _, w, _ = orc.velset(19)
    out = {}
    for storage, unshifted in RUNS:
        arith = "fp64" if storage == "fp64" else "fp32"
        p = lbm.make_params(N, N, N, q=19, collision="srt", storage=storage, arith=arith, tau=TAU,
                            wall_u=(0.0, U0, 0.0), unshifted=unshifted)
        with lbm.Lattices(p) as g:
            g.set_boundaries(0, flags)
            g.set_launch(mode=0, block=256, graph_steps=1000)
            g.step(STEPS)
            rho, u = g.get_rho_u(0)
            rec = {"rho_max": float(rho[fluid].max())}
            if storage == "fp32":
                f = g.get_ddf(0)[:, fluid].astype(np.float64)
                rec["f_absmax"] = float(np.abs(f).max())
                rec["median"] = np.median(f, axis=1)
        u = u.reshape(3, N, N, N)                                # [component, z, y, x]
        rec["vert"] = u[1, :, N // 2, N // 2]
        rec["hor"] = u[2, N // 2, :, N // 2]
        out[(storage, unshifted)] = rec
    ref = out[("fp64", False)]
    for key, rec in out.items():
        rec["dev"] = max(np.abs(rec["vert"] - ref["vert"]).max(), np.abs(rec["hor"] - ref["hor"]).max()) / U0
        say(f"cavity128 {key}: max deviation {rec['dev']:.2e} u0")
    out["w"] = w
    return out


def test_shifted_deviations_in_the_fourth_digit(runs):
    assert runs[("fp32", False)]["dev"] < 1e-4
    for storage in ("fp16", "fp16s", "fp16c", "p16_1s", "p16_2c"):
        assert runs[(storage, False)]["dev"] < 5e-4, storage
    fp16c = runs[("fp16c", False)]["dev"]
    assert fp16c < runs[("fp16", False)]["dev"] and fp16c < runs[("fp16s", False)]["dev"]
    assert runs[("p16_1s", False)]["dev"] < runs[("fp16s", False)]["dev"]


def test_unshifted_deviations_grow(runs):
    for storage in ("fp16", "fp16s", "fp16c"):
        plain, shifted = runs[(storage, True)]["dev"], runs[(storage, False)]["dev"]
        assert plain > 5 * shifted and plain > 1e-3, (storage, plain, shifted)
    assert runs[("fp32", True)]["dev"] > 1e-3
    assert runs[("fp64", True)]["dev"] < 1e-9


def test_ddf_ranges(runs):
    w = runs["w"]
    plain, shifted = runs[("fp32", True)], runs[("fp32", False)]
    assert np.all(np.abs(plain["median"] / w - 1) < 0.10), plain["median"] / w
    assert np.all(np.abs(shifted["median"]) < 0.1 * w), shifted["median"] / w
    assert plain["f_absmax"] <= 2 * plain["rho_max"] * DELTA
    assert shifted["f_absmax"] <= 2 * shifted["rho_max"] * DELTA_SHIFTED
