"""Parity at the full sizes of the workloads, in the launch configurations the
benchmark times: the lid-driven cavity 512^3 (D3Q19 TRT, tau 0.6, lid 0.1;
every storage format the benchmark reports), the ensemble of 256 lattices of
32^3..96^3 (D3Q19 SRT, FP16S, batched and persistent launches, HIP graph) and
the Karman channel 1024 x 256 x 64 (D3Q27 TRT, FP16S, cylinder of radius 16,
equilibrium inflow/outflow cells).

The reference cannot step these lattices in seconds, so one GPU step from a
seeded synthetic state (every DDF drawn from a table of values w_i a, a
uniform in +-0.05, stored through the format by the reference) is compared
cell by cell on a sample.  A cell's update depends only on its 3x3x3
neighbourhood, which the reference steps as a small periodic lattice (the
sampled neighbourhoods side by side along x) from the same stored codes.
Wall cells hold the code of 0 and EQ cells the stored equilibrium of their
fixed density and velocity, as in the model.  The samples cover the
interior, every face, edge and corner, the lid, the ends of 256-cell row
segments and the cylinder surface; wall cells must keep their codes.  Properties that hold at any size complete it: the
persistent launch in a HIP graph equals one launch per lattice bit for bit
over 100 steps, and no step produces a non-finite value."""
import numpy as np
import pytest

import lbm_workloads as wl
from lbm_testlib import MIN_SAME_SYNTHETIC, TABLE, check_samples, model_walls, sample_points, say, synthetic_codes

pytestmark = pytest.mark.gpu

LAUNCH_FIELDS = ("mode", "block", "cells_per_lane", "persistent")


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def _arith(storage):
    return "fp64" if storage == "fp64" else "fp32"


# ------------------------------------------------------------ cavity 512^3
N_CAV = 512
CAVITY_EXTRA_CONFIGS = {
    "fp16s": [("rows256", dict(mode=0, block=256, cells_per_lane=1, persistent=0)),
              ("dense256", dict(mode=2, block=256, cells_per_lane=1, persistent=0)),
              ("rows64_cpl2", dict(mode=0, block=64, cells_per_lane=2, persistent=0))],
    "fp32": [("rows256", dict(mode=0, block=256, cells_per_lane=1, persistent=0))],
}


@pytest.fixture(scope="module")
def cavity_indices(lbm):
    """Table indices of the cavity state, shared by every format."""
    say("cavity 512^3: drawing the state's table indices")
    return [wl.table_indices(N_CAV ** 3, 512, i, TABLE) for i in range(19)]


@pytest.mark.parametrize("storage", ["fp16s", "fp32", "fp16", "fp16c", "p16_0s", "p16_1s", "p16_2c", "fp64"])
def test_cavity_512_sampled_parity(lbm, orc, cavity_indices, storage):
    n = N_CAV
    dims = (n, n, n)
    say(f"cavity 512^3 {storage}: generating state")
    flags = wl.cavity_flags(n, n, n)
    codes = model_walls(orc, storage, 19, synthetic_codes(orc, storage, 19, n ** 3, seed=512,
                                                           indices=cavity_indices), flags)
    pts = sample_points(dims, np.random.default_rng(5))
    p = lbm.make_params(n, n, n, q=19, collision="trt", storage=storage, arith=_arith(storage), tau=0.6,
                        wall_u=(0.0, 0.1, 0.0))
    with lbm.Lattices(p) as g:
        g.set_boundaries(0, flags)
        g.set_ddf(0, codes)
        best = g.autotune(2)                      # as the benchmark: reads the state, leaves it unchanged
        configs = [("autotuned", {k: best[k] for k in LAUNCH_FIELDS})] + CAVITY_EXTRA_CONFIGS.get(storage, [])
        for name, cfg in configs:
            g.set_ddf(0, codes)
            g.set_launch(**cfg)
            g.step(1)
            out = g.get_ddf(0)
            same, m = check_samples(orc, storage, 19, "trt", 0.6, dims, flags, codes, out, pts,
                                    f"cavity {storage} {name}", wall_u=(0.0, 0.1, 0.0))
            say(f"  {name} {cfg}: {m} sampled fluid cells, identical codes {same:.4f}")
            del out
        assert g.diagnostics(0)["nonfinite_cells"] == 0


# ------------------------------------------------------------ ensemble of 256 lattices
def test_ensemble_full_sampled_parity_and_graph(lbm, orc):
    specs = wl.ensemble_specs(count=256, seed=2112, lo=32, hi=96)
    storage = "fp16s"
    params = [lbm.make_params(sp["nx"], sp["ny"], sp["nz"], q=19, collision="srt", storage=storage,
                              tau=sp["tau"], force=sp["force"]) for sp in specs]
    say(f"ensemble of {len(specs)}: generating states")
    flags = [wl.ensemble_member_inputs(sp)[0] for sp in specs]
    codes = [model_walls(orc, storage, 19, synthetic_codes(orc, storage, 19, sp["nx"] * sp["ny"] * sp["nz"],
                                                           seed=7000 + k), flags[k])
             for k, sp in enumerate(specs)]
    rng = np.random.default_rng(9)
    finals = {}
    with lbm.Lattices(params) as g:
        for k in range(len(specs)):
            g.set_boundaries(k, flags[k])
            g.set_ddf(k, codes[k])
        g.set_launch(graph_steps=0)
        best = g.autotune(2)
        say("  autotuned", {k: best[k] for k in LAUNCH_FIELDS})
        # one step of the autotuned launch, sampled cells of every lattice
        g.step(1)
        total, same_total = 0, 0.0
        for k, sp in enumerate(specs):
            dims = (sp["nx"], sp["ny"], sp["nz"])
            out = g.get_ddf(k)
            pts = sample_points(dims, rng, n_random=16)[::5]
            # every value within the bar; the share of identical codes is
            # taken over all lattices together (~70 cells per lattice alone
            # spread too much)
            same, m = check_samples(orc, storage, 19, "srt", sp["tau"], dims, flags[k], codes[k], out, pts,
                                    f"ensemble lattice {k} {dims}", force=sp["force"], min_same=0.0)
            total += m
            same_total += same * m
        say(f"  autotuned one step: {total} sampled fluid cells over {len(specs)} lattices, "
            f"identical codes {same_total / total:.4f}")
        assert same_total / total >= MIN_SAME_SYNTHETIC
        # 100 steps: persistent launch replayed as a HIP graph vs one launch per lattice
        for name, cfg in [("per_lattice", dict(mode=0, block=128, cells_per_lane=1, persistent=0,
                                               graph_steps=0)),
                          ("persistent_graph100", dict(mode=2, block=256, cells_per_lane=1,
                                                       persistent=8, graph_steps=100)),
                          ("autotuned_graph100", dict({k: best[k] for k in LAUNCH_FIELDS}, graph_steps=100))]:
            for k in range(len(specs)):
                g.set_ddf(k, codes[k])
            g.set_launch(**cfg)
            g.step(100)
            finals[name] = [g.get_ddf(k) for k in range(len(specs))]
            say(f"  {name}: 100 steps done")
        for k in range(len(specs)):
            assert g.diagnostics(k)["nonfinite_cells"] == 0, k
    for name in ("persistent_graph100", "autotuned_graph100"):
        for k in range(len(specs)):
            assert np.array_equal(finals[name][k], finals["per_lattice"][k]), (name, k)


# ------------------------------------------------------------ Karman channel 1024 x 256 x 64
def test_karman_full_sampled_parity(lbm, orc):
    nx, ny, nz, R = 1024, 256, 64, 16.0
    cx, cy = nx / 4, ny / 2
    dims = (nx, ny, nz)
    storage, tau, u0 = "fp16s", 0.532, 0.05
    say("karman 1024x256x64: generating state")
    flags = wl.karman_flags(nx, ny, nz, R, cx, cy)
    codes = model_walls(orc, storage, 27, synthetic_codes(orc, storage, 27, nx * ny * nz, seed=1024), flags,
                        eq_u=(u0, 0.0, 0.0))
    ang = np.linspace(0, 2 * np.pi, 240, endpoint=False)
    ring = []
    for rr in (R - 1.0, R, R + 1.0):
        xs = np.floor(cx + rr * np.cos(ang)).astype(np.int64)
        ys = np.floor(cy + rr * np.sin(ang)).astype(np.int64)
        for z in (0, nz // 2, nz - 1):
            ring.append(np.stack([xs, ys, np.full_like(xs, z)], axis=1))
    pts = sample_points(dims, np.random.default_rng(11), extra=np.concatenate(ring))
    p = lbm.make_params(nx, ny, nz, q=27, collision="trt", storage=storage, arith="fp32", tau=tau,
                        eq_rho=1.0, eq_u=(u0, 0.0, 0.0))
    with lbm.Lattices(p) as g:
        g.set_boundaries(0, flags)
        g.set_ddf(0, codes)
        best = g.autotune(2)
        g.set_launch(**{k: best[k] for k in LAUNCH_FIELDS})
        g.step(1)
        out = g.get_ddf(0)
        same, m = check_samples(orc, storage, 27, "trt", tau, dims, flags, codes, out, pts, "karman fp16s")
        say(f"  autotuned {dict((k, best[k]) for k in LAUNCH_FIELDS)}: {m} sampled fluid cells, "
            f"identical codes {same:.4f}")
        assert g.diagnostics(0)["nonfinite_cells"] == 0
