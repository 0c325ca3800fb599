"""Device memory per lattice point against the paper's memory table (Sec. 5,
memory requirements of the one-step-pull scheme with two DDF copies): the
paper keeps the velocity (d values), the density and one flag byte per
point besides the two copies of the q DDFs, that is 8 d + 9 + 16 q bytes for
FP64/FP64, 8 d + 9 + 8 q for FP64/FP32, 4 d + 5 + 8 q for FP32/FP32 and
4 d + 5 + 4 q for FP32/16-bit.  This library computes velocity and density
on demand and keeps one flag byte, a 32-bit wall-source mask and one bit per
64 cells instead, plus the FP64 partial sums of its diagnostics (12 doubles
per row tile of up to 512 cells: 96 / min(nx, 512) bytes per cell), so a
handle holds 2 q b + 5 + 96 / min(nx, 512) bytes per cell plus plane padding
and small tables (checked here within half a byte), below the paper's
figure for every variant.  Going from FP32 to 16-bit storage cuts the
footprint by 48 % for D3Q19 (the paper: about 45 %, with velocity and
density stored)."""
import pytest

pytestmark = pytest.mark.gpu

N3 = 128
D = 3


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def paper_bytes(arith, b, q):
    ab = 8 if arith == "fp64" else 4
    return ab * D + ab + 1 + 2 * b * q


def per_cell(lbm, q, storage, arith):
    p = lbm.make_params(N3, N3, N3, q=q, storage=storage, arith=arith)
    with lbm.Lattices(p) as g:
        info = g.info()
    return info["device_bytes"] / N3 ** 3, info["bytes_per_ddf"]


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,arith", [("fp64", "fp64"), ("fp32", "fp64"), ("fp32", "fp32"), ("fp16s", "fp32"),
                                           ("p16_1s", "fp32")])
def test_bytes_per_cell(lbm, q, storage, arith):
    per, b = per_cell(lbm, q, storage, arith)
    assert b == {"fp64": 8, "fp32": 4}.get(storage, 2)
    diag = 12 * 8 / min(N3, 512)
    assert 2 * q * b + 5 + diag <= per <= 2 * q * b + 5.5 + diag, (q, storage, arith, per)
    assert per < paper_bytes(arith, b, q), (q, storage, arith, per, paper_bytes(arith, b, q))


def test_sixteen_bit_footprint_reduction(lbm):
    fp32, _ = per_cell(lbm, 19, "fp32", "fp32")
    fp16, _ = per_cell(lbm, 19, "fp16s", "fp32")
    paper = 1 - paper_bytes("fp32", 2, 19) / paper_bytes("fp32", 4, 19)
    assert abs(paper - 0.45) < 0.01
    assert 0.47 < 1 - fp16 / fp32 < 0.49, (fp32, fp16)


def test_device_bytes_stay_exact_through_relaunches(lbm):
    """The handle's device-memory figure follows its allocations: switching
    between launch kinds (each builds a tile table and frees the old one) and
    autotuning (tens of tables) leave it where the same configuration had it
    before, so nothing is counted twice or leaked."""
    p = lbm.make_params(96, 64, 48, q=19, storage="fp16s")
    with lbm.Lattices(p) as g:
        g.set_launch(mode=0, block=512)
        base = g.info()["device_bytes"]
        g.set_launch(mode=2, block=256)
        dense = g.info()["device_bytes"]
        assert dense != base             # a table of 256-cell runs replaced one of 512-cell row tiles
        for _ in range(5):
            g.set_launch(mode=0, block=512)
            assert g.info()["device_bytes"] == base
            g.set_launch(mode=2, block=256)
            assert g.info()["device_bytes"] == dense
        g.autotune(2)
        g.set_launch(mode=2, block=256, cells_per_lane=1, persistent=0)
        assert g.info()["device_bytes"] == dense
        g.set_launch(mode=0, block=512)
        assert g.info()["device_bytes"] == base
