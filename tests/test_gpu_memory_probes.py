"""The memory microbenchmarks (the paper's appendix memory benchmarks,
Fig. 13): the write kernels store exactly the documented elements, the
misaligned ones shifted by one 4-byte element, the read kernels leave their
sink alone on a zero source, and every kind sustains a plausible share of
HBM bandwidth on a 1 GiB buffer."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return torch, lbm


@pytest.mark.parametrize("nbytes", [8, 4 * 1000 + 4, 4 * 256 * 3001])
@pytest.mark.parametrize("kind,shift", [("write", 0), ("write_misaligned", 1)])
def test_write_kernels_store_the_documented_elements(torch_lbm, nbytes, kind, shift):
    torch, lbm = torch_lbm
    n = nbytes // 4
    dst = torch.full((n + 64,), 0xA5A5A5A5 - (1 << 32), dtype=torch.int32, device="cuda")
    lbm.lbm_memory_probe(kind, None, dst.data_ptr(), nbytes)
    torch.cuda.synchronize()
    got = dst.cpu().numpy().view(np.uint32)
    expect = np.full(n + 64, 0xA5A5A5A5, dtype=np.uint32)
    expect[shift:n] = np.arange(n - shift, dtype=np.uint32)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("kind", ["read", "read_misaligned"])
def test_read_kernels_leave_the_sink_alone(torch_lbm, kind):
    torch, lbm = torch_lbm
    n = 256 * 5000 + 17
    src = torch.zeros(n, dtype=torch.int32, device="cuda")
    dst = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    lbm.lbm_memory_probe(kind, src.data_ptr(), dst.data_ptr(), 4 * n)
    torch.cuda.synchronize()
    assert bool((dst == 7).all())


def test_copy_kind_is_the_copy_probe(torch_lbm):
    torch, lbm = torch_lbm
    src = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    lbm.lbm_memory_probe("copy", src.data_ptr(), dst.data_ptr(), src.numel())
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_bandwidths_are_plausible(torch_lbm):
    """Every kind moves 1 GiB at more than 2 TB/s and at most the 8 TB/s
    peak (loose bounds: a sanity check of the timing, not a performance bar)."""
    torch, lbm = torch_lbm
    nbytes = 1 << 30
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for kind in ("copy", "read", "read_misaligned", "write", "write_misaligned"):
        lbm.lbm_memory_probe(kind, a.data_ptr(), b.data_ptr(), nbytes)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            lbm.lbm_memory_probe(kind, a.data_ptr(), b.data_ptr(), nbytes)
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / 5 * 1e-3
        moved = (2 if kind == "copy" else 1) * nbytes
        gbs = moved / s / 1e9
        print(f"{kind}: {gbs:.0f} GB/s", flush=True)
        assert 2000 < gbs < 8000, (kind, gbs)
