"""GPU storage codecs against the FP64 reference, exhaustively: every one of
the 2^32 FP32 inputs is encoded on the GPU; encoding is monotone in the bit
pattern of |x|, so the GPU result is fully described by the bit patterns at
which the code changes, which are compared with the reference's (found by
bisection with the reference encoder).  Negative inputs must give the code of
|x| with the sign bit; NaN inputs give NaN (FP16, FP16S) or the largest
magnitude (FP16C, posits)."""
import numpy as np
import pytest

from lbm_testlib import say

pytestmark = pytest.mark.gpu

FMTS = ["fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c"]
INF_BITS = 0x7F800000
CHUNK = 1 << 28


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_08926_amd as lbm
    return lbm


def reference_thresholds(orc, fmt):
    """First non-negative FP32 bit pattern of each positive magnitude code."""
    top = int(orc.encode(fmt, np.array([np.inf], np.float32))[0])
    codes = np.arange(1, top + 1, dtype=np.int64)
    lo = np.zeros(codes.size, np.int64)               # encode(lo) < c
    hi = np.full(codes.size, INF_BITS, np.int64)      # encode(hi) >= c
    while np.any(hi - lo > 1):
        mid = (lo + hi) // 2
        enc = orc.encode(fmt, mid.astype(np.uint32).view(np.float32)).astype(np.int64)
        ge = enc >= codes
        hi = np.where(ge, mid, hi)
        lo = np.where(ge, lo, mid)
    return hi, codes


def gpu_transitions(lbm, fmt):
    """(bit pattern, code) wherever the GPU code changes over [0, +Inf], and
    a check of the negative half and of the NaN range on the way."""
    import torch
    pos_b, pos_c = [], []
    prev_last = None
    out = torch.empty(CHUNK, dtype=torch.int16, device="cuda")
    outn = torch.empty(CHUNK, dtype=torch.int16, device="cuda")
    for s in range(0, INF_BITS + 1, CHUNK):
        e = min(s + CHUNK, INF_BITS + 1)
        bits = torch.arange(s, e, dtype=torch.int64, device="cuda").to(torch.int32)
        n = e - s
        lbm.lbm_encode(fmt, bits.data_ptr(), out.data_ptr(), n)
        nbits = bits | torch.tensor(-(1 << 31), dtype=torch.int32, device="cuda")
        lbm.lbm_encode(fmt, nbits.data_ptr(), outn.data_ptr(), n)
        c = out[:n].to(torch.int32) & 0xFFFF
        cn = outn[:n].to(torch.int32) & 0xFFFF
        assert torch.equal(cn, c | 0x8000), (fmt, "sign", s)
        first = int(c[0])
        if prev_last is None:
            assert first == 0, (fmt, "encode(+0)")
        elif first != prev_last:
            pos_b.append(s)
            pos_c.append(first)
        change = torch.nonzero(c[1:] != c[:-1]).flatten() + 1
        assert bool(torch.all(c[1:] >= c[:-1])), (fmt, "monotone", s)
        pos_b.extend((change + s).tolist())
        pos_c.extend(c[change].tolist())
        prev_last = int(c[-1])
    # NaN inputs
    for s in range(INF_BITS + 1, 1 << 31, CHUNK):
        e = min(s + CHUNK, 1 << 31)
        bits = torch.arange(s, e, dtype=torch.int64, device="cuda").to(torch.int32)
        n = e - s
        lbm.lbm_encode(fmt, bits.data_ptr(), out.data_ptr(), n)
        c = out[:n].to(torch.int32) & 0xFFFF
        if fmt in ("fp16", "fp16s"):
            assert bool(torch.all(((c & 0x7C00) == 0x7C00) & ((c & 0x3FF) != 0))), (fmt, "NaN")
        else:
            assert bool(torch.all(c == 0x7FFF)), (fmt, "NaN")
    torch.cuda.synchronize()
    return np.array(pos_b, np.int64), np.array(pos_c, np.int64)


@pytest.mark.parametrize("fmt", FMTS)
def test_encode_all_fp32_inputs(lbm, orc, fmt):
    say("exhaustive encode", fmt)
    thr, codes = reference_thresholds(orc, fmt)
    # expected transitions: at each distinct threshold, the largest code reached
    ub, idx = np.unique(thr, return_index=True)
    last = np.searchsorted(thr, ub, side="right") - 1
    exp_b, exp_c = ub, codes[last]
    got_b, got_c = gpu_transitions(lbm, fmt)
    assert got_b.size == exp_b.size, (fmt, got_b.size, exp_b.size)
    assert np.array_equal(got_b, exp_b) and np.array_equal(got_c, exp_c), fmt
