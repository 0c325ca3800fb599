"""The library's 16-bit codecs compiled for the host (the same header the
kernels include) against the oracle, without a GPU: the decoders on all
65,536 codes of FP16C and the three posit formats, and the encoders (FP16C's
arithmetic one, the posits' sign-and-exponent table) on every code value,
its float neighbours, the midpoints between neighbouring codes and their
float neighbours, specials and a million random floats.  The driver also
checks the shortcuts against the general codec on their whole range (the
posits' zeros-run decoders on every such code, P16_0S's fixed-range encoder
on every float below 2^-7 in magnitude).  The GPU tests repeat the encoder
comparison on all 2^32 floats."""
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIB_FMT = {"fp16c": 4, "p16_0s": 5, "p16_1s": 6, "p16_2c": 7}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    exe = tmp_path_factory.mktemp("codec") / "codec_host"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2112_08926_amd", "csrc"),
                    os.path.join(ROOT, "tests", "codec_host.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def _inputs(fmt):
    codes = np.arange(0x8000, dtype=np.uint16)
    v = oracle.decode(fmt, codes).astype(np.float32)
    v = np.unique(v[np.isfinite(v)])
    mids = ((v[1:].astype(np.float64) + v[:-1]) / 2).astype(np.float32)
    pts = np.concatenate([v, mids])
    pts = np.concatenate([pts, np.nextafter(pts, np.float32(np.inf)), np.nextafter(pts, np.float32(0))])
    rng = np.random.default_rng(5)
    rnd = rng.integers(0, 2 ** 32, size=1 << 20, dtype=np.uint64).astype(np.uint32).view(np.float32)
    special = np.array([0.0, np.inf, np.nan, 1e-45, 1e-40, 3.4e38, 1e-20, 1e20], dtype=np.float32)
    x = np.concatenate([pts, special, rnd]).astype(np.float32)
    return np.concatenate([x, -x])


@pytest.mark.parametrize("fmt", ["fp16c", "p16_0s", "p16_1s", "p16_2c"])
def test_host_codecs_match_oracle(driver, tmp_path, fmt):
    x = _inputs(fmt)
    x.tofile(tmp_path / "in.bin")
    subprocess.run([str(driver), str(LIB_FMT[fmt]), str(tmp_path / "dec.bin"), str(tmp_path / "in.bin"),
                    str(tmp_path / "out.bin")], check=True)
    dec = np.fromfile(tmp_path / "dec.bin", dtype=np.float32)
    ref = oracle.decode(fmt, np.arange(65536, dtype=np.uint16))
    assert np.array_equal(dec.view(np.uint32), ref.astype(np.float32).view(np.uint32))   # bitwise, -0 too
    got = np.fromfile(tmp_path / "out.bin", dtype=np.uint16)
    want = oracle.encode(fmt, x)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(float(x[i]), int(got[i]), int(want[i])) for i in bad[:8]]
