"""The C interface (include/lbm.h) without a GPU: the library loads, exports
every function the header declares, its structures have the layout the
Python binding assumes, and argument checks that need no device fail with
the documented status."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    import paper_2112_08926_amd as lbm
    L = lbm.library()
    names = _declared_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding wraps each under the same name
    assert all(hasattr(lbm, n) for n in names)


def test_struct_layout_matches_header(tmp_path):
    import paper_2112_08926_amd as lbm
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(lbm_params),"
                   " sizeof(lbm_diag), sizeof(lbm_launch), sizeof(lbm_info), offsetof(lbm_params, tau),"
                   " offsetof(lbm_params, eq_u), offsetof(lbm_diag, nonfinite_cells), offsetof(lbm_diag, nonfinite_updates));return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    expect = [ctypes.sizeof(lbm.LbmParams), ctypes.sizeof(lbm.LbmDiag), ctypes.sizeof(lbm.LbmLaunch),
              ctypes.sizeof(lbm.LbmInfo), lbm.LbmParams.tau.offset, lbm.LbmParams.eq_u.offset,
              lbm.LbmDiag.nonfinite_cells.offset, lbm.LbmDiag.nonfinite_updates.offset]
    assert got == expect


@pytest.mark.parametrize("field,value", [("tau", 0.5), ("tau", 0.3), ("nx", 0), ("q", 13), ("q", 7), ("q", 9),
                                         ("storage", 9), ("unshifted", 2), ("nz", 70000)])
def test_create_rejects_invalid_params_without_device(field, value):
    import paper_2112_08926_amd as lbm
    p = lbm.make_params(8, 8, 8)
    setattr(p, field, value)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(p)
    assert ei.value.code == -1


def test_create_rejects_unsupported_combinations_without_device():
    import paper_2112_08926_amd as lbm
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(lbm.make_params(8, 8, 8, storage="fp16", arith="fp64"))
    assert ei.value.code == -4
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create([lbm.make_params(8, 8, 8), lbm.make_params(8, 8, 8, q=27)])
    assert ei.value.code == -4
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(lbm.make_params(8, 8, 8, q=27, collision="mrt"))
    assert ei.value.code == -4


def test_codec_entry_points_reject_bad_arguments_without_device():
    import paper_2112_08926_amd as lbm
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_encode("fp32", 16, 16, 4)
    assert ei.value.code == -1
    with pytest.raises(lbm.LbmError):
        lbm.lbm_decode("fp16c", 16, 16, -1)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_copy_probe(16, 32, 17)
    for kind, src, dst, n in [(7, 16, 32, 64), (-1, 16, 32, 64), ("read", 16, 32, 18), ("read", 18, 32, 64),
                              ("write", 16, 34, 64), ("write_misaligned", 0, 0, 64), ("read", 0, 32, 64),
                              ("read_misaligned", 16, 32, 4)]:
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_memory_probe(kind, src, dst, n)
        assert ei.value.code == -1, (kind, src, dst, n)
    # n == 0 is a no-op and touches no device
    lbm.lbm_encode("fp16c", 0, 0, 0)
    assert np.dtype(np.uint16).itemsize == 2


@pytest.mark.parametrize("dims,storage", [((1024, 1024, 1024), "fp32"),      # N * 4 = 2^32
                                          ((2048, 1024, 1024), "fp16s"),     # N = 2^31
                                          ((1024, 1024, 512), "fp64")])      # N * 8 = 2^32
def test_create_rejects_lattices_past_the_offset_limits_without_device(dims, storage):
    """One past the largest lattices the 32-bit in-plane offsets allow (the
    largest ones themselves are stepped by the GPU tests)."""
    import paper_2112_08926_amd as lbm
    arith = "fp64" if storage == "fp64" else "fp32"
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(lbm.make_params(*dims, storage=storage, arith=arith))
    assert ei.value.code == -1 and "32-bit" in str(ei.value)


def test_create_rejects_an_empty_ensemble_without_device():
    import paper_2112_08926_amd as lbm
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create([])
    assert ei.value.code == -1
