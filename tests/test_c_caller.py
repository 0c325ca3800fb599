"""The library called from a plain C99 program (tests/c_caller.c) rather
than through the Python binding: the header compiles warning-free as C99 and
the program links against liblbm.so (CPU); on the GPU it steps a 48^3 cavity
and its device FP64 diagnostics agree with sums over the moments it copied
out, mass is conserved and the lid has set the fluid moving."""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2112_08926_amd")


def build_caller(tmp_path) -> str:
    exe = str(tmp_path / "c_caller")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-O1",
                    "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "c_caller.c"),
                    "-L", PKG, "-llbm", f"-Wl,-rpath,{PKG}", "-lm", "-o", exe], check=True)
    return exe


def test_c_caller_builds(tmp_path):
    if not os.path.exists(os.path.join(PKG, "liblbm.so")):
        pytest.skip("liblbm.so not built")
    assert os.access(build_caller(tmp_path), os.X_OK)


@pytest.mark.gpu
def test_c_caller_runs(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = build_caller(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.returncode, r.stderr)
    v = {k: float(x) for k, x in re.findall(r"(\w+)=([-+0-9.e]+)", r.stdout)}
    assert v["steps"] == 300 and v["nonfinite"] == 0 and v["fluid"] == 46 ** 3
    assert abs(v["mass"] - v["host_mass"]) <= 1e-9 * v["fluid"]
    assert abs(v["momentum_y"] - v["host_momentum_y"]) <= 1e-9 * v["fluid"]
    assert abs(v["mass"] / v["fluid"] - 1) < 1e-4
    assert 1e-3 < v["u_max"] < 0.05
    assert v["fused_same"] == 1 and v["steps_after"] == 301      # lbm_step_diagnostics: same sums, one more step
