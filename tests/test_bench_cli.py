"""Host behaviour of the benchmark (no GPU needed): more than one GPU is
refused with a message before anything touches a device, and the committed
counter readings are used only for the kernel code they were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_source_hash_is_stable_hex():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert h == bench.kernel_source_hash()


def test_committed_traffic_matches_the_current_kernels(monkeypatch):
    """The committed counter summary is used while it names the current
    kernel sources, and dropped (traffic null) once they differ."""
    sys.path.insert(0, ROOT)
    import json
    import bench
    with open(os.path.join(ROOT, "profiles", "ldc512_fp16s_traffic.json")) as fh:
        rec = json.load(fh)
    t = bench.traffic_from_profile("fp16s")
    if rec["kernel_source_hash"] == bench.kernel_source_hash():
        assert t is not None and 10.0e9 < t < 12.0e9    # 512^3 FP16S: 10.33 GB algorithmic per step
    else:
        assert t is None                                # taken on other kernel sources: not used
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.traffic_from_profile("fp16s") is None
    assert bench.traffic_from_profile("fp32") is None   # no summary for that format


def test_hash_ignores_comments_but_not_code():
    """The kernel hash reads the code without its comments: a comment-only
    edit keeps the stored counter readings, any change of code (string and
    character literals included) drops them."""
    sys.path.insert(0, ROOT)
    import bench
    src = 'int a = 1; // one\n/* two\n   lines */ const char* s = "//x /*y*/"; char c = \'/\';\n\nint b;\n'
    assert bench.code_only(src) == 'int a = 1;\n const char* s = "//x /*y*/"; char c = \'/\';\nint b;'
    assert bench.code_only(src.replace("// one", "// changed")) == bench.code_only(src)
    assert bench.code_only(src.replace("a = 1", "a = 2")) != bench.code_only(src)
    assert bench.code_only(src.replace('"//x /*y*/"', '"//x /*z*/"')) != bench.code_only(src)
