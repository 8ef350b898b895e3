"""The benchmark's command line without a GPU: asking for more than one GPU
ends at once with a message and a nonzero status (the solve is not sharded
across GPUs), before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_roofline_traffic_from_committed_profile():
    """roofline.traffic comes from the committed counter summary of the
    finest-level RM kernel, scaled by the copy kernel's counters, and only
    while that summary's source hash matches the kernel source; the scaled
    bytes then lie within a few percent of the algorithmic bytes the summary
    states ((k + 6) N 8 averaged over the solve's launches: 7.791 GB)."""
    b = _bench_module()
    alg = 7.791e9
    tr = b.profile_traffic(alg)
    text = open(b.PROFILE_RM).read()
    if b.rm_kernel_sha() not in text:
        assert tr is None
        return
    assert tr is not None
    assert 0.95 <= tr["ratio_to_algorithmic"] <= 1.1, tr
    assert abs(tr["bytes"] / alg - tr["ratio_to_algorithmic"]) < 1e-3
    # a summary taken on another source is not used
    orig = b.rm_kernel_sha
    b.rm_kernel_sha = lambda: "0" * 64
    try:
        assert b.profile_traffic(alg) is None
    finally:
        b.rm_kernel_sha = orig
