"""Host-side logic of bench.py (no GPU): the one-GPU refusal, and the
reading of the committed rocprofv3 counter summary that fills the bench
line's roofline.traffic -- the traffic is reported only when the summary
was taken on the current kernel source and names the timed kernel, and it
is then the summary's HBM bytes per launch."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _summary():
    vals = {}
    for line in open(os.path.join(ROOT, "profiles", "schur_f16_32x32x32x64.txt")):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    return vals


def test_traffic_read_from_the_matching_summary():
    vals = _summary()
    tag = vals["kernel"] + " (64 threads)"
    got = bench._traffic_from_profile(tag)
    if vals["kernel_source_hash"] == bench._kernel_source_hash():
        assert got == float(vals["hbm_bytes_per_launch"])
        # and the counters are consistent with the summary's own ratio
        alg = float(vals["algorithmic_bytes_per_launch"])
        assert abs(got / alg - float(vals["ratio_to_algorithmic"])) < 1e-3
    else:
        assert got is None
    # another kernel's tag never takes these counters
    assert bench._traffic_from_profile("FP32 Schur operator (64 threads)") is None


def test_summary_states_its_commands():
    text = open(os.path.join(ROOT, "profiles", "schur_f16_32x32x32x64.txt")).read()
    assert "rocprofv3 --kernel-trace --stats" in text and "--pmc <COUNTERS>" in text
    assert "bench.py --profile schur_f16" in text
