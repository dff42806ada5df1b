"""Host logic of the benchmark (no GPU): the one-GPU contract, the byte models
behind the roofline figures, and the committed rocprofv3 summaries they are
checked against."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("s", [4, 2, 1])
@pytest.mark.parametrize("iters", [1, 3])
@pytest.mark.parametrize("shape", [(1280, 384, 128), (1920, 1080, 256), (37, 23, 11)])
def test_solve_byte_model_is_the_sum_of_its_launches(shape, iters, s):
    """B_ref counts the volume crossing memory 4 I - 2 times plus the images and
    the disparities; the launches of one solve (cost + L/R, then U/D and L/R
    pairs, the last U/D pair with the WTA) add one guide read per pass pair."""
    w, h, d = shape
    ab = lambda k: bench.algorithmic_bytes(k, s, w, h, d)  # noqa: E731
    launches = ab("zncc_hpair") + (iters - 1) * (ab("dt_vpair") + ab("dt_hpair")) + ab("dt_vpair_wta")
    assert launches == bench.b_ref(s, iters, w, h, d) + (2 * iters - 1) * w * h


def test_config_1_byte_model():
    # 1280 x 384 x 128 FP32, three sweeps: 2.5195 GB; 16-bit: 1.2612 GB
    assert bench.b_ref(4, 3) == 1280 * 384 * 128 * 4 * 10 + 6 * 1280 * 384 == 2519531520
    assert bench.b_ref(2, 3) == 1261240320


def _summaries():
    return sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))


def test_counter_summaries_are_complete_and_at_least_compulsory():
    """Every committed traffic summary names its kernel, workload and source
    hash, its bytes are FETCH + WRITE, and no kernel moves less than its
    compulsory bytes (the counters see every L2 miss and write-back)."""
    files = _summaries()
    assert files
    for f in files:
        rec = json.load(open(f))
        for key in ("kernel", "launch", "vol_dtype", "workload", "bytes_per_launch", "fetch_bytes", "write_bytes",
                    "algorithmic_bytes", "avg_us_rocprof", "kernel_source_hash", "source"):
            assert key in rec, (f, key)
        # each is an average over the counted launches, rounded to a byte
        assert abs(rec["bytes_per_launch"] - rec["fetch_bytes"] - rec["write_bytes"]) <= 2
        assert rec["bytes_per_launch"] >= 0.98 * rec["algorithmic_bytes"], f
        assert os.path.exists(os.path.join(ROOT, rec["source"])), f


def test_profile_summaries_give_their_commands():
    for f in glob.glob(os.path.join(ROOT, "profiles", "kernels_*.md")):
        text = open(f).read()
        assert "rocprofv3 --kernel-trace --stats" in text
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
        assert "python3 -m paper_2212_00476_amd.timing" in text
