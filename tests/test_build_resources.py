"""The built kernels keep their working set in registers and LDS: the
compiler's per-kernel resource report (written by the build) shows no kernel
that needs more than a few words of scratch per lane.  A kernel that needs tens
of KB per lane cannot be dispatched at all."""
import json
import os

import pytest

from paper_2212_00476_amd import build

pytestmark = pytest.mark.skipif(not os.path.exists(build.RESOURCES), reason="library not built")


def _resources():
    with open(build.RESOURCES) as f:
        return json.load(f)


def test_every_kernel_reported():
    res = _resources()
    names = " ".join(res)
    for k in ("hpass_kernel", "vpass_kernel", "wta_kernel", "wta_combine_kernel"):
        assert k in names, k


def test_scratch_per_lane_bounded():
    res = _resources()
    worst = max(res.items(), key=lambda kv: kv[1].get("scratch_bytes", 0))
    assert worst[1].get("scratch_bytes", 0) <= build.MAX_SCRATCH_BYTES, worst


def test_report_parser():
    text = ("x.hpp:1:1: remark: Function Name: _Zfoo [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hpp:1:1: remark:     VGPRs: 74 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hpp:1:1: remark:     ScratchSize [bytes/lane]: 40 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hpp:1:1: remark:     Occupancy [waves/SIMD]: 6 [-Rpass-analysis=kernel-resource-usage]\n")
    assert build.parse_resources(text) == {"_Zfoo": {"vgprs": 74, "scratch_bytes": 40, "waves_per_simd": 6}}
