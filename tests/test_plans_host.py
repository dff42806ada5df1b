"""Host-side logic of tile plans, the autotuner's plan cache and the batch
entry point: all of it runs before any device work, so it is tested here
without a GPU."""
import ctypes

import pytest

import paper_2212_00476_amd as zdt
from paper_2212_00476_amd import _lib

SHAPES = [(1280, 384, 128), (640, 192, 64), (1920, 1080, 256), (320, 96, 32), (90, 200, 8), (1000, 500, 64),
          (37, 23, 11), (7, 5, 9), (1280, 1152, 16)]


def _valid(W, H, plan):
    lanes, hseg, vlanes, vseg = plan
    if lanes == 32:
        h_ok = hseg in (8, 20, 40, 60) and W % hseg == 0 and (W // hseg) % 2 == 0 and W // hseg <= 32
    else:
        h_ok = lanes == 64 and hseg in (16, 40, 80) and -(-W // hseg) <= 16
    if vlanes == 32:
        v_ok = vseg in (12, 24, 36) and H % vseg == 0 and (H // vseg) % 2 == 0 and H // vseg <= 32
    else:
        v_ok = vlanes == 64 and vseg in (8, 12, 24, 48, 72) and -(-H // vseg) <= 16
    return h_ok and v_ok


@pytest.mark.parametrize("shape", SHAPES, ids=["%dx%d_d%d" % s for s in SHAPES])
def test_plan_candidates_are_valid_and_distinct(shape):
    W, H, D = shape
    p = zdt.params(W, H, D)
    c = zdt.plan_candidates(p)
    assert c and len(set(c)) == len(c)
    assert c[0] == zdt.get_plan(p)                   # the default comes first
    assert all(_valid(W, H, pl) for pl in c), c
    # the default prefers two 32-lane segments per wave when the row allows it
    if any(pl[0] == 32 for pl in c):
        assert c[0][0] == 32


def test_known_candidates():
    p = zdt.params(1280, 384, 128)
    assert zdt.plan_candidates(p)[0] == (32, 40, 64, 48)   # 8 waves of 48 rows
    v = {(32, 12), (32, 24), (64, 24), (64, 48), (64, 72)}   # 384 = 32 x 12 = 16 x 24
    assert set(zdt.plan_candidates(p)) == {h + vv for h in ((32, 40), (64, 80)) for vv in v}
    # 1080 rows: no 8-wave split; the floating-point volumes default to 30 half-waves of 36 rows with 15
    # waves of 72 as the other candidate, the integer volumes the other way round
    for dt in (zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16):
        assert zdt.plan_candidates(zdt.params(1920, 1080, 256, vol_dtype=dt)) == [(32, 60, 32, 36), (32, 60, 64, 72)]
    for dt in (zdt.ZDT_I16, zdt.ZDT_I8):
        p = zdt.params(1920, 1080, 256, sigma_s=5.0, dt_iters=1, vol_dtype=dt)
        assert zdt.plan_candidates(p) == [(32, 60, 64, 72), (32, 60, 32, 36)]


def test_set_plan_round_trip_and_rejects_misfits():
    p = zdt.params(640, 192, 64, vol_dtype=zdt.ZDT_F16)
    default = zdt.get_plan(p)
    other = zdt.plan_candidates(p)[-1]
    try:
        zdt.set_plan(p, other)
        assert zdt.get_plan(p) == other
        # the plan is per shape and volume type: another dtype keeps its default
        assert zdt.get_plan(zdt.params(640, 192, 64)) == default
        for bad in ((32, 60, 64, 12), (64, 16, 64, 12), (32, 20, 64, 8), (48, 20, 64, 12), (32, 20, 64, 13),
                    (32, 20, 32, 36), (32, 20, 16, 12)):
            with pytest.raises(zdt.ZdtError) as e:
                zdt.set_plan(p, bad)
            assert e.value.code == _lib.ZDT_EINVAL
        assert zdt.get_plan(p) == other
    finally:
        zdt.set_plan(p, None)
    assert zdt.get_plan(p) == default


def test_autotune_takes_a_cached_plan_without_timing(tmp_path):
    p = zdt.params(640, 192, 64, vol_dtype=zdt.ZDT_F16)
    want = (64, 40, 32, 24)
    cache = tmp_path / "plans.txt"
    cache.write_text("zdt-plan 640 192 64 4 1 : 32 20 64 12  (1.0 us)\n"
                     "zdt-plan 640 192 64 4 0 : 32 40 64 48  (1.0 us)\n"   # other dtype
                     "zdt-plan 640 192 64 4 1 : 64 40 32 24  (0.9 us)\n"   # the last match wins
                     "zdt-plan 640 192 64 4 1 : 32 60 64 12  (0.1 us)\n")  # does not fit: ignored
    try:
        got = zdt.autotune(p, str(cache), stream=0)
        assert got == want and zdt.get_plan(p) == want
    finally:
        zdt.set_plan(p, None)


def _job(p, ptr=0x1000):
    return _lib.ZdtJob(p, ptr, ptr, ptr, ptr, ptr)


def test_batch_validation_before_any_device_work():
    lib = zdt.load()
    good = zdt.params(64, 32, 16)
    assert lib.stereo_solve_batch(None, 0, None) == _lib.ZDT_OK
    assert lib.stereo_solve_batch(None, 3, None) == _lib.ZDT_EINVAL
    assert lib.stereo_solve_batch((_lib.ZdtJob * 1)(_job(good)), -1, None) == _lib.ZDT_EINVAL
    # job 1 has a NULL volume: rejected, naming the job, nothing launched
    jobs = (_lib.ZdtJob * 2)(_job(good), _job(good))
    jobs[1].vol = None
    assert lib.stereo_solve_batch(jobs, 2, None) == _lib.ZDT_EINVAL
    assert "job 1" in lib.zdt_last_error().decode()
    # bad parameters and unsupported shapes keep their codes
    jobs = (_lib.ZdtJob * 2)(_job(good), _job(zdt.params(64, 32, 0)))
    assert lib.stereo_solve_batch(jobs, 2, None) == _lib.ZDT_EINVAL
    jobs = (_lib.ZdtJob * 2)(_job(good), _job(zdt.params(64, 32, 16, radius=9)))
    assert lib.stereo_solve_batch(jobs, 2, None) == _lib.ZDT_EUNSUPPORTED
    # a job that needs a workspace must bring one
    f16 = zdt.params(64, 32, 16, vol_dtype=zdt.ZDT_F16)
    assert zdt.workspace_size(f16) > 0
    jobs = (_lib.ZdtJob * 1)(_job(f16))
    jobs[0].ws = None
    assert lib.stereo_solve_batch(jobs, 1, None) == _lib.ZDT_EINVAL


def test_job_struct_layout_matches_header():
    # zdt_job: zdt_params (56 B) then five pointers
    assert ctypes.sizeof(_lib.ZdtParams) == 56
    assert _lib.ZdtJob.left.offset == 56 and ctypes.sizeof(_lib.ZdtJob) == 56 + 5 * 8
    assert ctypes.sizeof(_lib.ZdtPlan) == 16
