"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Bars (derivations in the design notes):
  - integer sums and WTA indices: bit-exact;
  - raw FP32 cost: |d cost| <= 1e-5; FP16 / BF16 storage: half an ulp of [1, 2) + 1e-6;
  - DT volume (FP32 state): |d C| <= DT_REL * max_d |C_oracle(x, y, :)| per pixel;
  - end-to-end FP32 disparity: every mismatch is a near-tie of the oracle's own
    aggregated costs, C(d_gpu) - min_d C <= DT_REL * max_d C;
  - end-to-end FP16 / BF16: every mismatch is a near-tie within the storage
    type's rounding, propagated (_narrow_tol); at full size at most 0.1 % of
    FP16 disparities differ;
  - integer volumes (Sec. IV-C): against the oracle's statement of the
    paper's per-pass FastDT (Sec. V-C), the stored state and the disparities.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2212_00476_amd import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2212_00476_amd as zdt  # noqa: E402

# FP32 DT state: every state is non-negative (costs in [0, 2], weights > 0),
# so the rounding of each of the 12 passes (2^-24 of the value it writes)
# reaches the final value as at most 2^-24 of that final value: 12 * 6e-8 =
# 7.2e-7.  The float weights and the composed segment carries add errors of
# the same kind along each line; 1e-5 (the parity contract for the
# aggregated volume) leaves a factor ~10 over the largest error measured
# (9.1e-7).
DT_REL = 1e-5
HALF_ULP = {zdt.ZDT_F16: 2.0 ** -11, zdt.ZDT_BF16: 2.0 ** -8}
ORACLE_THREADS = min(16, os.cpu_count() or 1)


def note(msg):
    print(msg, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.float().cpu().numpy() if t.dtype in (torch.float16, torch.bfloat16) else t.cpu().numpy()


def pair_for(W, H, D, seed=0):
    ds = tuple(sorted({max(0, min(D - 1, k)) for k in (1, D // 3, (2 * D) // 3)}))
    return scenes.bands_pair(W=W, H=H, D=D, seed=seed, band_disps=ds)


# (W, H, D, r): config-0 shape, ragged sizes, D not a multiple of 64, D = 1,
# D > W, image smaller than the window, r = 0, r = 6, the widest row.
SHAPES = [(320, 96, 32, 4), (37, 23, 11, 2), (100, 17, 65, 3), (50, 40, 1, 1), (30, 12, 45, 4), (7, 5, 9, 4),
          (129, 33, 130, 0), (640, 24, 20, 6), (1280, 9, 16, 5), (333, 70, 64, 1), (100, 40, 20, 7)]


def ids(shapes):
    return ["%dx%d_d%d_r%d" % s for s in shapes]


@pytest.mark.parametrize("shape", SHAPES, ids=ids(SHAPES))
def test_window_sums_bit_exact(shape):
    W, H, D, r = shape
    note(f"window sums {shape}")
    pr = pair_for(W, H, D)
    p = zdt.params(W, H, D, r)
    i32 = dict(dtype=torch.int32, device="cuda")
    s_l, s_ll = torch.full((H, W), -7, **i32), torch.full((H, W), -7, **i32)
    s_t, s_tt = torch.full((H, W + D - 1), -7, **i32), torch.full((H, W + D - 1), -7, **i32)
    s_rt = torch.full((H, W, D), -7, **i32)
    zdt.zncc_window_sums(p, dev(pr.left), dev(pr.right), s_l, s_ll, s_t, s_tt, s_rt)
    torch.cuda.synchronize()
    o_l, o_ll, o_t, o_tt = oracle.window_sums(pr.left, pr.right, D, r)
    assert np.array_equal(host(s_l), o_l)
    assert np.array_equal(host(s_ll), o_ll)
    assert np.array_equal(host(s_t), o_t)
    assert np.array_equal(host(s_tt), o_tt)
    assert np.array_equal(host(s_rt), oracle.cross_sums(pr.left, pr.right, D, r))


def test_window_sums_with_pitch():
    W, H, D, r, pitch = 90, 20, 24, 3, 128
    note("window sums with pitch")
    pr = pair_for(W, H, D, seed=5)
    rng = np.random.default_rng(0)
    Lp = rng.integers(0, 256, (H, pitch)).astype(np.uint8)
    Rp = rng.integers(0, 256, (H, pitch)).astype(np.uint8)
    Lp[:, :W], Rp[:, :W] = pr.left, pr.right
    p = zdt.params(W, H, D, r, pitch=pitch)
    s_rt = torch.empty((H, W, D), dtype=torch.int32, device="cuda")
    zdt.zncc_window_sums(p, dev(Lp), dev(Rp), s_rt=s_rt)
    cost = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, dev(Lp), dev(Rp), cost)
    torch.cuda.synchronize()
    assert np.array_equal(host(s_rt), oracle.cross_sums(pr.left, pr.right, D, r))
    assert np.abs(host(cost) - oracle.zncc_cost(pr.left, pr.right, D, r)).max() <= 1e-5


@pytest.mark.parametrize("shape", SHAPES, ids=ids(SHAPES))
def test_cost_fp32(shape):
    W, H, D, r = shape
    note(f"cost fp32 {shape}")
    pr = pair_for(W, H, D, seed=1)
    p = zdt.params(W, H, D, r)
    cost = torch.full((H, W, D), math.nan, dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, dev(pr.left), dev(pr.right), cost)
    torch.cuda.synchronize()
    err = np.abs(host(cost).astype(np.float64) - oracle.zncc_cost(pr.left, pr.right, D, r))
    note(f"  max |d cost| = {err.max():.3e}")
    assert err.max() <= 1e-5


def test_cost_special_cases():
    """Flat images (zero variance) give cost 1; an exact shifted copy gives 0 at its shift."""
    W, H, D, r = 64, 16, 8, 2
    note("cost special cases")
    flat = np.full((H, W), 90, np.uint8)
    rng = np.random.default_rng(3)
    tex = rng.integers(0, 256, (H, W + 8)).astype(np.uint8)
    left, right = tex[:, :W], tex[:, 5:5 + W]          # right(x') = left(x'+5): d = 5
    p = zdt.params(W, H, D, r)
    cost = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, dev(flat), dev(left), cost)
    torch.cuda.synchronize()
    assert np.all(host(cost) == 1.0)
    zdt.zncc_cost_volume(p, dev(left), dev(right), cost)
    torch.cuda.synchronize()
    c = host(cost)
    assert np.all(c >= 0.0) and np.all(c <= 2.0)
    assert np.abs(c[r:H - r, 5 + r:W - r, 5]).max() <= 1e-6


@pytest.mark.parametrize("dtype", [zdt.ZDT_F16, zdt.ZDT_BF16], ids=["f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES[:4], ids=ids(SHAPES[:4]))
def test_cost_narrow(shape, dtype):
    W, H, D, r = shape
    note(f"cost narrow {shape} dtype={dtype}")
    pr = pair_for(W, H, D, seed=2)
    p = zdt.params(W, H, D, r, vol_dtype=dtype)
    cost = torch.empty((H, W, D), dtype=zdt.torch_dtype(dtype), device="cuda")
    zdt.zncc_cost_volume(p, dev(pr.left), dev(pr.right), cost)
    torch.cuda.synchronize()
    err = np.abs(host(cost).astype(np.float64) - oracle.zncc_cost(pr.left, pr.right, D, r))
    note(f"  max |d cost| = {err.max():.3e}")
    assert err.max() <= HALF_ULP[dtype] + 1e-6


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16], ids=["f32", "f16", "bf16"])
@pytest.mark.parametrize("D", [1, 7, 64, 65, 128, 200])
def test_wta_bit_exact_with_ties(D, dtype):
    W, H = 53, 11
    note(f"wta D={D} dtype={dtype}")
    rng = np.random.default_rng(D)
    vol = rng.integers(0, 5, (H, W, D)).astype(np.float32)      # many exact ties
    vol[:, :, -1] = np.minimum(vol[:, :, -1], 0.0)               # a tie at the last d
    t = dev(vol).to(zdt.torch_dtype(dtype))
    disp = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
    zdt.wta_disparity(zdt.params(W, H, D, vol_dtype=dtype), t, disp)
    torch.cuda.synchronize()
    assert np.array_equal(host(disp), np.argmin(host(t), axis=2))
    vol = rng.standard_normal((H, W, D)).astype(np.float32)
    t = dev(vol).to(zdt.torch_dtype(dtype))
    zdt.wta_disparity(zdt.params(W, H, D, vol_dtype=dtype), t, disp)
    torch.cuda.synchronize()
    assert np.array_equal(host(disp), np.argmin(host(t), axis=2))


def _dt_check(got, want):
    scale = np.abs(want).max(axis=2, keepdims=True)
    rel = (np.abs(got - want) / np.maximum(scale, 1e-300)).max()
    return rel


DT_SHAPES = [(320, 96, 32, 4), (37, 23, 11, 2), (100, 17, 65, 3), (50, 40, 1, 1), (7, 5, 9, 4), (129, 33, 130, 0),
             (1280, 9, 16, 5), (90, 200, 8, 2), (60, 1000, 4, 1)]


@pytest.mark.parametrize("iters", [1, 3])
@pytest.mark.parametrize("shape", DT_SHAPES, ids=ids(DT_SHAPES))
def test_dt_aggregate_fp32(shape, iters):
    W, H, D, r = shape
    note(f"dt_aggregate {shape} iters={iters}")
    pr = pair_for(W, H, D, seed=3)
    c0 = oracle.zncc_cost(pr.left, pr.right, D, r).astype(np.float32)
    wh, wv = oracle.dt_weights(pr.left, 20.0, 0.1)
    want = oracle.dt_aggregate(c0.astype(np.float64), wh, wv, iters)
    p = zdt.params(W, H, D, r, dt_iters=iters)
    vol = dev(c0)
    scale = zdt.dt_aggregate(p, dev(pr.left), vol)
    torch.cuda.synchronize()
    assert scale == 1.0
    rel = _dt_check(host(vol).astype(np.float64), want)
    note(f"  max rel err = {rel:.3e}")
    assert rel <= DT_REL
    # normalised form: the same volume times the reported scale
    p = zdt.params(W, H, D, r, dt_iters=iters, flags=zdt.ZDT_FLAG_NORMALIZE)
    vol = dev(c0)
    scale = zdt.dt_aggregate(p, dev(pr.left), vol)
    torch.cuda.synchronize()
    assert scale == pytest.approx((1.0 - math.exp(-1.0 / 20.0)) ** (4 * iters), rel=1e-12)
    rel = _dt_check(host(vol).astype(np.float64) / scale, want)
    assert rel <= DT_REL


def test_dt_constant_guide_and_range_off():
    """With sigma_r = +inf the weights are the constant K; the GPU result then
    also matches the oracle run on a flat guide."""
    W, H, D = 80, 30, 5
    note("dt range term off")
    rng = np.random.default_rng(9)
    c0 = rng.uniform(0, 2, (H, W, D)).astype(np.float32)
    G = rng.integers(0, 256, (H, W)).astype(np.uint8)
    p = zdt.params(W, H, D, 1, sigma_s=5.0, sigma_r=math.inf, dt_iters=2)
    vol = dev(c0)
    zdt.dt_aggregate(p, dev(G), vol)
    torch.cuda.synchronize()
    wh, wv = oracle.dt_weights(np.zeros((H, W), np.uint8), 5.0, 0.1)
    want = oracle.dt_aggregate(c0.astype(np.float64), wh, wv, 2)
    assert _dt_check(host(vol).astype(np.float64), want) <= DT_REL


def _near_tie_ok(disp_gpu, cagg):
    """Every GPU/oracle disagreement is a near-tie in the oracle's own costs."""
    H, W, D = cagg.shape
    dmin = cagg.min(axis=2)
    dmax = np.abs(cagg).max(axis=2)
    picked = np.take_along_axis(cagg, disp_gpu[:, :, None].astype(np.int64), axis=2)[:, :, 0]
    slack = picked - dmin
    return slack, slack <= DT_REL * dmax


# Per-element relative rounding of a stored 16-bit state: FP16 keeps 11
# significant bits (the working volume is scaled per pixel by a power of two
# so that no state overflows or leaves the normal range), BF16 keeps 8.
NARROW_REL = {zdt.ZDT_F16: 2.0 ** -11, zdt.ZDT_BF16: 2.0 ** -9}


def _narrow_tol(dtype, iters, cagg):
    """Near-tie bar of a 16-bit working volume.  Every state is non-negative,
    so a store's rounding (at most NARROW_REL of the stored value) reaches the
    final value as at most NARROW_REL of that final value; stereo_solve stores
    2 I - 1 states (the last V pair feeds the WTA).  With the FP32 arithmetic
    (DT_REL), each aggregated cost is within eps = (2I-1) NARROW_REL + DT_REL
    of itself, and a disparity picked on the device satisfies
    C(d_gpu) - min_d C <= 2 eps max_d C."""
    eps = (2 * iters - 1) * NARROW_REL[dtype] + DT_REL
    return 2.0 * eps * np.abs(cagg).max(axis=2)


def _narrow_check(disp, cagg, dtype, iters=3):
    slack, _ = _near_tie_ok(disp, cagg)
    tol = _narrow_tol(dtype, iters, cagg)
    return slack, slack <= tol


def _solve_gpu(pr, D, r, dtype, iters=3, flags=0):
    H, W = pr.left.shape
    p = zdt.params(W, H, D, r, dt_iters=iters, vol_dtype=dtype, flags=flags)
    solver = zdt.Solver(p)
    disp = solver(dev(pr.left), dev(pr.right))
    torch.cuda.synchronize()
    return host(disp)


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16], ids=["f32", "f16", "bf16"])
def test_stereo_solve_bands(dtype):
    note(f"stereo_solve bands 320x96 D=32 dtype={dtype}")
    pr = scenes.bands_pair()
    D, r = 32, 4
    disp = _solve_gpu(pr, D, r, dtype)
    o_disp, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, 20.0, 0.1, 3, keep_volume=True)
    mism = (disp != o_disp).mean()
    note(f"  mismatch vs oracle = {100 * mism:.4f} %")
    if dtype == zdt.ZDT_F32:
        slack, ok = _near_tie_ok(disp, cagg)
    else:
        slack, ok = _narrow_check(disp, cagg, dtype)
    assert ok.all(), slack[~ok].max()
    if dtype == zdt.ZDT_F16:
        assert mism <= 1e-3
    gt = pr.gt.astype(np.int32)
    for k, d in enumerate(pr.band_disps):
        lo, hi = pr.band_edges[k], pr.band_edges[k + 1]
        q = (hi - lo) // 4
        assert np.all(disp[:, max(lo + q, d + r):hi - q] == d)


ODD = [(37, 23, 11, 2), (100, 17, 65, 3), (50, 40, 1, 1), (30, 12, 45, 4), (7, 5, 9, 4), (129, 33, 130, 0),
       (200, 150, 200, 2), (64, 700, 16, 3), (120, 50, 30, 7)]


@pytest.mark.parametrize("iters", [0, 1, 2])
@pytest.mark.parametrize("shape", ODD, ids=ids(ODD))
def test_stereo_solve_odd_shapes_fp32(shape, iters):
    W, H, D, r = shape
    note(f"stereo_solve odd {shape} iters={iters}")
    pr = pair_for(W, H, D, seed=4)
    disp = _solve_gpu(pr, D, r, zdt.ZDT_F32, iters=iters)
    o_disp, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, 20.0, 0.1, iters, keep_volume=True)
    slack, ok = _near_tie_ok(disp, cagg)
    note(f"  mismatch {100 * (disp != o_disp).mean():.4f} %")
    assert ok.all(), slack[~ok].max()


NARROW = [(160, 48, 128, 4), (96, 40, 96, 2), (200, 64, 200, 3), (640, 32, 130, 4), (37, 23, 70, 1)]


@pytest.mark.parametrize("dtype", [zdt.ZDT_F16, zdt.ZDT_BF16], ids=["f16", "bf16"])
@pytest.mark.parametrize("shape", NARROW, ids=ids(NARROW))
def test_stereo_solve_narrow_several_chunks(shape, dtype):
    """16-bit working volumes with several 32- and 64-disparity chunks (odd
    counts included): every disparity that differs from the FP64 oracle's is
    a near-tie within the storage type's propagated rounding (_narrow_tol)."""
    W, H, D, r = shape
    note(f"stereo_solve narrow {shape} dtype={dtype}")
    pr = pair_for(W, H, D, seed=11)
    disp = _solve_gpu(pr, D, r, dtype)
    o_disp, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, 20.0, 0.1, 3, keep_volume=True)
    mism = (disp != o_disp).mean()
    slack, ok = _narrow_check(disp, cagg, dtype)
    rel = (slack / np.maximum(np.abs(cagg).max(axis=2), 1e-300)).max()
    note(f"  mismatch {100 * mism:.4f} %, worst relative slack {rel:.2e}")
    assert ok.all(), (slack - _narrow_tol(dtype, 3, cagg)).max()


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_F16], ids=["f32", "f16"])
def test_widest_row_largest_window(dtype):
    """The largest LDS layout of the fused cost pass: a 1920-wide row (32
    segments of 60) with the 15x15 window, whose column records are 7 words
    (about 145 KB of LDS with the FP16 gain lines).  Disparities against the
    FP64 oracle, with the bars of the other end-to-end tests."""
    W, H, D, r = 1920, 24, 64, 7
    note(f"stereo_solve {W}x{H} D={D} r={r} dtype={dtype}")
    pr = pair_for(W, H, D, seed=21)
    disp = _solve_gpu(pr, D, r, dtype)
    o_disp, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, 20.0, 0.1, 3, keep_volume=True)
    slack, ok = _near_tie_ok(disp, cagg)
    mism = (disp != o_disp).mean()
    note(f"  mismatch {100 * mism:.4f} %")
    if dtype != zdt.ZDT_F32:
        slack, ok = _narrow_check(disp, cagg, dtype)
    assert ok.all(), slack[~ok].max()


def test_fused_equals_unfused_fp32():
    """stereo_solve (cost fused into the first H pair, WTA into the last V
    pair) equals zncc_cost_volume + dt_aggregate + wta_disparity bit for bit."""
    W, H, D, r = 333, 70, 96, 3
    note("fused vs unfused")
    pr = pair_for(W, H, D, seed=6)
    p = zdt.params(W, H, D, r, dt_iters=2)
    L, R = dev(pr.left), dev(pr.right)
    d_fused = zdt.Solver(p)(L, R)
    vol = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, L, R, vol)
    zdt.dt_aggregate(p, L, vol)
    d_unf = torch.empty((H, W), dtype=torch.int32, device="cuda")
    zdt.wta_disparity(p, vol, d_unf)
    torch.cuda.synchronize()
    assert torch.equal(d_fused, d_unf)


def test_guide_target_flag():
    W, H, D, r = 120, 40, 24, 2
    note("guide = target")
    pr = pair_for(W, H, D, seed=8)
    disp = _solve_gpu(pr, D, r, zdt.ZDT_F32, iters=1, flags=zdt.ZDT_FLAG_GUIDE_TARGET)
    o_disp, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, 20.0, 0.1, 1, guide_target=True, keep_volume=True)
    slack, ok = _near_tie_ok(disp, cagg)
    assert ok.all(), slack[~ok].max()


# ----------------------------------------------------------------- full size
_FULL = {}


def _full_oracle():
    if not _FULL:
        pr = scenes.workload("planes_1280x384_d128")
        note(f"oracle: 128 aggregated slices of 1280x384 on {ORACLE_THREADS} threads")
        c = oracle.solve_slices(pr.left, pr.right, 4, range(128), 20.0, 0.1, 3, threads=ORACLE_THREADS)
        _FULL["pair"] = pr
        _FULL["cagg"] = np.ascontiguousarray(np.moveaxis(c, 0, 2))      # [H][W][D]
        _FULL["disp"] = np.argmin(_FULL["cagg"], axis=2).astype(np.int32)
    return _FULL


def test_full_size_sums_and_cost():
    """1280x384, D = 128, 9x9: the launch configuration the benchmark times."""
    W, H, D, r = 1280, 384, 128, 4
    pr = scenes.workload("planes_1280x384_d128")
    note("full-size sums")
    p = zdt.params(W, H, D, r)
    i32 = dict(dtype=torch.int32, device="cuda")
    s_l, s_ll = torch.empty((H, W), **i32), torch.empty((H, W), **i32)
    s_t, s_tt = torch.empty((H, W + D - 1), **i32), torch.empty((H, W + D - 1), **i32)
    s_rt = torch.empty((H, W, D), **i32)
    L, R = dev(pr.left), dev(pr.right)
    zdt.zncc_window_sums(p, L, R, s_l, s_ll, s_t, s_tt, s_rt)
    torch.cuda.synchronize()
    o = oracle.window_sums(pr.left, pr.right, D, r)
    for g, w in zip((s_l, s_ll, s_t, s_tt), o):
        assert np.array_equal(host(g), w)
    rng = np.random.default_rng(0)
    srt = host(s_rt)
    for _ in range(3000):
        x, y, d = int(rng.integers(0, W)), int(rng.integers(0, H)), int(rng.integers(0, D))
        assert srt[y, x, d] == oracle.cross_sum_at(pr.left, pr.right, r, x, y, d), (x, y, d)
    del srt, s_rt
    note("full-size cost")
    cost = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, L, R, cost)
    torch.cuda.synchronize()
    c = host(cost)
    for d in (0, 1, 37, 64, 100, 127):
        err = np.abs(c[:, :, d].astype(np.float64) - oracle.zncc_cost_slice(pr.left, pr.right, r, d)).max()
        assert err <= 1e-5, (d, err)


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16], ids=["f32", "f16", "bf16"])
def test_full_size_end_to_end(dtype):
    W, H, D, r = 1280, 384, 128, 4
    full = _full_oracle()
    pr = full["pair"]
    note(f"full-size stereo_solve dtype={dtype}")
    disp = _solve_gpu(pr, D, r, dtype)
    mism = (disp != full["disp"]).mean()
    note(f"  disparity mismatch vs FP64 oracle: {100 * mism:.4f} % (all pixels)")
    if dtype == zdt.ZDT_F32:
        slack, ok = _near_tie_ok(disp, full["cagg"])
    else:
        slack, ok = _narrow_check(disp, full["cagg"], dtype)
    assert ok.all(), slack[~ok].max()
    if dtype == zdt.ZDT_F16:
        assert mism <= 1e-3


def test_full_size_dt_slices_fp32():
    """Aggregated volume at full size on sampled disparity slices."""
    W, H, D, r = 1280, 384, 128, 4
    full = _full_oracle()
    pr = full["pair"]
    note("full-size dt_aggregate slices")
    p = zdt.params(W, H, D, r, dt_iters=3)
    L, R = dev(pr.left), dev(pr.right)
    vol = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, L, R, vol)
    zdt.dt_aggregate(p, L, vol)
    torch.cuda.synchronize()
    got = host(vol).astype(np.float64)
    rel = _dt_check(got, full["cagg"])
    note(f"  max rel err = {rel:.3e}")
    assert rel <= DT_REL


def _oracle_slices(fn, ds):
    """fn(d) -> [H][W] for each d in ds, on ORACLE_THREADS threads (each call
    single-threaded; ctypes releases the GIL) -> [H][W][len(ds)]."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=ORACLE_THREADS) as ex:
        return np.ascontiguousarray(np.stack(list(ex.map(fn, ds)), axis=2))


def test_full_size_raw_cost_every_element():
    """1280x384, D = 128, 9x9: the whole raw cost volume in FP32, FP16 and
    BF16 against the FP64 oracle, element by element (FP32 <= 1e-5; 16-bit:
    half an ulp of [1, 2) + 1e-6)."""
    W, H, D, r = 1280, 384, 128, 4
    pr = scenes.workload("planes_1280x384_d128")
    note("full-size raw cost volume, every element")
    L, R = dev(pr.left), dev(pr.right)
    got = {}
    for dt in (zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16):
        t = torch.empty((H, W, D), dtype=zdt.torch_dtype(dt), device="cuda")
        zdt.zncc_cost_volume(zdt.params(W, H, D, r, vol_dtype=dt), L, R, t)
        torch.cuda.synchronize()
        got[dt] = host(t)
        del t
    for d0 in range(0, D, 32):
        ds = list(range(d0, d0 + 32))
        want = _oracle_slices(lambda d: oracle.zncc_cost_slice(pr.left, pr.right, r, d), ds)
        for dt, bar in ((zdt.ZDT_F32, 1e-5), (zdt.ZDT_F16, HALF_ULP[zdt.ZDT_F16] + 1e-6),
                        (zdt.ZDT_BF16, HALF_ULP[zdt.ZDT_BF16] + 1e-6)):
            err = np.abs(got[dt][:, :, d0:d0 + 32].astype(np.float64) - want).max()
            note(f"  d {d0}..{d0 + 31} dtype={dt}: max |d cost| = {err:.3e}")
            assert err <= bar, (dt, d0, err)


def _canonical_gap(v):
    return v - v.min(axis=2, keepdims=True)


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_BF16], ids=["f32", "bf16"])
def test_full_size_aggregated_volume_canonical_gap(dtype):
    """The aggregated volume of dt_aggregate at 1280x384, D = 128, three
    sweeps, in canonical form: G = C - min_d C, the device volume divided by
    the reported global scale.  The raw cost is stored once and each of the
    2 I pass pairs stores its output, every state non-negative, so each
    element is within eps = (2I + 1) NARROW_REL + DT_REL of itself (FP32:
    DT_REL) and |dG| <= 2 eps max_d C."""
    W, H, D, r = 1280, 384, 128, 4
    full = _full_oracle()
    pr = full["pair"]
    note(f"full-size aggregated volume, canonical gap, dtype={dtype}")
    p = zdt.params(W, H, D, r, dt_iters=3, vol_dtype=dtype)
    L, R = dev(pr.left), dev(pr.right)
    vol = torch.empty((H, W, D), dtype=zdt.torch_dtype(dtype), device="cuda")
    zdt.zncc_cost_volume(p, L, R, vol)
    scale = zdt.dt_aggregate(p, L, vol)
    torch.cuda.synchronize()
    got = host(vol).astype(np.float64) / scale
    del vol
    cmax = np.abs(full["cagg"]).max(axis=2)
    err = np.abs(_canonical_gap(got) - _canonical_gap(full["cagg"])).max(axis=2) / cmax
    eps = DT_REL if dtype == zdt.ZDT_F32 else 7 * NARROW_REL[dtype] + DT_REL
    note(f"  max |dG| / max_d C = {err.max():.3e} (bar {2 * eps:.3e})")
    assert err.max() <= 2 * eps


def test_full_size_fp16_working_volume_canonical_gap():
    """The FP16 working volume of stereo_solve at 1280x384, D = 128, three
    sweeps: after the call it holds the last H pair's output (10 passes),
    stored as C 2^(13 - k) with k = floor(log2 G) of the gain map the pass
    leaves in the workspace.  Decoded, in canonical form, against the
    oracle's first 10 passes: 2 I - 1 stores of relative rounding 2^-11 on
    non-negative states, so |dG| <= 2 ((2I-1) 2^-11 + DT_REL) max_d C."""
    W, H, D, r = 1280, 384, 128, 4
    pr = scenes.workload("planes_1280x384_d128")
    note("full-size FP16 working volume after the last H pair, canonical gap")
    p = zdt.params(W, H, D, r, dt_iters=3, vol_dtype=zdt.ZDT_F16)
    s = zdt.Solver(p)
    s(dev(pr.left), dev(pr.right))
    torch.cuda.synchronize()
    gain = s.ws[:W * H * 4].view(torch.float32).reshape(H, W).cpu().numpy()
    _, e = np.frexp(gain)                                     # gain = m 2^e, m in [0.5, 1)
    got = host(s.vol).astype(np.float64) * np.ldexp(1.0, (e - 1) - 13)[:, :, None]
    wh, wv = oracle.dt_weights(pr.left, 20.0, 0.1)
    want = _oracle_slices(lambda d: oracle.dt_passes(oracle.zncc_cost_slice(pr.left, pr.right, r, d), wh, wv, 0, 10),
                          range(D))
    cmax = np.abs(want).max(axis=2)
    err = np.abs(_canonical_gap(got) - _canonical_gap(want)).max(axis=2) / cmax
    eps = 5 * NARROW_REL[zdt.ZDT_F16] + DT_REL
    note(f"  max |dG| / max_d C = {err.max():.3e} (bar {2 * eps:.3e})")
    assert err.max() <= 2 * eps


# ------------------------------------------------ the paper's own configuration
PAPER = dict(r=1, sigma_s=5.0, sigma_r=52.0 / 255.0, iters=1)   # 3x3, one sweep, sigma_r = 52 on 0..255


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16], ids=["f32", "f16", "bf16"])
def test_paper_configuration_full_size(dtype):
    """1280x384, D = 128 with the paper's system parameters (3x3 ZNCC, one
    L-R-U-D sweep, sigma_s = 5, sigma_r = 52 in raw intensity units): FP32
    disagreements are near-ties of the FP64 oracle; 16-bit within 0.1 % / 2 %."""
    W, H, D = 1280, 384, 128
    pr = scenes.workload("planes_1280x384_d128")
    if "paper" not in _FULL:
        note(f"oracle: 128 slices at the paper's parameters on {ORACLE_THREADS} threads")
        c = oracle.solve_slices(pr.left, pr.right, PAPER["r"], range(D), PAPER["sigma_s"], PAPER["sigma_r"],
                                PAPER["iters"], threads=ORACLE_THREADS)
        _FULL["paper"] = np.ascontiguousarray(np.moveaxis(c, 0, 2))
    cagg = _FULL["paper"]
    o_disp = np.argmin(cagg, axis=2)
    p = zdt.params(W, H, D, PAPER["r"], PAPER["sigma_s"], PAPER["sigma_r"], PAPER["iters"], vol_dtype=dtype)
    disp = zdt.Solver(p)(dev(pr.left), dev(pr.right)).cpu().numpy()
    mism = (disp != o_disp).mean()
    note(f"  paper configuration dtype={dtype}: mismatch {100 * mism:.4f} %")
    if dtype == zdt.ZDT_F32:
        slack, ok = _near_tie_ok(disp, cagg)
    else:
        slack, ok = _narrow_check(disp, cagg, dtype, iters=PAPER["iters"])
    assert ok.all(), slack[~ok].max()
    if dtype == zdt.ZDT_F16:
        assert mism <= 1e-3


def test_cost_bright_15x15_window_wraps_exactly():
    """l = 15 on bright textured images: l^2 S_RT exceeds 2^31 (up to 3.3e9),
    so the numerator is formed in wrapping 32-bit arithmetic; sums stay
    bit-exact and costs match the oracle's int64 / FP64 evaluation."""
    W, H, D, r = 90, 40, 24, 7
    rng = np.random.default_rng(15)
    left = rng.integers(190, 256, (H, W)).astype(np.uint8)
    left[rng.random((H, W)) < 0.05] = 0                        # a few dark pixels keep the variance up
    right = np.roll(np.clip(left.astype(np.int32) - 3, 0, 255).astype(np.uint8), -4, axis=1)   # match at d = 4
    p = zdt.params(W, H, D, r)
    i32 = dict(dtype=torch.int32, device="cuda")
    s_rt = torch.empty((H, W, D), **i32)
    zdt.zncc_window_sums(p, dev(left), dev(right), s_rt=s_rt)
    cost = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
    zdt.zncc_cost_volume(p, dev(left), dev(right), cost)
    torch.cuda.synchronize()
    srt = host(s_rt)
    assert int(srt.max()) * (2 * r + 1) ** 2 > 2 ** 31           # the case is really past int32
    assert np.array_equal(srt, oracle.cross_sums(left, right, D, r))
    want = oracle.zncc_cost(left, right, D, r)
    err = np.abs(host(cost).astype(np.float64) - want).max()
    note(f"  l=15 bright: max |d cost| = {err:.2e}")
    assert err <= 1e-5


# ------------------------------------------------ integer volumes (Sec. IV-C)
def test_i8_codec_on_device_matches_oracle():
    """The device's 8-bit code, over every int16 value, bit for bit."""
    v = torch.arange(-32768, 32768, dtype=torch.int32).to(torch.int16).cuda()
    codes = torch.empty(v.shape, dtype=torch.uint8, device="cuda")
    dec = torch.empty(v.shape, dtype=torch.int16, device="cuda")
    zdt.i8_codec(v, codes, dec)
    torch.cuda.synchronize()
    want_codes = oracle.i8_encode(v.cpu().numpy())
    assert np.array_equal(codes.cpu().numpy(), want_codes)
    assert np.array_equal(dec.cpu().numpy(), oracle.i8_decode(want_codes))


@pytest.mark.parametrize("dtype", [zdt.ZDT_I16, zdt.ZDT_I8], ids=["i16", "i8"])
@pytest.mark.parametrize("W,r", [(160, 2), (157, 0), (133, 4), (101, 5), (96, 6), (77, 7), (1920, 7)])
def test_integer_volume_d_arb_slice_is_zero(dtype, W, r):
    """The first sweep's normalization (Int16: U2D, Int8: R2L) subtracts the
    d_arb = 0 slice of a stored state taken from disparity chunk 0; the
    passes map a zero slice to zero, so after two sweeps the stored state (the
    second R2L output) has an all-zero slice d = 0 -- which also checks that
    the subtracted map equals chunk 0's own values bit for bit, at every
    radius and at widths that are not a multiple of a segment."""
    H, D = 60, 40
    pr = pair_for(W, H, D, seed=13 + r)
    p = zdt.params(W, H, D, r, 2.0, 52.0 / 255.0, 2, vol_dtype=dtype)
    s = zdt.Solver(p)
    disp = s(dev(pr.left), dev(pr.right))
    torch.cuda.synchronize()
    vol = s.vol.cpu().numpy()
    assert np.all(vol[:, :, 0] == 0)
    if r > 0:  # a 1x1 window has no variance: every cost is 1, the normalized volume 0
        assert np.any(vol[:, :, 1:] != 0)
    else:
        assert np.all(vol == 0)
    d = disp.cpu().numpy()
    assert d.min() >= 0 and d.max() < D


T_INT = 21.0
_DECODE = None


def _decoded(codes):
    """int16 values of 8-bit codes, by a table of the oracle's decoding."""
    global _DECODE
    if _DECODE is None:
        _DECODE = oracle.i8_decode(np.arange(256, dtype=np.uint8)).astype(np.int64)
    return _DECODE[codes.astype(np.int64)]


def _stored_state(s, dtype):
    v = s.vol.cpu().numpy()
    return v.astype(np.int64) if dtype == zdt.ZDT_I16 else _decoded(v)


def _int_compare(pr, D, r, ss, sr, iters, dtype):
    """Run the device's integer path and the oracle's paper form.  Returns the
    device disparities, the share of identical elements of the stored state
    the device leaves in its volume (the last R2L output: the oracle's state
    after 4 I - 2 passes, as integers), its largest difference, the share of
    differing disparities, and whether every differing disparity is a
    near-tie of the oracle's final values within the bar derived from the
    stored states' differences: the last V pair maps a stored difference
    field Dst (T units) to at most D(U(Dst) + 1) -- U and D linear with
    non-negative weights, and the U2D output's rounding moving a value at
    most one unit further -- plus FP32 arithmetic (DT_REL of the values)."""
    H, W = pr.left.shape
    code8 = dtype == zdt.ZDT_I8
    s = zdt.Solver(zdt.params(W, H, D, r, ss, sr, iters, vol_dtype=dtype))
    disp = s(dev(pr.left), dev(pr.right)).cpu().numpy()
    torch.cuda.synchronize()
    o = oracle.int_solve(pr.left, pr.right, D, r, ss, sr, iters, T=T_INT, code8=code8, keep_volume=True)
    st = oracle.int_solve(pr.left, pr.right, D, r, ss, sr, iters, T=T_INT, code8=code8, keep_volume=True,
                          npasses=4 * iters - 2)
    assert o.saturated == 0 and st.saturated == 0
    want = np.rint(st.volume * T_INT).astype(np.int64)
    got = _stored_state(s, dtype)
    same = float((got == want).mean())
    dst = np.abs(got - want).max(axis=2).astype(np.float64)
    del got, want, st
    wh, wv = oracle.dt_weights(pr.left, ss, sr)
    e = oracle.dt_passes(oracle.dt_passes(dst, wh, wv, 2, 1) + 1.0, wh, wv, 3, 1)
    fin = o.volume * T_INT
    tol = 2.0 * (e + DT_REL * np.abs(fin).max(axis=2))
    slack, _ = _near_tie_ok(disp, fin)
    ok = bool(np.all(slack <= tol))
    return disp, same, float(dst.max()), float((disp != o.disp).mean()), ok, float((slack / tol).max())


INT_CASES = [(160, 60, 40, 2, 5.0, 1), (97, 41, 65, 1, 2.0, 2), (64, 48, 24, 3, 8.0, 1), (120, 50, 70, 4, 1.0, 3)]


@pytest.mark.parametrize("dtype", [zdt.ZDT_I16, zdt.ZDT_I8], ids=["i16", "i8"])
@pytest.mark.parametrize("case", INT_CASES, ids=["%dx%d_d%d_r%d_s%g_i%d" % c for c in INT_CASES])
def test_integer_volumes_match_the_paper_form(case, dtype):
    """The device runs the paper's per-pass FastDT (Sec. V-C): its fused pass
    pairs round the in-register L2R and U2D outputs exactly as those kernels'
    stores would, so it computes the oracle's paper form up to FP32 rounding.
    Where FP32 and FP64 round a state to different integers, values differ by
    one unit there and by what the later passes make of it.  Bars: at most
    0.1 % of the elements of the last stored state differ, and every
    differing disparity is a near-tie within the bar of _int_compare (the
    share of differing disparities is reported; on these small images a
    handful of pixels is already 0.1 %)."""
    W, H, D, r, ss, iters = case
    sr = 52.0 / 255.0
    pr = pair_for(W, H, D, seed=W + iters)
    note(f"integer path {case} dtype={dtype}")
    _, same, dmax, mism, ok, worst = _int_compare(pr, D, r, ss, sr, iters, dtype)
    note(f"  stored state identical: {100 * same:.4f} % (max |d| {dmax:g}); disparities differing from the "
         f"paper form: {100 * mism:.4f} %; worst slack / bar {worst:.3f}")
    assert same >= 0.999 and ok


def _paper_int_error_field(wh, wv, iters, T):
    """Componentwise bound on |Int16 paper form - DT(C - C0)| (cost units):
    each store rounds by at most 1/(2T), a pass maps a bound field to the
    same pass of it, the U2D normalization doubles it."""
    e = np.zeros(wh.shape)
    for n in range(4 * iters):
        k = n % 4
        if k == 2:
            e = 2.0 * e
        e = oracle.dt_passes(e, wh, wv, k, 1)
        if n + 1 < 4 * iters:
            e = e + 0.5 / T
    return e


@pytest.mark.parametrize("ss,iters", [(8.0, 1), (1.0, 3)])
def test_int16_against_the_float_path(ss, iters):
    """Int16 against the FP64 float DT of the cost (no integer oracle
    involved): the device rounds every state but the last to a multiple of
    1/T, so its aggregated costs lie within the propagated rounding field E
    of the float ones (plus FP32 arithmetic, DT_REL of the un-normalized
    magnitude 2 G, G the DT of ones), and every disparity that differs is a
    near-tie within twice that."""
    W, H, D, r, sr = 200, 80, 48, 3, 52.0 / 255.0
    pr = pair_for(W, H, D, seed=77)
    note(f"Int16 vs the float path, sigma_s={ss}, {iters} sweeps")
    p = zdt.params(W, H, D, r, ss, sr, iters, vol_dtype=zdt.ZDT_I16)
    disp = zdt.Solver(p)(dev(pr.left), dev(pr.right)).cpu().numpy()
    _, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, ss, sr, iters, keep_volume=True)
    wh, wv = oracle.dt_weights(pr.left, ss, sr)
    e = _paper_int_error_field(wh, wv, iters, T_INT)
    g = oracle.dt_slice(np.ones((H, W)), wh, wv, iters)
    tol = 2.0 * (e + DT_REL * 2.0 * g)
    slack, _ = _near_tie_ok(disp, cagg)
    mism = float((disp != np.argmin(cagg, axis=2)).mean())
    note(f"  differing from the float path: {100 * mism:.3f} %; worst slack / bar "
         f"{(slack / tol).max():.3f}")
    assert np.all(slack <= tol)


def test_integer_volumes_refuse_parameters_that_could_saturate():
    """sigma_s = 20 with three sweeps: a stored int16 state could leave the
    int16 range (the bound grows by 1/(1-K) = 20.5 per pass), so the call is
    refused with ZDT_EUNSUPPORTED before anything runs."""
    W, H, D = 64, 32, 16
    for dt in (zdt.ZDT_I16, zdt.ZDT_I8):
        p = zdt.params(W, H, D, 4, 20.0, 0.1, 3, vol_dtype=dt)
        with pytest.raises(zdt.ZdtError) as ei:
            zdt.Solver(p)(torch.zeros((H, W), dtype=torch.uint8, device="cuda"),
                          torch.zeros((H, W), dtype=torch.uint8, device="cuda"))
        assert ei.value.code == -4


@pytest.mark.parametrize("dtype", [zdt.ZDT_I16, zdt.ZDT_I8], ids=["i16", "i8"])
def test_integer_volumes_paper_configuration(dtype):
    """1280x384, D = 128 at the paper's parameters with its narrow integer
    volumes (T = 21, d_arb = 0; Int8 = 6-bit code + 2-bit flag): against the
    oracle's paper form (stored state and disparities), and, for the accuracy
    the narrow volumes cost, against the FP64 float path (reported)."""
    D = 128
    pr = scenes.workload("planes_1280x384_d128")
    disp, same, dmax, mism_int, ok, worst = _int_compare(pr, D, PAPER["r"], PAPER["sigma_s"], PAPER["sigma_r"],
                                                         PAPER["iters"], dtype)
    if "paper" not in _FULL:
        c = oracle.solve_slices(pr.left, pr.right, PAPER["r"], range(D), PAPER["sigma_s"], PAPER["sigma_r"],
                                PAPER["iters"], threads=ORACLE_THREADS)
        _FULL["paper"] = np.ascontiguousarray(np.moveaxis(c, 0, 2))
    o_disp = np.argmin(_FULL["paper"], axis=2)
    mism = (disp != o_disp).mean()
    note(f"  paper configuration dtype={dtype}: stored state identical {100 * same:.4f} % (max |d| {dmax:g}); "
         f"{100 * mism_int:.4f} % of disparities differ from the paper form (worst slack / bar {worst:.3f}); "
         f"{100 * mism:.3f} % from the float oracle")
    assert same >= 0.999 and ok and mism_int <= 1e-3
    assert mism <= 0.1


def _random_cases(n, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        W, H = int(rng.integers(1, 301)), int(rng.integers(1, 151))
        D, r = int(rng.integers(1, 161)), int(rng.integers(0, 8))
        sigma_s = float(rng.uniform(2.0, 40.0))
        sigma_r = float(rng.choice([0.05, 0.2, np.inf]))
        iters = int(rng.integers(0, 4))
        flags = zdt.ZDT_FLAG_GUIDE_TARGET if rng.random() < 0.3 else 0
        out.append((W, H, D, r, round(sigma_s, 3), sigma_r, iters, flags))
    return out


RANDOM = _random_cases(16)


@pytest.mark.parametrize("case", RANDOM, ids=["%dx%d_d%d_r%d_s%g_%g_i%d_g%d" % c for c in RANDOM])
def test_random_shapes_and_parameters_end_to_end(case):
    """Seeded random shapes and parameters, FP32 end to end.  Bar: the DT bound
    for this sigma_s and sweep count, 2 x (4 I) x 2^-24 x 1/(1 - K) relative to
    the pixel's largest aggregated cost (K = exp(-1/sigma_s)); with I = 0 the
    raw-cost bar (1e-5, doubled for the two sides of a near-tie)."""
    W, H, D, r, sigma_s, sigma_r, iters, flags = case
    note("random case %s" % (case,))
    k = min(D - 1, max(1, D // 3))
    pr = scenes.bands_pair(W=W, H=H, D=max(D, 2), seed=W * 7 + H, band_disps=tuple(sorted({0, k})))
    p = zdt.params(W, H, D, r, sigma_s=sigma_s, sigma_r=sigma_r, dt_iters=iters, flags=flags)
    solver = zdt.Solver(p)
    disp = host(solver(dev(pr.left), dev(pr.right)))
    torch.cuda.synchronize()
    _, cagg = oracle.stereo_solve(pr.left, pr.right, D, r, sigma_s, sigma_r, iters,
                                  guide_target=bool(flags & zdt.ZDT_FLAG_GUIDE_TARGET), keep_volume=True)
    picked = np.take_along_axis(cagg, disp[:, :, None].astype(np.int64), axis=2)[:, :, 0]
    slack = picked - cagg.min(axis=2)
    if iters == 0:
        tol = 2e-5 * np.ones_like(slack)
    else:
        gain = 1.0 / -np.expm1(-1.0 / sigma_s)
        tol = 2 * (4 * iters) * 2.0 ** -24 * gain * np.abs(cagg).max(axis=2)
    assert disp.min() >= 0 and disp.max() < D
    assert np.all(slack <= tol), (slack - tol).max()
