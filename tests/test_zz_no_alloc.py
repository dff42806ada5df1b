"""The workspace-free entry point stereo_solve_static_ws, called through the C
ABI, against stereo_solve with a caller workspace: identical disparities on
two calls in a row, the second with a smaller pair (the library's array keeps
the first call's contents), for every volume type; parameters whose workspace
exceeds the array are refused."""
import ctypes

import numpy as np
import pytest

from paper_2212_00476_amd import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2212_00476_amd as zdt  # noqa: E402
from paper_2212_00476_amd import _lib  # noqa: E402


def _pair(W, H, D, seed):
    ds = tuple(sorted({max(0, min(D - 1, k)) for k in (1, D // 3, (2 * D) // 3)}))
    pr = scenes.bands_pair(W=W, H=H, D=D, seed=seed, band_disps=ds)
    return (torch.from_numpy(np.ascontiguousarray(pr.left)).cuda(),
            torch.from_numpy(np.ascontiguousarray(pr.right)).cuda())


def _both(p, left, right):
    """(disparities from stereo_solve with its own workspace, from stereo_solve_static_ws)."""
    H, W = p.height, p.width
    vol = torch.empty((H, W, p.max_disp), dtype=zdt.torch_dtype(p.vol_dtype), device="cuda")
    ws_n = zdt.workspace_size(p)
    ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda") if ws_n else None
    d_ref = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
    zdt.stereo_solve(p, left, right, d_ref, vol, ws)
    d_sta = torch.full((H, W), -2, dtype=torch.int32, device="cuda")
    lib = zdt.load()
    rc = lib.stereo_solve_static_ws(ctypes.byref(p), ctypes.c_void_p(left.data_ptr()),
                                    ctypes.c_void_p(right.data_ptr()), ctypes.c_void_p(d_sta.data_ptr()),
                                    ctypes.c_void_p(vol.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.ZDT_OK, lib.zdt_last_error().decode()
    torch.cuda.synchronize()
    return d_ref.cpu().numpy(), d_sta.cpu().numpy()


@pytest.mark.parametrize("dtype", [zdt.ZDT_F32, zdt.ZDT_F16, zdt.ZDT_BF16, zdt.ZDT_I16, zdt.ZDT_I8],
                         ids=["f32", "f16", "bf16", "i16", "i8"])
def test_static_workspace_equals_caller_workspace_twice(dtype):
    ss, iters = (5.0, 1) if dtype in (zdt.ZDT_I16, zdt.ZDT_I8) else (20.0, 3)
    print(f"static workspace, dtype={dtype}", flush=True)
    for (W, H, D, seed) in ((1280, 384, 128, 1), (333, 70, 96, 2)):   # the second call smaller
        p = zdt.params(W, H, D, 4, sigma_s=ss, dt_iters=iters, vol_dtype=dtype)
        assert 0 < zdt.workspace_size(p) <= zdt.STATIC_WS_BYTES
        left, right = _pair(W, H, D, seed)
        d_ref, d_sta = _both(p, left, right)
        assert d_ref.min() >= 0 and np.array_equal(d_ref, d_sta), (W, H, D)


def test_static_workspace_raw_cost_path():
    """dt_iters = 0 needs no workspace at all."""
    p = zdt.params(200, 64, 40, 3, dt_iters=0)
    left, right = _pair(200, 64, 40, 3)
    d_ref, d_sta = _both(p, left, right)
    assert np.array_equal(d_ref, d_sta)


def test_static_workspace_too_large_is_refused():
    p = zdt.params(1920, 1080, 256, 4, vol_dtype=zdt.ZDT_F16)
    assert zdt.workspace_size(p) > zdt.STATIC_WS_BYTES
    lib = zdt.load()
    rc = lib.stereo_solve_static_ws(ctypes.byref(p), None, None, None, None, None)
    assert rc == _lib.ZDT_EUNSUPPORTED
    assert b"workspace" in lib.zdt_last_error()
