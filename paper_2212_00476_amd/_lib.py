"""ctypes binding of ``libzdt.so`` (the C ABI in ``include/zdt.h``).

Argument marshalling only: tensors are passed as raw device pointers and every
step runs in the library's HIP kernels.  There is no CPU fallback; if the
library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# ZDT_LIBRARY names another build of the same library (e.g. to compare two
# builds side by side); by default the in-tree libzdt.so.
LIB_PATH = os.environ.get("ZDT_LIBRARY") or os.path.join(HERE, "libzdt.so")

ZDT_OK, ZDT_EINVAL, ZDT_ENOMEM, ZDT_EHIP, ZDT_EUNSUPPORTED = 0, -1, -2, -3, -4
ZDT_F32, ZDT_F16, ZDT_BF16, ZDT_I16, ZDT_I8 = 0, 1, 2, 3, 4
ZDT_FLAG_NORMALIZE = 1
ZDT_FLAG_GUIDE_TARGET = 2

EXPORTED = ("zdt_workspace_size", "zdt_volume_size", "zncc_cost_volume", "dt_aggregate", "wta_disparity",
            "stereo_solve", "stereo_solve_static_ws", "stereo_solve_batch", "zdt_graph_create",
            "zdt_graph_launch", "zdt_graph_destroy", "zdt_plan_candidates", "zdt_get_plan", "zdt_set_plan",
            "zdt_autotune", "zncc_window_sums", "zdt_i8_codec", "sgm_aggregate", "sgm_disparity",
            "stereo_solve_sgm", "zdt_integral_workspace_size", "zncc_window_sums_integral", "zdt_last_error", "zdt_profile_enable", "zdt_profile_collect", "zdt_profile_entry")


class ZdtParams(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("max_disp", ctypes.c_int32), ("radius", ctypes.c_int32), ("sigma_s", ctypes.c_float),
                ("sigma_r", ctypes.c_float), ("dt_iters", ctypes.c_int32), ("vol_dtype", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class ZdtJob(ctypes.Structure):
    _fields_ = [("params", ZdtParams), ("left", ctypes.c_void_p), ("right", ctypes.c_void_p),
                ("disp", ctypes.c_void_p), ("vol", ctypes.c_void_p), ("ws", ctypes.c_void_p)]


class ZdtPlan(ctypes.Structure):
    _fields_ = [("h_lanes", ctypes.c_int32), ("h_seg", ctypes.c_int32), ("v_lanes", ctypes.c_int32),
                ("v_seg", ctypes.c_int32)]

    def astuple(self):
        return (self.h_lanes, self.h_seg, self.v_lanes, self.v_seg)


class ZdtError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


_lib = None


def load():
    """Load libzdt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run `python -m paper_2212_00476_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, PP = ctypes.c_void_p, ctypes.POINTER(ZdtParams)
    lib.zdt_workspace_size.argtypes = [PP]
    lib.zdt_workspace_size.restype = ctypes.c_size_t
    lib.zdt_volume_size.argtypes = [PP]
    lib.zdt_volume_size.restype = ctypes.c_size_t
    lib.zncc_cost_volume.argtypes = [PP, P, P, P, P]
    lib.dt_aggregate.argtypes = [PP, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.wta_disparity.argtypes = [PP, P, P, P]
    lib.stereo_solve.argtypes = [PP, P, P, P, P, P, P]
    lib.stereo_solve_static_ws.argtypes = [PP, P, P, P, P, P]
    lib.zncc_window_sums.argtypes = [PP, P, P, P, P, P, P, P, P]
    lib.stereo_solve_batch.argtypes = [ctypes.POINTER(ZdtJob), ctypes.c_int32, P]
    lib.zdt_graph_create.argtypes = [ctypes.POINTER(ZdtJob), ctypes.c_int32, P, ctypes.POINTER(ctypes.c_void_p)]
    lib.zdt_graph_launch.argtypes = [P, P]
    lib.zdt_graph_destroy.argtypes = [P]
    PL = ctypes.POINTER(ZdtPlan)
    lib.zdt_plan_candidates.argtypes = [PP, PL, ctypes.c_int]
    lib.zdt_get_plan.argtypes = [PP, PL]
    lib.zdt_set_plan.argtypes = [PP, PL]
    lib.zdt_autotune.argtypes = [PP, ctypes.c_char_p, PL, P]
    lib.zdt_i8_codec.argtypes = [P, P, P, ctypes.c_int64, P]
    F = ctypes.c_float
    lib.sgm_aggregate.argtypes = [PP, P, P, F, F, F, P]
    lib.zdt_integral_workspace_size.argtypes = [PP]
    lib.zdt_integral_workspace_size.restype = ctypes.c_size_t
    lib.zncc_window_sums_integral.argtypes = [PP, P, P, P, P, P, P, P, P]
    lib.sgm_disparity.argtypes = [PP, P, P, P, F, F, F, P]
    lib.stereo_solve_sgm.argtypes = [PP, P, P, P, P, P, F, F, F, P]
    lib.zdt_last_error.restype = ctypes.c_char_p
    lib.zdt_profile_enable.argtypes = [ctypes.c_int]
    lib.zdt_profile_entry.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for f in ("zncc_cost_volume", "dt_aggregate", "wta_disparity", "stereo_solve", "stereo_solve_static_ws",
              "stereo_solve_batch", "zdt_graph_create", "zdt_graph_launch", "zdt_graph_destroy",
              "zdt_plan_candidates", "zdt_get_plan", "zdt_set_plan", "zdt_autotune", "zncc_window_sums", "zdt_i8_codec",
              "sgm_aggregate", "sgm_disparity", "stereo_solve_sgm", "zncc_window_sums_integral", "zdt_profile_enable",
              "zdt_profile_collect",
              "zdt_profile_entry"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def params(width, height, max_disp, radius=4, sigma_s=20.0, sigma_r=0.1, dt_iters=3, vol_dtype=ZDT_F32, flags=0,
           pitch=None):
    return ZdtParams(int(width), int(height), int(pitch if pitch is not None else width), int(max_disp), int(radius),
                     float(sigma_s), float(sigma_r), int(dt_iters), int(vol_dtype), int(flags),
                     (ctypes.c_int32 * 4)(0, 0, 0, 0))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check(fn, rc):
    if rc != ZDT_OK:
        raise ZdtError(fn, rc, load().zdt_last_error().decode())


def workspace_size(p):
    return int(load().zdt_workspace_size(ctypes.byref(p)))


def volume_size(p):
    return int(load().zdt_volume_size(ctypes.byref(p)))


def zncc_cost_volume(p, left, right, cost, stream=None):
    _check("zncc_cost_volume",
           load().zncc_cost_volume(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(cost), _stream(stream)))


def dt_aggregate(p, guide, cost, stream=None):
    scale = ctypes.c_double(math.nan)
    _check("dt_aggregate",
           load().dt_aggregate(ctypes.byref(p), _ptr(guide), _ptr(cost), ctypes.byref(scale), _stream(stream)))
    return scale.value


def wta_disparity(p, cost, disp, stream=None):
    _check("wta_disparity", load().wta_disparity(ctypes.byref(p), _ptr(cost), _ptr(disp), _stream(stream)))


def stereo_solve(p, left, right, disp, vol, ws=None, stream=None):
    _check("stereo_solve", load().stereo_solve(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(disp), _ptr(vol),
                                               _ptr(ws), _stream(stream)))


def stereo_solve_static_ws(p, left, right, disp, vol, stream=None):
    _check("stereo_solve_static_ws", load().stereo_solve_static_ws(ctypes.byref(p), _ptr(left), _ptr(right),
                                                                   _ptr(disp), _ptr(vol), _stream(stream)))


STATIC_WS_BYTES = 32 << 20


def stereo_solve_batch(jobs, stream=None):
    """jobs: sequence of (params, left, right, disp, vol, ws) with device tensors (ws may be None)."""
    arr = (ZdtJob * max(1, len(jobs)))()
    for i, (p, left, right, disp, vol, ws) in enumerate(jobs):
        arr[i] = ZdtJob(p, _ptr(left), _ptr(right), _ptr(disp), _ptr(vol), _ptr(ws))
    _check("stereo_solve_batch", load().stereo_solve_batch(arr, len(jobs), _stream(stream)))


def _job_array(jobs):
    arr = (ZdtJob * len(jobs))()
    for i, (p, left, right, disp, vol, ws) in enumerate(jobs):
        arr[i] = ZdtJob(p, _ptr(left), _ptr(right), _ptr(disp), _ptr(vol), _ptr(ws))
    return arr


class Graph:
    """stereo_solve_batch(jobs) captured by the library into a HIP graph
    (zdt_graph_create); launch() replays it on a stream.  The jobs' tensors
    must stay alive as long as the graph."""

    def __init__(self, jobs, stream):
        self._jobs = list(jobs)
        h = ctypes.c_void_p()
        _check("zdt_graph_create", load().zdt_graph_create(_job_array(self._jobs), len(self._jobs),
                                                            _stream(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check("zdt_graph_launch", load().zdt_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            _check("zdt_graph_destroy", load().zdt_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_candidates(p):
    """Every tile plan (h_lanes, h_seg, v_lanes, v_seg) that fits the shape, the default first."""
    lib = load()
    n = lib.zdt_plan_candidates(ctypes.byref(p), None, 0)
    if n < 0:
        _check("zdt_plan_candidates", n)
    out = (ZdtPlan * n)()
    n = lib.zdt_plan_candidates(ctypes.byref(p), out, n)
    return [out[i].astuple() for i in range(n)]


def get_plan(p):
    out = ZdtPlan()
    _check("zdt_get_plan", load().zdt_get_plan(ctypes.byref(p), ctypes.byref(out)))
    return out.astuple()


def set_plan(p, plan):
    """Pin plan = (h_lanes, h_seg, v_lanes, v_seg) for p's shape; None restores the default."""
    pl = None if plan is None else ctypes.byref(ZdtPlan(*plan))
    _check("zdt_set_plan", load().zdt_set_plan(ctypes.byref(p), pl))


def autotune(p, cache_path=None, stream=None):
    out = ZdtPlan()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check("zdt_autotune", load().zdt_autotune(ctypes.byref(p), path, ctypes.byref(out), _stream(stream)))
    return out.astuple()


def i8_codec(values, codes, decoded, stream=None):
    """Device test entry of the 8-bit code: codes = encode(values), decoded = decode(codes)."""
    _check("zdt_i8_codec", load().zdt_i8_codec(_ptr(values), _ptr(codes), _ptr(decoded), values.numel(),
                                              _stream(stream)))


def zncc_window_sums(p, left, right, s_l=None, s_ll=None, s_t=None, s_tt=None, s_rt=None, stream=None):
    _check("zncc_window_sums",
           load().zncc_window_sums(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(s_l), _ptr(s_ll), _ptr(s_t),
                                   _ptr(s_tt), _ptr(s_rt), _stream(stream)))


def profile_enable(on):
    _check("zdt_profile_enable", load().zdt_profile_enable(int(bool(on))))


def profile_collect():
    """{kernel name: (total ms, launches)} for the launches recorded since profile_enable(True)."""
    lib = load()
    n = lib.zdt_profile_collect()
    if n < 0:
        _check("zdt_profile_collect", n)
    out = {}
    for i in range(n):
        name, ms, cnt = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_int64()
        _check("zdt_profile_entry", lib.zdt_profile_entry(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt)))
        out[name.value.decode()] = (ms.value, cnt.value)
    return out


def sgm_aggregate(p, cost, out_sum, p1, p2, cost_scale, stream=None):
    """Four-path SGM of an [H][W][D] cost volume (FP32 or FP16, p.vol_dtype) into the FP32 out_sum."""
    _check("sgm_aggregate", load().sgm_aggregate(ctypes.byref(p), _ptr(cost), _ptr(out_sum), float(p1), float(p2),
                                                 float(cost_scale), _stream(stream)))


def sgm_disparity(p, cost, out_sum, disp, p1, p2, cost_scale, stream=None):
    """Four-path SGM of a cost volume (FP32 or FP16) and its WTA into disp (out_sum: FP32 working memory)."""
    _check("sgm_disparity", load().sgm_disparity(ctypes.byref(p), _ptr(cost), _ptr(out_sum), _ptr(disp), float(p1),
                                                 float(p2), float(cost_scale), _stream(stream)))


def stereo_solve_sgm(p, left, right, disp, cost, out_sum, p1, p2, cost_scale, stream=None):
    """ZNCC cost, four-path SGM and WTA for one pair (the paper's system S1)."""
    _check("stereo_solve_sgm", load().stereo_solve_sgm(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(disp),
                                                       _ptr(cost), _ptr(out_sum), float(p1), float(p2),
                                                       float(cost_scale), _stream(stream)))


def integral_workspace_size(p):
    return load().zdt_integral_workspace_size(ctypes.byref(p))


def zncc_window_sums_integral(p, left, right, s_l=None, s_ll=None, s_t=None, s_tt=None, ws=None, stream=None):
    """Window sums by integral images (the paper's Method 2); allocates the workspace if none is given."""
    if ws is None:
        import torch
        ws = torch.empty(integral_workspace_size(p), dtype=torch.uint8, device=left.device)
    _check("zncc_window_sums_integral",
           load().zncc_window_sums_integral(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(s_l), _ptr(s_ll),
                                            _ptr(s_t), _ptr(s_tt), _ptr(ws), _stream(stream)))
