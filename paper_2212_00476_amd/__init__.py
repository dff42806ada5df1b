"""MI355X-native ZNCC + domain-transform + WTA stereo matching.

The compute path is the HIP library ``libzdt.so`` (C ABI: ``include/zdt.h``);
this package is its thin Python binding plus the seeded scene generator used by
the tests and the benchmark.  PyTorch provides device memory and streams only.

    import torch, paper_2212_00476_amd as zdt
    p = zdt.params(1280, 384, 128, radius=4, sigma_s=20, sigma_r=0.1, dt_iters=3)
    solver = zdt.Solver(p)
    disp = solver(left_u8_cuda, right_u8_cuda)      # int32 [H][W] on the device
"""
from __future__ import annotations

from ._lib import (ZDT_BF16, ZDT_F16, ZDT_F32, ZDT_FLAG_GUIDE_TARGET, ZDT_FLAG_NORMALIZE, ZDT_I8, ZDT_I16, ZdtError,
                   Graph,
                   ZdtParams, autotune, dt_aggregate, get_plan, i8_codec, load, params, plan_candidates,
                   profile_collect, profile_enable,
                   set_plan, sgm_aggregate, sgm_disparity, stereo_solve, stereo_solve_batch, stereo_solve_sgm,
                   stereo_solve_static_ws, STATIC_WS_BYTES,
                   volume_size, workspace_size, wta_disparity,
                   zncc_cost_volume, zncc_window_sums, zncc_window_sums_integral, integral_workspace_size)

__all__ = ["ZDT_F32", "ZDT_F16", "ZDT_BF16", "ZDT_I16", "ZDT_I8", "ZDT_FLAG_NORMALIZE", "ZDT_FLAG_GUIDE_TARGET",
           "ZdtError", "ZdtParams", "Graph", "i8_codec",
           "params", "load", "zncc_cost_volume", "dt_aggregate", "wta_disparity", "stereo_solve",
           "stereo_solve_static_ws", "STATIC_WS_BYTES",
           "stereo_solve_batch", "sgm_aggregate", "sgm_disparity", "stereo_solve_sgm",
           "plan_candidates", "get_plan", "set_plan", "autotune", "zncc_window_sums",
           "zncc_window_sums_integral", "integral_workspace_size", "workspace_size", "volume_size", "profile_enable",
           "profile_collect", "torch_dtype", "Solver"]


def torch_dtype(vol_dtype):
    import torch
    return {ZDT_F32: torch.float32, ZDT_F16: torch.float16, ZDT_BF16: torch.bfloat16, ZDT_I16: torch.int16,
            ZDT_I8: torch.uint8}[vol_dtype]


class Solver:
    """One pair shape: owns the working volume and workspace on the device."""

    def __init__(self, p, device="cuda"):
        import torch
        load()
        self.p = p
        self.device = torch.device(device)
        self.vol = torch.empty((p.height, p.width, p.max_disp), dtype=torch_dtype(p.vol_dtype), device=self.device)
        ws = workspace_size(p)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=self.device) if ws else None

    def __call__(self, left, right, disp=None, stream=None):
        import torch
        if disp is None:
            disp = torch.empty((self.p.height, self.p.width), dtype=torch.int32, device=self.device)
        stereo_solve(self.p, left, right, disp, self.vol, self.ws, stream)
        return disp
