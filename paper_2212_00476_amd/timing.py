"""Time ``stereo_solve`` on one of the named synthetic workloads.

    python -m paper_2212_00476_amd.timing planes_1920x1080_d256 --dtype f32 --dtype f16 --steps 10

Prints one line per volume type: milliseconds per pair (wall clock over
`steps` solves after `warmup` untimed ones, default plan, 9x9 window, three
sweeps) and each kernel's average time from HIP events that the library
records on its launch stream.  sgm_f32 / sgm_f16 time the paper's system S1
instead (ZNCC costs of that type, four-path SGM with P1 = 18, P2 = 185 on
costs times 21, WTA).  Inputs stay resident on the device; nothing
is checked (the tests do that).  Also serves as the program to run under
rocprofv3 for a per-kernel summary of a workload.
"""
from __future__ import annotations

import argparse
import time

DTYPES = ("f32", "f16", "bf16", "i16", "i8", "sgm_f32", "sgm_f16")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload", help="planes_1280x384_d128, planes_1920x1080_d256, planes_640x192_d64, ...")
    ap.add_argument("--dtype", action="append", choices=DTYPES, help="volume type (repeatable; default f32)")
    ap.add_argument("--radius", type=int, default=4)
    ap.add_argument("--plan", action="append", default=[],
                    help="dtype:h_lanes,h_seg,v_lanes,v_seg -- pin a tile plan for that volume type (repeatable)")
    ap.add_argument("--sigma-s", type=float, default=20.0)
    ap.add_argument("--sigma-r", type=float, default=0.1)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy three times (reference for byte counters)")
    args = ap.parse_args(argv)

    import torch

    from . import (ZDT_BF16, ZDT_F16, ZDT_F32, ZDT_I8, ZDT_I16, Solver, params, profile_collect, profile_enable,
                   set_plan, stereo_solve_sgm, torch_dtype)
    from . import scenes

    codes = {"f32": ZDT_F32, "f16": ZDT_F16, "bf16": ZDT_BF16, "i16": ZDT_I16, "i8": ZDT_I8}
    pr = scenes.workload(args.workload)
    H, W = pr.left.shape
    D = int(args.workload.rsplit("_d", 1)[1])
    left, right = torch.from_numpy(pr.left).cuda(), torch.from_numpy(pr.right).cuda()
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    plans = {k: tuple(int(v) for v in p.split(",")) for k, p in (x.split(":") for x in args.plan)}
    for name in args.dtype or ["f32"]:
        if name.startswith("sgm_"):
            ct = codes[name[4:]]
            p = params(W, H, D, args.radius, vol_dtype=ct)
            cost = torch.empty((H, W, D), dtype=torch_dtype(ct), device="cuda")
            sums = torch.empty((H, W, D), dtype=torch.float32, device="cuda")
            disp = torch.empty((H, W), dtype=torch.int32, device="cuda")

            def solver(left, right, p=p, cost=cost, sums=sums, disp=disp):
                stereo_solve_sgm(p, left, right, disp, cost, sums, 18.0, 185.0, 21.0)
        else:
            p = params(W, H, D, args.radius, args.sigma_s, args.sigma_r, args.iters, vol_dtype=codes[name])
            if name in plans:
                set_plan(p, plans[name])
            solver = Solver(p)
        for _ in range(args.warmup):
            solver(left, right)
        torch.cuda.synchronize()
        profile_enable(True)
        t = time.perf_counter()
        for _ in range(args.steps):
            solver(left, right)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / args.steps * 1e3
        profile_enable(False)
        kernels = {k: round(1e3 * v / n, 1) for k, (v, n) in profile_collect().items()}
        plan = f" plan {plans[name]}" if name in plans else ""
        print(f"{args.workload} {name}{plan}: {ms:.3f} ms per pair; kernel avg us {kernels}", flush=True)
        del solver
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
