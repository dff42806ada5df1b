"""Build the gfx950 HIP library ``libzdt.so`` in-tree with hipcc.

Usage: ``python -m paper_2212_00476_amd.build`` (also called by
``__graft_entry__.build()``).  The object files are compiled in parallel, one
translation unit per source in ``csrc/``.
"""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libzdt.so")
ARCH = os.environ.get("ZDT_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU forms.
# kernel-resource-usage remarks: parsed into a per-kernel report (below).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Rpass-analysis=kernel-resource-usage"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC] + DEVICE_FLAGS
# Per-source flags.  The SGM kernels take minima of values that are never NaN
# for finite costs; without NaN semantics the compiler drops the quieting of
# every operand (one extra VALU instruction per minimum on the serial path).
SOURCE_FLAGS = {"zdt_sgm.hip": ["-fno-honor-nans"]}
# Per-lane scratch above this fails the build: every kernel here keeps its
# working set in registers and LDS, so more than a few spilled words means the
# register allocation went wrong.  (One way it has gone wrong: the compiler
# promoted a kernel's per-lane value array to one wide vector value before the
# loops over it were unrolled, then copied and spilled whole vectors -- tens of
# KB of scratch per lane, more than a dispatch can be given.)
MAX_SCRATCH_BYTES = 1024
RESOURCES = os.path.join(HERE, "_build", "kernel_resources.json")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]"
                     r"|LDS Size \[bytes/block\]):\s+(\S+)")
_KEYS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch_bytes",
         "Occupancy [waves/SIMD]": "waves_per_simd", "LDS Size [bytes/block]": "static_lds_bytes"}


def parse_resources(text):
    """{kernel symbol: {vgprs, agprs, scratch_bytes, waves_per_simd, ...}} from
    the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val)
    return out


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC] + COMMON + SOURCE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        text = r.stdout + r.stderr
        msgs, held, in_remark = [], [], False
        for l in text.splitlines():
            if l.startswith("In file included from"):
                held.append(l)
                continue
            if "remark:" in l:  # drop remarks with their include chain and source context
                held, in_remark = [], True
                continue
            if in_remark and re.match(r"^\s*(\d+\s*)?\|", l):
                continue
            in_remark = False
            if "packed-fp32-ops' is not a recognized feature" not in l:
                msgs += held + [l]
            held = []
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, "\n".join(msgs)))
        if verbose and msgs:
            print("\n".join(msgs), file=sys.stderr)
        return obj, parse_resources(text)

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, sources()))
    objs = [o for o, _ in results]
    resources = {}
    for _, res in results:
        resources.update(res)
    with open(RESOURCES, "w") as f:
        json.dump(resources, f, indent=1, sort_keys=True)
    bad = {k: v for k, v in resources.items() if v.get("scratch_bytes", 0) > MAX_SCRATCH_BYTES}
    if bad:
        raise RuntimeError("kernels need more than %d B of scratch per lane: %s" % (MAX_SCRATCH_BYTES, bad))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t = __import__("time").time()
    print(build(verbose=True), "%.1fs" % (__import__("time").time() - t))
