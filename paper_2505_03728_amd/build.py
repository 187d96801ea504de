"""Builds libpkmi.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpkmi.so")
SOURCES = ["pk_api.hip", "pk_debug.hip", "lm_lane.hip", "lm_lane_chain_a.hip", "lm_lane_chain_b.hip",
           "lm_lane_chain_c.hip", "lm_wave.hip", "lm_wave_d8.hip",
           "lm_wave_d16.hip", "lm_wave_d32.hip", "lm_wave_d64.hip", "lm_path.hip", "lm_path_d16.hip", "seeder.hip",
           "pipeline.hip", "sched.hip", "lm_mixed.hip", "beam.hip", "traj.hip"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 VALU ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused only within one source expression: the same device
    # function then rounds the same way in every kernel it is inlined into
    # (the mixed-batch kernel and the per-robot kernels give identical results)
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _stale(obj, src):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, f) for f in os.listdir(CSRC)
                                        if f.endswith((".hpp", ".h"))]
    deps.append(os.path.join(ROOT, "include", "pkmi.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile each source to an object (in parallel), then link.

    incremental=True recompiles only objects older than their sources or
    any header (a development shortcut; the default rebuilds everything)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and not _stale(obj, src):
            continue
        cmd = ["hipcc", "-c", *[f for f in FLAGS if f != "-shared"], os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"--- {src}\n{text}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
