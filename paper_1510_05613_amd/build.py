"""Builds libperch.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libperch.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the float32 vertex stage is part of the rasterisation rule.
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
                "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature",
                "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]
# The network's kernels keep MFMA accumulators in ordinary VGPRs, so the bias can
# seed the accumulation and the epilogue reads the results without AGPR moves.
CNN_FLAGS = DEVICE_FLAGS + ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
# roctx ranges (search expansions, parent materialisation, successor launches) for
# rocprofv3 --marker-trace
LINK_FLAGS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
# host-only sources still go through hipcc: pin the offload target to gfx950 too
HOST_FLAGS = ["--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = (("perch_kernels.hip", DEVICE_FLAGS), ("perch_cnn.hip", CNN_FLAGS),
             ("perch_select.hip", DEVICE_FLAGS), ("perch_noalloc.hip", DEVICE_FLAGS),
             ("perch_posenet.hip", DEVICE_FLAGS), ("perch_posenet_api.cpp", HOST_FLAGS),
             ("perch_cnn_api.cpp", HOST_FLAGS), ("perch_api.cpp", HOST_FLAGS),
             ("perch_search.cpp", HOST_FLAGS), ("perch_batch.cpp", HOST_FLAGS),
             ("perch_tune.cpp", HOST_FLAGS))
    cmds, objs = [], []
    for src, flags in units:
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        cmds.append([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # one compiler process per source file, at most `jobs` at a time
    n = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=n) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, *LINK_FLAGS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
