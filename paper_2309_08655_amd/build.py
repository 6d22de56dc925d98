"""Build the gfx950 HIP library librt.so in-tree with hipcc."""
from __future__ import annotations

import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librt.so")
SOURCES = ["rt_api.hip", "rt_forward.hip", "rt_backward.hip", "rt_batched.hip", "rt_adjoint.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Per-file additions.  With -ffp-contract=on, multiply-adds are fused only within one
# source expression, decided by the front end, never by the backend across the inlined
# context, so every copy of the step code produces the same bits: the adjoint's recompute
# replays its forward pass's accept/reject decisions exactly, and the tracing kernels
# specialised at compile time for one plasma, density and rotation round exactly like the
# generic ones (results do not depend on the schedule).
# The kernels also keep the backend's loop-invariant code motion off.  Hoisting FP64 constants
# and invariant products out of their nested loops (rays, segments, steps, stages) kept them
# live across the whole kernel, and the kernels that run short of registers spilled them: the
# adjoint's reverse kernel, at one wave per SIMD, 547 spilled registers (56 without; its phase
# of the 1e6-ray gradient 75 ms -> 40 ms), and the generic tracing kernel 34-142 (0-6 without;
# the GR-dipole variant 17.1 -> 13.8 ms per step).  The specialised tracing kernels, which did
# not spill, time the same either way.  It moves instructions only, not arithmetic.
NO_MLICM = ["-mllvm", "-disable-machine-licm"]
FILE_FLAGS = {"rt_adjoint.hip": ["-ffp-contract=on", *NO_MLICM], "rt_forward.hip": ["-ffp-contract=on", *NO_MLICM],
              "rt_backward.hip": ["-ffp-contract=on", *NO_MLICM]}

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # never emit packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


FLOPS_JSON = os.path.join(HERE, "flops.json")


def build_flop_table(verbose: bool = False) -> str:
    """Compile and run the host-side operation counter of the device templates
    (csrc/flopcount.cpp) and store its table next to the library."""
    exe = os.path.join(HERE, "_flopcount.bin")
    cmd = [HIPCC, "-std=c++17", "-O1", "-o", exe, os.path.join(CSRC, "flopcount.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    json.loads(out)
    with open(FLOPS_JSON, "w") as f:
        f.write(out)
    os.remove(exe)
    return FLOPS_JSON


def build(verbose: bool = False) -> str:
    import concurrent.futures as cf
    import tempfile
    inc = os.path.join(HERE, "..", "include")
    with tempfile.TemporaryDirectory(prefix="rt_build_") as tmpdir:
        cmds, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), "-I", inc, "-c", os.path.join(CSRC, src),
                         "-o", obj])
        with cf.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            for cmd in cmds:
                if verbose:
                    print(" ".join(cmd), flush=True)
            list(ex.map(lambda c: subprocess.run(c, check=True), cmds))
        tmp = LIB + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    build_flop_table(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
