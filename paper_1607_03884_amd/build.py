"""Build step of the HIP library (hipcc, gfx950)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["rk_api.cpp", "rk_kernels.hip", "rk_group.hip", "rk_group16.hip", "rk_group64.hip", "rk_block.hip",
           "rk_mlp.hip", "rk_pred.hip", "rk_noalloc.hip", "rk_ros.hip"]
# per-source extra flags: the block kernel's elimination loops (51 register
# columns, nested) must unroll completely so every register index is constant
EXTRA_FLAGS = {"rk_block.hip": ["-mllvm", "-pragma-unroll-threshold=400000"]}
OUT = os.path.join(HERE, "librkchem.so")

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               # no packed-FP32 instructions anywhere in the device code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function"]


def build_library(verbose: bool = False, csrc: str = CSRC, out: str = OUT) -> str:
    """Compile every source to an object (in parallel), then link the shared
    library.  Objects go to _build/ next to the output."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    procs = []
    for s in SOURCES:
        obj = os.path.join(objdir, s + f".{os.getpid()}.o")
        cmd = [hipcc] + compile_flags + EXTRA_FLAGS.get(s, []) + ["-c", os.path.join(csrc, s), "-o", obj]
        procs.append((s, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    objs, errors = [], []
    for s, obj, p in procs:
        so, se = p.communicate()
        if p.returncode != 0:
            errors.append(f"{s}:\n{so}{se}")
        elif verbose and se:
            print(se)
        objs.append(obj)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = out + f".tmp{os.getpid()}"
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp],
                       capture_output=True, text=True)
    for o in objs:
        os.remove(o)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
