"""Builds libcodag.so (HIP, gfx950) in the package directory."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("codag.hip", "batch.hip", "sched.hip", "split.hip", "ablation.hip", "typed.hip")]
OUT = os.path.join(HERE, "libcodag.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.stderr


def build(verbose: bool = False) -> str:
    """Compiles each source to an object (in parallel), then links the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in SOURCES]
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        logs = list(ex.map(_run, [[hipcc, *HIPCC_FLAGS, "-c", s, "-o", o]
                                  for s, o in zip(SOURCES, objs)]))
    tmp = OUT + ".tmp"
    logs.append(_run([hipcc, "--offload-arch=gfx950", "-shared", *objs, "-o", tmp]))
    if verbose:
        print("".join(logs))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
