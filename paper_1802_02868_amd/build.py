"""Build the HIP library libdugks2p.so for gfx950 (in-tree).

Two translation units, compiled in parallel and linked into one library:
  csrc/dugks2p.hip      the runtime and every exact kernel, -ffp-contract=off
                        (FP64 in a fixed order without FMA contraction, so the
                        fused, staged and batched forms are reproducible bit
                        for bit);
  csrc/dugks2p_fma.hip  the fused step again with -ffp-contract=fast
                        (DUGKS2P_KERNEL_FUSED_FMA), in its own namespace.
Packed FP32 instructions are disabled in both.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdugks2p.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fno-fast-math",
          "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]
UNITS = [("dugks2p.hip", ["-ffp-contract=off"]),
         ("dugks2p_fma.hip", ["-ffp-contract=fast"])]


def build(verbose: bool = False, out: str = LIB, objdir: str = OBJ) -> str:
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src, flags in UNITS:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + COMMON + flags + ["-I", os.path.join(ROOT, "include"), "-c", "-o",
                                          obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd))
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = "%s.tmp%d" % (out, os.getpid())
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
