"""Build libsg.so (HIP kernels for gfx950 + host library) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = os.environ.get("CLANGXX", "/opt/rocm/llvm/bin/clang++")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# keep the compiler from forming packed fp32 instructions
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    objs = []
    jobs = []
    for src, dev in (("sg_kernels.hip", True), ("sg_host.cpp", False), ("sg_seed.cpp", False)):
        obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + ".o")
        if dev:
            cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip"]
        else:  # host-only C++ against the HIP runtime API
            cmd = [CLANGXX] + COMMON + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in jobs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed:\n{text}")
        if verbose and text.strip():
            print(text)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
