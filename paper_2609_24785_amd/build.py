"""Build liblee.so for gfx950: the host builder with g++ (FP64, no contraction,
so set-up predicates are reproducible), the kernels and the C ABI with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblee.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-Wno-unused-value", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def _run(cmd):
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    host_o = os.path.join(OUT, "lee_host.o")
    cmds = [["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "lee_host.cpp"), "-o", host_o]]
    objs = [host_o]
    for src in ("lee_kernels.hip", "lee_api.hip"):
        o = os.path.join(OUT, src.replace(".hip", ".o"))
        cmds.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    # the three translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
        list(pool.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
