"""Build libmbamg.so (HIP, gfx950) in the package directory.

    python -m paper_2103_07537_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbamg.so")
OBJ = os.path.join(HERE, "_build")
ARCH = "gfx950"

# (source, extra flags).  The setup unit keeps every floating-point operation
# separately rounded so its sums follow the written order exactly.
UNITS = [
    ("setup_kernels.hip", ["-ffp-contract=off"]),
    ("solve_kernels.hip", []),
    ("learned_kernels.hip", []),
    ("hierarchy.hip", []),
    ("memory.hip", []),
]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # no packed FP32 instructions in any kernel
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    p = os.path.join(rocm, "bin", "hipcc")
    return p if os.path.exists(p) else "hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    procs = []
    objs = []
    for src, extra in UNITS:
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc()] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()
                 and "warning: feature flag" not in l]
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


def build_test_driver(verbose: bool = False) -> str:
    """The tests' C-ABI driver (tests/abi_driver.cpp): a plain HIP program that
    links libmbamg.so and uses include/mbamg.h only."""
    root = os.path.dirname(HERE)
    out_dir = os.path.join(root, "tests", "_build")
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "abi_driver")
    cmd = [hipcc(), "-O2", "-std=c++17", "-I", os.path.join(root, "include"),
           os.path.join(root, "tests", "abi_driver.cpp"), "-L", HERE, "-lmbamg",
           "-Wl,-rpath,$ORIGIN/../../paper_2103_07537_amd", "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if p.returncode != 0:
        print(p.stdout.decode(errors="replace"), file=sys.stderr)
        raise RuntimeError("hipcc failed for tests/abi_driver.cpp")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_test_driver(verbose=True))
