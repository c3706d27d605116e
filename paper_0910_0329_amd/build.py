"""Builds libmcdose.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmcdose.so")
SOURCES = ("k_plain.hip", "k_regroup.hip", "k_final.hip", "runtime.hip", "sched.hip", "serve.hip")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # no packed-FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Production (non-diagnostic) transport kernels: checked for private scratch.
HOT_KERNELS = ("_ZN3mcd7k_plainILb0EEEvNS_6KPlainE", "_ZN3mcd7k_phaseILb0ELb1EEEvNS_6KPhaseE",
               "_ZN3mcd7k_phaseILb0ELb0EEEvNS_6KPhaseE")


def resource_usage(remarks: str) -> dict:
    """Per-kernel register/scratch usage from hipcc's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+)", line)
        if m and cur is not None:
            cur[m.group(1).replace(" ", "")] = int(m.group(2))
    return out


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    """Compiles every HIP source and links the shared library; returns its path."""
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, "-Rpass-analysis=kernel-resource-usage", "-I", INCLUDE,
               "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        usage = resource_usage(r.stderr)
        if verbose:
            for k, v in usage.items():
                print(k, v, file=sys.stderr)
        for name, u in usage.items():
            # the production transport kernels must keep their state in registers:
            # private scratch in the step loop costs several times the runtime
            if name in HOT_KERNELS and u.get("ScratchSize", 0) > 0:
                raise RuntimeError(f"{name} uses {u['ScratchSize']} bytes/lane of private scratch")
        return obj

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    r = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
