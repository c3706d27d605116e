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
SOURCES = ("k_plain.hip", "k_regroup.hip", "k_final.hip", "k_check.hip", "runtime.hip", "sched.hip",
           "serve.hip", "noalloc.hip", "k_wave.hip")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # no packed-FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# The production (no-diagnostics) transport kernels, checked for private
# scratch: with and without the refinement code, k_plain<false, REF>,
# k_phase<false, PHOTONS, REF>, and k_wave<false, REF, GTAB> for both table
# placements.  Every name must be found in the build.
HOT_KERNELS = ("_ZN3mcd7k_plainILb0ELb0EEEvNS_6KPlainE", "_ZN3mcd7k_plainILb0ELb1EEEvNS_6KPlainE",
               "_ZN3mcd7k_phaseILb0ELb0ELb0EEEvNS_6KPhaseE", "_ZN3mcd7k_phaseILb0ELb0ELb1EEEvNS_6KPhaseE",
               "_ZN3mcd7k_phaseILb0ELb1ELb0EEEvNS_6KPhaseE", "_ZN3mcd7k_phaseILb0ELb1ELb1EEEvNS_6KPhaseE",
               "_ZN3mcd6k_waveILb0ELb0ELb0EEEvNS_6KPhaseE", "_ZN3mcd6k_waveILb0ELb1ELb0EEEvNS_6KPhaseE",
               "_ZN3mcd6k_waveILb0ELb0ELb1EEEvNS_6KPhaseE", "_ZN3mcd6k_waveILb0ELb1ELb1EEEvNS_6KPhaseE")


def resource_usage(asm: str) -> dict:
    """Per-kernel register and scratch figures from the code-object metadata
    at the end of the device assembly."""
    out, cur = {}, None
    keys = {"private_segment_fixed_size": "ScratchSize", "sgpr_count": "SGPRs",
            "sgpr_spill_count": "SGPRsSpill", "vgpr_count": "VGPRs", "vgpr_spill_count": "VGPRsSpill"}
    for line in asm.splitlines():
        m = re.match(r"\s+\.name:\s+(\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.match(r"\s+\.(\w+):\s+(\d+)\s*$", line)
        if m and cur is not None and m.group(1) in keys:
            cur[keys[m.group(1)]] = int(m.group(2))
    return out


def scratch_instructions(asm: str) -> dict:
    """Private-memory instructions (scratch_*, buffer_*) per kernel in device assembly."""
    out, cur = {}, None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            cur = m.group(1)
            out.setdefault(cur, 0)
            continue
        if cur and re.match(r"\s+(scratch|buffer)_(load|store)", line):
            out[cur] += 1
    return out


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    """Compiles every HIP source and links the shared library; returns its path."""
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    found = set()

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, "-save-temps=obj",
               "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True, cwd=objdir)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        asm_path = os.path.join(objdir, src.replace(".hip", "") + "-hip-amdgcn-amd-amdhsa-gfx950.s")
        with open(asm_path) as f:
            asm = f.read()
        usage = resource_usage(asm)
        priv = scratch_instructions(asm)
        found.update(k for k in HOT_KERNELS if k in usage)
        if verbose:
            for k, v in usage.items():
                print(k, v, "scratch instructions:", priv.get(k, 0), file=sys.stderr)
        for name in HOT_KERNELS:
            # the production transport kernels must keep their state in registers:
            # private-memory traffic in the step loop costs several times the
            # runtime (a frame the compiler reserves but never touches is harmless)
            if priv.get(name, 0) > 0:
                raise RuntimeError(f"{name} has {priv[name]} private-memory instructions "
                                   f"({usage.get(name, {}).get('ScratchSize', 0)} bytes/lane)")
        return obj

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    missing = set(HOT_KERNELS) - found
    if missing:
        raise RuntimeError(f"production kernels not in the build: {sorted(missing)}")
    tmp = LIB + ".tmp"
    r = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
