"""Build libstag.so (HIP, gfx950) in-tree.

    python paper_1010_5433_amd/build.py

Every HIP source under csrc/ is compiled for gfx950 with hipcc and linked
into paper_1010_5433_amd/libstag.so.  Packed FP32 instructions are turned
off for all device code (-packed-fp32-ops).

The sources whose kernels have committed byte counters (ASM_SOURCES) are
also compiled to device assembly, and the instructions of every kernel are
hashed into libstag.kernels.json beside the library: a counter summary is
only valid for the build whose kernel hash it names.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstag.so")
KERNEL_HASHES = os.path.join(HERE, "libstag.kernels.json")
ASM_SOURCES = ["dslash.hip", "force.hip", "bdslash.hip", "rhmc.hip"]
ARCH = os.environ.get("STAG_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]
# roctx, for the named ranges of the solver phases in rocprofv3's marker trace
ROCM_LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(HIPCC))), "lib")
LDFLAGS = [f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-c", src, "-o", obj] + CFLAGS + list(extra)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _kernel_hashes(src: str, extra) -> dict:
    """Demangled kernel name -> hash of its instructions (comments dropped,
    block labels numbered within the function only)."""
    asm = os.path.join(BUILD, os.path.basename(src) + ".s")
    cmd = [HIPCC, "--cuda-device-only", "-S", src, "-o", asm] + CFLAGS + list(extra)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"device assembly failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    out, name, body = {}, None, []
    for line in open(asm):
        m = re.match(r"\s*\.type\s+(\S+),@function", line)
        if m:
            name, body = m.group(1), []
            continue
        if name is None:
            continue
        if line.startswith(".Lfunc_end"):
            out[name] = hashlib.sha256("".join(body).encode()).hexdigest()[:16]
            name = None
            continue
        text = line.split(";", 1)[0].strip()
        if text:
            # block labels carry the function's position in the file: drop it
            body.append(re.sub(r"\.LBB\d+_", ".LBB_", text) + "\n")
    if not out:
        return {}
    dem = subprocess.run(["c++filt"], input="\n".join(out), capture_output=True, text=True, check=True)
    return dict(zip(dem.stdout.split("\n"), out.values()))


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    asm_srcs = [os.path.join(CSRC, f) for f in ASM_SOURCES if os.path.exists(os.path.join(CSRC, f))]
    with cf.ThreadPoolExecutor(jobs) as ex:
        hashes = ex.map(lambda s: _kernel_hashes(s, extra), asm_srcs)
        objs = list(ex.map(lambda s: _compile(s, extra), srcs))
        kernels = {}
        for h in hashes:
            kernels.update(h)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + LDFLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    with open(KERNEL_HASHES + ".tmp", "w") as fh:
        json.dump(kernels, fh, indent=0, sort_keys=True)
    os.replace(KERNEL_HASHES + ".tmp", KERNEL_HASHES)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
