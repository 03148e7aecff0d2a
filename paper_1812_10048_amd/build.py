"""Build libdpmm.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import re
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdpmm.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["api.hip", "bookkeeping.hip", "layout.hip", "redraw.hip", "assign.hip", "assign_mfma.hip", "substats.hip",
           "laysub.hip", "splitmerge.hip", "dm.hip", "prep.hip"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled in every HIP object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    # per-kernel registers, scratch and occupancy, checked below
    "-Rpass-analysis=kernel-resource-usage",
]
RESOURCES = os.path.join(BUILD_DIR, "kernel_resources.txt")
# kernels allowed to use scratch: off the sweep's path (the log joint of
# dpmm_stats) or debug variants (the per-cell score dump, first template flag
# DUMP of the sub-cluster passes)
SCRATCH_OK = (re.compile(r"k_log_joint"), re.compile(r"k_sub_stats<\w+, \w+, true,"),
              re.compile(r"k_lay_sub<true,"), re.compile(r"k_mov_span<true,"))


def _resources(text: str) -> list[dict]:
    """Parse -Rpass-analysis=kernel-resource-usage remarks."""
    out, cur = [], None
    for line in text.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = {"name": m.group(1)}
            out.append(cur)
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]): (\d+)", line)
        if m and cur is not None:
            cur[m.group(1).split()[0]] = int(m.group(2))
    return out


def _demangle(names: list[str]) -> list[str]:
    exe = shutil.which("c++filt") or shutil.which("llvm-cxxfilt")
    if not exe or not names:
        return names
    r = subprocess.run([exe], input="\n".join(names), capture_output=True, text=True)
    got = r.stdout.splitlines()
    return got if len(got) == len(names) else names


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src: str):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, _resources(r.stderr)


def check_resources(kernels: list[dict]) -> None:
    """Write the per-kernel table and fail if a kernel on the sweep's path
    spills to scratch."""
    names = _demangle([k["name"] for k in kernels])
    rows, bad = [], []
    for k, name in zip(kernels, names):
        sc = k.get("ScratchSize", 0)
        rows.append(f"{name:<72} VGPRs {k.get('VGPRs', 0):4d} AGPRs {k.get('AGPRs', 0):4d} "
                    f"scratch {sc:4d} B/lane  waves/SIMD {k.get('Occupancy', 0)}  LDS {k.get('LDS', 0)} B")
        if sc and not any(p.search(name) for p in SCRATCH_OK):
            bad.append(name)
    with open(RESOURCES, "w") as f:
        f.write("\n".join(sorted(set(rows))) + "\n")
    if bad:
        raise RuntimeError("kernels spill to scratch: " + ", ".join(bad) + f" (see {RESOURCES})")


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libdpmm.so next to this file."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        done = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in done]
    check_resources([k for _, ks in done for k in ks])
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
