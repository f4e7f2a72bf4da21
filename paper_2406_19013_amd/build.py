"""Build libxcorr.so (HIP kernels + C ABI) for gfx950 with hipcc.

    python -m paper_2406_19013_amd.build [--verbose] [--changed]

Every call compiles every unit (--changed: only units whose object is older
than a source or header, for editing sessions); the library is written next
to this file.  The
compiler's per-kernel resource report (registers, scratch, occupancy, LDS) is
written to _build/kernel_resources.txt; a kernel that spills registers to
scratch is named on stderr.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libxcorr.so")
ARCH = "gfx950"

# (source, extra flags, object name).  The 8+8-bit and the three-product
# 4+4-bit MFMA kernels are compiled once per diagonal block size so that the
# objects build in parallel.
UNITS = [("xcorr_kernels.hip", [], "xcorr_kernels.o"), ("xcorr_api.cpp", [], "xcorr_api.o"),
         ("xcorr_pipe.cpp", [], "xcorr_pipe.o"), ("xcorr_reorder.cpp", [], "xcorr_reorder.o"), ("xcorr_cns.cpp", [], "xcorr_cns.o"),
         ("xcorr_mfma4.hip", [], "xcorr_mfma4.o"), ("xcorr_mfma4f.hip", [], "xcorr_mfma4f.o"),
         ("xcorr_batch.hip", [], "xcorr_batch.o"),
         ("xcorr_gauss4.hip", [], "xcorr_gauss4.o"), ("xcorr_gauss4_batch.hip", [], "xcorr_gauss4_batch.o"),
         ("xcorr_static.hip", [], "xcorr_static.o"),
         ("xcorr_ceiling.hip", [], "xcorr_ceiling.o"),
         ("xcorr_fengine.hip", [], "xcorr_fengine.o"),
         ("xcorr_stokes.hip", [], "xcorr_stokes.o")] + [
    ("xcorr_mfma8.hip", [f"-DXC_D={d}"], f"xcorr_mfma8_d{d}.o") for d in range(1, 7)] + [
    ("xcorr_gauss4.hip", [f"-DXC_G3_D={d}"], f"xcorr_gauss4_d{d}.o") for d in range(1, 7)]
RESOURCES = "kernel_resources.txt"

# Packed FP32 VALU ops are disabled for every device compile.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]"
                     r"|LDS Size \[bytes/block\]): (\S+)")


def _run(cmd, verbose):
    """Run one compiler step; return its kernel resource remarks as
    [(kernel, {field: value})]."""
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    kernels, rest = [], []
    for line in r.stdout.splitlines():
        m = _REMARK.search(line)
        if m:
            if m.group(1) == "Function Name":
                kernels.append((m.group(2), {}))
            elif kernels:
                kernels[-1][1][m.group(1).split(" ")[0]] = m.group(2)
        elif "packed-fp32-ops" not in line and "kernel-resource-usage" not in line:
            rest.append(line)
    out = "\n".join(rest)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}):\n{' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)
    return kernels


def read_resources(path: str | None = None) -> dict:
    """{kernel symbol: {"VGPRs", "AGPRs", "ScratchSize", "Occupancy", "LDS": int}}
    from the report of the last build."""
    path = path or os.path.join(HERE, "_build", RESOURCES)
    res = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2 and not line.startswith("#"):
                res[parts[0]] = {k: int(v) for k, v in (f.split("=") for f in parts[1:])}
    return res


def _stale(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")] + \
        [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE) if h.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, jobs: int | None = None, changed_only: bool = False) -> str:
    cc = hipcc()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, o) for _, _, o in UNITS]
    cmds = [[cc, *COMMON, *flags, "-Rpass-analysis=kernel-resource-usage", "-c",
             os.path.join(CSRC, src), "-o", obj]
            for (src, flags, _), obj in zip(UNITS, objs)
            if not changed_only or _stale(obj, src)]
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max(1, jobs)) as ex:
        reports = list(ex.map(lambda c: _run(c, verbose), cmds))
    # per-unit resource reports, merged into one file
    for c, kernels in zip(cmds, reports):
        with open(c[-1] + ".res", "w") as fh:
            for name, f in kernels:
                fh.write(name + " " + " ".join(f"{k}={v}" for k, v in f.items()) + "\n")
    with open(os.path.join(bdir, RESOURCES), "w") as fh:
        fh.write("# kernel VGPRs AGPRs ScratchSize(bytes/lane) Occupancy(waves/SIMD) LDS(bytes)\n")
        for obj in objs:
            kernels = []
            if os.path.exists(obj + ".res"):
                for line in open(obj + ".res"):
                    parts = line.split()
                    if parts:
                        kernels.append((parts[0], dict(p.split("=", 1) for p in parts[1:])))
            for name, f in kernels:
                fields = " ".join(f"{k}={f[k]}" for k in ("VGPRs", "AGPRs", "ScratchSize", "Occupancy", "LDS")
                                  if k in f)
                fh.write(f"{name} {fields}\n")
                if int(f.get("ScratchSize", "0")):
                    print(f"build: kernel {name} spills {f['ScratchSize']} bytes/lane to scratch",
                          file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv, changed_only="--changed" in sys.argv))
