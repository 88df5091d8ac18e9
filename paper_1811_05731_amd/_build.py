"""Compile the HIP/C++ sources into paper_1811_05731_amd/libh2dlp.so (gfx950).

Run as ``python -m paper_1811_05731_amd._build``; called by the repository's
build entry point.  Host structure code is compiled without floating-point
contraction so that cluster splits and admissibility are reproducible.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libh2dlp.so")

ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="h2dlp_build_")
    try:
        objs = []
        jobs = []
        for src, extra in (("structure.cpp", ["-ffp-contract=off", "-x", "c++"]),
                           ("api.cpp", ["-x", "c++"]),
                           ("build_kernels.hip", []),
                           ("apply_kernels.hip", []),
                           ("recompress.hip", []),
                           ("noalloc.hip", []),
                           ("fem.cpp", ["-x", "c++"]),
                           ("fem_kernels.hip", [])):
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
            if src.endswith(".cpp"):
                cmd = [c for c in cmd if not c.startswith("--offload-arch")]
                cmd += ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
                cmd = [c for c in cmd if c not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
            jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
            objs.append(obj)
        for j, o in zip(jobs, objs):
            out, _ = j.communicate()
            if j.returncode != 0:
                raise RuntimeError(f"compiling {os.path.basename(o)} failed:\n{out}")
            if verbose and out.strip():
                print(out)
        tmp_lib = LIB + ".tmp"
        _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp_lib, *objs,
              "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"])
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
