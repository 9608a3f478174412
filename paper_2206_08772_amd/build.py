"""Build libotm.so (HIP, gfx950) in the package directory.

    python -m paper_2206_08772_amd.build
"""
from __future__ import annotations

import concurrent.futures
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libotm.so")
SOURCES = ["api.hip", "search.hip", "lme.hip", "mp_update.hip", "scatter.hip", "adjoint.hip",
           "erode.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed-FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def kernel_resources(remarks):
    """{kernel: {"VGPRs": n, "AGPRs": n, "VGPRs Spill": n, "ScratchSize": n}}
    from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: (.*?) \[-Rpass-analysis", line)
        if not m:
            continue
        t = m.group(1).strip()
        if t.startswith("Function Name:"):
            cur = t.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None:
            k = re.match(r"(VGPRs|AGPRs|VGPRs Spill|ScratchSize)( \[bytes/lane\])?: (\d+)$", t)
            if k:
                out[cur][k.group(1)] = int(k.group(3))
    return out


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    # Every kernel must fit its live values in architectural VGPRs: spills
    # (to AGPRs or scratch) inside divergent code have been placed ahead of
    # the exec-mask restore by the compiler, corrupting the lanes that
    # skipped the branch.  Refuse such a build instead of running it.
    bad = {k: v for k, v in kernel_resources(r.stderr).items()
           if v.get("AGPRs", 0) > 0 or v.get("VGPRs Spill", 0) > 0 or v.get("ScratchSize", 0) > 0}
    if bad:
        raise RuntimeError(f"{src}: kernels spill registers (AGPR or scratch): {bad}")
    return obj


def build_library(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build_library(verbose=True)
    sys.exit(0)
