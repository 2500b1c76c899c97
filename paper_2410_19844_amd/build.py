"""Build libsos.so (gfx950) in-tree with hipcc.

Usage: python paper_2410_19844_amd/build.py   (or __graft_entry__.build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsos.so")
SOURCES = ["kernels.hip", "gemm_bf3.hip", "gemm_x64.hip", "gemm_i8.hip", "batch.hip", "net.hip", "api.cpp", "plan.cpp"]

# -packed-fp32-ops: never emit packed FP32 VALU instructions (they have given
# silent wrong results on this hardware); hipcc's host pass warns that it does
# not know the feature, which is harmless.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-inline-asm",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: libsos needs ROCm's hipcc to build")


# the compiler's per-kernel resource report (registers, scratch, occupancy),
# kept in _build/kernel_resources.tsv; it does not change the generated code
REPORT_FLAGS = ["-Rpass-analysis=kernel-resource-usage"]
RESOURCES = os.path.join(HERE, "_build", "kernel_resources.tsv")


def parse_resources(text: str) -> list[dict]:
    """Kernels and their resource figures from hipcc's remarks."""
    out, cur = [], None
    for line in text.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = {"kernel": body.split(":", 1)[1].strip()}
            out.append(cur)
        elif cur is not None and ":" in body:
            key, val = body.rsplit(":", 1)
            cur[key.strip()] = val.strip()
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link libsos.so; returns the library path."""
    objs = []
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    cc = hipcc()
    report = []
    for src in SOURCES:
        obj = os.path.join(obj_dir, src.rsplit(".", 1)[0] + ".o")
        cmd = [cc, *HIP_FLAGS, *REPORT_FLAGS, "-I", os.path.join(HERE, "..", "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if not src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        report += [dict(r, source=src) for r in parse_resources(res.stderr)]
        objs.append(obj)
    cols = ["source", "kernel", "VGPRs", "AGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]",
            "LDS Size [bytes/block]"]
    with open(RESOURCES, "w") as f:
        f.write("\t".join(cols) + "\n")
        for r in report:
            f.write("\t".join(str(r.get(c, "")) for c in cols) + "\n")
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
