"""Build libctd.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libctd.so")
SOURCES = ["cfe1d.cpp", "fdiag.cpp", "kernels.hip", "actd.hip", "solver.hip", "batch.hip", "serve.hip", "noalloc.hip", "wsep.hip"]
ARCH = os.environ.get("CTD_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 VALU ops are kept off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.isabs(cand) and os.path.exists(cand):
            return cand
    return "hipcc"


# the compiler's per-kernel resource report (registers, scratch, LDS,
# occupancy), taken from the same compile and kept beside the library
RESOURCE_FLAG = "-Rpass-analysis=kernel-resource-usage"
RESOURCE_REPORT = os.path.join(HERE, "_build", "kernel_resources.txt")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON]
    if src.endswith(".hip"):
        cmd += [RESOURCE_FLAG]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr


def kernel_resources(text: str) -> dict:
    """Per-kernel fields of the compiler's resource remarks:
    {mangled name: {"VGPRs": .., "ScratchSize [bytes/lane]": .., ...}}."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark:\s+(.*?)\s*\[-Rpass-analysis=kernel-resource-usage\]", line)
        if not m:
            continue
        field = m.group(1)
        if field.startswith("Function Name:"):
            cur = field.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None and ":" in field:
            k, v = field.rsplit(":", 1)
            out[cur][k.strip()] = v.strip()
    return out


def _remarks_only(out: str) -> str:
    keep = []
    for l in out.splitlines():
        if "packed-fp32-ops" in l or "kernel-resource-usage" in l:
            continue
        keep.append(l)
    return "\n".join(keep)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    failed = [r for r in results if r[2] != 0]
    for src, _, rc, out in results:
        if verbose or rc != 0:
            msg = _remarks_only(out)
            if msg.strip():
                print(f"[{src}]\n{msg}", file=sys.stderr)
    if failed:
        raise RuntimeError("HIP compile failed: " + ", ".join(f[0] for f in failed))
    # no kernel may use scratch memory: a copy of a by-value argument, a
    # register spill or an outlined call shows up there first
    res = {}
    for src, _, _, out in results:
        res.update(kernel_resources(out))
    with open(RESOURCE_REPORT, "w") as f:
        for name in sorted(res):
            f.write(name + "\t" + "\t".join(f"{k}={v}" for k, v in res[name].items()) + "\n")
    scratch = sorted(n for n, r in res.items() if r.get("ScratchSize [bytes/lane]", "0") != "0")
    if scratch:
        raise RuntimeError("kernels using scratch memory: " + ", ".join(scratch))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[r[1] for r in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
