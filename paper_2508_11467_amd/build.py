"""Builds libbdc.so (the HIP kernels and the C ABI) in place for gfx950."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbdc.so")

ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the deflation decisions must be reproducible bit for bit: no contraction
SOURCES = {
    "k_leaf.hip": [],
    "k_deflate.hip": ["-ffp-contract=off"],
    "k_secular.hip": [],
    "k_update.hip": [],
    "k_mlp.hip": [],
    "k_ozaki.hip": [],
    "k_crt.hip": [],
    "k_backtr.hip": [],
    "k_qr.hip": [],
    "k_gebrd.hip": [],
    "plan.cpp": [],
    "api.cpp": [],
    "api_steps.cpp": [],
}


def source_hash(files=None) -> str:
    """SHA-256 of the kernel and ABI sources (identifies a build's kernels);
    with `files` (names under csrc/), of those files and the shared device
    header only (identifies the kernels a measurement was taken of)."""
    import hashlib
    h = hashlib.sha256()
    if files:
        paths = [os.path.join(CSRC, f) for f in sorted(set(files) | {"bdc_internal.h"})]
    else:
        paths = [os.path.join(d, name) for d in (CSRC, INCLUDE) for name in sorted(os.listdir(d))
                 if name.endswith((".hip", ".h", ".cpp"))]
    for path in paths:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_sources(names) -> list:
    """The csrc/*.hip files that define the named kernels."""
    out = set()
    for fn in sorted(os.listdir(CSRC)):
        if fn.endswith(".hip"):
            text = open(os.path.join(CSRC, fn)).read()
            out.update(fn for k in names if f"void {k}(" in text)
    return sorted(out)


def rocm() -> str:
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc() -> str:
    for c in (os.path.join(rocm(), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        host = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm(), "include")]
        flags = COMMON + extra + (DEVICE if src.endswith(".hip") else host)
        cmd = [cc] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 feature: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if p.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        print(r.stdout.decode(errors="replace"), file=sys.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
