"""Compile libqsim.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_2305_14398_amd.build

Each source in csrc/ is compiled by hipcc to an object under _build/ (in
parallel), then linked into paper_2305_14398_amd/libqsim.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libqsim.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed fp32 instructions are disabled for all device code; hipcc's host pass
# warns that it does not know the feature, which is harmless.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def build_id() -> str:
    """Hash of the kernel and host sources and the public header: a tile cache records it and is only loaded
    by a library built from the same sources."""
    import hashlib
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(CSRC, "*"))) + [os.path.join(ROOT, "include", "qsim.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# Per-source extra flags.  fsv.hip: branches on uniform values (the operation
# dispatch of the full-state pass) are left unstructured, so each dispatch
# target updates the state registers in place and jumps straight to the loop
# latch; structuring them joins every target through flow blocks whose merges
# the register allocator resolves with whole-state copies.
EXTRA_FLAGS = {"fsv.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions"]}


def _compile(src: str, bid: str):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA_FLAGS.get(os.path.basename(src), []), f"-DQSIM_BUILD_ID=\"{bid}\"",
           "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # Every kernel is written to keep its working set in registers; report any
    # that the compiler sent to scratch memory (a large slowdown, never intended).
    spills, name = [], None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            spills.append(f"{name}: {m.group(1)} B/lane")
    return obj, spills


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    bid = build_id()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        done = list(ex.map(lambda s: _compile(s, bid), srcs))
    objs = [o for o, _ in done]
    spills = [x for _, sp in done for x in sp]
    if spills:
        print("warning: kernels using scratch memory:\n  " + "\n  ".join(spills), file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
