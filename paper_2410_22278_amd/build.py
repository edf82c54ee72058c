"""Builds libpbcjk.so (HIP for gfx950) in-tree.

Each source is compiled to an object in parallel, then linked.  Flags:
  --offload-arch=gfx950            MI355X only
  -munsafe-fp-atomics              hardware FP64 atomic add
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                   no packed FP32 instructions
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpbcjk.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["sr_slice_dp.hip", "sr_slice.hip", "sr_jk.hip", "sr_coop.hip", "sr_j.hip", "setup.cpp", "nbr.hip", "lr.hip",
           "one_e.hip", "becke.hip", "api.hip", "server.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{INCLUDE}", f"-I{CSRC}"]
HIP_FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _deps_mtime(src: str) -> float:
    """Newest modification time of a source and every header it may include."""
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in [os.path.join(CSRC, src)] + hdrs + [os.path.abspath(__file__)])


def _compile(src: str, with_d: bool, force: bool = True) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    stamp = obj + (".d1" if with_d else ".d0")
    if not force and os.path.exists(obj) and os.path.exists(stamp) and os.path.getmtime(obj) >= _deps_mtime(src):
        return obj
    cmd = [HIPCC] + COMMON + HIP_FLAGS + [f"-DPBCJK_WITH_D={1 if with_d else 0}",
                                          "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    for other in (".d0", ".d1"):
        if os.path.exists(obj + other):
            os.remove(obj + other)
    open(stamp, "w").close()
    return obj


def build(with_d: bool = True, verbose: bool = False, force: bool = True) -> str:
    """Compiles every source (force) or only those older than their
    dependencies, then links libpbcjk.so."""
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, with_d, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(with_d="--no-d" not in sys.argv, verbose=True, force="--incremental" not in sys.argv)
