"""Build libtto.so (all HIP sources, gfx950 only) in-tree with hipcc.

``build(sanitize=True)`` (``python -m paper_2605_10128_amd.build --sanitize``)
writes _build/libtto_san.so instead: the host code of every source built with
AddressSanitizer and UndefinedBehaviorSanitizer (device code is unchanged;
the sanitizer flags reach only the host pass).  Load it by setting TTO_LIBRARY
to its path, with the ASan runtime preloaded into the interpreter."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtto.so")
LIB_SAN = os.path.join(BUILD, "libtto_san.so")
SOURCES = ["tto_api.hip", "k_grid.hip", "k_eval.hip", "k_archive.hip", "k_evolve.hip", "k_busbar.hip", "k_ptdf.hip", "k_mlp.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 VALU ops are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
# host pass only: each -fsanitize= follows its own -Xarch_host
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, sanitize: bool = False) -> str:
    stem = os.path.splitext(src)[0] + ("_san" if sanitize else "")
    obj = os.path.join(BUILD, stem + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, sanitize: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), SOURCES))
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    # a shared library does not carry the sanitizer runtimes: the host process
    # preloads the ASan runtime (which also holds the UBSan handlers)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}", file=sys.stderr)
    return out


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
