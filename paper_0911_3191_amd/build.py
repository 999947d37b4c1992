"""Build libwdslash.so for gfx950 with hipcc (in-tree, next to this file).

Every translation unit under csrc/ is compiled separately (in parallel) and
linked into one shared library.  Packed FP32 instructions are disabled for
all device code.

`--sanitize` builds libwdslash_san.so instead, with the host code (API,
validation, solver driver, tuner, scheduler) instrumented by AddressSanitizer
and UndefinedBehaviorSanitizer; device code is built as usual.  It is loaded
through WD_LIB_PATH with clang's ASan runtime preloaded (tests/sanitize.sh).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwdslash.so")
OBJ_SAN = os.path.join(HERE, "_build_san")
LIB_SAN = os.path.join(HERE, "libwdslash_san.so")
ARCH = "gfx950"
# host-side sanitizers only: each -fsanitize= applies to the host pass
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall",
          "-Wno-unused-function", "-Wno-unused-result"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-munsafe-fp-atomics"]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(OBJ_SAN if sanitize else OBJ, os.path.basename(src) + ".o")
    extra = SANITIZE if sanitize else []
    cmd = [hipcc(), *COMMON, *DEVICE, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), *COMMON, "-x", "hip", *DEVICE, *extra, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{res.stdout}\n{res.stderr}")
    if res.stderr.strip():
        warn = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if warn:
            sys.stderr.write("\n".join(warn) + "\n")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link libwdslash.so (libwdslash_san.so with
    sanitize); returns the library path."""
    obj_dir, lib = (OBJ_SAN, LIB_SAN) if sanitize else (OBJ, LIB)
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sources()
    workers = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), srcs))
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SANITIZE if sanitize else []), "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
