"""Build libnbhip.so (the HIP library behind include/nbhip.h) in-tree for gfx950.

    python -m paper_0902_0827_amd.build_lib

Always recompiles: every source to an object file in parallel (``_build/``, kept out
of version control), then one link.  Packed FP32 instructions are disabled
(-packed-fp32-ops): hipcc's automatic v_pk_* FP32 forms are not used anywhere in this
library.
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
LIB = os.path.join(HERE, "libnbhip.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["nb_api.cpp", "nb_build.hip", "nb_pair.hip", "nb_pair_cluster_f32.hip", "nb_pair_cluster_f64.hip",
           "nb_ewald.hip", "nb_pme.hip", "nb_noalloc.hip", "nb_md.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]
LIBS = ["-lhipfft"]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer build (`--sanitize`): the host
# code only (each flag after -Xarch_host; the device code is built as usual), into
# _build/sanitize/libnbhip_sanitize.so, for CPU tests of the host runtime run with the
# sanitizer runtime preloaded.
SAN_DIR = os.path.join(OBJDIR, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libnbhip_sanitize.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, verbose: bool, objdir: str = OBJDIR, extra=()) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    objdir, lib, extra = (SAN_DIR, SAN_LIB, SAN_FLAGS) if sanitize else (OBJDIR, LIB, [])
    os.makedirs(objdir, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, objdir, extra), SOURCES))
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LIBS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link libnbhip.so")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
