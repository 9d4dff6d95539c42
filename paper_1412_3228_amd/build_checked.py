"""Host-checked build of the HIP library: the host side of the hand-written
sources (argument checks, plans, tables, grouping, the filter's sphere
tables) compiled with AddressSanitizer and UndefinedBehaviorSanitizer, the
device code unchanged.  The kernel-table sources are linked from the plain
build's objects (build.py), so that build runs first.

The result, csrc/_build/checked/libhm_checked.so, is for host-only checks
without a GPU; it needs the sanitizer runtime preloaded
(``LD_PRELOAD=$(runtime_path())``) and is never loaded by the package.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess

from .build import ARCH, CSRC, FLAGS, OUT, _compile, _hipcc

CHECKED = os.path.join(OUT, "checked")
LIB = os.path.join(CHECKED, "libhm_checked.so")
# hand-written host code; the other sources only build kernel tables
HOST_SOURCES = ("hm_api.hip", "hm_filter.hip", "hm_extrapolate.hip", "hm_adjoint.hip")
# sanitizers for the host pass only (each flag behind -Xarch_host)
HOST_CHECKS = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def runtime_path() -> str:
    """The sanitizer runtime to preload (the compiler's own)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("sanitizer runtime not found (%s)" % path)
    return path


def build_checked(jobs: int = 0) -> str:
    """Compiles the host-checked objects and links libhm_checked.so."""
    hipcc = _hipcc()
    os.makedirs(CHECKED, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    plain = [os.path.join(OUT, os.path.splitext(f)[0] + ".o") for f in srcs if f not in HOST_SOURCES]
    missing = [o for o in plain if not os.path.exists(o)]
    if missing:
        raise RuntimeError("plain objects missing (run build.build_library first): %s" % missing[:3])
    work, objs = [], []
    for f in HOST_SOURCES:
        o = os.path.join(CHECKED, os.path.splitext(f)[0] + ".o")
        objs.append(o)
        work.append(([hipcc] + FLAGS + HOST_CHECKS + ["-c", os.path.join(CSRC, f), "-o", o], f))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs or min(4, os.cpu_count() or 2)) as ex:
        list(ex.map(_compile, work))
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", LIB + ".tmp"] + objs + plain
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("linking libhm_checked.so failed:\n%s" % r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB
