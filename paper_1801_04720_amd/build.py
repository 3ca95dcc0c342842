"""Build libsf.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with FP contraction off
(the FP32 stages perform exactly the stated operations) and packed-FP32
instructions disabled; the objects are linked into
paper_1801_04720_amd/libsf.so, which the Python binding loads.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsf.so")
# The same library with the kernels' index checks compiled in (sf_check.hpp).
LIB_CHECKED = os.path.join(PKG, "libsf_checked.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# Host code only: AddressSanitizer and UndefinedBehaviorSanitizer for the
# library's host side (argument validation, plans, task tables); the device
# code is built as usual.  The sanitizer runtime must be preloaded by the
# process that loads such a build.
SANITIZE = ["-g", "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + CFLAGS + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + src)
    return obj


def build(jobs: int = 8, sanitize: bool = False, out: str | None = None, build_dir: str | None = None,
          checked: bool = False) -> str:
    """Compile every HIP source and link libsf.so; returns its path.  With
    sanitize=True the host code is instrumented (SANITIZE) and the library goes
    to `out` (default: a separate build folder), never over the product build.
    checked=True compiles the kernels' index checks in (-DSF_CHECKED) and links
    libsf_checked.so next to libsf.so."""
    if checked:
        lib = out or LIB_CHECKED
        bdir = build_dir or BUILD + "_checked"
    else:
        lib = out or (os.path.join(BUILD + "_sanitize", "libsf.so") if sanitize else LIB)
        bdir = build_dir or (BUILD + "_sanitize" if sanitize else BUILD)
    os.makedirs(bdir, exist_ok=True)
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    srcs = sources()
    extra = (SANITIZE if sanitize else []) + (["-DSF_CHECKED"] if checked else [])
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, bdir, extra), srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libsf.so failed")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
