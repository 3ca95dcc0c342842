"""CPU-side hygiene: the oracle and the library's host code under
AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (plain C) is built with gcc -fsanitize=address,undefined together
  with a driver (tests/native/oracle_sanitize.c) that runs every oracle entry
  on small and degenerate shapes; out-of-bounds accesses, leaks and undefined
  operations abort the run.
* The library is rebuilt with its host code instrumented (build.SANITIZE: each
  -fsanitize= after -Xarch_host, device code unchanged) into a temporary
  folder, and the host-only C-ABI tests run against it with the sanitizer
  runtime preloaded.  Skipped where a preload is already set (it is not ours
  to replace) or hipcc / the runtime is missing."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_asan")
    srcs = sorted(glob.glob(os.path.join(ROOT, "oracle", "*.c"))) + [os.path.join(ROOT, "tests", "native",
                                                                                   "oracle_sanitize.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"] + srcs + ["-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "clean" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preload is already set for this process tree")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None:
        pytest.skip("hipcc or the clang sanitizer runtime missing")
    sys.path.insert(0, ROOT)
    from paper_1801_04720_amd import build

    lib = build.build(sanitize=True, out=str(tmp_path / "libsf.so"), build_dir=str(tmp_path / "obj"))
    env = dict(os.environ, SF_LIB_PATH=lib, LD_PRELOAD=rt[-1], ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")], capture_output=True, text=True,
                       env=env, cwd=str(tmp_path), timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
