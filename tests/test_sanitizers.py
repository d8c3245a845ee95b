"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C-ABI's host paths (line factors of the wind and product bispectra,
argument validation before any device work) from a host-only sanitized build
of the library, and every entry point of the FP64 oracle from a sanitized
build of its C source.  Each runs as its own process; any sanitizer report
fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2310_03979_amd", "csrc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang", shutil.which("clang")):
        if c and os.path.exists(c):
            return c
    pytest.skip("clang not found")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
          "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "srm3_oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_host_library_under_asan_ubsan(tmp_path):
    from paper_2310_03979_amd import build as b
    cc = b.hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    procs = []
    for src in b.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [cc, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={b.ARCH}",
               "-I", b.INCLUDE, "-I", CSRC] + san + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), cmd))
        objs.append(obj)
    for p, cmd in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, f"{' '.join(cmd)}\n{err}"
    lib = str(tmp_path / "libsrm3_san.so")
    _run([cc, "-shared", "-fPIC", f"--offload-arch={b.ARCH}"] + san + objs + ["-o", lib])
    exe = str(tmp_path / "host_driver")
    _run([_clang(), "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", b.INCLUDE, os.path.join(HERE, "host_driver.c"), lib, "-o", exe, "-lm",
          f"-Wl,-rpath,{tmp_path}", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "host driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
