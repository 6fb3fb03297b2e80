"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds, with the sanitizers on the host side only, the solver library (its validation,
CSR transpose, panel layout builder, presolve and postsolve, option handling) and the C
oracle, then runs the CPU tests of those parts against the instrumented builds in a child
process (the binding and the oracle module load the libraries named by LPGPU_LIB_OVERRIDE
and ORACLE_LIB_OVERRIDE; the panel layout checker is compiled with the same sanitizers).
Any sanitizer report stops the child with a failure. No GPU is touched: device code is
compiled as usual, and these tests never launch it."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_23951_amd", "csrc")
LLVM = "/opt/rocm/llvm/bin"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-shared-libsan"]
TESTS = ["tests/test_abi.py", "tests/test_presolve.py", "tests/test_panel_layout.py", "tests/test_oracle_pins.py",
         "tests/test_oracle_exact.py", "tests/test_oracle_structure.py", "tests/test_oracle_infeasible.py",
         "tests/test_oracle_halpern.py", "tests/test_oracle_restarts.py", "tests/test_oracle_polish.py"]


def _runtime():
    clang = os.path.join(LLVM, "clang")
    if not os.path.exists(clang) or shutil.which("hipcc") is None:
        return None
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not os.path.isabs(path):
        lib = subprocess.run([clang, "-print-resource-dir"], capture_output=True, text=True).stdout.strip()
        path = os.path.join(lib, "lib", "linux", "libclang_rt.asan-x86_64.so")
    return path if os.path.exists(path) else None


@pytest.mark.skipif(_runtime() is None, reason="needs ROCm's clang with its sanitizer runtimes")
def test_host_code_under_sanitizers(tmp_path):
    rt = _runtime()
    lib = str(tmp_path / "liblpgpu_san.so")
    host_san = [f for flag in SAN for f in ("-Xarch_host", flag)]
    from paper_2604_23951_amd.build import HIPCC_FLAGS, SOURCES
    flags = [f for f in HIPCC_FLAGS if f != "-O3"]
    r = subprocess.run(["hipcc", "-O1", "-g", *flags, *host_san, "-I", os.path.join(ROOT, "include"), "-o", lib,
                        *SOURCES], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    ora = str(tmp_path / "liboracle_san.so")
    r = subprocess.run([os.path.join(LLVM, "clang"), "-O1", "-g", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                        "-ffp-contract=off", "-fPIC", "-shared", *SAN, "-o", ora,
                        os.path.join(ROOT, "oracle", "pdhg_oracle.c"), "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", LPGPU_LIB_OVERRIDE=lib, ORACLE_LIB_OVERRIDE=ora,
               HOST_CXX=" ".join([os.path.join(LLVM, "clang++"), *SAN]))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stdout + r.stderr
