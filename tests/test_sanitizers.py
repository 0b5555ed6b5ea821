"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

- The oracle (plain C) is rebuilt with gcc's sanitizers and its pins run
  against that build.
- libnnsort's host code (argument checks, workspace planning, the BF16 form's
  operand preparation, model files) is rebuilt with the sanitizers on the host
  side only (the device code is unchanged) and the CPU-side library tests run
  against that build.
Any report aborts the child process, which fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env_extra, cwd=ROOT, timeout=600):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    r = subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_pins_under_asan_ubsan(tmp_path):
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", so, os.path.join(ROOT, "oracle", "nnsort_oracle.c"),
                           "-lm"])
    pre = " ".join(subprocess.check_output(["gcc", f"-print-file-name={lib}"], text=True).strip()
                   for lib in ("libasan.so", "libubsan.so"))
    _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_oracle_pins.py",
          "-k", "not mutated"], {"LD_PRELOAD": pre, "NNSORT_ORACLE_LIB": so, "OMP_NUM_THREADS": "2"})


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_1907_08817_amd import build as B
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang AddressSanitizer runtime not found")
    B.build()  # the device-side objects are reused as built
    objs = []
    for src in B.SOURCES:
        obj = os.path.join(B.BUILD, os.path.splitext(src)[0] + ".o")
        if src == "api.cpp":
            obj = str(tmp_path / "api_san.o")
            san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
            subprocess.check_call([B.hipcc(), "-x", "hip", *B.COMMON, *san, "-c", os.path.join(B.CSRC, src),
                                   "-o", obj])
        objs.append(obj)
    so = str(tmp_path / "libnnsort_san.so")
    subprocess.check_call([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-shared-libsan",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-o", so, *objs])
    code = ("import sys, pytest; sys.path.insert(0, %r); import paper_1907_08817_amd as nn; "
            "nn.LIB_PATH = %r; sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', "
            "'tests/test_lib_cpu.py', 'tests/test_sanitizers_probe.py']))") % (ROOT, so)
    _run([sys.executable, "-c", code], {"LD_PRELOAD": rt[-1]})
