"""Sanitizer builds of the host code, on the CPU.

- The oracle (oracle/oracle.c) built with AddressSanitizer and UndefinedBehaviorSanitizer
  (gcc, any error fatal), with its pins run against that build.
- The C-ABI library built with both sanitizers on its host code only (hipcc, each
  -fsanitize after -Xarch_host; the gfx950 code is unchanged), with the ABI tests run against
  it: without a GPU they reach the argument checks and error paths of the entry points.

A canary program with a planted heap overflow first shows that the runtime reports it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def clang_asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def preload_env(libs, **extra):
    env = dict(os.environ)
    old = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = ":".join(libs + ([old] if old else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    env.update(extra)
    return env


SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def test_canary_overflow_is_reported(tmp_path):
    src = tmp_path / "canary.c"
    src.write_text("#include <stdlib.h>\nint main(int c, char** v) { int* a = malloc(4 * sizeof(int));"
                   " a[c + 3] = 1; int r = a[0]; free(a); return r; }\n")
    exe = tmp_path / "canary"
    subprocess.run(["gcc", *SAN, str(src), "-o", str(exe)], check=True)
    p = subprocess.run([str(exe)], capture_output=True, text=True)
    # UndefinedBehaviorSanitizer's object-size check or AddressSanitizer stops it
    assert p.returncode != 0 and ("heap-buffer-overflow" in p.stderr or "insufficient space" in p.stderr)


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = gcc_runtime("libasan.so"), gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    so = tmp_path / "liborc_san.so"
    subprocess.run(["gcc", *SAN, "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    env = preload_env([asan, ubsan], PB_ORACLE_LIB=str(so))
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_grid_energy.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (p.stdout + p.stderr)[-3000:]
    assert p.returncode == 0, tail
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, tail
    assert " passed" in p.stdout


def test_abi_host_code_under_asan_ubsan(tmp_path):
    rt = clang_asan_runtime()
    if not rt or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or its sanitizer runtime not installed")
    so = tmp_path / "libpb_san.so"
    csrc = os.path.join(ROOT, "paper_2502_09323_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc)) if f.endswith(".hip")]
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize=function", "-Xarch_host", "-shared-libsan",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", csrc, *srcs, "-o", str(so)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = preload_env([rt], PB_LIB_PATH=str(so))
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (p.stdout + p.stderr)[-3000:]
    assert p.returncode == 0, tail
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, tail
