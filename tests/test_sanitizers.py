"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (lane_oracle.c) built with gcc -fsanitize=address,undefined runs
  its pins (tests/test_oracle_pins.py) in a child process with the sanitizer
  runtime preloaded: any out-of-bounds access, overflow of a signed integer or
  other undefined behaviour in the oracle aborts that run.
* The C ABI's host side (argument validation, plan and admission logic in
  liblane.so) built with hipcc, host code sanitized and device code as usual,
  runs the contract tests (tests/test_capi.py, tests/test_serve_host.py) the
  same way; none of them reaches a kernel.
* A deliberately out-of-bounds C function built the same way must abort, so
  the set-up demonstrably catches what it is for.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_09460_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_GCC = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
# host-side sanitizers only (device code is built as usual)
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def gcc_asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def clang_asan_runtime():
    found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def run_pytest(files, env_extra, timeout=600):
    env = dict(os.environ, **ENV_SAN, **env_extra)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           "-m", "not gpu", *files], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=timeout)


def test_sanitizer_catches_a_planted_overflow(tmp_path):
    rt = gcc_asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\nint bad(int n) { int *a = malloc(4 * n); int s = a[n]; "
                   "free(a); return s; }\n")
    lib = tmp_path / "libbad.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", *SAN_GCC, str(src), "-o", str(lib)])
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).bad(8)"
    p = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, **ENV_SAN, LD_PRELOAD=rt),
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0 and "AddressSanitizer" in p.stderr


def test_oracle_pins_under_asan_ubsan(tmp_path):
    rt = gcc_asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = tmp_path / "liblane_oracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", *SAN_GCC,
                           os.path.join(ROOT, "oracle", "lane_oracle.c"), "-o", str(lib), "-lm"])
    p = run_pytest(["tests/test_oracle_pins.py"], {"LD_PRELOAD": rt, "LANE_ORACLE_LIB": str(lib)})
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-3000:]


def _hipcc_object(args):
    src, obj = args
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang",
           "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN_HOST, "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return obj


def test_c_abi_host_side_under_asan_ubsan(tmp_path):
    rt = clang_asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    from paper_2212_09460_amd import build

    jobs = [(os.path.join(CSRC, s), str(tmp_path / (s + ".o"))) for s in build.SOURCES]
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(_hipcc_object, jobs))
    lib = tmp_path / "liblane_san.so"
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *SAN_HOST, *objs,
                        "-o", str(lib), "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    p = run_pytest(["tests/test_capi.py", "tests/test_serve_host.py"],
                   {"LD_PRELOAD": rt, "LANE_LIB_PATH": str(lib)})
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-3000:]
