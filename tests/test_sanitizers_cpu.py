"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle.cpp) built with g++ and both sanitizers, loaded in place
  of the plain build, runs its pin tests and the paper-mode pins.
* The library's host code (mesh ingest, neighbour and boundary tables,
  convexity checks, BVH and R*-tree builds, the C interface) built with both
  sanitizers on the host side only, linked with the regular device objects,
  runs the host-only ingest and R*-tree tests.

Each run is a child process with the sanitizer runtime preloaded; any report
aborts it (no recovery), so a zero exit status means a clean run.
"""

import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(ROOT, "_build", "san")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run_pytest(env_extra, files):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *files], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    print(tail)
    return r.returncode, tail


def test_oracle_pins_under_asan_ubsan():
    os.makedirs(SAN, exist_ok=True)
    lib = os.path.join(SAN, "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "oracle.cpp")
    flags = ["-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
    san = ["-fsanitize=address,undefined"]
    subprocess.run(["g++", *flags, *san, src, "-o", lib], check=True)
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    rt_ub = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    rc, tail = _run_pytest({"LD_PRELOAD": f"{rt}:{rt_ub}", "TCT_ORACLE_LIB": lib},
                           ["tests/test_oracle_pins.py", "tests/test_oracle_paper_mode.py"])
    assert rc == 0, tail
    assert "passed" in tail


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    return hits[-1]


def test_host_library_under_asan_ubsan():
    from paper_1908_06909_amd import build as lib_build

    dev_objs = [os.path.join(lib_build.BUILD, s.replace(".hip", ".o")) for s in lib_build.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev_objs):
        lib_build.build()
    os.makedirs(SAN, exist_ok=True)
    # Host side only: every sanitizer flag is passed through -Xarch_host, so
    # the device code is built exactly as in the library.
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("mesh.cpp", "rstar.cpp", "capi.cpp"):
        obj = os.path.join(SAN, src.replace(".cpp", ".o"))
        flags = [f for f in lib_build.FLAGS if f != "-O3"] + ["-O1", "-g"]
        subprocess.run([HIPCC, "-x", "hip", *flags, *host_san, "-c", os.path.join(lib_build.CSRC, src), "-o", obj],
                       check=True, capture_output=True)
        objs.append(obj)
    lib = os.path.join(SAN, "libtetct_san.so")
    subprocess.run([HIPCC, f"--offload-arch={lib_build.ARCH}", "-shared", "-fPIC", *host_san, "-shared-libsan",
                    *objs, *dev_objs, "-o", lib], check=True, capture_output=True)
    rc, tail = _run_pytest({"LD_PRELOAD": _clang_asan_runtime(), "TCT_LIB_PATH": lib},
                           ["tests/test_lib_cpu.py", "tests/test_rstar_cpu.py"])
    assert rc == 0, tail
    assert "passed" in tail
