"""AddressSanitizer and UndefinedBehaviorSanitizer builds, run on the CPU.

* The oracle (plain C) built with gcc -fsanitize=address,undefined, driven
  through binary and ternary lattices with walls, moving walls, a solid box
  and a roller, consistent initialisation, observation and population
  read/write (tests/sanitize/oracle_main.c).
* The library's host code (parameter validation, the buffer and batch plans,
  argument checks, error reporting) built by hipcc with the sanitizers on the
  host side only, linked into a driver that calls the C ABI with valid and
  invalid arguments and no device present (tests/sanitize/host_main.cpp).

Either driver aborts on the first invalid access, leak or undefined
operation; leak detection is on."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2212_01617_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), (r.stdout[-3000:], r.stderr[-6000:])
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
                           "-Wno-unknown-pragmas", os.path.join(SAN, "oracle_main.c"), "-o", exe, "-lm"])
    out = _run(exe)
    assert out.count("ternary=1") == 2


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


def test_host_library_under_asan_ubsan(tmp_path):
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not found")
    # device code as usual; sanitizers on the host compilation only
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=on",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san]
    objs = []
    for src in ("api.hip", "kernels.hip"):
        o = str(tmp_path / src.replace(".hip", ".o"))
        subprocess.check_call([_hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", o],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        objs.append(o)
    main_o = str(tmp_path / "host_main.o")
    subprocess.check_call([clang, "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-c", os.path.join(SAN, "host_main.cpp"), "-o", main_o])
    exe = str(tmp_path / "host_asan")
    subprocess.check_call([clang, "-fsanitize=address,undefined", main_o, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                           "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    _run(exe)
