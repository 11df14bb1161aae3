"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU call): tests/host/host_checks.cpp fuzzes lb_validate against the
documented constraints, builds the per-grid constants of every valid grid, checks
the moving-shock cell count cell by cell, the batch work lists, the tile and
partition arithmetic and the early error returns of the entry points. The
sanitizers apply to host code only (each -fsanitize= behind -Xarch_host); the
build is cached under _build/ and redone when a source is newer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT_DIR = os.path.join(ROOT, "_build", "host_sanitize")
BIN = os.path.join(OUT_DIR, "host_checks")
CSRC = os.path.join(ROOT, "paper_0706_0405_amd", "csrc")
SOURCES = [os.path.join(CSRC, n) for n in ("lbkt.hip", "vn.hip", "noalloc.hip")] + \
    [os.path.join(ROOT, "tests", "host", "host_checks.cpp")]
DEPS = SOURCES + [os.path.join(CSRC, "kt_site.hpp"), os.path.join(CSRC, "lbkt_internal.hpp"),
                  os.path.join(ROOT, "include", "lbkt.h")]


def _build():
    if os.path.exists(BIN) and os.path.getmtime(BIN) > max(os.path.getmtime(p) for p in DEPS):
        return
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmd = [hipcc, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-o", BIN + ".tmp"] + SOURCES
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)
    os.replace(BIN + ".tmp", BIN)


@pytest.mark.slow
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    _build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([BIN, "100000"], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "all host checks passed" in out, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
