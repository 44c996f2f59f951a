"""Host code under the address and undefined-behaviour sanitizers (CPU only):
the smoothed-aggregation set-up (csrc/amg.cpp with tests/host/amg_check.cpp),
the reference and mesh tables (csrc/tables.cpp with tests/host/tables_check.cpp),
the one-sided face flux against the two-sided one (tests/host/pointwise_check.cpp),
and the C ABI's argument handling (tests/host/abi_check.c against the whole
library built with sanitized host code).  Only host code is instrumented: every
sanitizer flag goes to the host pass."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_09271_amd", "csrc")
INC = os.path.join(ROOT, "include")
HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
LINK_SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-gpu-sanitize"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _build(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.fail("build failed:\n" + " ".join(cmd) + "\n" + res.stderr[-3000:])


def _run(args):
    res = subprocess.run(args, capture_output=True, text=True, timeout=600, env=ENV)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and res.stdout.startswith("ok"), out[-4000:]
    return out


def _driver(tmp, name, sources, flags=()):
    exe = os.path.join(tmp, name)
    _build(["hipcc", "-O1", "-g", "-std=c++17", "-pthread", *SAN, *flags, "-I", CSRC, "-I", INC, *sources,
            *LINK_SAN, "-o", exe])
    return exe


def test_amg_setup_under_sanitizers(tmp_path):
    exe = _driver(str(tmp_path), "amg_check", [os.path.join(HOST, "amg_check.cpp"), os.path.join(CSRC, "amg.cpp")])
    _run([exe])


def test_tables_under_sanitizers(tmp_path):
    exe = _driver(str(tmp_path), "tables_check",
                  [os.path.join(HOST, "tables_check.cpp"), os.path.join(CSRC, "tables.cpp")])
    _run([exe])


def test_one_sided_face_flux_under_sanitizers(tmp_path):
    exe = _driver(str(tmp_path), "pointwise_check", [os.path.join(HOST, "pointwise_check.cpp")])
    print(_run([exe]))


def test_abi_argument_handling_under_sanitizers(tmp_path):
    """The whole library with sanitized host code, driven from plain C: every
    argument error dgnp_setup reports before using a device, NULL arguments,
    and a valid set-up (OK with a GPU, DGNP_E_HIP without one)."""
    from paper_2112_09271_amd import build as B
    tmp = str(tmp_path)

    def compile_one(src):
        obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _build(["hipcc", *B.FLAGS, "-g", *SAN, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = os.path.join(tmp, "libdgnp_san.so")
    _build(["hipcc", f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-pthread", *objs, *LINK_SAN, "-o", lib])
    exe = os.path.join(tmp, "abi_check")
    _build(["hipcc", "-O1", "-g", "-x", "c", *SAN, "-I", INC, os.path.join(HOST, "abi_check.c"), "-x", "none",
            lib, f"-Wl,-rpath,{tmp}", *LINK_SAN, "-o", exe])
    _run([exe])
