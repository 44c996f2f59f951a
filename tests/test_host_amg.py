"""Host logic of the potential-block multigrid set-up (smoothed aggregation,
csrc/amg.cpp), compiled for the CPU with a small driver (tests/host/amg_check.cpp):
SpGEMM/transpose against dense products, aggregation coverage, symmetric
Galerkin operators, the coarsest inverse, repeatability across runs of the
threaded set-up, and the set-up that keeps an earlier hierarchy's prolongators
(same Galerkin levels bit for bit, a warm eigenvalue estimate between the cold
one and the Gershgorin bound, exact scaling for 2 A, refusal of another size)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_09271_amd", "csrc")


@pytest.fixture(scope="module")
def amg_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("amg") / "amg_check")
    cmd = ["hipcc", "-O2", "-std=c++17", "-pthread", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "amg_check.cpp"), os.path.join(CSRC, "amg.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.fail("host build failed:\n" + res.stderr[-3000:])
    return exe


def test_smoothed_aggregation_setup(amg_check):
    res = subprocess.run([amg_check], capture_output=True, text=True, timeout=300)
    print(res.stdout)
    assert res.returncode == 0 and res.stdout.startswith("ok"), res.stdout + res.stderr


@pytest.mark.parametrize("threads", ["1", "3"])
def test_setup_independent_of_thread_count(amg_check, threads):
    """The chunked reductions and products give bitwise the same hierarchy for
    any number of host workers (checksum over every value of the hierarchy)."""
    env = dict(os.environ)
    env.pop("DGNP_HOST_THREADS", None)
    base = subprocess.run([amg_check], capture_output=True, text=True, timeout=300, env=env).stdout
    env["DGNP_HOST_THREADS"] = threads
    res = subprocess.run([amg_check], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0 and res.stdout == base and "checksum" in base, (base, res.stdout)
