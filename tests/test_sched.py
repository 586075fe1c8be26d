"""CPU test of the serving loop's admission rules: tests/sched_check.cpp drives the library's
own scheduling header with random arrivals and a fake completion source (no GPU involved;
this checks the scheduling logic only, not a compute path)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2301_08068_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("sched") / "sched_check")
    src = os.path.join(HERE, "sched_check.cpp")
    base = [gxx, "-std=c++17", "-O1", "-g", "-Wall", "-I", CSRC, src, "-o", exe]
    # host-only build with the address and undefined-behaviour sanitizers where available
    r = subprocess.run(base[:1] + ["-fsanitize=address,undefined"] + base[1:], capture_output=True, text=True)
    if r.returncode != 0:
        subprocess.run(base, check=True)
    return exe


@pytest.mark.parametrize("seed", range(12))
def test_admission_rules(checker, seed):
    r = subprocess.run([checker, str(seed), "20000"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr


def test_checker_catches_out_of_order_start(tmp_path):
    """The checker itself: a scheduler that lets a later request overtake a waiting one must
    be reported."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    hdr = open(os.path.join(CSRC, "rmpc_sched.h")).read()
    broken = hdr.replace("if (!staging.alloc(r.stage_bytes, &off)) {\n                f.staging_wait = true;\n"
                         "                break;\n",
                         "if (!staging.alloc(r.stage_bytes, &off)) {\n                f.staging_wait = true;\n"
                         "                std::swap(pending.front(), pending.back());\n                break;\n")
    assert broken != hdr
    (tmp_path / "rmpc_sched.h").write_text(broken)
    exe = str(tmp_path / "chk")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", str(tmp_path), os.path.join(HERE, "sched_check.cpp"), "-o", exe],
                   check=True)
    bad = [subprocess.run([exe, str(s), "20000"], capture_output=True, text=True, timeout=120).returncode
           for s in range(6)]
    assert any(rc == 1 for rc in bad)
