"""CPU check of the work ring of the device-side iteration loop (csrc/loop_ring.h).

The header's protocol is compiled with g++ against a host policy (GCC atomics on plain
memory) and driven by host threads that play the leaders of workgroups on a model solve with
random delays (tests/loop_ring_check.cpp): every tile of every update processed exactly once,
an interval's next update only after its last update was applied, every interval finished,
and no wait running out -- with the smallest ring the protocol allows (one slot per tile) and
with spare slots.  A zero wait bound forces the abort path: every thread must still end.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1502_06974_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("ring") / "loop_ring_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-I", CSRC, os.path.join(HERE, "loop_ring_check.cpp"),
                    "-o", exe], check=True)
    return exe


# seed, threads, intervals, max tiles per interval, max updates, spare ring slots
CASES = [(s, 8, 60, 5, 10, 0) for s in range(1, 9)] + [
    (21, 16, 300, 3, 20, 0), (22, 32, 6, 40, 8, 0), (23, 4, 500, 2, 4, 7), (24, 24, 40, 12, 30, 64),
    (25, 2, 30, 30, 5, 0), (26, 12, 1, 64, 50, 0)]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_ring_processes_every_update_once(checker, case):
    r = subprocess.run([checker, *map(str, case), str(20_000_000)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("seed", [31, 32])
def test_ring_abort_ends_every_wait(checker, seed):
    r = subprocess.run([checker, str(seed), "16", "100", "4", "10", "0", "0"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "aborted=1" in r.stdout


@pytest.mark.parametrize("seed", [41, 42])
def test_ring_runaway_interval_ends_every_thread(checker, seed):
    """A position limit below what the intervals need (as if an interval kept putting its tiles
    back past its update cap): the put beyond the limit sets ABORT and every thread ends."""
    r = subprocess.run([checker, str(seed), "16", "40", "4", "12", "0", str(20_000_000), "60"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "aborted=1" in r.stdout
