"""Host checks of the LDS lane schedule (schedule.cpp), compiled with g++ and
run on the CPU: every edge appears once, in its own class, and no LDS bank is
touched twice by the u-rows, or by the v-rows, of one group of lanes that the
gfx950 LDS serves together (reads: 256 bytes of lanes, 32 lanes for 4-byte
rows; writes: 128 bytes of lanes; the model is written out in
sched_check.cpp); and the rows outside the last class, which the twist visits
inside that class's sub-sweep, are exactly the rows its edges leave out."""
import os
import subprocess

import pytest

import cosm_inputs as ci
import paper_2605_30355_amd as cosm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    # built per test process (parallel workers must not share the binary)
    out = str(tmp_path_factory.mktemp("bin") / "sched_check")
    src = os.path.join(ROOT, "tests", "cpp", "sched_check.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2605_30355_amd", "csrc"),
                           "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", src,
                           os.path.join(ROOT, "paper_2605_30355_amd", "csrc", "schedule.cpp"),
                           "-o", out])
    return out


CASES = [(ci.random_regular(2000, 3, seed=2), cosm.COLOR_BALANCED, None),
         (ci.torus(20), cosm.COLOR_TORUS, [20, 20]),
         (ci.torus(141, seed=4), cosm.COLOR_TORUS, [141, 141]),
         (ci.random_regular(20000, 5, seed=1000, weights="pm1"), cosm.COLOR_GREEDY, None),
         (ci.erdos_renyi_capped(10000, 4, 8, seed=3), cosm.COLOR_MISRA_GRIES, None),
         (ci.small_random(37, 150, seed=5), cosm.COLOR_GREEDY, None),
         (ci.torus(101, seed=6, weights="pm12"), cosm.COLOR_TORUS, [101, 101])]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0].name)
@pytest.mark.parametrize("W", [4, 2, 1])
def test_schedule_conflict_free_and_complete(checker, case, W):
    inst, method, sides = case
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, method, sides)
    txt = f"{inst.n} {inst.m} {C}\n" + "\n".join(
        f"{u} {v} {J} {c}" for u, v, J, c in zip(inst.eu, inst.ev, inst.J, colour))
    r = subprocess.run([checker, str(W)], input=txt, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "conflicts=0" in r.stdout and "equal=1" in r.stdout and "fuse_ok=1" in r.stdout \
        and "bad_dummy=0" in r.stdout, r.stdout
    # the streamed word form (long schedules): same edges, dummies, no conflicts
    assert "stream_ok=1" in r.stdout and "stream_conflicts=0" in r.stdout, r.stdout
