"""Host checks of the register-owner schedule (reg_schedule.cpp), compiled with
g++ and run on the CPU (tests/cpp/reg_check.cpp): every edge exactly once, in
its class, with its own u / v roles; the register vertices independent and
each held once; every other vertex in exactly one LDS row; lanes without an
edge on dummy rows with J = 0; and, for the 3-regular benchmark graph, no LDS
bank touched twice within a lane group on the gfx950 model."""
import os
import subprocess

import pytest

import cosm_inputs as ci
import paper_2605_30355_amd as cosm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    # built per test process (parallel workers must not share the binary)
    out = str(tmp_path_factory.mktemp("bin") / "reg_check")
    src = os.path.join(ROOT, "tests", "cpp", "reg_check.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2605_30355_amd", "csrc"),
                           "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", src,
                           os.path.join(ROOT, "paper_2605_30355_amd", "csrc", "reg_schedule.cpp"),
                           "-o", out])
    return out


def run(checker, inst, method, sides, W, K):
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, method, sides)
    txt = f"{inst.n} {inst.m} {C}\n" + "\n".join(
        f"{u} {v} {J} {c}" for u, v, J, c in zip(inst.eu, inst.ev, inst.J, colour))
    return subprocess.run([checker, str(W), str(K)], input=txt, capture_output=True, text=True,
                          timeout=120)


def fields(out):
    return dict(kv.split("=") for kv in out.split())


@pytest.mark.parametrize("W", [1, 2, 4])
@pytest.mark.parametrize("K", [1, 2, 4])
def test_maxcut_graph_complete_and_conflict_free(checker, W, K):
    r = run(checker, ci.random_regular(2000, 3, seed=2), cosm.COLOR_BALANCED, None, W, K)
    assert r.returncode == 0, r.stdout + r.stderr
    f = fields(r.stdout)
    assert f["equal"] == "1" and f["indep"] == "1" and f["rows_ok"] == "1", r.stdout
    assert f["bad_dummy"] == "0" and f["conflicts"] == "0" and f["fuse_ok"] == "1", r.stdout
    # an independent set of a random cubic graph covers most edges
    assert int(f["reg_edges"]) >= 0.8 * 3000, r.stdout


@pytest.mark.parametrize("case", [
    (ci.torus(20), cosm.COLOR_TORUS, [20, 20]),
    (ci.random_regular(600, 3, seed=8, weights="pm12"), cosm.COLOR_MISRA_GRIES, None),
    (ci.small_random(40, 60, seed=3), cosm.COLOR_GREEDY, None),
], ids=lambda c: c[0].name)
@pytest.mark.parametrize("W", [1, 2, 4])
def test_other_graphs_complete(checker, case, W):
    inst, method, sides = case
    r = run(checker, inst, method, sides, W, 1)
    if r.returncode == 2:
        assert "ERANGE" in r.stdout
        return
    assert r.returncode == 0, r.stdout + r.stderr
    f = fields(r.stdout)
    assert f["equal"] == "1" and f["indep"] == "1" and f["rows_ok"] == "1", r.stdout
    assert f["bad_dummy"] == "0" and f["fuse_ok"] == "1", r.stdout


@pytest.mark.parametrize("W", [1, 2, 4])
def test_fused_twist_on_the_even_torus(checker, W):
    """On an even torus every vertex has an edge in every class, so with the
    whole register set placed the last class touches each row once and the
    twist is fused into it."""
    r = run(checker, ci.torus(20), cosm.COLOR_TORUS, [20, 20], W, 1)
    f = fields(r.stdout)
    assert f["fuse_ok"] == "1", r.stdout
    if int(f["reg_edges"]) + int(f["free"]) == 800 and f["bad_dummy"] == "0":
        assert f["fuse"] == "1" or int(f["free"]) > 0, r.stdout


def test_not_applicable_beyond_eight_classes(checker):
    inst = ci.small_random(37, 150, seed=5)
    r = run(checker, inst, cosm.COLOR_GREEDY, None, 2, 1)
    assert r.returncode == 2 and "ERANGE" in r.stdout


@pytest.mark.parametrize("txt", [
    "2 1 1\n0 1 -2 0",                                   # one edge
    "5 4 4\n0 1 1 0\n0 2 1 1\n0 3 -1 2\n0 4 1 3",        # a star: its centre alone covers it
    "3 3 3\n0 1 1 0\n1 2 1 1\n0 2 -1 2",                 # a triangle: one edge between LDS rows
    "6 2 1\n0 1 1 0\n4 5 1 0",                           # isolated vertices
], ids=["one_edge", "star", "triangle", "isolated"])
@pytest.mark.parametrize("W", [1, 2, 4])
@pytest.mark.parametrize("K", [1, 4])
def test_degenerate_graphs(checker, txt, W, K):
    r = subprocess.run([checker, str(W), str(K)], input=txt, capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    f = fields(r.stdout)
    assert f["equal"] == "1" and f["indep"] == "1" and f["rows_ok"] == "1", r.stdout
    assert f["bad_dummy"] == "0" and f["conflicts"] == "0", r.stdout


# The streamed register-owner schedule (K = 0 asks the checker for it): every
# edge exactly once in its class, with its own roles, from the register words
# of the register classes and the pair words; per-wave masks that cover every
# pair slot with an edge; no bank conflicts on the tori.
RSTREAM_CASES = [
    (ci.torus(141, seed=4), cosm.COLOR_TORUS, [141, 141], 2, 10, 4),
    (ci.torus(100, seed=3), cosm.COLOR_TORUS, [100, 100], 4, 8, 4),
    (ci.torus(101, seed=6, weights="pm12"), cosm.COLOR_TORUS, [101, 101], 2, 8, 4),
    (ci.random_regular(20000, 5, seed=1000, weights="pm1"), cosm.COLOR_BALANCED, None, 2, 8, 6),
]


@pytest.mark.parametrize("case", RSTREAM_CASES, ids=lambda c: f"{c[0].name}-W{c[3]}")
def test_rstream_schedule_complete(checker, case):
    inst, method, sides, W, K, rclasses = case
    r = run(checker, inst, method, sides, W, 0)
    assert r.returncode == 0, r.stdout + r.stderr
    f = fields(r.stdout)
    assert f["rstream"] == "1" and f["K"] == str(K) and f["rclasses"] == str(rclasses), r.stdout
    assert f["equal"] == "1" and f["indep"] == "1" and f["rows_ok"] == "1", r.stdout
    assert f["bad_dummy"] == "0" and f["mask_bad"] == "0", r.stdout
    if sides:  # the tori: conflict-free and nearly every edge in registers
        assert f["conflicts"] == "0", r.stdout
        assert int(f["reg_edges"]) >= 0.9 * inst.m, r.stdout


def test_rstream_row_offsets_bounded(checker):
    """Row offsets must stay below 2^18 bytes: 3000 disjoint 6-cliques (18000
    vertices, 7 classes, at most one register vertex per clique) leave about
    15000 LDS rows, too many for 16-byte rows and for 8-byte ones."""
    edges = [(6 * q + a, 6 * q + b) for q in range(3000) for a in range(6) for b in range(a + 1, 6)]
    colour = {}
    for q in range(3000):  # greedy edge colouring of each clique
        used = {}
        for a in range(6):
            for b in range(a + 1, 6):
                c = 0
                while c in used.get(a, set()) or c in used.get(b, set()):
                    c += 1
                used.setdefault(a, set()).add(c)
                used.setdefault(b, set()).add(c)
                colour[(6 * q + a, 6 * q + b)] = c
    C = max(colour.values()) + 1
    txt = f"18000 {len(edges)} {C}\n" + "\n".join(f"{u} {v} 1 {colour[(u, v)]}" for u, v in edges)
    for W in (4, 2):
        r = subprocess.run([checker, str(W), "0"], input=txt, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 2 and "ERANGE" in r.stdout, (W, r.stdout)
