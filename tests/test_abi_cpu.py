"""Host-side checks of libcosm that need no GPU: the library loads and exports
every function include/cosm.h declares, the three colourings are proper and
within their bounds, and bad graphs are rejected with the documented codes."""
import os
import re

import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm
from paper_2605_30355_amd.cosm import CosmError

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cosm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cosm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    declared = header_functions()
    assert len(declared) >= 10
    exported = cosm.exported_symbols()
    assert sorted(exported) == declared
    assert "gfx950" in cosm.version()


def test_default_params_match_tables_ix_x():
    p = cosm.default_params()
    assert p.alpha0_deg == 14.0 and p.dwt_window_deg == 90.0 and p.n_bisectors == 100
    assert p.dwt_ratio == 0.5 and p.dwt_period == 3
    assert p.schedule == cosm.SCHED_GRID and p.storage == cosm.STORE_FP32


INSTANCES = [ci.torus(6, seed=1), ci.torus(7, seed=2), ci.torus(20, seed=1),
             ci.random_regular(2000, 3, seed=2), ci.random_regular(600, 5, seed=3, weights="pm1"),
             ci.erdos_renyi_capped(3000, 4, 8, seed=3), ci.small_random(40, 300, seed=4),
             ci.trap_triangle(), ci.cycle(9)]


@pytest.mark.parametrize("inst", INSTANCES, ids=lambda i: i.name)
def test_greedy_equals_oracle_greedy(inst):
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_GREEDY)
    ref, Cref = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    assert C == Cref and np.array_equal(colour, ref)


@pytest.mark.parametrize("inst", INSTANCES, ids=lambda i: i.name)
def test_misra_gries_proper_and_at_most_delta_plus_one(inst):
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_MISRA_GRIES)
    delta = int(inst.degrees().max())
    assert oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, colour, C)
    assert C <= delta + 1
    assert np.all(np.bincount(colour, minlength=C) > 0)


@pytest.mark.parametrize("inst", INSTANCES, ids=lambda i: i.name)
def test_balanced_is_proper_equalised_and_same_count(inst):
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
    _, Cmg = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_MISRA_GRIES)
    assert C == Cmg
    assert oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, colour, C)
    sizes = np.bincount(colour, minlength=C)
    if inst.m >= 100:
        assert sizes.max() - sizes.min() <= 1


def test_misra_gries_many_random_graphs():
    rng = np.random.default_rng(0)
    for k in range(60):
        n = int(rng.integers(3, 40))
        m = int(rng.integers(0, n * (n - 1) // 2 + 1))
        inst = ci.small_random(n, m, seed=k)
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_MISRA_GRIES)
        delta = int(inst.degrees().max()) if m else 0
        assert oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, colour, C)
        assert C <= delta + 1


@pytest.mark.parametrize("L", [(4, 4), (6, 8), (5, 5), (141, 141), (7, 6), (100, 100)])
def test_torus_pattern(L):
    Lx, Ly = L
    inst = ci.torus(Lx, Ly, seed=3)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [Lx, Ly])
    assert oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, colour, C)
    assert C == 4 + (Lx % 2) + (Ly % 2)
    sizes = np.bincount(colour)
    if Lx % 2 == 0 and Ly % 2 == 0:  # regular pattern: N/2 edges per class (Sec. II-B)
        assert np.all(sizes == inst.n // 2)


def test_torus_rejects_non_lattice_edge():
    inst = ci.torus(6, seed=1)
    eu = np.append(inst.eu, 0)
    ev = np.append(inst.ev, 14)
    with pytest.raises(CosmError) as e:
        cosm.build_partitions(inst.n, eu, ev, cosm.COLOR_TORUS, [6, 6])
    assert e.value.status == -1


@pytest.mark.parametrize("eu,ev,status", [
    ([0, 1], [1, 1], -1),      # self-loop
    ([0, 1], [1, 5], -1),      # endpoint out of range
    ([0, 1, 1], [1, 2, 0], -2),  # duplicate undirected edge
    ([-1], [1], -1),
])
def test_bad_graphs_rejected(eu, ev, status):
    with pytest.raises(CosmError) as e:
        cosm.build_partitions(3, eu, ev, cosm.COLOR_GREEDY)
    assert e.value.status == status


def test_empty_graph():
    colour, C = cosm.build_partitions(5, [], [], cosm.COLOR_GREEDY)
    assert C == 0 and len(colour) == 0


def test_minimum_colouring():
    """MINIMUM: Delta colours on random 3- and 5-regular graphs (class 1),
    Delta + 1 on the Petersen graph (class 2); always proper and equalised."""
    import cosm_inputs as ci
    for g, delta in ((ci.random_regular(400, 3, seed=3), 3), (ci.random_regular(300, 5, seed=4), 5)):
        c, C = cosm.build_partitions(g.n, g.eu, g.ev, cosm.COLOR_MINIMUM)
        assert C == delta and oracle.is_proper_colouring(g.n, g.eu, g.ev, c, C)
        sizes = np.bincount(c, minlength=C)
        assert sizes.max() - sizes.min() <= 1
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    E = np.array(outer + spokes + inner, np.int32)
    c, C = cosm.build_partitions(10, E[:, 0], E[:, 1], cosm.COLOR_MINIMUM)
    assert C == 4 and oracle.is_proper_colouring(10, E[:, 0], E[:, 1], c, C)


@pytest.mark.parametrize("case", [("torus141", cosm.COLOR_TORUS), ("er", cosm.COLOR_GREEDY),
                                  ("rr3", cosm.COLOR_BALANCED)])
def test_largest_class_last(case):
    """COSM_ORDER_LARGEST_LAST swaps two labels only: the same classes, the
    largest one applied last, still a proper colouring."""
    name, method = case
    inst = {"torus141": ci.torus(141, seed=4), "er": ci.erdos_renyi_capped(3000, 4, 8, seed=7),
            "rr3": ci.random_regular(2000, 3, seed=2)}[name]
    sides = [141, 141] if name == "torus141" else None
    c0, C0 = cosm.build_partitions(inst.n, inst.eu, inst.ev, method, sides)
    c1, C1 = cosm.build_partitions(inst.n, inst.eu, inst.ev, method | cosm.ORDER_LARGEST_LAST, sides)
    assert C1 == C0 and oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, c1, C1)
    s0, s1 = np.bincount(c0, minlength=C0), np.bincount(c1, minlength=C1)
    assert s1[-1] == s0.max()
    big = int(np.argmax(s0)) if s0.max() > s0[-1] else C0 - 1
    relabel = np.arange(C0)
    relabel[[big, C0 - 1]] = [C0 - 1, big]
    assert np.array_equal(c1, relabel[c0])


def test_params_validation_on_host():
    """cosm_workspace_bytes validates the parameters without a device: storage
    formats (FIX32 needs the grid schedule) and the LDS layout selector."""
    import ctypes
    lib = cosm.load_library()

    def status(**kw):
        p = cosm.Params(**kw)._c()
        out = ctypes.c_size_t(0)
        return lib.cosm_workspace_bytes(100, 200, 4, 8, ctypes.byref(p), ctypes.byref(out)), out.value

    assert status()[0] == 0 and status()[1] > 0
    assert status(storage=cosm.STORE_FIX32)[0] == 0
    assert status(storage=cosm.STORE_FIX32, schedule=cosm.SCHED_CONTINUOUS)[0] == -1
    assert status(storage=cosm.STORE_FP16_PK)[0] == 0
    assert status(storage=6)[0] == -1
    # FP16 with FP16 arithmetic stores 2 bytes per replica-vertex, as FP16
    assert status(storage=cosm.STORE_FP16_PK)[1] == status(storage=cosm.STORE_FP16)[1]
    for form in (cosm.LDS_FORM_AUTO, cosm.LDS_FORM_PAIR, cosm.LDS_FORM_REGISTER,
                 cosm.LDS_FORM_REGISTER_STREAM):
        assert status(lds_form=form)[0] == 0
    assert status(lds_form=4)[0] == -1
    # FIX32 phases take 4 bytes per replica-vertex, FIX16 2
    assert status(storage=cosm.STORE_FIX32)[1] > status(storage=cosm.STORE_FIX16)[1]


def test_fix32_step_bound_checked_after_rounding():
    """FIX32 takes alpha0 * |J| in 2^-32 turn units as a signed 32-bit step:
    alpha0 just below 180 degrees rounds to half a turn on the 2^-22 turn step
    grid and is rejected (ERANGE) before any device work; slightly smaller
    values pass the check (they fail later only for want of a device)."""
    import ctypes
    lib = cosm.load_library()
    inst = ci.torus(4, seed=1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [4, 4])

    from paper_2605_30355_amd.cosm import _ptr
    eu, ev, J, col = (np.ascontiguousarray(a, dtype=np.int32)
                      for a in (inst.eu, inst.ev, inst.J, colour))

    def init_status(alpha0, storage):
        p = cosm.Params(alpha0_deg=alpha0, storage=storage)._c()
        st = ctypes.c_void_p(None)
        rc = lib.cosm_init(ctypes.byref(st), inst.n, inst.m, _ptr(eu), _ptr(ev), _ptr(J), None,
                           _ptr(col), C, ctypes.byref(p), 1, 4, None, None, 0)
        if rc == 0:
            lib.cosm_destroy(st)
        return rc

    assert init_status(180.0 - 2e-5, cosm.STORE_FIX32) == -4
    assert init_status(179.9, cosm.STORE_FIX32) != -4
    # FP32 storage has no such bound below a full turn
    assert init_status(180.0 - 2e-5, cosm.STORE_FP32) != -4
