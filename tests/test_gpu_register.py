"""The register-owner layout of the LDS sweep (an independent set of vertices
in registers, each edge at it applied by that vertex's thread) applies the
same updates in the same class order as the pair layout, so phases, energies
and spins must be bit-identical to the pair layout and to the oracle's GRID
schedule, for every storage format the layout takes (FP32, FIX32, FIX16)."""
import sys

import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm
from paper_2605_30355_amd.cosm import CosmError

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(inst, colour, C, p, seed, R, steps):
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed, replicas=R,
                    h=inst.h) as st:
        for k in steps:
            st.sweep(k)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
        info = st.info()
    return x, H, cut, spins, info


def both(inst, colour, C, seed, R, steps, **kw):
    say(f"[gpu] register vs pair {inst.name} R={R} steps={steps} {kw}")
    a = run(inst, colour, C, cosm.Params(lds_form=cosm.LDS_FORM_REGISTER, **kw), seed, R, steps)
    b = run(inst, colour, C, cosm.Params(lds_form=cosm.LDS_FORM_PAIR, **kw), seed, R, steps)
    say(f"[gpu]   register: {a[4]}")
    assert a[4]["lds_form"] == cosm.LDS_FORM_REGISTER and a[4]["register_rows"] > 0
    assert b[4]["lds_form"] == cosm.LDS_FORM_PAIR
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    return a


def oracle_rows(inst, colour, C, p, seed, rows, sweeps, x):
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    op = oracle.Params(alpha0_deg=p.alpha0_deg, dwt_ratio=p.dwt_ratio, dwt_period=p.dwt_period,
                       sweeps=p.sweeps_per_trial,
                       schedule=oracle.SCHED_GRID16 if p.storage == cosm.STORE_FIX16
                       else oracle.SCHED_GRID)
    for r in rows:
        xr = oracle.init_phases(inst.n, seed, r, 1, op.schedule)
        oracle.sweeps(prob, op, seed, r, xr, 0, sweeps, n_threads=1)
        assert np.array_equal(x[r] * 360.0, xr[0]), f"replica {r}"


@pytest.mark.parametrize("storage", [cosm.STORE_FP32, cosm.STORE_FIX32, cosm.STORE_FIX16])
def test_maxcut_full_size(storage):
    """3-regular N=2000, 1024 replicas, 10^4 sweeps: the benchmark's shape."""
    inst = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
    kw = dict(storage=storage, sweeps_per_trial=10000, dwt_ratio=1.0, dwt_period=6)
    x = both(inst, colour, C, 42, 1024, [10000], **kw)[0]
    oracle_rows(inst, colour, C, cosm.Params(**kw), 42, [0, 777, 1023], 10000, x)


@pytest.mark.parametrize("rw", [1, 2, 4])
def test_torus20_every_row_width(rw):
    inst = ci.torus(20, seed=1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [20, 20])
    kw = dict(sweeps_per_trial=2000, dwt_ratio=0.5, dwt_period=3, residency=cosm.RES_LDS,
              replicas_per_wg=rw)
    x = both(inst, colour, C, 42, 64, [2000], **kw)[0]
    oracle_rows(inst, colour, C, cosm.Params(**kw), 42, range(64), 2000, x)


def test_ragged_resumed_pm12():
    """R not a multiple of the row width, +-1/+-2 couplings, sweeps split over
    calls, and the twist every sweep."""
    inst = ci.random_regular(600, 3, seed=8, weights="pm12")
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_MISRA_GRIES)
    kw = dict(sweeps_per_trial=500, alpha0_deg=25.0, dwt_ratio=1.0, dwt_period=1)
    x = both(inst, colour, C, 9, 37, [1, 2, 97, 100, 300], **kw)[0]
    oracle_rows(inst, colour, C, cosm.Params(**kw), 9, [0, 18, 36], 500, x)
    kw["storage"] = cosm.STORE_FIX32
    both(inst, colour, C, 9, 37, [250, 250], **kw)


@pytest.mark.parametrize("threads,rows", [(448, 2), (256, 4)])
def test_two_and_four_register_rows(threads, rows):
    """Fewer threads than register vertices: 2 or 4 register rows per thread."""
    inst = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
    for storage in (cosm.STORE_FP32, cosm.STORE_FIX16):
        kw = dict(storage=storage, sweeps_per_trial=1200, dwt_ratio=1.0, dwt_period=6,
                  replicas_per_wg=2 if storage == cosm.STORE_FP32 else 4, threads_per_wg=threads)
        a = both(inst, colour, C, 5, 200, [600, 600], **kw)
        assert a[4]["register_rows"] == rows and a[4]["threads_per_wg"] == threads
    oracle_rows(inst, colour, C, cosm.Params(**kw), 5, [0, 199], 1200, a[0])


@pytest.mark.parametrize("case", ["torus21", "rr4"])
def test_five_and_six_classes(case):
    """More than four classes (the odd torus pattern, a 4-regular graph)."""
    if case == "torus21":
        inst = ci.torus(21, seed=2)
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [21, 21])
        assert C == 6
    else:
        inst = ci.random_regular(1000, 4, seed=8, weights="pm1")
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_MISRA_GRIES)
        assert C == 5
    kw = dict(sweeps_per_trial=900, dwt_ratio=0.5, dwt_period=3)
    x = both(inst, colour, C, 3, 96, [900], **kw)[0]
    oracle_rows(inst, colour, C, cosm.Params(**kw), 3, [0, 95], 900, x)
    kw.update(threads_per_wg=128 if case == "torus21" else 256, replicas_per_wg=2)
    a = both(inst, colour, C, 3, 96, [450, 450], **kw)
    assert a[4]["register_rows"] == 2


@pytest.mark.parametrize("case", ["maxcut", "torus"])
def test_auto_layout_equals_pair(case):
    """AUTO times both layouts and keeps the faster; whichever it keeps, the
    result equals the pair layout's (the probes leave no state behind)."""
    if case == "maxcut":
        inst = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
        kw, R = dict(sweeps_per_trial=800, dwt_ratio=1.0, dwt_period=6), 1024
    else:
        inst = ci.torus(40, seed=6)
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [40, 40])
        kw, R = dict(sweeps_per_trial=800, dwt_ratio=0.5, dwt_period=3), 512
    say(f"[gpu] auto vs pair {inst.name}")
    a = run(inst, colour, C, cosm.Params(lds_form=cosm.LDS_FORM_AUTO, **kw), 13, R, [400, 400])
    b = run(inst, colour, C, cosm.Params(lds_form=cosm.LDS_FORM_PAIR, **kw), 13, R, [400, 400])
    say(f"[gpu]   auto kept: {a[4]}")
    assert a[4]["lds_form"] in (cosm.LDS_FORM_PAIR, cosm.LDS_FORM_REGISTER)
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)


def test_not_applicable():
    inst = ci.torus(8)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [8, 8])
    p = cosm.Params(storage=cosm.STORE_BF16, lds_form=cosm.LDS_FORM_REGISTER)
    with pytest.raises(CosmError) as e:
        cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, replicas=4)
    assert e.value.status == -4
    h = np.ones(inst.n, np.int32)
    p = cosm.Params(lds_form=cosm.LDS_FORM_REGISTER)
    with pytest.raises(CosmError) as e:
        cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, replicas=4, h=h)
    assert e.value.status == -4


@pytest.mark.parametrize("storage", [cosm.STORE_FP32, cosm.STORE_FIX32, cosm.STORE_FIX16])
def test_fused_twist_four_register_rows(storage):
    """The register kernel with 4 register rows per thread and the twist fused
    into the last class (the form the large even tori run): 64 threads hold
    the 200 register vertices of the 20 x 20 torus, four each; twist every 3
    sweeps; equal to the pair layout and to the oracle."""
    inst = ci.torus(20, seed=1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [20, 20])
    kw = dict(storage=storage, sweeps_per_trial=1500, dwt_ratio=0.5, dwt_period=3,
              residency=cosm.RES_LDS, replicas_per_wg=2 if storage != cosm.STORE_FIX16 else 4,
              threads_per_wg=64)
    a = both(inst, colour, C, 17, 40, [700, 800], **kw)
    assert a[4]["register_rows"] == 4 and a[4]["threads_per_wg"] == 64
    assert a[4]["twist_fused"] == 1
    oracle_rows(inst, colour, C, cosm.Params(**kw), 17, [0, 19, 39], 1500, a[0])
