"""FIX32 phase storage (32-bit fixed point, integer wrap) against the oracle's
GRID schedule: on the 2^-23 turn grid the FP32 trajectory is exact, and the
integer update of Eq. (6) (difference by wrapping subtraction, sign bit as the
biased sign of Eq. (4), wrap to one turn by overflow) reaches the same phases,
so phases, spins, energies and cuts must be bit-identical to the oracle and to
FP32 storage in every sweep form."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm
from paper_2605_30355_amd.cosm import CosmError

pytestmark = pytest.mark.gpu

GRID = oracle.SCHED_GRID


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(inst, method=cosm.COLOR_GREEDY, sides=None):
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, method, sides)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C, h=inst.h)
    return colour, C, prob


def fix32(**kw):
    return cosm.Params(storage=cosm.STORE_FIX32, schedule=cosm.SCHED_GRID, **kw)


def oparams(p):
    return oracle.Params(alpha0_deg=p.alpha0_deg, dwt_ratio=p.dwt_ratio, dwt_period=p.dwt_period,
                         dwt_window_deg=p.dwt_window_deg, n_bisectors=p.n_bisectors,
                         sweeps=p.sweeps_per_trial, schedule=GRID, update=p.update)


def run(inst, colour, C, p, seed, R, sweeps):
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed, replicas=R,
                    h=inst.h) as st:
        x0 = st.get_phases(cosm.UNIT_DEGREES)
        st.sweep(sweeps)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
        info = st.info()
    return x0, x, H, cut, spins, info


def check(inst, colour, C, prob, p, seed, R, sweeps, sample=None, optimal=False):
    say(f"[gpu] fix32 {inst.name} R={R} sweeps={sweeps} res={p.residency} "
        f"rw={p.replicas_per_wg} update={p.update} readout={p.readout}")
    x0, x, H, cut, spins, info = run(inst, colour, C, p, seed, R, sweeps)
    say(f"[gpu]   done: {info}")
    assert np.array_equal(x0, oracle.init_phases(inst.n, seed, 0, R, GRID))
    op = oparams(p)
    rows = list(range(R)) if sample is None else list(sample)

    def one(r):
        xr = oracle.init_phases(inst.n, seed, r, 1, GRID)
        oracle.sweeps(prob, op, seed, r, xr, 0, sweeps, n_threads=1)
        return xr

    with ThreadPoolExecutor(max_workers=8) as pool:
        ref = list(pool.map(one, rows))
    for r, xr in zip(rows, ref):
        if optimal:
            sr, Hr, cr, _ = oracle.readout_optimal(prob, xr)
        else:
            sr, Hr, cr, _ = oracle.readout(prob, op, xr)
        assert np.array_equal(x[r] * 360.0, xr[0]), f"replica {r}: phases differ"
        assert H[r] == Hr[0] and cut[r] == cr[0], f"replica {r}: energy differs"
        assert np.array_equal(spins[r], sr[0]), f"replica {r}: spins differ"
    return info


@pytest.mark.parametrize("rw", [1, 2, 4])
def test_torus20_lds_every_row_width(rw):
    inst = ci.torus(20, seed=1)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [20, 20])
    p = fix32(sweeps_per_trial=2000, dwt_ratio=0.5, dwt_period=3, residency=cosm.RES_LDS,
              replicas_per_wg=rw)
    info = check(inst, colour, C, prob, p, seed=42, R=64, sweeps=2000)
    assert info["residency"] == cosm.RES_LDS and info["replicas_per_wg"] == rw


@pytest.mark.parametrize("res", [cosm.RES_HBM, cosm.RES_PLAIN])
def test_torus20_hbm_and_plain(res):
    inst = ci.torus(20, seed=1)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [20, 20])
    p = fix32(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3, residency=res)
    check(inst, colour, C, prob, p, seed=5, R=8 if res == cosm.RES_PLAIN else 70, sweeps=300)


def test_maxcut_full_size_sampled_and_equal_to_fp32():
    """3-regular N=2000, 1024 replicas, 10^4 sweeps in the benchmark's shape:
    sampled replicas against the oracle, every replica against FP32 storage."""
    inst = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
    colour, C, prob = make(inst, cosm.COLOR_BALANCED)
    p = fix32(sweeps_per_trial=10000, dwt_ratio=1.0, dwt_period=6)
    info = check(inst, colour, C, prob, p, seed=42, R=1024, sweeps=10000,
                 sample=[0, 1, 511, 512, 1022, 1023])
    assert info["residency"] == cosm.RES_LDS
    say("[gpu] fix32 vs fp32 at full size")
    q = cosm.Params(storage=cosm.STORE_FP32, schedule=cosm.SCHED_GRID, sweeps_per_trial=10000,
                    dwt_ratio=1.0, dwt_period=6)
    a = run(inst, colour, C, p, 42, 1024, 10000)
    b = run(inst, colour, C, q, 42, 1024, 10000)
    for u, v in zip(a[:5], b[:5]):
        assert np.array_equal(u, v)


def test_ragged_streamed_pm12():
    """R not a multiple of the row width, +-1/+-2 couplings, a larger graph on
    the streamed schedule."""
    inst = ci.erdos_renyi_capped(3000, 4, 8, seed=7)
    colour, C, prob = make(inst, cosm.COLOR_GREEDY)
    p = fix32(sweeps_per_trial=400, dwt_ratio=1.5, dwt_period=3, residency=cosm.RES_LDS,
              replicas_per_wg=4)
    check(inst, colour, C, prob, p, seed=9, R=37, sweeps=400, sample=[0, 17, 36])
    inst = ci.torus(12, seed=3, weights="pm12")
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [12, 12])
    p = fix32(sweeps_per_trial=600, alpha0_deg=25.0, dwt_ratio=1.0, dwt_period=3)
    check(inst, colour, C, prob, p, seed=11, R=50, sweeps=600)


def test_bias_fields_and_full_gradient():
    inst = ci.small_random(40, 100, seed=3, weights="pm12")
    inst.h = np.random.default_rng(4).integers(-2, 3, size=inst.n).astype(np.int32)
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    for res in (cosm.RES_LDS, cosm.RES_HBM):
        p = fix32(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3, residency=res)
        check(inst, colour, C, prob, p, seed=2, R=20, sweeps=300)
    inst.h = None
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    p = fix32(sweeps_per_trial=200, dwt_ratio=0.5, dwt_period=3,
              update=cosm.UPDATE_FULL_GRADIENT)
    check(inst, colour, C, prob, p, seed=3, R=12, sweeps=200)


def test_optimal_readout():
    inst = ci.torus(16, seed=5)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [16, 16])
    p = fix32(sweeps_per_trial=150, dwt_ratio=0.5, dwt_period=3,
              readout=cosm.READOUT_OPTIMAL)
    check(inst, colour, C, prob, p, seed=8, R=24, sweeps=40, optimal=True)


def test_batch_equals_single_states():
    gs = []
    t = ci.torus(20, seed=1)
    c, C = cosm.build_partitions(t.n, t.eu, t.ev, cosm.COLOR_TORUS, [20, 20])
    gs.append((t, c, C, fix32(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3), 11, 64))
    g = ci.random_regular(2000, 3, seed=2)
    c, C = cosm.build_partitions(g.n, g.eu, g.ev, cosm.COLOR_BALANCED)
    gs.append((g, c, C, fix32(sweeps_per_trial=200, dwt_ratio=1.0, dwt_period=6), 12, 100))
    with cosm.Batch(storage=cosm.STORE_FIX32, max_graphs=4, max_n=4000) as b:
        ids = [b.add(i.n, i.eu, i.ev, i.J, c, C, p, seed=s, replicas=R) for i, c, C, p, s, R in gs]
        say("[gpu] fix32 batch run")
        b.run(ids)
        b.wait()
        for gid, (i, c, C, p, s, R) in zip(ids, gs):
            H, cut, sp = b.results(gid, return_spins=True)
            with cosm.State(i.n, i.eu, i.ev, i.J, c, C, p, seed=s, replicas=R) as st:
                st.sweep(p.sweeps_per_trial)
                Hs, cs, ss = st.energy()
            assert np.array_equal(H, Hs) and np.array_equal(cut, cs) and np.array_equal(sp, ss)


def test_validation_and_rounding():
    inst = ci.torus(6)
    colour, C, _ = make(inst, cosm.COLOR_TORUS, [6, 6])
    p = cosm.Params(storage=cosm.STORE_FIX32, schedule=cosm.SCHED_CONTINUOUS)
    with pytest.raises(CosmError) as e:
        cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, replicas=2)
    assert e.value.status == -1
    J2 = (inst.J * 13).astype(np.int32)  # 14 degrees * 13 = 182 degrees: above half a turn
    with pytest.raises(CosmError) as e:
        cosm.State(inst.n, inst.eu, inst.ev, J2, colour, C, fix32(), replicas=2)
    assert e.value.status == -4
    # phases set from outside are rounded to 2^-32 turn
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, fix32(), replicas=2) as st:
        x = np.full((2, inst.n), 0.3, np.float64)
        st.set_phases(x, cosm.UNIT_TURNS, 0)
        y = st.get_phases(cosm.UNIT_TURNS)
    f = np.float64(np.float32(0.3))
    assert np.array_equal(y, np.float64(np.float32(np.round(f * 2.0**32) / 2.0**32)) * np.ones_like(x))


def test_resume_across_calls_and_degenerate():
    """Sweeps split over several calls, an edgeless instance (twist only) and a
    single edge."""
    inst = ci.random_regular(300, 3, seed=8, weights="pm1")
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    p = fix32(sweeps_per_trial=500, dwt_ratio=1.5, dwt_period=3, residency=cosm.RES_LDS,
              replicas_per_wg=4)
    say("[gpu] fix32 resume")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=9, replicas=36) as st:
        for step in (1, 2, 97, 100, 300):
            st.sweep(step)
        x = st.get_phases(cosm.UNIT_TURNS)
    op = oparams(p)
    xr = oracle.init_phases(inst.n, 9, 0, 36, GRID)
    oracle.sweeps(prob, op, 9, 0, xr, 0, 500)
    assert np.array_equal(x * 360.0, xr)
    none = ci.Instance("no_edges", 17, np.zeros(0, np.int32), np.zeros(0, np.int32),
                       np.zeros(0, np.int32))
    c, C, prob = make(none)
    check(none, c, C, prob, fix32(sweeps_per_trial=30, dwt_period=1, dwt_ratio=1.0), 2, 10, 30)
    one = ci.Instance("one_edge", 2, np.array([0], np.int32), np.array([1], np.int32),
                      np.array([-2], np.int32))
    c, C, prob = make(one)
    check(one, c, C, prob, fix32(sweeps_per_trial=50, dwt_period=2), 1, 6, 50)
