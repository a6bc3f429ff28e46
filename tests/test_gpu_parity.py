"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Grid schedule (every value on the 2^-23 turn grid): phases, spins, energies and
cuts must be bit-identical to the oracle's for whole trials.  Phases compare as
turns (GPU) against degrees / 360 (oracle), which is exact on the grid.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

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


def make(inst, method=cosm.COLOR_GREEDY, sides=None):
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, method, sides)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C, h=inst.h)
    return colour, C, prob


def oparams(p: cosm.Params):
    return oracle.Params(alpha0_deg=p.alpha0_deg, dwt_ratio=p.dwt_ratio, dwt_period=p.dwt_period,
                         dwt_window_deg=p.dwt_window_deg, n_bisectors=p.n_bisectors,
                         sweeps=p.sweeps_per_trial, schedule=p.schedule, update=p.update)


def run_gpu(inst, colour, C, params, seed, R, sweeps, chunks=1):
    say(f"[gpu] {inst.name} R={R} sweeps={sweeps} res={params.residency} "
        f"rw={params.replicas_per_wg} store={params.storage} sched={params.schedule}")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, params, seed=seed, replicas=R,
                    h=inst.h) as st:
        done = 0
        for k in range(chunks):
            step = sweeps // chunks + (1 if k < sweeps % chunks else 0)
            st.sweep(step)
            done += step
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
        info = st.info()
    say(f"[gpu]   done: {info}")
    return x, H, cut, spins, info


# ---------------------------------------------------------------------------
def test_init_matches_oracle():
    inst = ci.random_regular(124, 3, seed=5)
    colour, C, prob = make(inst)
    for sched in (cosm.SCHED_GRID, cosm.SCHED_CONTINUOUS):
        p = cosm.Params(schedule=sched, sweeps_per_trial=10)
        say(f"[gpu] init sched={sched}")
        with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=77, replicas=37) as st:
            x = st.get_phases(cosm.UNIT_DEGREES)
            st.reset(78, 1000)
            x2 = st.get_phases(cosm.UNIT_DEGREES)
        assert np.array_equal(x, oracle.init_phases(inst.n, 77, 0, 37, sched))
        assert np.array_equal(x2, oracle.init_phases(inst.n, 78, 1000, 37, sched))


@pytest.mark.parametrize("inst", [ci.torus(20, seed=1), ci.random_regular(2000, 3, seed=2),
                                  ci.small_random(30, 200, seed=3, weights="pm12"),
                                  ci.erdos_renyi_capped(1000, 4, 8, seed=4)],
                         ids=lambda i: i.name)
def test_energy_of_given_spins(inst):
    colour, C, prob = make(inst)
    R = 19
    rng = np.random.default_rng(1)
    s = rng.choice(np.array([-1, 1], np.int8), size=(R, inst.n))
    s[0] = 1
    s[1] = -1
    say(f"[gpu] energy {inst.name}")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, cosm.Params(), replicas=R) as st:
        H, cut, back = st.energy(s)
    Hr, cr = oracle.energy(prob, s)
    assert np.array_equal(H, Hr) and np.array_equal(cut, cr)


def test_energy_with_bias_fields():
    inst = ci.small_random(25, 60, seed=9)
    inst.h = np.random.default_rng(2).integers(-2, 3, size=inst.n).astype(np.int32)
    colour, C, prob = make(inst)
    s = np.random.default_rng(3).choice(np.array([-1, 1], np.int8), size=(5, inst.n))
    say("[gpu] energy with h")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, cosm.Params(), replicas=5,
                    h=inst.h) as st:
        H, cut, _ = st.energy(s)
    Hr, cr = oracle.energy(prob, s)
    assert np.array_equal(H, Hr) and np.array_equal(cut, cr)


def test_energy_rejects_bad_spins():
    inst = ci.torus(4)
    colour, C, _ = make(inst)
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, cosm.Params(), replicas=2) as st:
        s = np.ones((2, inst.n), np.int8)
        s[1, 3] = 0
        with pytest.raises(CosmError) as e:
            st.energy(s)
        assert e.value.status == -1


# ---------------------------------------------------------------------------
# Whole trials in the grid schedule: bit-exact.
# ---------------------------------------------------------------------------
def check_trial(inst, colour, C, prob, params, seed, R, sweeps, chunks=1, sample=None):
    x, H, cut, spins, info = run_gpu(inst, colour, C, params, seed, R, sweeps, chunks)
    op = oparams(params)
    rows = list(range(R)) if sample is None else [int(r) for r in sample]
    say(f"[oracle] {len(rows)} replicas x {sweeps} sweeps")

    def one(r):  # ctypes releases the GIL, so rows run in parallel
        xr = oracle.init_phases(inst.n, seed, r, 1, params.schedule)
        oracle.sweeps(prob, op, seed, r, xr, 0, sweeps, n_threads=1)
        return xr

    with ThreadPoolExecutor(max_workers=8) as pool:
        ref = list(pool.map(one, rows))
    for r, xr in zip(rows, ref):
        sr, Hr, cr, _ = oracle.readout(prob, op, xr)
        assert np.array_equal(x[r] * 360.0, xr[0]), f"replica {r}: phases differ"
        assert H[r] == Hr[0] and cut[r] == cr[0], f"replica {r}: energy differs"
        assert np.array_equal(spins[r], sr[0]), f"replica {r}: spins differ"
    return info


@pytest.mark.parametrize("rw", [1, 2, 4])
def test_c1_torus20_full_trial_lds(rw):
    """20x20 +-1 torus, 4 classes, 64 replicas, 2000 sweeps (the small workload)."""
    inst = ci.torus(20, seed=1)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [20, 20])
    p = cosm.Params(sweeps_per_trial=2000, dwt_ratio=0.5, dwt_period=3, residency=cosm.RES_LDS,
                    replicas_per_wg=rw)
    info = check_trial(inst, colour, C, prob, p, seed=42, R=64, sweeps=2000)
    assert info["residency"] == cosm.RES_LDS and info["replicas_per_wg"] == rw


@pytest.mark.parametrize("res", [cosm.RES_HBM, cosm.RES_PLAIN])
def test_c1_torus20_other_forms(res):
    inst = ci.torus(20, seed=1)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [20, 20])
    p = cosm.Params(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3, residency=res)
    check_trial(inst, colour, C, prob, p, seed=5, R=8 if res == cosm.RES_PLAIN else 70, sweeps=300)


def test_ragged_replicas_and_resume():
    """R not a multiple of the row width; sweeps split over several calls."""
    inst = ci.random_regular(300, 3, seed=8, weights="pm1")
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    p = cosm.Params(sweeps_per_trial=500, dwt_ratio=1.5, dwt_period=3, residency=cosm.RES_LDS,
                    replicas_per_wg=4)
    check_trial(inst, colour, C, prob, p, seed=9, R=37, sweeps=500, chunks=7)


def check_all(inst, colour, C, prob, params, seed, R, sweeps, phase_rows):
    """Every replica's energy, cut and spins, and the phases of phase_rows,
    against the oracle run on all host cores."""
    x, H, cut, spins, info = run_gpu(inst, colour, C, params, seed, R, sweeps)
    op = oparams(params)
    say(f"[oracle] all {R} replicas x {sweeps} sweeps")
    xr, sr, Hr, cr = oracle.solve(prob, op, seed, 0, R, n_threads=16)
    bad = np.nonzero((H != Hr) | (cut != cr))[0]
    assert len(bad) == 0, f"energies differ at replicas {bad[:10].tolist()}"
    assert np.array_equal(spins, sr), "spins differ"
    for r in phase_rows:
        assert np.array_equal(x[r] * 360.0, xr[r]), f"replica {r}: phases differ"
    return info


def xcd_sample(R, rw, per_block=3):
    """Replicas spread over the 8 XCD ranges of the sweep's workgroup map: the
    kernel gives XCD x the replica blocks [x q, (x + 1) q), q = blocks / 8."""
    blocks = (R + rw - 1) // rw
    q = blocks // 8
    rows = set()
    for x in range(8):
        lo, hi = x * q * rw, (x + 1) * q * rw - 1
        rows.update(np.linspace(lo, hi, per_block).round().astype(int).tolist())
    rows.add(R - 1)
    return sorted(r for r in rows if r < R)


def test_c2_full_size_bench_shape():
    """3-regular N=2000 Max-Cut (+1 weights), equalised Misra-Gries colouring,
    1024 replicas, 1e4 sweeps, in the shape the benchmark times (2 replicas
    and 768 threads per workgroup, one slot per class, the twist fused into the
    last class): energies, cuts and spins of all 1024 replicas, phases of
    replicas spread over the XCD blocks."""
    inst = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
    colour, C, prob = make(inst, cosm.COLOR_BALANCED)
    p = cosm.Params(sweeps_per_trial=10000, dwt_ratio=1.0, dwt_period=6, replicas_per_wg=2,
                    threads_per_wg=768, lds_form=cosm.LDS_FORM_PAIR)
    info = check_all(inst, colour, C, prob, p, seed=42, R=1024, sweeps=10000,
                     phase_rows=xcd_sample(1024, 2))
    assert info["residency"] == cosm.RES_LDS
    assert info["replicas_per_wg"] == 2 and info["threads_per_wg"] == 768
    assert info["lds_form"] == cosm.LDS_FORM_PAIR and info["twist_fused"] == 1


def test_torus141_full_width():
    """The 141 x 141 +-1 torus (N = 19881, 6 classes) at 4096 replicas in the
    benchmark's shape and trial length (10^4 sweeps): energies, cuts and spins
    of replicas sampled from every XCD block of the workgroup map, and their
    phases, against the oracle."""
    import bench
    cfg = bench.HEADLINE
    inst = bench.headline_instance()
    colour, C, prob = make(inst, cfg["colouring"], cfg["sides"])
    S = cfg["sweeps"]
    p = bench.headline_params(cosm, sweeps_per_trial=S)
    R = cfg["replicas"]
    rows = xcd_sample(R, p.replicas_per_wg or 2)
    info = check_trial(inst, colour, C, prob, p, seed=3, R=R, sweeps=S, sample=rows)
    assert info["residency"] == cosm.RES_LDS and info["replicas"] == R
    assert info["replicas_per_wg"] == p.replicas_per_wg
    assert info["threads_per_wg"] == p.threads_per_wg
    assert info["streamed"] == 1 and info["lazy_wrap"] == 1


@pytest.mark.parametrize("order", [0, cosm.ORDER_LARGEST_LAST])
def test_large_torus_odd_side_sampled(order):
    """141x141 torus (N=19881, 6 classes): the largest LDS-resident replica block,
    in the colour order given and with the largest class last."""
    inst = ci.torus(141, seed=4)
    colour, C, prob = make(inst, cosm.COLOR_TORUS | order, [141, 141])
    p = cosm.Params(sweeps_per_trial=200, dwt_ratio=0.5, dwt_period=3)
    info = check_trial(inst, colour, C, prob, p, seed=3, R=96, sweeps=200, sample=[0, 95])
    assert info["residency"] == cosm.RES_LDS


def test_five_regular_20000_sampled():
    inst = ci.random_regular(20000, 5, seed=1000, weights="pm1")
    colour, C, prob = make(inst, cosm.COLOR_GREEDY)
    p = cosm.Params(sweeps_per_trial=100, dwt_ratio=1.5, dwt_period=3)
    check_trial(inst, colour, C, prob, p, seed=6, R=64, sweeps=100, sample=[0, 33, 63])


def test_five_regular_20000_seed_study_shape():
    """The 5-regular N = 20000 +-1 family of the time-to-target study at full
    size: 2048 replicas x 10^4 sweeps, equalised colouring, the streamed pair
    form at 2 replicas and 1024 threads per workgroup; replicas sampled from
    every XCD block against the oracle."""
    inst = ci.random_regular(20000, 5, seed=1000, weights="pm1")
    colour, C, prob = make(inst, cosm.COLOR_BALANCED)
    p = cosm.Params(sweeps_per_trial=10000, dwt_ratio=1.5, dwt_period=3,
                    lds_form=cosm.LDS_FORM_PAIR, replicas_per_wg=2, threads_per_wg=1024)
    info = check_trial(inst, colour, C, prob, p, seed=1, R=2048, sweeps=10000,
                       sample=xcd_sample(2048, 2, per_block=1))
    assert info["residency"] == cosm.RES_LDS and info["streamed"] == 1
    assert info["replicas_per_wg"] == 2 and info["threads_per_wg"] == 1024


def test_degenerate_instances():
    # one edge; no edges (twist only); an empty class in the middle
    one = ci.Instance("one_edge", 2, np.array([0], np.int32), np.array([1], np.int32),
                      np.array([1], np.int32))
    c, C, prob = make(one)
    check_trial(one, c, C, prob, cosm.Params(sweeps_per_trial=50, dwt_period=2), 1, 5, 50)
    none = ci.Instance("no_edges", 17, np.zeros(0, np.int32), np.zeros(0, np.int32),
                       np.zeros(0, np.int32))
    c, C, prob = make(none)
    check_trial(none, c, C, prob, cosm.Params(sweeps_per_trial=30, dwt_period=1, dwt_ratio=1.0), 2, 9, 30)
    inst = ci.cycle(10, weights="antiferro")
    c = np.array([0, 2, 0, 2, 0, 2, 0, 2, 0, 2], np.int32)  # class 1 empty
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=c, C=3)
    check_trial(inst, c, 3, prob, cosm.Params(sweeps_per_trial=40), 3, 4, 40)


def test_trap_triangle_scs_escapes_on_gpu():
    inst = ci.trap_triangle()
    colour, C, prob = make(inst)
    p = cosm.Params(sweeps_per_trial=1000, dwt_period=0)
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, replicas=1) as st:
        st.set_phases(np.array([[0.0, 15.0, 0.0]]), cosm.UNIT_DEGREES, 0)
        st.sweep(1)
        H, _, _ = st.energy()
    assert H[0] == -3


def test_schedule_limits_and_errors():
    inst = ci.torus(4)
    colour, C, _ = make(inst)
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C,
                    cosm.Params(sweeps_per_trial=10), replicas=2) as st:
        st.sweep(10)
        with pytest.raises(CosmError) as e:
            st.sweep(1)
        assert e.value.status == -4
    with pytest.raises(CosmError) as e:
        big = ci.torus(150, seed=1)
        cb, Cb, _ = make(big, cosm.COLOR_TORUS, [150, 150])
        cosm.State(big.n, big.eu, big.ev, big.J, cb, Cb,
                   cosm.Params(residency=cosm.RES_LDS, replicas_per_wg=4), replicas=4)
    assert e.value.status == -4
    bad = colour.copy()
    bad[0] = bad[1] if inst.eu[0] == inst.eu[1] else bad[0]
    k0, k1 = np.nonzero((inst.eu == 0) | (inst.ev == 0))[0][:2]
    bad[k1] = bad[k0]
    with pytest.raises(CosmError) as e:
        cosm.State(inst.n, inst.eu, inst.ev, inst.J, bad, C, cosm.Params(), replicas=1)
    assert e.value.status == -3


def test_set_get_phases_roundtrip():
    inst = ci.torus(5)
    colour, C, _ = make(inst, cosm.COLOR_TORUS, [5, 5])
    x = oracle.init_phases(inst.n, 3, 0, 3)
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, cosm.Params(), replicas=3) as st:
        st.set_phases(x, cosm.UNIT_DEGREES, 0)
        assert np.array_equal(st.get_phases(cosm.UNIT_DEGREES), x)


# ---------------------------------------------------------------------------
# Continuous schedule: within 1e-4 rad for 8 sweeps, away from near-ties.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("inst", [ci.torus(20, seed=1), ci.random_regular(2000, 3, seed=2)],
                         ids=lambda i: i.name)
def test_continuous_first_sweeps_within_tolerance(inst):
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    p = cosm.Params(sweeps_per_trial=2000, schedule=cosm.SCHED_CONTINUOUS, dwt_period=3)
    R, seed = 64, 21
    x, *_ = run_gpu(inst, colour, C, p, seed, R, 8)
    xr = oracle.init_phases(inst.n, seed, 0, R, oracle.SCHED_CONTINUOUS)
    margin = oracle.sweeps(prob, oparams(p), seed, 0, xr, 0, 8, diag_sweeps=8)
    d = np.abs(x * 360.0 - xr) % 360.0
    err = np.deg2rad(np.minimum(d, 360.0 - d)).max(axis=1)
    clean = margin > 1e-3  # degrees: replicas with no decision within 1e-3 deg of a threshold
    say(f"continuous: {clean.sum()} of {R} replicas clear of ties; max err {err[clean].max():.2e} rad")
    assert clean.sum() >= R // 2
    assert np.all(err[clean] <= 1e-4)


def test_pm12_torus_alpha25():
    """+-1/+-2 torus (the scaling study's instances) with Appendix C's
    parameters: alpha0 = 25 degrees, ratio 1, period 3; |alpha J| up to 50."""
    inst = ci.torus(16, seed=16001, weights="pm12")
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [16, 16])
    p = cosm.Params(alpha0_deg=25.0, sweeps_per_trial=800, dwt_ratio=1.0, dwt_period=3)
    check_trial(inst, colour, C, prob, p, seed=31, R=96, sweeps=800)


def test_erdos_renyi_capped_sampled():
    """Erdos-Renyi N = 10000, mean degree 4, degree cap 8 (the irregular
    bounded-degree workload), equalised colouring, 2048 replicas in the LDS form;
    3 replicas checked against the oracle."""
    inst = ci.erdos_renyi_capped(10000, 4, 8, seed=3)
    colour, C, prob = make(inst, cosm.COLOR_BALANCED)
    p = cosm.Params(sweeps_per_trial=120, dwt_ratio=1.5, dwt_period=3)
    info = check_trial(inst, colour, C, prob, p, seed=8, R=2048, sweeps=120, sample=[0, 1023, 2047])
    assert info["residency"] == cosm.RES_LDS


def test_erdos_renyi_seed_study_shape():
    """The capped Erdos-Renyi N = 10000 family of the time-to-target study at
    full size: 2048 replicas x 10^4 sweeps, Misra-Gries colouring, the pair form
    at 4 replicas and 1024 threads per workgroup; replicas sampled from every
    XCD block against the oracle."""
    inst = ci.erdos_renyi_capped(10000, 4, 8, seed=1000)
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    p = cosm.Params(sweeps_per_trial=10000, dwt_ratio=1.5, dwt_period=3,
                    lds_form=cosm.LDS_FORM_PAIR, replicas_per_wg=4, threads_per_wg=1024)
    info = check_trial(inst, colour, C, prob, p, seed=1, R=2048, sweeps=10000,
                       sample=xcd_sample(2048, 4, per_block=1))
    assert info["residency"] == cosm.RES_LDS
    assert info["replicas_per_wg"] == 4 and info["threads_per_wg"] == 1024


def test_beyond_lds_capacity_uses_hbm_form():
    """A 300 x 300 torus (N = 90000) does not fit one replica in 160 KB of LDS:
    AUTO residency must fall back to the HBM form and still match the oracle."""
    inst = ci.torus(300, seed=9)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [300, 300])
    p = cosm.Params(sweeps_per_trial=30, dwt_ratio=0.5, dwt_period=3)
    info = check_trial(inst, colour, C, prob, p, seed=4, R=64, sweeps=30, sample=[0, 63])
    assert info["residency"] == cosm.RES_HBM


def test_library_owned_memory_and_small_workspace():
    """cosm_init with device_workspace = NULL (the library's own hipMalloc) gives
    the same trial as a caller workspace; a caller workspace smaller than
    cosm_workspace_bytes() is refused with ENOMEM before any device work."""
    import ctypes
    import torch
    inst = ci.torus(12, seed=2)
    colour, C, _ = make(inst, cosm.COLOR_TORUS, [12, 12])
    p = cosm.Params(sweeps_per_trial=200, dwt_ratio=0.5, dwt_period=3)
    res = []
    for own in (False, True):
        with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=5, replicas=16,
                        torch_workspace=not own) as st:
            st.sweep(200)
            res.append(st.energy())
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][2], res[1][2])
    L = cosm.load_library()
    cp = cosm.cosm._CParams()
    L.cosm_default_params(ctypes.byref(cp))
    need = ctypes.c_size_t(0)
    assert L.cosm_workspace_bytes(inst.n, inst.m, C, 16, ctypes.byref(cp), ctypes.byref(need)) == 0
    ws = torch.empty(max(need.value // 2, 1), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    eu, ev, J, col = (np.ascontiguousarray(a, np.int32) for a in (inst.eu, inst.ev, inst.J, colour))
    rc = L.cosm_init(ctypes.byref(h), inst.n, inst.m, eu.ctypes.data, ev.ctypes.data, J.ctypes.data,
                     None, col.ctypes.data, C, ctypes.byref(cp), 1, 16, None,
                     ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(need.value // 2))
    assert rc == -5 and not h.value


@pytest.mark.parametrize("form", [cosm.LDS_FORM_REGISTER, cosm.LDS_FORM_PAIR])
def test_torus100_full_size(form):
    """The 100 x 100 +-1 torus (N = 10000, 4 classes) at full size: 4096
    replicas x 10^4 sweeps, 4 replicas and 1024 threads per workgroup, in the
    register-owner layout the autotuner keeps for FP32 (4 register rows per
    thread, the twist fused into the last class) and in the pair layout;
    replicas from every XCD block against the oracle."""
    inst = ci.torus(100, seed=3)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [100, 100])
    p = cosm.Params(sweeps_per_trial=10000, dwt_ratio=0.5, dwt_period=3, lds_form=form,
                    replicas_per_wg=4, threads_per_wg=1024, residency=cosm.RES_LDS)
    info = check_trial(inst, colour, C, prob, p, seed=2, R=4096, sweeps=10000,
                       sample=xcd_sample(4096, 4, per_block=2))
    assert info["lds_form"] == form and info["replicas_per_wg"] == 4
    if form == cosm.LDS_FORM_REGISTER:
        assert info["register_rows"] == 4 and info["twist_fused"] == 1
