"""The streamed sweep form (long lane schedules: the large graphs), bit-exact
against the oracle's grid schedules on sampled replicas: uniform and varying
|J| (a second stream of magnitudes), classes with an odd number of slots (a
padding slot of dummy pairs) and final pairs that only the first waves run,
the twist as a pass after the last class, one, two and four FP32 replicas per
workgroup, the fixed-point and 16-bit storage formats, and FP32 phases wrapped
only at the twists (at the edge of the drift bound that keeps them exact)."""
import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm
from test_gpu_parity import check_trial, make, say

pytestmark = pytest.mark.gpu


def run_case(inst, colour, C, prob, p, seed, R, S, rows, oracle_sched=None):
    info = check_trial(inst, colour, C, prob, p, seed=seed, R=R, sweeps=S, sample=rows) \
        if oracle_sched is None else None
    if oracle_sched is not None:  # FIX16: the oracle's 16-bit grid schedule
        with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed,
                        replicas=R) as st:
            st.sweep(S // 2)
            st.sweep(S - S // 2)
            x = st.get_phases(cosm.UNIT_TURNS)
            H, cut, spins = st.energy()
            info = st.info()
        op = oracle.Params(alpha0_deg=p.alpha0_deg, dwt_ratio=p.dwt_ratio,
                           dwt_period=p.dwt_period, sweeps=p.sweeps_per_trial,
                           schedule=oracle_sched)
        for r in rows:
            xr = oracle.init_phases(inst.n, seed, r, 1, oracle_sched)
            oracle.sweeps(prob, op, seed, r, xr, 0, S, n_threads=1)
            assert np.array_equal(x[r] * 360.0, xr[0]), f"replica {r}"
            sr, Hr, cr, _ = oracle.readout(prob, op, xr)
            assert H[r] == Hr[0] and cut[r] == cr[0] and np.array_equal(spins[r], sr[0])
    say(f"[gpu]   streamed={info['streamed']} fused={info['twist_fused']}")
    assert info["streamed"] == 1
    return info


@pytest.mark.parametrize("storage", [cosm.STORE_FP32, cosm.STORE_FIX32])
def test_torus141_seam_classes(storage):
    """6 classes: four of 9870 edges (10 slots per thread) and the two seams of
    141 edges (one slot, padded to a pair that only the first waves run)."""
    inst = ci.torus(141, seed=4)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [141, 141])
    p = cosm.Params(sweeps_per_trial=400, dwt_ratio=0.5, dwt_period=3, storage=storage,
                    replicas_per_wg=2, threads_per_wg=1024, residency=cosm.RES_LDS)
    info = run_case(inst, colour, C, prob, p, 5, 96, 400, [0, 47, 95])
    assert info["twist_fused"] == 0


def test_torus141_fix16():
    inst = ci.torus(141, seed=4)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [141, 141])
    p = cosm.Params(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3,
                    storage=cosm.STORE_FIX16, replicas_per_wg=4, threads_per_wg=1024,
                    residency=cosm.RES_LDS)
    run_case(inst, colour, C, prob, p, 6, 64, 300, [0, 33, 63], oracle.SCHED_GRID16)


def test_varying_coupling_magnitude():
    """+-1/+-2 couplings: the step magnitudes come from their own stream."""
    inst = ci.torus(101, seed=6, weights="pm12")
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [101, 101])
    p = cosm.Params(alpha0_deg=25.0, sweeps_per_trial=300, dwt_ratio=1.0, dwt_period=3,
                    replicas_per_wg=2, threads_per_wg=1024, residency=cosm.RES_LDS)
    run_case(inst, colour, C, prob, p, 7, 64, 300, [0, 31, 63])


def test_five_regular_twist_pass():
    """5-regular N = 20000, equalised colouring: the rows outside the last class
    are few, but the streamed form keeps the twist as a pass of its own."""
    inst = ci.random_regular(20000, 5, seed=1000, weights="pm1")
    colour, C, prob = make(inst, cosm.COLOR_BALANCED)
    p = cosm.Params(sweeps_per_trial=150, dwt_ratio=1.5, dwt_period=3, replicas_per_wg=2,
                    threads_per_wg=1024, residency=cosm.RES_LDS)
    info = run_case(inst, colour, C, prob, p, 8, 64, 150, [0, 63])
    assert info["twist_fused"] == 0


@pytest.mark.parametrize("rw", [1, 4])
def test_row_widths(rw):
    """One and four FP32 replicas per workgroup (4- and 16-byte rows) on the
    capped Erdos-Renyi graph, twist every sweep, sweeps over several calls."""
    inst = ci.erdos_renyi_capped(6000, 4, 8, seed=11)
    colour, C, prob = make(inst, cosm.COLOR_MISRA_GRIES)
    p = cosm.Params(sweeps_per_trial=200, dwt_ratio=1.5, dwt_period=1, replicas_per_wg=rw,
                    threads_per_wg=512, residency=cosm.RES_LDS)
    info = check_trial(inst, colour, C, prob, p, seed=9, R=37, sweeps=200, chunks=3,
                       sample=[0, 18, 36])
    assert info["streamed"] == 1 and info["replicas_per_wg"] == rw


@pytest.mark.parametrize("case", [(14.3, 3, 1, 0), (14.3, 3, 1, cosm.ORDER_LARGEST_LAST),
                                  (14.5, 3, 0, 0), (14.0, 4, 0, 0)],
                         ids=["lazy-drift-0.4965", "lazy-largest-last", "eager-drift-0.5035",
                              "eager-drift-0.642"])
def test_lazy_wrap_bound(case):
    """FP32 phases wrapped to [0, 1) turn only at the twists stay exact while no
    phase can drift by 1/2 turn from [0, 1) between two twists: the twist
    (ratio x alpha0, left unwrapped) plus period x alpha0 x 4 on a +-1 torus.
    alpha0 = 14.3 deg with a twist every 3 sweeps and ratio 1/2 sits just
    inside the bound (0.4965 turn), also with the classes reordered;
    14.5 deg (0.5035) and every 4 sweeps at 14 deg (0.642) lie outside it and
    keep the wrap at every update.  All bit-exact against the oracle."""
    a0, T, lazy, order = case
    inst = ci.torus(101, seed=9)
    colour, C, prob = make(inst, cosm.COLOR_TORUS | order, [101, 101])
    p = cosm.Params(alpha0_deg=a0, sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=T,
                    replicas_per_wg=2, threads_per_wg=1024, residency=cosm.RES_LDS)
    info = run_case(inst, colour, C, prob, p, 11, 64, 300, [0, 31, 63])
    assert info["lazy_wrap"] == lazy
    assert info["twist_fused"] == 0
