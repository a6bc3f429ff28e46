"""Trial statistics on the GPU (Appendix A, Eqs. (15)-(17); Sec. III-B):
cosm_solve_to_target runs successive batches of R replicas (global replica
indices 0, R, 2R, ...) and reports trials, successes, P_s with its Wilson 95%
interval, R99, STT = S R99, t_trial and TTT = t_trial R99, and the best energy,
cut and spins.  Every count and statistic must equal what the same replicas
give when the oracle recomputes them one by one (grid schedule: the energies
are exact, so successes are exact too)."""
import math
import sys

import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm
from stats_util import wilson

pytestmark = pytest.mark.gpu

S, R, TRIALS, SEED = 300, 64, 256, 23


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torus_case():
    inst = ci.torus(20, seed=1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [20, 20])
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    op = oracle.Params(sweeps=S, dwt_ratio=0.5, dwt_period=3)
    say(f"[oracle] torus20 {TRIALS} replicas x {S} sweeps")
    _, spins, H, cut = oracle.solve(prob, op, SEED, 0, TRIALS, n_threads=16)
    return inst, colour, C, spins, H, cut


def expected(H, cut, spins, target, upto):
    """Statistics of replicas 0 .. upto-1 as the oracle gives them."""
    Hs = H[:upto]
    k = int((Hs <= target).sum())
    ps = k / upto
    lo, hi = wilson(k, upto)
    r99 = oracle.r99(ps)
    best = int(np.argmin(Hs))  # the first replica with the lowest energy
    return dict(trials=upto, successes=k, ps=ps, lo=max(0.0, lo), hi=min(1.0, hi), r99=r99,
                best_H=int(Hs[best]), best_cut=int(cut[best]), best_spins=spins[best])


def check(res, best_spins, exp):
    assert res.trials == exp["trials"]
    assert res.successes == exp["successes"]
    assert res.ps == exp["ps"]
    assert res.ps_lo == pytest.approx(exp["lo"], rel=1e-12, abs=1e-15)
    assert res.ps_hi == pytest.approx(exp["hi"], rel=1e-12, abs=1e-15)
    if math.isinf(exp["r99"]):
        assert math.isinf(res.r99) and math.isinf(res.ttt_s) and math.isinf(res.stt_sweeps)
    else:
        assert res.r99 == pytest.approx(exp["r99"], rel=1e-12)
        assert res.stt_sweeps == pytest.approx(S * exp["r99"], rel=1e-12)
        assert res.ttt_s == pytest.approx(res.t_trial_s * exp["r99"], rel=1e-12)
    assert res.t_trial_s > 0.0
    assert res.best_H == exp["best_H"] and res.best_cut == exp["best_cut"]
    assert np.array_equal(best_spins, exp["best_spins"])


def solve(inst, colour, C, target, max_trials, stop):
    p = cosm.Params(sweeps_per_trial=S, dwt_ratio=0.5, dwt_period=3)
    say(f"[gpu] solve_to_target torus20 target={target} max_trials={max_trials} stop={stop}")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=SEED, replicas=R) as st:
        return st.solve_to_target(target, max_trials, stop_at_first_hit=stop)


def test_statistics_equal_oracle_trials(torus_case):
    inst, colour, C, spins, H, cut = torus_case
    target = int(np.quantile(H, 0.25))  # some replicas of every batch reach it
    res, best = solve(inst, colour, C, target, TRIALS, False)
    exp = expected(H, cut, spins, target, TRIALS)
    say(f"P_s {res.successes}/{res.trials}, R99 {res.r99:.3f}, t_trial {res.t_trial_s:.3e} s")
    assert 0 < exp["successes"] < TRIALS
    check(res, best, exp)


def test_stop_at_first_hit(torus_case):
    inst, colour, C, spins, H, cut = torus_case
    target = int(H.min())  # the best energy of the 256 replicas
    first = int(np.nonzero(H <= target)[0][0])
    upto = (first // R + 1) * R  # batches run until the one holding the first hit
    res, best = solve(inst, colour, C, target, TRIALS, True)
    say(f"first hit at replica {first}: {res.trials} trials run")
    check(res, best, expected(H, cut, spins, target, upto))
    # without stopping, all batches run
    res2, best2 = solve(inst, colour, C, target, TRIALS, False)
    check(res2, best2, expected(H, cut, spins, target, TRIALS))


def test_no_success_and_all_success(torus_case):
    """P_s = 0 gives R99 = inf (and TTT, STT inf); P_s = 1 gives R99 = 1."""
    inst, colour, C, spins, H, cut = torus_case
    res, best = solve(inst, colour, C, int(H.min()) - 10**6, 2 * R, False)
    check(res, best, expected(H, cut, spins, int(H.min()) - 10**6, 2 * R))
    assert res.successes == 0 and math.isinf(res.r99)
    res, best = solve(inst, colour, C, 10**6, 2 * R, False)
    check(res, best, expected(H, cut, spins, 10**6, 2 * R))
    assert res.ps == 1.0 and res.r99 == 1.0 and res.stt_sweeps == S
    assert res.ttt_s == res.t_trial_s


def test_ragged_max_trials(torus_case):
    """max_trials not a multiple of R: whole batches run until at least
    max_trials replicas have, so 100 requested gives 128 trials."""
    inst, colour, C, spins, H, cut = torus_case
    target = int(np.quantile(H, 0.5))
    res, best = solve(inst, colour, C, target, 100, False)
    check(res, best, expected(H, cut, spins, target, 128))
