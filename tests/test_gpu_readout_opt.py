"""The optimal-bisector readout on the GPU (keys, segmented sort, difference
array) against the oracle's brute force over every distinct bisector: exact H,
cut and spins, with ties and repeated keys, and never worse than the 100
bisectors of Algorithm 1 on the same phases."""
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


def _state(inst, colour, C, R, S, readout, seed=3, **kw):
    p = cosm.Params(sweeps_per_trial=S, readout=readout, **kw)
    return cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed, replicas=R)


def _check_against_oracle(inst, colour, C, x_turns, H, cut, spins, rows):
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    so, Ho, co, _ = oracle.readout_optimal(prob, x_turns[rows] * 360.0)
    assert np.array_equal(H[rows], Ho) and np.array_equal(cut[rows], co)
    assert np.array_equal(spins[rows], so)


def test_torus20_trial_matches_oracle():
    inst = ci.torus(20, seed=1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [20, 20])
    with _state(inst, colour, C, 64, 300, cosm.READOUT_OPTIMAL, dwt_ratio=0.5, dwt_period=3) as st:
        st.sweep(300)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
    _check_against_oracle(inst, colour, C, x, H, cut, spins, list(range(64)))


def test_repeated_keys_and_ties():
    """Phases on a coarse grid (many equal keys, including x and x + 180) and
    antipodal duplicates: ranks over distinct keys and the smallest-angle tie
    rule must agree with the oracle."""
    inst = ci.random_regular(200, 3, seed=5, weights="pm1")
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_GREEDY)
    rng = np.random.default_rng(7)
    x = rng.integers(0, 16, (40, inst.n)) * (360.0 / 16)
    x[:5] = 0.0  # every key equal
    with _state(inst, colour, C, 40, 10, cosm.READOUT_OPTIMAL) as st:
        st.set_phases(x, cosm.UNIT_DEGREES, 0)
        H, cut, spins = st.energy()
        xt = st.get_phases(cosm.UNIT_TURNS)
    _check_against_oracle(inst, colour, C, xt, H, cut, spins, list(range(40)))


def test_maxcut_full_size_sampled_and_never_worse():
    """3-regular N = 2000, 1024 replicas after 10^4 sweeps: sampled replicas
    exact against the oracle; every replica's optimal H <= its 100-bisector H."""
    inst = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
    with _state(inst, colour, C, 1024, 10000, cosm.READOUT_OPTIMAL, dwt_ratio=1.0,
                dwt_period=6) as st:
        st.sweep(10000)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
    with _state(inst, colour, C, 1024, 10000, cosm.READOUT_BISECTORS) as sb:
        sb.set_phases(x, cosm.UNIT_TURNS, 10000)
        HB, _, _ = sb.energy(return_spins=False)
    say(f"mean H optimal {H.mean():.2f}  100 bisectors {HB.mean():.2f}; "
        f"better on {(H < HB).sum()} of 1024")
    assert np.all(H <= HB)
    _check_against_oracle(inst, colour, C, x, H, cut, spins, [0, 1, 511, 1023])


def test_optimal_readout_rejects_fields():
    inst = ci.torus(4)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_GREEDY)
    p = cosm.Params(readout=cosm.READOUT_OPTIMAL)
    with pytest.raises(CosmError) as e:
        cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, replicas=2,
                   h=np.ones(inst.n, np.int32))
    assert e.value.status == -1
