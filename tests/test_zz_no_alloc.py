"""cosm_init_static (a state whose device buffers live in the library's static
per-device array) against cosm_init: the same trial must give the same
phases, energies, cuts and spins bit for bit, on two calls in a row, the
second with a smaller instance; a second live static state on the device and
an instance too large for the array are refused."""
import sys

import numpy as np
import pytest

import cosm_inputs as ci
import paper_2605_30355_amd as cosm
from paper_2605_30355_amd.cosm import CosmError

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def trial(inst, colour, C, p, seed, R, sweeps, static):
    say(f"[gpu] {'cosm_init_static' if static else 'cosm_init'} {inst.name} R={R} S={sweeps}")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed, replicas=R,
                    static_scratch=static) as st:
        st.sweep(sweeps // 2)
        st.sweep(sweeps - sweeps // 2)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
        info = st.info()
    return x, H, cut, spins, info


def check_pair(inst, colour, C, p, seed, R, sweeps):
    a = trial(inst, colour, C, p, seed, R, sweeps, True)
    b = trial(inst, colour, C, p, seed, R, sweeps, False)
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    return a[4]


def test_static_state_equals_cosm_init_twice():
    # first call: the 3-regular Max-Cut graph, 1024 replicas (about 12 MB of
    # buffers), in the benchmark's shape
    big = ci.random_regular(2000, 3, seed=2, weights="maxcut1")
    colour, C = cosm.build_partitions(big.n, big.eu, big.ev, cosm.COLOR_BALANCED)
    p = cosm.Params(sweeps_per_trial=3000, dwt_ratio=1.0, dwt_period=6, replicas_per_wg=2,
                    threads_per_wg=768)
    info = check_pair(big, colour, C, p, 42, 1024, 3000)
    assert info["residency"] == cosm.RES_LDS
    # second call, smaller: the 20 x 20 torus, 64 replicas, default (untimed) shape
    small = ci.torus(20, seed=1)
    colour, C = cosm.build_partitions(small.n, small.eu, small.ev, cosm.COLOR_TORUS, [20, 20])
    p = cosm.Params(sweeps_per_trial=2000, dwt_ratio=0.5, dwt_period=3)
    check_pair(small, colour, C, p, 7, 64, 2000)


def test_static_state_limits():
    small = ci.torus(8, seed=2)
    colour, C = cosm.build_partitions(small.n, small.eu, small.ev, cosm.COLOR_TORUS, [8, 8])
    p = cosm.Params(sweeps_per_trial=100)
    with cosm.State(small.n, small.eu, small.ev, small.J, colour, C, p, replicas=8,
                    static_scratch=True) as st:
        with pytest.raises(CosmError) as e:  # the array is taken
            cosm.State(small.n, small.eu, small.ev, small.J, colour, C, p, replicas=8,
                       static_scratch=True)
        assert e.value.status == -7
        st.sweep(100)
    # released by cosm_destroy: usable again
    with cosm.State(small.n, small.eu, small.ev, small.J, colour, C, p, replicas=8,
                    static_scratch=True) as st:
        st.sweep(10)
    # larger than the array: refused before any device work
    huge = ci.torus(141, seed=4)
    colour, C = cosm.build_partitions(huge.n, huge.eu, huge.ev, cosm.COLOR_TORUS, [141, 141])
    with pytest.raises(CosmError) as e:
        cosm.State(huge.n, huge.eu, huge.ev, huge.J, colour, C, p, replicas=4096,
                   static_scratch=True)
    assert e.value.status == -4
