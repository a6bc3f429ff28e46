"""Bias fields on the GPU (the virtual-spin reading of h; twist direction drawn
per event; single-semicircle readout) against the FP64 oracle, bit-exact in the
grid schedule for every sweep form, and the QUBO boundary mapping used on a
GPU solve."""
import sys

import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _with_fields(inst, seed, lo=-2, hi=2):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, inst.n).astype(np.int32)


def _compare(inst, h, colour, C, params, R, S, seed):
    say(f"[gpu] fields {inst.name} R={R} S={S} res={params.residency} rw={params.replicas_per_wg} "
        f"update={params.update}")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, params, seed=seed, replicas=R,
                    h=h) as st:
        st.sweep(S)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C, h=h)
    op = oracle.Params(alpha0_deg=params.alpha0_deg, dwt_ratio=params.dwt_ratio,
                       dwt_period=params.dwt_period, n_bisectors=1, sweeps=S,
                       update=params.update)
    xo = oracle.init_phases(inst.n, seed, 0, R)
    oracle.sweeps(prob, op, seed, 0, xo, 0, S)
    so, Ho, co, _ = oracle.readout(prob, op, xo)
    assert np.array_equal(x * 360.0, xo)
    assert np.array_equal(H, Ho) and np.array_equal(cut, co) and np.array_equal(spins, so)


@pytest.mark.parametrize("rw", [1, 2, 4])
def test_fields_lds_form_matches_oracle(rw):
    inst = ci.torus(20, seed=1)
    h = _with_fields(inst, 3)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [20, 20])
    p = cosm.Params(sweeps_per_trial=600, dwt_ratio=0.5, dwt_period=3, residency=cosm.RES_LDS,
                    replicas_per_wg=rw)
    _compare(inst, h, colour, C, p, R=40, S=600, seed=12)


@pytest.mark.parametrize("form", ["hbm", "plain", "full_gradient"])
def test_fields_other_forms_match_oracle(form):
    inst = ci.random_regular(300, 3, seed=8, weights="pm1")
    h = _with_fields(inst, 4, -1, 1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_MISRA_GRIES)
    p = cosm.Params(sweeps_per_trial=300, dwt_ratio=1.5, dwt_period=3)
    if form == "hbm":
        p.residency = cosm.RES_HBM
    elif form == "plain":
        p.residency = cosm.RES_PLAIN
    else:
        p.update = cosm.UPDATE_FULL_GRADIENT
    _compare(inst, h, colour, C, p, R=3 if form == "plain" else 65, S=300, seed=13)


def test_fields_large_graph_sampled():
    """N = 10000 torus with fields, the LDS form at two replicas per workgroup."""
    inst = ci.torus(100, seed=3)
    h = _with_fields(inst, 5, -1, 1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [100, 100])
    p = cosm.Params(sweeps_per_trial=60, dwt_ratio=0.5, dwt_period=3)
    _compare(inst, h, colour, C, p, R=8, S=60, seed=14)


def test_qubo_solved_on_gpu():
    """A random 16-variable QUBO through cosm_qubo_to_ising and a GPU solve: the
    best trial's x attains the enumerated minimum of E."""
    import itertools
    rng = np.random.default_rng(21)
    n = 16
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.25]
    qi = np.array([p[0] for p in pairs] + list(range(n)), np.int32)
    qj = np.array([p[1] for p in pairs] + list(range(n)), np.int32)
    qv = rng.integers(-3, 4, len(qi)).astype(np.int32)
    eu, ev, J, h, offset = cosm.qubo_to_ising(n, qi, qj, qv)
    xs = np.array(list(itertools.product((0, 1), repeat=n)), np.int64)
    E = (xs[:, qi] * xs[:, qj] * qv).sum(axis=1)
    colour, C = cosm.build_partitions(n, eu, ev, cosm.COLOR_GREEDY)
    p = cosm.Params(sweeps_per_trial=1000, dwt_ratio=1.5, dwt_period=3)
    with cosm.State(n, eu, ev, J, colour, C, p, seed=3, replicas=256, h=h) as st:
        st.sweep(1000)
        H, _, spins = st.energy()
    k = int(np.argmin(H))
    x = (spins[k].astype(np.int64) + 1) // 2
    e = int((x[qi] * x[qj] * qv).sum())
    assert 4 * e == int(H[k]) + offset
    assert e == int(E.min())
