"""Exact ties of Eq. (4) on the grid schedule, in every LDS sweep form: phases
set to quarter turns plus -1, 0 or +1 grid steps (2^-23 turn), so that many
edges start at x_u - x_v of exactly 0, +-1/4, +-1/2 or one step either side.
On the grid the FP32 kernels take the step's sign from the parity of
floor(2(x_u - x_v)) under round-toward-minus-infinity; the oracle takes it from
fract(x_u - x_v) < 1/2 in FP64.  Both must agree bit for bit on every phase
after a few sweeps (twists included), also where the lazy wrap lets a phase
leave [0, 1) and where the register-owner layouts flip the edge's roles.  FP16
and BF16 storage (FP32 arithmetic, rounded to 16 bits on store) take the same
step in the streamed form; there the device-memory form, which does not,
is the reference."""
import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm
from test_gpu_parity import make, oparams, say

pytestmark = pytest.mark.gpu

STEP = 2.0 ** -23


def tie_phases(n, R, seed):
    """[R][n] turns: k/4 + e 2^-23 (mod 1), k in 0..3, e in -1..1."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 4, size=(R, n))
    e = rng.integers(-1, 2, size=(R, n))
    return np.mod(k / 4.0 + e * STEP, 1.0)


def run(inst, colour, C, prob, p, R, S, seed, want):
    x0 = tie_phases(inst.n, R, seed)
    say(f"[gpu] {inst.name} R={R} S={S} form={p.lds_form} rw={p.replicas_per_wg} "
        f"threads={p.threads_per_wg}")
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed,
                    replicas=R) as st:
        st.set_phases(x0, cosm.UNIT_TURNS, 0)
        st.sweep(1)
        x1 = st.get_phases(cosm.UNIT_TURNS)
        st.sweep(S - 1)
        x = st.get_phases(cosm.UNIT_TURNS)
        info = st.info()
    for key, val in want.items():
        assert info[key] == val, (key, info[key], info)
    op = oparams(p)
    xr = np.ascontiguousarray(x0 * 360.0)
    oracle.sweeps(prob, op, seed, 0, xr, 0, 1)
    assert np.array_equal(x1 * 360.0, xr), "after the first sweep"
    oracle.sweeps(prob, op, seed, 0, xr, 1, S - 1)
    assert np.array_equal(x * 360.0, xr), f"after {S} sweeps"
    # the pattern really holds ties: count the exact ones the first class saw
    d = np.mod(x0[:, inst.eu] - x0[:, inst.ev], 1.0)
    say(f"[ties] {int(np.sum(d == 0.0))} at 0, {int(np.sum(d == 0.5))} at 1/2 of {d.size}")
    assert np.sum(d == 0.0) > 0 and np.sum(d == 0.5) > 0
    return info


@pytest.mark.parametrize("form", [cosm.LDS_FORM_PAIR, cosm.LDS_FORM_REGISTER])
def test_even_torus_pair_and_register(form):
    inst = ci.torus(20, seed=2)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [20, 20])
    p = cosm.Params(sweeps_per_trial=60, dwt_ratio=1.0, dwt_period=3, lds_form=form,
                    residency=cosm.RES_LDS, replicas_per_wg=2, threads_per_wg=256)
    info = run(inst, colour, C, prob, p, 32, 7, 31, {"lds_form": form})
    assert (info["register_rows"] > 0) == (form == cosm.LDS_FORM_REGISTER)


def test_three_regular_register_flips():
    """A non-bipartite graph: register vertices on either end of their edges."""
    inst = ci.random_regular(2000, 3, seed=2)
    colour, C, prob = make(inst, cosm.COLOR_BALANCED)
    p = cosm.Params(sweeps_per_trial=60, dwt_ratio=1.0, dwt_period=6,
                    lds_form=cosm.LDS_FORM_REGISTER, residency=cosm.RES_LDS,
                    replicas_per_wg=2, threads_per_wg=768)
    info = run(inst, colour, C, prob, p, 16, 7, 32, {"lds_form": cosm.LDS_FORM_REGISTER})
    assert info["register_rows"] > 0


def test_streamed_register_owner():
    inst = ci.torus(100, seed=3)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [100, 100])
    p = cosm.Params(sweeps_per_trial=60, dwt_ratio=0.5, dwt_period=3,
                    lds_form=cosm.LDS_FORM_REGISTER_STREAM, residency=cosm.RES_LDS,
                    replicas_per_wg=4, threads_per_wg=640)
    run(inst, colour, C, prob, p, 8, 7, 33,
        {"lds_form": cosm.LDS_FORM_REGISTER_STREAM, "streamed": 1, "lazy_wrap": 1})


@pytest.mark.parametrize("alpha0,lazy", [(14.0, 1), (40.0, 0)], ids=["lazy", "eager"])
def test_streamed_pair_torus141(alpha0, lazy):
    """The headline's form (wrapped at the twists) and, with a step too large
    for the drift bound, the form that wraps after every update."""
    inst = ci.torus(141, seed=4)
    colour, C, prob = make(inst, cosm.COLOR_TORUS, [141, 141])
    p = cosm.Params(alpha0_deg=alpha0, sweeps_per_trial=60, dwt_ratio=0.5, dwt_period=3,
                    residency=cosm.RES_LDS, replicas_per_wg=2, threads_per_wg=1024)
    run(inst, colour, C, prob, p, 4, 7, 34,
        {"lds_form": cosm.LDS_FORM_PAIR, "streamed": 1, "lazy_wrap": lazy})


@pytest.mark.parametrize("storage", [cosm.STORE_FP16, cosm.STORE_BF16])
@pytest.mark.parametrize("alpha0,lazy", [(14.0, 1), (40.0, 0)], ids=["lazy", "eager"])
def test_streamed_pair_sixteen_bit_against_device_memory_form(storage, alpha0, lazy):
    """FP16 and BF16 storage on the grid: the streamed form takes the parity
    step, the device-memory form compares fract(x_u - x_v) with 1/2; from the
    same tie-laden phases both give the same phases bit for bit."""
    inst = ci.torus(141, seed=4)
    colour, C, _ = make(inst, cosm.COLOR_TORUS, [141, 141])
    R, S = 8, 7
    x0 = tie_phases(inst.n, R, 35)
    out = {}
    for res in (cosm.RES_LDS, cosm.RES_HBM):
        p = cosm.Params(alpha0_deg=alpha0, sweeps_per_trial=60, dwt_ratio=0.5, dwt_period=3,
                        storage=storage, residency=res,
                        **({"replicas_per_wg": 4, "threads_per_wg": 1024}
                           if res == cosm.RES_LDS else {}))
        with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=35,
                        replicas=R) as st:
            st.set_phases(x0, cosm.UNIT_TURNS, 0)
            st.sweep(1)
            x1 = st.get_phases(cosm.UNIT_TURNS)
            st.sweep(S - 1)
            out[res] = (x1, st.get_phases(cosm.UNIT_TURNS), st.info())
        say(f"[gpu] storage={storage} residency={res} lazy={out[res][2]['lazy_wrap']} "
            f"streamed={out[res][2]['streamed']}")
        assert out[res][2]["lazy_wrap"] == lazy
    assert out[cosm.RES_LDS][2]["streamed"] == 1
    assert np.array_equal(out[cosm.RES_LDS][0], out[cosm.RES_HBM][0]), "after the first sweep"
    assert np.array_equal(out[cosm.RES_LDS][1], out[cosm.RES_HBM][1]), f"after {S} sweeps"
