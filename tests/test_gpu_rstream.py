"""The streamed register-owner form of the LDS sweep (an independent set of
vertices in registers, the schedule streamed from memory; the large graphs),
bit-exact against the oracle's grid schedule on sampled replicas: the odd
141 x 141 torus (four register classes, the seams and the rows next to them as
pair slots) with FP32 phases wrapped only at the twists and at every update,
the even 100 x 100 torus at four replicas per workgroup, varying |J|, and a
5-regular graph whose edges outside the register set fill three pair slots
per class."""
import pytest

import cosm_inputs as ci
import paper_2605_30355_amd as cosm
from test_gpu_parity import check_trial, make, say

pytestmark = pytest.mark.gpu


def run(inst, method, sides, p, seed, R, S, rows):
    colour, C, prob = make(inst, method, sides)
    info = check_trial(inst, colour, C, prob, p, seed=seed, R=R, sweeps=S, sample=rows)
    say(f"[gpu]   form={info['lds_form']} rows/thread={info['register_rows']} "
        f"register edges={info['register_edges']} lazy={info['lazy_wrap']}")
    assert info["lds_form"] == cosm.LDS_FORM_REGISTER_STREAM
    assert info["streamed"] == 1
    return info


@pytest.mark.parametrize("period,lazy", [(3, 1), (4, 0)], ids=["lazy-wrap", "wrap-each-update"])
def test_torus141(period, lazy):
    inst = ci.torus(141, seed=4)
    p = cosm.Params(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=period,
                    lds_form=cosm.LDS_FORM_REGISTER_STREAM, replicas_per_wg=2,
                    threads_per_wg=1024, residency=cosm.RES_LDS)
    info = run(inst, cosm.COLOR_TORUS, [141, 141], p, 5, 96, 300, [0, 47, 95])
    assert info["register_rows"] == 10 and info["lazy_wrap"] == lazy


def test_torus100_four_replicas_per_workgroup():
    inst = ci.torus(100, seed=3)
    p = cosm.Params(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3,
                    lds_form=cosm.LDS_FORM_REGISTER_STREAM, replicas_per_wg=4,
                    threads_per_wg=1024, residency=cosm.RES_LDS)
    run(inst, cosm.COLOR_TORUS, [100, 100], p, 6, 70, 300, [0, 35, 69])


def test_varying_coupling_magnitude():
    inst = ci.torus(101, seed=6, weights="pm12")
    p = cosm.Params(alpha0_deg=25.0, sweeps_per_trial=300, dwt_ratio=1.0, dwt_period=3,
                    lds_form=cosm.LDS_FORM_REGISTER_STREAM, replicas_per_wg=2,
                    threads_per_wg=1024, residency=cosm.RES_LDS)
    run(inst, cosm.COLOR_TORUS, [101, 101], p, 7, 64, 300, [0, 31, 63])


def test_five_regular_pair_slots():
    inst = ci.random_regular(20000, 5, seed=1000, weights="pm1")
    p = cosm.Params(sweeps_per_trial=150, dwt_ratio=1.5, dwt_period=3,
                    lds_form=cosm.LDS_FORM_REGISTER_STREAM, replicas_per_wg=2,
                    threads_per_wg=1024, residency=cosm.RES_LDS)
    run(inst, cosm.COLOR_BALANCED, None, p, 8, 64, 150, [0, 63])
