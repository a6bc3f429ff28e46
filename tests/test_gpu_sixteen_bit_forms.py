"""FP16 / BF16 phase storage gives the same trajectory in every form: the
register-resident and streamed LDS forms, the device-memory (HBM) form and the
plain one-replica form all wrap the centred 16-bit values at the twists only
(while no phase can drift by 1/2 turn between two twists), or all at every
update (outside that bound), and round the same FP32 results to 16 bits, so
their phases, energies and spins agree bit for bit.  FP16_PK (FP16 arithmetic)
computes packed on the LDS words and step by step in FP32 with a rounding to
FP16 after each step in the element-wise forms; those agree bit for bit too.  (Parity with the FP64
oracle for these formats is distributional: test_gpu_distribution.py.)"""
import numpy as np
import pytest

import cosm_inputs as ci
import paper_2605_30355_amd as cosm
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def run(inst, colour, C, p, seed, R):
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=seed, replicas=R) as st:
        st.sweep(p.sweeps_per_trial)
        x = st.get_phases(cosm.UNIT_TURNS)
        H, cut, spins = st.energy()
        return x, H, spins, st.info()


@pytest.mark.parametrize("storage", [cosm.STORE_FP16, cosm.STORE_BF16, cosm.STORE_FP16_PK])
@pytest.mark.parametrize("period,lazy", [(3, 1), (6, 0)], ids=["wrap-at-twists", "wrap-each-update"])
def test_forms_agree(storage, period, lazy):
    inst = ci.torus(20, seed=1)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [20, 20])
    R, S = 8, 300
    out = {}
    for res in (cosm.RES_LDS, cosm.RES_HBM, cosm.RES_PLAIN):
        p = cosm.Params(sweeps_per_trial=S, dwt_ratio=0.5, dwt_period=period, storage=storage,
                        residency=res)
        out[res] = run(inst, colour, C, p, 21, R)
        say(f"[gpu] storage={storage} residency={res} lazy={out[res][3]['lazy_wrap']}")
        assert out[res][3]["lazy_wrap"] == lazy
    for res in (cosm.RES_HBM, cosm.RES_PLAIN):
        assert np.array_equal(out[res][0], out[cosm.RES_LDS][0]), res
        assert np.array_equal(out[res][1], out[cosm.RES_LDS][1]), res
        assert np.array_equal(out[res][2], out[cosm.RES_LDS][2]), res


@pytest.mark.parametrize("storage", [cosm.STORE_FP16, cosm.STORE_BF16, cosm.STORE_FP16_PK])
def test_streamed_form_agrees_with_device_memory_form(storage):
    """The 141 x 141 torus: the streamed LDS form against the HBM form."""
    inst = ci.torus(141, seed=4)
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [141, 141])
    R, S = 8, 60
    lds = run(inst, colour, C, cosm.Params(sweeps_per_trial=S, dwt_ratio=0.5, dwt_period=3,
                                           storage=storage, residency=cosm.RES_LDS,
                                           replicas_per_wg=4, threads_per_wg=1024), 22, R)
    hbm = run(inst, colour, C, cosm.Params(sweeps_per_trial=S, dwt_ratio=0.5, dwt_period=3,
                                           storage=storage, residency=cosm.RES_HBM), 22, R)
    assert lds[3]["streamed"] == 1 and lds[3]["lazy_wrap"] == 1 and hbm[3]["lazy_wrap"] == 1
    assert np.array_equal(lds[0], hbm[0])
    assert np.array_equal(lds[1], hbm[1]) and np.array_equal(lds[2], hbm[2])
