"""Write tests/golden/targets.json: the best Ising energy the FP64 oracle finds
on each synthetic workload instance, used as the time-to-target goal.

Calls only oracle/ and the seeded instance generators.  The oracle searches with
its own greedy colouring; the target is a property of the instance (its best
known energy), not of the colouring used to find it.

    python tests/golden/make_targets.py [workload ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cosm_inputs as ci  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "targets.json")

# workload -> (instance, params, [(replicas, sweeps_per_trial), ...])
WORKLOADS = {
    "torus20-pm1": (lambda: ci.torus(20, seed=1), dict(dwt_ratio=0.5, dwt_period=3),
                    [(512, 2000), (128, 20000)]),
    "maxcut-3reg-n2000": (lambda: ci.random_regular(2000, 3, seed=2, weights="maxcut1"),
                          dict(dwt_ratio=1.0, dwt_period=6), [(512, 10000), (64, 100000)]),
    # G70-shaped stand-in for the ablation of Table VII: N = 10000, mean degree 2
    # (m ~ 10000), degree cap 9, unweighted Max-Cut
    "maxcut-er-n10000": (lambda: ci.erdos_renyi_capped(10000, 2.0, 9, seed=70, weights="maxcut1"),
                         dict(dwt_ratio=1.0, dwt_period=6), [(256, 10000), (32, 100000)]),
}
# +-1/+-2 tori for the TTS scaling study (the shape of the tile-planted set:
# L x L, periodic, weights in {+-1, +-2}; random, not planted); Appendix C's
# parameters alpha0 = 25, ratio 1.0, period 3
for _L in (12, 14, 16, 18, 20):
    for _s in range(1, 16):
        WORKLOADS[f"torus-pm12-L{_L}-s{_s}"] = (
            (lambda L=_L, sd=_s: ci.torus(L, seed=1000 * L + sd, weights="pm12")),
            dict(alpha0_deg=25.0, dwt_ratio=1.0, dwt_period=3), [(512, 2000), (128, 10000)])


def run(name):
    make, kw, runs = WORKLOADS[name]
    inst = make()
    colour, C = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    rec = {"instance": inst.name, "n": inst.n, "m": inst.m, "sum_w": int(-inst.J.sum()),
           "runs": []}
    best_H, best_cut = None, None
    rid = 0
    for R, S in runs:
        P = oracle.Params(sweeps=S, **kw)
        t0 = time.time()
        _, spins, H, cut = oracle.solve(prob, P, seed=1234, rid0=rid, R=R)
        rid += R
        b = int(H.min())
        rec["runs"].append({"replicas": R, "sweeps": S, "best_H": b,
                            "hits_of_best": int((H == b).sum()), "seconds": round(time.time() - t0, 1),
                            **kw})
        if best_H is None or b < best_H:
            best_H, best_cut = b, int(cut[H == b][0])
        print(name, rec["runs"][-1], flush=True)
    rec["target_H"] = best_H
    rec["target_cut"] = best_cut
    return rec


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {
        "source": "best energy found by the FP64 oracle (tests/golden/make_targets.py), seed 1234"}
    for nm in names:
        data[nm] = run(nm)
        json.dump(data, open(OUT, "w"), indent=1)
