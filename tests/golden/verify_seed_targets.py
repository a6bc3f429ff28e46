"""Re-evaluate the per-instance targets of the time-to-target study over
instance seeds with the FP64 oracle.

`bench.py --seeds N --seeds-jsonl FILE` appends one record per instance to FILE,
carrying the Ising energy of the instance's best target trial as the GPU
computed it and that trial's spins (packed bits, hex).  This script regenerates
each instance from its seed with the shared seeded generators, evaluates the
same spins with `oracle.energy`, and writes seed_targets.json: per family and
sweep count, each instance's GPU energy, the oracle's energy and whether they
agree.  Calls only oracle/ and the seeded instance generators.

    python tests/golden/verify_seed_targets.py FILE.jsonl [FILE.jsonl ...]
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cosm_inputs as ci  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "seed_targets.json")

# the instance families of the study (the same generator calls and seeds)
FAMILIES = {
    "rr5": lambda s: ci.random_regular(20000, 5, seed=s, weights="pm1"),
    "er": lambda s: ci.erdos_renyi_capped(10000, 4, 8, seed=s),
}


def verify(path):
    out = {}
    with open(path) as f:
        for line in f:
            rec = json.loads(line)
            inst = FAMILIES[rec["family"]](rec["seed"])
            bits = np.unpackbits(np.frombuffer(bytes.fromhex(rec["target_spins_hex"]),
                                               dtype=np.uint8))[:inst.n]
            spins = np.where(bits == 1, 1, -1).astype(np.int8)
            prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J)
            H, _ = oracle.energy(prob, spins)
            key = f"{rec['family']}-{rec['sweeps']}sweeps"
            out.setdefault(key, []).append({"seed": rec["seed"], "target_H": rec["target_H"],
                                            "oracle_H": int(H[0])})
    return out


def main(paths):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for p in paths:
        for key, recs in verify(p).items():
            recs.sort(key=lambda r: r["seed"])
            data[key] = {"instances": len(recs),
                         "all_equal": all(r["target_H"] == r["oracle_H"] for r in recs),
                         "records": recs}
            print(key, len(recs), "instances, all equal:", data[key]["all_equal"])
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
