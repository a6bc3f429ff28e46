"""The oracle's check of the time-to-target study's targets
(tests/golden/verify_seed_targets.py): the verifier decodes the packed spins the
way bench.py writes them and catches a wrong energy; and every recorded target
in tests/golden/seed_targets.json equals the oracle's energy of its spins."""
import json
import os
import sys

import numpy as np
import pytest

import cosm_inputs as ci
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import verify_seed_targets as vst  # noqa: E402


def test_verifier_decodes_bench_records(tmp_path):
    inst = ci.erdos_renyi_capped(10000, 4, 8, seed=1003)
    rng = np.random.default_rng(7)
    spins = rng.choice(np.array([-1, 1], dtype=np.int8), size=inst.n)
    H, _ = oracle.energy(oracle.Problem(inst.n, inst.eu, inst.ev, inst.J), spins)
    hexbits = np.packbits(spins > 0).tobytes().hex()  # as bench.py writes them
    path = tmp_path / "er.jsonl"
    with open(path, "w") as f:
        f.write(json.dumps({"seed": 1003, "family": "er", "sweeps": 10000,
                            "target_H": int(H[0]), "target_spins_hex": hexbits}) + "\n")
        # a wrong energy (a planted mistake) must show as a mismatch
        f.write(json.dumps({"seed": 1003, "family": "er", "sweeps": 1,
                            "target_H": int(H[0]) + 4, "target_spins_hex": hexbits}) + "\n")
    out = vst.verify(str(path))
    assert out["er-10000sweeps"][0]["oracle_H"] == out["er-10000sweeps"][0]["target_H"]
    assert out["er-1sweeps"][0]["oracle_H"] != out["er-1sweeps"][0]["target_H"]


def test_recorded_targets_equal_the_oracle():
    if not os.path.exists(vst.OUT):
        pytest.skip("no recorded study")
    with open(vst.OUT) as f:
        data = json.load(f)
    assert data
    for key, entry in data.items():
        assert entry["instances"] == len(entry["records"]) > 0, key
        for r in entry["records"]:
            assert r["target_H"] == r["oracle_H"], (key, r)
        assert entry["all_equal"], key
