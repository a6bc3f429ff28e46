"""Pins of the oracle's optimal-bisector readout (the exact best line through
the origin among all bisectors, the rounding the paper cites next to its B
equally spaced bisectors): hand-worked cases, the containment of the B-bisector
family, dense sampling of the angle, and the tie rule."""
import numpy as np
import pytest

import cosm_inputs as ci
import oracle


def _H(prob, s):
    H, _ = oracle.energy(prob, s[None, :].astype(np.int8))
    return int(H[0])


def _spins_at(x, beta):
    return np.where(np.mod(x - beta, 360.0) < 180.0, 1, -1).astype(np.int8)


def test_narrow_gap_missed_by_100_bisectors():
    """One antiferromagnetic bond (J = -1) with phases 0.5 and 1.0 degrees: only
    a bisector in (0.5, 1.0] (or its antipode) separates them.  The optimum is
    beta = 1.0, H = -1; none of the 100 bisectors at multiples of 1.8 degrees
    separates them, so that readout gives H = +1."""
    prob = oracle.Problem(2, np.array([0], np.int32), np.array([1], np.int32),
                          np.array([-1], np.int32))
    x = np.array([[0.5, 1.0]])
    s, H, cut, beta = oracle.readout_optimal(prob, x)
    assert H[0] == -1 and cut[0] == 1 and beta[0] == 1.0 and list(s[0]) == [-1, 1]
    _, HB, _, _ = oracle.readout(prob, oracle.Params(n_bisectors=100), x)
    assert HB[0] == 1


def test_tie_takes_the_smallest_angle():
    """A ferromagnetic bond at 10 degrees and an isolated vertex at 5 degrees:
    every bisector gives H = -1, so the smallest candidate angle, 5, is kept."""
    prob = oracle.Problem(3, np.array([0], np.int32), np.array([1], np.int32),
                          np.array([1], np.int32))
    s, H, _, beta = oracle.readout_optimal(prob, np.array([[10.0, 10.0, 5.0]]))
    assert H[0] == -1 and beta[0] == 5.0 and list(s[0]) == [1, 1, 1]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_never_worse_than_bisectors_and_dense_angles(seed):
    """Random phases on a random +-1 graph: the optimum is no worse than the
    100-bisector readout, no angle of a dense sweep (all keys, their
    neighbours, and 20000 uniform angles) does better, and the returned spins
    are those of the returned angle with energy H."""
    inst = ci.small_random(40, 90, seed=seed, weights="pm1")
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J)
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << 15, (3, inst.n)) * (360.0 / (1 << 15))
    s, H, cut, beta = oracle.readout_optimal(prob, x)
    _, HB, _, _ = oracle.readout(prob, oracle.Params(n_bisectors=100), x)
    assert np.all(H <= HB)
    eps = 360.0 / (1 << 20)
    for r in range(x.shape[0]):
        keys = np.mod(x[r], 180.0)
        angles = np.concatenate([keys, keys + eps, keys - eps, rng.random(20000) * 180.0])
        dense = min(_H(prob, _spins_at(x[r], b)) for b in angles)
        assert dense == H[r]
        assert np.array_equal(s[r], _spins_at(x[r], beta[r]))
        assert _H(prob, s[r]) == H[r]
        # cut identity of Appendix A with w = -J
        assert cut[r] == (-int(inst.J.sum()) - H[r]) // 2


def test_rejects_bias_fields():
    prob = oracle.Problem(2, np.array([0], np.int32), np.array([1], np.int32),
                          np.array([1], np.int32), h=np.array([1, 0], np.int32))
    with pytest.raises(ValueError):
        oracle.readout_optimal(prob, np.zeros((1, 2)))
