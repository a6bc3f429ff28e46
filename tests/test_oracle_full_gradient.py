"""Pins of the oracle's full-gradient update (Eq. (8), the "without SCS" row of
Table VII) that a sign error, a dropped contribution or a swapped endpoint
fails:

- on a graph whose edges form one matching, Eq. (8) and one sub-sweep of
  Eq. (6) are the same map (every variable has at most one contribution), so
  a full-gradient sweep must equal an SCS sweep bit for bit, twist included;
- away from the kinks of v (Eq. (2)), one Eq. (8) step with the selected
  generalized gradient of Eq. (5) changes the relaxed objective f of Eq. (7)
  by exactly -(alpha / 90) sum_i g_i^2, where g_i is the (unscaled) sum of
  J_k s_k over the edges at i, signed by i's role; gradient ascent would raise
  f by the same amount.
"""
import numpy as np
import pytest

import cosm_inputs as ci
import oracle

Q_DEG = 360.0 / (1 << 23)


def _matching(n, seed, weights):
    """n/2 disjoint edges on a random pairing of the vertices, random roles."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    eu = perm[0::2].astype(np.int32)
    ev = perm[1::2].astype(np.int32)
    J = rng.choice(np.array(weights, np.int32), size=len(eu))
    return eu, ev, J


@pytest.mark.parametrize("weights,period", [((-1, 1), 0), ((-2, -1, 1, 2), 0),
                                            ((-1, 1), 1), ((-2, 1, 2), 2)])
def test_full_gradient_equals_scs_on_one_matching(weights, period):
    n = 96
    eu, ev, J = _matching(n, seed=len(weights) + 10 * period, weights=weights)
    colour = np.zeros(len(eu), np.int32)
    prob = oracle.Problem(n, eu, ev, J, colour=colour, C=1)
    S = 40
    Ps = oracle.Params(alpha0_deg=14, dwt_ratio=0.5, dwt_period=period, sweeps=S)
    Pf = oracle.Params(alpha0_deg=14, dwt_ratio=0.5, dwt_period=period, sweeps=S,
                       update=oracle.UPDATE_FULL_GRADIENT)
    x0 = oracle.init_phases(n, 5, 0, 6)
    xs, xf = x0.copy(), x0.copy()
    oracle.sweeps(prob, Ps, 5, 0, xs, 0, S)
    oracle.sweeps(prob, Pf, 5, 0, xf, 0, S)
    assert not np.array_equal(xs, x0)
    assert np.array_equal(xs, xf)
    # and one sweep at a time, from the same start
    xs1, xf1 = x0.copy(), x0.copy()
    oracle.sweeps(prob, Ps, 5, 0, xs1, 0, 1)
    oracle.sweeps(prob, Pf, 5, 0, xf1, 0, 1)
    assert np.array_equal(xs1, xf1)


def _signed_gradient(eu, ev, J, x):
    """g_i = sum over edges k at i of J_k s_k (+1 for i = u_k, -1 for i = v_k),
    s_k = sgn_b of the minimum angular difference x_u - x_v (Eqs. (4), (5))."""
    d = x[eu] - x[ev]
    dw = d - 360.0 * np.floor((d + 180.0) / 360.0)
    s = np.where(dw >= 0.0, 1.0, -1.0)
    g = np.zeros(len(x))
    np.add.at(g, eu, J * s)
    np.add.at(g, ev, -J * s)
    return g, dw


@pytest.mark.parametrize("name,inst", [
    ("3reg-pm1", ci.random_regular(30, 3, seed=4, weights="pm1")),
    ("3reg-pm12", ci.random_regular(24, 3, seed=6, weights="pm12")),
    ("small-pm12", ci.small_random(14, 20, seed=3, weights="pm12")),
])
def test_full_gradient_step_descends_objective_exactly(name, inst):
    S = 1000
    P = oracle.Params(alpha0_deg=0.25, dwt_period=0, sweeps=S, update=oracle.UPDATE_FULL_GRADIENT)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J,
                          colour=np.zeros(inst.m, np.int32), C=1)
    a = oracle.alpha(P, 1)
    J = inst.J.astype(np.float64)
    rng = np.random.default_rng(17)
    checked = 0
    for _ in range(600):
        x0 = (rng.integers(0, 1 << 23, size=(1, inst.n)) * Q_DEG).astype(np.float64)
        g, dw = _signed_gradient(inst.eu, inst.ev, J, x0[0])
        # the change of every pair's difference under Eq. (8)
        dx = -a * g
        ddiff = np.abs(dx[inst.eu] - dx[inst.ev])
        clear = (np.abs(dw) > ddiff + 1e-9) & (180.0 - np.abs(dw) > ddiff + 1e-9)
        if not clear.all():
            continue  # some pair would cross a kink of v
        x1 = x0.copy()
        oracle.sweeps(prob, P, 1, 0, x1, 0, 1)
        f0 = oracle.relaxed_objective(prob, x0)[0]
        f1 = oracle.relaxed_objective(prob, x1)[0]
        predicted = -(a / 90.0) * float((g * g).sum())
        assert predicted < 0.0
        assert f1 - f0 == pytest.approx(predicted, abs=1e-9), name
        # the step itself: every variable moved by -alpha g_i (mod 360)
        moved = (x1[0] - x0[0] + 180.0) % 360.0 - 180.0
        np.testing.assert_allclose(moved, dx, atol=1e-9)
        checked += 1
    assert checked >= 40, checked
