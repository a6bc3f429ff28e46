"""Pins of the oracle's 16-bit grid schedule (phases on 360 * 2^-16 degrees,
steps on 360 * 2^-15), the reference for phases held in 16-bit fixed point:
the same draws truncated to 16 bits, the step ramp of Sec. II-B / Appendix B on
the coarser grid, trajectories that stay on the grid, and the two-spin closed
form of Eq. (6) in exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

import cosm_inputs as ci
import oracle

Q16 = Fraction(360, 1 << 16)
Q23 = Fraction(360, 1 << 23)


def _on(v, q):
    return (Fraction(float(v)) / q).denominator == 1


def test_init_is_the_23_bit_draw_truncated():
    x23 = oracle.init_phases(3000, seed=42, rid0=3, R=4)
    x16 = oracle.init_phases(3000, seed=42, rid0=3, R=4, schedule=oracle.SCHED_GRID16)
    assert x16.min() >= 0 and x16.max() < 360
    # w >> 16 == (w >> 9) >> 7: the 16-bit phase is the 23-bit one rounded down
    expect = np.floor(x23 / float(Q16)) * float(Q16)
    assert np.array_equal(x16, expect)
    assert all(_on(v, Q16) for v in x16.ravel()[:500])


def test_theta_is_the_23_bit_draw_truncated():
    for t in range(1, 60):
        for r in range(5):
            a = oracle.theta_ref(9, t, r)
            b = oracle.theta_ref(9, t, r, oracle.SCHED_GRID16)
            assert _on(b, Q16)
            assert b == float(int(Fraction(a) / Q16) * Q16)


def test_alpha_ramp_on_the_coarse_grid():
    S = 777
    P = oracle.Params(alpha0_deg=14.0, sweeps=S, schedule=oracle.SCHED_GRID16)
    a = [Fraction(oracle.alpha(P, t)) for t in range(1, S + 2)]
    assert a[-1] == 0
    assert all(x >= y for x, y in zip(a, a[1:]))
    assert all((v / (2 * Q16)).denominator == 1 for v in a)  # half a step stays on q16
    # alpha0 rounded to the 2 q16 grid, then the ramp rounded: within 2 q16 of the ideal
    for t in (1, 2, 100, 400, 777):
        ideal = Fraction(14) * (S - t + 1) / S
        assert abs(a[t - 1] - ideal) <= 2 * Q16


def test_trajectories_stay_on_the_grid():
    inst = ci.random_regular(200, 3, seed=4, weights="pm1")
    colour, C = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    P = oracle.Params(alpha0_deg=14, dwt_ratio=0.5, dwt_period=3, sweeps=300,
                      schedule=oracle.SCHED_GRID16)
    x = oracle.init_phases(inst.n, 5, 0, 3, schedule=oracle.SCHED_GRID16)
    oracle.sweeps(prob, P, 5, 0, x, 0, 150)
    units = x / float(Q16)
    assert np.array_equal(units, np.round(units))
    assert x.min() >= 0 and x.max() < 360


@pytest.mark.parametrize("J", [1, -2])
def test_two_spin_closed_form_grid16(J):
    prob = oracle.Problem(2, [0], [1], [J], colour=[0], C=1)
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=100, schedule=oracle.SCHED_GRID16)
    alpha = Fraction(oracle.alpha(P, 1))
    rng = np.random.default_rng(8)
    for _ in range(100):
        x0 = [k * Q16 for k in rng.integers(0, 1 << 16, size=2)]
        x = np.array([[float(v) for v in x0]])
        oracle.sweeps(prob, P, 1, 0, x, 0, 1)
        dw = (x0[0] - x0[1] + 180) % 360 - 180
        s = 1 if dw >= 0 else -1
        assert Fraction(x[0, 0]) == (x0[0] - alpha * J * s) % 360
        assert Fraction(x[0, 1]) == (x0[1] + alpha * J * s) % 360
