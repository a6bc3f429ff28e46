"""Pins of the oracle's relaxed coupling v (Eq. (2)) and relaxed objective f
(Eqs. (3), (7)): a second definition of the angular distance, closed values,
symmetries, agreement with the Ising energy of Eq. (1) at binary phases, and
the descent of f by one sub-sweep of Eq. (6) away from its kinks."""
import numpy as np
import pytest

import cosm_inputs as ci
import oracle

Q_DEG = 360.0 / (1 << 23)


def _v_by_distance(a, b):
    # shortest arc between two points of the circle, by trying the three lifts
    d = min(abs(a - b + 360.0 * k) for k in (-1, 0, 1))
    return 1.0 - d / 90.0


def test_v_closed_values():
    for a in (0.0, 17.5, 179.0, 359.0):
        assert oracle.coupling_v(a, a) == 1.0
        assert oracle.coupling_v(a, (a + 180.0) % 360.0) == -1.0
        assert oracle.coupling_v(a, (a + 90.0) % 360.0) == 0.0
        assert oracle.coupling_v(a, (a + 270.0) % 360.0) == 0.0
    assert oracle.coupling_v(10.0, 350.0) == pytest.approx(1.0 - 20.0 / 90.0, abs=1e-15)
    assert oracle.coupling_v(350.0, 10.0) == pytest.approx(1.0 - 20.0 / 90.0, abs=1e-15)
    assert oracle.coupling_v(0.0, 45.0) == 0.5
    assert oracle.coupling_v(0.0, 135.0) == -0.5


def test_v_matches_shortest_arc_and_symmetries():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        a, b, c = rng.uniform(0.0, 360.0, size=3)
        v = oracle.coupling_v(a, b)
        assert -1.0 <= v <= 1.0
        assert v == pytest.approx(_v_by_distance(a, b), abs=1e-12)
        assert oracle.coupling_v(b, a) == pytest.approx(v, abs=1e-12)
        # periodic in either argument, invariant under a common rotation
        assert oracle.coupling_v(a + 360.0, b) == pytest.approx(v, abs=1e-12)
        assert oracle.coupling_v(a, b - 720.0) == pytest.approx(v, abs=1e-12)
        assert oracle.coupling_v((a + c) % 360.0, (b + c) % 360.0) == pytest.approx(v, abs=1e-11)
        # half a turn on one side flips the sign
        assert oracle.coupling_v((a + 180.0) % 360.0, b) == pytest.approx(-v, abs=1e-11)


@pytest.mark.parametrize("with_h", [False, True])
def test_objective_equals_ising_energy_at_binary_phases(with_h):
    """Phases restricted to 0 (s = +1) and 180 (s = -1) make v = s_i s_j, so f
    is H of Eq. (1) exactly; the field term pins the sign of h."""
    rng = np.random.default_rng(3)
    for inst in (ci.torus(6, seed=2), ci.random_regular(40, 3, seed=5, weights="pm1"),
                 ci.small_random(12, 30, seed=6, weights="pm12")):
        h = rng.integers(-3, 4, size=inst.n).astype(np.int32) if with_h else None
        prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, h=h)
        s = rng.choice(np.array([-1, 1], np.int8), size=(16, inst.n))
        x = np.where(s > 0, 0.0, 180.0)
        f = oracle.relaxed_objective(prob, x)
        H, _ = oracle.energy(prob, s)
        assert np.array_equal(f, H.astype(np.float64)), inst.name
        # a common rotation keeps f without fields (couplings see differences only)
        if not with_h:
            f_rot = oracle.relaxed_objective(prob, (x + 77.25) % 360.0)
            np.testing.assert_allclose(f_rot, f, atol=1e-9)


def test_objective_bounds():
    rng = np.random.default_rng(8)
    inst = ci.random_regular(60, 3, seed=9, weights="pm12")
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J)
    x = rng.uniform(0.0, 360.0, size=(32, inst.n))
    f = oracle.relaxed_objective(prob, x)
    bound = float(np.abs(inst.J).sum())
    assert np.all(f >= -bound - 1e-9) and np.all(f <= bound + 1e-9)
    # all phases equal: every v is 1
    assert oracle.relaxed_objective(prob, np.full(inst.n, 123.0))[0] == -float(inst.J.sum())


@pytest.mark.parametrize("J", [1, -1, 2, -2])
def test_one_subsweep_descends_objective(J):
    """Eq. (6) moves the pair along the selected generalized gradient of f, so
    one edge and one sub-sweep lower f by 2 alpha J^2 / 90 whenever the pair's
    angular distance stays clear of its kinks at 0 and 180 degrees."""
    prob = oracle.Problem(2, [0], [1], [J], colour=[0], C=1)
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=100)
    a = oracle.alpha(P, 1)
    rng = np.random.default_rng(21)
    checked = 0
    for _ in range(400):
        x0 = (rng.integers(0, 1 << 23, size=(1, 2)) * Q_DEG).astype(np.float64)
        d = abs(((x0[0, 0] - x0[0, 1] + 180.0) % 360.0) - 180.0)
        if d < 2 * a * abs(J) + 1e-6 or d > 180.0 - 2 * a * abs(J) - 1e-6:
            continue  # the step would cross a kink
        x1 = x0.copy()
        oracle.sweeps(prob, P, 1, 0, x1, 0, 1)
        f0 = oracle.relaxed_objective(prob, x0)[0]
        f1 = oracle.relaxed_objective(prob, x1)[0]
        assert f1 - f0 == pytest.approx(-2.0 * a * J * J / 90.0, abs=1e-9)
        checked += 1
    assert checked > 100
