"""Pins of the oracle's bias-field dynamics (the virtual-spin reading: h_i is a
coupling of x_i to a fixed spin at phase 0, applied as one more conflict-free
sub-sweep; with fields the twist direction is drawn per event) and of the
QUBO -> Ising mapping at the boundary.  The paper prints nothing for fields
(its instances have h = 0), so these pins are exact invariants, brute-force
ground states and enumeration; the dynamics with h are otherwise parity
unpinned."""
import itertools

import numpy as np
import pytest

import cosm_inputs as ci
import oracle


def _problem(n, eu, ev, J, h):
    colour, C = oracle.greedy_colouring(n, eu, ev)
    return oracle.Problem(n, eu, ev, J, colour=colour, C=C, h=h)


def _enumerate(n, eu, ev, J, h):
    best = None
    for bits in itertools.product((-1, 1), repeat=n):
        s = np.array(bits)
        H = -int((J * s[eu] * s[ev]).sum()) - int((h * s).sum())
        best = H if best is None else min(best, H)
    return best


@pytest.mark.parametrize("sign", [1, -1])
def test_strong_uniform_field_aligns_every_spin(sign):
    """A +-1 ring with h_i = 3 sign: each spin's field beats its two couplings,
    so the unique ground state is s_i = sign.  Pulling x_i towards the virtual
    spin at 0 (or away from it for sign -1) must reach it in nearly every
    trial; the opposite sign of the field term would not."""
    inst = ci.cycle(12, weights="pm1", seed=3)
    h = np.full(inst.n, 3 * sign, np.int32)
    prob = _problem(inst.n, inst.eu, inst.ev, inst.J, h)
    gs_spins, gs = oracle.brute_force_ground_state(prob)
    assert np.all(gs_spins == sign) and gs == _enumerate(inst.n, inst.eu, inst.ev, inst.J, h)
    P = oracle.Params(alpha0_deg=14, dwt_ratio=0.5, dwt_period=3, n_bisectors=1, sweeps=300)
    _, spins, H, _ = oracle.solve(prob, P, seed=5, rid0=0, R=64)
    assert (H == gs).mean() >= 0.9
    assert np.all(spins[H == gs] == sign)


def test_fields_reach_brute_force_ground_state():
    """Random +-1 couplings and fields in {-1, 0, 1} on 14 spins: the best of
    256 trials is the exhaustive ground state."""
    inst = ci.small_random(14, 30, seed=11, weights="pm1")
    rng = np.random.default_rng(4)
    h = rng.integers(-1, 2, inst.n).astype(np.int32)
    prob = _problem(inst.n, inst.eu, inst.ev, inst.J, h)
    _, gs = oracle.brute_force_ground_state(prob)
    assert gs == _enumerate(inst.n, inst.eu, inst.ev, inst.J, h)
    P = oracle.Params(alpha0_deg=14, dwt_ratio=1.5, dwt_period=3, n_bisectors=1, sweeps=1000)
    _, _, H, _ = oracle.solve(prob, P, seed=6, rid0=0, R=256)
    assert H.min() == gs


def test_field_gauge_symmetry_exact():
    """Flip a vertex set G: J' = -J on edges with one end in G, h' = -h on G and
    x' = x + 180 on G.  The field term is an edge to the virtual spin, so the
    trajectory maps exactly (twists included) and the energy is equal."""
    inst = ci.random_regular(40, 3, seed=12, weights="pm1")
    rng = np.random.default_rng(2)
    h = rng.integers(-2, 3, inst.n).astype(np.int32)
    G = rng.random(inst.n) < 0.5
    Jg = inst.J * np.where(G[inst.eu] ^ G[inst.ev], -1, 1).astype(np.int32)
    hg = np.where(G, -h, h).astype(np.int32)
    colour, C = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    p1 = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C, h=h)
    p2 = oracle.Problem(inst.n, inst.eu, inst.ev, Jg, colour=colour, C=C, h=hg)
    P = oracle.Params(alpha0_deg=14, dwt_ratio=1.5, dwt_period=3, n_bisectors=1, sweeps=240)
    x0 = oracle.init_phases(inst.n, 8, 0, 4)
    x0g = x0.copy()
    x0g[:, G] = (x0g[:, G] + 180.0) % 360.0
    x1, x1g = x0.copy(), x0g.copy()
    oracle.sweeps(p1, P, 8, 0, x1, 0, 240)
    oracle.sweeps(p2, P, 8, 0, x1g, 0, 240)
    assert np.array_equal((x1[:, G] + 180.0) % 360.0, x1g[:, G])
    assert np.array_equal(x1[:, ~G], x1g[:, ~G])
    s1, H1, _, _ = oracle.readout(p1, P, x1)
    s2, H2, _, _ = oracle.readout(p2, P, x1g)
    assert np.array_equal(H1, H2)


def test_twist_direction_draw():
    """The drawn twist sense is +-1 with probability 1/2 and independent of the
    reference angle's word (binomial and sign-agreement bounds)."""
    d = np.array([oracle.twist_direction(9, t, r) for t in range(1, 301) for r in range(20)])
    assert set(np.unique(d)) == {-1, 1}
    n = len(d)
    assert abs((d == 1).sum() - n / 2) < 4 * np.sqrt(n / 4)
    th = np.array([oracle.theta_ref(9, t, r) for t in range(1, 301) for r in range(20)])
    agree = ((th < 180.0) == (d == 1)).sum()
    assert abs(agree - n / 2) < 4 * np.sqrt(n / 4)


def test_fields_off_leave_dynamics_unchanged():
    """h = 0 everywhere behaves as no fields in the sweeps (the twist keeps
    its + direction only without fields, so compare with the twist off)."""
    inst = ci.torus(6, seed=2)
    colour, C = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    p0 = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    pz = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C,
                        h=np.zeros(inst.n, np.int32))
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=100)
    x0 = oracle.init_phases(inst.n, 3, 0, 2)
    a, b = x0.copy(), x0.copy()
    oracle.sweeps(p0, P, 3, 0, a, 0, 100)
    oracle.sweeps(pz, P, 3, 0, b, 0, 100)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# QUBO -> Ising at the boundary (host code of the library; no GPU needed)
# ---------------------------------------------------------------------------
def _qubo_energy(x, qi, qj, qv):
    return int(sum(int(v) * int(x[i]) * int(x[j]) for i, j, v in zip(qi, qj, qv)))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_qubo_mapping_by_enumeration(seed):
    """4 E(x) = H(s) + offset for every x in {0,1}^n (n = 10), with repeated,
    reversed and diagonal terms; H from the oracle's energy of Eq. (1)."""
    import paper_2605_30355_amd as cosm
    rng = np.random.default_rng(seed)
    n, nnz = 10, 40
    qi = rng.integers(0, n, nnz).astype(np.int32)
    qj = rng.integers(0, n, nnz).astype(np.int32)
    qj[:6] = qi[:6]  # diagonal terms
    qv = rng.integers(-5, 6, nnz).astype(np.int32)
    eu, ev, J, h, offset = cosm.qubo_to_ising(n, qi, qj, qv)
    assert np.all(eu < ev)
    prob = oracle.Problem(n, eu, ev, J, h=h)
    xs = np.array(list(itertools.product((0, 1), repeat=n)), np.int8)
    H, _ = oracle.energy(prob, (2 * xs - 1).astype(np.int8))
    E = np.array([_qubo_energy(x, qi, qj, qv) for x in xs])
    assert np.array_equal(4 * E, H + offset)


def test_qubo_mapping_errors():
    import paper_2605_30355_amd as cosm
    from paper_2605_30355_amd.cosm import CosmError
    with pytest.raises(CosmError):
        cosm.qubo_to_ising(3, [0], [3], [1])
    eu, ev, J, h, off = cosm.qubo_to_ising(3, [0, 1], [1, 0], [2, -2])  # cancels
    assert len(J) == 0 and off == 0 and np.array_equal(h, [0, 0, 0])
