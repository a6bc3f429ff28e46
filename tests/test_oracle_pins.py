"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these tests compares the oracle with itself or with the HIP path; each
checks a printed value, a closed form, an invariant of the method's equations,
or a brute-force answer computed here by independent means (numpy enumeration,
exact rational arithmetic).
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import cosm_inputs as ci
import oracle

Q_DEG = Fraction(360, 1 << 23)  # grid quantum in degrees


def load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Philox (random numbers the method draws)
# --------------------------------------------------------------------------
def test_philox_known_answer_vectors(golden_dir):
    kat = load(golden_dir, "philox4x32_10_kat.json")
    for v in kat["vectors"]:
        ctr = [int(w, 16) for w in v["ctr"]]
        key = [int(w, 16) for w in v["key"]]
        out = [int(w) for w in oracle.philox4x32_10(ctr, key)]
        assert out == [int(w, 16) for w in v["out"]]


# --------------------------------------------------------------------------
# Greedy colouring, Sec. II-B; partitions, Eqs. (9)-(11)
# --------------------------------------------------------------------------
def test_greedy_hand_worked(golden_dir):
    for case in load(golden_dir, "greedy_small.json")["cases"]:
        e = np.array(case["edges"], dtype=np.int32)
        colour, C = oracle.greedy_colouring(case["n"], e[:, 0], e[:, 1])
        assert colour.tolist() == case["colour"], case["name"]
        assert C == max(case["colour"]) + 1


@pytest.mark.parametrize("inst", [
    ci.torus(6, seed=1), ci.torus(7, seed=2), ci.random_regular(200, 3, seed=4),
    ci.random_regular(300, 5, seed=5, weights="pm1"), ci.erdos_renyi_capped(500, 4, 8, seed=6),
    ci.small_random(30, 120, seed=8)])
def test_greedy_is_proper_and_bounded(inst):
    colour, C = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    delta = int(inst.degrees().max())
    assert oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, colour, C)
    assert delta <= C <= 2 * delta - 1
    # classes are matchings (checked independently here) covering every edge once
    for c in range(C):
        sel = colour == c
        ends = np.concatenate([inst.eu[sel], inst.ev[sel]])
        assert len(np.unique(ends)) == len(ends)
    assert np.bincount(colour, minlength=C).sum() == inst.m


def test_colouring_checker_rejects_planted_mistakes():
    inst = ci.torus(4, seed=3)
    colour, C = oracle.greedy_colouring(inst.n, inst.eu, inst.ev)
    bad = colour.copy()
    # two edges sharing vertex 0 in the same class
    k0, k1 = np.nonzero((inst.eu == 0) | (inst.ev == 0))[0][:2]
    bad[k1] = bad[k0]
    assert not oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, bad, C)
    bad = colour.copy()
    bad[0] = C  # out of range
    assert not oracle.is_proper_colouring(inst.n, inst.eu, inst.ev, bad, C)


def test_table_viii_class_sizes_cover_edges(golden_dir):
    """Table VIII rows sum to |E| of Table III and the greedy used Delta colours."""
    t = load(golden_dir, "paper_printed_values.json")["greedy_class_sizes_table_VIII"]
    for g in ("G61", "G70"):
        assert sum(t[g]["sizes"]) == t[g]["edges"]
        assert len(t[g]["sizes"]) == t[g]["max_degree"]
        assert t[g]["sizes"] == sorted(t[g]["sizes"], reverse=True)  # greedy fills low colours first


# --------------------------------------------------------------------------
# Energy, Eq. (1); cut, Eq. (14) with w = -J (Appendix A)
# --------------------------------------------------------------------------
def _prob(inst, h=None):
    return oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, h=h)


def test_energy_closed_forms():
    fer = ci.torus(4, weights="ferro")
    p = _prob(fer)
    H, cut = oracle.energy(p, np.ones((1, fer.n), np.int8))
    assert H[0] == -fer.m and cut[0] == 0
    for n in (6, 8):
        afm = ci.cycle(n, weights="antiferro")
        alt = np.array([1 if i % 2 == 0 else -1 for i in range(n)], np.int8)
        H, cut = oracle.energy(_prob(afm), alt)
        assert H[0] == -n and cut[0] == n  # every edge cut, weight w = +1
        H, cut = oracle.energy(_prob(afm), np.ones(n, np.int8))
        assert H[0] == n and cut[0] == 0


def test_energy_g70_worked_example(golden_dir):
    """Unweighted graph with 9999 edges: cut 9595 <-> Ising energy -9191."""
    g = load(golden_dir, "paper_printed_values.json")["g70_energy_cut"]
    n = g["n"]
    # a path on n vertices has exactly n - 1 = 9999 edges, like G70
    inst = ci.Instance("path", n, np.arange(n - 1, dtype=np.int32),
                       np.arange(1, n, dtype=np.int32), np.full(n - 1, -g["weight"], np.int32))
    assert inst.m == g["edges"]
    # spins that cut exactly 9595 of the path's edges
    flips = np.zeros(n - 1, bool)
    flips[: g["cut"]] = True
    np.random.default_rng(0).shuffle(flips)
    s = np.ones(n, np.int8)
    for k in range(n - 1):
        s[k + 1] = -s[k] if flips[k] else s[k]
    H, cut = oracle.energy(_prob(inst), s)
    assert cut[0] == g["cut"]
    assert H[0] == g["ising_energy"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_energy_cut_identity_and_flip_symmetry(seed):
    inst = ci.small_random(40, 150, seed=seed)
    p = _prob(inst)
    rng = np.random.default_rng(seed)
    s = rng.choice(np.array([-1, 1], np.int8), size=(16, inst.n))
    H, cut = oracle.energy(p, s)
    W = -int(inst.J.sum())
    assert np.array_equal(2 * cut, W - H)  # cut = (sum w - H)/2 with h = 0
    H2, _ = oracle.energy(p, -s)
    assert np.array_equal(H, H2)
    h = rng.integers(-3, 4, size=inst.n).astype(np.int32)
    ph = _prob(inst, h=h)
    Hh, _ = oracle.energy(ph, s)
    Hh2, _ = oracle.energy(ph, -s)
    assert np.array_equal(Hh - Hh2, -2 * (s.astype(np.int64) @ h.astype(np.int64)))


def _numpy_exhaustive_min(inst, h=None):
    n = inst.n
    codes = np.arange(1 << n, dtype=np.int64)
    S = 1 - 2 * ((codes[:, None] >> np.arange(n)) & 1)  # [2^n, n]
    E = -(S[:, inst.eu] * S[:, inst.ev] * inst.J[None, :].astype(np.int64)).sum(1)
    if h is not None:
        E -= S @ h.astype(np.int64)
    return int(E.min())


@pytest.mark.parametrize("inst", [ci.torus(4, seed=9), ci.random_regular(20, 3, seed=11, weights="pm1"),
                                  ci.small_random(14, 30, seed=12), ci.trap_triangle()])
def test_brute_force_ground_state(inst):
    s, H = oracle.brute_force_ground_state(_prob(inst))
    assert H == _numpy_exhaustive_min(inst)
    Hs, _ = oracle.energy(_prob(inst), s)
    assert Hs[0] == H


def test_brute_force_closed_forms():
    assert oracle.brute_force_ground_state(_prob(ci.torus(4, weights="ferro")))[1] == -32
    assert oracle.brute_force_ground_state(_prob(ci.cycle(5, weights="antiferro")))[1] == -3
    s, H = oracle.brute_force_ground_state(_prob(ci.trap_triangle()))
    assert H == -3 and s.tolist() in ([1, -1, -1], [-1, 1, 1])  # Fig. 2 ground states


# --------------------------------------------------------------------------
# Trial statistics, Appendix A, Eqs. (15)-(17)
# --------------------------------------------------------------------------
def test_r99_table_ii_and_sts(golden_dir):
    for row in load(golden_dir, "paper_printed_values.json")["r99_table_II"]["rows"]:
        ps = row["successes"] / row["trials"]
        assert round(ps, 4) == pytest.approx(row["ps_printed"], abs=1e-9)
        r = oracle.r99(ps)
        assert round(r, 2) == pytest.approx(row["r99"], abs=1e-9)
        # STS = S_trial * R99, printed to 0.1 M (within one unit of the last
        # printed digit: the paper rounds its intermediate values)
        assert abs(row["sweeps_per_trial"] * r / 1e6 - row["sts_millions"]) <= 0.1 + 1e-9


def test_r99_table_vi_and_stt(golden_dir):
    for row in load(golden_dir, "paper_printed_values.json")["r99_table_VI"]["rows"]:
        r = oracle.r99(row["ps"])
        assert round(r, 1) == pytest.approx(row["r99"], abs=1e-9)
        stt = row["sweeps_per_trial"] * r / 1e6
        assert abs(stt - row["stt_millions"]) <= 0.5 * row["stt_printed_step"] + 1e-9


def test_tts_is_t_trial_times_r99(golden_dir):
    for row in load(golden_dir, "paper_printed_values.json")["tts_sec_III_A"]["rows"]:
        # t_trial is printed to 0.01 s, so the product is known to +-0.005 * R99
        assert abs(row["t_trial_s"] * row["r99"] - row["tts_s"]) <= 0.005 * row["r99"] + 0.05


def test_r99_sec_iii_c_and_edges(golden_dir):
    g = load(golden_dir, "paper_printed_values.json")["sts_sec_III_C"]
    assert round(g["sweeps_per_trial"] * oracle.r99(g["ps"]), -3) == g["sts"]
    assert oracle.r99(1.0) == 1.0
    assert oracle.r99(0.0) == float("inf")


# --------------------------------------------------------------------------
# Schedule, bisectors, initial state
# --------------------------------------------------------------------------
def test_alpha_schedule_linear_ramp(golden_dir):
    tab = load(golden_dir, "paper_printed_values.json")["parameters_tables_IX_X"]
    S = 1000
    for sched in (oracle.SCHED_GRID, oracle.SCHED_CONTINUOUS):
        P = oracle.Params(alpha0_deg=tab["alpha0_deg"], sweeps=S, schedule=sched)
        a = np.array([oracle.alpha(P, t) for t in range(1, S + 2)])
        assert abs(a[0] - tab["alpha0_deg"]) <= float(Q_DEG)
        assert a[-1] == tab["final_alpha_deg"]  # value after the last sweep
        assert np.all(np.diff(a) <= 0)
        ideal = tab["alpha0_deg"] * (S - np.arange(1, S + 2) + 1) / S
        # grid: alpha0 rounded to the 2q step (<= q) plus the ramp rounded (<= q)
        assert np.max(np.abs(a - ideal)) <= 2 * float(Q_DEG)
        if sched == oracle.SCHED_GRID:  # on the 2q grid, so half a step is on the q grid
            for v in a[:50]:
                assert (Fraction(v) / (2 * Q_DEG)).denominator == 1


def test_bisectors_cover_semicircle(golden_dir):
    tab = load(golden_dir, "paper_printed_values.json")["parameters_tables_IX_X"]
    P = oracle.Params(n_bisectors=tab["bisectors"])
    for sched in (oracle.SCHED_GRID, oracle.SCHED_CONTINUOUS):
        P.schedule = sched
        b = np.array([oracle.bisector(P, k) for k in range(P.n_bisectors)])
        assert b[0] == 0.0
        assert np.max(np.abs(b - tab["bisector_spacing_deg"] * np.arange(P.n_bisectors))) <= float(Q_DEG)
        assert b[-1] + tab["bisector_spacing_deg"] == pytest.approx(180.0, abs=1e-4)


def test_init_phases_on_grid_and_uniform():
    from scipy import stats
    x = oracle.init_phases(5000, seed=42, rid0=0, R=20)
    assert x.min() >= 0 and x.max() < 360
    units = x / float(Q_DEG)
    assert np.array_equal(units, np.round(units))
    assert stats.kstest(x.ravel() / 360.0, "uniform").pvalue > 1e-3
    xc = oracle.init_phases(5000, seed=42, rid0=0, R=2, schedule=oracle.SCHED_CONTINUOUS)
    assert np.max(np.abs(xc - x[:2])) < float(Q_DEG)  # same draw, one more bit
    # replicas and seeds give different streams
    assert not np.array_equal(x[0], x[1])
    assert not np.array_equal(x[0], oracle.init_phases(5000, seed=43, rid0=0, R=1)[0])
    assert np.array_equal(x[5], oracle.init_phases(5000, seed=42, rid0=5, R=1)[0])


def test_theta_ref_on_grid_and_uniform():
    from scipy import stats
    th = np.array([oracle.theta_ref(7, t, r) for t in range(1, 400) for r in range(10)])
    assert th.min() >= 0 and th.max() < 360
    assert stats.kstest(th / 360.0, "uniform").pvalue > 1e-3
    units = th / float(Q_DEG)
    assert np.array_equal(units, np.round(units))


# --------------------------------------------------------------------------
# Sweep invariants: Eqs. (4)-(6), (12)-(13), the dual window twist
# --------------------------------------------------------------------------
def _run(prob, params, x0, n_sweeps, seed=1, rid0=0, t_from=0):
    x = np.array(x0, dtype=np.float64, copy=True)
    oracle.sweeps(prob, params, seed, rid0, x, t_from, n_sweeps)
    return x


def _frac_mod(v, period):
    return v - period * (v // period)


def test_two_spin_closed_form():
    """One edge, one sweep, exact rational arithmetic: the pair difference moves
    by -2 alpha J sgn_b(dw) and the pair sum is conserved mod 360."""
    inst = ci.Instance("pair", 2, np.array([0], np.int32), np.array([1], np.int32),
                       np.array([1], np.int32))
    rng = np.random.default_rng(5)
    for J in (1, -1, 2, -2):
        inst.J[0] = J
        prob = oracle.Problem(2, inst.eu, inst.ev, inst.J, colour=[0], C=1)
        P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=100)
        alpha = Fraction(oracle.alpha(P, 1))
        for _ in range(200):
            x0 = rng.integers(0, 1 << 23, size=2) * Q_DEG
            x1 = _run(prob, P, [[float(v) for v in x0]], 1)[0]
            dw = _frac_mod(x0[0] - x0[1] + 180, 360) - 180
            s = 1 if dw >= 0 else -1
            exp_u = _frac_mod(x0[0] - alpha * J * s, 360)
            exp_v = _frac_mod(x0[1] + alpha * J * s, 360)
            assert Fraction(x1[0]) == exp_u and Fraction(x1[1]) == exp_v
            assert _frac_mod(Fraction(x1[0]) + Fraction(x1[1]) - x0[0] - x0[1], 360) == 0


def test_ties_follow_biased_sign():
    """dw = 0 -> sgn_b = +1 (Eq. (4)); dw = +-180 wraps to -180 -> -1."""
    prob = oracle.Problem(2, [0], [1], [1], colour=[0], C=1)
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=100)
    a = oracle.alpha(P, 1)
    x = _run(prob, P, [[100.0, 100.0]], 1)[0]
    assert x[0] == 100.0 - a and x[1] == 100.0 + a  # J=+1, s=+1: u moves down, v up
    x = _run(prob, P, [[280.0, 100.0]], 1)[0]  # difference +180 -> -180 -> s = -1
    assert x[0] == 280.0 + a and x[1] == 100.0 - a
    x = _run(prob, P, [[100.0, 280.0]], 1)[0]  # difference -180 -> s = -1
    assert x[0] == 100.0 + a and x[1] == 280.0 - a


def _circ(a, b):
    d = np.abs(a - b) % 360.0
    return np.minimum(d, 360.0 - d)


@pytest.mark.parametrize("J", [1, -1, 2])
def test_single_class_step_magnitude(J):
    """A perfect matching is one class: one sweep moves every spin by alpha*|J|."""
    n = 64
    eu = np.arange(0, n, 2, dtype=np.int32)
    ev = eu + 1
    prob = oracle.Problem(n, eu, ev, np.full(len(eu), J, np.int32), colour=np.zeros(len(eu)), C=1)
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=50)
    x0 = oracle.init_phases(n, 3, 0, 4)
    x1 = _run(prob, P, x0, 1)
    assert np.all(_circ(x1, x0) == oracle.alpha(P, 1) * abs(J))


def test_alpha_zero_is_identity():
    inst = ci.torus(6, seed=4)
    prob = _prob(inst)
    P = oracle.Params(alpha0_deg=0.0, dwt_ratio=1.5, dwt_period=1, sweeps=40)
    x0 = oracle.init_phases(inst.n, 5, 0, 3)
    assert np.array_equal(_run(prob, P, x0, 40), x0)


@pytest.mark.parametrize("inst", [ci.torus(8, seed=2), ci.random_regular(60, 3, seed=3, weights="pm1"),
                                  ci.torus(5, seed=6, weights="pm12")])
def test_sum_of_phases_conserved_by_subsweeps(inst):
    prob = _prob(inst)
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=200)
    x0 = oracle.init_phases(inst.n, 9, 0, 4)
    x1 = _run(prob, P, x0, 200)
    for r in range(4):
        d = sum(Fraction(v) for v in x1[r]) - sum(Fraction(v) for v in x0[r])
        assert _frac_mod(d, 360) == 0


def test_dwt_rotates_exactly_the_window_members():
    """No edges: each sweep is only the twist.  Members (computed here in exact
    arithmetic) rotate by ratio*alpha; the rest stay; the two windows cover
    exactly half of the circle (Sec. II-D)."""
    n = 1024
    prob = oracle.Problem(n, [], [], [], colour=[], C=0)
    seed, ratio = 11, 1.5
    P = oracle.Params(alpha0_deg=14, dwt_ratio=ratio, dwt_period=1, sweeps=10)
    x0 = np.array([[360.0 * k / n for k in range(n)]])  # evenly spaced on the circle
    for t in range(1, 6):
        x1 = _run(prob, P, x0, 1, seed=seed, t_from=t - 1)
        theta = Fraction(oracle.theta_ref(seed, t, 0))
        tw = Fraction(ratio) * Fraction(oracle.alpha(P, t))
        inside = [_frac_mod(Fraction(v) - theta + 45, 180) < 90 for v in x0[0]]
        assert sum(inside) == n // 2
        for k in range(n):
            want = _frac_mod(Fraction(x0[0, k]) + (tw if inside[k] else 0), 360)
            assert Fraction(x1[0, k]) == want


def test_gauge_symmetry_exact():
    """Flip a vertex set G: J' = -J on edges with one end in G and x' = x + 180
    on G.  The trajectory maps exactly, twist included, and H is equal."""
    inst = ci.torus(6, seed=8)
    rng = np.random.default_rng(1)
    G = rng.random(inst.n) < 0.5
    Jg = inst.J * np.where(G[inst.eu] ^ G[inst.ev], -1, 1).astype(np.int32)
    p1 = _prob(inst)
    p2 = oracle.Problem(inst.n, inst.eu, inst.ev, Jg, colour=p1.colour, C=p1.C)
    P = oracle.Params(alpha0_deg=14, dwt_ratio=0.5, dwt_period=3, sweeps=300)
    x0 = oracle.init_phases(inst.n, 4, 0, 3)
    x0g = x0.copy()
    x0g[:, G] = (x0g[:, G] + 180.0) % 360.0
    x1 = _run(p1, P, x0, 300, seed=4)
    x1g = _run(p2, P, x0g, 300, seed=4)
    assert np.array_equal((x1[:, G] + 180.0) % 360.0, x1g[:, G])
    assert np.array_equal(x1[:, ~G], x1g[:, ~G])
    _, H1, _, _ = oracle.readout(p1, P, x1)
    _, H2, _, _ = oracle.readout(p2, P, x1g)
    assert np.array_equal(H1, H2)


def test_rotation_commutes_with_scs():
    inst = ci.random_regular(50, 3, seed=9, weights="pm1")
    prob = _prob(inst)
    P = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=100)
    x0 = oracle.init_phases(inst.n, 2, 0, 2)
    c = 123.0 + float(Q_DEG) * 77
    a = (_run(prob, P, x0, 100) + c) % 360.0
    b = _run(prob, P, (x0 + c) % 360.0, 100)
    assert np.array_equal(a, b)


def test_conflict_trap_triangle():
    """Figs. 2 and 4: from a force-cancelling state the full gradient (Eq. (8))
    stays frozen, while sequential conflict-free search reaches the ground
    state in one sweep.  The paper's figure values are not available; this
    state is constructed (zero full gradient at every spin)."""
    inst = ci.trap_triangle()
    prob = _prob(inst)
    x0 = np.array([[0.0, 15.0, 0.0]])
    Pf = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=1000, update=oracle.UPDATE_FULL_GRADIENT)
    Ps = oracle.Params(alpha0_deg=14, dwt_period=0, sweeps=1000)
    assert np.array_equal(_run(prob, Pf, x0, 50), x0)
    _, Hf, _, _ = oracle.readout(prob, Ps, x0)
    assert Hf[0] == 1  # frozen above the ground state
    _, Hs, _, _ = oracle.readout(prob, Ps, _run(prob, Ps, x0, 1))
    assert Hs[0] == -3


def test_resume_equals_one_run():
    inst = ci.torus(6, seed=1)
    prob = _prob(inst)
    P = oracle.Params(alpha0_deg=14, dwt_period=3, sweeps=100)
    x0 = oracle.init_phases(inst.n, 1, 0, 2)
    a = _run(prob, P, x0, 60)
    b = _run(prob, P, _run(prob, P, x0, 31), 29, t_from=31)
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# Readout, Algorithm 1 (binarization) and Appendix B
# --------------------------------------------------------------------------
def test_readout_two_clusters():
    """Two antipodal clusters are separated by some bisector: H equals the energy
    of the cluster labelling, which for these instances is the ground state."""
    for inst, lab in ((ci.torus(4, weights="ferro"), np.ones(16, np.int8)),
                      (ci.cycle(8, weights="antiferro"), np.array([1, -1] * 4, np.int8))):
        prob = _prob(inst)
        P = oracle.Params()
        x = np.where(lab > 0, 37.0, 217.0)[None, :]
        spins, H, cut, _ = oracle.readout(prob, P, x)
        assert H[0] == -inst.m
        assert np.array_equal(spins[0], lab) or np.array_equal(spins[0], -lab)
        He, ce = oracle.energy(prob, spins)
        assert He[0] == H[0] and ce[0] == cut[0]


def test_readout_not_below_ground_state_and_consistent():
    inst = ci.random_regular(16, 3, seed=2, weights="pm1")
    prob = _prob(inst)
    _, gs = oracle.brute_force_ground_state(prob)
    P = oracle.Params(sweeps=300, dwt_ratio=1.5, dwt_period=3)
    x, spins, H, cut = oracle.solve(prob, P, seed=3, rid0=0, R=16)
    assert np.all(H >= gs)
    He, ce = oracle.energy(prob, spins)
    assert np.array_equal(He, H) and np.array_equal(ce, cut)
    assert np.any(H == gs)  # a 16-spin instance is solved by some of 16 trials


def test_readout_lowest_index_on_ties():
    inst = ci.torus(4, weights="ferro")
    prob = _prob(inst)
    x = np.full((1, inst.n), 100.0)  # every bisector before 100 and after 100-180 ties
    _, H, _, bp = oracle.readout(prob, oracle.Params(), x)
    assert H[0] == -inst.m and bp[0] == 0


def test_tts_scaling_fit_reproduces_appendix_c(golden_dir):
    """The fit of log10 TTS = a + b L used by bench.py's scaling study, on the
    median TTS values Appendix C prints for L = 12..20, gives the printed
    slope 0.139, R^2 0.981 and 95 % interval 0.104-0.175."""
    import bench
    ref = load(golden_dir, "paper_printed_values.json")["tts_scaling_appendix_C"]
    fit = bench.fit_log_tts(ref["L"], ref["tts_ms"])
    assert abs(fit["b"] - ref["slope_b"]) < 5e-4
    assert abs(fit["r_squared"] - ref["r_squared"]) < 5e-4
    assert abs(fit["b_ci95"][0] - ref["slope_ci95"][0]) < 1.5e-3
    assert abs(fit["b_ci95"][1] - ref["slope_ci95"][1]) < 1.5e-3
