"""The multi-instance persistent launch (cosm_batch_*) against single-instance
states and the oracle: instances of uneven sizes, families and parameters run
in one launch must give exactly the trajectories, energies and spins they give
alone (grid schedule), including on replays of the captured hipGraph with new
seeds and subsets of the instances."""
import sys
import time

import numpy as np
import pytest

import cosm_inputs as ci
import oracle
import paper_2605_30355_amd as cosm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def graphs():
    out = []
    t = ci.torus(20, seed=1)
    c, C = cosm.build_partitions(t.n, t.eu, t.ev, cosm.COLOR_TORUS, [20, 20])
    out.append((t, c, C, cosm.Params(sweeps_per_trial=300, dwt_ratio=0.5, dwt_period=3), 11, 64))
    g = ci.random_regular(2000, 3, seed=2)
    c, C = cosm.build_partitions(g.n, g.eu, g.ev, cosm.COLOR_BALANCED)
    out.append((g, c, C, cosm.Params(sweeps_per_trial=200, dwt_ratio=1.0, dwt_period=6), 12, 100))
    g = ci.random_regular(600, 5, seed=3, weights="pm1")
    c, C = cosm.build_partitions(g.n, g.eu, g.ev, cosm.COLOR_GREEDY)
    out.append((g, c, C, cosm.Params(sweeps_per_trial=150, dwt_ratio=1.5, dwt_period=3), 13, 37))
    g = ci.small_random(30, 90, seed=4, weights="pm12")
    c, C = cosm.build_partitions(g.n, g.eu, g.ev, cosm.COLOR_MISRA_GRIES)
    out.append((g, c, C, cosm.Params(sweeps_per_trial=500, dwt_ratio=0.5, dwt_period=2), 14, 5))
    t = ci.torus(141, seed=4)
    c, C = cosm.build_partitions(t.n, t.eu, t.ev, cosm.COLOR_TORUS, [141, 141])
    out.append((t, c, C, cosm.Params(sweeps_per_trial=20, dwt_ratio=0.5, dwt_period=3), 15, 3))
    return out


def single(inst, c, C, p, seed, R, rid0=0):
    with cosm.State(inst.n, inst.eu, inst.ev, inst.J, c, C, p, seed=seed, replicas=R) as st:
        st.reset(seed, rid0)
        st.sweep(p.sweeps_per_trial)
        return st.energy()


@pytest.mark.parametrize("storage", [cosm.STORE_FP32, cosm.STORE_BF16, cosm.STORE_FP16_PK])
def test_batch_equals_single_states(storage):
    gs = graphs()
    with cosm.Batch(storage=storage, max_graphs=16, max_n=20000) as b:
        ids, lazy = [], []
        for inst, c, C, p, seed, R in gs:
            p.storage = storage
            ids.append(b.add(inst.n, inst.eu, inst.ev, inst.J, c, C, p, seed=seed, replicas=R))
            lazy.append(b.shape(ids[-1])["lazy_wrap"])
        say(f"[gpu] batch run of {len(ids)} graphs, storage {storage}, wrapped at the twists only: "
            f"{lazy}")
        # 16-bit phases: the tori stay within the drift bound (T = 3, twist 7 deg,
        # degree 4: 175 deg between wraps), the 3- and 5-regular graphs and the
        # +-2 graph do not; FP32 phases are wrapped after every update here
        assert lazy == ([0] * 5 if storage == cosm.STORE_FP32 else [1, 0, 0, 0, 1])
        b.run(ids)
        ms = b.wait()
        say(f"[gpu] batch took {ms:.2f} ms")
        for gid, (inst, c, C, p, seed, R) in zip(ids, gs):
            H, cut, sp = b.results(gid, return_spins=True)
            Hs, cs, ss = single(inst, c, C, p, seed, R)
            assert np.array_equal(H, Hs) and np.array_equal(cut, cs), inst.name
            assert np.array_equal(sp, ss), inst.name
        # replay the captured graph on a subset with new seeds and replica offsets
        sub = [ids[1], ids[3]]
        b.set_seed(ids[1], 99, 1000)
        b.set_seed(ids[3], 98, 7)
        b.run(sub)
        b.wait()
        for gid, rid0, seed in ((ids[1], 1000, 99), (ids[3], 7, 98)):
            inst, c, C, p, _, R = gs[gid]
            H, cut, _ = b.results(gid)
            Hs, cs, _ = single(inst, c, C, p, seed, R, rid0)
            assert np.array_equal(H, Hs) and np.array_equal(cut, cs), inst.name


def test_batch_matches_oracle_sample():
    inst, c, C, p, seed, R = graphs()[0]
    with cosm.Batch(max_graphs=4, max_n=400) as b:
        gid = b.add(inst.n, inst.eu, inst.ev, inst.J, c, C, p, seed=seed, replicas=R)
        assert b.poll()  # nothing submitted yet
        b.run([gid])
        # the non-blocking poll turns true once the run has drained
        deadline = time.monotonic() + 60.0
        while not b.poll():
            assert time.monotonic() < deadline, "batch run did not finish within 60 s"
            time.sleep(0.001)
        b.wait()
        H, cut, sp = b.results(gid, return_spins=True)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=c, C=C)
    op = oracle.Params(sweeps=p.sweeps_per_trial, dwt_ratio=p.dwt_ratio, dwt_period=p.dwt_period)
    _, so, Ho, co = oracle.solve(prob, op, seed, 0, R)
    assert np.array_equal(H, Ho) and np.array_equal(cut, co) and np.array_equal(sp, so)


def test_batch_shape_tuned_and_cached():
    """The row width of each instance is measured when more than one fits,
    taken from the per-process cache for an identical instance, and fixed by
    replicas_per_wg when given; the tuned shape still gives the single-state
    trajectory."""
    # an instance and sweep count no other test in the process adds (the cache
    # lives as long as the process)
    t = ci.torus(22, seed=41)
    c, C = cosm.build_partitions(t.n, t.eu, t.ev, cosm.COLOR_TORUS, [22, 22])
    p = cosm.Params(sweeps_per_trial=301, dwt_ratio=0.5, dwt_period=3)
    with cosm.Batch(max_graphs=4, max_n=500) as b:
        g0 = b.add(t.n, t.eu, t.ev, t.J, c, C, p, seed=3, replicas=64)
        g1 = b.add(t.n, t.eu, t.ev, t.J, c, C, p, seed=3, replicas=64)
        q = cosm.Params(sweeps_per_trial=301, dwt_ratio=0.5, dwt_period=3, replicas_per_wg=1)
        g2 = b.add(t.n, t.eu, t.ev, t.J, c, C, q, seed=3, replicas=64)
        s0, s1, s2 = b.shape(g0), b.shape(g1), b.shape(g2)
        say(f"[gpu] shapes {s0} {s1} {s2}")
        assert s0["tuned"] == 1 and s0["probe_ms"] > 0.0
        assert s1["tuned"] == 2 and s1["replicas_per_set"] == s0["replicas_per_set"]
        assert s1["probe_ms"] == s0["probe_ms"]
        assert s2["tuned"] == 0 and s2["replicas_per_set"] == 1
        b.run([g0, g1, g2])
        b.wait()
        Hs, cs, ss = single(t, c, C, p, 3, 64)
        for gid in (g0, g1, g2):
            H, cut, sp = b.results(gid, return_spins=True)
            assert np.array_equal(H, Hs) and np.array_equal(cut, cs) and np.array_equal(sp, ss)


# The mixed request stream's workload at full size: the largest request of each
# family (256 replicas x 10^4 sweeps, the families' twist parameters, the
# colourings the stream uses), run together in one batch launch with their
# tuned row widths; sampled replicas (the first and the last of each request)
# against the FP64 oracle.
STREAM_FAMILY_PARAMS = {"torus": dict(dwt_ratio=0.5, dwt_period=3),
                        "3-regular": dict(dwt_ratio=1.0, dwt_period=6),
                        "5-regular": dict(dwt_ratio=1.5, dwt_period=3)}


def test_stream_requests_full_size_sampled():
    from concurrent.futures import ThreadPoolExecutor

    reqs = ci.request_stream(256, 400, 20000, 5)
    largest = {}
    for k, (_, inst) in enumerate(reqs):
        fam = inst.meta["family"]
        if fam not in largest or inst.n > reqs[largest[fam]][1].n:
            largest[fam] = k
    S, R = 10000, 256
    picked = []
    with cosm.Batch(max_graphs=4, max_n=20001) as b:
        for fam, k in sorted(largest.items()):
            inst = reqs[k][1]
            if fam == "torus":
                L = inst.meta["Lx"]
                c, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [L, L])
            else:
                c, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
            p = cosm.Params(sweeps_per_trial=S, **STREAM_FAMILY_PARAMS[fam])
            gid = b.add(inst.n, inst.eu, inst.ev, inst.J, c, C, p, seed=k, replicas=R)
            say(f"[gpu] request {k} ({fam}, n={inst.n}, m={inst.m}): shape {b.shape(gid)}")
            picked.append((gid, k, inst, c, C, fam))
        b.run([g[0] for g in picked])
        say(f"[gpu] batch of {len(picked)} full-size requests took {b.wait():.0f} ms")
        res = {gid: b.results(gid, return_spins=True) for gid, *_ in picked}

    def oracle_one(job):
        gid, k, inst, c, C, fam, r = job
        prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=c, C=C)
        op = oracle.Params(sweeps=S, **STREAM_FAMILY_PARAMS[fam])
        _, so, Ho, co = oracle.solve(prob, op, k, r, 1, n_threads=1)
        return gid, r, so[0], int(Ho[0]), int(co[0])

    jobs = [g + (r,) for g in picked for r in (0, R - 1)]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for gid, r, so, Ho, co in ex.map(oracle_one, jobs):
            H, cut, sp = res[gid]
            say(f"[oracle] graph {gid} replica {r}: H {Ho} (gpu {int(H[r])})")
            assert int(H[r]) == Ho and int(cut[r]) == co and np.array_equal(sp[r], so), (gid, r)
