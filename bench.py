#!/usr/bin/env python3
"""Benchmark of the Cosm sweep on one MI355X.

A step is one whole trial batch of the hot path on the largest single-GPU
workload: the 141 x 141 +-1 toroidal spin glass (N = 19881, 39762 edges, the
torus colouring's 6 classes, 4096 replicas, FP32 phases, grid schedule, 10^4
sweeps): phase init, the sweeps (SCS sub-sweeps, twist, schedule) and the
bisector readout with int64 energies.

Prints one JSON line: edge-updates/s of the batched LDS-resident form (value),
replica-sweeps/s, the roofline of the sweep kernel, and the CPU oracle timed on
the host on a bounded sample of the same workload.  Extra keys: the Max-Cut
workload (random 3-regular, N = 2000, 1024 replicas, 10^4 sweeps) with the
plain one-replica-per-launch form and time-to-target at 99% for the batched,
plain and reduced-precision forms; the other large graphs' sweep rates.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz.  LDS peak taken as 128 B/clk/CU (the CDNA figure;
# 78.6 TB/s).  On gfx950 conflict-free reads measure up to ~190 B/clk/CU and
# writes ~72-78 B/clk/CU, so the sweep's 50/50 read/write mix has a lower
# measured ceiling, which the run also reports (cosm_lds_probe).
LDS_PEAK_GBS = 128 * 256 * 2.4          # 78643 GB/s
HBM_PEAK_GBS = 8000.0
VALU_PEAK_OPS = 256 * 64 * 2.4e9        # lane-ops per second, non-packed FP32

# HBM bytes per launch of the sweep kernel at this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the counter
# reads for a 256 MiB device copy (FETCH_SIZE 131087 KiB -> x2.0; WRITE_SIZE
# 262144 KiB -> x1.0).  Valid only for the kernel sources they were taken on.
TRAFFIC = dict(fetch_kib=1002863.8, write_kib=1295563.3, fetch_factor=2.0, write_factor=1.0,
               sources_sha256="2fae1109e931794c28948c2b1b0b357f98e857ff7afc6988202b2461ab46c449")
TRAFFIC_SOURCES = ('paper_2605_30355_amd/csrc/sweep_stream.hip', 'paper_2605_30355_amd/csrc/device_common.hpp', 'paper_2605_30355_amd/csrc/schedule.cpp', 'paper_2605_30355_amd/csrc/internal.hpp')


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes():
    """HBM bytes per sweep launch from the recorded counters, or None when the
    kernel sources changed since they were taken."""
    if sources_sha256() != TRAFFIC["sources_sha256"]:
        return None
    return round(1024 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_factor"]
                         + TRAFFIC["write_kib"] * TRAFFIC["write_factor"]))


# The timed workload: the 141 x 141 +-1 torus (the size of the paper's largest
# toroidal instance, with an odd side, so the torus colouring has 6 classes),
# 4096 replicas, FP32 phases, in the kernel shape given here (2 replicas and
# 1024 threads per workgroup: one workgroup fills a CU's LDS).
HEADLINE = dict(name="torus141-pm1", L=141, seed=4, weights="pm1", replicas=4096, sweeps=10000,
                alpha0_deg=14.0, dwt_ratio=0.5, dwt_period=3, window_deg=90.0, bisectors=100,
                colouring=2, sides=[141, 141], replicas_per_wg=2, threads_per_wg=1024)

# The Max-Cut workload of the time-to-target legs.
WORKLOAD = dict(name="maxcut-3reg-n2000", n=2000, degree=3, seed=2, weights="maxcut1",
                replicas=1024, sweeps=10000, alpha0_deg=14.0, dwt_ratio=1.0, dwt_period=6,
                window_deg=90.0, bisectors=100)


def headline_instance():
    import cosm_inputs as ci
    return ci.torus(HEADLINE["L"], seed=HEADLINE["seed"], weights=HEADLINE["weights"])


def headline_params(cosm, **over):
    h = HEADLINE
    p = cosm.Params(alpha0_deg=h["alpha0_deg"], dwt_ratio=h["dwt_ratio"],
                    dwt_period=h["dwt_period"], dwt_window_deg=h["window_deg"],
                    n_bisectors=h["bisectors"], sweeps_per_trial=h["sweeps"],
                    replicas_per_wg=h["replicas_per_wg"], threads_per_wg=h["threads_per_wg"],
                    residency=cosm.RES_LDS)
    for k, v in over.items():
        setattr(p, k, v)
    return p


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_instance():
    import cosm_inputs as ci
    return ci.random_regular(WORKLOAD["n"], WORKLOAD["degree"], seed=WORKLOAD["seed"],
                             weights=WORKLOAD["weights"])


def params(cosm, **over):
    p = cosm.Params(alpha0_deg=WORKLOAD["alpha0_deg"], dwt_ratio=WORKLOAD["dwt_ratio"],
                    dwt_period=WORKLOAD["dwt_period"], dwt_window_deg=WORKLOAD["window_deg"],
                    n_bisectors=WORKLOAD["bisectors"], sweeps_per_trial=WORKLOAD["sweeps"])
    for k, v in over.items():
        setattr(p, k, v)
    return p


def load_target():
    path = os.path.join(ROOT, "tests", "golden", "targets.json")
    try:
        with open(path) as f:
            return json.load(f)[WORKLOAD["name"]]["target_H"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model name (as lscpu prints it) with its family and model
    numbers, from /proc/cpuinfo (a virtual machine may report a generic name)."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key = line.split(":", 1)[0].strip()
                if key in ("model name", "cpu family", "model") and key not in fields:
                    fields[key] = line.split(":", 1)[1].strip()
                if not line.strip() and fields:
                    break
    except OSError:
        return None
    if "model name" not in fields:
        return None
    extra = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model") if k in fields)
    return fields["model name"] + (f" ({extra})" if extra else "")


def cpu_baseline(inst, colour, C, work, seconds_goal=12.0):
    """The FP64 oracle on the host cores, on a bounded sample of the workload
    `work`: whole trials (init, all sweeps, readout) of as many replicas as fit
    in about seconds_goal, one replica per thread at a time; then one replica
    on one core."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    S = work["sweeps"]
    op = oracle.Params(alpha0_deg=work["alpha0_deg"], dwt_ratio=work["dwt_ratio"],
                       dwt_period=work["dwt_period"], dwt_window_deg=work["window_deg"],
                       n_bisectors=work["bisectors"], sweeps=S)
    prob = oracle.Problem(inst.n, inst.eu, inst.ev, inst.J, colour=colour, C=C)
    # calibrate on one replica per thread for 100 sweeps, then size the sample
    x = oracle.init_phases(inst.n, 7, 0, threads)
    t0 = time.perf_counter()
    oracle.sweeps(prob, op, 7, 0, x, 0, 100, n_threads=threads)
    rate = threads * 100 * inst.m / (time.perf_counter() - t0)
    R = max(threads, int(seconds_goal * rate / (inst.m * S)) // threads * threads)
    t0 = time.perf_counter()
    x = oracle.init_phases(inst.n, 7, 0, R)
    oracle.sweeps(prob, op, 7, 0, x, 0, S, n_threads=threads)
    oracle.readout(prob, op, x)
    dt = time.perf_counter() - t0
    # and one core: one replica, the whole trial
    t1 = time.perf_counter()
    x1 = oracle.init_phases(inst.n, 7, 0, 1)
    oracle.sweeps(prob, op, 7, 0, x1, 0, S, n_threads=1)
    oracle.readout(prob, op, x1)
    dt1 = time.perf_counter() - t1
    return {"value": R * S * inst.m / dt, "unit": "edge-updates/s",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{R} replicas x {S} sweeps of {work['name']} "
                      f"(init, sweeps, readout), {dt:.1f} s wall",
            "seconds": round(dt, 2),
            "replica_sweeps_per_s": R * S / dt,
            "one_core": {"value": S * inst.m / dt1, "unit": "edge-updates/s",
                         "sample": f"1 replica x {S} sweeps, {dt1:.2f} s wall"}}


STREAM = dict(name="mixed-stream-256", requests=256, n_min=400, n_max=20000, seed=5,
              replicas=256, sweeps=10000, load=0.7)
FAMILY_PARAMS = {"torus": dict(dwt_ratio=0.5, dwt_period=3),
                 "3-regular": dict(dwt_ratio=1.0, dwt_period=6),
                 "5-regular": dict(dwt_ratio=1.5, dwt_period=3)}


ABLATION = dict(replicas=1024, batches=2, sweeps=10000, seed=11)


def wilson(k, n, z=1.959964):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def ablation_bench():
    """Table VII's ablation on synthetic stand-ins: the full method against the
    same sweeps without SCS (Eq. (8) full-gradient update, all edges reading
    the phases of the previous sweep), without the dual window twist (T = 0)
    and without both.  Per variant: energies of R x batches trials at S sweeps,
    P_s at the oracle's best energy and at 0.5 % above it (Wilson CI), R99 and
    TTT with t_trial from HIP events around each batch (init, sweeps, readout)."""
    import numpy as np
    import torch

    import cosm_inputs as ci
    import paper_2605_30355_amd as cosm

    torch.cuda.set_device(0)
    with open(os.path.join(ROOT, "tests", "golden", "targets.json")) as f:
        targets = json.load(f)
    work = [("maxcut-3reg-n2000", make_instance(), dict(dwt_ratio=1.0, dwt_period=6)),
            ("maxcut-er-n10000", ci.erdos_renyi_capped(10000, 2.0, 9, seed=70, weights="maxcut1"),
             dict(dwt_ratio=1.0, dwt_period=6))]
    R, nb, S = ABLATION["replicas"], ABLATION["batches"], ABLATION["sweeps"]
    out = {"metric": "ablation (Table VII): P_s and TTT @99% without SCS / without DWT",
           "replicas_per_batch": R, "batches": nb, "sweeps": S, "instances": {}}
    stream = torch.cuda.current_stream()
    for name, inst, kw in work:
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
        tH = targets[name]["target_H"]
        relaxed = int(math.floor(tH * 0.995))  # H < 0: 0.5 % above the best energy
        rec = {"n": inst.n, "m": inst.m, "classes": C, "target_H": tH, "relaxed_target_H": relaxed,
               "variants": {}}
        for vname, over in (("full", {}), ("without_dwt", {"dwt_period": 0}),
                            ("without_scs", {"update": cosm.UPDATE_FULL_GRADIENT}),
                            ("without_both", {"update": cosm.UPDATE_FULL_GRADIENT, "dwt_period": 0})):
            p = cosm.Params(sweeps_per_trial=S, **kw)
            for k, v in over.items():
                setattr(p, k, v)
            st = cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=ABLATION["seed"],
                            replicas=R)
            Hs, ms = [], 0.0
            for k in range(nb):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                st.reset(ABLATION["seed"], k * R)
                st.sweep(S)
                H, _, _ = st.energy(return_spins=False)
                e1.record(stream)
                torch.cuda.synchronize()
                ms += e0.elapsed_time(e1)
                Hs.append(H.copy())
            info = st.info()
            st.close()
            H = np.concatenate(Hs)
            t_trial = ms * 1e-3 / (R * nb)
            v = {"form": {cosm.RES_LDS: "lds", cosm.RES_HBM: "hbm"}.get(info["residency"], "plain"),
                 "mean_H": float(H.mean()), "best_H": int(H.min()), "t_trial_s": t_trial}
            for label, thr in (("target", tH), ("relaxed", relaxed)):
                k = int((H <= thr).sum())
                ps = k / len(H)
                r99 = (1.0 if ps >= 1.0 else math.log(0.01) / math.log(1.0 - ps)) if ps > 0 else None
                v[label] = {"hits": k, "ps": ps, "ps_ci95": list(wilson(k, len(H))), "r99": r99,
                            "ttt_s": t_trial * r99 if r99 is not None else None}
            rec["variants"][vname] = v
            log(f"ablation {name} {vname}: {v}")
        out["instances"][name] = rec
    return out


SCALING = dict(sizes=(12, 14, 16, 18, 20), seeds=tuple(range(1, 16)), trials=4096,
               sweep_options=(25, 50, 100, 200, 400, 800, 1600), single_trials=200,
               alpha0_deg=25.0, dwt_ratio=1.0, dwt_period=3)


def fit_log_tts(L, tts):
    """Least-squares fit of log10 TTS = a + b L (the fit used for the
    tile-planted scaling, Appendix C).  Returns a, b, R^2 and the 95 %
    t-interval of b."""
    import numpy as np
    from scipy import stats
    L = np.asarray(L, dtype=np.float64)
    y = np.log10(np.asarray(tts, dtype=np.float64))
    n = len(L)
    Lm, ym = L.mean(), y.mean()
    sxx = ((L - Lm) ** 2).sum()
    b = ((L - Lm) * (y - ym)).sum() / sxx
    a = ym - b * Lm
    res = y - (a + b * L)
    ss_res, ss_tot = (res ** 2).sum(), ((y - ym) ** 2).sum()
    r2 = 1.0 - ss_res / ss_tot
    se = math.sqrt(ss_res / (n - 2) / sxx)
    t = stats.t.ppf(0.975, n - 2)
    return {"a": a, "b": b, "r_squared": r2, "b_ci95": [b - t * se, b + t * se]}


def scaling_bench():
    """TTS scaling on +-1/+-2 tori (the shape of the tile-planted set; random,
    not planted), L in {12, ..., 20}, fifteen instances per size, Appendix C's
    parameters.  Per instance: P_s of 4096 batched trials at each sweep budget,
    the budget with the fewest sweeps-to-solution kept (the paper tuned its
    sweeps the same way), then t_trial measured two ways: batched (device time
    of 4096 parallel trials / 4096) and single-replica latency (one trial at a
    time, init + sweeps + readout, averaged over sequential trials).  TTS =
    t_trial x R99; the median over instances per size is fitted to
    log10 TTS = a + b L."""
    import numpy as np
    import torch

    import cosm_inputs as ci
    import paper_2605_30355_amd as cosm

    torch.cuda.set_device(0)
    with open(os.path.join(ROOT, "tests", "golden", "targets.json")) as f:
        targets = json.load(f)
    cfg = SCALING
    stream = torch.cuda.current_stream()

    def params(S, R_form=None):
        return cosm.Params(alpha0_deg=cfg["alpha0_deg"], dwt_ratio=cfg["dwt_ratio"],
                           dwt_period=cfg["dwt_period"], sweeps_per_trial=S)

    def timed_batch(st, S, rid0):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st.reset(7, rid0)
        st.sweep(S)
        H, _, _ = st.energy(return_spins=False)
        e1.record(stream)
        torch.cuda.synchronize()
        return H.copy(), e0.elapsed_time(e1) * 1e-3

    out = {"metric": "TTS scaling on +-1/+-2 tori: median TTS vs L, fit log10 TTS = a + b L",
           "parameters": {k: v for k, v in cfg.items() if k != "sizes"}, "sizes": {}}
    med_b, med_s = [], []
    for L in cfg["sizes"]:
        per = []
        for sd in cfg["seeds"]:
            inst = ci.torus(L, seed=1000 * L + sd, weights="pm12")
            colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [L, L])
            target = targets[f"torus-pm12-L{L}-s{sd}"]["target_H"]
            R = cfg["trials"]
            best = None
            for S in cfg["sweep_options"]:
                with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, params(S), seed=7,
                                replicas=R) as st:
                    H, secs = timed_batch(st, S, 0)
                ps = float((H <= target).mean())
                if ps <= 0.0:
                    continue
                r99 = 1.0 if ps >= 1.0 else math.log(0.01) / math.log(1.0 - ps)
                if best is None or S * r99 < best["sts"]:
                    best = {"sweeps": S, "ps": ps, "r99": r99, "sts": S * r99,
                            "t_trial_batched_s": secs / R}
            if best is None:
                per.append({"seed": sd, "reached": False})
                continue
            S = best["sweeps"]
            # single-replica latency: one trial at a time on its own state
            with cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, params(S), seed=7,
                            replicas=1) as s1:
                timed_batch(s1, S, 0)
                tot = 0.0
                for k in range(cfg["single_trials"]):
                    _, secs = timed_batch(s1, S, k + 1)
                    tot += secs
            best["t_trial_single_s"] = tot / cfg["single_trials"]
            best["tts_batched_s"] = best["t_trial_batched_s"] * best["r99"]
            best["tts_single_s"] = best["t_trial_single_s"] * best["r99"]
            best.update({"seed": sd, "target_H": target, "reached": True})
            per.append(best)
            log(f"scaling L={L} seed={sd}: {best}")
        ok = [p for p in per if p["reached"]]
        rec = {"instances": per,
               "median_tts_batched_s": float(np.median([p["tts_batched_s"] for p in ok])) if ok else None,
               "median_tts_single_s": float(np.median([p["tts_single_s"] for p in ok])) if ok else None}
        out["sizes"][str(L)] = rec
        med_b.append(rec["median_tts_batched_s"])
        med_s.append(rec["median_tts_single_s"])
    Ls = list(cfg["sizes"])
    if all(v is not None for v in med_b):
        out["fit_batched"] = fit_log_tts(Ls, med_b)
        out["fit_single_replica"] = fit_log_tts(Ls, med_s)
    return out


def stream_bench():
    """Mixed request stream: 256 solve requests (N uniform in [400, 20000]; torus,
    3-regular Max-Cut and 5-regular +-1 graphs), each a whole trial of 256
    replicas x 10^4 sweeps, served by one batch (one persistent sweep launch per
    micro-batch, replayed from a hipGraph).  First all requests at t = 0 (the
    burst gives the capacity), then Poisson arrivals at 70 % of that capacity."""
    import numpy as np
    import torch

    import cosm_inputs as ci
    import paper_2605_30355_amd as cosm

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    reqs = ci.request_stream(STREAM["requests"], STREAM["n_min"], STREAM["n_max"], STREAM["seed"])
    b = cosm.Batch(max_graphs=STREAM["requests"], max_n=STREAM["n_max"] + 1)
    ids, updates, lds_bytes = [], 0, 0
    for k, (_, inst) in enumerate(reqs):
        fam = inst.meta["family"]
        if fam == "torus":
            L = inst.meta["Lx"]
            colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_TORUS, [L, L])
        else:
            colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
        p = cosm.Params(sweeps_per_trial=STREAM["sweeps"], **FAMILY_PARAMS[fam])
        ids.append(b.add(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=k,
                         replicas=STREAM["replicas"]))
        updates += inst.m * STREAM["sweeps"] * STREAM["replicas"]
        # algorithmic LDS bytes (FP32): 16 per edge update, 8 per vertex and twist
        lds_bytes += (16 * inst.m + 8 * inst.n / FAMILY_PARAMS[fam]["dwt_period"]) \
            * STREAM["sweeps"] * STREAM["replicas"]
    shapes = [b.shape(g) for g in ids]
    widths = {}
    for sh in shapes:
        widths[str(sh["replicas_per_set"])] = widths.get(str(sh["replicas_per_set"]), 0) + 1
    log(f"stream: {len(ids)} requests prepared in {time.perf_counter() - t0:.1f} s "
        f"(replicas per set: {widths})")
    b.run(ids[:4])  # warm-up (captures the graph)
    b.wait()
    # burst: every request at t = 0, one launch
    t0 = time.perf_counter()
    b.run(ids)
    dev_ms = b.wait()
    burst_s = time.perf_counter() - t0
    capacity = len(ids) / burst_s
    log(f"stream burst: {burst_s:.2f} s ({dev_ms:.0f} ms device), {capacity:.1f} requests/s")
    # Poisson arrivals at STREAM["load"] x capacity, micro-batched when the GPU is idle
    rng = np.random.default_rng(STREAM["seed"])
    arrivals = np.cumsum(rng.exponential(1.0 / (STREAM["load"] * capacity), size=len(ids)))
    done = np.zeros(len(ids))
    nxt, launches, pois_dev_ms = 0, 0, 0.0
    start = time.perf_counter()
    while nxt < len(ids):
        now = time.perf_counter() - start
        if arrivals[nxt] > now:
            time.sleep(min(arrivals[nxt] - now, 0.002))
            continue
        batch = []
        while nxt < len(ids) and arrivals[nxt] <= now:
            batch.append(nxt)
            nxt += 1
        for k in batch:
            b.set_seed(ids[k], 1000 + k, 0)
        b.run([ids[k] for k in batch])
        pois_dev_ms += b.wait()
        launches += 1
        done[batch] = time.perf_counter() - start
    lat = (done - arrivals) * 1e3
    span = done.max() - arrivals[0]
    b.close()
    return {
        "metric": "mixed request stream on one MI355X (latency and throughput)",
        "workload": STREAM["name"], "requests": len(ids), "replicas_per_request": STREAM["replicas"],
        "sweeps_per_request": STREAM["sweeps"], "n_range": [STREAM["n_min"], STREAM["n_max"]],
        "families": list(FAMILY_PARAMS), "total_edge_updates": updates,
        "shapes": {"replicas_per_set": widths,
                   "tuned_by_probes": sum(1 for sh in shapes if sh["tuned"] == 1),
                   "from_cache": sum(1 for sh in shapes if sh["tuned"] == 2)},
        "burst": {"seconds": round(burst_s, 3), "device_ms": round(dev_ms, 1),
                  "requests_per_s": round(capacity, 2),
                  "edge_updates_per_s": round(updates / burst_s, 1),
                  "lds_roofline_frac": round(lds_bytes / (dev_ms * 1e-3) / (LDS_PEAK_GBS * 1e9), 4)},
        "poisson": {"rate_per_s": round(STREAM["load"] * capacity, 2), "launches": launches,
                    "p50_ms": round(float(np.percentile(lat, 50)), 1),
                    "p99_ms": round(float(np.percentile(lat, 99)), 1),
                    "mean_ms": round(float(lat.mean()), 1),
                    "requests_per_s": round(len(ids) / span, 2),
                    "edge_updates_per_s": round(updates / span, 1),
                    "device_ms": round(pois_dev_ms, 1),
                    "lds_roofline_frac": round(lds_bytes / (pois_dev_ms * 1e-3)
                                               / (LDS_PEAK_GBS * 1e9), 4)},
    }


LARGE = dict(sweeps=300, reps=2, seed=1)

# Time to target over many instances of the 5-regular N = 20000 +-1 family
# (instance seeds first .. first + count - 1).  Per instance: the target is the
# best energy of target_batches batches of replicas trials (solver seed 1); the
# time to target is then measured on ttt_batches fresh batches (solver seed 2),
# at that energy and 0.5 % above it.
SEEDS = dict(first=1000, count=100, replicas=2048, sweeps=10000, target_batches=2,
             ttt_batches=4, relax=0.005)
SEED_FAMILIES = {
    # instance generator, colouring, the shape the autotuner keeps on the family
    "rr5": dict(n=20000, make=lambda ci, s: ci.random_regular(20000, 5, seed=s, weights="pm1"),
                colouring="balanced", rw=2),
    "er": dict(n=10000, make=lambda ci, s: ci.erdos_renyi_capped(10000, 4, 8, seed=s),
               colouring="misra-gries", rw=4),
}


def seeds_bench(count=None, jsonl=None, family="rr5", sweeps=None):
    """Median and interquartile range of TTT @99% over instance seeds.  With a
    JSONL file, each instance's record there also carries the spins of its
    target trial (packed bits, hex), for tests/golden/verify_seed_targets.py to
    re-evaluate with the FP64 oracle."""
    import numpy as np
    import torch

    import cosm_inputs as ci
    import paper_2605_30355_amd as cosm

    torch.cuda.set_device(0)
    cfg = dict(SEEDS)
    if count is not None:
        cfg["count"] = count
    if sweeps is not None:
        cfg["sweeps"] = sweeps
    fam = SEED_FAMILIES[family]
    cfg.update(family=family, n=fam["n"], colouring=fam["colouring"])
    R, S = cfg["replicas"], cfg["sweeps"]
    stream = torch.cuda.current_stream()
    recs = []
    for k in range(cfg["count"]):
        seed = cfg["first"] + k
        inst = fam["make"](ci, seed)
        colour, C = cosm.build_partitions(
            inst.n, inst.eu, inst.ev,
            cosm.COLOR_BALANCED if fam["colouring"] == "balanced" else cosm.COLOR_MISRA_GRIES)
        # the shape the autotuner keeps on this family, fixed so that every
        # instance runs the same kernel
        p = cosm.Params(sweeps_per_trial=S, dwt_ratio=1.5, dwt_period=3,
                        lds_form=cosm.LDS_FORM_PAIR, replicas_per_wg=fam["rw"],
                        threads_per_wg=1024)
        st = cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=1, replicas=R)
        best, best_spins = None, None
        for b in range(cfg["target_batches"]):
            st.reset(1, b * R)
            st.sweep(S)
            H, _, sp = st.energy(return_spins=True)
            i = int(np.argmin(H))
            if best is None or int(H[i]) < best:
                best, best_spins = int(H[i]), sp[i].copy()
        Hs, ms = [], 0.0
        for b in range(cfg["ttt_batches"]):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st.reset(2, b * R)
            st.sweep(S)
            H, _, _ = st.energy(return_spins=False)
            e1.record(stream)
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            Hs.append(H.copy())
        st.close()
        H = np.concatenate(Hs)
        t_trial = ms * 1e-3 / len(H)
        relaxed = int(math.floor(best * (1.0 - cfg["relax"])))  # H < 0
        rec = {"seed": seed, "classes": C, "target_H": best, "relaxed_target_H": relaxed,
               "t_trial_s": t_trial, "best_H_ttt_run": int(H.min())}
        for label, thr in (("target", best), ("relaxed", relaxed)):
            hits = int((H <= thr).sum())
            ps = hits / len(H)
            r99 = (1.0 if ps >= 1.0 else math.log(0.01) / math.log(1.0 - ps)) if ps > 0 else None
            rec[label] = {"hits": hits, "ps": ps, "r99": r99,
                          "ttt_s": t_trial * r99 if r99 is not None else None}
        recs.append(rec)
        log(f"seeds {rec}")
        if jsonl is not None:
            with open(jsonl, "a") as f:
                f.write(json.dumps(dict(rec, family=family, sweeps=S, target_spins_hex=np.packbits(
                    best_spins > 0).tobytes().hex())) + "\n")

    def summary(label):
        # nearest-rank quartiles over every instance, an instance without a hit
        # counting as an unbounded TTT (null when a quartile falls on one)
        v = sorted(r[label]["ttt_s"] if r[label]["ttt_s"] is not None else math.inf
                   for r in recs)

        def rank(p):
            x = v[max(0, min(len(v) - 1, math.ceil(p / 100 * len(v)) - 1))]
            return x if math.isfinite(x) else None

        return {"instances_with_hits": sum(1 for x in v if math.isfinite(x)),
                "instances": len(recs), "median_ttt_s": rank(50),
                "iqr_ttt_s": [rank(25), rank(75)]}

    return {"metric": f"time to target @99% over instance seeds, {family} +-1 graphs, 1 MI355X",
            "config": {k: v for k, v in cfg.items()}, "solver": f"FP32, grid schedule, pair layout "
            f"{fam['rw']} replicas x 1024 threads, alpha0 14, dwt ratio 1.5 period 3, 100 bisectors",
            "fidelity": f"{S} sweeps per trial; the targets are the best of "
            f"{cfg['target_batches'] * R} GPU trials per instance, not oracle ground states (their "
            "spins, written to the JSONL file, are re-evaluated by the FP64 oracle in "
            "tests/golden/verify_seed_targets.py)",
            "t_trial_s_median": float(np.median([r["t_trial_s"] for r in recs])),
            "target": summary("target"), "relaxed": summary("relaxed"), "instances": recs}


def lds_bytes(info, inst, R, S, period, storage_bytes):
    """LDS bytes of S sweeps of R replicas: the algorithmic count (2 reads and
    2 writes of a phase per edge update, a read and a write of every phase per
    twist) and the bytes the kernel's layout moves (the register layout reads
    and writes one LDS row for an edge with an endpoint in registers, and the
    twist touches only the LDS rows)."""
    b = storage_bytes
    twists = S // period if period > 0 else 0
    algo = R * (S * 4 * b * inst.m + twists * 2 * b * inst.n)
    if info.get("lds_form") in (2, 3):
        er, nr = info["register_edges"], info["register_vertices"]
        moved = R * (S * b * (2 * er + 4 * (inst.m - er)) + twists * 2 * b * (inst.n - nr))
    else:
        moved = algo
    return algo, moved


def large_bench(cases_wanted=None, S=None, reps=None):
    """The large-graph configurations: the 100x100 and 141x141 +-1 tori at 4096
    replicas (FP32, FIX32, FP16, FP16 with FP16 arithmetic, BF16 and FIX16 storage) and
    the 5-regular N = 20000 and capped Erdos-Renyi N = 10000 graphs at 2048 replicas
    (FP32, FIX32): edge-updates/s
    of the sweep kernel (HIP events around whole sweep calls after a warm-up),
    the shape and layout the autotuner kept, and the LDS roofline fraction of the
    algorithmic bytes (16 B, or 8 B for 16-bit storage, per edge update plus a
    read and a write of every phase per twist) and of the bytes the layout moves."""
    import torch

    import cosm_inputs as ci
    import paper_2605_30355_amd as cosm

    torch.cuda.set_device(0)
    cases = [("torus-100x100", lambda: ci.torus(100, seed=3), cosm.COLOR_TORUS, [100, 100], 4096,
              dict(dwt_ratio=0.5, dwt_period=3), ("fp32", "fix32", "fp16", "fp16pk", "bf16", "fix16")),
             ("torus-141x141", lambda: ci.torus(141, seed=4), cosm.COLOR_TORUS, [141, 141], 4096,
              dict(dwt_ratio=0.5, dwt_period=3), ("fp32", "fix32", "fp16", "fp16pk", "bf16", "fix16")),
             ("rr5-n20000", lambda: ci.random_regular(20000, 5, seed=1000, weights="pm1"),
              cosm.COLOR_BALANCED, None, 2048, dict(dwt_ratio=1.5, dwt_period=3), ("fp32", "fix32")),
             ("er-n10000", lambda: ci.erdos_renyi_capped(10000, 4, 8, seed=3),
              cosm.COLOR_MISRA_GRIES, None, 2048, dict(dwt_ratio=1.5, dwt_period=3),
              ("fp32", "fix32"))]
    storages = {"fp32": cosm.STORE_FP32, "fix32": cosm.STORE_FIX32, "fp16": cosm.STORE_FP16,
                "bf16": cosm.STORE_BF16, "fix16": cosm.STORE_FIX16, "fp16pk": cosm.STORE_FP16_PK}
    S = S or LARGE["sweeps"]
    reps = reps or LARGE["reps"]
    stream = torch.cuda.current_stream()
    out = {"metric": "edge-updates/s of the sweep on the large-graph configurations, 1 MI355X",
           "sweeps_per_call": S, "calls": reps, "cases": []}
    for name, make_inst, meth, sides, R, kw, sts in cases:
        want = None if cases_wanted is None else cases_wanted.get(name)
        if cases_wanted is not None and want is None:
            continue
        inst = make_inst()
        colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, meth, sides)
        for st_name in sts:
            if want is not None and st_name not in want:
                continue
            p = cosm.Params(sweeps_per_trial=S * (reps + 1), storage=storages[st_name], **kw)
            st = cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, p, seed=LARGE["seed"],
                            replicas=R)
            st.sweep(S)  # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                st.sweep(S)
            e1.record(stream)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / reps
            info = st.info()
            st.close()
            rate = inst.m * S * R / sec
            b = 2 if st_name in ("fp16", "fp16pk", "bf16", "fix16") else 4
            algo, moved = lds_bytes(info, inst, R, S, kw["dwt_period"], b)
            form = {cosm.RES_LDS: "lds", cosm.RES_HBM: "hbm"}.get(info["residency"], "plain")
            rec = {"workload": name, "n": inst.n, "m": inst.m, "classes": C, "replicas": R,
                   "storage": st_name, "edge_updates_per_s": round(rate, 1),
                   "replica_sweeps_per_s": round(S * R / sec, 1), "form": form,
                   "layout": {1: "pair", 2: "register", 3: "register-stream"}.get(info["lds_form"], None),
                   "register_rows": info["register_rows"], "twist_fused": info["twist_fused"],
                   "streamed": info["streamed"], "lazy_wrap": info["lazy_wrap"],
                   "replicas_per_wg": info["replicas_per_wg"],
                   "threads_per_wg": info["threads_per_wg"],
                   "lds_roofline_frac": round(algo / sec / (LDS_PEAK_GBS * 1e9), 3),
                   "lds_moved_frac": round(moved / sec / (LDS_PEAK_GBS * 1e9), 3)}
            out["cases"].append(rec)
            log(f"large {rec}")
    return out


def maxcut_legs(args):
    """The Max-Cut workload: the batched sweep kernel's rate, the plain
    one-replica-per-launch form, and time to target at 99 % for the batched
    FP32, reduced-precision and other forms (cosm_solve_to_target)."""
    import torch

    import paper_2605_30355_amd as cosm

    inst = make_instance()
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, cosm.COLOR_BALANCED)
    R, S, m = WORKLOAD["replicas"], WORKLOAD["sweeps"], inst.m
    stream = torch.cuda.current_stream()
    # the shape the autotuner picks on this workload (2 replicas and 768
    # threads per workgroup, one slot per class), fixed so that every launch
    # of the batched leg is a full trial
    st = cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C,
                    params(cosm, lds_form=cosm.LDS_FORM_PAIR, replicas_per_wg=2,
                           threads_per_wg=768), seed=1, replicas=R)
    info = st.info()
    st.sweep(S)  # warm-up
    st.reset(1, R)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    st.sweep(S)
    e1.record(stream)
    torch.cuda.synchronize()
    kernel_s = e0.elapsed_time(e1) * 1e-3
    batched_rate = m * S * R / kernel_s
    algo, _ = lds_bytes(info, inst, R, S, WORKLOAD["dwt_period"], 4)
    out = {"workload": WORKLOAD["name"], "n": inst.n, "edges": m, "classes": C, "replicas": R,
           "sweeps": S, "colouring": "misra-gries, class sizes equalised",
           "replicas_per_wg": info["replicas_per_wg"], "threads_per_wg": info["threads_per_wg"],
           "layout": {1: "pair", 2: "register", 3: "register-stream"}.get(info["lds_form"], None),
           "sweep_kernel_edge_updates_per_s": round(batched_rate, 1),
           "sweep_kernel_lds_roofline_frac": round(algo / kernel_s / (LDS_PEAK_GBS * 1e9), 4)}
    log(f"maxcut batched: {batched_rate:.3e} edge-updates/s, shape {info}")

    # plain form: one replica per launch, one launch per colour class
    plain_sweeps = 500
    sp = cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C,
                    params(cosm, residency=cosm.RES_PLAIN), seed=1, replicas=1)
    sp.sweep(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp.sweep(plain_sweeps)
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t0
    plain_rate = m * plain_sweeps / plain_dt
    plain_t_trial = plain_dt / plain_sweeps * S
    sp.close()
    out["plain_edge_updates_per_s"] = round(plain_rate, 1)
    out["batched_over_plain"] = round(batched_rate / plain_rate, 1)
    log(f"plain: {plain_rate:.3e} edge-updates/s, t_trial {plain_t_trial:.3f} s")

    target = load_target()
    if args.no_ttt or target is None:
        st.close()
        return out
    ttt = {"target_H": target, "target_cut": (int(-inst.J.sum()) - target) // 2}
    for name, over in (("batched_fp32", {}), ("batched_fp16", {"storage": cosm.STORE_FP16}),
                       ("batched_fp16_pk", {"storage": cosm.STORE_FP16_PK}),
                       ("batched_bf16", {"storage": cosm.STORE_BF16}),
                       ("batched_fix16", {"storage": cosm.STORE_FIX16}),
                       ("batched_fix32", {"storage": cosm.STORE_FIX32}),
                       ("batched_fp32_register_layout", {"lds_form": cosm.LDS_FORM_REGISTER}),
                       ("batched_fp32_optimal_readout", {"readout": cosm.READOUT_OPTIMAL}),
                       ("batched_fp32_minimum_colouring", {"colouring": cosm.COLOR_MINIMUM})):
        col2, C2 = colour, C
        if "colouring" in over:  # 3 classes of 1000 instead of 4 of 750
            col2, C2 = cosm.build_partitions(inst.n, inst.eu, inst.ev, over.pop("colouring"))
        s2 = st if not over and col2 is colour else cosm.State(
            inst.n, inst.eu, inst.ev, inst.J, col2, C2, params(cosm, **over), seed=1,
            replicas=R)
        res, _ = s2.solve_to_target(target, 8 * R)
        ttt[name] = {"ps": res.ps, "ps_ci95": [res.ps_lo, res.ps_hi], "trials": res.trials,
                     "r99": res.r99, "t_trial_s": res.t_trial_s, "ttt_s": res.ttt_s,
                     "best_H": res.best_H,
                     # whole trials (init, sweeps, readout) per second, as edge updates
                     "edge_updates_per_s": round(m * S / res.t_trial_s, 1)}
        if col2 is not colour:
            ttt[name]["classes"] = C2
        if s2 is not st:
            s2.close()
        log(f"{name}: {ttt[name]}")
    ps = ttt["batched_fp32"]["ps"]
    r99 = ttt["batched_fp32"]["r99"]
    # the plain form runs the same trajectories (bit-exact), so it shares P_s
    ttt["plain_fp32"] = {"ps": ps, "r99": r99, "t_trial_s": plain_t_trial,
                         "ttt_s": plain_t_trial * r99 if math.isfinite(r99) else None}
    for k, v in ttt.items():
        if isinstance(v, dict) and v.get("ttt_s") is not None and not math.isfinite(v["ttt_s"]):
            v["ttt_s"] = None
            v["r99"] = None
    st.close()
    out["ttt"] = ttt
    return out


def copy_probe():
    """One 256 MiB device copy whose source is first evicted from the caches by
    1 GiB of other writes: the reference for the HBM byte counters."""
    import torch

    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    evict = torch.empty(256 << 20, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    evict.fill_(2.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b, evict


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttt", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="time the headline workload only (no Max-Cut legs or other graphs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (reference for HBM counters)")
    ap.add_argument("--stream", action="store_true",
                    help="measure the mixed request stream instead (prints its own JSON line)")
    ap.add_argument("--ablation", action="store_true",
                    help="run the Table VII ablation instead (prints its own JSON line)")
    ap.add_argument("--scaling", action="store_true",
                    help="run the TTS scaling study on +-1/+-2 tori instead (own JSON line)")
    ap.add_argument("--maxcut", action="store_true",
                    help="run the Max-Cut legs only (batched, plain, time to target; own JSON line)")
    ap.add_argument("--large", action="store_true",
                    help="measure the large tori and bounded-degree graphs instead (own JSON line)")
    ap.add_argument("--only", nargs="+", default=None, metavar="CASE:STORAGE",
                    help="with --large: just these cases, e.g. torus-141x141:bf16")
    ap.add_argument("--seeds", type=int, nargs="?", const=SEEDS["count"], default=None,
                    help="time to target over N instance seeds of the 5-regular family instead")
    ap.add_argument("--sweeps", type=int, default=None,
                    help="with --seeds: sweeps per trial (default %d)" % SEEDS["sweeps"])
    ap.add_argument("--seeds-jsonl", default=None,
                    help="with --seeds: also append each instance's record to this file")
    ap.add_argument("--family", default="rr5", choices=sorted(SEED_FAMILIES),
                    help="with --seeds: 5-regular N=20000 (rr5) or capped Erdos-Renyi N=10000 (er)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the method's replicas are independent, so several "
              "GPUs would each run this same single-GPU job on their own replicas; "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.stream:
        print(json.dumps(stream_bench()), flush=True)
        return
    if args.ablation:
        print(json.dumps(ablation_bench()), flush=True)
        return
    if args.scaling:
        print(json.dumps(scaling_bench()), flush=True)
        return
    if args.large:
        wanted = None
        if args.only:
            wanted = {}
            for item in args.only:
                case, st_name = item.split(":")
                wanted[case] = wanted.get(case, ()) + (st_name,)
        print(json.dumps(large_bench(wanted)), flush=True)
        return
    if args.maxcut:
        import torch
        torch.cuda.set_device(0)
        if args.copy_probe:
            copy_probe()
        print(json.dumps(maxcut_legs(args)), flush=True)
        return
    if args.seeds is not None:
        print(json.dumps(seeds_bench(args.seeds, args.seeds_jsonl, args.family, args.sweeps)),
              flush=True)
        return

    import torch

    import paper_2605_30355_amd as cosm

    torch.cuda.set_device(0)
    h = HEADLINE
    inst = headline_instance()
    colour, C = cosm.build_partitions(inst.n, inst.eu, inst.ev, h["colouring"], h["sides"])
    R, S, m = h["replicas"], h["sweeps"], inst.m
    log(f"workload {h['name']}: n={inst.n} m={m} C={C} R={R} S={S}")

    if args.copy_probe:
        copy_probe()

    # ---- the timed steps: whole trials of the batched LDS-resident form --------------
    st = cosm.State(inst.n, inst.eu, inst.ev, inst.J, colour, C, headline_params(cosm), seed=1,
                    replicas=R)
    info = st.info()
    log(f"shape: {info}")
    stream = torch.cuda.current_stream()

    def step(k, ev=None):
        st.reset(1, k * R)
        if ev:
            ev[0].record(stream)
        st.sweep(S)
        if ev:
            ev[1].record(stream)
        st.energy(return_spins=False)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in events]
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    updates = m * S * R * args.steps
    value = updates / elapsed
    st.close()
    log(f"batched: {elapsed * 1e3 / args.steps:.2f} ms/step, sweep kernel {avg_kernel_s * 1e3:.2f} ms, "
        f"{value:.3e} edge-updates/s")

    algo, moved = lds_bytes(info, inst, R, S, h["dwt_period"], 4)
    achieved = algo / avg_kernel_s / 1e9
    row_words = info["replicas_per_wg"]  # FP32: one word per replica
    measured = max(cosm.lds_probe(row_words, bpc) for bpc in (1, 2))
    layout = {1: "pair", 2: "register", 3: "register-stream"}.get(info["lds_form"], None)
    if info["streamed"] and info["lds_form"] == 1:
        layout = "streamed pair"
    roofline = {"bound": "lds", "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1),
                "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBS, 4),
                "traffic": traffic_bytes(), "traffic_unit": "HBM bytes per launch",
                "measured_peak": round(measured, 1),
                "measured_peak_note": "cosm_lds_probe: 2 reads + 2 writes per lane of "
                                      f"{4 * row_words}-byte rows, no arithmetic or barriers",
                "frac_of_measured": round(achieved / measured, 4),
                "moved_frac": round(moved / avg_kernel_s / 1e9 / LDS_PEAK_GBS, 4),
                "kernel": f"sweep kernel, fp32, {row_words} words/row, {layout} layout"
                          + (", wrapped at the twists" if info["lazy_wrap"] else ""),
                "bytes_per_edge_update": 16,
                "bytes_per_launch": algo,
                "kernel_ms": round(avg_kernel_s * 1e3, 4),
                "edge_updates_per_s_kernel": round(m * S * R / avg_kernel_s, 1),
                "valu_peak_lane_ops_per_s": VALU_PEAK_OPS}

    out = {
        "metric": "edge-updates/s (batched vs plain) + time-to-target @99% success, 1 MI355X",
        "value": round(value, 1),
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": h["name"], "n": inst.n, "edges": m, "classes": C,
                   "colouring": "torus pattern", "replicas": R, "sweeps": S,
                   "alpha0_deg": h["alpha0_deg"], "dwt_ratio": h["dwt_ratio"],
                   "dwt_period": h["dwt_period"], "bisectors": h["bisectors"],
                   "schedule": "grid", "storage": "fp32", "residency": "lds", "layout": layout,
                   "replicas_per_wg": info["replicas_per_wg"],
                   "threads_per_wg": info["threads_per_wg"], "workgroups": info["workgroups"],
                   "step": "init + sweeps + 100-bisector readout of all replicas"},
        "replica_sweeps_per_s": round(S * R * args.steps / elapsed, 1),
        "roofline": roofline,
    }
    if not args.no_extra:
        out["maxcut"] = maxcut_legs(args)
        out["large"] = large_bench({"torus-100x100": ("fp32", "fp16", "fp16pk", "bf16", "fix16"),
                                    "torus-141x141": ("fp16", "fp16pk", "bf16", "fix16"),
                                    "rr5-n20000": ("fp32",), "er-n10000": ("fp32",)})["cases"]
        if "maxcut" in out:
            mc = out["maxcut"]
            out["plain_edge_updates_per_s"] = mc["plain_edge_updates_per_s"]
            out["batched_over_plain"] = mc["batched_over_plain"]
            out["ttt"] = mc.get("ttt")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, colour, C, h)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
