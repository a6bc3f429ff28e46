"""Seeded synthetic Ising instances.

This module only builds inputs: graphs, couplings and request streams.  It holds
none of the solver's arithmetic, so both the product path and the CPU oracle
may use it.

Every generator is deterministic in its seed (numpy PCG64) and returns an
``Instance`` with ``n`` spins and edge arrays ``eu``, ``ev``, ``J`` (int32, Ising
sign of Eq. (1): H = -sum J s_i s_j).  A Max-Cut weight w maps to J = -w
(Appendix A).

Shapes follow the paper's workloads, whose own files are not available here:
  * 2D +-J tori with periodic boundaries (the Gset G72/G77/G81 family, Sec. III-A);
  * random regular graphs (bounded degree, unweighted or +-1, stand-ins for the
    non-lattice Gset graphs G61/G70, Table III);
  * Erdos-Renyi graphs with a degree cap (bounded-degree irregular graphs);
  * tori with J in {+-1, +-2} (the shape of the tile-planted set, Sec. III-C);
  * the three-spin conflict-trap instance of Fig. 2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Instance:
    name: str
    n: int
    eu: np.ndarray
    ev: np.ndarray
    J: np.ndarray
    h: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(len(self.eu))

    def degrees(self) -> np.ndarray:
        d = np.zeros(self.n, dtype=np.int64)
        np.add.at(d, self.eu, 1)
        np.add.at(d, self.ev, 1)
        return d


def _couplings(rng: np.random.Generator, m: int, weights: str) -> np.ndarray:
    if weights == "pm1":  # J uniform in {-1, +1}
        return rng.choice(np.array([-1, 1], dtype=np.int32), size=m)
    if weights == "maxcut1":  # Max-Cut weight +1 on every edge -> J = -1
        return np.full(m, -1, dtype=np.int32)
    if weights == "ferro":
        return np.full(m, 1, dtype=np.int32)
    if weights == "antiferro":
        return np.full(m, -1, dtype=np.int32)
    if weights == "pm12":  # J uniform in {-2, -1, +1, +2}
        return rng.choice(np.array([-2, -1, 1, 2], dtype=np.int32), size=m)
    raise ValueError(f"unknown weights {weights!r}")


def torus(Lx: int, Ly: int | None = None, seed: int = 1, weights: str = "pm1") -> Instance:
    """Lx x Ly torus, vertex (r, c) -> r*Lx + c.  For each vertex in row-major order
    the edge to its right neighbour, then the edge to the neighbour below, both
    with periodic wrap.  Needs Lx, Ly >= 3 (smaller sides would repeat edges)."""
    Ly = Lx if Ly is None else Ly
    if Lx < 3 or Ly < 3:
        raise ValueError("torus sides must be >= 3")
    rng = np.random.default_rng(seed)
    r, c = np.divmod(np.arange(Lx * Ly, dtype=np.int64), Lx)
    v = r * Lx + c
    right = r * Lx + (c + 1) % Lx
    down = ((r + 1) % Ly) * Lx + c
    eu = np.stack([v, v], axis=1).reshape(-1).astype(np.int32)
    ev = np.stack([right, down], axis=1).reshape(-1).astype(np.int32)
    J = _couplings(rng, len(eu), weights)
    return Instance(f"torus{Lx}x{Ly}_s{seed}_{weights}", Lx * Ly, eu, ev, J,
                    meta={"family": "torus", "Lx": Lx, "Ly": Ly, "seed": seed,
                          "weights": weights})


def random_regular(n: int, d: int, seed: int = 2, weights: str = "maxcut1",
                   max_restarts: int = 1000) -> Instance:
    """Random simple d-regular graph by stub pairing: repeatedly join two random
    free stubs whose vertices are distinct and not yet adjacent; restart if the
    pairing gets stuck.  Edges are emitted in the order they are formed."""
    if (n * d) % 2 or d >= n:
        raise ValueError("n*d must be even and d < n")
    rng = np.random.default_rng(seed)
    for _ in range(max_restarts):
        stubs = np.repeat(np.arange(n, dtype=np.int64), d)
        rng.shuffle(stubs)
        stubs = list(stubs)
        adj = [set() for _ in range(n)]
        edges = []
        stuck = False
        while stubs:
            ok = False
            for _try in range(100):
                i = int(rng.integers(len(stubs)))
                j = int(rng.integers(len(stubs)))
                if i == j:
                    continue
                a, b = stubs[i], stubs[j]
                if a != b and b not in adj[a]:
                    ok = True
                    break
            if not ok:
                stuck = True
                break
            adj[a].add(b)
            adj[b].add(a)
            edges.append((a, b))
            for idx in sorted((i, j), reverse=True):
                stubs[idx] = stubs[-1]
                stubs.pop()
        if not stuck:
            e = np.array(edges, dtype=np.int32)
            J = _couplings(rng, len(e), weights)
            return Instance(f"rr{d}_n{n}_s{seed}_{weights}", n, e[:, 0].copy(), e[:, 1].copy(), J,
                            meta={"family": f"{d}-regular", "d": d, "seed": seed,
                                  "weights": weights})
    raise RuntimeError("random_regular: too many restarts")


def erdos_renyi_capped(n: int, mean_degree: float = 4.0, max_degree: int = 8, seed: int = 3,
                       weights: str = "pm1") -> Instance:
    """G(n, p) with p = mean_degree / (n - 1): candidate pairs (i < j) in
    lexicographic order, drawn by geometric skipping; a pair is dropped when
    either endpoint already has max_degree edges."""
    rng = np.random.default_rng(seed)
    p = mean_degree / (n - 1)
    deg = np.zeros(n, dtype=np.int64)
    eu, ev = [], []
    total = n * (n - 1) // 2
    pos = -1
    lp = np.log1p(-p)
    # enumerate pair index -> (i, j) for i < j, row by row
    row_start = np.concatenate([[0], np.cumsum(np.arange(n - 1, 0, -1))])
    while True:
        pos += 1 + int(np.floor(np.log(1.0 - rng.random()) / lp))
        if pos >= total:
            break
        i = int(np.searchsorted(row_start, pos, side="right") - 1)
        j = i + 1 + int(pos - row_start[i])
        if deg[i] >= max_degree or deg[j] >= max_degree:
            continue
        deg[i] += 1
        deg[j] += 1
        eu.append(i)
        ev.append(j)
    eu = np.array(eu, dtype=np.int32)
    ev = np.array(ev, dtype=np.int32)
    J = _couplings(rng, len(eu), weights)
    return Instance(f"er_n{n}_k{mean_degree}_cap{max_degree}_s{seed}_{weights}", n, eu, ev, J,
                    meta={"family": "erdos-renyi", "mean_degree": mean_degree,
                          "max_degree": max_degree, "seed": seed, "weights": weights})


def small_random(n: int, m: int, seed: int = 7, weights: str = "pm1") -> Instance:
    """m distinct random edges on n vertices (no self-loops), random orientation."""
    rng = np.random.default_rng(seed)
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    seen = set()
    eu, ev = [], []
    while len(eu) < m:
        a, b = (int(v) for v in rng.integers(n, size=2))
        if a == b or (min(a, b), max(a, b)) in seen:
            continue
        seen.add((min(a, b), max(a, b)))
        eu.append(a)
        ev.append(b)
    J = _couplings(rng, m, weights)
    return Instance(f"rand_n{n}_m{m}_s{seed}_{weights}", n, np.array(eu, dtype=np.int32),
                    np.array(ev, dtype=np.int32), J, meta={"family": "random", "seed": seed})


def trap_triangle() -> Instance:
    """Fig. 2: three spins, no frustration, two ground states (+,-,-) and (-,+,+)
    with Ising energy -3: J_01 = J_02 = -1, J_12 = +1."""
    eu = np.array([0, 0, 1], dtype=np.int32)
    ev = np.array([1, 2, 2], dtype=np.int32)
    J = np.array([-1, -1, 1], dtype=np.int32)
    return Instance("trap_triangle", 3, eu, ev, J, meta={"family": "trap"})


def cycle(n: int, weights: str = "ferro", seed: int = 0) -> Instance:
    rng = np.random.default_rng(seed)
    eu = np.arange(n, dtype=np.int32)
    ev = ((np.arange(n) + 1) % n).astype(np.int32)
    return Instance(f"cycle{n}_{weights}", n, eu, ev, _couplings(rng, n, weights),
                    meta={"family": "cycle"})


def request_stream(count: int = 256, n_min: int = 400, n_max: int = 20000, seed: int = 5,
                   rate_per_s: float | None = None):
    """Mixed solve requests: N uniform in [n_min, n_max], family uniform over
    {torus (side round(sqrt N)), 3-regular (+1 Max-Cut weights), 5-regular (+-1)};
    arrival times Poisson at rate_per_s (all at t = 0 when None).
    Returns a list of (arrival_s, Instance)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(count):
        n = int(rng.integers(n_min, n_max + 1))
        fam = int(rng.integers(3))
        s = int(rng.integers(1 << 30))
        if fam == 0:
            L = max(3, int(round(np.sqrt(n))))
            inst = torus(L, seed=s)
        elif fam == 1:
            inst = random_regular(n + (n % 2), 3, seed=s, weights="maxcut1")
        else:
            inst = random_regular(n + (n % 2), 5, seed=s, weights="pm1")
        if rate_per_s:
            t += float(rng.exponential(1.0 / rate_per_s))
        out.append((t, inst))
    return out
