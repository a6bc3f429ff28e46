// graph.cpp -- graph validation and the three edge colourings of
// cosm_build_partitions (Sec. II-B: "a proper edge coloring of the input
// graph"; classes are the matchings E_1..E_C of Eqs. (9)-(11)).
#include <algorithm>
#include <random>
#include <cstdio>
#include <numeric>

#include "internal.hpp"

namespace cosm {

int validate_graph(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                   std::vector<int32_t> *degree) {
  if (n < 1) return set_error(COSM_EINVAL, "n must be >= 1");
  if (m < 0) return set_error(COSM_EINVAL, "m must be >= 0");
  if (m > 0 && (eu == nullptr || ev == nullptr))
    return set_error(COSM_EINVAL, "edge arrays must not be NULL");
  std::vector<int64_t> keys((size_t)m);
  if (degree) degree->assign((size_t)n, 0);
  for (int64_t k = 0; k < m; k++) {
    int32_t a = eu[k], b = ev[k];
    if (a < 0 || b < 0 || a >= n || b >= n) {
      char buf[128];
      snprintf(buf, sizeof buf, "edge %lld has an endpoint out of range", (long long)k);
      return set_error(COSM_EINVAL, buf);
    }
    if (a == b) {
      char buf[128];
      snprintf(buf, sizeof buf, "edge %lld is a self-loop", (long long)k);
      return set_error(COSM_EINVAL, buf);
    }
    keys[(size_t)k] = (int64_t)std::min(a, b) * n + std::max(a, b);
    if (degree) {
      (*degree)[(size_t)a]++;
      (*degree)[(size_t)b]++;
    }
  }
  std::sort(keys.begin(), keys.end());
  for (size_t k = 1; k < keys.size(); k++)
    if (keys[k] == keys[k - 1]) {
      char buf[160];
      snprintf(buf, sizeof buf, "duplicate undirected edge (%lld, %lld)",
               (long long)(keys[k] / n), (long long)(keys[k] % n));
      return set_error(COSM_EDUP, buf);
    }
  return COSM_OK;
}

int validate_colouring(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                       const int32_t *colour, int32_t C) {
  if (m > 0 && colour == nullptr) return set_error(COSM_ECOLOR, "colour must not be NULL");
  if (C < 0 || (m > 0 && C < 1)) return set_error(COSM_ECOLOR, "bad number of colours");
  // last[v] = 1 + the last class seen at v; classes are checked one at a time
  std::vector<int64_t> order((size_t)m);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t k = 0; k < m; k++)
    if (colour[k] < 0 || colour[k] >= C)
      return set_error(COSM_ECOLOR, "colour index out of range");
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return colour[a] < colour[b]; });
  std::vector<int32_t> mark((size_t)n, -1);
  for (int64_t idx : order) {
    int32_t c = colour[idx];
    if (mark[(size_t)eu[idx]] == c || mark[(size_t)ev[idx]] == c) {
      char buf[160];
      snprintf(buf, sizeof buf, "class %d is not a matching (edge %lld shares a vertex)", c,
               (long long)idx);
      return set_error(COSM_ECOLOR, buf);
    }
    mark[(size_t)eu[idx]] = c;
    mark[(size_t)ev[idx]] = c;
  }
  return COSM_OK;
}

// Greedy: edges in input order, lowest colour absent at both endpoints.
int32_t colour_greedy(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                      int32_t *colour) {
  // colours present at each vertex, kept as a growable bitset
  std::vector<std::vector<uint64_t>> present((size_t)n);
  int32_t C = 0;
  auto has = [&](int32_t v, int32_t c) {
    const auto &b = present[(size_t)v];
    size_t w = (size_t)c >> 6;
    return w < b.size() && ((b[w] >> (c & 63)) & 1u);
  };
  auto add = [&](int32_t v, int32_t c) {
    auto &b = present[(size_t)v];
    size_t w = (size_t)c >> 6;
    if (b.size() <= w) b.resize(w + 1, 0);
    b[w] |= (uint64_t)1 << (c & 63);
  };
  for (int64_t k = 0; k < m; k++) {
    int32_t c = 0;
    while (has(eu[k], c) || has(ev[k], c)) c++;
    colour[k] = c;
    add(eu[k], c);
    add(ev[k], c);
    C = std::max(C, c + 1);
  }
  return C;
}

// Misra-Gries: a constructive proof of Vizing's theorem that colours every
// simple graph with at most Delta + 1 colours.  Edges are taken in input order.
int32_t colour_misra_gries(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                           int32_t *colour) {
  std::vector<int32_t> deg((size_t)n, 0);
  for (int64_t k = 0; k < m; k++) {
    deg[(size_t)eu[k]]++;
    deg[(size_t)ev[k]]++;
  }
  const int32_t delta = m ? *std::max_element(deg.begin(), deg.end()) : 0;
  const int32_t K = delta + 1;  // palette size
  // at[v*K + c] = edge with colour c at v, or -1
  std::vector<int64_t> at((size_t)n * K, -1);
  std::vector<int32_t> col((size_t)m, -1);
  // incident edges per vertex
  std::vector<int64_t> start((size_t)n + 1, 0), inc((size_t)(2 * m));
  for (int64_t k = 0; k < m; k++) {
    start[(size_t)eu[k] + 1]++;
    start[(size_t)ev[k] + 1]++;
  }
  for (int32_t v = 0; v < n; v++) start[(size_t)v + 1] += start[(size_t)v];
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t k = 0; k < m; k++) {
      inc[(size_t)fill[(size_t)eu[k]]++] = k;
      inc[(size_t)fill[(size_t)ev[k]]++] = k;
    }
  }
  auto other = [&](int64_t e, int32_t v) { return eu[e] == v ? ev[e] : eu[e]; };
  auto is_free = [&](int32_t v, int32_t c) { return at[(size_t)v * K + c] < 0; };
  auto first_free = [&](int32_t v) {
    for (int32_t c = 0; c < K; c++)
      if (is_free(v, c)) return c;
    return -1;  // cannot happen: deg(v) <= delta < K
  };
  auto set_col = [&](int64_t e, int32_t c) {
    if (col[(size_t)e] >= 0) {
      at[(size_t)eu[e] * K + col[(size_t)e]] = -1;
      at[(size_t)ev[e] * K + col[(size_t)e]] = -1;
    }
    col[(size_t)e] = c;
    if (c >= 0) {
      at[(size_t)eu[e] * K + c] = e;
      at[(size_t)ev[e] * K + c] = e;
    }
  };
  auto edge_between = [&](int32_t u, int32_t x) -> int64_t {
    for (int64_t a = start[(size_t)u]; a < start[(size_t)u + 1]; a++)
      if (other(inc[(size_t)a], u) == x) return inc[(size_t)a];
    return -1;
  };

  std::vector<int32_t> fan;
  std::vector<char> in_fan((size_t)n, 0);
  std::vector<int64_t> path;
  for (int64_t e0 = 0; e0 < m; e0++) {
    const int32_t u = eu[e0], v = ev[e0];
    // maximal fan of u starting at v: colour(u, F[i+1]) is free on F[i]
    fan.assign(1, v);
    in_fan[(size_t)v] = 1;
    for (bool grown = true; grown;) {
      grown = false;
      const int32_t last = fan.back();
      for (int32_t c = 0; c < K && !grown; c++) {
        if (!is_free(last, c)) continue;
        const int64_t e = at[(size_t)u * K + c];
        if (e < 0) continue;
        const int32_t x = other(e, u);
        if (in_fan[(size_t)x]) continue;
        fan.push_back(x);
        in_fan[(size_t)x] = 1;
        grown = true;
      }
    }
    const int32_t c = first_free(u);
    const int32_t d = first_free(fan.back());
    // invert the cd_u path: from u follow d, c, d, ... and swap c <-> d
    if (c != d) {
      path.clear();
      int32_t cur = u, want = d;
      while (true) {
        const int64_t e = at[(size_t)cur * K + want];
        if (e < 0) break;
        path.push_back(e);
        cur = other(e, cur);
        want = (want == d) ? c : d;
      }
      std::vector<int32_t> newc(path.size());
      for (size_t a = 0; a < path.size(); a++) newc[a] = col[(size_t)path[a]] == c ? d : c;
      for (int64_t e : path) set_col(e, -1);
      for (size_t a = 0; a < path.size(); a++) set_col(path[a], newc[a]);
    }
    // w: first fan vertex with d free such that F[0..w] is still a fan
    int32_t wi = -1;
    for (size_t i = 0; i < fan.size() && wi < 0; i++) {
      if (!is_free(fan[i], d)) continue;
      bool ok = true;
      for (size_t j = 0; j + 1 <= i && ok; j++) {
        const int64_t e = edge_between(u, fan[j + 1]);
        ok = e >= 0 && col[(size_t)e] >= 0 && is_free(fan[j], col[(size_t)e]);
      }
      if (ok) wi = (int32_t)i;
    }
    if (wi < 0) wi = 0;  // unreachable for a correct fan; keeps the loop total
    // rotate F[0..w]: colour(u, F[i]) <- colour(u, F[i+1]), then (u, F[w]) gets d
    for (int32_t i = 0; i < wi; i++) {
      const int64_t ei = edge_between(u, fan[(size_t)i]);
      const int64_t ej = edge_between(u, fan[(size_t)i + 1]);
      const int32_t cj = col[(size_t)ej];
      set_col(ej, -1);
      set_col(ei, cj);
    }
    set_col(edge_between(u, fan[(size_t)wi]), d);
    for (int32_t x : fan) in_fan[(size_t)x] = 0;
  }
  // renumber the colours in use to 0..C-1, keeping their order
  std::vector<int32_t> remap((size_t)K, -1);
  for (int64_t k = 0; k < m; k++) remap[(size_t)col[(size_t)k]] = 0;
  int32_t C = 0;
  for (int32_t c = 0; c < K; c++)
    if (remap[(size_t)c] == 0) remap[(size_t)c] = C++;
  for (int64_t k = 0; k < m; k++) colour[k] = remap[(size_t)col[(size_t)k]];
  return C;
}

// Equalise class sizes of a proper colouring without adding colours: while the
// largest class a exceeds the smallest b by more than one edge, swap a <-> b on
// a maximal a/b alternating path that holds one more a-edge than b-edges (one
// exists whenever |a| > |b|).  Every swap keeps the colouring proper.
void equalise_classes(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, int32_t C,
                      int32_t *colour) {
  if (C < 2 || m == 0) return;
  std::vector<int64_t> size((size_t)C, 0);
  for (int64_t k = 0; k < m; k++) size[(size_t)colour[k]]++;
  // edge of colour c at vertex v
  std::vector<int64_t> at((size_t)n * C, -1);
  for (int64_t k = 0; k < m; k++) {
    at[(size_t)eu[k] * C + colour[k]] = k;
    at[(size_t)ev[k] * C + colour[k]] = k;
  }
  auto other = [&](int64_t e, int32_t v) { return eu[e] == v ? ev[e] : eu[e]; };
  std::vector<int64_t> path;
  for (int64_t guard = 0; guard < 4 * m + 16; guard++) {
    int32_t a = 0, b = 0;
    for (int32_t c = 1; c < C; c++) {
      if (size[(size_t)c] > size[(size_t)a]) a = c;
      if (size[(size_t)c] < size[(size_t)b]) b = c;
    }
    if (size[(size_t)a] - size[(size_t)b] <= 1) break;
    bool swapped = false;
    // a path with more a- than b-edges starts at a vertex with an a-edge and no b-edge
    for (int32_t v0 = 0; v0 < n && !swapped; v0++) {
      if (at[(size_t)v0 * C + a] < 0 || at[(size_t)v0 * C + b] >= 0) continue;
      path.clear();
      int32_t v = v0, want = a;
      int64_t na = 0, nb = 0;
      while (true) {
        const int64_t e = at[(size_t)v * C + want];
        if (e < 0) break;
        path.push_back(e);
        (want == a ? na : nb)++;
        v = other(e, v);
        want = (want == a) ? b : a;
      }
      if (na <= nb) continue;
      for (int64_t e : path) {
        at[(size_t)eu[e] * C + colour[e]] = -1;
        at[(size_t)ev[e] * C + colour[e]] = -1;
      }
      for (int64_t e : path) {
        colour[e] = colour[e] == a ? b : a;
        at[(size_t)eu[e] * C + colour[e]] = e;
        at[(size_t)ev[e] * C + colour[e]] = e;
      }
      size[(size_t)a]--;
      size[(size_t)b]++;
      swapped = true;
    }
    if (!swapped) break;
  }
}

// Regular lattice pattern for an Lx x Ly torus (vertex r*Lx + c).
int32_t colour_torus(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, int32_t Lx,
                     int32_t Ly, int32_t *colour) {
  if (Lx < 3 || Ly < 3 || (int64_t)Lx * Ly != n)
    return set_error(COSM_EINVAL, "TORUS needs {Lx, Ly} with Lx, Ly >= 3 and Lx*Ly == n");
  // raw classes: 0 H-even, 1 H-odd, 2 V-even, 3 V-odd, 4 H-wrap (odd Lx), 5 V-wrap (odd Ly)
  bool used[6] = {false, false, false, false, false, false};
  for (int64_t k = 0; k < m; k++) {
    const int32_t ra = eu[k] / Lx, ca = eu[k] % Lx, rb = ev[k] / Lx, cb = ev[k] % Lx;
    int32_t cls = -1;
    if (ra == rb) {
      int32_t left = -1;
      if (cb == (ca + 1) % Lx) left = ca;
      else if (ca == (cb + 1) % Lx) left = cb;
      if (left >= 0) cls = (Lx % 2 == 1 && left == Lx - 1) ? 4 : (left % 2);
    } else if (ca == cb) {
      int32_t up = -1;
      if (rb == (ra + 1) % Ly) up = ra;
      else if (ra == (rb + 1) % Ly) up = rb;
      if (up >= 0) cls = (Ly % 2 == 1 && up == Ly - 1) ? 5 : 2 + (up % 2);
    }
    if (cls < 0) {
      char buf[160];
      snprintf(buf, sizeof buf, "edge %lld does not join torus neighbours", (long long)k);
      return set_error(COSM_EINVAL, buf);
    }
    colour[k] = cls;
    used[cls] = true;
  }
  int32_t remap[6], C = 0;
  for (int c = 0; c < 6; c++) remap[c] = used[c] ? C++ : -1;
  for (int64_t k = 0; k < m; k++) colour[k] = remap[colour[k]];
  return C;
}

// Delta-edge-colouring attempt ("minimum colouring", which the paper reports
// its greedy heuristic reached on its non-lattice graphs).  Start from
// Misra-Gries (<= Delta + 1 colours).  If it used colour Delta, move each edge
// e = (u, v) of that colour into [0, Delta): with a free at u and b free at v,
// either one colour is free at both, or swapping the (a, b)-alternating path
// that starts at v (v lacks b, so the path ends there) frees a at v while a
// stays free at u -- unless the path ends at u.  Edges left over after a pass
// wait for the next one, after a random Kempe-chain swap elsewhere changes the
// colouring.  Gives up after a fixed number of passes and then keeps
// Delta + 1 colours (graphs of class 2, such as the Petersen graph, need them).
// Returns the number of colours.
int32_t colour_minimum(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                       int32_t *colour) {
  int32_t C = colour_misra_gries(n, m, eu, ev, colour);
  if (m == 0) return C;
  std::vector<int32_t> deg((size_t)n, 0);
  for (int64_t k = 0; k < m; k++) {
    deg[(size_t)eu[k]]++;
    deg[(size_t)ev[k]]++;
  }
  const int32_t delta = *std::max_element(deg.begin(), deg.end());
  if (C <= delta) return C;
  const int32_t K = delta + 1;
  std::vector<int64_t> at((size_t)n * K, -1);
  for (int64_t k = 0; k < m; k++) {
    at[(size_t)eu[k] * K + colour[k]] = k;
    at[(size_t)ev[k] * K + colour[k]] = k;
  }
  auto other = [&](int64_t e, int32_t v) { return eu[e] == v ? ev[e] : eu[e]; };
  auto set_colour = [&](int64_t e, int32_t c) {
    at[(size_t)eu[e] * K + colour[e]] = -1;
    at[(size_t)ev[e] * K + colour[e]] = -1;
    colour[e] = c;
    at[(size_t)eu[e] * K + c] = e;
    at[(size_t)ev[e] * K + c] = e;
  };
  // the maximal (a, b)-alternating path from v, which must lack b
  std::vector<int64_t> path;
  auto chain_from = [&](int32_t v, int32_t a, int32_t b) {
    path.clear();
    int32_t want = a;
    while (true) {
      const int64_t e = at[(size_t)v * K + want];
      if (e < 0) break;
      path.push_back(e);
      v = other(e, v);
      want = want == a ? b : a;
    }
    return v;  // the other end
  };
  auto swap_path = [&](int32_t a, int32_t b) {
    for (int64_t e : path) {
      at[(size_t)eu[e] * K + colour[e]] = -1;
      at[(size_t)ev[e] * K + colour[e]] = -1;
    }
    for (int64_t e : path) {
      colour[e] = colour[e] == a ? b : a;
      at[(size_t)eu[e] * K + colour[e]] = e;
      at[(size_t)ev[e] * K + colour[e]] = e;
    }
  };
  std::vector<int64_t> extra;
  for (int64_t k = 0; k < m; k++)
    if (colour[k] == delta) extra.push_back(k);
  std::mt19937_64 rng(0x5eed5eedull);
  for (int pass = 0; pass < 400 && !extra.empty(); pass++) {
    std::vector<int64_t> left;
    for (int64_t e : extra) {
      const int32_t u = eu[e], v = ev[e];
      bool done = false;
      for (int32_t a = 0; a < delta && !done; a++) {
        if (at[(size_t)u * K + a] >= 0) continue;
        if (at[(size_t)v * K + a] < 0) {
          set_colour(e, a);
          done = true;
          break;
        }
        for (int32_t b = 0; b < delta && !done; b++) {
          if (b == a || at[(size_t)v * K + b] >= 0) continue;
          if (chain_from(v, a, b) == u) continue;
          bool touches_u = false;
          for (int64_t f : path) touches_u |= (eu[f] == u || ev[f] == u);
          if (touches_u) continue;
          swap_path(a, b);
          set_colour(e, a);
          done = true;
        }
      }
      if (!done) left.push_back(e);
    }
    extra.swap(left);
    if (extra.empty()) break;
    // perturb: swap a random Kempe chain that starts at a chain end
    for (int tries = 0; tries < 64; tries++) {
      const int32_t x = (int32_t)(rng() % (uint64_t)n);
      const int32_t a = (int32_t)(rng() % (uint64_t)delta), b = (int32_t)(rng() % (uint64_t)delta);
      if (a == b || at[(size_t)x * K + a] < 0 || at[(size_t)x * K + b] >= 0) continue;
      chain_from(x, a, b);
      swap_path(a, b);
      break;
    }
  }
  if (!extra.empty()) return C;
  return delta;
}

}  // namespace cosm
