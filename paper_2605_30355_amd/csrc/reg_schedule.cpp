// reg_schedule.cpp -- the register-owner form of the LDS-resident sweep.
//
// In the pair form every edge update reads and writes both endpoint rows in
// LDS.  Here an independent set I of vertices is held in registers: thread t
// owns up to K of them, and every edge with an endpoint in I is updated by
// that endpoint's owner, which reads and writes only the other endpoint's row
// (no two vertices of I are adjacent, so each edge has at most one register
// endpoint).  Edges with no endpoint in I keep the pair form, one slot per
// class.  On a bipartite graph (the even tori) one side is I and every update
// touches LDS once instead of twice; on a random 3-regular graph about 0.43 n
// vertices cover about 86 % of the edges.
//
// Bank layout (the gfx950 LDS model of schedule.cpp): in each aligned group of
// G lanes (G = 64 / W, 32 for W = 1) the rows of one access must be distinct
// mod G, and in each aligned half of H = 32 / W lanes distinct mod H.  Rows
// are numbered residue-major (row = rho + G i), and the residue rho of each
// LDS vertex is chosen while the register vertices are packed into groups:
// a vertex joins a group only if, class by class, its neighbours' residues are
// still free there (unassigned neighbours take a free residue).  Lanes without
// an edge get dummy rows n_rows + rho with residues free in their group, so the
// register slots' accesses are conflict-free and need no branch.  The pair
// slot's edges are packed the same way, group by group from lane 0 (a wave
// without one skips the slot); edges that find no conflict-free lane take any
// free lane and are counted in reg_conflicts.
//
// The class order and the edge set per class are unchanged: only which thread
// applies an update, and in which register or LDS row the phases sit, differ.
#include <algorithm>
#include <map>
#include <numeric>

#include "internal.hpp"

namespace cosm {

namespace {

struct Adj {
  int32_t other;
  int32_t edge;
  int32_t cls;
};

// Vertices of one side of a 2-colouring per connected component (the side
// with fewer vertices), or an empty result when the graph has an odd cycle.
bool bipartite_side(int32_t n, const std::vector<std::vector<Adj>> &adj,
                    std::vector<uint8_t> *in_set) {
  std::vector<int8_t> side((size_t)n, -1);
  std::vector<int32_t> queue, comp;
  in_set->assign((size_t)n, 0);
  for (int32_t s0 = 0; s0 < n; s0++) {
    if (side[(size_t)s0] >= 0 || adj[(size_t)s0].empty()) continue;
    side[(size_t)s0] = 0;
    queue.assign(1, s0);
    comp.clear();
    int32_t count[2] = {0, 0};
    for (size_t h = 0; h < queue.size(); h++) {
      const int32_t v = queue[h];
      comp.push_back(v);
      count[side[(size_t)v]]++;
      for (const Adj &a : adj[(size_t)v]) {
        if (side[(size_t)a.other] < 0) {
          side[(size_t)a.other] = (int8_t)(1 - side[(size_t)v]);
          queue.push_back(a.other);
        } else if (side[(size_t)a.other] == side[(size_t)v]) {
          return false;
        }
      }
    }
    const int8_t pick = count[1] < count[0] ? 1 : 0;
    for (int32_t v : comp)
      if (side[(size_t)v] == pick) (*in_set)[(size_t)v] = 1;
  }
  return true;
}

// Greedy independent set: repeatedly take a vertex of minimum remaining
// degree (isolated vertices excluded: they have nothing to cover).
void greedy_independent(int32_t n, const std::vector<std::vector<Adj>> &adj,
                        std::vector<uint8_t> *in_set) {
  in_set->assign((size_t)n, 0);
  std::vector<int32_t> deg((size_t)n);
  int32_t dmax = 0;
  for (int32_t v = 0; v < n; v++) {
    deg[(size_t)v] = (int32_t)adj[(size_t)v].size();
    dmax = std::max(dmax, deg[(size_t)v]);
  }
  std::vector<std::vector<int32_t>> bucket((size_t)dmax + 1);
  for (int32_t v = n - 1; v >= 0; v--)
    if (deg[(size_t)v] > 0) bucket[(size_t)deg[(size_t)v]].push_back(v);
  std::vector<uint8_t> gone((size_t)n, 0);
  for (int32_t v = 0; v < n; v++)
    if (deg[(size_t)v] == 0) gone[(size_t)v] = 1;
  int32_t d = 0;
  while (true) {
    while (d <= dmax && bucket[(size_t)d].empty()) d++;
    if (d > dmax) break;
    const int32_t v = bucket[(size_t)d].back();
    bucket[(size_t)d].pop_back();
    if (gone[(size_t)v] || deg[(size_t)v] != d) continue;  // stale entry
    (*in_set)[(size_t)v] = 1;
    gone[(size_t)v] = 1;
    for (const Adj &a : adj[(size_t)v]) {
      const int32_t w = a.other;
      if (gone[(size_t)w]) continue;
      gone[(size_t)w] = 1;
      for (const Adj &b : adj[(size_t)w]) {
        const int32_t x = b.other;
        if (gone[(size_t)x]) continue;
        deg[(size_t)x]--;
        bucket[(size_t)deg[(size_t)x]].push_back(x);
        d = std::min(d, deg[(size_t)x]);
      }
    }
  }
}

// Enlarges an independent set by 2-improvements (the local search of Andrade,
// Resende and Werneck, 2012): a set vertex x leaves when two of its
// neighbours that have x as their only set neighbour, and are not adjacent to
// each other, can enter instead.  Repeated until no vertex offers such a pair;
// every step keeps the set independent and grows it by one.
void improve_independent(int32_t n, const std::vector<std::vector<Adj>> &adj,
                         std::vector<uint8_t> *in_set) {
  std::vector<uint8_t> &I = *in_set;
  std::vector<int32_t> tight((size_t)n, 0);  // set neighbours of a vertex
  for (int32_t v = 0; v < n; v++)
    if (I[(size_t)v])
      for (const Adj &a : adj[(size_t)v]) tight[(size_t)a.other]++;
  auto adjacent = [&](int32_t a, int32_t b) {
    for (const Adj &e : adj[(size_t)a])
      if (e.other == b) return true;
    return false;
  };
  std::vector<int32_t> queue;
  std::vector<uint8_t> queued((size_t)n, 0);
  for (int32_t v = 0; v < n; v++)
    if (I[(size_t)v]) {
      queue.push_back(v);
      queued[(size_t)v] = 1;
    }
  std::vector<int32_t> one;
  for (size_t h = 0; h < queue.size(); h++) {
    const int32_t x = queue[h];
    queued[(size_t)x] = 0;
    if (!I[(size_t)x]) continue;
    one.clear();
    for (const Adj &a : adj[(size_t)x])
      if (!I[(size_t)a.other] && tight[(size_t)a.other] == 1) one.push_back(a.other);
    int32_t w1 = -1, w2 = -1;
    for (size_t i = 0; i < one.size() && w1 < 0; i++)
      for (size_t j = i + 1; j < one.size(); j++)
        if (one[i] != one[j] && !adjacent(one[i], one[j])) {
          w1 = one[i];
          w2 = one[j];
          break;
        }
    if (w1 < 0) continue;
    // x leaves, w1 and w2 enter
    I[(size_t)x] = 0;
    for (const Adj &a : adj[(size_t)x]) tight[(size_t)a.other]--;
    for (int32_t w : {w1, w2}) {
      I[(size_t)w] = 1;
      for (const Adj &a : adj[(size_t)w]) tight[(size_t)a.other]++;
    }
    // the set vertices near the change may now offer a pair
    for (int32_t w : {x, w1, w2})
      for (const Adj &a : adj[(size_t)w])
        for (const Adj &b : adj[(size_t)a.other])
          if (I[(size_t)b.other] && !queued[(size_t)b.other]) {
            queued[(size_t)b.other] = 1;
            queue.push_back(b.other);
          }
    for (int32_t w : {w1, w2})
      if (!queued[(size_t)w]) {
        queued[(size_t)w] = 1;
        queue.push_back(w);
      }
  }
}

// An independent set for a graph that is not bipartite: the larger of (a) the
// minimum-degree greedy set and (b) a side of the breadth-first parity
// colouring with the vertices that have a neighbour on their own side dropped
// (first come, first kept) and the set then made maximal -- nearly half of a
// graph that is bipartite but for a few odd cycles, as an odd torus is --
// each enlarged by 2-improvements.
void large_independent(int32_t n, const std::vector<std::vector<Adj>> &adj,
                       std::vector<uint8_t> *in_set) {
  greedy_independent(n, adj, in_set);
  improve_independent(n, adj, in_set);
  int64_t best = 0;
  for (uint8_t b : *in_set) best += b;
  std::vector<int32_t> depth((size_t)n, -1), queue;
  for (int32_t s0 = 0; s0 < n; s0++) {
    if (depth[(size_t)s0] >= 0 || adj[(size_t)s0].empty()) continue;
    depth[(size_t)s0] = 0;
    queue.assign(1, s0);
    for (size_t h = 0; h < queue.size(); h++)
      for (const Adj &a : adj[(size_t)queue[h]])
        if (depth[(size_t)a.other] < 0) {
          depth[(size_t)a.other] = depth[(size_t)queue[h]] + 1;
          queue.push_back(a.other);
        }
  }
  for (int32_t side : {0, 1}) {
    std::vector<uint8_t> S((size_t)n, 0);
    for (int32_t v = 0; v < n; v++) S[(size_t)v] = depth[(size_t)v] >= 0 && depth[(size_t)v] % 2 == side;
    auto has_set_neighbour = [&](int32_t v) {
      for (const Adj &a : adj[(size_t)v])
        if (S[(size_t)a.other]) return true;
      return false;
    };
    for (int32_t v = 0; v < n; v++)
      if (S[(size_t)v] && has_set_neighbour(v)) S[(size_t)v] = 0;
    for (int32_t v = 0; v < n; v++)
      if (!S[(size_t)v] && depth[(size_t)v] >= 0 && !has_set_neighbour(v)) S[(size_t)v] = 1;
    improve_independent(n, adj, &S);
    int64_t size = 0;
    for (uint8_t b : S) size += b;
    if (size > best) {
      best = size;
      *in_set = std::move(S);
    }
  }
}

inline uint64_t bit(int32_t r) { return 1ull << r; }

// Options of one attempt.  pre: every LDS vertex takes residue (its rank among
// the LDS vertices, in vertex order) mod G before the packing, which keeps
// lattice neighbourhoods aligned; otherwise residues are chosen during the
// packing.  rstream: the streamed form (up to kRStreamKMax register rows and
// kRStreamPairs pair slots per class, and its own encoding); the register
// vertices are then ordered by their pattern (the classes they have an edge
// in, and those where they are the edge's v), most common pattern first, so
// that vertices with the same pattern share waves and a class leaves the
// register slots of the rare patterns (the seams of an odd torus) to a few
// waves.
struct RegOptions {
  int32_t W = 0, K = 0, nth_request = 0;
  bool pre = false;
  bool rstream = false;
};

// One lane's entry in a register slot: the LDS endpoint's row (or a dummy
// row), whether the register vertex is the edge's v, and J (0: no edge).
struct RegEntry {
  int32_t row = 0;
  bool flip = false;
  int32_t J = 0;
};
// One lane's entry in a pair slot (rows of u and v, J; 0: dummy rows).
struct PairEntry {
  int32_t ru = 0, rv = 0;
  int32_t J = 0;
};

int build_reg_impl(const cosm_state &s, const RegOptions &o, LdsSchedule *out) {
  const int32_t n = s.n, C = s.C, W = o.W, K = o.K;
  const int64_t m = s.m;
  const int32_t P = o.rstream ? kRStreamPairs : 1;  // pair slots per class
  if (W != 1 && W != 2 && W != 4) return set_error(COSM_EINVAL, "bad row width");
  if (K < 1 || K > (o.rstream ? kRStreamKMax : kRegKMax))
    return set_error(COSM_EINVAL, "bad register count");
  if (C > (o.rstream ? kRStreamClassesMax : kRegClassesMax))
    return set_error(COSM_ERANGE, "too many classes for the register form");
  if (s.has_h) return set_error(COSM_ERANGE, "the register form runs without bias fields");
  if (m == 0) return set_error(COSM_ERANGE, "no edges");
  if (o.rstream) {
    // the pair slots' words hold J in 14 bits and row offsets in 18
    for (int64_t k = 0; k < m; k++)
      if (s.h_J[(size_t)k] >= 8192 || s.h_J[(size_t)k] < -8192)
        return set_error(COSM_ERANGE, "the streamed register form needs |J| < 2^13");
  }
  const int32_t G = W == 1 ? 32 : 64 / W;  // lanes and residues of a read group
  const int32_t H = 32 / W;                // lanes and residues of a write half

  std::vector<std::vector<Adj>> adj((size_t)n);
  for (int64_t k = 0; k < m; k++) {
    const int32_t u = s.h_eu[(size_t)k], v = s.h_ev[(size_t)k], c = s.h_colour[(size_t)k];
    adj[(size_t)u].push_back({v, (int32_t)k, c});
    adj[(size_t)v].push_back({u, (int32_t)k, c});
  }

  // 1. the register set
  std::vector<uint8_t> inI;
  if (!bipartite_side(n, adj, &inI)) large_independent(n, adj, &inI);
  std::vector<int32_t> cand;
  for (int32_t v = 0; v < n; v++)
    if (inI[(size_t)v]) cand.push_back(v);
  int32_t nth = o.nth_request;
  if (nth <= 0) {
    const int64_t need = ((int64_t)cand.size() + K - 1) / K;
    nth = (int32_t)std::min<int64_t>(1024, std::max<int64_t>(64, (need + 63) / 64 * 64));
  }
  if (nth % 64 != 0 || nth < 64 || nth > 1024) return set_error(COSM_EINVAL, "bad thread count");
  const int64_t cap = (int64_t)K * nth;
  const int64_t set_size = (int64_t)cand.size();
  if ((int64_t)cand.size() > cap) {
    // keep the vertices that cover the most edges
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
      return adj[(size_t)a].size() > adj[(size_t)b].size();
    });
    for (size_t i = (size_t)cap; i < cand.size(); i++) inI[(size_t)cand[i]] = 0;
    cand.resize((size_t)cap);
    std::sort(cand.begin(), cand.end());
  }
  std::vector<uint8_t> rclass((size_t)C, 1);  // classes with register slots
  if (o.rstream) {
    // The streamed form runs a class's register slots on every wave or on
    // none: only classes where at least half of the register set has an edge
    // get them, and a vertex with an edge in another class (the seams of an
    // odd torus) goes back to LDS.
    for (int iter = 0; iter < 8; iter++) {
      std::vector<int64_t> cnt((size_t)C, 0);
      for (int32_t v : cand)
        for (const Adj &a : adj[(size_t)v]) cnt[(size_t)a.cls]++;
      bool changed = false;
      for (int32_t c = 0; c < C; c++) {
        const uint8_t r = cnt[(size_t)c] * 2 >= (int64_t)cand.size() ? 1 : 0;
        if (r != rclass[(size_t)c]) changed = true;
        rclass[(size_t)c] = r;
      }
      std::vector<int32_t> keep;
      for (int32_t v : cand) {
        bool ok = true;
        for (const Adj &a : adj[(size_t)v])
          if (!rclass[(size_t)a.cls]) ok = false;
        if (ok) keep.push_back(v);
        else inI[(size_t)v] = 0;
      }
      if (keep.size() != cand.size()) changed = true;
      cand.swap(keep);
      if (!changed) break;
    }
    if (cand.empty()) return set_error(COSM_ERANGE, "no register set for the streamed form");
    std::vector<uint64_t> pattern((size_t)n, 0);
    std::map<uint64_t, int64_t> freq;
    for (int32_t v : cand) {
      uint64_t sig = 0, flips = 0;
      for (const Adj &a : adj[(size_t)v]) {
        sig |= 1ull << a.cls;
        if (s.h_ev[(size_t)a.edge] == v) flips |= 1ull << a.cls;
      }
      pattern[(size_t)v] = sig << 32 | flips;
      freq[pattern[(size_t)v]]++;
    }
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
      const uint64_t pa = pattern[(size_t)a], pb = pattern[(size_t)b];
      const int64_t fa = freq[pa], fb = freq[pb];
      return fa != fb ? fa > fb : pa < pb;
    });
  }

  // 2. pack the register vertices into lane groups, choosing residues
  const int32_t groups_per_k = nth / G;
  const int32_t ngroups = groups_per_k * K;
  std::vector<int32_t> res((size_t)n, -1);
  std::vector<int64_t> load((size_t)G, 0);
  std::vector<uint64_t> usedG((size_t)ngroups * C, 0);
  std::vector<uint64_t> usedH((size_t)ngroups * 2 * C, 0);
  std::vector<int32_t> pos_vertex((size_t)K * nth, -1);  // [k][t]
  auto pick_free = [&](uint64_t gmask, uint64_t hmask) {
    int32_t best = -1;
    for (int32_t r = 0; r < G; r++) {
      if ((gmask >> r) & 1u) continue;
      if ((hmask >> (r % H)) & 1u) continue;
      if (best < 0 || load[(size_t)r] < load[(size_t)best]) best = r;
    }
    return best;
  };
  if (o.pre) {
    int32_t rank = 0;
    for (int32_t v = 0; v < n; v++) {
      if (inI[(size_t)v]) continue;
      res[(size_t)v] = rank++ % G;
      load[(size_t)res[(size_t)v]]++;
    }
  }
  std::vector<uint8_t> placed((size_t)n, 0);
  size_t first_open = 0;  // cand[0 .. first_open) are all placed
  for (int32_t gi = 0; gi < ngroups && first_open < cand.size(); gi++) {
    const int32_t k = gi / groups_per_k, tg = gi % groups_per_k;
    for (int32_t p = 0; p < G; p++) {
      const int32_t half = p / H;
      int32_t chosen = -1;
      int32_t scanned = 0;
      for (size_t i = first_open; i < cand.size() && scanned < 2048; i++) {
        const int32_t v = cand[i];
        if (placed[(size_t)v]) continue;
        scanned++;
        bool ok = true;
        for (const Adj &a : adj[(size_t)v]) {
          const uint64_t gm = usedG[(size_t)gi * C + a.cls];
          const uint64_t hm = usedH[((size_t)gi * 2 + half) * C + a.cls];
          const int32_t r = res[(size_t)a.other];
          if (r >= 0 ? (((gm >> r) & 1u) || ((hm >> (r % H)) & 1u)) : pick_free(gm, hm) < 0) {
            ok = false;
            break;
          }
        }
        if (ok) {
          chosen = v;
          break;
        }
      }
      if (chosen < 0) {  // nothing fits this half any more: on to the next half
        p = (half + 1) * H - 1;
        continue;
      }
      placed[(size_t)chosen] = 1;
      pos_vertex[(size_t)k * nth + tg * G + p] = chosen;
      for (const Adj &a : adj[(size_t)chosen]) {
        uint64_t &gm = usedG[(size_t)gi * C + a.cls];
        uint64_t &hm = usedH[((size_t)gi * 2 + half) * C + a.cls];
        int32_t &r = res[(size_t)a.other];
        if (r < 0) {
          r = pick_free(gm, hm);
          load[(size_t)r]++;
        }
        gm |= bit(r);
        hm |= bit(r % H);
      }
      while (first_open < cand.size() && placed[(size_t)cand[first_open]]) first_open++;
    }
  }
  // register vertices that found no place go back to LDS
  int64_t reg_edges = 0;
  for (int32_t v : cand) {
    if (!placed[(size_t)v]) inI[(size_t)v] = 0;
    else reg_edges += (int64_t)adj[(size_t)v].size();
  }

  // 3. edges between two LDS rows: P slots per class
  std::vector<std::vector<int32_t>> free_edges((size_t)C);
  for (int64_t k = 0; k < m; k++) {
    const int32_t u = s.h_eu[(size_t)k], v = s.h_ev[(size_t)k];
    if (!inI[(size_t)u] && !inI[(size_t)v]) free_edges[(size_t)s.h_colour[(size_t)k]].push_back((int32_t)k);
  }
  int32_t reg_free = 0;
  for (int32_t c = 0; c < C; c++) {
    if ((int64_t)free_edges[(size_t)c].size() > (int64_t)P * nth)
      return set_error(COSM_ERANGE, "too many edges outside the register set");
    if (!free_edges[(size_t)c].empty()) reg_free = 1;
  }
  // per class and pair slot: lane of each free edge; u-rows and v-rows
  // conflict-free per group (masks per class, slot and group; halves apart)
  const size_t nps = (size_t)C * P;  // (class, pair slot) pairs
  std::vector<int32_t> free_at(nps * nth, -1);
  std::vector<uint64_t> fG(nps * groups_per_k * 2, 0), fH(nps * groups_per_k * 4, 0);
  auto fmask = [&](size_t cp, int32_t tg, int32_t half, uint64_t **gU, uint64_t **gV,
                   uint64_t **hU, uint64_t **hV) {
    *gU = &fG[(cp * groups_per_k + tg) * 2];
    *gV = *gU + 1;
    *hU = &fH[((cp * groups_per_k + tg) * 2 + half) * 2];
    *hV = *hU + 1;
  };
  int64_t conflicts = 0;
  for (int32_t c = 0; c < C; c++) {
    std::vector<int32_t> &list = free_edges[(size_t)c];
    std::vector<uint8_t> done(list.size(), 0);
    size_t left = list.size();
    for (int32_t ps = 0; ps < P && left > 0; ps++) {
      const size_t cp = (size_t)c * P + ps;
      for (int32_t tg = 0; tg < groups_per_k && left > 0; tg++) {
        for (int32_t p = 0; p < G && left > 0; p++) {
          const int32_t half = p / H;
          uint64_t *gU, *gV, *hU, *hV;
          fmask(cp, tg, half, &gU, &gV, &hU, &hV);
          int32_t chosen = -1;
          for (size_t i = 0; i < list.size(); i++) {
            if (done[i]) continue;
            const int32_t e = list[i];
            const int32_t u = s.h_eu[(size_t)e], v = s.h_ev[(size_t)e];
            const int32_t ru = res[(size_t)u], rv = res[(size_t)v];
            const bool uok = ru >= 0 ? !(((*gU >> ru) & 1u) || ((*hU >> (ru % H)) & 1u))
                                     : pick_free(*gU, *hU) >= 0;
            const bool vok = rv >= 0 ? !(((*gV >> rv) & 1u) || ((*hV >> (rv % H)) & 1u))
                                     : pick_free(*gV, *hV) >= 0;
            if (uok && vok) {
              chosen = (int32_t)i;
              break;
            }
          }
          if (chosen < 0) continue;  // leave this lane for a dummy
          done[(size_t)chosen] = 1;
          left--;
          const int32_t e = list[(size_t)chosen];
          free_at[cp * nth + tg * G + p] = e;
          int32_t &ru = res[(size_t)s.h_eu[(size_t)e]];
          if (ru < 0) { ru = pick_free(*gU, *hU); load[(size_t)ru]++; }
          *gU |= bit(ru); *hU |= bit(ru % H);
          int32_t &rv = res[(size_t)s.h_ev[(size_t)e]];
          if (rv < 0) { rv = pick_free(*gV, *hV); load[(size_t)rv]++; }
          *gV |= bit(rv); *hV |= bit(rv % H);
        }
      }
    }
    // edges no conflict-free lane took: any empty lane, counted as conflicts
    for (size_t i = 0; i < list.size(); i++) {
      if (done[i]) continue;
      size_t at = (size_t)c * P * nth;
      while (free_at[at] >= 0) at++;  // fits: at most P nth edges
      const int32_t e = list[i];
      free_at[at] = e;
      const size_t cp = at / (size_t)nth;
      const int32_t t = (int32_t)(at % (size_t)nth);
      const int32_t tg = t / G, half = (t % G) / H;
      uint64_t *gU, *gV, *hU, *hV;
      fmask(cp, tg, half, &gU, &gV, &hU, &hV);
      for (int q = 0; q < 2; q++) {
        int32_t &r = res[(size_t)(q == 0 ? s.h_eu[(size_t)e] : s.h_ev[(size_t)e])];
        uint64_t *gm = q == 0 ? gU : gV, *hm = q == 0 ? hU : hV;
        if (r < 0) {
          r = pick_free(*gm, *hm);
          if (r < 0) r = 0;
          load[(size_t)r]++;
        }
        if (((*gm >> r) & 1u) || ((*hm >> (r % H)) & 1u)) conflicts++;
        *gm |= bit(r);
        *hm |= bit(r % H);
      }
    }
  }

  // 4. residues of the remaining LDS vertices, then rows residue-major
  for (int32_t v = 0; v < n; v++) {
    if (inI[(size_t)v] || res[(size_t)v] >= 0) continue;
    int32_t r = 0;
    for (int32_t q = 1; q < G; q++)
      if (load[(size_t)q] < load[(size_t)r]) r = q;
    res[(size_t)v] = r;
    load[(size_t)r]++;
  }
  int64_t per = 0;
  for (int32_t r = 0; r < G; r++) per = std::max(per, load[(size_t)r]);
  const int64_t n_rows = ((int64_t)G * per + 63) / 64 * 64;
  if (n_rows + kDummyRows > 65535 || n_rows > (int64_t)n + kRegRowsSlack - kDummyRows)
    return set_error(COSM_ERANGE, "too many rows for the register form");
  // the streamed form's pair words hold row offsets in 18 bits
  if (o.rstream && (size_t)(n_rows + kDummyRows) * 4 * W > ((size_t)1 << 18))
    return set_error(COSM_ERANGE, "the streamed register form needs rows below 2^18 bytes");
  std::vector<int32_t> row((size_t)n, -1), fill((size_t)G, 0);
  LdsSchedule L;
  L.G = G;
  L.nth = nth;
  L.n_rows = (int32_t)n_rows;
  L.slot_vertex.assign((size_t)n_rows, -1);
  for (int32_t v = 0; v < n; v++) {
    if (inI[(size_t)v]) continue;
    const int32_t r = res[(size_t)v];
    row[(size_t)v] = r + G * fill[(size_t)r]++;
    L.slot_vertex[(size_t)row[(size_t)v]] = v;
  }

  // 5. the entries: register slots [C][K][nth] and pair slots [C][P][nth];
  // lanes without an edge take dummy rows whose residues are free in their
  // group and half, so every access of a slot stays conflict-free
  std::vector<RegEntry> reg((size_t)C * K * nth);
  std::vector<PairEntry> pair((size_t)C * P * nth);
  for (int32_t k = 0; k < K; k++) {
    for (int32_t tg = 0; tg < groups_per_k; tg++) {
      const int32_t gi = k * groups_per_k + tg;
      for (int32_t c = 0; c < C; c++) {
        uint64_t gm = usedG[(size_t)gi * C + c];
        uint64_t hm[2] = {usedH[((size_t)gi * 2) * C + c], usedH[((size_t)gi * 2 + 1) * C + c]};
        for (int32_t p = 0; p < G; p++) {
          const int32_t t = tg * G + p;
          const int32_t v = pos_vertex[(size_t)k * nth + t];
          int32_t e = -1;
          if (v >= 0)
            for (const Adj &a : adj[(size_t)v])
              if (a.cls == c) e = a.edge;
          if (e < 0) continue;
          RegEntry &d = reg[((size_t)c * K + k) * nth + t];
          d.flip = s.h_ev[(size_t)e] == v;
          d.row = row[(size_t)(d.flip ? s.h_eu[(size_t)e] : s.h_ev[(size_t)e])];
          d.J = s.h_J[(size_t)e];
        }
        for (int32_t half = 0; half < 2 && half * H < G; half++) {
          for (int32_t p = half * H; p < (half + 1) * H && p < G; p++) {
            const int32_t t = tg * G + p;
            const int32_t v = pos_vertex[(size_t)k * nth + t];
            bool active = false;
            if (v >= 0)
              for (const Adj &a : adj[(size_t)v])
                if (a.cls == c) active = true;
            if (active) continue;
            int32_t r = -1;
            for (int32_t q = 0; q < G && r < 0; q++)
              if (!((gm >> q) & 1u) && !((hm[half] >> (q % H)) & 1u)) r = q;
            if (r < 0) return set_error(COSM_ERANGE, "no free dummy row");
            gm |= bit(r);
            hm[half] |= bit(r % H);
            RegEntry &d = reg[((size_t)c * K + k) * nth + t];
            d.row = (int32_t)n_rows + r;
            d.flip = false;
            d.J = 0;
          }
        }
      }
    }
  }
  for (size_t cp = 0; cp < nps; cp++) {
    for (int32_t tg = 0; tg < groups_per_k; tg++) {
      uint64_t gU = fG[(cp * groups_per_k + tg) * 2], gV = fG[(cp * groups_per_k + tg) * 2 + 1];
      for (int32_t p = 0; p < G; p++) {
        const int32_t t = tg * G + p, half = p / H;
        uint64_t &hU = fH[((cp * groups_per_k + tg) * 2 + half) * 2];
        uint64_t &hV = fH[((cp * groups_per_k + tg) * 2 + half) * 2 + 1];
        PairEntry &d = pair[cp * nth + t];
        const int32_t e = free_at[cp * nth + t];
        if (e >= 0) {
          d.ru = row[(size_t)s.h_eu[(size_t)e]];
          d.rv = row[(size_t)s.h_ev[(size_t)e]];
          d.J = s.h_J[(size_t)e];
          continue;
        }
        int32_t ru = -1, rv = -1;
        for (int32_t q = 0; q < G && ru < 0; q++)
          if (!((gU >> q) & 1u) && !((hU >> (q % H)) & 1u)) ru = q;
        for (int32_t q = 0; q < G && rv < 0; q++)
          if (!((gV >> q) & 1u) && !((hV >> (q % H)) & 1u)) rv = q;
        if (ru < 0 || rv < 0) {  // a group with conflicts: any dummy row
          ru = ru < 0 ? 0 : ru;
          rv = rv < 0 ? 0 : rv;
        }
        gU |= bit(ru); hU |= bit(ru % H);
        gV |= bit(rv); hV |= bit(rv % H);
        d.ru = (int32_t)n_rows + ru;
        d.rv = (int32_t)n_rows + rv;
        d.J = 0;
      }
    }
  }

  // 6. the encoding
  if (o.rstream) {
    const uint32_t rowb = 4u * (uint32_t)W;
    const int32_t nw = nth / 64;
    int32_t nr = 0;
    for (int32_t c = 0; c < C; c++) nr += rclass[(size_t)c];
    L.rs_words.assign((size_t)nr * K * nth * 2, 0u);
    L.rs_pwords.assign((size_t)C * P * nth * 2, 0u);
    L.rs_act.assign((size_t)C * nw, 0u);
    int32_t j = 0;  // register classes so far
    for (int32_t c = 0; c < C; c++) {
      if (rclass[(size_t)c]) {
        for (int32_t k = 0; k < K; k++)
          for (int32_t t = 0; t < nth; t++) {
            const RegEntry &d = reg[((size_t)c * K + k) * nth + t];
            const size_t i = ((size_t)j * K + k) * nth + t;
            L.rs_words[2 * i] = (uint32_t)d.row * rowb | (d.flip ? 0x80000000u : 0u);
            L.rs_words[2 * i + 1] = __builtin_bit_cast(uint32_t, (float)d.J);
          }
        for (int32_t w = 0; w < nw; w++) L.rs_act[(size_t)c * nw + w] |= 1u;
        j++;
      }
      for (int32_t ps = 0; ps < P; ps++)
        for (int32_t t = 0; t < nth; t++) {
          const size_t i = ((size_t)c * P + ps) * nth + t;
          const PairEntry &d = pair[i];
          // u row offset with J in the top 14 bits (|J| < 2^13), v row offset
          L.rs_pwords[2 * i] = (uint32_t)d.ru * rowb | (uint32_t)d.J << 18;
          L.rs_pwords[2 * i + 1] = (uint32_t)d.rv * rowb;
          if (d.J != 0) L.rs_act[(size_t)c * nw + t / 64] |= 2u << ps;
        }
    }
    L.rstream = true;
    L.fuse = false;
  } else {
    // descriptors: [C][K + 1][nth], a register slot's row with the flip in
    // bit 16, then the pair slot (u | v << 16)
    const int32_t per_class = K + 1;
    L.desc.assign((size_t)C * per_class * nth, EdgeDesc{0u, 0.0f});
    for (int32_t c = 0; c < C; c++) {
      for (int32_t k = 0; k < K; k++)
        for (int32_t t = 0; t < nth; t++) {
          const RegEntry &d = reg[((size_t)c * K + k) * nth + t];
          L.desc[((size_t)c * per_class + k) * nth + t] =
              EdgeDesc{(uint32_t)d.row | (d.flip ? 1u << 16 : 0u), (float)d.J};
        }
      for (int32_t t = 0; t < nth; t++) {
        const PairEntry &d = pair[(size_t)c * nth + t];
        L.desc[((size_t)c * per_class + K) * nth + t] =
            EdgeDesc{(uint32_t)d.ru | ((uint32_t)d.rv << 16), (float)d.J};
      }
    }
    // The twist can run inside the last class when that class touches every
    // vertex row exactly once (each row is then final for the sweep right after
    // its update there), as on the even tori, where every vertex has an edge in
    // every class.
    std::vector<int32_t> hit((size_t)n_rows, 0);
    const int32_t c = C - 1;
    for (int32_t k = 0; k <= K; k++)
      for (int32_t t = 0; t < nth; t++) {
        const EdgeDesc &d = L.desc[((size_t)c * per_class + k) * nth + t];
        if (d.J == 0.0f) continue;  // dummy (or a no-op edge)
        const uint32_t a = d.slots & 0xffffu;
        if (a < (uint32_t)n_rows) hit[a]++;
        if (k == K) {
          const uint32_t b = d.slots >> 16;
          if (b < (uint32_t)n_rows) hit[b]++;
        }
      }
    bool all = true;
    for (int64_t r = 0; r < n_rows && all; r++)
      if (L.slot_vertex[(size_t)r] >= 0 && hit[(size_t)r] != 1) all = false;
    L.fuse = all;
  }
  L.total_slots = C * (K + P);
  L.K.assign((size_t)C, K + P);
  L.padded.assign((size_t)C, (K + P) * nth);
  L.reg_k = K;
  L.reg_free = reg_free;
  L.reg_vertex = pos_vertex;
  L.reg_set = set_size;
  L.reg_edges = reg_edges;
  L.reg_conflicts = conflicts;
  L.fuse_k = 0;
  L.dummy_pairs = true;
  *out = std::move(L);
  return COSM_OK;
}

}  // namespace

int build_reg_schedule(const cosm_state &s, int32_t W, int32_t K, int32_t nth_request,
                       LdsSchedule *out) {
  RegOptions a, b;
  a.W = b.W = W;
  a.K = b.K = K;
  a.nth_request = b.nth_request = nth_request;
  a.pre = true;
  LdsSchedule la, lb;
  const int ra = build_reg_impl(s, a, &la);
  const int rb = build_reg_impl(s, b, &lb);
  if (ra && rb) return ra;
  clear_error();
  // more edges in registers first, then fewer bank conflicts
  const bool take_a = rb || (ra == 0 && (la.reg_edges > lb.reg_edges ||
                                         (la.reg_edges == lb.reg_edges &&
                                          la.reg_conflicts <= lb.reg_conflicts)));
  *out = std::move(take_a ? la : lb);
  return COSM_OK;
}

int build_rstream_schedule(const cosm_state &s, int32_t W, int32_t nth_request,
                           LdsSchedule *out) {
  // the fewest register rows (8, 10, 12 or 16) that hold the independent set
  // at the thread count asked for (1024 when none is)
  const int32_t nth = nth_request > 0 ? nth_request : 1024;
  std::vector<std::vector<Adj>> adj((size_t)s.n);
  for (int64_t k = 0; k < s.m; k++) {
    adj[(size_t)s.h_eu[(size_t)k]].push_back({s.h_ev[(size_t)k], (int32_t)k, 0});
    adj[(size_t)s.h_ev[(size_t)k]].push_back({s.h_eu[(size_t)k], (int32_t)k, 0});
  }
  std::vector<uint8_t> inI;
  if (!bipartite_side(s.n, adj, &inI)) large_independent(s.n, adj, &inI);
  int64_t set = 0;
  for (uint8_t b : inI) set += b;
  int32_t K = kRStreamKMax;
  for (int32_t k : {8, 10, 12, 16})
    if ((int64_t)k * nth >= set) {
      K = k;
      break;
    }
  RegOptions a, b;
  a.W = b.W = W;
  a.K = b.K = K;
  a.nth_request = b.nth_request = nth;
  a.rstream = b.rstream = true;
  a.pre = true;
  LdsSchedule la, lb;
  const int ra = build_reg_impl(s, a, &la);
  const int rb = build_reg_impl(s, b, &lb);
  if (ra && rb) return ra;
  clear_error();
  const bool take_a = rb || (ra == 0 && (la.reg_edges > lb.reg_edges ||
                                         (la.reg_edges == lb.reg_edges &&
                                          la.reg_conflicts <= lb.reg_conflicts)));
  *out = std::move(take_a ? la : lb);
  return COSM_OK;
}

size_t rstream_lds_bytes(const LdsSchedule &L, int W, int32_t C) {
  // rows and dummy rows, the twist angles of kThetaChunk twists (FP32: W
  // replicas per row), the slot masks
  return (size_t)(L.n_rows + kDummyRows) * W * 4 + (size_t)kThetaChunk * W * 4 +
         (size_t)C * (L.nth / 64) * 4;
}

}  // namespace cosm
