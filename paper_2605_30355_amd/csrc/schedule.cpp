// schedule.cpp -- LDS layout and lane schedule of the LDS-resident sweep.
//
// The sweep kernel keeps a replica block as LDS rows (one row per slot) and
// lets consecutive lanes take consecutive entries of a class's edge list.  The
// gfx950 LDS has 64 banks of 4 bytes.  Measured on the part: a wave's reads
// are served in groups of 256 bytes of lanes (16 lanes of ds_read_b128, 32 of
// _b64, 32 of _b32) and its writes in groups of 128 bytes (8 lanes of
// ds_write_b128, 16 of _b64, 32 of _b32); an access runs at full speed when
// the rows of every group lie in distinct banks.  With rows of 4 W bytes that
// means distinct residues slot mod G within each aligned group of G = 64 / W
// lanes (32 for W = 1), and distinct residues mod H = 32 / W within each
// aligned half of H lanes.  Within a colour class the edges are a matching, so
// their order is free; this file picks
//   1. a vertex -> slot map that spreads every class's u-endpoints, and its
//      v-endpoints, evenly over the G residues;
//   2. per class, an order made of aligned groups of G entries in which the
//      u-residues are distinct and the v-residues are distinct: a proper edge
//      colouring of the bipartite multigraph (u-residue, v-residue), which
//      König's theorem gives with as many colours as its maximum degree;
//      unused lanes of a group are masked off;
//   3. within each group, the split into two halves of H lanes: two entries
//      whose u-residues (or v-residues) agree mod H must go to different
//      halves.  Each entry has at most one such partner of each kind, so the
//      constraints form paths and even cycles and a 2-colouring exists.
// None of this changes the dynamics: each class is still applied in full, in
// the class order given by the caller.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>

#include "internal.hpp"

namespace cosm {

namespace {

// Edge colouring of a bipartite multigraph with Delta colours (alternating-path
// recolouring).  left/right in [0, G); returns colour per edge and the count.
int32_t bipartite_edge_colouring(int32_t G, const std::vector<int32_t> &left,
                                 const std::vector<int32_t> &right, std::vector<int32_t> *col) {
  const size_t E = left.size();
  std::vector<int32_t> degL((size_t)G, 0), degR((size_t)G, 0);
  for (size_t e = 0; e < E; e++) {
    degL[(size_t)left[e]]++;
    degR[(size_t)right[e]]++;
  }
  int32_t D = 0;
  for (int32_t g = 0; g < G; g++) D = std::max({D, degL[(size_t)g], degR[(size_t)g]});
  // atL[a*D + c] = edge coloured c at left node a (or -1); same for atR
  std::vector<int32_t> atL((size_t)G * D, -1), atR((size_t)G * D, -1);
  col->assign(E, -1);
  auto freeL = [&](int32_t a) {
    for (int32_t c = 0; c < D; c++)
      if (atL[(size_t)a * D + c] < 0) return c;
    return -1;
  };
  auto freeR = [&](int32_t b) {
    for (int32_t c = 0; c < D; c++)
      if (atR[(size_t)b * D + c] < 0) return c;
    return -1;
  };
  std::vector<int32_t> path;
  for (size_t e = 0; e < E; e++) {
    const int32_t a = left[e], b = right[e];
    const int32_t al = freeL(a), be = freeR(b);
    if (atR[(size_t)b * D + al] >= 0) {
      // swap al <-> be along the path from b that starts with b's al-edge
      path.clear();
      int32_t node = b, c = al;
      bool on_right = true;
      while (true) {
        const int32_t f = on_right ? atR[(size_t)node * D + c] : atL[(size_t)node * D + c];
        if (f < 0) break;
        path.push_back(f);
        node = on_right ? left[(size_t)f] : right[(size_t)f];
        on_right = !on_right;
        c = (c == al) ? be : al;
      }
      for (int32_t f : path) {
        atL[(size_t)left[(size_t)f] * D + (*col)[(size_t)f]] = -1;
        atR[(size_t)right[(size_t)f] * D + (*col)[(size_t)f]] = -1;
      }
      for (int32_t f : path) {
        const int32_t nc = (*col)[(size_t)f] == al ? be : al;
        (*col)[(size_t)f] = nc;
        atL[(size_t)left[(size_t)f] * D + nc] = f;
        atR[(size_t)right[(size_t)f] * D + nc] = f;
      }
    }
    (*col)[e] = al;
    atL[(size_t)a * D + al] = (int32_t)e;
    atR[(size_t)b * D + al] = (int32_t)e;
  }
  return D;
}

}  // namespace

int build_lds_schedule(const cosm_state &s, int32_t W, int32_t nth_request, LdsSchedule *out,
                       bool dummy_pairs, bool allow_stream) {
  const int32_t n = s.n, C = s.C, G = W == 1 ? 32 : 64 / W, H = 32 / W;
  const int64_t m = s.m;
  *out = LdsSchedule();  // nothing of an earlier schedule (e.g. register rows) survives
  LdsSchedule &L = *out;
  L.G = G;
  L.n_rows = n;
  if (n > 65536) return set_error(COSM_ERANGE, "too many LDS rows");

  // 1. residue of every vertex: greedy balancing of the per-class, per-side
  // residue counts; residue g owns the slots g, g + G, ... below n.
  // inc[i] lists (class, side) pairs of vertex i.
  std::vector<std::vector<int32_t>> inc((size_t)n);
  for (int64_t k = 0; k < m; k++) {
    inc[(size_t)s.h_eu[(size_t)k]].push_back(2 * s.h_colour[(size_t)k]);
    inc[(size_t)s.h_ev[(size_t)k]].push_back(2 * s.h_colour[(size_t)k] + 1);
  }
  std::vector<int32_t> cnt((size_t)2 * C * G, 0), cap((size_t)G, 0), res((size_t)n, 0);
  for (int32_t g = 0; g < G; g++) cap[(size_t)g] = (n - g + G - 1) / G;
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937 rng(12345u);
  std::shuffle(order.begin(), order.end(), rng);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return inc[(size_t)a].size() > inc[(size_t)b].size();
  });
  for (int32_t i : order) {
    int32_t best = -1;
    int64_t best_cost = 0;
    for (int32_t g = 0; g < G; g++) {
      if (cap[(size_t)g] == 0) continue;
      int64_t cost = 0;  // sum of squares of the counts this choice raises
      for (int32_t cs : inc[(size_t)i]) {
        const int64_t v = cnt[(size_t)cs * G + g];
        cost += 2 * v + 1;
      }
      if (best < 0 || cost < best_cost) {
        best = g;
        best_cost = cost;
      }
    }
    res[(size_t)i] = best;
    cap[(size_t)best]--;
    for (int32_t cs : inc[(size_t)i]) cnt[(size_t)cs * G + best]++;
  }
  // 1b. local search: exchange the residues of two vertices when that lowers
  // sum(cnt^2) + 64 sum(max(0, cnt - T)^2), T = ceil(class-side total / G), the
  // least maximum a class-side can have.  Stops once no count exceeds its T.
  {
    std::vector<int32_t> T((size_t)2 * C, 0);
    for (int32_t cs = 0; cs < 2 * C; cs++) {
      int64_t tot = 0;
      for (int32_t g = 0; g < G; g++) tot += cnt[(size_t)cs * G + g];
      T[(size_t)cs] = (int32_t)((tot + G - 1) / G);
    }
    auto cell = [&](int32_t cs, int32_t c) {
      const int64_t e = std::max(0, c - T[(size_t)cs]);
      return (int64_t)c * c + 64 * e * e;
    };
    int64_t excess = 0;
    for (int32_t cs = 0; cs < 2 * C; cs++)
      for (int32_t g = 0; g < G; g++) excess += std::max(0, cnt[(size_t)cs * G + g] - T[(size_t)cs]);
    // move vertex i from residue a to b; returns the change of the objective
    auto move = [&](int32_t i, int32_t a, int32_t b) {
      int64_t d = 0;
      for (int32_t cs : inc[(size_t)i]) {
        int32_t &ca = cnt[(size_t)cs * G + a], &cb = cnt[(size_t)cs * G + b];
        d += cell(cs, ca - 1) - cell(cs, ca) + cell(cs, cb + 1) - cell(cs, cb);
        excess += std::max(0, ca - 1 - T[(size_t)cs]) - std::max(0, ca - T[(size_t)cs]);
        excess += std::max(0, cb + 1 - T[(size_t)cs]) - std::max(0, cb - T[(size_t)cs]);
        ca--;
        cb++;
      }
      return d;
    };
    std::uniform_int_distribution<int32_t> pick(0, n - 1);
    const int64_t tries = 60 * (int64_t)n;
    for (int64_t it = 0; it < tries && excess > 0; it++) {
      const int32_t x = pick(rng), y = pick(rng);
      const int32_t gx = res[(size_t)x], gy = res[(size_t)y];
      if (gx == gy) continue;
      const int64_t d = move(x, gx, gy) + move(y, gy, gx);
      if (d < 0) {
        res[(size_t)x] = gy;
        res[(size_t)y] = gx;
      } else {
        move(y, gx, gy);
        move(x, gy, gx);
      }
    }
  }
  // slots: residue g holds slots g, g + G, g + 2G, ... in vertex order
  L.slot_vertex.assign((size_t)L.n_rows, -1);
  std::vector<int32_t> slot((size_t)n), next_in_res((size_t)G, 0);
  for (int32_t i = 0; i < n; i++) {
    const int32_t g = res[(size_t)i];
    slot[(size_t)i] = g + G * next_in_res[(size_t)g]++;
    L.slot_vertex[(size_t)slot[(size_t)i]] = i;
  }

  // 2. per class: bipartite colouring of (u residue, v residue) -> groups of G
  std::vector<std::vector<int64_t>> by_class((size_t)C);
  for (int64_t k = 0; k < m; k++) by_class[(size_t)s.h_colour[(size_t)k]].push_back(k);
  L.K.assign((size_t)C, 0);
  L.padded.assign((size_t)C, 0);
  std::vector<std::vector<EdgeDesc>> lists((size_t)C);
  for (int32_t c = 0; c < C; c++) {
    const auto &E = by_class[(size_t)c];
    if (E.empty()) continue;
    std::vector<int32_t> lft(E.size()), rgt(E.size()), col;
    for (size_t a = 0; a < E.size(); a++) {
      lft[a] = slot[(size_t)s.h_eu[(size_t)E[a]]] % G;
      rgt[a] = slot[(size_t)s.h_ev[(size_t)E[a]]] % G;
    }
    const int32_t D = bipartite_edge_colouring(G, lft, rgt, &col);
    auto &lst = lists[(size_t)c];
    lst.assign((size_t)D * G, EdgeDesc{kEmptySlot, 0.0f});  // unfilled lanes stay masked
    std::vector<std::vector<int32_t>> group((size_t)D);
    for (size_t a = 0; a < E.size(); a++) group[(size_t)col[a]].push_back((int32_t)a);
    std::vector<int32_t> half(E.size(), -1), uo((size_t)H), vo((size_t)H), stack;
    for (int32_t g = 0; g < D; g++) {
      const auto &grp = group[(size_t)g];
      int32_t fill[2] = {0, 0};
      if (H < G) {
        // partner of each entry through a shared u- or v-residue mod H
        std::fill(uo.begin(), uo.end(), -1);
        std::fill(vo.begin(), vo.end(), -1);
        std::vector<int32_t> pu(grp.size(), -1), pv(grp.size(), -1);
        for (size_t q = 0; q < grp.size(); q++) {
          const int32_t ru = lft[(size_t)grp[q]] % H, rv = rgt[(size_t)grp[q]] % H;
          if (uo[(size_t)ru] >= 0) {
            pu[q] = uo[(size_t)ru];
            pu[(size_t)uo[(size_t)ru]] = (int32_t)q;
          }
          uo[(size_t)ru] = (int32_t)q;
          if (vo[(size_t)rv] >= 0) {
            pv[q] = vo[(size_t)rv];
            pv[(size_t)vo[(size_t)rv]] = (int32_t)q;
          }
          vo[(size_t)rv] = (int32_t)q;
        }
        for (size_t q0 = 0; q0 < grp.size(); q0++) {
          if (half[(size_t)grp[q0]] >= 0) continue;
          half[(size_t)grp[q0]] = 0;
          stack.assign(1, (int32_t)q0);
          while (!stack.empty()) {
            const int32_t q = stack.back();
            stack.pop_back();
            for (int32_t r : {pu[(size_t)q], pv[(size_t)q]}) {
              if (r < 0 || half[(size_t)grp[(size_t)r]] >= 0) continue;
              half[(size_t)grp[(size_t)r]] = 1 - half[(size_t)grp[(size_t)q]];
              stack.push_back(r);
            }
          }
        }
      }
      for (int32_t a : grp) {
        const int32_t hf = H < G ? half[(size_t)a] : 0;
        const int64_t k = E[(size_t)a];
        const uint32_t su = (uint32_t)slot[(size_t)s.h_eu[(size_t)k]];
        const uint32_t sv = (uint32_t)slot[(size_t)s.h_ev[(size_t)k]];
        lst[(size_t)g * G + (size_t)hf * H + fill[hf]++] =
            EdgeDesc{su | (sv << 16), (float)s.h_J[(size_t)k]};
      }
    }
    L.padded[(size_t)c] = (int32_t)lst.size();
  }
  // threads: enough for the largest class in one pass, a multiple of 64, <= 1024
  int32_t maxp = 0;
  for (int32_t c = 0; c < C; c++) maxp = std::max(maxp, L.padded[(size_t)c]);
  int32_t nth = nth_request;
  if (nth <= 0) nth = std::min(1024, std::max(64, (maxp + 63) / 64 * 64));
  L.nth = nth;
  for (int32_t c = 0; c < C; c++) L.K[(size_t)c] = (L.padded[(size_t)c] + nth - 1) / nth;
  // 3. flatten: entry (j, tid) of the per-thread slot list, j running over
  // classes in order and K[c] slots per class.
  L.total_slots = 0;
  for (int32_t c = 0; c < C; c++) L.total_slots += L.K[(size_t)c];
  L.desc.assign((size_t)L.total_slots * nth, EdgeDesc{kEmptySlot, 0.0f});
  int32_t j = 0;
  for (int32_t c = 0; c < C; c++) {
    const auto &lst = lists[(size_t)c];
    for (int32_t k = 0; k < L.K[(size_t)c]; k++, j++)
      for (int32_t t = 0; t < nth; t++) {
        const size_t pos = (size_t)k * nth + t;
        if (pos < lst.size()) L.desc[(size_t)j * nth + t] = lst[pos];
      }
  }
  int64_t pad = 0;
  for (int32_t c = 0; c < C; c++) pad += L.padded[(size_t)c] - (int64_t)by_class[(size_t)c].size();
  L.pad_entries = pad;
  // 3b. register-resident schedules: a masked lane gets a no-op edge (J = 0)
  // between two dummy rows (after the n vertex rows) whose residues no other
  // lane of its group uses, so that it costs no bank conflict.  u-dummies are
  // dummy rows [0, 32), v-dummies [32, 64).
  // The streamed word form replaces the streamed schedule when the sweep has
  // no field pass (it needs the dummy pairs too).
  L.stream = dummy_pairs && allow_stream && L.total_slots > kRegisterSlotsMax && !s.has_h &&
             n + kDummyRows <= 65536;
  L.dummy_pairs = dummy_pairs && (L.total_slots <= kRegisterSlotsMax || L.stream) &&
                  n + kDummyRows <= 65536;
  if (L.dummy_pairs) {
    std::vector<char> used_u((size_t)G), used_v((size_t)G);
    for (int32_t jj = 0; jj < L.total_slots; jj++)
      for (int32_t g0 = 0; g0 < nth; g0 += G) {
        std::fill(used_u.begin(), used_u.end(), 0);
        std::fill(used_v.begin(), used_v.end(), 0);
        const size_t row = (size_t)jj * nth;
        const int32_t g1 = std::min(nth, g0 + G);
        for (int32_t t = g0; t < g1; t++) {
          const EdgeDesc &d = L.desc[row + t];
          if (d.slots == kEmptySlot) continue;
          used_u[(size_t)((d.slots & 0xffffu) % (uint32_t)G)] = 1;
          used_v[(size_t)((d.slots >> 16) % (uint32_t)G)] = 1;
        }
        int32_t ru = 0, rv = 0;
        for (int32_t t = g0; t < g1; t++) {
          EdgeDesc &d = L.desc[row + t];
          if (d.slots != kEmptySlot) continue;
          while (ru < G && used_u[(size_t)ru]) ru++;
          while (rv < G && used_v[(size_t)rv]) rv++;
          // a group has as many free residues as masked lanes
          const int32_t q = n % G;
          const uint32_t du = (uint32_t)(n + (ru - q + G) % G);
          const uint32_t dv = (uint32_t)(n + 32 + (rv - q + G) % G);
          d = EdgeDesc{du | (dv << 16), 0.0f};
          ru++;
          rv++;
        }
      }
  }
  // 4. kStreamRepeat slots after the last repeat slots 0, 1, ... (mod
  // total), so that a schedule streamed one or two slots ahead never wraps.
  if (L.total_slots > 0) {
    L.desc.resize((size_t)(L.total_slots + kStreamRepeat) * nth);
    for (int32_t q = 0; q < kStreamRepeat; q++)
      for (int32_t t = 0; t < nth; t++)
        L.desc[(size_t)(L.total_slots + q) * nth + t] =
            L.desc[(size_t)(q % L.total_slots) * nth + t];
  } else {
    L.desc.assign((size_t)kStreamRepeat * nth, EdgeDesc{kEmptySlot, 0.0f});
  }
  // 5. rows outside the last class, in slot order (consecutive lanes read
  // consecutive rows), kFuseRowsMax per thread at most.
  L.fuse = false;
  L.fuse_k = 0;
  if (C > 0) {
    std::vector<char> touched((size_t)n, 0);
    for (const EdgeDesc &d : lists[(size_t)C - 1]) {
      if (d.slots == kEmptySlot) continue;
      touched[(size_t)(d.slots & 0xffffu)] = 1;
      touched[(size_t)(d.slots >> 16)] = 1;
    }
    std::vector<int32_t> rest;
    for (int32_t r = 0; r < n; r++)
      if (!touched[(size_t)r]) rest.push_back(r);
    const int32_t fk = (int32_t)(((int64_t)rest.size() + nth - 1) / nth);
    if (fk <= kFuseRowsMax) {
      L.fuse = true;
      L.fuse_k = fk;
      const size_t base = (size_t)(L.total_slots + kStreamRepeat) * nth;
      L.desc.resize(base + (size_t)fk * nth, EdgeDesc{kEmptySlot, 0.0f});
      // deal the rows by bank residue (row mod G): consecutive lanes take
      // rows of distinct residues while every residue has rows left
      std::vector<std::vector<int32_t>> bucket((size_t)G);
      for (int32_t r : rest) bucket[(size_t)(r % G)].push_back(r);
      std::vector<size_t> next((size_t)G, 0);
      for (size_t q = 0; q < rest.size(); q++) {
        size_t g = q % (size_t)G;
        if (next[g] == bucket[g].size()) {  // residue exhausted: the fullest one
          size_t best = 0, left = 0;
          for (size_t h = 0; h < (size_t)G; h++)
            if (bucket[h].size() - next[h] > left) {
              left = bucket[h].size() - next[h];
              best = h;
            }
          g = best;
        }
        L.desc[base + q] = EdgeDesc{(uint32_t)bucket[g][next[g]++], 0.0f};
      }
    }
  }
  // 6. the streamed word form: byte offsets, the sign of J, |J| when it
  // varies; every class padded to an even number of slots (an added slot holds
  // dummy pairs and is never run), so that a class always starts on an even
  // slot.
  if (L.stream) {
    const uint32_t rowb = (uint32_t)(4 * W);
    float mag = -1.0f;
    L.junit = true;
    for (int64_t k = 0; k < m; k++) {
      const float a = std::fabs((float)s.h_J[(size_t)k]);
      if (mag < 0.0f) mag = a;
      if (a != mag || a == 0.0f) L.junit = false;
    }
    L.jscale = L.junit && mag > 0.0f ? mag : 1.0f;
    auto word = [&](const EdgeDesc &d, uint32_t *w, float *jm) {
      const uint32_t su = d.slots & 0xffffu, sv = d.slots >> 16;
      w[0] = su * rowb | (std::signbit(d.J) ? 0x80000000u : 0u);
      w[1] = sv * rowb;
      *jm = std::fabs(d.J);
    };
    // an added slot: lane t pairs the dummy rows of residue t mod G (distinct
    // in every lane group, so conflict-free), J = 0
    const int32_t q0 = n % L.G;
    L.last_lanes.assign((size_t)C, 0);
    std::vector<uint32_t> words;
    std::vector<float> mags;
    int32_t j0 = 0;
    for (int32_t c = 0; c < C; c++) {
      const int32_t K = L.K[(size_t)c];
      const int32_t Kp = (K + kWordGroup - 1) / kWordGroup * kWordGroup;
      // lanes holding entries in the last slot; with an even slot count every
      // wave runs the final pair, so all of them count
      const int32_t last = K > 0 ? std::min(nth, L.padded[(size_t)c] - (K - 1) * nth) : 0;
      L.last_lanes[(size_t)c] = K % 2 == 0 ? nth : last;
      for (int32_t k = 0; k < Kp; k++)
        for (int32_t t = 0; t < nth; t++) {
          uint32_t w[2];
          float jm;
          if (k < K) {
            word(L.desc[(size_t)(j0 + k) * nth + t], w, &jm);
          } else {
            const uint32_t r = (uint32_t)((t % L.G - q0 + L.G) % L.G);
            word(EdgeDesc{((uint32_t)n + r) | (((uint32_t)n + 32u + r) << 16), 0.0f}, w, &jm);
          }
          words.push_back(w[0]);
          words.push_back(w[1]);
          mags.push_back(jm);
        }
      j0 += K;
    }
    L.stotal = (int32_t)(mags.size() / (size_t)nth);
    // the first slots again after the last, then the rows outside the last class
    for (int32_t q = 0; q < kWordRepeat; q++)
      for (int32_t t = 0; t < nth; t++) {
        const size_t e = (size_t)(q % std::max(1, L.stotal)) * nth + t;
        words.push_back(words[2 * e]);
        words.push_back(words[2 * e + 1]);
        mags.push_back(mags[e]);
      }
    const size_t rows_at = (size_t)(L.total_slots + kStreamRepeat) * nth;
    for (size_t e = rows_at; e < L.desc.size(); e++) {
      const EdgeDesc &d = L.desc[e];
      words.push_back(d.slots == kEmptySlot ? kEmptySlot : d.slots * rowb);
      words.push_back(0u);
    }
    L.sdesc = std::move(words);
    if (L.junit) L.sjmag.clear();
    else L.sjmag = std::move(mags);
  }
  return COSM_OK;
}

}  // namespace cosm
