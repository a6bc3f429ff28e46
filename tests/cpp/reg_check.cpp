// Host-only check of the register-owner schedule built by reg_schedule.cpp.
// Input on stdin: "n m C" then m lines "u v J colour"; arguments: W K.
// Prints one summary line; exit status 0 when the schedule was built (1-2:
// bad input or the form does not apply, printed as "ERANGE").  The caller
// checks equal=1 (every edge exactly once, in its class, with its own u / v
// roles), indep=1 (no edge joins two register vertices, each register vertex
// once), rows_ok=1 (every other vertex in exactly one LDS row), bad_dummy=0
// (lanes without an edge use dummy rows with J = 0) and the bank conflicts,
// counted on the gfx950 LDS model written out in sched_check.cpp: 64 banks of
// 4 bytes, reads served in groups of 256 bytes of lanes (32 lanes for 4-byte
// rows), writes in groups of 128 bytes of lanes.
#include "internal.hpp"
#include <cstdio>
#include <cstdlib>
#include <set>
#include <tuple>
#include <vector>
int cosm::set_error(int st, const std::string &m) { fprintf(stderr, "err %s\n", m.c_str()); return st; }
void cosm::clear_error() {}
int main(int argc, char **argv) {
  if (argc < 3) return 1;
  const int W = atoi(argv[1]), K = atoi(argv[2]);
  int n; long m; int C;
  if (scanf("%d %ld %d", &n, &m, &C) != 3) return 1;
  cosm_state s; s.n = n; s.m = m; s.C = C;
  for (long k = 0; k < m; k++) {
    int u, v, J, c;
    if (scanf("%d %d %d %d", &u, &v, &J, &c) != 4) return 1;
    s.h_eu.push_back(u); s.h_ev.push_back(v); s.h_J.push_back(J); s.h_colour.push_back(c);
  }
  cosm::LdsSchedule L;
  if (cosm::build_reg_schedule(s, W, K, 0, &L)) { puts("ERANGE"); return 2; }
  const int nth = L.nth, nr = L.n_rows;
  // register vertices: each once, independent
  std::vector<int> isreg(n, 0);
  int indep = 1;
  if ((int)L.reg_vertex.size() != K * nth) indep = 0;
  for (int v : L.reg_vertex) {
    if (v < -1 || v >= n) { indep = 0; continue; }
    if (v >= 0 && isreg[v]++) indep = 0;
  }
  for (long k = 0; k < m; k++)
    if (isreg[s.h_eu[k]] && isreg[s.h_ev[k]]) indep = 0;
  // rows: every other vertex exactly once
  int rows_ok = nr % 64 == 0 && (int)L.slot_vertex.size() == nr;
  std::vector<int> seen(n, 0);
  for (int r = 0; r < nr && rows_ok; r++) {
    const int v = L.slot_vertex[r];
    if (v < -1 || v >= n || (v >= 0 && isreg[v])) rows_ok = 0;
    else if (v >= 0) seen[v]++;
  }
  for (int v = 0; v < n && rows_ok; v++) if (!isreg[v] && seen[v] != 1) rows_ok = 0;
  // edges per class
  std::multiset<std::tuple<int, int, int, float>> want, got;
  for (long k = 0; k < m; k++) want.insert({s.h_colour[k], s.h_eu[k], s.h_ev[k], (float)s.h_J[k]});
  const int rlanes = W == 1 ? 32 : 256 / (4 * W), wlanes = 128 / (4 * W);
  long conflicts = 0, bad_dummy = 0, reg_active = 0, free_active = 0;
  auto banks = [&](const std::vector<int> &rows) {  // rows per lane of one access
    for (int lanes : {rlanes, wlanes})
      for (int g0 = 0; g0 < nth; g0 += lanes) {
        int b[64] = {0};
        for (int t = g0; t < g0 + lanes; t++)
          for (int w = 0; w < W; w++) b[(rows[t] * W + w) % 64]++;
        for (int q = 0; q < 64; q++) conflicts += b[q] > 1 ? b[q] - 1 : 0;
      }
  };
  if ((int)L.desc.size() != C * (K + 1) * nth) bad_dummy++;
  for (int c = 0; c < C && !bad_dummy; c++) {
    for (int k = 0; k < K; k++) {
      std::vector<int> rows(nth);
      for (int t = 0; t < nth; t++) {
        const auto d = L.desc[((size_t)c * (K + 1) + k) * nth + t];
        const int row = d.slots & 0xffff, flip = (d.slots >> 16) & 1;
        rows[t] = row;
        if ((d.slots >> 17) != 0) bad_dummy++;
        if (row >= nr) {
          if (row >= nr + cosm::kDummyRows || d.J != 0.0f || flip) bad_dummy++;
          continue;
        }
        const int v = L.reg_vertex[(size_t)k * nth + t], w = L.slot_vertex[row];
        if (v < 0 || w < 0) { bad_dummy++; continue; }
        reg_active++;
        got.insert({c, flip ? w : v, flip ? v : w, d.J});
      }
      banks(rows);
    }
    std::vector<int> ru(nth), rv(nth);
    for (int t = 0; t < nth; t++) {
      const auto d = L.desc[((size_t)c * (K + 1) + K) * nth + t];
      const int a = d.slots & 0xffff, b = d.slots >> 16;
      ru[t] = a; rv[t] = b;
      if (a >= nr || b >= nr) {
        if (a < nr || b < nr || a >= nr + cosm::kDummyRows || b >= nr + cosm::kDummyRows ||
            d.J != 0.0f) bad_dummy++;
        continue;
      }
      const int u = L.slot_vertex[a], v = L.slot_vertex[b];
      if (u < 0 || v < 0 || !L.reg_free) { bad_dummy++; continue; }
      free_active++;
      got.insert({c, u, v, d.J});
    }
    if (L.reg_free) { banks(ru); banks(rv); }
  }
  // a fused twist needs every vertex row touched exactly once in the last class
  int fuse_ok = 1;
  if (L.fuse) {
    std::vector<int> hit(nr, 0);
    for (int k = 0; k <= K; k++)
      for (int t = 0; t < nth; t++) {
        const auto d = L.desc[((size_t)(C - 1) * (K + 1) + k) * nth + t];
        const int a = d.slots & 0xffff, b = d.slots >> 16;
        if (a < nr && d.J != 0.0f) hit[a]++;
        if (k == K && b < nr && d.J != 0.0f) hit[b]++;
      }
    for (int r = 0; r < nr; r++)
      if (L.slot_vertex[r] >= 0 && hit[r] != 1) fuse_ok = 0;
  }
  printf("W=%d K=%d nth=%d rows=%d reg_edges=%ld reg_active=%ld free=%ld reg_free=%d "
         "conflicts=%ld equal=%d indep=%d rows_ok=%d bad_dummy=%ld fuse=%d fuse_ok=%d\n",
         W, K, nth, nr, (long)L.reg_edges, reg_active, free_active, L.reg_free, conflicts,
         (int)(want == got), indep, rows_ok, bad_dummy, (int)L.fuse, fuse_ok);
  return 0;
}
