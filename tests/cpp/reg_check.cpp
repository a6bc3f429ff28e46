// Host-only check of the register-owner schedule built by reg_schedule.cpp.
// Input on stdin: "n m C" then m lines "u v J colour"; arguments: W K (K = 0:
// the streamed register-owner schedule, which picks its own K).
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
#include <cstring>
#include <set>
#include <tuple>
#include <vector>
int cosm::set_error(int st, const std::string &m) { fprintf(stderr, "err %s\n", m.c_str()); return st; }
void cosm::clear_error() {}
int main(int argc, char **argv) {
  if (argc < 3) return 1;
  const int W = atoi(argv[1]);
  int K = atoi(argv[2]);
  int n; long m; int C;
  if (scanf("%d %ld %d", &n, &m, &C) != 3) return 1;
  cosm_state s; s.n = n; s.m = m; s.C = C;
  for (long k = 0; k < m; k++) {
    int u, v, J, c;
    if (scanf("%d %d %d %d", &u, &v, &J, &c) != 4) return 1;
    s.h_eu.push_back(u); s.h_ev.push_back(v); s.h_J.push_back(J); s.h_colour.push_back(c);
  }
  cosm::LdsSchedule L;
  // K = 0: the streamed register-owner schedule (it picks its own K)
  const bool rstream = K == 0;
  if (rstream ? cosm::build_rstream_schedule(s, W, 0, &L) : cosm::build_reg_schedule(s, W, K, 0, &L)) {
    puts("ERANGE");
    return 2;
  }
  if (rstream) K = L.reg_k;
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
  long mask_bad = 0;
  int rclasses = 0;
  if (rstream) {
    // register classes (bit 0 of every wave's mask), their K slots of word
    // pairs (row offset | flip << 31, J as a float), then kRStreamPairs pair
    // slots per class (u offset | J << 18, v offset) with per-wave mask bits
    const int nw = nth / 64, P = cosm::kRStreamPairs;
    const uint32_t rowb = 4u * W;
    if ((int)L.rs_act.size() != C * nw || (int)L.rs_pwords.size() != C * P * nth * 2) bad_dummy++;
    std::vector<int> rc(C, 0);
    for (int c = 0; c < C && !bad_dummy; c++) {
      rc[c] = L.rs_act[(size_t)c * nw] & 1u;
      for (int w = 1; w < nw; w++) if ((int)(L.rs_act[(size_t)c * nw + w] & 1u) != rc[c]) mask_bad++;
      rclasses += rc[c];
    }
    if ((long)L.rs_words.size() != (long)rclasses * K * nth * 2) bad_dummy++;
    int j = 0;
    for (int c = 0; c < C && !bad_dummy; c++) {
      if (rc[c]) {
        for (int k = 0; k < K; k++) {
          std::vector<int> rows(nth);
          for (int t = 0; t < nth; t++) {
            const size_t i = ((size_t)j * K + k) * nth + t;
            const uint32_t x = L.rs_words[2 * i], y = L.rs_words[2 * i + 1];
            float J;
            memcpy(&J, &y, 4);
            const uint32_t off = x & 0x7fffffffu;
            const int flip = (int)(x >> 31), row = (int)(off / rowb);
            rows[t] = row;
            if (off % rowb) bad_dummy++;
            if (J == 0.0f) {
              if (row < nr || row >= nr + cosm::kDummyRows || flip) bad_dummy++;
              continue;
            }
            if (row >= nr) { bad_dummy++; continue; }
            const int v = L.reg_vertex[(size_t)k * nth + t], w = L.slot_vertex[row];
            if (v < 0 || w < 0) { bad_dummy++; continue; }
            reg_active++;
            got.insert({c, flip ? w : v, flip ? v : w, J});
          }
          banks(rows);
        }
        j++;
      }
      for (int p = 0; p < P; p++) {
        std::vector<int> ru(nth), rv(nth);
        for (int t = 0; t < nth; t++) {
          const size_t i = ((size_t)c * P + p) * nth + t;
          const uint32_t x = L.rs_pwords[2 * i], y = L.rs_pwords[2 * i + 1];
          const uint32_t ou = x & ((1u << 18) - 1u);
          const int J = (int32_t)x >> 18;
          ru[t] = (int)(ou / rowb);
          rv[t] = (int)(y / rowb);
          if (ou % rowb || y % rowb) bad_dummy++;
          if (J == 0) {
            if (ru[t] < nr || rv[t] < nr || ru[t] >= nr + cosm::kDummyRows ||
                rv[t] >= nr + cosm::kDummyRows) bad_dummy++;
            continue;
          }
          if (!((L.rs_act[(size_t)c * nw + t / 64] >> (1 + p)) & 1u)) mask_bad++;
          if (ru[t] >= nr || rv[t] >= nr) { bad_dummy++; continue; }
          const int u = L.slot_vertex[ru[t]], v = L.slot_vertex[rv[t]];
          if (u < 0 || v < 0) { bad_dummy++; continue; }
          free_active++;
          got.insert({c, u, v, (float)J});
        }
        banks(ru);
        banks(rv);
      }
    }
  }
  if (!rstream && (int)L.desc.size() != C * (K + 1) * nth) bad_dummy++;
  for (int c = 0; c < C && !bad_dummy && !rstream; c++) {
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
         "conflicts=%ld equal=%d indep=%d rows_ok=%d bad_dummy=%ld fuse=%d fuse_ok=%d "
         "rstream=%d rclasses=%d mask_bad=%ld\n",
         W, K, nth, nr, (long)L.reg_edges, reg_active, free_active, L.reg_free, conflicts,
         (int)(want == got), indep, rows_ok, bad_dummy, (int)L.fuse, fuse_ok, (int)rstream,
         rclasses, mask_bad);
  return 0;
}
