// Host-only check of the LDS lane schedule built by schedule.cpp.
// Input on stdin: "n m C" then m lines "u v J colour".  Prints a summary line;
// exit status 0 only if the slot map is a permutation.  The caller checks
// "conflicts=0" and "equal=1" (every edge exactly once).  Conflicts are counted
// on a model of the gfx950 LDS written out here, not on the schedule's own
// group size: 64 banks of 4 bytes; a read of 4 W bytes per lane is served in
// groups of 256 bytes of lanes (W >= 2) or 32 lanes (W = 1), a write in groups
// of 128 bytes of lanes, and every bank touched twice within a group is one
// conflict (u-rows and v-rows separately, reads and writes separately).
#include "internal.hpp"
#include <cstdio>
#include <set>
#include <fstream>
#include <vector>
int cosm::set_error(int st, const std::string& m){ fprintf(stderr,"err %s\n",m.c_str()); return st; }
void cosm::clear_error(){}
int main(int argc, char** argv) {
  // reads n m C then m lines u v J colour from stdin
  int n; long m; int C; int W = atoi(argv[1]);
  if (scanf("%d %ld %d", &n, &m, &C) != 3) return 1;
  cosm_state s; s.n = n; s.m = m; s.C = C;
  for (long k = 0; k < m; k++) { int u, v, J, c; if (scanf("%d %d %d %d", &u, &v, &J, &c) != 4) return 1;
    s.h_eu.push_back(u); s.h_ev.push_back(v); s.h_J.push_back(J); s.h_colour.push_back(c); }
  cosm::LdsSchedule L;
  if (cosm::build_lds_schedule(s, W, 0, &L, true)) return 2;
  // permutation
  std::vector<int> seen(n, 0); for (int sl = 0; sl < L.n_rows; sl++) { if (L.slot_vertex[sl] < 0 || L.slot_vertex[sl] >= n) { puts("BAD slot map"); return 3; } seen[L.slot_vertex[sl]]++; }
  for (int i = 0; i < n; i++) if (seen[i] != 1) { puts("BAD perm"); return 3; }
  std::vector<int> vslot(n); for (int sl = 0; sl < n; sl++) vslot[L.slot_vertex[sl]] = sl;
  // each edge once, in its class, conflict-free groups
  // (class, slot_u, slot_v, J) of every edge, expected and scheduled
  std::multiset<std::tuple<int,int,int,float>> want, got;
  for (long k = 0; k < m; k++) want.insert({s.h_colour[k], vslot[s.h_eu[k]] , vslot[s.h_ev[k]], (float)s.h_J[k]});
  const int rlanes = W == 1 ? 32 : 256 / (4 * W), wlanes = 128 / (4 * W);
  int j = 0; long conflicts = 0, active = 0, dummies = 0, bad_dummy = 0;
  auto count = [&](int jj, int g0, int lanes, bool record) {
    int bu[64] = {0}, bv[64] = {0};
    for (int t = g0; t < g0 + lanes && t < L.nth; t++) {
      auto d = L.desc[(size_t)jj * L.nth + t];
      if (d.slots == cosm::kEmptySlot) continue;
      int su = d.slots & 0xffff, sv = d.slots >> 16;
      // dummy no-op edges of masked lanes: dummy rows only, J = 0, counted for
      // bank conflicts like the edges
      const bool dummy = su >= n || sv >= n;
      if (dummy && !(su >= n && sv >= n && su < n + cosm::kDummyRows && sv < n + cosm::kDummyRows &&
                     d.J == 0.0f && su != sv)) bad_dummy++;
      if (record && !dummy) { active++; got.insert({0, su, sv, d.J}); }
      if (record && dummy) dummies++;
      for (int w = 0; w < W; w++) { bu[(su * W + w) % 64]++; bv[(sv * W + w) % 64]++; }
    }
    for (int b = 0; b < 64; b++) conflicts += (bu[b] > 1 ? bu[b] - 1 : 0) + (bv[b] > 1 ? bv[b] - 1 : 0);
  };
  std::multiset<std::tuple<int,int,int,float>> got_c;
  for (int c = 0; c < C; c++) {
    for (int k = 0; k < L.K[c]; k++, j++) {
      got.clear();
      for (int g0 = 0; g0 < L.nth; g0 += rlanes) count(j, g0, rlanes, true);
      for (int g0 = 0; g0 < L.nth; g0 += wlanes) count(j, g0, wlanes, false);
      for (auto &e : got) got_c.insert({c, std::get<1>(e), std::get<2>(e), std::get<3>(e)});
    }
  }
  got = got_c;
  // rows outside the last class (after the repeated slots): together with the
  // last class's rows, every row exactly once (without fuse the twist keeps
  // its own pass)
  int fuse_ok = 1;
  long fuse_conflicts = 0;
  // the kStreamRepeat slots after the last repeat slots 0, 1, ... mod total
  const size_t rep = (size_t)(L.total_slots + cosm::kStreamRepeat) * L.nth;
  if (L.desc.size() < rep) fuse_ok = 0;
  for (int q = 0; q < cosm::kStreamRepeat && fuse_ok && L.total_slots > 0; q++)
    for (int t = 0; t < L.nth; t++) {
      auto a = L.desc[(size_t)(L.total_slots + q) * L.nth + t];
      auto b = L.desc[(size_t)(q % L.total_slots) * L.nth + t];
      if (a.slots != b.slots || a.J != b.J) { fuse_ok = 0; break; }
    }
  if (L.fuse) {
    if (L.desc.size() != rep + (size_t)L.fuse_k * L.nth) fuse_ok = 0;
    std::vector<int> hit(n, 0);
    for (int k = 0; k < L.K[C - 1]; k++)
      for (int t = 0; t < L.nth; t++) {
        auto d = L.desc[(size_t)(L.total_slots - L.K[C - 1] + k) * L.nth + t];
        if (d.slots == cosm::kEmptySlot || (int)(d.slots & 0xffff) >= n) continue;  // masked lane
        hit[d.slots & 0xffff]++; hit[d.slots >> 16]++;
      }
    for (int q = 0; q < L.fuse_k && fuse_ok; q++)
      for (int t = 0; t < L.nth; t++) {
        auto d = L.desc[rep + (size_t)q * L.nth + t];
        if (d.slots == cosm::kEmptySlot) continue;
        if (d.slots >= (uint32_t)n) { fuse_ok = 0; break; }
        hit[d.slots]++;
      }
    for (int r = 0; r < n; r++) if (hit[r] != 1) fuse_ok = 0;
    // bank collisions of those rows within the lane groups of the model
    for (int q = 0; q < L.fuse_k; q++)
      for (int lanes : {rlanes, wlanes})
        for (int g0 = 0; g0 < L.nth; g0 += lanes) {
          int b[64] = {0};
          for (int t = g0; t < g0 + lanes && t < L.nth; t++) {
            auto d = L.desc[rep + (size_t)q * L.nth + t];
            if (d.slots == cosm::kEmptySlot) continue;
            for (int w = 0; w < W; w++) b[(d.slots * W + w) % 64]++;
          }
          for (int k = 0; k < 64; k++) fuse_conflicts += b[k] > 1 ? b[k] - 1 : 0;
        }
  } else if (L.desc.size() != rep) {
    fuse_ok = 0;
  }
  // The streamed word form: decode (u_off | Jneg << 31, v_off) back to rows;
  // every class holds an even number of slots whose real entries are exactly
  // the class's edges (sign and magnitude of J), dummy entries pair dummy rows
  // only, lanes past last_lanes in a class's last slot and every lane of a
  // padding slot hold dummies only, the
  // first slots repeat after the last, the rows outside the last class follow
  // as byte offsets, and no group of the LDS model touches a bank twice.
  int stream_ok = 1;
  long stream_conflicts = 0;
  if (L.stream) {
    const uint32_t rowb = 4u * W;
    std::multiset<std::tuple<int,int,int,float>> sgot;
    const size_t nth = (size_t)L.nth;
    auto dec = [&](size_t e, int &ru, int &rv, float &J) {
      const uint32_t x = L.sdesc[2 * e], y = L.sdesc[2 * e + 1];
      if ((x & 0x7fffffffu) % rowb || y % rowb) stream_ok = 0;
      ru = (int)((x & 0x7fffffffu) / rowb);
      rv = (int)(y / rowb);
      const float mag = L.junit ? L.jscale : L.sjmag[e];
      J = (x >> 31) ? -mag : mag;
    };
    int jj = 0;
    for (int c = 0; c < C && stream_ok; c++) {
      const int K = L.K[c], Kp = (K + cosm::kWordGroup - 1) / cosm::kWordGroup * cosm::kWordGroup;
      if (K % 2 == 0 && L.last_lanes[c] != L.nth) stream_ok = 0;
      for (int k = 0; k < Kp; k++, jj++) {
        for (size_t t = 0; t < nth; t++) {
          int ru, rv; float J;
          dec((size_t)jj * nth + t, ru, rv, J);
          const bool dummy = ru >= n || rv >= n;
          if (dummy) {
            if (!(ru >= n && rv >= n && ru < n + cosm::kDummyRows && rv < n + cosm::kDummyRows &&
                  ru != rv)) stream_ok = 0;
            if (!L.junit && J != 0.0f) stream_ok = 0;
          } else {
            // padding slots and lanes past last_lanes in the last slot are not run
            if (k >= K || (k == K - 1 && (int)t >= L.last_lanes[c])) stream_ok = 0;
            sgot.insert({c, ru, rv, J});
          }
        }
        for (int lanes : {rlanes, wlanes})
          for (size_t g0 = 0; g0 < nth; g0 += lanes) {
            int bu[64] = {0}, bv[64] = {0};
            for (size_t t = g0; t < g0 + lanes && t < nth; t++) {
              int ru, rv; float J;
              dec((size_t)jj * nth + t, ru, rv, J);
              for (int w = 0; w < W; w++) { bu[(ru * W + w) % 64]++; bv[(rv * W + w) % 64]++; }
            }
            for (int b = 0; b < 64; b++)
              stream_conflicts += (bu[b] > 1 ? bu[b] - 1 : 0) + (bv[b] > 1 ? bv[b] - 1 : 0);
          }
      }
    }
    if (jj != L.stotal) stream_ok = 0;
    if (sgot != got) stream_ok = 0;
    const size_t rep = (size_t)(L.stotal + cosm::kWordRepeat) * nth;
    if (L.sdesc.size() != 2 * (rep + (L.fuse ? (size_t)L.fuse_k * nth : 0))) stream_ok = 0;
    if (!L.junit && L.sjmag.size() != rep) stream_ok = 0;
    for (int q = 0; q < cosm::kWordRepeat && stream_ok; q++)
      for (size_t t = 0; t < nth; t++) {
        const size_t a = (size_t)(L.stotal + q) * nth + t, b = (size_t)(q % L.stotal) * nth + t;
        if (L.sdesc[2 * a] != L.sdesc[2 * b] || L.sdesc[2 * a + 1] != L.sdesc[2 * b + 1]) stream_ok = 0;
      }
    if (L.fuse)
      for (size_t e = 0; e < (size_t)L.fuse_k * nth; e++) {
        const cosm::EdgeDesc d = L.desc[(size_t)(L.total_slots + cosm::kStreamRepeat) * nth + e];
        const uint32_t want_w = d.slots == cosm::kEmptySlot ? cosm::kEmptySlot : d.slots * rowb;
        if (L.sdesc[2 * (rep + e)] != want_w) stream_ok = 0;
      }
  }
  printf("W=%d G=%d nth=%d slots=%d rows=%d active=%ld pad=%ld (%.1f%%) conflicts=%ld equal=%d fuse=%d fuse_k=%d fuse_ok=%d fuse_conflicts=%ld dummies=%ld bad_dummy=%ld stream=%d stream_ok=%d stream_conflicts=%ld junit=%d\n", W, L.G, L.nth, L.total_slots, L.n_rows, active, L.pad_entries, 100.0*L.pad_entries/m, conflicts, (int)(want==got), (int)L.fuse, L.fuse_k, fuse_ok, fuse_conflicts, dummies, bad_dummy, (int)L.stream, stream_ok, stream_conflicts, (int)L.junit);
  return 0;
}
