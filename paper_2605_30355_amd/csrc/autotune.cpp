// autotune.cpp -- picks the LDS sweep kernel's shape by measurement.
//
// Candidates: every LDS row width that fits (1, 2 or 4 words per row, i.e. 1-4
// FP32 or 2-8 16-bit replicas per workgroup) crossed with a few thread counts
// (pair layout; a long schedule in both streamed forms: the word form with two
// slots in flight per wave, and the classic one), with 1, 2 or 4 register
// rows per thread (register layout, where it applies), and the streamed
// register-owner form (FP32; 512 to 1024 threads); a requested layout
// restricts the candidates to its own.
// Each candidate runs a short timed probe on the state's own phases (which are
// re-drawn afterwards, so the probe leaves no trace in the trajectory), and the
// fastest shape is kept.  Results are cached per process, keyed by the
// instance's signature (sizes, storage, layout request, bias fields and a hash
// of the edge list and colouring).  None of the candidates changes the dynamics: they
// differ only in how the same class-by-class updates are laid out on the GPU.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.hpp"

namespace cosm {

namespace {

// Instance signature: sizes, storage, layout request, bias fields, the kernel
// variant the parameters select (grid schedule: the parity step; drift bound:
// the wrap at the twists), and an FNV-1a hash of the edge list and its
// colouring (the schedules are built from exactly these, so two instances with
// the same key accept the same shapes and run the same kernels).
using Key = std::tuple<int32_t, int64_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t,
                       uint64_t>;
// (W, threads, register rows (kShapeRStream: the streamed register-owner form,
// 0: the pair form), 1 = the classic streamed schedule instead of the streamed
// word form)
using Shape = std::tuple<int32_t, int32_t, int32_t, int32_t>;
std::mutex g_cache_mu;
std::map<Key, Shape> g_cache;

Key make_key(const cosm_state &s) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint32_t v) {
    for (int b = 0; b < 4; b++) h = (h ^ ((v >> (8 * b)) & 0xffu)) * 1099511628211ull;
  };
  for (int64_t k = 0; k < s.m; k++) {
    mix((uint32_t)s.h_eu[(size_t)k]);
    mix((uint32_t)s.h_ev[(size_t)k]);
    mix((uint32_t)s.h_colour[(size_t)k]);
  }
  const int32_t variant = (s.sched.grid ? 1 : 0) |
                          (s.sched.dwt_period > 0 && wrap_drift_turns(s) < 0.5 ? 2 : 0);
  return Key{s.n, s.m, s.C, s.R, s.p.storage, s.p.lds_form, s.has_h ? 1 : 0, variant, h};
}


// K > 0: the register form with K rows; K = kShapeRStream: the streamed
// register-owner form; 0: the pair form.
constexpr int32_t kShapeRStream = -1;

int apply_shape(cosm_state *s, int32_t W, int32_t nth, int32_t pw, int32_t K,
                int32_t classic = 0) {
  if (K > 0) {
    if (int rc = reg_schedule_for(*s, W, K, nth, &s->lds)) return rc;
  } else if (K == kShapeRStream) {
    if (int rc = rstream_schedule_for(*s, W, nth, &s->lds)) return rc;
  } else {
    if (int rc = build_lds_schedule(*s, W, nth, &s->lds, true, classic == 0)) return rc;
  }
  s->shape.residency = COSM_RES_LDS;
  s->shape.rw = W * pw;
  s->shape.blocks = (s->R + s->shape.rw - 1) / s->shape.rw;
  s->shape.lds_bytes = (int32_t)(K == kShapeRStream ? rstream_lds_bytes(s->lds, W, s->C)
                                 : lds_sweep_bytes(K > 0 ? s->lds.n_rows : s->n_slots, W, s->C));
  s->shape.threads = s->lds.nth;
  return upload_lds_schedule(s);
}

}  // namespace

int upload_lds_schedule(cosm_state *s) {
  const LdsSchedule &L = s->lds;
  if (L.rstream) {
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.rs_words, L.rs_words.data(), L.rs_words.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.rs_pwords, L.rs_pwords.data(), L.rs_pwords.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.rs_act, L.rs_act.data(), L.rs_act.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.slot_vertex, L.slot_vertex.data(),
                                  L.slot_vertex.size() * 4, hipMemcpyHostToDevice, s->stream));
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.reg_vertex, L.reg_vertex.data(), L.reg_vertex.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
    COSM_HIP_CHECK(hipStreamSynchronize(s->stream));  // host vectors may change next
    return COSM_OK;
  }
  if (L.stream) {
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.desc, L.sdesc.data(), L.sdesc.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
    if (!L.sjmag.empty())
      COSM_HIP_CHECK(hipMemcpyAsync(s->d.jmag, L.sjmag.data(), L.sjmag.size() * 4,
                                    hipMemcpyHostToDevice, s->stream));
  } else {
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.desc, L.desc.data(), L.desc.size() * sizeof(EdgeDesc),
                                  hipMemcpyHostToDevice, s->stream));
  }
  // slots per class, then (streamed word form) the lanes of each class's last slot
  std::vector<int32_t> cls(L.K);
  if (L.stream) cls.insert(cls.end(), L.last_lanes.begin(), L.last_lanes.end());
  if (!cls.empty())
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.class_off, cls.data(), cls.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
  COSM_HIP_CHECK(hipMemcpyAsync(s->d.slot_vertex, L.slot_vertex.data(),
                                L.slot_vertex.size() * 4, hipMemcpyHostToDevice, s->stream));
  if (L.reg_k > 0)
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.reg_vertex, L.reg_vertex.data(), L.reg_vertex.size() * 4,
                                  hipMemcpyHostToDevice, s->stream));
  if (int rc = upload_h_slot(s)) return rc;
  COSM_HIP_CHECK(hipStreamSynchronize(s->stream));  // host vectors may change next
  return COSM_OK;
}

int upload_h_slot(cosm_state *s) {
  if (!s->has_h) return COSM_OK;
  const LdsSchedule &L = s->lds;
  s->h_slot.assign(L.slot_vertex.size(), 0);
  for (size_t k = 0; k < L.slot_vertex.size(); k++) s->h_slot[k] = s->h_h[(size_t)L.slot_vertex[k]];
  COSM_HIP_CHECK(hipMemcpyAsync(s->d.h_slot, s->h_slot.data(), s->h_slot.size() * 4,
                                hipMemcpyHostToDevice, s->stream));
  return COSM_OK;
}

bool reg_form_supported(const cosm_state &s) {
  const int32_t st = s.p.storage;
  return (st == COSM_STORE_FP32 || st == COSM_STORE_FIX32 || st == COSM_STORE_FIX16) && !s.has_h &&
         s.C <= kRegClassesMax && s.m > 0 && s.p.update == COSM_UPDATE_SCS;
}

int reg_schedule_for(const cosm_state &s, int32_t W, int32_t K, int32_t nth, LdsSchedule *out) {
  if (!reg_form_supported(s))
    return set_error(COSM_ERANGE, "the register form needs FP32, FIX32 or FIX16 storage, at most "
                                  "8 classes, edges and no bias fields");
  if (K == 4 && s.C > 4) return set_error(COSM_ERANGE, "4 register rows need at most 4 classes");
  LdsSchedule L;
  if (int rc = build_reg_schedule(s, W, K, nth, &L)) return rc;
  if (lds_sweep_bytes(L.n_rows, W, s.C) > (size_t)lds_capacity_bytes())
    return set_error(COSM_ERANGE, "register form: rows do not fit in LDS");
  *out = std::move(L);
  return COSM_OK;
}

int rstream_schedule_for(const cosm_state &s, int32_t W, int32_t nth, LdsSchedule *out) {
  if (s.p.storage != COSM_STORE_FP32 || s.has_h || s.C > kRStreamClassesMax || s.m == 0 ||
      s.p.update != COSM_UPDATE_SCS)
    return set_error(COSM_ERANGE, "the streamed register form needs FP32 storage, at most 32 "
                                  "classes, edges and no bias fields");
  LdsSchedule L;
  if (int rc = build_rstream_schedule(s, W, nth, &L)) return rc;
  if (!rstream_shape_supported(s.p.storage, W, L.reg_k))
    return set_error(COSM_ERANGE, "streamed register form: no kernel for this row width and "
                                  "register count");
  if (rstream_lds_bytes(L, W, s.C) > (size_t)lds_capacity_bytes())
    return set_error(COSM_ERANGE, "streamed register form: rows do not fit in LDS");
  *out = std::move(L);
  return COSM_OK;
}

// The register form for a fixed row width: the fewest register rows per
// thread that hold the whole independent set (with a thread count given,
// the set may need 2 or 4 rows per thread), else the most that give one.
int pick_reg_schedule(cosm_state *s, int32_t W, int32_t nth) {
  int rc = COSM_ERANGE;
  bool any = false;
  LdsSchedule best;
  for (int32_t K : {1, 2, 4}) {
    LdsSchedule L;
    if (reg_schedule_for(*s, W, K, nth, &L) != COSM_OK) continue;
    any = true;
    const bool whole = L.reg_set <= (int64_t)K * L.nth;
    best = std::move(L);
    if (whole) break;
  }
  if (!any) return set_error(COSM_ERANGE, "the register form does not apply to this shape");
  clear_error();
  s->lds = std::move(best);
  rc = COSM_OK;
  return rc;
}

int autotune_lds_shape(cosm_state *s, const std::vector<int32_t> &widths) {
  const int32_t pw = (s->p.storage == COSM_STORE_FP32 || s->p.storage == COSM_STORE_FIX32) ? 1 : 2;
  const Key key = make_key(*s);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      if (apply_shape(s, std::get<0>(it->second), std::get<1>(it->second), pw,
                      std::get<2>(it->second), std::get<3>(it->second)) == COSM_OK)
        return COSM_OK;
      // the cached shape does not apply to this instance: measure afresh
      clear_error();
      g_cache.erase(it);
    }
  }
  const int64_t probe = std::min<int64_t>(256, s->p.sweeps_per_trial);
  hipEvent_t e0, e1;
  COSM_HIP_CHECK(hipEventCreate(&e0));
  COSM_HIP_CHECK(hipEventCreate(&e1));
  float best_ms = 0.0f;
  int32_t best_W = 0, best_nth = 0, best_K = 0, best_classic = 0;
  int rc = COSM_OK;
  const bool timing = s->timing;
  s->timing = false;
  // candidates: (W, requested threads, register rows); pair form first
  std::vector<Shape> cands;
  // (the pair form with a long schedule is timed in both streamed forms)
  const int32_t form = s->p.lds_form;
  if (form == COSM_LDS_FORM_AUTO || form == COSM_LDS_FORM_PAIR)
    for (int32_t W : widths)
      for (int32_t req : {0, 512, 768, 1024})
        for (int32_t classic : {0, 1}) cands.emplace_back(W, req, 0, classic);
  if ((form == COSM_LDS_FORM_AUTO || form == COSM_LDS_FORM_REGISTER) && reg_form_supported(*s))
    for (int32_t W : widths)
      for (int32_t K : {1, 2, 4}) cands.emplace_back(W, 0, K, 0);
  // (fewer threads hold more register rows each, and may leave room for a
  // second workgroup per CU)
  if (form == COSM_LDS_FORM_AUTO || form == COSM_LDS_FORM_REGISTER_STREAM)
    for (int32_t W : widths)
      for (int32_t req : {1024, 768, 640, 512}) cands.emplace_back(W, req, kShapeRStream, 0);
  std::vector<Shape> tried;
  int32_t auto_nth = 0;
  for (const Shape &cand : cands) {
    const int32_t W = std::get<0>(cand), req = std::get<1>(cand), K = std::get<2>(cand);
    const int32_t classic = std::get<3>(cand);
    if (K == 0 && req > 0 && req < auto_nth / 2) continue;  // far too few threads for one pass
    rc = apply_shape(s, W, req, pw, K, classic);
    if (rc && K != 0) {  // a register form does not apply to this shape
      rc = COSM_OK;
      clear_error();
      continue;
    }
    if (rc) break;
    if (K == 0 && req == 0) auto_nth = s->lds.nth;
    // a short schedule (or one with a field pass) has no word form: the two
    // candidates are one
    const bool long_sched = K == 0 && s->lds.total_slots > kRegisterSlotsMax && !s->has_h;
    const Shape got{W, s->lds.nth, K, classic != 0 && long_sched ? 1 : 0};
    if (std::find(tried.begin(), tried.end(), got) != tried.end()) continue;
    tried.push_back(got);
    const int64_t t_saved = s->t;
    rc = launch_sweeps(s, probe);  // warm-up
    s->t = t_saved;
    if (rc) break;
    // the faster of two timed probes (single probes of a few hundred
    // microseconds vary by several per cent)
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && rc == COSM_OK; rep++) {
      if (hipEventRecord(e0, s->stream) != hipSuccess) { rc = set_error(COSM_EDEVICE, "event"); break; }
      rc = launch_sweeps(s, probe);
      s->t = t_saved;
      if (rc) break;
      if (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = set_error(COSM_EDEVICE, "event");
        break;
      }
      float one = 0.0f;
      (void)hipEventElapsedTime(&one, e0, e1);
      ms = rep == 0 ? one : std::min(ms, one);
    }
    if (rc) break;
    if (best_W == 0 || ms < best_ms) {
      best_ms = ms;
      best_W = W;
      best_nth = s->lds.nth;
      best_K = K;
      best_classic = std::get<3>(got);
    }
  }
  if (rc == COSM_OK && best_W == 0)
    rc = set_error(COSM_ERANGE, "no LDS shape applies (register form requested)");
  s->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  s->launches = 0;
  s->kernel_ms = 0.0;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = Shape{best_W, best_nth, best_K, best_classic};
  }
  rc = apply_shape(s, best_W, best_nth, pw, best_K, best_classic);
  if (rc) return rc;
  return launch_init(s);  // the probes moved the phases: draw them again
}

}  // namespace cosm
