// api.cpp -- the C ABI of libcosm (include/cosm.h): argument checks, state
// lifetime, device memory plan, kernel-shape choice and trial statistics.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>

#include "internal.hpp"

namespace cosm {

static thread_local std::string g_last_error;

int set_error(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}
void clear_error() { g_last_error.clear(); }

namespace {

bool wide_storage(int32_t storage) {
  return storage == COSM_STORE_FP32 || storage == COSM_STORE_FIX32;
}
int storage_bytes(int32_t storage) { return wide_storage(storage) ? 4 : 2; }  // FP16, BF16, FIX16: 2
int per_word(int32_t storage) { return wide_storage(storage) ? 1 : 2; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offsets of every device buffer inside one allocation.
struct MemPlan {
  size_t phases, desc, jmag, class_off, slot_vertex, reg_vertex, rs_words, rs_pwords, rs_act, h_slot, eu, ev, J, h, peu, pev, pJ, spins, H, cut, best_p,
      inc_off, inc_nbr, inc_J, phases_alt, opt_keys, opt_keys2, opt_vals, opt_vals2, opt_off,
      opt_temp, opt_temp_bytes, codes, total;
};

MemPlan plan_memory(int32_t n, int64_t m, int32_t C, int32_t R, const cosm_params &p) {
  MemPlan mp{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1), 256);
    return at;
  };
  const size_t nr = (size_t)n * (size_t)R;
  mp.phases = take(nr * storage_bytes(p.storage));
  // lane schedule: at most 32 lanes per edge group plus one partial pass per
  // class, the repeated slots, then the rows outside the last class
  // (or the register-owner form's [C][K + 1][nth])
  // (the streamed word form pads each class to a multiple of kWordGroup slots)
  const size_t pair_desc = (size_t)32 * m + (size_t)kWordGroup * 1024 * C + 1024 +
                           (size_t)(kWordRepeat + kFuseRowsMax) * 1024;
  const size_t reg_desc = (size_t)std::min(C, kRegClassesMax) * (kRegKMax + 1) * 1024;
  mp.desc = take(std::max(pair_desc, reg_desc) * sizeof(EdgeDesc));
  mp.jmag = take(pair_desc * 4);
  mp.class_off = take(((size_t)2 * C + 1) * 4);
  mp.slot_vertex = take(((size_t)n + kRegRowsSlack) * 4);
  mp.reg_vertex = take((size_t)kRStreamKMax * 1024 * 4);
  const size_t rs_classes = (size_t)std::min(C, kRStreamClassesMax);
  mp.rs_words = take(rs_classes * kRStreamKMax * 1024 * 8);
  mp.rs_pwords = take(rs_classes * kRStreamPairs * 1024 * 8);
  mp.rs_act = take(rs_classes * 16 * 4);
  mp.h_slot = take(((size_t)n + 1) * 4);
  mp.eu = take((size_t)m * 4);
  mp.ev = take((size_t)m * 4);
  mp.J = take((size_t)m * 4);
  mp.h = take((size_t)n * 4);
  mp.peu = take((size_t)m * 4);
  mp.pev = take((size_t)m * 4);
  mp.pJ = take((size_t)m * 4);
  mp.spins = take(nr);
  mp.H = take((size_t)R * 8);
  mp.cut = take((size_t)R * 8);
  mp.best_p = take((size_t)R * 4);
  const bool fg = p.update == COSM_UPDATE_FULL_GRADIENT;
  mp.inc_off = take(fg ? ((size_t)n + 1) * 4 : 0);
  mp.inc_nbr = take(fg ? (size_t)(2 * m) * 4 : 0);
  mp.inc_J = take(fg ? (size_t)(2 * m) * 4 : 0);
  mp.phases_alt = take(fg ? nr * storage_bytes(p.storage) : 0);
  const bool opt = p.readout == COSM_READOUT_OPTIMAL;
  mp.opt_keys = take(opt ? nr * 4 : 0);
  mp.opt_keys2 = take(opt ? nr * 4 : 0);
  mp.opt_vals = take(opt ? nr * 4 : 0);
  mp.opt_vals2 = take(opt ? nr * 4 : 0);
  mp.opt_off = take(opt ? ((size_t)R + 1) * 4 : 0);
  mp.opt_temp_bytes = opt ? opt_readout_temp_bytes(n, R) : 0;
  mp.opt_temp = take(mp.opt_temp_bytes);
  // readout codes in device memory when n is too large for them to sit in LDS
  const bool codes = readout_lds_bytes(n, p.n_bisectors) > kReadoutLdsLimit;
  mp.codes = take(codes ? nr * 2 : 0);
  mp.total = off;
  return mp;
}

}  // namespace

int check_params_public(const cosm_params *p);

namespace {

int check_params(const cosm_params *p) {
  if (p == nullptr) return set_error(COSM_EINVAL, "params must not be NULL");
  auto bad = [](const char *m) { return set_error(COSM_EINVAL, m); };
  if (!(p->alpha0_deg >= 0.0) || !std::isfinite(p->alpha0_deg)) return bad("alpha0_deg must be >= 0");
  if (!(p->dwt_ratio >= 0.0) || !std::isfinite(p->dwt_ratio)) return bad("dwt_ratio must be >= 0");
  if (p->dwt_period < 0) return bad("dwt_period must be >= 0");
  if (!(p->dwt_window_deg > 0.0 && p->dwt_window_deg <= 180.0))
    return bad("dwt_window_deg must be in (0, 180]");
  if (p->n_bisectors < 1 || p->n_bisectors > 32767) return bad("n_bisectors must be in [1, 32767]");
  if (p->sweeps_per_trial < 1 || p->sweeps_per_trial > ((int64_t)1 << 31))
    return bad("sweeps_per_trial must be in [1, 2^31]");
  if (p->schedule != COSM_SCHED_GRID && p->schedule != COSM_SCHED_CONTINUOUS) return bad("bad schedule");
  if (p->storage < COSM_STORE_FP32 || p->storage > COSM_STORE_FP16_PK) return bad("bad storage");
  if (p->storage == COSM_STORE_FIX16 && p->schedule != COSM_SCHED_GRID)
    return bad("FIX16 storage needs the GRID schedule");
  if (p->storage == COSM_STORE_FIX32 && p->schedule != COSM_SCHED_GRID)
    return bad("FIX32 storage needs the GRID schedule");
  if (p->residency < COSM_RES_AUTO || p->residency > COSM_RES_PLAIN) return bad("bad residency");
  if (p->update != COSM_UPDATE_SCS && p->update != COSM_UPDATE_FULL_GRADIENT) return bad("bad update");
  if (p->lds_form < COSM_LDS_FORM_AUTO || p->lds_form > COSM_LDS_FORM_REGISTER_STREAM)
    return bad("bad lds_form");
  if (p->readout != COSM_READOUT_BISECTORS && p->readout != COSM_READOUT_OPTIMAL)
    return bad("bad readout");
  if (p->replicas_per_wg < 0 || p->threads_per_wg < 0 || p->threads_per_wg > 1024)
    return bad("bad workgroup shape");
  return COSM_OK;
}

}  // namespace

// Schedule constants shared by every sweep form; the grid reading of the step
// ramp and of the twist (see the header of kernels.hip).
int make_schedule(const cosm_params &p, int32_t max_abs_J, Schedule *sc) {
  if (p.alpha0_deg * max_abs_J >= 360.0)
    return set_error(COSM_ERANGE, "alpha0 * |J| must stay below a full turn");
  // FIX32 steps are signed 32-bit integers of 2^-32 turn
  if (p.storage == COSM_STORE_FIX32 && p.alpha0_deg * max_abs_J >= 180.0)
    return set_error(COSM_ERANGE, "FIX32 needs alpha0 * |J| below half a turn");
  if (p.alpha0_deg * p.dwt_ratio >= 360.0)
    return set_error(COSM_ERANGE, "dwt_ratio * alpha0 must stay below a full turn");
  sc->grid = p.schedule == COSM_SCHED_GRID;
  const bool fix16 = p.storage == COSM_STORE_FIX16;
  // grid of the phases (2^-bits turn) and of the steps (twice as coarse)
  const int bits = fix16 ? 16 : 23;
  const double step_per_turn = std::ldexp(1.0, bits - 1);
  sc->aunit = (float)std::ldexp(1.0, 1 - bits);
  sc->tunit = (float)std::ldexp(1.0, -bits);
  sc->tshift = 32 - bits;
  sc->tscale = (float)std::ldexp(1.0, -bits);
  sc->ishift = sc->grid ? 32 - bits : 8;
  sc->iscale = sc->grid ? (float)std::ldexp(1.0, -bits) : (float)std::ldexp(1.0, -24);
  sc->S = p.sweeps_per_trial;
  sc->a0_units = (int64_t)std::floor(p.alpha0_deg / 360.0 * step_per_turn + 0.5);
  // FIX32: the largest step, alpha0 rounded to the step grid times |J|, in
  // units of 2^-32 turn (2^10 per step unit) must stay a positive int32, so
  // the bound is checked after the rounding
  if (p.storage == COSM_STORE_FIX32 && sc->a0_units * (int64_t)max_abs_J >= ((int64_t)1 << 21))
    return set_error(COSM_ERANGE, "FIX32 needs alpha0 * |J| (on the step grid) below half a turn");
  const double r2 = 2.0 * p.dwt_ratio;
  sc->twist_num2 = (int32_t)std::llround(r2);
  // the window on the step grid keeps the twist's membership test exact
  const double w_units = p.dwt_window_deg / 360.0 * (fix16 ? std::ldexp(1.0, 16) : step_per_turn);
  if (sc->grid) {
    if (std::fabs(r2 - sc->twist_num2) > 1e-12)
      return set_error(COSM_ERANGE, "GRID schedule needs 2 * dwt_ratio to be an integer");
    if (std::fabs(w_units - std::round(w_units)) > 1e-6)
      return set_error(COSM_ERANGE, fix16 ? "FIX16 needs the window on the 2^-16 turn grid"
                                          : "GRID schedule needs the window on the 2^-22 turn grid");
  }
  sc->alpha0_turns = (float)(p.alpha0_deg / 360.0);
  sc->dwt_ratio = (float)p.dwt_ratio;
  sc->dwt_period = p.dwt_period;
  sc->window = (float)(p.dwt_window_deg / 360.0);
  sc->window2 = 2.0f * sc->window;
  return COSM_OK;
}

namespace {

}  // namespace

int check_params_public(const cosm_params *p) { return check_params(p); }

namespace {

int device_cu_count() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
  return v > 0 ? v : 256;
}


// Choose residency, replicas per workgroup and threads.  The LDS form is used
// when a replica block fits; among fitting shapes prefer the widest rows that
// still give every CU a workgroup, else the most workgroups.
int choose_shape(cosm_state *s) {
  const cosm_params &p = s->p;
  KernelShape sh;
  sh.residency = p.residency;
  if (p.update == COSM_UPDATE_FULL_GRADIENT) {
    if (p.residency == COSM_RES_LDS || p.residency == COSM_RES_PLAIN)
      return set_error(COSM_ERANGE, "the full-gradient update runs in the HBM form only");
    sh.residency = COSM_RES_HBM;
  }
  const int pw = per_word(p.storage);
  if (sh.residency == COSM_RES_AUTO || sh.residency == COSM_RES_LDS) {
    const size_t cap = (size_t)lds_capacity_bytes();
    const bool slots_ok = s->n_slots <= 65535;
    int chosen = 0;
    if (p.replicas_per_wg > 0) {
      if (p.replicas_per_wg % pw != 0)
        return set_error(COSM_EINVAL, "replicas_per_wg must be a multiple of 2 for 16-bit storage");
      const int W = p.replicas_per_wg / pw;
      if (W != 1 && W != 2 && W != 4)
        return set_error(COSM_EINVAL, "replicas_per_wg must be 1, 2 or 4 words per row");
      if (slots_ok && lds_sweep_bytes(s->n_slots, W, s->C) <= cap) chosen = W;
      else if (sh.residency == COSM_RES_LDS)
        return set_error(COSM_ERANGE, "requested replicas per workgroup do not fit in LDS");
    } else if (slots_ok) {
      const int cus = device_cu_count();
      int best_full = 0, smallest_fit = 0;
      for (int W : {4, 2, 1}) {
        if (lds_sweep_bytes(s->n_slots, W, s->C) > cap) continue;
        s->lds_widths.push_back(W);
        const int64_t blocks = (s->R + W * pw - 1) / (W * pw);
        if (blocks >= cus && best_full == 0) best_full = W;
        smallest_fit = W;
      }
      chosen = best_full ? best_full : smallest_fit;
    }
    if (chosen == 0) {
      if (sh.residency == COSM_RES_LDS)
        return set_error(COSM_ERANGE, "a replica does not fit in LDS");
      sh.residency = COSM_RES_HBM;
    } else {
      sh.residency = COSM_RES_LDS;
      sh.rw = chosen * pw;
      sh.blocks = (s->R + sh.rw - 1) / sh.rw;
      sh.lds_bytes = (int32_t)lds_sweep_bytes(s->n_slots, chosen, s->C);
      if (int rc = build_lds_schedule(*s, chosen, p.threads_per_wg, &s->lds, true)) return rc;
      sh.threads = s->lds.nth;
      if (p.lds_form == COSM_LDS_FORM_REGISTER) {
        // the autotuner, when it runs, chooses among register shapes only
        if (int rc = pick_reg_schedule(s, chosen, p.threads_per_wg)) return rc;
        sh.threads = s->lds.nth;
        sh.lds_bytes = (int32_t)lds_sweep_bytes(s->lds.n_rows, chosen, s->C);
      } else if (p.lds_form == COSM_LDS_FORM_REGISTER_STREAM) {
        if (int rc = rstream_schedule_for(*s, chosen, p.threads_per_wg, &s->lds)) return rc;
        sh.threads = s->lds.nth;
        sh.lds_bytes = (int32_t)rstream_lds_bytes(s->lds, chosen, s->C);
      }
    }
  }
  if (sh.residency != COSM_RES_LDS) {
    sh.rw = 1;
    sh.threads = 256;
    sh.blocks = 0;
    sh.lds_bytes = 0;
  }
  s->shape = sh;
  return COSM_OK;
}

template <typename T>
T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

int sync(cosm_state *s) {
  COSM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return COSM_OK;
}

}  // namespace
}  // namespace cosm

using namespace cosm;

extern "C" {

const char *cosm_last_error(void) { return g_last_error.c_str(); }
const char *cosm_version(void) { return "cosm-mi355x 0.1 (gfx950)"; }

void cosm_default_params(cosm_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->alpha0_deg = 14.0;
  p->dwt_ratio = 0.5;
  p->dwt_period = 3;
  p->dwt_window_deg = 90.0;
  p->n_bisectors = 100;
  p->sweeps_per_trial = 1000;
  p->schedule = COSM_SCHED_GRID;
  p->storage = COSM_STORE_FP32;
  p->residency = COSM_RES_AUTO;
  p->replicas_per_wg = 0;
  p->threads_per_wg = 0;
  p->update = COSM_UPDATE_SCS;
  p->readout = COSM_READOUT_BISECTORS;
  p->lds_form = COSM_LDS_FORM_AUTO;
}

int cosm_build_partitions(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                          int32_t method, const int32_t *method_args, int32_t *colour_out,
                          int32_t *num_colours_out) {
  clear_error();
  if (num_colours_out == nullptr || (m > 0 && colour_out == nullptr))
    return set_error(COSM_EINVAL, "output pointers must not be NULL");
  if (int rc = validate_graph(n, m, eu, ev, nullptr)) return rc;
  const bool largest_last = (method & COSM_ORDER_LARGEST_LAST) != 0;
  method &= ~COSM_ORDER_LARGEST_LAST;
  int32_t C = 0;
  switch (method) {
    case COSM_COLOR_GREEDY: C = colour_greedy(n, m, eu, ev, colour_out); break;
    case COSM_COLOR_MISRA_GRIES: C = colour_misra_gries(n, m, eu, ev, colour_out); break;
    case COSM_COLOR_BALANCED:
      C = colour_misra_gries(n, m, eu, ev, colour_out);
      equalise_classes(n, m, eu, ev, C, colour_out);
      break;
    case COSM_COLOR_MINIMUM:
      C = colour_minimum(n, m, eu, ev, colour_out);
      equalise_classes(n, m, eu, ev, C, colour_out);
      break;
    case COSM_COLOR_TORUS:
      if (method_args == nullptr) return set_error(COSM_EINVAL, "TORUS needs {Lx, Ly}");
      C = colour_torus(n, m, eu, ev, method_args[0], method_args[1], colour_out);
      if (C < 0) return C;
      break;
    default: return set_error(COSM_EINVAL, "unknown colouring method");
  }
  if (largest_last && C > 1) {
    // swap the labels of the largest class (lowest index on ties) and the last
    std::vector<int64_t> size((size_t)C, 0);
    for (int64_t k = 0; k < m; k++) size[(size_t)colour_out[k]]++;
    int32_t big = 0;
    for (int32_t c = 1; c < C; c++)
      if (size[(size_t)c] > size[(size_t)big]) big = c;
    if (size[(size_t)big] > size[(size_t)C - 1])
      for (int64_t k = 0; k < m; k++) {
        if (colour_out[k] == big) colour_out[k] = C - 1;
        else if (colour_out[k] == C - 1) colour_out[k] = big;
      }
  }
  if (validate_colouring(n, m, eu, ev, colour_out, C) != COSM_OK)
    return set_error(COSM_ECOLOR, "internal error: colouring is not proper: " + g_last_error);
  *num_colours_out = C;
  return COSM_OK;
}

int cosm_workspace_bytes(int32_t n, int64_t m, int32_t num_colours, int32_t replicas,
                         const cosm_params *p, size_t *bytes_out) {
  clear_error();
  if (bytes_out == nullptr) return set_error(COSM_EINVAL, "bytes_out must not be NULL");
  if (int rc = check_params(p)) return rc;
  if (n < 1 || m < 0 || num_colours < 0 || replicas < 1)
    return set_error(COSM_EINVAL, "bad sizes");
  *bytes_out = plan_memory(n, m, num_colours, replicas, *p).total;
  return COSM_OK;
}

int cosm_init(cosm_state **out, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
              const int32_t *J, const int32_t *h, const int32_t *colour, int32_t num_colours,
              const cosm_params *p, uint64_t seed, int32_t replicas, void *hip_stream,
              void *device_workspace, size_t workspace_bytes) {
  clear_error();
  return init_state(out, n, m, eu, ev, J, h, colour, num_colours, p, seed, replicas, hip_stream,
                    device_workspace, workspace_bytes, -1);
}

}  // extern "C"

namespace cosm {

int init_state(cosm_state **out, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
               const int32_t *J, const int32_t *h, const int32_t *colour, int32_t num_colours,
               const cosm_params *p, uint64_t seed, int32_t replicas, void *hip_stream,
               void *device_workspace, size_t workspace_bytes, int32_t static_dev) {
  if (out == nullptr) return set_error(COSM_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (int rc = check_params(p)) return rc;
  if (replicas < 1) return set_error(COSM_EINVAL, "replicas must be >= 1");
  if (m > 0 && J == nullptr) return set_error(COSM_EINVAL, "J must not be NULL");
  if (m >= ((int64_t)1 << 31)) return set_error(COSM_ERANGE, "m must be below 2^31");
  if ((int64_t)n * replicas >= ((int64_t)1 << 40)) return set_error(COSM_ERANGE, "n * R too large");
  if (int rc = validate_graph(n, m, eu, ev, nullptr)) return rc;
  if (int rc = validate_colouring(n, m, eu, ev, colour, num_colours)) return rc;
  if (p->readout == COSM_READOUT_OPTIMAL) {
    if (h != nullptr)
      return set_error(COSM_EINVAL, "the optimal-bisector readout needs h = NULL (with bias "
                                    "fields the semicircle is fixed)");
    if (n > kOptReadoutMaxN)
      return set_error(COSM_ERANGE, "the optimal-bisector readout supports n <= 32768");
    if ((int64_t)n * replicas >= ((int64_t)1 << 31))
      return set_error(COSM_ERANGE, "the optimal-bisector readout needs n * replicas < 2^31");
  }

  int32_t max_abs_J = 0;
  int64_t sum_abs = 0;
  for (int64_t k = 0; k < m; k++) {
    const int64_t a = std::llabs((int64_t)J[k]);
    max_abs_J = (int32_t)std::max<int64_t>(max_abs_J, a);
    sum_abs += a;
  }
  if (h != nullptr)
    for (int32_t i = 0; i < n; i++) {
      // a field is the coupling to the virtual spin: the same step bound applies
      const int64_t a = std::llabs((int64_t)h[i]);
      max_abs_J = (int32_t)std::max<int64_t>(max_abs_J, a);
      sum_abs += a;
    }
  if (sum_abs >= ((int64_t)1 << 60)) return set_error(COSM_ERANGE, "couplings too large");

  cosm_state *s = new (std::nothrow) cosm_state();
  if (s == nullptr) return set_error(COSM_ENOMEM, "out of host memory");
  s->n = n;
  s->m = m;
  s->C = num_colours;
  s->R = replicas;
  s->p = *p;
  if (h != nullptr) s->p.n_bisectors = 1;
  s->seed = seed;
  s->rid0 = 0;
  s->t = 0;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->has_h = h != nullptr;
  if (int rc = make_schedule(s->p, max_abs_J, &s->sched)) {
    delete s;
    return rc;
  }
  s->h_eu.assign(eu, eu + m);
  s->h_ev.assign(ev, ev + m);
  s->h_J.assign(J, J + m);
  s->sumJ = 0;
  for (int64_t k = 0; k < m; k++) s->sumJ += J[k];
  {
    std::vector<int64_t> wdeg((size_t)n, 0);
    for (int64_t k = 0; k < m; k++) {
      const int64_t a = J[k] < 0 ? -(int64_t)J[k] : (int64_t)J[k];
      wdeg[(size_t)eu[k]] += a;
      wdeg[(size_t)ev[k]] += a;
    }
    if (h != nullptr)
      for (int32_t i = 0; i < n; i++) wdeg[(size_t)i] += std::llabs((int64_t)h[i]);
    s->wdeg_max = 0;
    for (int64_t w : wdeg) s->wdeg_max = std::max(s->wdeg_max, w);
  }
  if (h) s->h_h.assign(h, h + n);
  s->h_colour.assign(colour, colour + m);

  // group the edges by class (stable): the plain / HBM arrays and LDS descriptors
  s->class_sizes.assign((size_t)num_colours, 0);
  for (int64_t k = 0; k < m; k++) s->class_sizes[(size_t)colour[k]]++;
  s->class_begin.assign((size_t)num_colours, 0);
  for (int32_t c = 1; c < num_colours; c++)
    s->class_begin[(size_t)c] = s->class_begin[(size_t)c - 1] + s->class_sizes[(size_t)c - 1];
  s->max_class = num_colours ? *std::max_element(s->class_sizes.begin(), s->class_sizes.end()) : 0;
  std::vector<int32_t> peu((size_t)m), pev((size_t)m);
  std::vector<float> pJ((size_t)m);
  {
    std::vector<int32_t> fill(s->class_begin);
    for (int64_t k = 0; k < m; k++) {
      const int32_t pos = fill[(size_t)colour[k]]++;
      peu[(size_t)pos] = eu[k];
      pev[(size_t)pos] = ev[k];
      pJ[(size_t)pos] = (float)J[k];
    }
  }
  s->n_slots = n;

  // incidence lists (full-gradient form)
  std::vector<int32_t> inc_off;
  std::vector<uint32_t> inc_nbr;
  std::vector<float> inc_J;
  if (s->p.update == COSM_UPDATE_FULL_GRADIENT) {
    inc_off.assign((size_t)n + 1, 0);
    for (int64_t k = 0; k < m; k++) {
      inc_off[(size_t)eu[k] + 1]++;
      inc_off[(size_t)ev[k] + 1]++;
    }
    for (int32_t i = 0; i < n; i++) inc_off[(size_t)i + 1] += inc_off[(size_t)i];
    inc_nbr.assign((size_t)(2 * m), 0);
    inc_J.assign((size_t)(2 * m), 0.0f);
    std::vector<int32_t> fill(inc_off.begin(), inc_off.end() - 1);
    for (int64_t k = 0; k < m; k++) {
      int32_t a = fill[(size_t)eu[k]]++;
      inc_nbr[(size_t)a] = (uint32_t)ev[k] | 0x80000000u;
      inc_J[(size_t)a] = (float)J[k];
      a = fill[(size_t)ev[k]]++;
      inc_nbr[(size_t)a] = (uint32_t)eu[k];
      inc_J[(size_t)a] = (float)J[k];
    }
  }

  if (int rc = choose_shape(s)) {
    delete s;
    return rc;
  }
  const char *tune_env = std::getenv("COSM_AUTOTUNE");
  const bool autotune = static_dev < 0 && s->shape.residency == COSM_RES_LDS && p->replicas_per_wg == 0 &&
                        p->threads_per_wg == 0 && s->lds_widths.size() > 0 &&
                        !(tune_env && tune_env[0] == '0');

  const MemPlan mp = plan_memory(n, m, num_colours, replicas, s->p);
  if (device_workspace != nullptr) {
    if (workspace_bytes < mp.total) {
      delete s;
      return set_error(COSM_ENOMEM, "workspace smaller than cosm_workspace_bytes()");
    }
    s->base = device_workspace;
    s->own_memory = false;
  } else {
    if (hipMalloc(&s->base, mp.total) != hipSuccess) {
      (void)hipGetLastError();
      delete s;
      return set_error(COSM_ENOMEM, "hipMalloc of the state's buffers failed");
    }
    s->own_memory = true;
  }
  s->base_bytes = mp.total;
  DeviceBuffers &d = s->d;
  d.phases = at<void>(s->base, mp.phases);
  d.desc = at<EdgeDesc>(s->base, mp.desc);
  d.class_off = at<int32_t>(s->base, mp.class_off);
  d.jmag = at<float>(s->base, mp.jmag);
  d.slot_vertex = at<int32_t>(s->base, mp.slot_vertex);
  d.reg_vertex = at<int32_t>(s->base, mp.reg_vertex);
  d.rs_words = at<uint32_t>(s->base, mp.rs_words);
  d.rs_pwords = at<uint32_t>(s->base, mp.rs_pwords);
  d.rs_act = at<uint32_t>(s->base, mp.rs_act);
  d.h_slot = at<int32_t>(s->base, mp.h_slot);
  d.eu = at<int32_t>(s->base, mp.eu);
  d.ev = at<int32_t>(s->base, mp.ev);
  d.J = at<int32_t>(s->base, mp.J);
  d.h = at<int32_t>(s->base, mp.h);
  d.peu = at<int32_t>(s->base, mp.peu);
  d.pev = at<int32_t>(s->base, mp.pev);
  d.pJ = at<float>(s->base, mp.pJ);
  d.spins = at<int8_t>(s->base, mp.spins);
  d.H = at<int64_t>(s->base, mp.H);
  d.cut = at<int64_t>(s->base, mp.cut);
  d.best_p = at<int32_t>(s->base, mp.best_p);
  d.inc_off = at<int32_t>(s->base, mp.inc_off);
  d.inc_nbr = at<uint32_t>(s->base, mp.inc_nbr);
  d.inc_J = at<float>(s->base, mp.inc_J);
  d.phases_alt = at<void>(s->base, mp.phases_alt);
  d.opt_keys = at<uint32_t>(s->base, mp.opt_keys);
  d.opt_keys2 = at<uint32_t>(s->base, mp.opt_keys2);
  d.opt_vals = at<uint32_t>(s->base, mp.opt_vals);
  d.opt_vals2 = at<uint32_t>(s->base, mp.opt_vals2);
  d.opt_off = at<int32_t>(s->base, mp.opt_off);
  d.opt_temp = at<void>(s->base, mp.opt_temp);
  d.codes = readout_lds_bytes(n, s->p.n_bisectors) > kReadoutLdsLimit
                ? at<uint16_t>(s->base, mp.codes) : nullptr;
  s->opt_temp_bytes = mp.opt_temp_bytes;

  auto up = [&](void *dst, const void *src, size_t bytes) -> int {
    if (bytes == 0) return COSM_OK;
    COSM_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream));
    return COSM_OK;
  };
  int rc = COSM_OK;
  if (s->shape.residency == COSM_RES_LDS) rc = upload_lds_schedule(s);
  rc = rc ? rc : up(d.eu, eu, (size_t)m * 4);
  rc = rc ? rc : up(d.ev, ev, (size_t)m * 4);
  rc = rc ? rc : up(d.J, J, (size_t)m * 4);
  if (h) rc = rc ? rc : up(d.h, h, (size_t)n * 4);
  rc = rc ? rc : up(d.peu, peu.data(), (size_t)m * 4);
  rc = rc ? rc : up(d.pev, pev.data(), (size_t)m * 4);
  rc = rc ? rc : up(d.pJ, pJ.data(), (size_t)m * 4);
  if (s->p.update == COSM_UPDATE_FULL_GRADIENT) {
    rc = rc ? rc : up(d.inc_off, inc_off.data(), inc_off.size() * 4);
    rc = rc ? rc : up(d.inc_nbr, inc_nbr.data(), inc_nbr.size() * 4);
    rc = rc ? rc : up(d.inc_J, inc_J.data(), inc_J.size() * 4);
  }
  if (static_dev < 0) {
    if (rc == COSM_OK && hipEventCreate(&s->ev0) != hipSuccess) rc = set_error(COSM_EDEVICE, "hipEventCreate");
    if (rc == COSM_OK && hipEventCreate(&s->ev1) != hipSuccess) rc = set_error(COSM_EDEVICE, "hipEventCreate");
  }
  rc = rc ? rc : launch_init(s);
  rc = rc ? rc : sync(s);  // the host vectors above must outlive the copies
  if (rc == COSM_OK && autotune) rc = autotune_lds_shape(s, s->lds_widths);
  rc = rc ? rc : sync(s);
  if (rc) {
    // the caller keeps the static scratch array until this returns
    s->static_dev = -1;
    cosm_destroy(s);
    return rc;
  }
  s->static_dev = static_dev;
  *out = s;
  return COSM_OK;
}

}  // namespace cosm

extern "C" {

int cosm_destroy(cosm_state *s) {
  clear_error();
  if (s == nullptr) return COSM_OK;
  (void)hipStreamSynchronize(s->stream);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->own_memory && s->base) (void)hipFree(s->base);
  if (s->static_dev >= 0) release_static_scratch(s->static_dev);
  delete s;
  return COSM_OK;
}

int cosm_reset(cosm_state *s, uint64_t seed, int64_t replica_offset) {
  clear_error();
  if (s == nullptr) return set_error(COSM_EINVAL, "state must not be NULL");
  if (replica_offset < 0 || replica_offset + s->R > ((int64_t)1 << 32))
    return set_error(COSM_ERANGE, "replica indices must stay below 2^32");
  s->seed = seed;
  s->rid0 = replica_offset;
  s->t = 0;
  return launch_init(s);
}

int cosm_sweep(cosm_state *s, int64_t n_sweeps) {
  clear_error();
  if (s == nullptr) return set_error(COSM_EINVAL, "state must not be NULL");
  if (n_sweeps < 0) return set_error(COSM_EINVAL, "n_sweeps must be >= 0");
  if (s->t + n_sweeps > s->p.sweeps_per_trial)
    return set_error(COSM_ERANGE, "sweeps would run past the end of the schedule");
  if (n_sweeps == 0) return COSM_OK;
  if (int rc = launch_sweeps(s, n_sweeps)) return rc;
  s->t += n_sweeps;
  return COSM_OK;
}

int cosm_energy(cosm_state *s, const int8_t *spins, int8_t *spins_out, int64_t *H_out,
                int64_t *cut_out) {
  clear_error();
  if (s == nullptr || H_out == nullptr || cut_out == nullptr)
    return set_error(COSM_EINVAL, "state, H_out and cut_out must not be NULL");
  const size_t nr = (size_t)s->n * s->R;
  if (spins != nullptr) {
    for (size_t i = 0; i < nr; i++)
      if (spins[i] != 1 && spins[i] != -1) return set_error(COSM_EINVAL, "spins must be -1 or +1");
    COSM_HIP_CHECK(hipMemcpyAsync(s->d.spins, spins, nr, hipMemcpyHostToDevice, s->stream));
    if (int rc = launch_energy(s)) return rc;
  } else {
    if (int rc = launch_readout(s)) return rc;
  }
  COSM_HIP_CHECK(hipMemcpyAsync(H_out, s->d.H, (size_t)s->R * 8, hipMemcpyDeviceToHost, s->stream));
  COSM_HIP_CHECK(hipMemcpyAsync(cut_out, s->d.cut, (size_t)s->R * 8, hipMemcpyDeviceToHost, s->stream));
  if (spins_out != nullptr)
    COSM_HIP_CHECK(hipMemcpyAsync(spins_out, s->d.spins, nr, hipMemcpyDeviceToHost, s->stream));
  return sync(s);
}

int cosm_solve_to_target(cosm_state *s, int64_t target_H, int64_t max_trials,
                         int32_t stop_at_first_hit, cosm_tts_result *out, int8_t *best_spins) {
  clear_error();
  if (s == nullptr || out == nullptr) return set_error(COSM_EINVAL, "state and out must not be NULL");
  if (max_trials < 1) return set_error(COSM_EINVAL, "max_trials must be >= 1");
  if (max_trials + s->R > ((int64_t)1 << 32))
    return set_error(COSM_ERANGE, "trial indices must stay below 2^32");
  std::vector<int64_t> H((size_t)s->R), cut((size_t)s->R);
  int64_t trials = 0, succ = 0, best = std::numeric_limits<int64_t>::max(), best_cut = 0;
  double total_ms = 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  COSM_HIP_CHECK(hipEventCreate(&e0));
  COSM_HIP_CHECK(hipEventCreate(&e1));
  int rc = COSM_OK;
  while (trials < max_trials && rc == COSM_OK) {
    if (hipEventRecord(e0, s->stream) != hipSuccess) { rc = set_error(COSM_EDEVICE, "hipEventRecord"); break; }
    rc = cosm_reset(s, s->seed, trials);
    rc = rc ? rc : cosm_sweep(s, s->p.sweeps_per_trial);
    rc = rc ? rc : launch_readout(s);
    if (rc) break;
    if (hipEventRecord(e1, s->stream) != hipSuccess) { rc = set_error(COSM_EDEVICE, "hipEventRecord"); break; }
    if (hipMemcpyAsync(H.data(), s->d.H, (size_t)s->R * 8, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipMemcpyAsync(cut.data(), s->d.cut, (size_t)s->R * 8, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
      rc = set_error(COSM_EDEVICE, "copying batch results failed");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    total_ms += ms;
    int32_t arg = -1;
    for (int32_t r = 0; r < s->R; r++) {
      if (H[(size_t)r] <= target_H) succ++;
      if (H[(size_t)r] < best) {
        best = H[(size_t)r];
        best_cut = cut[(size_t)r];
        arg = r;
      }
    }
    trials += s->R;
    if (arg >= 0 && best_spins != nullptr) {
      if (hipMemcpy(best_spins, s->d.spins + (size_t)arg * s->n, (size_t)s->n,
                    hipMemcpyDeviceToHost) != hipSuccess) {
        rc = set_error(COSM_EDEVICE, "copying best spins failed");
        break;
      }
    }
    if (stop_at_first_hit && succ > 0) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const double n = (double)trials, ps = n > 0 ? succ / n : 0.0;
  const double z = 1.959963984540054;
  const double den = 1.0 + z * z / n;
  const double centre = (ps + z * z / (2 * n)) / den;
  const double half = z * std::sqrt(ps * (1 - ps) / n + z * z / (4 * n * n)) / den;
  out->trials = trials;
  out->successes = succ;
  out->ps = ps;
  out->ps_lo = std::max(0.0, centre - half);
  out->ps_hi = std::min(1.0, centre + half);
  out->r99 = ps >= 1.0 ? 1.0 : (ps <= 0.0 ? INFINITY : std::log(0.01) / std::log(1.0 - ps));
  out->t_trial_s = total_ms / 1000.0 / n;
  out->ttt_s = out->t_trial_s * out->r99;
  out->stt_sweeps = (double)s->p.sweeps_per_trial * out->r99;
  out->best_H = best;
  out->best_cut = best_cut;
  return COSM_OK;
}

int cosm_get_phases(cosm_state *s, int32_t unit, double *out) {
  clear_error();
  if (s == nullptr || out == nullptr) return set_error(COSM_EINVAL, "state and out must not be NULL");
  if (unit < COSM_UNIT_TURNS || unit > COSM_UNIT_RADIANS) return set_error(COSM_EINVAL, "bad unit");
  const size_t nr = (size_t)s->n * s->R;
  float *tmp = nullptr;
  COSM_HIP_CHECK(hipMalloc(&tmp, nr * 4));
  std::vector<float> host(nr);
  int rc = launch_to_turns(s, tmp);
  if (!rc && hipMemcpyAsync(host.data(), tmp, nr * 4, hipMemcpyDeviceToHost, s->stream) != hipSuccess)
    rc = set_error(COSM_EDEVICE, "hipMemcpy");
  if (!rc) rc = sync(s);
  (void)hipFree(tmp);
  if (rc) return rc;
  const double scale = unit == COSM_UNIT_TURNS ? 1.0 : unit == COSM_UNIT_DEGREES ? 360.0 : 2.0 * M_PI;
  for (int32_t i = 0; i < s->n; i++)
    for (int32_t r = 0; r < s->R; r++)
      out[(size_t)r * s->n + i] = (double)host[(size_t)i * s->R + r] * scale;
  return COSM_OK;
}

int cosm_set_phases(cosm_state *s, int32_t unit, const double *in, int64_t t) {
  clear_error();
  if (s == nullptr || in == nullptr) return set_error(COSM_EINVAL, "state and in must not be NULL");
  if (unit < COSM_UNIT_TURNS || unit > COSM_UNIT_RADIANS) return set_error(COSM_EINVAL, "bad unit");
  if (t < 0 || t > s->p.sweeps_per_trial) return set_error(COSM_ERANGE, "t outside the schedule");
  const size_t nr = (size_t)s->n * s->R;
  const double scale = unit == COSM_UNIT_TURNS ? 1.0 : unit == COSM_UNIT_DEGREES ? 360.0 : 2.0 * M_PI;
  std::vector<float> host(nr);
  for (int32_t r = 0; r < s->R; r++)
    for (int32_t i = 0; i < s->n; i++) {
      double x = in[(size_t)r * s->n + i] / scale;
      if (!std::isfinite(x)) return set_error(COSM_EINVAL, "phases must be finite");
      x -= std::floor(x);
      float f = (float)x;
      if (f >= 1.0f) f = 0.0f;
      host[(size_t)i * s->R + r] = f;
    }
  float *tmp = nullptr;
  COSM_HIP_CHECK(hipMalloc(&tmp, nr * 4));
  int rc = COSM_OK;
  if (hipMemcpyAsync(tmp, host.data(), nr * 4, hipMemcpyHostToDevice, s->stream) != hipSuccess)
    rc = set_error(COSM_EDEVICE, "hipMemcpy");
  if (!rc) rc = launch_from_turns(s, tmp);
  if (!rc) rc = sync(s);
  (void)hipFree(tmp);
  if (!rc) s->t = t;
  return rc;
}

int cosm_get_info(const cosm_state *s, cosm_info *out) {
  clear_error();
  if (s == nullptr || out == nullptr) return set_error(COSM_EINVAL, "state and out must not be NULL");
  out->n = s->n;
  out->num_colours = s->C;
  out->replicas = s->R;
  out->m = s->m;
  out->sweeps_done = s->t;
  out->residency = s->shape.residency;
  out->storage = s->p.storage;
  out->replicas_per_wg = s->shape.rw;
  out->threads_per_wg = s->shape.threads;
  out->workgroups = s->shape.blocks;
  out->lds_bytes = s->shape.lds_bytes;
  out->max_class_edges = s->max_class;
  out->sweep_launches = s->launches;
  out->sweep_kernel_ms = s->kernel_ms;
  out->lds_form = s->shape.residency != COSM_RES_LDS ? 0
                  : s->lds.rstream                   ? COSM_LDS_FORM_REGISTER_STREAM
                  : s->lds.reg_k > 0                 ? COSM_LDS_FORM_REGISTER
                                                     : COSM_LDS_FORM_PAIR;
  out->register_rows = s->shape.residency == COSM_RES_LDS ? s->lds.reg_k : 0;
  out->twist_fused = lds_twist_fused(*s) ? 1 : 0;
  out->register_vertices = 0;
  out->register_edges = 0;
  if (s->shape.residency == COSM_RES_LDS && s->lds.reg_k > 0) {
    for (int32_t v : s->lds.reg_vertex) out->register_vertices += v >= 0 ? 1 : 0;
    out->register_edges = s->lds.reg_edges;
  }
  out->streamed = s->shape.residency == COSM_RES_LDS && (s->lds.stream || s->lds.rstream) ? 1 : 0;
  out->lazy_wrap = lds_lazy_wrap(*s) ? 1 : 0;
  return COSM_OK;
}

int cosm_set_timing(cosm_state *s, int32_t on) {
  clear_error();
  if (s == nullptr) return set_error(COSM_EINVAL, "state must not be NULL");
  if (on && s->ev0 == nullptr) {  // a state made by cosm_init_static has no events yet
    COSM_HIP_CHECK(hipEventCreate(&s->ev0));
    COSM_HIP_CHECK(hipEventCreate(&s->ev1));
  }
  s->timing = on != 0;
  if (s->timing) {
    s->launches = 0;
    s->kernel_ms = 0.0;
  }
  return COSM_OK;
}

}  // extern "C"
