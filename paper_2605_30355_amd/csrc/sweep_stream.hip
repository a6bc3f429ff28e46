// sweep_stream.hip -- the LDS-resident sweep for schedules too long to keep in
// registers (the large graphs: 10^4 - 2 10^4 vertices, up to 2 replicas of
// FP32 phases per workgroup, tens of slots per thread and sweep).
//
// One workgroup owns RW = W kPerWord replicas as LDS rows of W words and runs
// every sweep of the call with workgroup barriers between the colour classes
// (Eqs. (12)-(13)); within a class the edges form a matching, so slot k and
// slot k + 1 of a thread touch disjoint rows, and the rows of slot k + 1 are
// read before slot k is computed and written: each wave keeps two slots in
// flight, so the LDS latency of one overlaps the arithmetic of the other.
//
// Schedule words (schedule.cpp, the streamed word form): per lane and slot
// (u_off | Jneg << 31, v_off), the LDS byte offsets of the two rows and the
// sign of J; the magnitude is one constant (JU) or a second stream of |J|.
// Dynamic LDS starts at address 0 (the kernel declares no static LDS), so the
// offsets are the rows' LDS addresses.  The words are read with buffer loads
// whose lane offset is fixed and whose slot offset is a scalar, one slot ahead
// of its rows' reads; masked lanes carry dummy-row pairs, so no lane branches.
// Each wave keeps two slots in flight: within a class the rows of slot k + 1
// are read before slot k is computed and written.  The stream pads every class
// to an even number of slots (a padding slot's words are passed, never run),
// so that a class starts in the same register set whatever came before it.
// The last slot of a class may hold fewer lanes than the workgroup: waves past
// them skip it.  The twist runs as a pass of its own after the last class
// (four rows in flight per thread); folded into a class's slots instead, its
// arithmetic lengthened that class by more than the pass costs.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace cosm {
namespace {

// v_bitop3 truth table of (a & c) | (b & ~c): the bits of a where c is set,
// the bits of b elsewhere.
constexpr int kSelectBits = 0xe4;

struct StreamArgs {
  void *phases;
  const uint32_t *desc;       // [entries][2] schedule words
  const float *jmag;          // [entries] |J| (when |J| varies), else null
  const int32_t *cls;         // [2C]: slots per thread of each class, then last_lanes
  const int32_t *slot_vertex; // [n_rows]
  int32_t R, n_rows, C, total_slots;  // total_slots: padded slots of a sweep
  uint32_t desc_bytes, jmag_bytes;
  float jscale;               // |J| of every edge (uniform magnitude)
  int64_t t0, nsw;
  SweepSchedule sch;
  uint32_t k0, k1, rid0;
};

// Eq. (6) on an edge's two rows of FP32 phases, without the wrap to [0, 1)
// turn (the lazy form).  On the grid schedule every phase is a multiple of
// 2^-23 turn and every step a multiple of 2^-22; while all phases stay inside
// (-1/2, 3/2) turn, each phase, each step result and each difference x_u - x_v
// (|.| < 2) is exact in FP32, so fract(x_u - x_v) and every later phase mod 1
// equal those of the wrapped form bit for bit.  The host enables this form
// only when the phases provably stay there: a twist wraps every row and adds
// at most twist_max, and until the next one a phase moves by at most
// period * alpha_max * (largest sum of |J| at one vertex), with the two
// together below 1/2 turn.
// FP16 / BF16 / FP16_PK (centred values y = x - 1/2) use the same form to save the two
// wraps y - rint(y) of every update: no exactness is claimed there, and a
// value that has drifted to |y| in [1/2, 1) is stored with one bit less of
// fraction (2^-11 turn for FP16, 2^-8 for BF16) until the next twist wraps it.
template <int ST, int W, bool RD>
__device__ __forceinline__ void update_words_lazy(uint32_t (&wu)[W], uint32_t (&wv)[W], float aJ,
                                                  float pm) {
  if constexpr (ST == COSM_STORE_FP16_PK) {  // packed FP16 arithmetic
    update_words<ST, W, true>(wu, wv, aJ);
    return;
  }
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  float xu[RW], xv[RW];
  F::template unpack<W>(wu, xu);
  F::template unpack<W>(wv, xv);
#pragma unroll
  for (int k = 0; k < RW; k++) {
    // RD (the grid schedule): every value exact, the classes run toward
    // minus infinity
    const float dl = RD ? step_by_parity(xu[k] - xv[k], aJ, pm)
                        : (fract1(xu[k] - xv[k]) < 0.5f) ? aJ : -aJ;
    xu[k] -= dl;
    xv[k] += dl;
  }
  F::template pack<W>(xu, wu);
  F::template pack<W>(xv, wv);
}

// One slot in flight: its rows, their addresses and the step alpha_t J.
template <int W>
struct Slot {
  uint32_t u[W], v[W];
  uint32_t au, av;
  float aJ;
};

template <int ST, int W, bool JU, bool LAZY, bool RD>
__global__ void __launch_bounds__(1024) k_sweep_stream(const StreamArgs a) {
  static_assert(!LAZY || lazy_storage(ST), "the lazy wrap is a floating-point form");
  static_assert(!RD || parity_storage(ST), "the parity step is a grid form of the float formats");
  static_assert(!LAZY || ST != COSM_STORE_FP32 || RD, "the lazy FP32 form runs on the grid");
  extern __shared__ uint32_t lds[];
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int32_t r0 = xcd_block(blockIdx.x, gridDim.x) * RW;
  const int32_t nvalid = min(RW, a.R - r0);

  // HBM [n][R] -> LDS rows, dummy rows zero
  for (int s = tid; s < a.n_rows; s += nth) {
    const size_t base = (size_t)a.slot_vertex[s] * a.R + r0;
    float v[RW];
#pragma unroll
    for (int k = 0; k < RW; k++) v[k] = (k < nvalid) ? F::load_elem(a.phases, base + k) : 0.0f;
    uint32_t w[W];
    F::template pack<W>(v, w);
    lds_store<W>(lds, s, w);
  }
  for (int s = tid; s < kDummyRows; s += nth) {
    const uint32_t z[W] = {};
    lds_store<W>(lds, a.n_rows + s, z);
  }
  float *theta_buf = reinterpret_cast<float *>(lds + (size_t)(a.n_rows + kDummyRows) * W);
  int32_t *cls = reinterpret_cast<int32_t *>(theta_buf + 2 * kThetaFloats);  // [2C]
  for (int c = tid; c < 2 * a.C; c += nth) cls[c] = a.cls[c];

  // schedule words: lane offset fixed, slot offset a scalar
  const __amdgpu_buffer_rsrc_t rdesc =
      __builtin_amdgcn_make_buffer_rsrc((void *)a.desc, (short)0, (int)a.desc_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rjmag =
      __builtin_amdgcn_make_buffer_rsrc((void *)a.jmag, (short)0, (int)a.jmag_bytes, 0x00020000);
  const uint32_t lane8 = (uint32_t)tid * 8u, lane4 = (uint32_t)tid * 4u;
  const uint32_t stride8 = (uint32_t)nth * 8u, stride4 = (uint32_t)nth * 4u;
  // (the slot offset is uniform; readfirstlane keeps it in a scalar register)
  auto word = [&](uint32_t slot) -> su2 {
    return __builtin_amdgcn_raw_buffer_load_b64(
        rdesc, lane8, __builtin_amdgcn_readfirstlane(slot * stride8), 0);
  };
  auto mag = [&](uint32_t slot) -> float {
    if constexpr (JU) {
      return 0.0f;
    } else {
      return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          rjmag, lane4, __builtin_amdgcn_readfirstlane(slot * stride4), 0));
    }
  };
  const int32_t wave_base = __builtin_amdgcn_readfirstlane(tid & ~63);
  __syncthreads();

  // Schedule words in flight: set p holds those of a slot of parity p.  A
  // set is refilled right after its rows are read, with the words of the slot
  // two ahead, so each load has about two slots of work to arrive in.
  su2 dw[2];
  float dm[2];
  uint32_t jsw = 0;  // the next slot whose rows are read, within the sweep
  dw[0] = word(0);
  dw[1] = word(1);
  dm[0] = mag(0);
  dm[1] = mag(1);
  Slot<W> sl[2];

  int32_t k_next = cls[0], last_next = cls[a.C];
  SweepSchedule sc = a.sch;
  float pm = 0.0f;  // RD: 1.5 * 2^23 from the switch, the parity fma's addend
  const uint32_t nsw = (uint32_t)a.nsw;
  uint32_t t = (uint32_t)a.t0;
  uint32_t tw = 0;
  ScheduleChunk chunk;
  for (uint32_t it = 0; it < nsw; it++) {
    t++;
    if ((it & 63u) == 0u) chunk.fill(sc, t);
    float alpha, twist;
    chunk.get(it & 63u, alpha, twist);
    // the step magnitude in storage units; its sign comes from the word
    const float amag = alpha * F::kStepScale * (JU ? a.jscale : 1.0f);
    const bool twist_now = chunk.twist_at(it & 63u);
    TwistOps<ST, W> op;
    if (twist_now) {
      const int q = (int)(tw % (uint32_t)kThetaChunk);
      if (q == 0) {
        theta_fill(theta_buf, nullptr, kThetaChunk, RW, t, sc.period, a.rid0 + (uint32_t)r0,
                   a.k0, a.k1, sc.win, sc.tshift, sc.tscale);
        __syncthreads();
      }
      float cth[RW], tws[RW];
#pragma unroll
      for (int k = 0; k < RW; k++) {
        cth[k] = theta_buf[q * RW + k];
        tws[k] = twist;
      }
      op.set(cth, tws, sc.win2);
      tw++;
    }

    // read the rows of slot jsw (words in set p), then fetch the words of
    // slot jsw + 2 into that set
    auto read = [&](int p) {
      Slot<W> &x = sl[p];
      // (both addresses are new values: the refill below may reuse the words'
      // registers at once, with no copy and no wait)
      x.au = dw[p].x & 0x7fffffffu;
      x.av = dw[p].y & 0x7fffffffu;
      const float m = JU ? amag : amag * dm[p];
      // (the sign bit from the word, the rest from m: one v_bitop3)
      x.aJ = __uint_as_float(
          __builtin_amdgcn_bitop3_b32(dw[p].x, __float_as_uint(m), 0x80000000u, kSelectBits));
      row_load<W>(x.au, x.u);
      row_load<W>(x.av, x.v);
      dw[p] = word(jsw + 2);
      dm[p] = mag(jsw + 2);
      jsw++;
    };
    // Eq. (6) on the slot in set p and store
    auto finish = [&](int p) {
      Slot<W> &x = sl[p];
      if constexpr (LAZY) {
        update_words_lazy<ST, W, RD>(x.u, x.v, x.aJ, pm);
      } else {
        update_words<ST, W, false, RD>(x.u, x.v, x.aJ, pm);
      }
      row_store<W>(x.au, x.u);
      row_store<W>(x.av, x.v);
    };
    // npairs pairs of slots of one class: slot 2i in set 0, 2i + 1 in set 1;
    // the rows of the next slot are read before the current one is written
    auto run_pairs = [&](int npairs) {
      read(0);  // slot 0
      read(1);  // slot 1
      finish(0);
      for (int i = 1; i < npairs; i++) {
        read(0);    // slot 2i
        finish(1);  // slot 2i - 1
        read(1);    // slot 2i + 1
        finish(0);  // slot 2i
      }
      finish(1);
    };
    // a pair this wave skips: its words are still consumed in order
    auto skip_pair = [&] {
      dw[0] = word(jsw + 2);
      dm[0] = mag(jsw + 2);
      dw[1] = word(jsw + 3);
      dm[1] = mag(jsw + 3);
      jsw += 2;
    };

    // one class of K slots (the stream pads it to an even number): its pairs,
    // then, for odd K, its last slot alone (the padding slot's words passed)
    auto run_class = [&](int K, bool act_final) {
      const int full = K >> 1;  // pairs of real slots
      const bool odd = (K & 1) != 0;
      // with even K every wave runs every pair; with odd K the last slot holds
      // entries in its first last_lanes lanes only
      if (full > 0) run_pairs(full);
      if (odd) {
        if (act_final) {
          read(0);
          finish(0);
          dw[1] = word(jsw + 2);  // past the padding slot
          dm[1] = mag(jsw + 2);
          jsw++;
        } else {
          skip_pair();
        }
      }
    };

    if constexpr (RD) pm = f32_round_down();
    for (int c = 0; c < a.C; c++) {
      // this class's slot count and last lanes, read one class ahead
      const int K = __builtin_amdgcn_readfirstlane(k_next);
      const int last = __builtin_amdgcn_readfirstlane(last_next);
      const int cn = c + 1 == a.C ? 0 : c + 1;
      k_next = cls[cn];
      last_next = cls[a.C + cn];
      if (K == 0) continue;
      const bool act_final = wave_base < last;
      run_class(K, act_final);
      __syncthreads();
    }
    if constexpr (RD) f32_round_nearest();
    jsw -= (uint32_t)a.total_slots;  // the next sweep's first words are in flight

    // Dual window twist every `period` sweeps, after the last class: whole
    // groups of four rows per thread with no bounds checks (branch-free, the
    // four reads in flight together), then the remaining rows checked
    if (twist_now) {
      const int groups = a.n_rows / (4 * nth);  // uniform
      int s0 = tid;
      for (int g = 0; g < groups; g++, s0 += 4 * nth) {
        uint32_t w[4][W];
#pragma unroll
        for (int q = 0; q < 4; q++) lds_load<W>(lds, s0 + q * nth, w[q]);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          twist_row<ST, W, LAZY>(op, w[q]);
          lds_store<W>(lds, s0 + q * nth, w[q]);
        }
      }
      if (s0 < a.n_rows) {
        uint32_t w[4][W];
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (s0 + q * nth < a.n_rows) lds_load<W>(lds, s0 + q * nth, w[q]);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          if (s0 + q * nth < a.n_rows) {
            twist_row<ST, W, LAZY>(op, w[q]);
            lds_store<W>(lds, s0 + q * nth, w[q]);
          }
        }
      }
      __syncthreads();
    }
  }

  // LDS rows -> HBM
  for (int s = tid; s < a.n_rows; s += nth) {
    const size_t base = (size_t)a.slot_vertex[s] * a.R + r0;
    uint32_t w[W];
    lds_load<W>(lds, s, w);
    float v[RW];
    F::template unpack<W>(w, v);
#pragma unroll
    for (int k = 0; k < RW; k++)
      if (k < nvalid)  // FP32 wraps exactly; 16-bit values go back as they are
        F::store_elem(a.phases, base + k, LAZY && ST == COSM_STORE_FP32 ? F::wrap(v[k]) : v[k]);
  }
}

template <int ST, int W, bool JU, bool LAZY, bool RD>
int launch_stream_k(cosm_state *s, const StreamArgs &a) {
  const size_t lds = s->shape.lds_bytes;
  (void)hipFuncSetAttribute((const void *)k_sweep_stream<ST, W, JU, LAZY, RD>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_sweep_stream<ST, W, JU, LAZY, RD>), dim3(s->shape.blocks),
                     dim3(s->shape.threads), lds, s->stream, a);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    return set_error(COSM_EDEVICE, std::string("k_sweep_stream: ") + hipGetErrorString(err));
  return COSM_OK;
}

template <int ST, int W, bool LAZY, bool RD = false>
int launch_stream_l(cosm_state *s, const StreamArgs &a) {
  if (s->lds.junit) return launch_stream_k<ST, W, true, LAZY, RD>(s, a);
  return launch_stream_k<ST, W, false, LAZY, RD>(s, a);
}

// On the grid schedule FP32, FP16 and BF16 take the parity step (under
// round-toward-minus-infinity), wrapped at the twists where the drift bound
// holds (FP32 wraps lazily only on the grid), else after every update
template <int ST, int W>
int launch_stream_w(cosm_state *s, const StreamArgs &a) {
  if constexpr (parity_storage(ST)) {
    if (grid_parity_step(*s)) {
      if (lds_lazy_wrap(*s)) return launch_stream_l<ST, W, true, true>(s, a);
      return launch_stream_l<ST, W, false, true>(s, a);
    }
  }
  if constexpr (lazy_storage(ST) && ST != COSM_STORE_FP32) {
    if (lds_lazy_wrap(*s)) return launch_stream_l<ST, W, true>(s, a);
  }
  return launch_stream_l<ST, W, false>(s, a);
}

template <int ST>
int launch_stream_st(cosm_state *s, int64_t n_sweeps) {
  const LdsSchedule &L = s->lds;
  StreamArgs a{};
  a.phases = s->d.phases;
  a.desc = reinterpret_cast<const uint32_t *>(s->d.desc);
  a.jmag = L.junit ? nullptr : s->d.jmag;
  a.cls = s->d.class_off;
  a.slot_vertex = s->d.slot_vertex;
  a.R = s->R;
  a.n_rows = L.n_rows;
  a.C = s->C;
  a.total_slots = L.stotal;
  a.desc_bytes = (uint32_t)(L.sdesc.size() * 4);
  a.jmag_bytes = (uint32_t)(L.sjmag.size() * 4);
  a.jscale = L.jscale;
  a.t0 = s->t;
  a.nsw = n_sweeps;
  a.sch = make_sweep_schedule(s->sched, s->t);
  a.k0 = (uint32_t)(s->seed & 0xffffffffu);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.rid0 = (uint32_t)s->rid0;
  const int W = s->shape.rw / Fmt<ST>::kPerWord;
  if (W == 4) return launch_stream_w<ST, 4>(s, a);
  if (W == 2) return launch_stream_w<ST, 2>(s, a);
  if (W == 1) return launch_stream_w<ST, 1>(s, a);
  return set_error(COSM_EINVAL, "unsupported replicas per workgroup");
}

}  // namespace

bool lds_lazy_wrap(const cosm_state &s) {
  const int32_t st = s.p.storage;
  if (st == COSM_STORE_FP16 || st == COSM_STORE_BF16 || st == COSM_STORE_FP16_PK) return lazy16(s);
  // FP32: exact on the grid schedule, in the streamed forms
  return st == COSM_STORE_FP32 && s.sched.grid && s.shape.residency == COSM_RES_LDS &&
         (s.lds.stream || s.lds.rstream) && s.sched.dwt_period > 0 && wrap_drift_turns(s) < 0.5;
}

int launch_sweeps_stream(cosm_state *s, int64_t n_sweeps) {
  switch (s->p.storage) {
    case COSM_STORE_FP32: return launch_stream_st<COSM_STORE_FP32>(s, n_sweeps);
    case COSM_STORE_FP16: return launch_stream_st<COSM_STORE_FP16>(s, n_sweeps);
    case COSM_STORE_FP16_PK: return launch_stream_st<COSM_STORE_FP16_PK>(s, n_sweeps);
    case COSM_STORE_BF16: return launch_stream_st<COSM_STORE_BF16>(s, n_sweeps);
    case COSM_STORE_FIX16: return launch_stream_st<COSM_STORE_FIX16>(s, n_sweeps);
    case COSM_STORE_FIX32: return launch_stream_st<COSM_STORE_FIX32>(s, n_sweeps);
  }
  return set_error(COSM_EINVAL, "unknown storage format");
}

}  // namespace cosm
