// sweep_rstream.hip -- the streamed register-owner form of the LDS-resident
// sweep, for the large graphs (10^4 - 2 10^4 vertices, long schedules).
//
// An independent set of vertices lives in registers: thread t owns K of them
// (K = 8, 10, 12 or 16), as W words each (RW replicas).  Every edge with an
// endpoint there is applied by that endpoint's owner, which reads and writes
// only the other endpoint's LDS row; since no two register vertices are
// adjacent, an edge has at most one register endpoint, and the LDS traffic of
// those edges is half that of the pair form.  Edges between two LDS rows take
// up to kRStreamPairs pair slots per class.  The classes run in order with a
// barrier after each (Eqs. (12)-(13)); the order of the edges within a class
// is free because the class is a matching.
//
// Schedule (reg_schedule.cpp): register slots exist in the register classes
// only (those where at least half of the register set has an edge; the seams
// of an odd torus are not, and their vertices stay in LDS), K per class, all
// run by every wave straight through, the row of slot k + 1 read before slot
// k is computed; a slot's word per lane is (the LDS endpoint's row offset |
// flip << 31, J as a float, 0 for no edge).  Pair slots, kRStreamPairs per
// class, hold 8 bytes per lane (u row offset with J in its top 14 bits, v row
// offset), and a wave runs only those with an edge in some lane (per-wave
// mask).  The words are read with scalar-offset buffer loads: a register
// slot's word a few slots ahead (into the ring register its own word has just
// left), a pair slot's one class ahead.  A class either runs all K register
// slots or none, so no register row is updated on one path and not on
// another, and the compiler keeps every row in one register.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace cosm {
namespace {

// Pair-slot words: (u row offset | J << kPairJShift, v row offset); row
// offsets are below 2^18 (LDS holds at most 160 KB).
constexpr uint32_t kRowOffsetMask = (1u << 18) - 1u;
constexpr int kPairJShift = 18;

struct RStreamArgs {
  void *phases;
  const uint32_t *words;      // [register classes][K][nth][2]
  const uint32_t *pwords;     // [C][kRStreamPairs][nth][2]
  const uint32_t *act;        // [C][nth / 64] slot masks
  const int32_t *slot_vertex; // [n_rows], -1 for padding rows
  const int32_t *reg_vertex;  // [K][nth], -1 for none
  int32_t R, n_rows, C, n_reg_classes;
  uint32_t words_bytes, pwords_bytes;
  int64_t t0, nsw;
  SweepSchedule sch;
  uint32_t k0, k1, rid0;
};

// Eq. (6) on register row r and LDS row w of one edge.  fm = flip << 31 (the
// register vertex is the edge's v); aJf = alpha_t J, negated when flipped.  The
// difference is taken as x_u - x_v, i.e. (x_r - x_w) with its sign bit
// flipped when r is v (IEEE subtraction is antisymmetric); the register row
// moves by -D and the LDS row by +D, D = +-aJf.  LAZY: no wrap (FP32 phases
// wrapped at the twists only, as in the streamed pair form; the grid schedule,
// so the sweeps run under f32_round_down and the sign comes from the parity of
// floor(2e), the flip folded into the fma's factor -2).
template <int ST, int W, bool LAZY>
__device__ __forceinline__ void update_owner(uint32_t (&r)[W], uint32_t (&w)[W], float aJf,
                                             uint32_t fm, float pm) {
  if constexpr (ST == COSM_STORE_FP32 && LAZY) {
    const float two = __uint_as_float(0x40000000u ^ fm);  // +-2
#pragma unroll
    for (int k = 0; k < W; k++) {
      const float xr = __uint_as_float(r[k]), xw = __uint_as_float(w[k]);
      const float p = __builtin_fmaf(xr - xw, two, pm);
      const float D = __uint_as_float((__float_as_uint(p) << 31) + __float_as_uint(aJf));
      r[k] = __float_as_uint(xr - D);
      w[k] = __float_as_uint(xw + D);
    }
  } else if constexpr (ST == COSM_STORE_FP32) {
#pragma unroll
    for (int k = 0; k < W; k++) {
      const float xr = __uint_as_float(r[k]), xw = __uint_as_float(w[k]);
      const float e = __uint_as_float(__float_as_uint(xr - xw) ^ fm);
      const float D = (fract1(e) < 0.5f) ? aJf : -aJf;
      r[k] = __float_as_uint(fract1(xr - D));
      w[k] = __float_as_uint(fract1(xw + D));
    }
  } else {
    static_assert(!LAZY, "the lazy wrap is an FP32 form");
    update_reg_words<ST, W>(r, w, __uint_as_float(__float_as_uint(aJf) ^ fm), fm >> 31);
  }
}

template <int ST, int W, bool LAZY>
__device__ __forceinline__ void update_pair(uint32_t (&u)[W], uint32_t (&v)[W], float aJ,
                                            float pm) {
  if constexpr (LAZY) {
#pragma unroll
    for (int k = 0; k < W; k++) {
      const float xu = __uint_as_float(u[k]), xv = __uint_as_float(v[k]);
      const float dl = step_by_parity(xu - xv, aJ, pm);
      u[k] = __float_as_uint(xu - dl);
      v[k] = __float_as_uint(xv + dl);
    }
  } else {
    update_words<ST, W>(u, v, aJ);
  }
}

// A register slot in flight: the LDS row, its address, the flip mask and step.
template <int W>
struct RSlot {
  uint32_t w[W];
  uint32_t off, fm;
  float aJ;
};
// A pair slot in flight.
template <int W>
struct PSlot {
  uint32_t u[W], v[W];
  uint32_t ou, ov;
  float aJ;
};

template <int ST, int W, int K, bool LAZY>
__global__ void __launch_bounds__(1024) k_sweep_rstream(const RStreamArgs a) {
  static_assert(!LAZY || ST == COSM_STORE_FP32, "the lazy wrap is an FP32 form");
  constexpr int P = kRStreamPairs;
  extern __shared__ uint32_t lds[];
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nw = nth >> 6;
  const int32_t r0 = xcd_block(blockIdx.x, gridDim.x) * RW;
  const int32_t nvalid = min(RW, a.R - r0);

  // HBM [n][R] -> LDS rows (padding rows and dummy rows zero)
  for (int s = tid; s < a.n_rows + kDummyRows; s += nth) {
    const int32_t v = s < a.n_rows ? a.slot_vertex[s] : -1;
    float x[RW];
#pragma unroll
    for (int k = 0; k < RW; k++)
      x[k] = (v >= 0 && k < nvalid) ? F::load_elem(a.phases, (size_t)v * a.R + r0 + k) : 0.0f;
    uint32_t w[W];
    F::template pack<W>(x, w);
    lds_store<W>(lds, s, w);
  }
  // the twist angles of kThetaChunk twists (no bias fields: no direction
  // table), then the slot masks
  float *theta_buf = reinterpret_cast<float *>(lds + (size_t)(a.n_rows + kDummyRows) * W);
  uint32_t *act = reinterpret_cast<uint32_t *>(theta_buf + kThetaChunk * RW);  // [C][nw]
  for (int i = tid; i < a.C * nw; i += nth) act[i] = a.act[i];
  // HBM -> register rows
  uint32_t own[K][W];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int32_t v = a.reg_vertex[k * nth + tid];
    float x[RW];
#pragma unroll
    for (int q = 0; q < RW; q++)
      x[q] = (v >= 0 && q < nvalid) ? F::load_elem(a.phases, (size_t)v * a.R + r0 + q) : 0.0f;
    F::template pack<W>(x, own[k]);
  }

  // schedule words: lane offset fixed, slot offset a scalar
  const __amdgpu_buffer_rsrc_t rw =
      __builtin_amdgcn_make_buffer_rsrc((void *)a.words, (short)0, (int)a.words_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rp =
      __builtin_amdgcn_make_buffer_rsrc((void *)a.pwords, (short)0, (int)a.pwords_bytes, 0x00020000);
  const uint32_t lane8 = (uint32_t)tid * 8u;
  const uint32_t stride8 = (uint32_t)nth * 8u;
  auto word = [&](uint32_t c, int k) -> su2 {
    return __builtin_amdgcn_raw_buffer_load_b64(
        rw, lane8, __builtin_amdgcn_readfirstlane((c * K + (uint32_t)k) * stride8), 0);
  };
  auto pword = [&](uint32_t c, int p) -> su2 {
    return __builtin_amdgcn_raw_buffer_load_b64(
        rp, lane8, __builtin_amdgcn_readfirstlane((c * P + (uint32_t)p) * stride8), 0);
  };
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t C = (uint32_t)a.C;
  __syncthreads();

  // Register-slot words in a ring of kRing: slot k's word sits in wr[k %
  // kRing] and, once decoded, makes room for the word kRing slots on (in this
  // register class or the next; K is a multiple of kRing).  Pair-slot words
  // are fetched one class ahead.
  constexpr int kRing = K % 4 == 0 ? 4 : 5;
  static_assert(K % kRing == 0, "register rows per thread must be a multiple of the ring");
  const uint32_t nreg = (uint32_t)a.n_reg_classes;
  su2 wr[kRing];
  su2 wp[P];
#pragma unroll
  for (int k = 0; k < kRing; k++) wr[k] = word(0u, k);
#pragma unroll
  for (int p = 0; p < P; p++) wp[p] = pword(0u, p);

  SweepSchedule sc = a.sch;
  const uint32_t nsw = (uint32_t)a.nsw;
  uint32_t t = (uint32_t)a.t0;
  uint32_t tw = 0;
  uint32_t j = 0;  // the register class whose words are in the ring
  ScheduleChunk chunk;
  // LAZY (the grid schedule): every operation of the sweeps is exact
  float pm = 0.0f;  // LAZY: 1.5 * 2^23 from the switch, the parity fma's addend
  if constexpr (LAZY) pm = f32_round_down();
  for (uint32_t it = 0; it < nsw; it++) {
    t++;
    if ((it & 63u) == 0u) chunk.fill(sc, t);
    float alpha, twist;
    chunk.get(it & 63u, alpha, twist);
    const float amag = alpha * F::kStepScale;
    const bool twist_now = chunk.twist_at(it & 63u);

    for (uint32_t c = 0; c < C; c++) {
      const uint32_t cn = c + 1 == C ? 0u : c + 1;
      const uint32_t m = __builtin_amdgcn_readfirstlane(act[c * (uint32_t)nw + wave]);
      if (m & 1u) {
        // a register class: all K slots on every wave, the row of slot k + 1
        // read before slot k is computed (all of a class's rows are distinct)
        const uint32_t jn = j + 1 == nreg ? 0u : j + 1;
        RSlot<W> rs[2];
        auto rread = [&](int k) {
          RSlot<W> &x = rs[k & 1];
          const su2 w = wr[k % kRing];
          x.off = w.x & 0x7fffffffu;
          x.fm = w.x & 0x80000000u;
          x.aJ = __uint_as_float(__float_as_uint(amag * __uint_as_float(w.y)) ^ x.fm);
          row_load<W>(x.off, x.w);
          wr[k % kRing] = k + kRing < K ? word(j, k + kRing) : word(jn, k + kRing - K);
        };
        auto rfinish = [&](int k) {
          RSlot<W> &x = rs[k & 1];
          update_owner<ST, W, LAZY>(own[k], x.w, x.aJ, x.fm, pm);
          row_store<W>(x.off, x.w);
        };
        rread(0);
#pragma unroll
        for (int k = 0; k < K; k++) {
          if (k + 1 < K) rread(k + 1);
          rfinish(k);
        }
        j = jn;
      }
      // edges between two LDS rows (a wave runs the slots with an edge)
#pragma unroll
      for (int p = 0; p < P; p++) {
        if ((m >> (1 + p)) & 1u) {
          PSlot<W> x;
          x.ou = wp[p].x & kRowOffsetMask;
          x.ov = wp[p].y & kRowOffsetMask;
          x.aJ = amag * (float)((int32_t)wp[p].x >> kPairJShift);
          row_load<W>(x.ou, x.u);
          row_load<W>(x.ov, x.v);
          update_pair<ST, W, LAZY>(x.u, x.v, x.aJ, pm);
          row_store<W>(x.ou, x.u);
          row_store<W>(x.ov, x.v);
        }
        wp[p] = pword(cn, p);
      }
      __syncthreads();
    }

    // Dual window twist every `period` sweeps, after the last class: the
    // register rows by their owners, the LDS rows by all threads
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
      TwistOps<ST, W> op;
      op.set(cth, tws, sc.win2);
      tw++;
#pragma unroll
      for (int k = 0; k < K; k++) twist_row<ST, W, LAZY>(op, own[k]);
      for (int s0 = tid; s0 < a.n_rows; s0 += 4 * nth) {
        uint32_t w[4][W];
#pragma unroll
        for (int j = 0; j < 4; j++)
          if (s0 + j * nth < a.n_rows) lds_load<W>(lds, s0 + j * nth, w[j]);
#pragma unroll
        for (int j = 0; j < 4; j++) {
          if (s0 + j * nth < a.n_rows) {
            twist_row<ST, W, LAZY>(op, w[j]);
            lds_store<W>(lds, s0 + j * nth, w[j]);
          }
        }
      }
      __syncthreads();
    }
  }
  if constexpr (LAZY) f32_round_nearest();

  // register rows and LDS rows -> HBM
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int32_t v = a.reg_vertex[k * nth + tid];
    if (v < 0) continue;
    float x[RW];
    F::template unpack<W>(own[k], x);
#pragma unroll
    for (int q = 0; q < RW; q++)
      if (q < nvalid) F::store_elem(a.phases, (size_t)v * a.R + r0 + q, LAZY ? fract1(x[q]) : x[q]);
  }
  for (int s = tid; s < a.n_rows; s += nth) {
    const int32_t v = a.slot_vertex[s];
    if (v < 0) continue;
    uint32_t w[W];
    lds_load<W>(lds, s, w);
    float x[RW];
    F::template unpack<W>(w, x);
#pragma unroll
    for (int q = 0; q < RW; q++)
      if (q < nvalid) F::store_elem(a.phases, (size_t)v * a.R + r0 + q, LAZY ? fract1(x[q]) : x[q]);
  }
}

template <int ST, int W, int K, bool LAZY>
int launch_rstream_k(cosm_state *s, const RStreamArgs &a) {
  const size_t lds = s->shape.lds_bytes;
  (void)hipFuncSetAttribute((const void *)k_sweep_rstream<ST, W, K, LAZY>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_sweep_rstream<ST, W, K, LAZY>), dim3(s->shape.blocks),
                     dim3(s->shape.threads), lds, s->stream, a);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    return set_error(COSM_EDEVICE, std::string("k_sweep_rstream: ") + hipGetErrorString(err));
  return COSM_OK;
}

template <int ST, bool LAZY>
int launch_rstream_l(cosm_state *s, const RStreamArgs &a, int W, int K) {
  if (W == 2 && K == 8) return launch_rstream_k<ST, 2, 8, LAZY>(s, a);
  if (W == 2 && K == 10) return launch_rstream_k<ST, 2, 10, LAZY>(s, a);
  if (W == 2 && K == 12) return launch_rstream_k<ST, 2, 12, LAZY>(s, a);
  if (W == 2 && K == 16) return launch_rstream_k<ST, 2, 16, LAZY>(s, a);
  if (W == 4 && K == 8) return launch_rstream_k<ST, 4, 8, LAZY>(s, a);
  return set_error(COSM_EINVAL, "streamed register form: unsupported row width or register count");
}

}  // namespace

bool rstream_shape_supported(int32_t storage, int32_t W, int32_t K) {
  if (storage != COSM_STORE_FP32) return false;
  return (W == 2 && (K == 8 || K == 10 || K == 12 || K == 16)) || (W == 4 && K == 8);
}

int launch_sweeps_rstream(cosm_state *s, int64_t n_sweeps) {
  const LdsSchedule &L = s->lds;
  if (s->p.storage != COSM_STORE_FP32)
    return set_error(COSM_EINVAL, "the streamed register form runs FP32 storage");
  RStreamArgs a{};
  a.phases = s->d.phases;
  a.words = s->d.rs_words;
  a.pwords = s->d.rs_pwords;
  a.act = s->d.rs_act;
  a.slot_vertex = s->d.slot_vertex;
  a.reg_vertex = s->d.reg_vertex;
  a.R = s->R;
  a.n_rows = L.n_rows;
  a.C = s->C;
  a.n_reg_classes = (int32_t)(L.rs_words.size() / ((size_t)2 * L.reg_k * L.nth));
  a.words_bytes = (uint32_t)(L.rs_words.size() * 4);
  a.pwords_bytes = (uint32_t)(L.rs_pwords.size() * 4);
  a.t0 = s->t;
  a.nsw = n_sweeps;
  a.sch = make_sweep_schedule(s->sched, s->t);
  a.k0 = (uint32_t)(s->seed & 0xffffffffu);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.rid0 = (uint32_t)s->rid0;
  const int W = s->shape.rw;  // FP32: one word per replica
  if (lds_lazy_wrap(*s)) return launch_rstream_l<COSM_STORE_FP32, true>(s, a, W, L.reg_k);
  return launch_rstream_l<COSM_STORE_FP32, false>(s, a, W, L.reg_k);
}

}  // namespace cosm
