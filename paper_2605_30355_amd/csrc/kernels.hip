// kernels.hip -- gfx950 kernels of libcosm and their launchers.
//
// Phases are turns (1 turn = 360 degrees).  FP32 storage keeps x in [0, 1) and
// wraps with v_fract_f32; FP16 / BF16 storage keeps the centred value
// y = x - 1/2 in [-1/2, 1/2] and wraps with y - rint(y) (one more bit of
// resolution than storing x); arithmetic is FP32 (FP16_PK: FP16, packed).
// When no phase can drift by 1/2 turn between two twists, the 16-bit float
// formats (every form) and FP32 (the
// streamed LDS forms, grid schedule) wrap at the twists only (lazy16,
// lds_lazy_wrap).  FIX16 storage keeps x as a
// 16-bit integer k (x = k 2^-16) and the LDS sweep updates it with packed
// 16-bit integer ops (other forms go through FP32, exact on that grid).  On
// the 2^-23 turn grid (2^-16 for FIX16) every add, subtract, fma by 2 and
// fract below is exact, so grid-schedule trajectories are bit-exact.
//
// The pair update of Eq. (6), with the biased sign of Eq. (4) taken on the
// minimum angular difference:  f = fract(x_u - x_v); s = +1 iff f < 1/2;
// delta = alpha_t * J * s; x_u <- wrap(x_u - delta); x_v <- wrap(x_v + delta).
// (fract(d) < 1/2 is exactly "the difference wrapped to [-1/2, 1/2) is >= 0".)
// On the grid schedule the FP32 sweeps (RD instantiations) take s from the
// parity of floor(2(x_u - x_v)) under round-toward-minus-infinity instead
// (step_by_parity): the same decision for every input, in fewer instructions.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"
#include "lds_args.hpp"

namespace cosm {
namespace {


// ---------------------------------------------------------------------------
// Phase initialisation, Algorithm 1 "Set x_i random".
// ---------------------------------------------------------------------------
template <int ST>
__global__ void __launch_bounds__(256) k_init(void *phases, int32_t n, int32_t R, uint32_t k0,
                                              uint32_t k1, uint32_t rid0, uint32_t shift,
                                              float scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * R) return;
  const int32_t i = (int32_t)(idx / R), r = (int32_t)(idx % R);
  const uint32_t w = philox_first_word((uint32_t)i, 0u, rid0 + (uint32_t)r, kTagInit, k0, k1);
  const float x = (float)(w >> shift) * scale;  // the top 32 - shift bits
  Fmt<ST>::store_elem(phases, (size_t)idx, Fmt<ST>::from_turn(x));
}

// ---------------------------------------------------------------------------
// The batched LDS-resident sweep: one workgroup owns RW = W * kPerWord whole
// replicas, stored as LDS rows of W 32-bit words (one row per slot), and runs
// every sweep of the call with workgroup barriers only.  Thread t handles the
// t-th entry of each slot of the lane schedule (consecutive lanes touch rows in
// distinct LDS bank groups).  EMAX > 0: the schedule (at most EMAX slots) is
// loaded into registers once; EMAX == 0: it streams from memory, one slot ahead.
// EXACT: one slot per class (EMAX of them), no bounds checks.  FUSE (EXACT or
// streamed, no bias fields): the twist runs inside the last class's sub-sweep.
// ---------------------------------------------------------------------------
template <int ST, int W, int EMAX, bool EXACT, bool FUSE, bool LAZY, bool RD>
__global__ void __launch_bounds__(1024) k_sweep_lds(const LdsArgs a) {
  static_assert(!LAZY || lazy_storage(ST), "the lazy wrap is a floating-point form");
  static_assert(!RD || ST == COSM_STORE_FP32, "the parity step is an FP32 grid form");
  static_assert(!FUSE || EXACT || EMAX == 0,
                "the fused twist runs in the one-slot-per-class and the streamed forms");
  extern __shared__ uint32_t lds[];
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  constexpr uint32_t ROWB = 4 * W;
  const int tid = threadIdx.x, nth = blockDim.x;
  // Workgroups go to the 8 XCDs round-robin; give each XCD a contiguous range
  // of replica blocks so that the workgroups sharing a cache line of a vertex
  // row ([n][R] layout) share one L2.
  const int32_t r0 = xcd_block(blockIdx.x, gridDim.x) * RW;
  const int32_t nvalid = min(RW, a.R - r0);

  // HBM [n][R] -> LDS rows
  for (int s = tid; s < a.n_rows; s += nth) {
    const size_t base = (size_t)a.slot_vertex[s] * a.R + r0;
    float v[RW];
#pragma unroll
    for (int k = 0; k < RW; k++) v[k] = (k < nvalid) ? F::load_elem(a.phases, base + k) : 0.0f;
    uint32_t w[W];
    F::template pack<W>(v, w);
    lds_store<W>(lds, s, w);
  }

  // dummy rows for masked lanes (zero, never stored back), the table of
  // reference angles (filled at the first twist of every chunk), then the slots
  // per class
  for (int s = tid; s < kDummyRows; s += nth) {
    const uint32_t z[W] = {};
    lds_store<W>(lds, a.n_rows + s, z);
  }
  float *theta_buf = reinterpret_cast<float *>(lds + (size_t)(a.n_rows + kDummyRows) * W);  // [kThetaChunk][RW]
  float *dir_buf = theta_buf + kThetaFloats;                                  // [kThetaChunk][RW]
  int32_t *Ks = reinterpret_cast<int32_t *>(dir_buf + kThetaFloats);          // [C]
  if constexpr (EMAX == 0)
    for (int c = tid; c < a.C; c += nth) Ks[c] = a.Kc[c];
  uint32_t tw = 0;  // twists done in this call

  // register-resident lane schedule; a masked lane updates two dummy rows
  // with J = 0 (a no-op), so the slots need no branches
  uint32_t ua[EMAX > 0 ? EMAX : 1], va[EMAX > 0 ? EMAX : 1];
  float jr[EMAX > 0 ? EMAX : 1];
  if constexpr (EMAX > 0) {
    const uint32_t du = (uint32_t)(a.n_rows + (tid & 31)) * ROWB;
    const uint32_t dv = (uint32_t)(a.n_rows + 32 + (tid & 31)) * ROWB;
#pragma unroll
    for (int j = 0; j < EMAX; j++) {
      EdgeDesc d{kEmptySlot, 0.0f};
      if (EXACT || j < a.total_slots) d = a.desc[(size_t)j * nth + tid];
      const bool empty = d.slots == kEmptySlot;
      ua[j] = empty ? du : (d.slots & 0xffffu) * ROWB;
      va[j] = empty ? dv : (d.slots >> 16) * ROWB;
      jr[j] = empty ? 0.0f : d.J;
    }
  }
  // rows outside the last class (twist only)
  uint32_t fr[FUSE && EXACT ? kFuseRowsMax : 1];
  if constexpr (FUSE && EXACT) {
#pragma unroll
    for (int q = 0; q < kFuseRowsMax; q++) {
      fr[q] = kEmptySlot;
      if (q < a.fuse_k) {
        const uint32_t sl = a.desc[(size_t)(a.total_slots + kStreamRepeat + q) * nth + tid].slots;
        if (sl != kEmptySlot) fr[q] = sl * ROWB;
      }
    }
  }
  // streamed schedule: the first two slots in flight
  EdgeDesc dA{kEmptySlot, 0.0f}, dB{kEmptySlot, 0.0f};
  int jslot = 0;
  if (EMAX == 0 && a.total_slots > 0) {
    dA = a.desc[tid];
    dB = a.desc[(size_t)(1 % a.total_slots) * nth + tid];
  }
  __syncthreads();

  SweepSchedule sc = a.sch;
  // 32-bit sweep counters (at most 2^31 sweeps)
  const uint32_t nsw = (uint32_t)a.nsw;
  uint32_t t = (uint32_t)a.t0;
  ScheduleChunk chunk;
  // RD: the grid schedule, on which every operation of the sweeps is exact
  // (the ramp, the twist angles and offsets, the updates and wraps), so the
  // rounding mode matters only to the step's parity fma
  float pm = 0.0f;  // RD: 1.5 * 2^23 from the switch, the parity fma's addend
  if constexpr (RD) pm = f32_round_down();
  for (uint32_t it = 0; it < nsw; it++) {
    t++;
    if ((it & 63u) == 0u) chunk.fill(sc, t);
    float alpha, twist;
    chunk.get(it & 63u, alpha, twist);
    const float alpha_s = alpha * F::kStepScale;  // the step in storage units
    // Sequential conflict-free search: classes in order, a barrier after each.
    if constexpr (FUSE && EXACT) {
      // EMAX slots, one class each.  On a twist sweep the last class twists
      // the rows it updates and, concurrently, the rows it leaves out.
      const bool fuse_now = chunk.twist_at(it & 63u);
      TwistOps<ST, W> op;
      if (fuse_now) {
        const int slot = (int)(tw % (uint32_t)kThetaChunk);
        tw++;
        if (slot == 0) {
          theta_fill(theta_buf, nullptr, kThetaChunk, RW, t, sc.period, a.rid0 + (uint32_t)r0,
                     a.k0, a.k1, sc.win, sc.tshift, sc.tscale);
          __syncthreads();
        }
        float cth[RW], tws[RW];
#pragma unroll
        for (int k = 0; k < RW; k++) {
          cth[k] = theta_buf[slot * RW + k];
          tws[k] = twist;
        }
        op.set(cth, tws, sc.win2);
      }
#pragma unroll
      for (int j = 0; j < EMAX - 1; j++) {
        edge_rows<ST, W, LAZY, RD>(lds, ua[j], va[j], alpha_s * jr[j], pm);
        __syncthreads();
      }
      if (fuse_now) {
        edge_rows_twist<ST, W, LAZY, RD>(lds, ua[EMAX - 1], va[EMAX - 1], alpha_s * jr[EMAX - 1],
                                         op, pm);
#pragma unroll
        for (int q = 0; q < kFuseRowsMax; q++)
          if (q < a.fuse_k && fr[q] != kEmptySlot) row_twist<ST, W, LAZY>(lds, fr[q], op);
      } else {
        edge_rows<ST, W, LAZY, RD>(lds, ua[EMAX - 1], va[EMAX - 1], alpha_s * jr[EMAX - 1], pm);
      }
      __syncthreads();
    } else if constexpr (EXACT) {
      // EMAX slots, one class each
#pragma unroll
      for (int j = 0; j < EMAX; j++) {
        edge_rows<ST, W, LAZY, RD>(lds, ua[j], va[j], alpha_s * jr[j], pm);
        __syncthreads();
      }
    } else if constexpr (EMAX > 0) {
#pragma unroll
      for (int j = 0; j < EMAX; j++) {
        if (j < a.total_slots) {
          edge_rows<ST, W, LAZY, RD>(lds, ua[j], va[j], alpha_s * jr[j], pm);
          if ((a.bar_mask >> j) & 1u) __syncthreads();
        }
      }
    } else if (a.total_slots > 0) {
      auto edge = [&](const EdgeDesc &d) {
        edge_rows<ST, W, LAZY, RD>(lds, (d.slots & 0xffffu) * ROWB, (d.slots >> 16) * ROWB,
                                   alpha_s * d.J, pm);
      };
      if constexpr (FUSE) {
        // streamed form: on a twist sweep the last class twists the rows it
        // updates, then each thread twists its fuse_k rows outside that class
        const bool fuse_now = chunk.twist_at(it & 63u);
        TwistOps<ST, W> op;
        if (fuse_now) {
          const int slot = (int)(tw % (uint32_t)kThetaChunk);
          tw++;
          if (slot == 0) {
            theta_fill(theta_buf, nullptr, kThetaChunk, RW, t, sc.period, a.rid0 + (uint32_t)r0,
                       a.k0, a.k1, sc.win, sc.tshift, sc.tscale);
            __syncthreads();
          }
          float cth[RW], tws[RW];
#pragma unroll
          for (int k = 0; k < RW; k++) {
            cth[k] = theta_buf[slot * RW + k];
            tws[k] = twist;
          }
          op.set(cth, tws, sc.win2);
        }
        const gptr<EdgeDesc> rest =
            as_global(a.desc) + (size_t)(a.total_slots + kStreamRepeat) * nth + tid;
        stream_classes(
            a.desc, Ks, a.C, a.total_slots, dA, dB, jslot, edge,
            [&](const EdgeDesc &d) {
              edge_rows_twist<ST, W, LAZY, RD>(lds, (d.slots & 0xffffu) * ROWB,
                                               (d.slots >> 16) * ROWB, alpha_s * d.J, op, pm);
            },
            [&] {
              for (int q = 0; q < a.fuse_k; q++) {
                const uint32_t row = rest[(size_t)q * nth].slots;
                if (row != kEmptySlot) row_twist<ST, W, LAZY>(lds, row * ROWB, op);
              }
            },
            fuse_now);
      } else {
        stream_classes(a.desc, Ks, a.C, a.total_slots, dA, dB, jslot, edge);
      }
    }
    // Bias fields: one more conflict-free sub-sweep against the virtual spin
    // at phase 0, after the classes (rows are final after the last barrier).
    if (!FUSE && a.h_slot != nullptr) {
      for (int s0 = tid; s0 < a.n_rows; s0 += 4 * nth) {
        int32_t hv[4];
        uint32_t w[4][W];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          hv[q] = s0 + q * nth < a.n_rows ? a.h_slot[s0 + q * nth] : 0;
          if (hv[q] != 0) lds_load<W>(lds, s0 + q * nth, w[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
          if (hv[q] != 0) {
            float v[RW];
            F::template unpack<W>(w[q], v);
            const float ah = alpha * (float)hv[q];
#pragma unroll
            for (int k = 0; k < RW; k++) field_update<ST, LAZY>(v[k], ah);
            F::template pack<W>(v, w[q]);
            lds_store<W>(lds, s0 + q * nth, w[q]);
          }
        }
      }
      __syncthreads();
    }
    // Dual window twist every `period` sweeps, on the phases after the last
    // class (a barrier ended it).  Reference angles (and, with bias fields,
    // directions) come from the LDS tables, refilled by the whole workgroup
    // every kThetaChunk twists.
    if constexpr (FUSE) {
      // the twist ran inside the last class
    } else if (chunk.twist_at(it & 63u)) {
      const int slot = (int)(tw % (uint32_t)kThetaChunk);
      if (slot == 0) {
        theta_fill(theta_buf, a.h_slot != nullptr ? dir_buf : nullptr, kThetaChunk, RW, t,
                   sc.period, a.rid0 + (uint32_t)r0, a.k0, a.k1, sc.win, sc.tshift, sc.tscale);
        __syncthreads();
      }
      tw++;
      float cth[RW], tws[RW];
#pragma unroll
      for (int k = 0; k < RW; k++) {
        cth[k] = theta_buf[slot * RW + k];
        tws[k] = a.h_slot != nullptr ? dir_buf[slot * RW + k] * twist : twist;
      }
      TwistOps<ST, W> op;
      op.set(cth, tws, sc.win2);
      // four rows per thread in flight: all loads, then the updates and stores
      for (int s0 = tid; s0 < a.n_rows; s0 += 4 * nth) {
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
  if constexpr (RD) f32_round_nearest();

  // LDS rows -> HBM.  16-bit float phases wrapped at the twists only go back
  // as they are (|y| < 1, within the drift bound): wrapping them here would
  // change how later steps round them, and with it the trajectory whenever a
  // trial is split over several calls
  for (int s = tid; s < a.n_rows; s += nth) {
    const size_t base = (size_t)a.slot_vertex[s] * a.R + r0;
    uint32_t w[W];
    lds_load<W>(lds, s, w);
    float v[RW];
    F::template unpack<W>(w, v);
#pragma unroll
    for (int k = 0; k < RW; k++)
      if (k < nvalid) F::store_elem(a.phases, base + k, v[k]);
  }
}

// ---------------------------------------------------------------------------
// VEC consecutive replicas of one vertex row in one access (8 or 16 bytes for
// FP32 and FIX32, 4 or 8 for the 16-bit formats); idx is a multiple of VEC.
typedef float hbm_f32x2 __attribute__((ext_vector_type(2)));
typedef float hbm_f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t hbm_u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t hbm_u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
using gvec = T __attribute__((address_space(1))) *;

template <int ST, int VEC>
__device__ __forceinline__ void load_vec(const void *p, size_t idx, float (&x)[VEC]) {
  using F = Fmt<ST>;
  if constexpr (VEC == 1) {
    x[0] = F::load_elem(p, idx);
  } else if constexpr (ST == COSM_STORE_FP32) {
    const float *q = static_cast<const float *>(p) + idx;
    if constexpr (VEC == 4) {
      const hbm_f32x4 v = *(gvec<const hbm_f32x4>)(q);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
      const hbm_f32x2 v = *(gvec<const hbm_f32x2>)(q);
      x[0] = v.x; x[1] = v.y;
    }
  } else if constexpr (ST == COSM_STORE_FIX32) {
    const uint32_t *q = static_cast<const uint32_t *>(p) + idx;
    if constexpr (VEC == 4) {
      const hbm_u32x4 v = *(gvec<const hbm_u32x4>)(q);
      x[0] = F::dec(v.x); x[1] = F::dec(v.y); x[2] = F::dec(v.z); x[3] = F::dec(v.w);
    } else {
      const hbm_u32x2 v = *(gvec<const hbm_u32x2>)(q);
      x[0] = F::dec(v.x); x[1] = F::dec(v.y);
    }
  } else {
    const uint16_t *q = static_cast<const uint16_t *>(p) + idx;
    if constexpr (VEC == 4) {
      const hbm_u32x2 v = *(gvec<const hbm_u32x2>)(q);
      x[0] = F::dec(v.x & 0xffffu); x[1] = F::dec(v.x >> 16);
      x[2] = F::dec(v.y & 0xffffu); x[3] = F::dec(v.y >> 16);
    } else {
      const uint32_t v = *(gvec<const uint32_t>)(q);
      x[0] = F::dec(v & 0xffffu); x[1] = F::dec(v >> 16);
    }
  }
}
template <int ST, int VEC>
__device__ __forceinline__ void store_vec(void *p, size_t idx, const float (&x)[VEC]) {
  using F = Fmt<ST>;
  if constexpr (VEC == 1) {
    F::store_elem(p, idx, x[0]);
  } else if constexpr (ST == COSM_STORE_FP32) {
    float *q = static_cast<float *>(p) + idx;
    if constexpr (VEC == 4) {
      *(gvec<hbm_f32x4>)(q) = hbm_f32x4{x[0], x[1], x[2], x[3]};
    } else {
      *(gvec<hbm_f32x2>)(q) = hbm_f32x2{x[0], x[1]};
    }
  } else if constexpr (ST == COSM_STORE_FIX32) {
    uint32_t *q = static_cast<uint32_t *>(p) + idx;
    if constexpr (VEC == 4) {
      *(gvec<hbm_u32x4>)(q) = hbm_u32x4{F::enc(x[0]), F::enc(x[1]), F::enc(x[2]), F::enc(x[3])};
    } else {
      *(gvec<hbm_u32x2>)(q) = hbm_u32x2{F::enc(x[0]), F::enc(x[1])};
    }
  } else {
    uint16_t *q = static_cast<uint16_t *>(p) + idx;
    if constexpr (VEC == 4) {
      *(gvec<hbm_u32x2>)(q) = hbm_u32x2{F::enc(x[0]) | (F::enc(x[1]) << 16),
                                        F::enc(x[2]) | (F::enc(x[3]) << 16)};
    } else {
      *(gvec<uint32_t>)(q) = F::enc(x[0]) | (F::enc(x[1]) << 16);
    }
  }
}

// ---------------------------------------------------------------------------
// Device-memory forms: one launch per colour class.  HBM form: a wave covers
// 64 VEC consecutive replicas of one edge (coalesced rows of the [n][R]
// layout, VEC per lane).  PLAIN form: one replica, a thread per edge.
// ---------------------------------------------------------------------------
template <int ST, int VEC>
__global__ void __launch_bounds__(256) k_class_hbm(void *phases, const int32_t *peu,
                                                   const int32_t *pev, const float *pJ,
                                                   int32_t beg, int32_t cnt, int32_t R,
                                                   int32_t rchunks, float alpha, int32_t lazy) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t e = wave / rchunks;
  const int32_t r = ((int32_t)(wave % rchunks) * 64 + lane) * VEC;
  if (e >= cnt || r >= R) return;
  const int32_t u = peu[beg + e], v = pev[beg + e];
  const float aJ = alpha * pJ[beg + e];
  float xu[VEC], xv[VEC];
  load_vec<ST, VEC>(phases, (size_t)u * R + r, xu);
  load_vec<ST, VEC>(phases, (size_t)v * R + r, xv);
  // (lazy: 16-bit float phases wrapped at the twists only)
  if (lazy) {
#pragma unroll
    for (int k = 0; k < VEC; k++) pair_update<ST, true>(xu[k], xv[k], aJ);
  } else {
#pragma unroll
    for (int k = 0; k < VEC; k++) pair_update<ST>(xu[k], xv[k], aJ);
  }
  store_vec<ST, VEC>(phases, (size_t)u * R + r, xu);
  store_vec<ST, VEC>(phases, (size_t)v * R + r, xv);
}

// Twist for replicas [rbeg, rbeg + rcount): thread = VEC replicas x a strip of
// `strip` vertices, so the reference angles are drawn once per strip.
template <int ST, int VEC>
__global__ void __launch_bounds__(256) k_dwt_hbm(void *phases, int32_t n, int32_t R, int32_t rbeg,
                                                 int32_t rcount, int32_t strip, uint32_t t,
                                                 float twist, float win, float win2, uint32_t k0,
                                                 uint32_t k1, uint32_t rid0, int32_t drawn_dir,
                                                 uint32_t tshift, float tscale, int32_t lazy) {
  using F = Fmt<ST>;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t rchunks = (rcount + 64 * VEC - 1) / (64 * VEC);
  const int64_t wave = g >> 6;
  const int lane = threadIdx.x & 63;
  const int32_t rloc = ((int32_t)(wave % rchunks) * 64 + lane) * VEC;
  const int64_t i0 = (wave / rchunks) * strip;
  if (rloc >= rcount || i0 >= n) return;
  const int32_t r = rbeg + rloc;
  float c[VEC], tw[VEC];
#pragma unroll
  for (int k = 0; k < VEC; k++) {
    const uint2 wd = philox_words01(0u, t, rid0 + (uint32_t)(r + k), kTagDwt, k0, k1);
    c[k] = 2.0f * ((float)(wd.x >> tshift) * tscale) - win;
    tw[k] = (drawn_dir && (wd.y >> 31)) ? -twist : twist;  // with bias fields: drawn direction
  }
  const int64_t i1 = min((int64_t)n, i0 + strip);
  for (int64_t i = i0; i < i1; i++) {
    const size_t idx = (size_t)i * R + r;
    float v[VEC];
    load_vec<ST, VEC>(phases, idx, v);
    bool any = lazy != 0;  // lazy: every phase is wrapped here, the twist added unwrapped
#pragma unroll
    for (int k = 0; k < VEC; k++) {
      if (lazy) {
        const float y = F::wrap(v[k]);
        v[k] = in_windows(y, c[k], win2) ? y + tw[k] : y;
      } else if (in_windows(v[k], c[k], win2)) {
        v[k] = F::wrap(v[k] + tw[k]);
        any = true;
      }
    }
    if (any) store_vec<ST, VEC>(phases, idx, v);
  }
}

// Bias-field sub-sweep for replicas [rbeg, rbeg + rcount) of the [n][R] array.
template <int ST>
__global__ void __launch_bounds__(256) k_field_hbm(void *phases, const int32_t *h, int32_t n,
                                                   int32_t R, int32_t rbeg, int32_t rcount,
                                                   float alpha, int32_t lazy) {
  using F = Fmt<ST>;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * rcount) return;
  const int32_t i = (int32_t)(g / rcount), r = rbeg + (int32_t)(g % rcount);
  const int32_t hv = h[i];
  if (hv == 0) return;
  const size_t idx = (size_t)i * R + r;
  float v = F::load_elem(phases, idx);
  if (lazy) field_update<ST, true>(v, alpha * (float)hv);
  else field_update<ST>(v, alpha * (float)hv);
  F::store_elem(phases, idx, v);
}

template <int ST>
__global__ void __launch_bounds__(256) k_class_plain(void *phases, const int32_t *peu,
                                                     const int32_t *pev, const float *pJ,
                                                     int32_t beg, int32_t cnt, int32_t R,
                                                     int32_t r, float alpha, int32_t lazy) {
  using F = Fmt<ST>;
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const int32_t u = peu[beg + e], v = pev[beg + e];
  const float aJ = alpha * pJ[beg + e];
  float xu = F::load_elem(phases, (size_t)u * R + r);
  float xv = F::load_elem(phases, (size_t)v * R + r);
  if (lazy) pair_update<ST, true>(xu, xv, aJ);
  else pair_update<ST>(xu, xv, aJ);
  F::store_elem(phases, (size_t)u * R + r, xu);
  F::store_elem(phases, (size_t)v * R + r, xv);
}

// Full-gradient update of Eq. (8) (the "without SCS" ablation): every edge
// reads the same state x_t; vertex i sums its incident contributions in CSR
// order and writes x_{t+1} to the other buffer.  inc_nbr holds the neighbour j
// with bit 31 set when i is the edge's first endpoint u; the sign decision
// always uses x_u - x_v of the edge's own orientation.
template <int ST>
__global__ void __launch_bounds__(256) k_full_gradient(const void *src, void *dst,
                                                       const int32_t *inc_off,
                                                       const uint32_t *inc_nbr,
                                                       const float *inc_J, const int32_t *h,
                                                       int32_t n, int32_t R, float alpha) {
  using F = Fmt<ST>;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * R) return;
  const int32_t i = (int32_t)(idx / R), r = (int32_t)(idx % R);
  const float xi = F::load_elem(src, (size_t)idx);
  float acc = 0.0f;
  for (int32_t a = inc_off[i]; a < inc_off[i + 1]; a++) {
    const uint32_t code = inc_nbr[a];
    const bool i_first = (code >> 31) != 0;
    const int32_t j = (int32_t)(code & 0x7fffffffu);
    const float xj = F::load_elem(src, (size_t)j * R + r);
    const float f = fract1(i_first ? xi - xj : xj - xi);
    const float aJs = (f < 0.5f) ? alpha * inc_J[a] : -alpha * inc_J[a];
    acc += i_first ? -aJs : aJs;
  }
  if (h != nullptr && h[i] != 0) {  // the virtual spin at phase 0 (bias field)
    const float ah = alpha * (float)h[i];
    acc += fract1(F::to_turn(xi)) < 0.5f ? -ah : ah;
  }
  F::store_elem(dst, (size_t)idx, F::wrap(xi + acc));
}


template <int ST>
__global__ void __launch_bounds__(256) k_readout(const ReadoutArgs a) {
  extern __shared__ int64_t sm64[];
  // one replica per workgroup; replicas sharing a cache line on one XCD
  readout_block<ST>(a, xcd_block(blockIdx.x, gridDim.x), sm64);
}

// Energy (Eq. (1)) and cut (Eq. (14), w = -J) of caller-supplied spins [R][n].
__global__ void __launch_bounds__(256) k_energy(const int8_t *spins, const int32_t *eu,
                                                const int32_t *ev, const int32_t *J,
                                                const int32_t *h, int32_t n, int64_t m,
                                                int64_t *H, int64_t *cut) {
  __shared__ int64_t red[16];
  const int r = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
  const int8_t *s = spins + (size_t)r * n;
  int64_t e = 0, c = 0;
  for (int64_t k = tid; k < m; k += nth) {
    const int su = s[eu[k]], sv = s[ev[k]];
    e -= (int64_t)J[k] * su * sv;
    if (su != sv) c -= J[k];
  }
  if (h != nullptr)
    for (int i = tid; i < n; i += nth) e -= (int64_t)h[i] * s[i];
  e = block_sum(e, red);
  c = block_sum(c, red);
  if (tid == 0) {
    H[r] = e;
    cut[r] = c;
  }
}

template <int ST>
__global__ void __launch_bounds__(256) k_to_turns(const void *phases, float *out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = Fmt<ST>::to_turn(Fmt<ST>::load_elem(phases, (size_t)i));
}

template <int ST>
__global__ void __launch_bounds__(256) k_from_turns(void *phases, const float *in, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) Fmt<ST>::store_elem(phases, (size_t)i, Fmt<ST>::from_turn(in[i]));
}

// ---------------------------------------------------------------------------
// Host-side helpers.
// ---------------------------------------------------------------------------
int launch_check(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    return set_error(COSM_EDEVICE, std::string(what) + ": " + hipGetErrorString(err));
  return COSM_OK;
}

// Step size of sweep t (1-based) in turns, exactly as the device evaluates it.
float host_alpha(const Schedule &sc, int64_t t) {
  if (sc.grid) {
    const int64_t q = (sc.a0_units * (sc.S - t + 1) + sc.S / 2) / sc.S;
    return (float)q * sc.aunit;
  }
  return (float)(sc.S - t + 1) * (sc.alpha0_turns / (float)sc.S);
}

float host_twist(const Schedule &sc, int64_t t) {
  if (sc.grid) {
    const int64_t q = (sc.a0_units * (sc.S - t + 1) + sc.S / 2) / sc.S;
    return (float)(sc.twist_num2 * q) * sc.tunit;
  }
  return sc.dwt_ratio * host_alpha(sc, t);
}

template <int ST, int W, int EMAX, bool EXACT, bool FUSE, bool LAZY, bool RD = false>
int launch_lds_k(cosm_state *s, const LdsArgs &a) {
  const size_t lds = s->shape.lds_bytes;
  (void)hipFuncSetAttribute((const void *)k_sweep_lds<ST, W, EMAX, EXACT, FUSE, LAZY, RD>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_sweep_lds<ST, W, EMAX, EXACT, FUSE, LAZY, RD>), dim3(s->shape.blocks),
                     dim3(s->shape.threads), lds, s->stream, a);
  return launch_check("k_sweep_lds");
}

// 16-bit float phases are wrapped at the twists only when the drift bound
// holds (lazy16); the other formats here wrap at every update.  FP32 on the
// grid schedule takes the step's sign from the parity form (exact_grid_fp32).
template <int ST, int W, int EMAX, bool EXACT, bool FUSE = false>
int launch_lds(cosm_state *s, const LdsArgs &a) {
  if constexpr (ST == COSM_STORE_FP16 || ST == COSM_STORE_BF16 || ST == COSM_STORE_FP16_PK) {
    if (lazy16(*s)) return launch_lds_k<ST, W, EMAX, EXACT, FUSE, true>(s, a);
  }
  if constexpr (ST == COSM_STORE_FP32) {
    if (exact_grid_fp32(*s)) return launch_lds_k<ST, W, EMAX, EXACT, FUSE, false, true>(s, a);
  }
  return launch_lds_k<ST, W, EMAX, EXACT, FUSE, false>(s, a);
}

template <int ST, int W>
int launch_lds_w(cosm_state *s, const LdsArgs &a) {
  if (s->lds.reg_k > 0) return launch_sweeps_reg(s, a, W);
  const int slots = a.total_slots;
  // one slot per class and exactly 4 / 8 slots: the unconditional form
  const bool one_each = slots == a.C && slots <= 32 && a.bar_mask == (uint32_t)((1ull << slots) - 1);
  const bool fuse = lds_twist_fused(*s);
  if (fuse && one_each && slots == 4) return launch_lds<ST, W, 4, true, true>(s, a);
  if (fuse && one_each && slots == 8) return launch_lds<ST, W, 8, true, true>(s, a);
  if (one_each && slots == 4) return launch_lds<ST, W, 4, true>(s, a);
  if (one_each && slots == 8) return launch_lds<ST, W, 8, true>(s, a);
  if (slots <= 4) return launch_lds<ST, W, 4, false>(s, a);
  if (slots <= 8) return launch_lds<ST, W, 8, false>(s, a);
  if (slots <= 16) return launch_lds<ST, W, 16, false>(s, a);
  if (fuse) return launch_lds<ST, W, 0, false, true>(s, a);
  return launch_lds<ST, W, 0, false>(s, a);
}

template <int ST>
int sweeps_lds_st(cosm_state *s, int64_t n_sweeps) {
  LdsArgs a{};
  a.phases = s->d.phases;
  a.desc = s->d.desc;
  a.Kc = s->d.class_off;
  a.slot_vertex = s->d.slot_vertex;
  a.h_slot = s->has_h ? s->d.h_slot : nullptr;
  a.R = s->R;
  a.n_rows = s->lds.n_rows;
  a.C = s->C;
  a.total_slots = s->lds.total_slots;
  a.t0 = s->t;
  a.nsw = n_sweeps;
  uint32_t mask = 0;
  {
    int j = 0;
    for (int c = 0; c < s->C; c++) {
      j += s->lds.K[(size_t)c];
      if (s->lds.K[(size_t)c] > 0 && j - 1 < 32) mask |= 1u << (j - 1);
    }
  }
  a.bar_mask = mask;
  a.fuse_k = s->lds.fuse_k;
  a.reg_vertex = s->d.reg_vertex;
  a.reg_free = s->lds.reg_free;
  a.sch = make_sweep_schedule(s->sched, s->t);
  a.k0 = (uint32_t)(s->seed & 0xffffffffu);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.rid0 = (uint32_t)s->rid0;
  const int W = s->shape.rw / Fmt<ST>::kPerWord;
  if (W == 4) return launch_lds_w<ST, 4>(s, a);
  if (W == 2) return launch_lds_w<ST, 2>(s, a);
  if (W == 1) return launch_lds_w<ST, 1>(s, a);
  return set_error(COSM_EINVAL, "unsupported replicas per workgroup");
}

// Replicas per lane of the HBM kernels: the widest of 4, 2, 1 that keeps every
// access aligned (R, the first replica and the count all multiples of it).
int hbm_vec(int32_t R, int32_t rbeg, int32_t rcount) {
  for (int v : {4, 2})
    if (R % v == 0 && rbeg % v == 0 && rcount % v == 0) return v;
  return 1;
}

template <int ST, int VEC>
int dwt_hbm_vec(cosm_state *s, int64_t t, int32_t rbeg, int32_t rcount) {
  const Schedule &sc = s->sched;
  const int32_t strip = 64;
  const int32_t rchunks = (rcount + 64 * VEC - 1) / (64 * VEC);
  const int64_t strips = ((int64_t)s->n + strip - 1) / strip;
  const int64_t threads = strips * rchunks * 64;
  const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
  hipLaunchKernelGGL((k_dwt_hbm<ST, VEC>), grid, block, 0, s->stream, s->d.phases, s->n, s->R,
                     rbeg, rcount, strip, (uint32_t)t, host_twist(sc, t), sc.window, sc.window2,
                     (uint32_t)(s->seed & 0xffffffffu), (uint32_t)(s->seed >> 32),
                     (uint32_t)s->rid0, (int32_t)s->has_h, (uint32_t)sc.tshift, sc.tscale,
                     (int32_t)lazy16(*s));
  return launch_check("k_dwt_hbm");
}

template <int ST>
int dwt_hbm_st(cosm_state *s, int64_t t, int32_t rbeg, int32_t rcount) {
  switch (hbm_vec(s->R, rbeg, rcount)) {
    case 4: return dwt_hbm_vec<ST, 4>(s, t, rbeg, rcount);
    case 2: return dwt_hbm_vec<ST, 2>(s, t, rbeg, rcount);
    default: return dwt_hbm_vec<ST, 1>(s, t, rbeg, rcount);
  }
}

template <int ST>
int field_hbm_st(cosm_state *s, float alpha, int32_t rbeg, int32_t rcount) {
  const int64_t threads = (int64_t)s->n * rcount;
  hipLaunchKernelGGL((k_field_hbm<ST>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                     s->stream, s->d.phases, s->d.h, s->n, s->R, rbeg, rcount, alpha,
                     (int32_t)lazy16(*s));
  return launch_check("k_field_hbm");
}

template <int ST, int VEC>
int class_hbm_vec(cosm_state *s, int32_t beg, int32_t cnt, float alpha) {
  const int32_t rchunks = (s->R + 64 * VEC - 1) / (64 * VEC);
  const int64_t threads = (int64_t)cnt * rchunks * 64;
  hipLaunchKernelGGL((k_class_hbm<ST, VEC>), dim3((unsigned)((threads + 255) / 256)), dim3(256),
                     0, s->stream, s->d.phases, s->d.peu, s->d.pev, s->d.pJ, beg, cnt, s->R,
                     rchunks, alpha, (int32_t)lazy16(*s));
  return launch_check("k_class_hbm");
}

template <int ST>
int sweeps_hbm_st(cosm_state *s, int64_t n_sweeps) {
  const Schedule &sc = s->sched;
  const int vec = hbm_vec(s->R, 0, s->R);
  for (int64_t t = s->t + 1; t <= s->t + n_sweeps; t++) {
    const float alpha = host_alpha(sc, t);
    if (s->p.update == COSM_UPDATE_FULL_GRADIENT) {
      const int64_t tot = (int64_t)s->n * s->R;
      hipLaunchKernelGGL((k_full_gradient<ST>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                         s->stream, s->d.phases, s->d.phases_alt, s->d.inc_off, s->d.inc_nbr,
                         s->d.inc_J, s->has_h ? s->d.h : nullptr, s->n, s->R, alpha);
      if (int rc = launch_check("k_full_gradient")) return rc;
      std::swap(s->d.phases, s->d.phases_alt);
    } else {
      for (int c = 0; c < s->C; c++) {
        const int32_t beg = s->class_begin[c], cnt = s->class_sizes[c];
        if (cnt == 0) continue;
        const int rc = vec == 4   ? class_hbm_vec<ST, 4>(s, beg, cnt, alpha)
                       : vec == 2 ? class_hbm_vec<ST, 2>(s, beg, cnt, alpha)
                                  : class_hbm_vec<ST, 1>(s, beg, cnt, alpha);
        if (rc) return rc;
      }
      if (s->has_h)
        if (int rc = field_hbm_st<ST>(s, alpha, 0, s->R)) return rc;
    }
    if (sc.dwt_period > 0 && t % sc.dwt_period == 0)
      if (int rc = dwt_hbm_st<ST>(s, t, 0, s->R)) return rc;
  }
  return COSM_OK;
}

template <int ST>
int sweeps_plain_st(cosm_state *s, int64_t n_sweeps) {
  const Schedule &sc = s->sched;
  for (int32_t r = 0; r < s->R; r++) {
    for (int64_t t = s->t + 1; t <= s->t + n_sweeps; t++) {
      const float alpha = host_alpha(sc, t);
      for (int c = 0; c < s->C; c++) {
        const int32_t beg = s->class_begin[c], cnt = s->class_sizes[c];
        if (cnt == 0) continue;
        hipLaunchKernelGGL((k_class_plain<ST>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                           s->stream, s->d.phases, s->d.peu, s->d.pev, s->d.pJ, beg, cnt, s->R, r,
                           alpha, (int32_t)lazy16(*s));
        if (int rc = launch_check("k_class_plain")) return rc;
      }
      if (s->has_h)
        if (int rc = field_hbm_st<ST>(s, alpha, r, 1)) return rc;
      if (sc.dwt_period > 0 && t % sc.dwt_period == 0)
        if (int rc = dwt_hbm_st<ST>(s, t, r, 1)) return rc;
    }
  }
  return COSM_OK;
}

template <int ST>
int readout_st(cosm_state *s) {
  ReadoutArgs a{};
  a.phases = s->d.phases;
  a.eu = s->d.eu;
  a.ev = s->d.ev;
  a.J = s->d.J;
  a.h = s->has_h ? s->d.h : nullptr;
  a.spins = s->d.spins;
  a.H = s->d.H;
  a.cut = s->d.cut;
  a.best_p = s->d.best_p;
  a.n = s->n;
  a.R = s->R;
  a.B = s->p.n_bisectors;
  a.grid = s->sched.grid;
  a.m = s->m;
  a.code_global = s->d.codes;
  const size_t lds = readout_lds_bytes(a.code_global != nullptr ? 0 : s->n, a.B);
  (void)hipFuncSetAttribute((const void *)k_readout<ST>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  hipLaunchKernelGGL((k_readout<ST>), dim3(s->R), dim3(256), lds, s->stream, a);
  return launch_check("k_readout");
}

template <int ST>
int init_st(cosm_state *s) {
  const int64_t tot = (int64_t)s->n * s->R;
  hipLaunchKernelGGL((k_init<ST>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s->stream,
                     s->d.phases, s->n, s->R, (uint32_t)(s->seed & 0xffffffffu),
                     (uint32_t)(s->seed >> 32), (uint32_t)s->rid0, (uint32_t)s->sched.ishift,
                     s->sched.iscale);
  return launch_check("k_init");
}

template <template <int> class Fn, typename... A>
int dispatch_storage(int storage, A &&...args) {
  switch (storage) {
    case COSM_STORE_FP32: return Fn<COSM_STORE_FP32>::run(args...);
    case COSM_STORE_FP16: return Fn<COSM_STORE_FP16>::run(args...);
    case COSM_STORE_FP16_PK: return Fn<COSM_STORE_FP16_PK>::run(args...);
    case COSM_STORE_BF16: return Fn<COSM_STORE_BF16>::run(args...);
    case COSM_STORE_FIX16: return Fn<COSM_STORE_FIX16>::run(args...);
    case COSM_STORE_FIX32: return Fn<COSM_STORE_FIX32>::run(args...);
  }
  return set_error(COSM_EINVAL, "unknown storage format");
}

template <int ST> struct InitFn { static int run(cosm_state *s) { return init_st<ST>(s); } };
template <int ST> struct ToTurnsFn {
  static int run(cosm_state *s, float *out) {
    const int64_t cnt = (int64_t)s->n * s->R;
    hipLaunchKernelGGL((k_to_turns<ST>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       s->stream, s->d.phases, out, cnt);
    return launch_check("k_to_turns");
  }
};
template <int ST> struct FromTurnsFn {
  static int run(cosm_state *s, const float *in) {
    const int64_t cnt = (int64_t)s->n * s->R;
    hipLaunchKernelGGL((k_from_turns<ST>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       s->stream, s->d.phases, in, cnt);
    return launch_check("k_from_turns");
  }
};
template <int ST> struct ReadoutFn { static int run(cosm_state *s) { return readout_st<ST>(s); } };
template <int ST> struct SweepFn {
  static int run(cosm_state *s, int64_t n) {
    switch (s->shape.residency) {
      case COSM_RES_LDS:
        if (s->lds.stream) return launch_sweeps_stream(s, n);
        if (s->lds.rstream) return launch_sweeps_rstream(s, n);
        return sweeps_lds_st<ST>(s, n);
      case COSM_RES_HBM: return sweeps_hbm_st<ST>(s, n);
      case COSM_RES_PLAIN: return sweeps_plain_st<ST>(s, n);
    }
    return set_error(COSM_EINVAL, "unknown residency");
  }
};

}  // namespace

// The fused twist exists in the register form with exactly 4 classes and in
// the pair form's one-slot-per-class (4 or 8 classes) and streamed schedules;
// it needs a twist period, no bias-field pass after the classes, and a
// schedule that lists the rows outside the last class (lds.fuse).
bool lds_twist_fused(const cosm_state &s) {
  if (s.shape.residency != COSM_RES_LDS || s.sched.dwt_period <= 0 || !s.lds.fuse) return false;
  // (the streamed word form runs its twist as a pass: measured faster than
  // the fused twist there, whose extra arithmetic lengthens the last class)
  if (s.lds.stream) return false;
  if (s.lds.reg_k > 0) return s.C == 4;
  if (s.has_h) return false;
  const int slots = s.lds.total_slots;
  bool one_each = slots == s.C;
  for (int32_t k : s.lds.K) one_each = one_each && k == 1;
  if (one_each && (slots == 4 || slots == 8)) return true;
  return slots > kRegisterSlotsMax;
}

double wrap_drift_turns(const cosm_state &s) {
  // the largest step and the largest twist in turns (grid: exact products of
  // small integers and powers of two), then the largest drift of one phase
  // from its wrapped range between two twists: the twist left unwrapped plus
  // every step of `period` sweeps, J and h alike
  const Schedule &sc = s.sched;
  const double alpha_max = sc.grid ? (double)sc.a0_units * (double)sc.aunit : (double)sc.alpha0_turns;
  const double twist_max = sc.grid ? (double)sc.twist_num2 * (double)sc.a0_units * (double)sc.tunit
                                   : (double)sc.dwt_ratio * alpha_max;
  return twist_max + (double)sc.dwt_period * alpha_max * (double)s.wdeg_max;
}

bool exact_grid_fp32(const cosm_state &s) {
  return s.p.storage == COSM_STORE_FP32 && s.sched.grid && s.p.update == COSM_UPDATE_SCS;
}

bool grid_parity_step(const cosm_state &s) {
  const int32_t st = s.p.storage;
  return (st == COSM_STORE_FP32 || st == COSM_STORE_FP16 || st == COSM_STORE_BF16) &&
         s.sched.grid && s.p.update == COSM_UPDATE_SCS;
}

bool lazy16(const cosm_state &s) {
  const int32_t st = s.p.storage;
  return (st == COSM_STORE_FP16 || st == COSM_STORE_BF16 || st == COSM_STORE_FP16_PK) &&
         s.p.update == COSM_UPDATE_SCS &&
         s.sched.dwt_period > 0 && wrap_drift_turns(s) < 0.5;
}

size_t readout_lds_bytes(int32_t n, int32_t B) {
  return 16 * 8 + (size_t)(B + 1) * 8 + (size_t)B * 4 + (size_t)n * 2 + 16;
}

int lds_capacity_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

int launch_init(cosm_state *s) { return dispatch_storage<InitFn>(s->p.storage, s); }
int launch_to_turns(cosm_state *s, float *out) {
  return dispatch_storage<ToTurnsFn>(s->p.storage, s, out);
}
int launch_from_turns(cosm_state *s, const float *in) {
  return dispatch_storage<FromTurnsFn>(s->p.storage, s, in);
}
int launch_readout(cosm_state *s) {
  if (s->p.readout == COSM_READOUT_OPTIMAL) return launch_readout_optimal(s);
  return dispatch_storage<ReadoutFn>(s->p.storage, s);
}

int launch_sweeps(cosm_state *s, int64_t n_sweeps) {
  if (s->timing) COSM_HIP_CHECK(hipEventRecord(s->ev0, s->stream));
  int rc = dispatch_storage<SweepFn>(s->p.storage, s, n_sweeps);
  if (rc) return rc;
  s->launches++;
  if (s->timing) {
    COSM_HIP_CHECK(hipEventRecord(s->ev1, s->stream));
    COSM_HIP_CHECK(hipEventSynchronize(s->ev1));
    float ms = 0.0f;
    COSM_HIP_CHECK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->kernel_ms += ms;
  }
  return COSM_OK;
}

int launch_energy(cosm_state *s) {
  hipLaunchKernelGGL(k_energy, dim3(s->R), dim3(256), 0, s->stream, s->d.spins, s->d.eu, s->d.ev,
                     s->d.J, s->has_h ? s->d.h : nullptr, s->n, s->m, s->d.H, s->d.cut);
  return launch_check("k_energy");
}

}  // namespace cosm
