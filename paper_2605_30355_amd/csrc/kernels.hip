// kernels.hip -- gfx950 kernels of libcosm and their launchers.
//
// Phase arithmetic is FP32 in turns (1 turn = 360 degrees).  FP32 storage keeps
// x in [0, 1) and wraps with v_fract_f32; FP16 / BF16 storage keeps the centred
// value y = x - 1/2 in [-1/2, 1/2] and wraps with y - rint(y) (one more bit of
// resolution than storing x).  On the 2^-23 turn grid every add, subtract, fma
// by 2 and fract below is exact, so grid-schedule trajectories are bit-exact.
//
// The pair update of Eq. (6), with the biased sign of Eq. (4) taken on the
// minimum angular difference:  f = fract(x_u - x_v); s = +1 iff f < 1/2;
// delta = alpha_t * J * s; x_u <- wrap(x_u - delta); x_v <- wrap(x_v + delta).
// (fract(d) < 1/2 is exactly "the difference wrapped to [-1/2, 1/2) is >= 0".)
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cosm {
namespace {

constexpr uint32_t kTagInit = 0x494E4954u;  // "INIT"
constexpr uint32_t kTagDwt = 0x44575420u;   // "DWT "
constexpr float kQ23 = 1.0f / 8388608.0f;   // 2^-23
constexpr float kQ22 = 1.0f / 4194304.0f;   // 2^-22
constexpr float kQ24 = 1.0f / 16777216.0f;  // 2^-24

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// Weyl key schedule; only output word 0 is used here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_first_word(uint32_t c0, uint32_t c1, uint32_t c2,
                                                      uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; i++) {
    const uint32_t ka = k0 + (uint32_t)i * 0x9E3779B9u;
    const uint32_t kb = k1 + (uint32_t)i * 0xBB67AE85u;
    const uint32_t p0lo = 0xD2511F53u * c0, p0hi = __umulhi(0xD2511F53u, c0);
    const uint32_t p1lo = 0xCD9E8D57u * c2, p1hi = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = p1hi ^ c1 ^ ka;
    const uint32_t n2 = p0hi ^ c3 ^ kb;
    c0 = n0;
    c1 = p1lo;
    c2 = n2;
    c3 = p0lo;
  }
  return c0;
}

__device__ __forceinline__ float fract1(float v) { return __builtin_amdgcn_fractf(v); }

// ---------------------------------------------------------------------------
// Storage formats.  "value" is x in [0,1) for FP32 and y = x - 1/2 otherwise.
// ---------------------------------------------------------------------------
template <int ST>
struct Fmt;

template <>
struct Fmt<COSM_STORE_FP32> {
  using elem_t = float;
  static constexpr int kPerWord = 1;
  __device__ __forceinline__ static float wrap(float v) { return fract1(v); }
  __device__ __forceinline__ static float from_turn(float x) { return x; }
  __device__ __forceinline__ static float to_turn(float v) { return v; }
  __device__ __forceinline__ static float load_elem(const void *p, size_t i) {
    return static_cast<const float *>(p)[i];
  }
  __device__ __forceinline__ static void store_elem(void *p, size_t i, float v) {
    static_cast<float *>(p)[i] = v;
  }
  template <int W>
  __device__ __forceinline__ static void unpack(const uint32_t (&w)[W], float (&v)[W]) {
#pragma unroll
    for (int k = 0; k < W; k++) v[k] = __uint_as_float(w[k]);
  }
  template <int W>
  __device__ __forceinline__ static void pack(const float (&v)[W], uint32_t (&w)[W]) {
#pragma unroll
    for (int k = 0; k < W; k++) w[k] = __float_as_uint(v[k]);
  }
};

template <int ST>
struct Fmt16 {
  static constexpr int kPerWord = 2;
  __device__ __forceinline__ static float wrap(float v) { return v - __builtin_rintf(v); }
  __device__ __forceinline__ static float from_turn(float x) { return x - 0.5f; }
  __device__ __forceinline__ static float to_turn(float v) { return fract1(v + 0.5f); }
  __device__ __forceinline__ static float dec(uint32_t bits16) {
    if constexpr (ST == COSM_STORE_FP16) {
      return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
    } else {
      return __uint_as_float(bits16 << 16);
    }
  }
  __device__ __forceinline__ static uint32_t enc(float v) {
    if constexpr (ST == COSM_STORE_FP16) {
      return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
    } else {
      return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v);
    }
  }
  __device__ __forceinline__ static float load_elem(const void *p, size_t i) {
    return dec(static_cast<const uint16_t *>(p)[i]);
  }
  __device__ __forceinline__ static void store_elem(void *p, size_t i, float v) {
    static_cast<uint16_t *>(p)[i] = (uint16_t)enc(v);
  }
  template <int W>
  __device__ __forceinline__ static void unpack(const uint32_t (&w)[W], float (&v)[2 * W]) {
#pragma unroll
    for (int k = 0; k < W; k++) {
      if constexpr (ST == COSM_STORE_FP16) {
        v[2 * k] = dec(w[k] & 0xffffu);
        v[2 * k + 1] = dec(w[k] >> 16);
      } else {
        v[2 * k] = __uint_as_float(w[k] << 16);
        v[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
      }
    }
  }
  template <int W>
  __device__ __forceinline__ static void pack(const float (&v)[2 * W], uint32_t (&w)[W]) {
#pragma unroll
    for (int k = 0; k < W; k++) w[k] = enc(v[2 * k]) | (enc(v[2 * k + 1]) << 16);
  }
};
template <>
struct Fmt<COSM_STORE_FP16> : Fmt16<COSM_STORE_FP16> {};
template <>
struct Fmt<COSM_STORE_BF16> : Fmt16<COSM_STORE_BF16> {};

// LDS row access with the widest ds_read / ds_write for W words.
template <int W>
__device__ __forceinline__ void lds_load(const uint32_t *base, int slot, uint32_t (&w)[W]) {
  if constexpr (W == 4) {
    const uint4 q = reinterpret_cast<const uint4 *>(base)[slot];
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else if constexpr (W == 2) {
    const uint2 q = reinterpret_cast<const uint2 *>(base)[slot];
    w[0] = q.x; w[1] = q.y;
  } else {
    w[0] = base[slot];
  }
}
template <int W>
__device__ __forceinline__ void lds_store(uint32_t *base, int slot, const uint32_t (&w)[W]) {
  if constexpr (W == 4) {
    reinterpret_cast<uint4 *>(base)[slot] = make_uint4(w[0], w[1], w[2], w[3]);
  } else if constexpr (W == 2) {
    reinterpret_cast<uint2 *>(base)[slot] = make_uint2(w[0], w[1]);
  } else {
    base[slot] = w[0];
  }
}

// Eq. (6) for one (edge, replica): values in the storage's convention.
template <int ST>
__device__ __forceinline__ void pair_update(float &xu, float &xv, float aJ) {
  const float f = fract1(xu - xv);
  const float dl = (f < 0.5f) ? aJ : -aJ;
  xu = Fmt<ST>::wrap(xu - dl);
  xv = Fmt<ST>::wrap(xv + dl);
}

// Dual window twist membership: mod_{1/2}(x - theta + w/2) < w, evaluated as
// fract(2x - c) < 2w with c = 2 theta - w (valid for x and for y = x - 1/2).
__device__ __forceinline__ bool in_windows(float v, float c, float win2) {
  return fract1(__builtin_fmaf(2.0f, v, -c)) < win2;
}

__device__ __forceinline__ float theta_turns(uint32_t t, uint32_t rid, uint32_t k0, uint32_t k1) {
  return (float)(philox_first_word(0u, t, rid, kTagDwt, k0, k1) >> 9) * kQ23;
}

// Per-sweep schedule evaluated on the device.  Grid: alpha = q * 2^-22 with
// q = floor(num / S), num = a0 (S - t + 1) + S/2, stepped by subtraction.
struct SweepSchedule {
  int32_t grid;
  int64_t S, q, r, aq, ar;
  float alpha_cont_per;  // alpha0 / S in turns (continuous)
  int32_t twist2;        // 2 * ratio (grid)
  float ratio;           // continuous
  int32_t period, phase; // twist when ++phase == period
  float win, win2;
};

struct LdsArgs {
  void *phases;
  const EdgeDesc *desc;       // [total_slots * nth] lane schedule
  const int32_t *Kc;          // [C] slots per thread of each class
  const int32_t *slot_vertex; // [n_rows]
  int32_t R, n_rows, C, total_slots;
  int64_t t0, nsw;
  SweepSchedule sch;
  uint32_t k0, k1, rid0;
  uint32_t bar_mask;          // register-resident schedule: barrier after slot j
};

// ---------------------------------------------------------------------------
// Phase initialisation, Algorithm 1 "Set x_i random".
// ---------------------------------------------------------------------------
template <int ST>
__global__ void __launch_bounds__(256) k_init(void *phases, int32_t n, int32_t R, uint32_t k0,
                                              uint32_t k1, uint32_t rid0, int32_t grid) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * R) return;
  const int32_t i = (int32_t)(idx / R), r = (int32_t)(idx % R);
  const uint32_t w = philox_first_word((uint32_t)i, 0u, rid0 + (uint32_t)r, kTagInit, k0, k1);
  const float x = grid ? (float)(w >> 9) * kQ23 : (float)(w >> 8) * kQ24;
  Fmt<ST>::store_elem(phases, (size_t)idx, Fmt<ST>::from_turn(x));
}

// ---------------------------------------------------------------------------
// The batched LDS-resident sweep: one workgroup owns RW = W * kPerWord whole
// replicas, stored as LDS rows of W 32-bit words (one row per slot), and runs
// every sweep of the call with workgroup barriers only.  Thread t handles the
// t-th entry of each slot of the lane schedule (consecutive lanes touch rows in
// distinct LDS bank groups).  EMAX > 0: the schedule (at most EMAX slots) is
// loaded into registers once; EMAX == 0: it streams from memory, one slot ahead.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void lds_load_at(const uint32_t *base, uint32_t byte, uint32_t (&w)[W]) {
  const char *p = reinterpret_cast<const char *>(base) + byte;
  if constexpr (W == 4) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else if constexpr (W == 2) {
    const uint2 q = *reinterpret_cast<const uint2 *>(p);
    w[0] = q.x; w[1] = q.y;
  } else {
    w[0] = *reinterpret_cast<const uint32_t *>(p);
  }
}
template <int W>
__device__ __forceinline__ void lds_store_at(uint32_t *base, uint32_t byte, const uint32_t (&w)[W]) {
  char *p = reinterpret_cast<char *>(base) + byte;
  if constexpr (W == 4) {
    *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
  } else if constexpr (W == 2) {
    *reinterpret_cast<uint2 *>(p) = make_uint2(w[0], w[1]);
  } else {
    *reinterpret_cast<uint32_t *>(p) = w[0];
  }
}

// Eq. (6) on every replica of one edge: rows at byte offsets bu, bv.
template <int ST, int W>
__device__ __forceinline__ void edge_rows(uint32_t *lds, uint32_t bu, uint32_t bv, float aJ) {
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  uint32_t wu[W], wv[W];
  lds_load_at<W>(lds, bu, wu);
  lds_load_at<W>(lds, bv, wv);
  float xu[RW], xv[RW];
  F::template unpack<W>(wu, xu);
  F::template unpack<W>(wv, xv);
#pragma unroll
  for (int k = 0; k < RW; k++) pair_update<ST>(xu[k], xv[k], aJ);
  F::template pack<W>(xu, wu);
  F::template pack<W>(xv, wv);
  lds_store_at<W>(lds, bu, wu);
  lds_store_at<W>(lds, bv, wv);
}

template <int ST, int W, int EMAX>
__global__ void __launch_bounds__(1024) k_sweep_lds(const LdsArgs a) {
  extern __shared__ uint32_t lds[];
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  constexpr uint32_t ROWB = 4 * W;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int32_t r0 = blockIdx.x * RW;
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

  // reference angles of the first twist of this call
  float *theta_buf = reinterpret_cast<float *>(lds + (size_t)a.n_rows * W);  // [2][RW]
  int tbuf = 0;
  if (a.sch.period > 0 && tid < RW) {
    const int64_t first = a.t0 + (a.sch.period - a.sch.phase);  // next t with t % period == 0
    theta_buf[tid] = 2.0f * theta_turns((uint32_t)first, a.rid0 + (uint32_t)(r0 + tid), a.k0,
                                        a.k1) - a.sch.win;
  }

  // register-resident lane schedule
  uint32_t ua[EMAX > 0 ? EMAX : 1], va[EMAX > 0 ? EMAX : 1];
  float jr[EMAX > 0 ? EMAX : 1];
  if constexpr (EMAX > 0) {
#pragma unroll
    for (int j = 0; j < EMAX; j++) {
      EdgeDesc d{kEmptySlot, 0.0f};
      if (j < a.total_slots) d = a.desc[(size_t)j * nth + tid];
      ua[j] = d.slots == kEmptySlot ? kEmptySlot : (d.slots & 0xffffu) * ROWB;
      va[j] = (d.slots >> 16) * ROWB;
      jr[j] = d.J;
    }
  }
  __syncthreads();

  SweepSchedule sc = a.sch;
  for (int64_t t = a.t0 + 1; t <= a.t0 + a.nsw; t++) {
    float alpha, twist;
    if (sc.grid) {
      alpha = (float)sc.q * kQ22;
      twist = (float)(sc.twist2 * sc.q) * kQ23;
      sc.q -= sc.aq;
      sc.r -= sc.ar;
      if (sc.r < 0) {
        sc.r += sc.S;
        sc.q -= 1;
      }
    } else {
      alpha = (float)(sc.S - t + 1) * sc.alpha_cont_per;
      twist = sc.ratio * alpha;
    }
    // Sequential conflict-free search: classes in order, a barrier after each.
    if constexpr (EMAX > 0) {
#pragma unroll
      for (int j = 0; j < EMAX; j++) {
        if (j < a.total_slots) {
          if (ua[j] != kEmptySlot) edge_rows<ST, W>(lds, ua[j], va[j], alpha * jr[j]);
          if ((a.bar_mask >> j) & 1u) __syncthreads();
        }
      }
    } else {
      int j = 0;
      EdgeDesc cur{kEmptySlot, 0.0f};
      if (a.total_slots > 0) cur = a.desc[tid];
      for (int c = 0; c < a.C; c++) {
        const int kc = a.Kc[c];
        for (int k = 0; k < kc; k++, j++) {
          const int jn = (j + 1 < a.total_slots) ? j + 1 : 0;
          const EdgeDesc nxt = a.desc[(size_t)jn * nth + tid];
          if (cur.slots != kEmptySlot)
            edge_rows<ST, W>(lds, (cur.slots & 0xffffu) * ROWB, (cur.slots >> 16) * ROWB,
                             alpha * cur.J);
          cur = nxt;
        }
        if (kc > 0) __syncthreads();
      }
    }
    // Dual window twist every `period` sweeps.  The reference angles of this
    // twist were drawn during the previous one (or at the start) by the first
    // RW lanes of the workgroup; those lanes now draw the next twist's angles
    // into the other buffer, read only after the barrier that ends this twist.
    if (sc.period > 0 && ++sc.phase == sc.period) {
      sc.phase = 0;
      float cth[RW];
#pragma unroll
      for (int k = 0; k < RW; k++) cth[k] = theta_buf[tbuf * RW + k];
      if (tid < RW)
        theta_buf[(tbuf ^ 1) * RW + tid] =
            2.0f * theta_turns((uint32_t)(t + sc.period), a.rid0 + (uint32_t)(r0 + tid), a.k0,
                               a.k1) - sc.win;
      tbuf ^= 1;
      for (int s = tid; s < a.n_rows; s += nth) {
        uint32_t w[W];
        lds_load<W>(lds, s, w);
        float v[RW];
        F::template unpack<W>(w, v);
#pragma unroll
        for (int k = 0; k < RW; k++)
          if (in_windows(v[k], cth[k], sc.win2)) v[k] = F::wrap(v[k] + twist);
        F::template pack<W>(v, w);
        lds_store<W>(lds, s, w);
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
      if (k < nvalid) F::store_elem(a.phases, base + k, v[k]);
  }
}

// ---------------------------------------------------------------------------
// Device-memory forms: one launch per colour class.  HBM form: a wave covers 64
// consecutive replicas of one edge (coalesced rows of the [n][R] layout).
// PLAIN form: one replica, a thread per edge.
// ---------------------------------------------------------------------------
template <int ST>
__global__ void __launch_bounds__(256) k_class_hbm(void *phases, const int32_t *peu,
                                                   const int32_t *pev, const float *pJ,
                                                   int32_t beg, int32_t cnt, int32_t R,
                                                   int32_t rchunks, float alpha) {
  using F = Fmt<ST>;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t e = wave / rchunks;
  const int32_t r = (int32_t)(wave % rchunks) * 64 + lane;
  if (e >= cnt || r >= R) return;
  const int32_t u = peu[beg + e], v = pev[beg + e];
  const float aJ = alpha * pJ[beg + e];
  float xu = F::load_elem(phases, (size_t)u * R + r);
  float xv = F::load_elem(phases, (size_t)v * R + r);
  pair_update<ST>(xu, xv, aJ);
  F::store_elem(phases, (size_t)u * R + r, xu);
  F::store_elem(phases, (size_t)v * R + r, xv);
}

// Twist for replicas [rbeg, rbeg + rcount): thread = one replica x a strip of
// `strip` vertices, so the reference angle is drawn once per strip.
template <int ST>
__global__ void __launch_bounds__(256) k_dwt_hbm(void *phases, int32_t n, int32_t R, int32_t rbeg,
                                                 int32_t rcount, int32_t strip, uint32_t t,
                                                 float twist, float win, float win2, uint32_t k0,
                                                 uint32_t k1, uint32_t rid0) {
  using F = Fmt<ST>;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t rchunks = (rcount + 63) / 64;
  const int64_t wave = g >> 6;
  const int lane = threadIdx.x & 63;
  const int32_t rloc = (int32_t)(wave % rchunks) * 64 + lane;
  const int64_t i0 = (wave / rchunks) * strip;
  if (rloc >= rcount || i0 >= n) return;
  const int32_t r = rbeg + rloc;
  const float c = 2.0f * theta_turns(t, rid0 + (uint32_t)r, k0, k1) - win;
  const int64_t i1 = min((int64_t)n, i0 + strip);
  for (int64_t i = i0; i < i1; i++) {
    const size_t idx = (size_t)i * R + r;
    const float v = F::load_elem(phases, idx);
    if (in_windows(v, c, win2)) F::store_elem(phases, idx, F::wrap(v + twist));
  }
}

template <int ST>
__global__ void __launch_bounds__(256) k_class_plain(void *phases, const int32_t *peu,
                                                     const int32_t *pev, const float *pJ,
                                                     int32_t beg, int32_t cnt, int32_t R,
                                                     int32_t r, float alpha) {
  using F = Fmt<ST>;
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const int32_t u = peu[beg + e], v = pev[beg + e];
  const float aJ = alpha * pJ[beg + e];
  float xu = F::load_elem(phases, (size_t)u * R + r);
  float xv = F::load_elem(phases, (size_t)v * R + r);
  pair_update<ST>(xu, xv, aJ);
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
                                                       const float *inc_J, int32_t n,
                                                       int32_t R, float alpha) {
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
  F::store_elem(dst, (size_t)idx, F::wrap(xi + acc));
}

// ---------------------------------------------------------------------------
// Block reductions (wave64 shuffles, then one LDS slot per wave).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ int64_t block_sum(int64_t v, int64_t *scratch /* >= 16 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wv] = v;
  __syncthreads();
  int64_t total = 0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int k = 0; k < nw; k++) total += scratch[k];
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------------------
// Readout, Algorithm 1 binarization: one workgroup per replica.  Bisector p is
// beta_p (increasing, beta_0 = 0); spin i is +1 on [beta_p, beta_p + 1/2).
// With x in [0,1): s_i(0) = +1 iff x < 1/2, and spin i flips exactly once, at
// q_i = #{p : beta_p <= y_i}, y_i = x_i mod 1/2.  An edge's term -J s_u s_v thus
// changes sign at min(q_u, q_v) and back at max(q_u, q_v): a difference array
// over p gives every H_p in O(n + m + B).
// ---------------------------------------------------------------------------
struct ReadoutArgs {
  const void *phases;
  const int32_t *eu, *ev, *J, *h;
  int8_t *spins;
  int64_t *H, *cut;
  int32_t *best_p;
  int32_t n, R, B, grid;
  int64_t m;
};

template <int ST>
__global__ void __launch_bounds__(256) k_readout(const ReadoutArgs a) {
  using F = Fmt<ST>;
  extern __shared__ int64_t sm64[];
  int64_t *red = sm64;            // 16
  int64_t *bins = sm64 + 16;      // B + 1
  float *beta = reinterpret_cast<float *>(bins + a.B + 1);  // B
  uint16_t *code = reinterpret_cast<uint16_t *>(beta + a.B); // n
  const int r = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
  const int B = a.B;
  __shared__ int32_t s_bp;
  __shared__ int64_t s_best;

  if (a.h != nullptr) {
    // bias fields: fixed semicircles, +1 on the half centred at 0
    int64_t e = 0;
    for (int i = tid; i < a.n; i += nth) {
      const float x = F::to_turn(F::load_elem(a.phases, (size_t)i * a.R + r));
      const int s = fract1(x + 0.25f) < 0.5f ? 1 : -1;
      a.spins[(size_t)r * a.n + i] = (int8_t)s;
      e -= (int64_t)a.h[i] * s;
    }
    __syncthreads();
    int64_t c = 0;
    for (int64_t k = tid; k < a.m; k += nth) {
      const int su = a.spins[(size_t)r * a.n + a.eu[k]], sv = a.spins[(size_t)r * a.n + a.ev[k]];
      e -= (int64_t)a.J[k] * su * sv;
      if (su != sv) c -= a.J[k];
    }
    e = block_sum(e, red);
    c = block_sum(c, red);
    if (tid == 0) {
      a.H[r] = e;
      a.cut[r] = c;
      a.best_p[r] = 0;
    }
    return;
  }

  for (int p = tid; p <= B; p += nth) bins[p] = 0;
  for (int p = tid; p < B; p += nth) {
    if (a.grid) {
      const int64_t units = (((int64_t)p << 23) + B) / (2 * (int64_t)B);
      beta[p] = (float)units * kQ23;
    } else {
      beta[p] = (float)p / (float)(2 * B);
    }
  }
  __syncthreads();
  for (int i = tid; i < a.n; i += nth) {
    const float x = F::to_turn(F::load_elem(a.phases, (size_t)i * a.R + r));
    const bool neg = !(x < 0.5f);
    const float y = neg ? x - 0.5f : x;
    int lo = 0, hi = B;  // count of beta <= y
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (beta[mid] <= y) lo = mid + 1; else hi = mid;
    }
    code[i] = (uint16_t)(lo | (neg ? 0x8000 : 0));
  }
  __syncthreads();
  int64_t h0 = 0;
  for (int64_t k = tid; k < a.m; k += nth) {
    const uint32_t cu = code[a.eu[k]], cv = code[a.ev[k]];
    const int su = (cu & 0x8000) ? -1 : 1, sv = (cv & 0x8000) ? -1 : 1;
    const int64_t e0 = -(int64_t)a.J[k] * su * sv;
    h0 += e0;
    const int qu = cu & 0x7fff, qv = cv & 0x7fff;
    const int lo = min(qu, qv), hi = max(qu, qv);
    if (lo != hi) {
      if (lo < B) atomicAdd((unsigned long long *)&bins[lo], (unsigned long long)(-2 * e0));
      if (hi < B) atomicAdd((unsigned long long *)&bins[hi], (unsigned long long)(2 * e0));
    }
  }
  h0 = block_sum(h0, red);
  if (tid == 0) {
    int64_t run = h0, best = h0;
    int bp = 0;
    for (int p = 1; p < B; p++) {
      run += bins[p];
      if (run < best) {
        best = run;
        bp = p;
      }
    }
    s_bp = bp;
    s_best = best;
  }
  __syncthreads();
  const int bp = s_bp;
  for (int i = tid; i < a.n; i += nth) {
    const uint32_t ci = code[i];
    const int s0 = (ci & 0x8000) ? -1 : 1;
    a.spins[(size_t)r * a.n + i] = (int8_t)((bp < (int)(ci & 0x7fff)) ? s0 : -s0);
  }
  int64_t c = 0;
  for (int64_t k = tid; k < a.m; k += nth) {
    const uint32_t cu = code[a.eu[k]], cv = code[a.ev[k]];
    const int su = ((cu & 0x8000) ? -1 : 1) * ((bp < (int)(cu & 0x7fff)) ? 1 : -1);
    const int sv = ((cv & 0x8000) ? -1 : 1) * ((bp < (int)(cv & 0x7fff)) ? 1 : -1);
    if (su != sv) c -= a.J[k];
  }
  c = block_sum(c, red);
  if (tid == 0) {
    a.H[r] = s_best;
    a.cut[r] = c;
    a.best_p[r] = bp;
  }
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
    return (float)q * kQ22;
  }
  return (float)(sc.S - t + 1) * (sc.alpha0_turns / (float)sc.S);
}

float host_twist(const Schedule &sc, int64_t t) {
  if (sc.grid) {
    const int64_t q = (sc.a0_units * (sc.S - t + 1) + sc.S / 2) / sc.S;
    return (float)(sc.twist_num2 * q) * kQ23;
  }
  return sc.dwt_ratio * host_alpha(sc, t);
}

template <int ST, int W, int EMAX>
int launch_lds(cosm_state *s, const LdsArgs &a) {
  const size_t lds = s->shape.lds_bytes;
  (void)hipFuncSetAttribute((const void *)k_sweep_lds<ST, W, EMAX>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_sweep_lds<ST, W, EMAX>), dim3(s->shape.blocks), dim3(s->shape.threads), lds,
                     s->stream, a);
  return launch_check("k_sweep_lds");
}

template <int ST, int W>
int launch_lds_w(cosm_state *s, const LdsArgs &a) {
  const int slots = a.total_slots;
  if (slots <= 4) return launch_lds<ST, W, 4>(s, a);
  if (slots <= 8) return launch_lds<ST, W, 8>(s, a);
  if (slots <= 16) return launch_lds<ST, W, 16>(s, a);
  return launch_lds<ST, W, 0>(s, a);
}

template <int ST>
int sweeps_lds_st(cosm_state *s, int64_t n_sweeps) {
  LdsArgs a{};
  a.phases = s->d.phases;
  a.desc = s->d.desc;
  a.Kc = s->d.class_off;
  a.slot_vertex = s->d.slot_vertex;
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
  const Schedule &sc = s->sched;
  SweepSchedule &w = a.sch;
  w.grid = sc.grid;
  w.S = sc.S;
  const int64_t num = sc.a0_units * (sc.S - s->t) + sc.S / 2;  // numerator at t0 + 1
  w.q = num / sc.S;
  w.r = num % sc.S;
  w.aq = sc.a0_units / sc.S;
  w.ar = sc.a0_units % sc.S;
  w.alpha_cont_per = sc.alpha0_turns / (float)sc.S;
  w.twist2 = sc.twist_num2;
  w.ratio = sc.dwt_ratio;
  w.period = sc.dwt_period;
  w.phase = sc.dwt_period > 0 ? (int32_t)(s->t % sc.dwt_period) : 0;
  w.win = sc.window;
  w.win2 = sc.window2;
  a.k0 = (uint32_t)(s->seed & 0xffffffffu);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.rid0 = (uint32_t)s->rid0;
  const int W = s->shape.rw / Fmt<ST>::kPerWord;
  if (W == 4) return launch_lds_w<ST, 4>(s, a);
  if (W == 2) return launch_lds_w<ST, 2>(s, a);
  if (W == 1) return launch_lds_w<ST, 1>(s, a);
  return set_error(COSM_EINVAL, "unsupported replicas per workgroup");
}

template <int ST>
int dwt_hbm_st(cosm_state *s, int64_t t, int32_t rbeg, int32_t rcount) {
  const Schedule &sc = s->sched;
  const int32_t strip = 64;
  const int32_t rchunks = (rcount + 63) / 64;
  const int64_t strips = ((int64_t)s->n + strip - 1) / strip;
  const int64_t threads = strips * rchunks * 64;
  const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
  hipLaunchKernelGGL((k_dwt_hbm<ST>), grid, block, 0, s->stream, s->d.phases, s->n, s->R, rbeg,
                     rcount, strip, (uint32_t)t, host_twist(sc, t), sc.window, sc.window2,
                     (uint32_t)(s->seed & 0xffffffffu), (uint32_t)(s->seed >> 32),
                     (uint32_t)s->rid0);
  return launch_check("k_dwt_hbm");
}

template <int ST>
int sweeps_hbm_st(cosm_state *s, int64_t n_sweeps) {
  const Schedule &sc = s->sched;
  const int32_t rchunks = (s->R + 63) / 64;
  for (int64_t t = s->t + 1; t <= s->t + n_sweeps; t++) {
    const float alpha = host_alpha(sc, t);
    if (s->p.update == COSM_UPDATE_FULL_GRADIENT) {
      const int64_t tot = (int64_t)s->n * s->R;
      hipLaunchKernelGGL((k_full_gradient<ST>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                         s->stream, s->d.phases, s->d.phases_alt, s->d.inc_off, s->d.inc_nbr,
                         s->d.inc_J, s->n, s->R, alpha);
      if (int rc = launch_check("k_full_gradient")) return rc;
      std::swap(s->d.phases, s->d.phases_alt);
    } else {
      for (int c = 0; c < s->C; c++) {
        const int32_t beg = s->class_begin[c], cnt = s->class_sizes[c];
        if (cnt == 0) continue;
        const int64_t threads = (int64_t)cnt * rchunks * 64;
        hipLaunchKernelGGL((k_class_hbm<ST>), dim3((unsigned)((threads + 255) / 256)), dim3(256),
                           0, s->stream, s->d.phases, s->d.peu, s->d.pev, s->d.pJ, beg, cnt, s->R,
                           rchunks, alpha);
        if (int rc = launch_check("k_class_hbm")) return rc;
      }
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
                           alpha);
        if (int rc = launch_check("k_class_plain")) return rc;
      }
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
  const size_t lds = readout_lds_bytes(s->n, a.B);
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
                     (uint32_t)(s->seed >> 32), (uint32_t)s->rid0, s->sched.grid);
  return launch_check("k_init");
}

template <template <int> class Fn, typename... A>
int dispatch_storage(int storage, A &&...args) {
  switch (storage) {
    case COSM_STORE_FP32: return Fn<COSM_STORE_FP32>::run(args...);
    case COSM_STORE_FP16: return Fn<COSM_STORE_FP16>::run(args...);
    case COSM_STORE_BF16: return Fn<COSM_STORE_BF16>::run(args...);
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
      case COSM_RES_LDS: return sweeps_lds_st<ST>(s, n);
      case COSM_RES_HBM: return sweeps_hbm_st<ST>(s, n);
      case COSM_RES_PLAIN: return sweeps_plain_st<ST>(s, n);
    }
    return set_error(COSM_EINVAL, "unknown residency");
  }
};

}  // namespace

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
int launch_readout(cosm_state *s) { return dispatch_storage<ReadoutFn>(s->p.storage, s); }

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
