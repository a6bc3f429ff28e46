// device_common.hpp -- device-side pieces shared by the sweep kernels:
// Philox, the storage formats, LDS row access, the pair update of Eq. (6), the
// dual-window membership test and the per-sweep schedule.
//
// Phases are turns (1 turn = 360 degrees).  FP32 storage keeps x in [0, 1) and
// wraps with v_fract_f32; FP16 / BF16 / FP16_PK storage keeps the centred value
// y = x - 1/2 in [-1/2, 1/2] and wraps with y - rint(y); FIX16 keeps x in 16-bit
// fixed point and wraps by integer overflow (update_words, twist_words).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cosm {
namespace {

constexpr uint32_t kTagInit = 0x494E4954u;  // "INIT"
constexpr uint32_t kTagDwt = 0x44575420u;   // "DWT "
constexpr float kQ23 = 1.0f / 8388608.0f;   // 2^-23
constexpr float kQ22 = 1.0f / 4194304.0f;   // 2^-22
constexpr float kQ24 = 1.0f / 16777216.0f;  // 2^-24

// Device pointers taken from tables in memory lose their address space and
// would be read with flat loads, which also count against the LDS wait
// counter; these casts keep such reads global.
template <typename T>
using gptr = const T __attribute__((address_space(1))) *;
template <typename T>
using gptr_mut = T __attribute__((address_space(1))) *;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
  return (gptr<T>)(p);
}
template <typename T>
__device__ __forceinline__ gptr_mut<T> as_global_mut(T *p) {
  return (gptr_mut<T>)(p);
}


// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// Weyl key schedule; only output word 0 is used here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint2 philox_words01(uint32_t c0, uint32_t c1, uint32_t c2,
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
  return make_uint2(c0, c1);
}

__device__ __forceinline__ uint32_t philox_first_word(uint32_t c0, uint32_t c1, uint32_t c2,
                                                      uint32_t c3, uint32_t k0, uint32_t k1) {
  return philox_words01(c0, c1, c2, c3, k0, k1).x;
}

// Logical index of workgroup b of nb when consecutive workgroups are dealt to
// the 8 XCDs in turn: XCD x runs logical indices [x q, x q + q), q = nb / 8
// (the nb % 8 workgroups past 8 q keep their own index).
__device__ __forceinline__ int32_t xcd_block(int32_t b, int32_t nb) {
  const int32_t q = nb >> 3;
  return b < 8 * q ? (b & 7) * q + (b >> 3) : b;
}

__device__ __forceinline__ float fract1(float v) { return __builtin_amdgcn_fractf(v); }

// The formats whose sweeps can take the parity step on the grid schedule
// (step_by_parity): the float formats with FP32 arithmetic.
constexpr bool parity_storage(int st) {
  return st == COSM_STORE_FP32 || st == COSM_STORE_FP16 || st == COSM_STORE_BF16;
}

// The FP32 rounding mode of the calling wave (MODE.FP_ROUND bits 1:0; each wave
// has its own MODE and starts in round-to-nearest-even).  Toward minus
// infinity, fma(d, 2, 1.5 * 2^23) is 1.5 * 2^23 + floor(2d) exactly for
// |2d| < 2^22, an integer whose lowest mantissa bit is the parity of floor(2d);
// exact sums and products do not depend on the mode.
// The compiler orders no instruction against a write of MODE (neither the
// arithmetic nor the memory accesses around s_setreg), so the switch is an asm
// statement that also yields the constant 1.5 * 2^23: every parity fma takes
// it as an operand and so cannot run before the switch.  The switch back is a
// volatile asm with a memory clobber, after the loops whose stores consume the
// parity results.  s_nop 1 gives the mode write its wait states before the
// next vector instruction.
__device__ __forceinline__ float f32_round_down() {
  float m;
  asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 2), 2\n\ts_nop 1\n\t"
               "s_mov_b32 %0, 0x4b400000"
               : "=s"(m)
               :
               : "memory");
  return m;
}
__device__ __forceinline__ void f32_round_nearest() {
  asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 2), 0\n\ts_nop 1" ::: "memory");
}

// Eq. (4)-(6)'s step sign on exact grid values, under f32_round_down (pm its
// 1.5 * 2^23): fract(d) < 1/2 exactly when floor(2d) is even, so the step is aJ
// with its sign bit flipped by that parity (one fma and one v_lshl_add instead
// of fract, compare and select).
__device__ __forceinline__ float step_by_parity(float d, float aJ, float pm) {
  const float r = __builtin_fmaf(d, 2.0f, pm);
  return __uint_as_float((__float_as_uint(r) << 31) + __float_as_uint(aJ));
}

// ---------------------------------------------------------------------------
// Storage formats.  "value" is x in [0,1) for FP32 and y = x - 1/2 otherwise.
// ---------------------------------------------------------------------------
template <int ST>
struct Fmt;

// kStepScale: the factor from turns to the step argument of update_words
// (1 for the FP32-arithmetic formats; the fixed-point formats take the step in
// their own integer units, scaled once per sweep instead of once per edge).
template <>
struct Fmt<COSM_STORE_FP32> {
  using elem_t = float;
  static constexpr int kPerWord = 1;
  static constexpr float kStepScale = 1.0f;
  __device__ __forceinline__ static float wrap(float v) { return fract1(v); }
  __device__ __forceinline__ static float from_turn(float x) { return x; }
  __device__ __forceinline__ static float to_turn(float v) { return v; }
  __device__ __forceinline__ static float load_elem(const void *p, size_t i) {
    return as_global(static_cast<const float *>(p))[i];
  }
  __device__ __forceinline__ static void store_elem(void *p, size_t i, float v) {
    as_global_mut(static_cast<float *>(p))[i] = v;
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
  static constexpr float kStepScale = 1.0f;
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
    return dec(as_global(static_cast<const uint16_t *>(p))[i]);
  }
  __device__ __forceinline__ static void store_elem(void *p, size_t i, float v) {
    as_global_mut(static_cast<uint16_t *>(p))[i] = (uint16_t)enc(v);
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
  // two values per word with one round-to-nearest-even packed conversion
  template <int W>
  __device__ __forceinline__ static void pack(const float (&v)[2 * W], uint32_t (&w)[W]) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int k = 0; k < W; k++) {
      const f32x2 p = {v[2 * k], v[2 * k + 1]};
      if constexpr (ST == COSM_STORE_FP16) {
        w[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector(p, f16x2));
      } else {
        w[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector(p, bf16x2));
      }
    }
  }
};
template <>
struct Fmt<COSM_STORE_FP16> : Fmt16<COSM_STORE_FP16> {};
// FP16 storage with FP16 arithmetic: the FP16 encoding, its own update paths
template <>
struct Fmt<COSM_STORE_FP16_PK> : Fmt16<COSM_STORE_FP16> {};
template <>
struct Fmt<COSM_STORE_BF16> : Fmt16<COSM_STORE_BF16> {};

// 16-bit fixed point: the stored integer k is x = k 2^-16 turn.  As a value
// x in [0, 1) is exact in FP32, so every FP32 form below works unchanged (on
// the 2^-16 grid its adds, fract and comparisons are exact); the LDS sweep
// also has an integer form (edge_rows_fix16).
template <>
struct Fmt<COSM_STORE_FIX16> {
  static constexpr int kPerWord = 2;
  static constexpr float kStepScale = 65536.0f;
  __device__ __forceinline__ static float wrap(float v) { return fract1(v); }
  __device__ __forceinline__ static float from_turn(float x) { return x; }
  __device__ __forceinline__ static float to_turn(float v) { return v; }
  __device__ __forceinline__ static float dec(uint32_t bits16) {
    return (float)bits16 * (1.0f / 65536.0f);
  }
  // nearest grid point, 1 turn wrapping to 0
  __device__ __forceinline__ static uint32_t enc(float v) {
    return (uint32_t)__builtin_rintf(v * 65536.0f) & 0xffffu;
  }
  __device__ __forceinline__ static float load_elem(const void *p, size_t i) {
    return dec(as_global(static_cast<const uint16_t *>(p))[i]);
  }
  __device__ __forceinline__ static void store_elem(void *p, size_t i, float v) {
    as_global_mut(static_cast<uint16_t *>(p))[i] = (uint16_t)enc(v);
  }
  template <int W>
  __device__ __forceinline__ static void unpack(const uint32_t (&w)[W], float (&v)[2 * W]) {
#pragma unroll
    for (int k = 0; k < W; k++) {
      v[2 * k] = dec(w[k] & 0xffffu);
      v[2 * k + 1] = dec(w[k] >> 16);
    }
  }
  template <int W>
  __device__ __forceinline__ static void pack(const float (&v)[2 * W], uint32_t (&w)[W]) {
#pragma unroll
    for (int k = 0; k < W; k++) w[k] = enc(v[2 * k]) | (enc(v[2 * k + 1]) << 16);
  }
};

// 32-bit fixed point: the stored integer k is x = k 2^-32 turn.  Under the
// GRID schedule every phase is a multiple of 2^-23 turn, so the value x is
// exact in FP32 and the FP32 forms below work unchanged; the LDS sweep updates
// the integers directly, where the wrap to [0, 1) turn is the overflow of the
// 32-bit add.  The trajectory is the FP32 one bit for bit.
template <>
struct Fmt<COSM_STORE_FIX32> {
  static constexpr int kPerWord = 1;
  static constexpr float kStepScale = 4294967296.0f;
  __device__ __forceinline__ static float wrap(float v) { return fract1(v); }
  __device__ __forceinline__ static float from_turn(float x) { return x; }
  __device__ __forceinline__ static float to_turn(float v) { return v; }
  __device__ __forceinline__ static float dec(uint32_t bits) {
    return (float)bits * (1.0f / 4294967296.0f);
  }
  // nearest multiple of 2^-32 turn (v in [0, 1) as FP32: below 2^32 - 2^8
  // after scaling, so no wrap is needed)
  __device__ __forceinline__ static uint32_t enc(float v) {
    return (uint32_t)__builtin_rintf(v * 4294967296.0f);
  }
  __device__ __forceinline__ static float load_elem(const void *p, size_t i) {
    return dec(as_global(static_cast<const uint32_t *>(p))[i]);
  }
  __device__ __forceinline__ static void store_elem(void *p, size_t i, float v) {
    as_global_mut(static_cast<uint32_t *>(p))[i] = enc(v);
  }
  template <int W>
  __device__ __forceinline__ static void unpack(const uint32_t (&w)[W], float (&v)[W]) {
#pragma unroll
    for (int k = 0; k < W; k++) v[k] = dec(w[k]);
  }
  template <int W>
  __device__ __forceinline__ static void pack(const float (&v)[W], uint32_t (&w)[W]) {
#pragma unroll
    for (int k = 0; k < W; k++) w[k] = enc(v[k]);
  }
};

// A value in turns (any sign) as a 32-bit fixed-point angle mod 1 turn; exact
// for multiples of 2^-32 turn whose fraction FP32 holds.
__device__ __forceinline__ uint32_t turns_fix32(float v) {
  return (uint32_t)(fract1(v) * 4294967296.0f);
}

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

// FP16 value of v (round to nearest even), as an FP32 number.
__device__ __forceinline__ float round_h(float v) { return (float)(_Float16)v; }

// Eq. (6) for one (edge, replica): values in the storage's convention.
// LAZY: no wrap (phases wrapped at the twists only; fract(x_u - x_v) does not
// need wrapped operands).
// FP16_PK storage computes in FP16 arithmetic, each step rounded to FP16 as the
// packed form in update_words does it: e = y_u - y_v; the coupling is positive
// (fract(e) < 1/2) when round(2e - 1/2) is even, round to nearest even (an
// exact half-turn difference counts as positive); step +-alpha J rounded to
// FP16; y_u - step, y_v + step rounded to FP16; the wrap y - rint(y) is then
// exact.  FP32 steps on FP16 operands give these results: an FP32 result of
// one operation rounded again to FP16 equals its direct FP16 rounding
// (24 >= 2 x 11 + 2 bits).
// RD (the grid schedule, under f32_round_down): every FP32 operand and result
// is exact (phases and steps are multiples of 2^-23 turn below 2 in
// magnitude), and the step's sign comes from step_by_parity.  FP16 and BF16
// storage take it too: their values are on the same grid, and the packed
// conversions that round them on store follow the 16-bit rounding field of
// MODE, not the FP32 one, so they still round to nearest even.
template <int ST, bool LAZY = false, bool RD = false>
__device__ __forceinline__ void pair_update(float &xu, float &xv, float aJ, float pm = 0.0f) {
  static_assert(!RD || parity_storage(ST), "the parity step is a grid form of the float formats");
  if constexpr (ST == COSM_STORE_FP16_PK) {
    const float e = round_h(xu - xv);
    const float t = round_h(__builtin_fmaf(2.0f, e, -0.5f));
    const float st = round_h(aJ);
    const float dl = ((int32_t)__builtin_rintf(t) & 1) ? -st : st;
    xu = round_h(xu - dl);
    xv = round_h(xv + dl);
    if constexpr (!LAZY) {
      xu -= __builtin_rintf(xu);
      xv -= __builtin_rintf(xv);
    }
  } else {
    const float dl = RD ? step_by_parity(xu - xv, aJ, pm) : (fract1(xu - xv) < 0.5f) ? aJ : -aJ;
    xu = LAZY ? xu - dl : Fmt<ST>::wrap(xu - dl);
    xv = LAZY ? xv + dl : Fmt<ST>::wrap(xv + dl);
  }
}

// Eq. (6) between x (storage convention) and a fixed virtual spin at phase 0
// coupled with h (the bias field read as one more edge): s = +1 iff x lies in
// [0, 1/2) turn, x <- wrap(x - alpha h s).
template <int ST, bool LAZY = false>
__device__ __forceinline__ void field_update(float &v, float ah) {
  const float f = fract1(Fmt<ST>::to_turn(v));
  const float d = (f < 0.5f) ? ah : -ah;
  v = LAZY ? v - d : Fmt<ST>::wrap(v - d);
}

// Dual window twist membership: mod_{1/2}(x - theta + w/2) < w, evaluated as
// fract(2x - c) < 2w with c = 2 theta - w (valid for x and for y = x - 1/2).
__device__ __forceinline__ bool in_windows(float v, float c, float win2) {
  return fract1(__builtin_fmaf(2.0f, v, -c)) < win2;
}


// The step-size ramp and the twist angle, evaluated on the device.  Grid:
// alpha = q * aunit (2^-22 turn; 2^-15 for FIX16) with
// q = floor((a0 (S - t + 1) + S/2) / S) (q < 2^22 and 2 rho q < 2^23, so the
// int32 products and conversions are exact).  Continuous: the literal ramp.
struct SweepSchedule {
  int32_t grid;
  uint32_t S;            // schedule length (<= 2^31)
  float alpha_cont_per;  // alpha0 / S in turns (continuous)
  int32_t twist2;        // 2 * ratio (grid)
  float ratio;           // continuous
  int32_t period, phase; // twist when ++phase == period
  float win, win2;
  int64_t a0;            // grid: alpha0 in step units
  float aunit, tunit;    // grid: turns per step unit and per twist unit
  uint32_t tshift;       // reference angle: (draw >> tshift) * tscale
  float tscale;
};

// alpha_t and the twist of sweep t (1 <= t <= S), exactly as the host
// evaluates them for the device-memory forms.
__device__ __forceinline__ void schedule_at(const SweepSchedule &sc, uint32_t t, float &alpha,
                                            float &twist) {
  const uint32_t u = sc.S - t + 1u;  // S - t + 1 >= 1
  if (sc.grid) {
    const int32_t q = (int32_t)((sc.a0 * (int64_t)u + (int64_t)(sc.S / 2u)) / (int64_t)sc.S);
    alpha = (float)q * sc.aunit;
    twist = (float)(sc.twist2 * q) * sc.tunit;
  } else {
    alpha = (float)u * sc.alpha_cont_per;
    twist = sc.ratio * alpha;
  }
}

// One wave's table of 64 sweeps: lane i holds alpha and the twist of sweep
// t_next + i (clamped to S); a sweep then reads its pair with two readlanes
// instead of stepping the ramp on the scalar and vector units every sweep.
// Bit i of twists is set when sweep t_next + i ends with a twist
// (t % period == 0), so a sweep tests one bit instead of stepping a counter.
struct ScheduleChunk {
  float alpha, twist;
  uint64_t twists;
  __device__ __forceinline__ void fill(const SweepSchedule &sc, uint32_t t_next) {
    const uint32_t lane = __lane_id();
    const uint32_t t = min(t_next + lane, sc.S);
    schedule_at(sc, t, alpha, twist);
    const uint32_t tl = t_next + lane;
    twists = __ballot(sc.period > 0 && tl <= sc.S && tl % (uint32_t)sc.period == 0u);
  }
  __device__ __forceinline__ void get(uint32_t i, float &a, float &tw) const {
    a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(alpha), i));
    tw = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(twist), i));
  }
  __device__ __forceinline__ bool twist_at(uint32_t i) const { return (twists >> i) & 1u; }
};

// The device schedule after t_done sweeps (host side).
SweepSchedule make_sweep_schedule(const Schedule &sc, int64_t t_done) {
  SweepSchedule w{};
  w.grid = sc.grid;
  w.S = (uint32_t)sc.S;
  w.alpha_cont_per = sc.alpha0_turns / (float)sc.S;
  w.twist2 = sc.twist_num2;
  w.ratio = sc.dwt_ratio;
  w.period = sc.dwt_period;
  w.phase = sc.dwt_period > 0 ? (int32_t)(t_done % sc.dwt_period) : 0;
  w.win = sc.window;
  w.win2 = sc.window2;
  w.a0 = sc.a0_units;
  w.aunit = sc.aunit;
  w.tunit = sc.tunit;
  w.tshift = (uint32_t)sc.tshift;
  w.tscale = sc.tscale;
  return w;
}

// Fills table[q * nrep + k] with c = 2 theta - w for the twist at sweep
// t_first + q * period (q < nch) and replica rid_base + k (k < nrep), and, when
// dirs is not null, dirs[q * nrep + k] with that twist's direction (+-1 from
// the top bit of word 1 of the same draw; used with bias fields).  Every thread
// of the workgroup takes part; the caller synchronises.
__device__ __forceinline__ void theta_fill(float *table, float *dirs, int nch, int nrep,
                                           uint32_t t_first, int32_t period, uint32_t rid_base,
                                           uint32_t k0, uint32_t k1, float win, uint32_t tshift,
                                           float tscale) {
  for (int i = threadIdx.x; i < nch * nrep; i += blockDim.x) {
    const int q = i / nrep, k = i - q * nrep;
    const uint2 w = philox_words01(0u, t_first + (uint32_t)(q * period),
                                   rid_base + (uint32_t)k, kTagDwt, k0, k1);
    table[i] = 2.0f * ((float)(w.x >> tshift) * tscale) - win;
    if (dirs != nullptr) dirs[i] = (w.y >> 31) ? -1.0f : 1.0f;
  }
}

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

typedef uint32_t su2 __attribute__((ext_vector_type(2)));
// Row access at an absolute LDS byte address, for kernels whose only LDS is
// the dynamic allocation (which then starts at address 0), so that a row's
// byte offset is its address (clang vector types: the HIP vector classes do
// not take an address-space qualifier).
typedef uint32_t su4 __attribute__((ext_vector_type(4)));
template <int W>
__device__ __forceinline__ void row_load(uint32_t addr, uint32_t (&w)[W]) {
  if constexpr (W == 4) {
    typedef __attribute__((address_space(3))) const su4 *P;
    const su4 q = *(P)(uintptr_t)addr;
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else if constexpr (W == 2) {
    typedef __attribute__((address_space(3))) const su2 *P;
    const su2 q = *(P)(uintptr_t)addr;
    w[0] = q.x; w[1] = q.y;
  } else {
    typedef __attribute__((address_space(3))) const uint32_t *P;
    w[0] = *(P)(uintptr_t)addr;
  }
}
template <int W>
__device__ __forceinline__ void row_store(uint32_t addr, const uint32_t (&w)[W]) {
  if constexpr (W == 4) {
    typedef __attribute__((address_space(3))) su4 *P;
    *(P)(uintptr_t)addr = su4{w[0], w[1], w[2], w[3]};
  } else if constexpr (W == 2) {
    typedef __attribute__((address_space(3))) su2 *P;
    *(P)(uintptr_t)addr = su2{w[0], w[1]};
  } else {
    typedef __attribute__((address_space(3))) uint32_t *P;
    *(P)(uintptr_t)addr = w[0];
  }
}

// Eq. (6) on the W words of an edge's two rows (every replica they hold); aJ
// is alpha_t J in turns times Fmt<ST>::kStepScale.
// FIX16: two replicas per word in 16-bit lanes, packed integer arithmetic; the
// lane difference u - v wraps to the signed difference in [-1/2, 1/2) turn,
// whose sign bit selects -step or +step, and the updates wrap by overflow.
// FIX32: the same on one 32-bit integer per replica.
// FP16_PK: two replicas per word in packed FP16 arithmetic (pair_update's steps):
// r = (2e - 1/2) + 1536 lies in [1024, 2048), where FP16 has unit spacing, so
// its lowest bit is the parity of round(2e - 1/2); shifted to the sign bit it
// flips the step's sign.  The wrap subtracts (y + 1536) - 1536 = rint(y).
// Other formats: unpack, the FP32 update, pack.
template <int ST, int W, bool LAZY = false, bool RD = false>
__device__ __forceinline__ void update_words(uint32_t (&wu)[W], uint32_t (&wv)[W], float aJ,
                                             float pm = 0.0f) {
  if constexpr (ST == COSM_STORE_FP16_PK) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const uint32_t sb = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)aJ);
    const uint32_t step = sb | (sb << 16);
    const h2 two = {(_Float16)2.0f, (_Float16)2.0f};
    const h2 mhalf = {(_Float16)-0.5f, (_Float16)-0.5f};
    const h2 mag = {(_Float16)1536.0f, (_Float16)1536.0f};
#pragma unroll
    for (int k = 0; k < W; k++) {
      const h2 u = __builtin_bit_cast(h2, wu[k]), v = __builtin_bit_cast(h2, wv[k]);
      const h2 r = __builtin_elementwise_fma(u - v, two, mhalf) + mag;
      const h2 dl = __builtin_bit_cast(h2, step ^ ((__builtin_bit_cast(uint32_t, r) << 15) &
                                                   0x80008000u));
      h2 nu = u - dl, nv = v + dl;
      if constexpr (!LAZY) {
        nu = nu - ((nu + mag) - mag);
        nv = nv - ((nv + mag) - mag);
      }
      wu[k] = __builtin_bit_cast(uint32_t, nu);
      wv[k] = __builtin_bit_cast(uint32_t, nv);
    }
  } else if constexpr (ST == COSM_STORE_FIX32) {
    // aJ is an integer of magnitude below 2^31 (|alpha J| < 1/2 turn on the
    // grid): the conversion is exact
    const uint32_t st = (uint32_t)(int32_t)aJ, nst = 0u - st;
#pragma unroll
    for (int k = 0; k < W; k++) {
      const uint32_t dl = (int32_t)(wu[k] - wv[k]) >= 0 ? st : nst;
      wu[k] -= dl;
      wv[k] += dl;
    }
  } else if constexpr (ST == COSM_STORE_FIX16) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    // aJ is an integer (2^-16 turn units) below one turn: the conversion is exact
    const uint32_t st = (uint32_t)(int32_t)aJ & 0xffffu;
    const u16x2 step = __builtin_bit_cast(u16x2, st | (st << 16));
#pragma unroll
    for (int k = 0; k < W; k++) {
      const u16x2 u = __builtin_bit_cast(u16x2, wu[k]), v = __builtin_bit_cast(u16x2, wv[k]);
      const u16x2 m = (u16x2)((s16x2)(u - v) >> (short)15);  // 0xffff where negative
      const u16x2 dl = (step ^ m) - m;                        // +step or -step
      wu[k] = __builtin_bit_cast(uint32_t, (u16x2)(u - dl));
      wv[k] = __builtin_bit_cast(uint32_t, (u16x2)(v + dl));
    }
  } else {
    using F = Fmt<ST>;
    constexpr int RW = W * F::kPerWord;
    float xu[RW], xv[RW];
    F::template unpack<W>(wu, xu);
    F::template unpack<W>(wv, xv);
#pragma unroll
    for (int k = 0; k < RW; k++) pair_update<ST, LAZY, RD>(xu[k], xv[k], aJ, pm);
    F::template pack<W>(xu, wu);
    F::template pack<W>(xv, wv);
  }
}

// Eq. (6) between a row held in registers (r) and one in LDS (w), for every
// replica they hold; flip says that the register vertex is the edge's v (the
// sign of Eq. (4) is taken on x_u - x_v, so the roles matter on ties).  With
// the change written r <- r - D, w <- w + D, the result is the pair update's
// bit for bit: D = delta when r is u, -delta when r is v.
// FIX32 / FIX16: d = r - w - flip (integer units) is >= 0 exactly when D is
// +step: for r = u that is the sign of u - v; for r = v, u - v = -(r - w) has
// the sign bit clear exactly when r - w is not in [1, 1/2 turn].
// FP32 arithmetic: the pair update on (w, r) when flipped, with -(r - w)
// standing for w - r (IEEE subtraction is antisymmetric).  RD (the grid
// schedule, under f32_round_down): the flip folded into the parity fma's
// factor (-2) and into the step's sign, so that D = step_by_parity on
// (r - w) x (-1)^flip with aJ x (-1)^flip.
template <int ST, int W, bool RD = false>
__device__ __forceinline__ void update_reg_words(uint32_t (&r)[W], uint32_t (&w)[W], float aJ,
                                                 uint32_t flip, float pm = 0.0f) {
  if constexpr (ST == COSM_STORE_FIX32) {
    const uint32_t st = (uint32_t)(int32_t)aJ, nst = 0u - st;
#pragma unroll
    for (int k = 0; k < W; k++) {
      const uint32_t D = (int32_t)(r[k] - w[k] - flip) >= 0 ? st : nst;
      r[k] -= D;
      w[k] += D;
    }
  } else if constexpr (ST == COSM_STORE_FIX16) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    const uint32_t st = (uint32_t)(int32_t)aJ & 0xffffu;
    const u16x2 step = __builtin_bit_cast(u16x2, st | (st << 16));
    const u16x2 f2 = __builtin_bit_cast(u16x2, flip * 0x00010001u);
#pragma unroll
    for (int k = 0; k < W; k++) {
      const u16x2 a = __builtin_bit_cast(u16x2, r[k]), b = __builtin_bit_cast(u16x2, w[k]);
      const u16x2 m = (u16x2)((s16x2)(a - b - f2) >> (short)15);  // 0xffff where negative
      const u16x2 D = (step ^ m) - m;
      r[k] = __builtin_bit_cast(uint32_t, (u16x2)(a - D));
      w[k] = __builtin_bit_cast(uint32_t, (u16x2)(b + D));
    }
  } else {
    using F = Fmt<ST>;
    constexpr int RW = W * F::kPerWord;
    float xr[RW], xw[RW];
    F::template unpack<W>(r, xr);
    F::template unpack<W>(w, xw);
#pragma unroll
    for (int k = 0; k < RW; k++) {
      const float e = xr[k] - xw[k];
      float D;
      if constexpr (RD) {
        const float p = __builtin_fmaf(e, flip ? -2.0f : 2.0f, pm);
        D = __uint_as_float((__float_as_uint(p) << 31) + (__float_as_uint(aJ) ^ (flip << 31)));
      } else {
        const float f = fract1(flip ? -e : e);
        const float dl = (f < 0.5f) ? aJ : -aJ;
        D = flip ? -dl : dl;
      }
      xr[k] = F::wrap(xr[k] - D);
      xw[k] = F::wrap(xw[k] + D);
    }
    F::template pack<W>(xr, r);
    F::template pack<W>(xw, w);
  }
}

// Eq. (6) on every replica of one edge: rows at byte offsets bu, bv.
template <int ST, int W, bool LAZY = false, bool RD = false>
__device__ __forceinline__ void edge_rows(uint32_t *lds, uint32_t bu, uint32_t bv, float aJ,
                                          float pm = 0.0f) {
  uint32_t wu[W], wv[W];
  lds_load_at<W>(lds, bu, wu);
  lds_load_at<W>(lds, bv, wv);
  update_words<ST, W, LAZY, RD>(wu, wv, aJ, pm);
  lds_store_at<W>(lds, bu, wu);
  lds_store_at<W>(lds, bv, wv);
}

// The dual window twist on the RW values of one row (membership tested on the
// values given, c and tws per replica).
template <int ST, int RW>
__device__ __forceinline__ void twist_values(float (&x)[RW], const float (&c)[RW],
                                             const float (&tws)[RW], float win2) {
#pragma unroll
  for (int k = 0; k < RW; k++)
    if (in_windows(x[k], c[k], win2)) x[k] = Fmt<ST>::wrap(x[k] + tws[k]);
}

// The twist's per-replica operands prepared once per twist for many rows: the
// fixed-point formats convert the reference offsets and the twist to their
// integer units here instead of at every row.
template <int ST, int W>
struct TwistOps {
  static constexpr int RW = W * Fmt<ST>::kPerWord;
  float c[RW], t[RW], win2;
  __device__ __forceinline__ void set(const float (&cth)[RW], const float (&tws)[RW], float w2) {
#pragma unroll
    for (int k = 0; k < RW; k++) {
      c[k] = cth[k];
      t[k] = tws[k];
    }
    win2 = w2;
  }
  __device__ __forceinline__ void apply(uint32_t (&w)[W]) const {
    using F = Fmt<ST>;
    float x[RW];
    F::template unpack<W>(w, x);
    twist_values<ST, RW>(x, c, t, win2);
    F::template pack<W>(x, w);
  }
};
template <int W>
struct TwistOps<COSM_STORE_FIX32, W> {
  uint32_t c[W], t[W], W2;
  bool all;
  __device__ __forceinline__ void set(const float (&cth)[W], const float (&tws)[W], float w2) {
    all = w2 >= 1.0f;
    W2 = all ? 0u : (uint32_t)(w2 * 4294967296.0f);
#pragma unroll
    for (int q = 0; q < W; q++) {
      c[q] = turns_fix32(cth[q]);
      t[q] = turns_fix32(tws[q]);
    }
  }
  __device__ __forceinline__ void apply(uint32_t (&w)[W]) const {
#pragma unroll
    for (int q = 0; q < W; q++) {
      const uint32_t d = (w[q] << 1) - c[q];
      if (all || d < W2) w[q] += t[q];
    }
  }
};
template <int W>
struct TwistOps<COSM_STORE_FIX16, W> {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  uint32_t c2[W], t2[W], k2;
  bool all;
  __device__ __forceinline__ void set(const float (&cth)[2 * W], const float (&tws)[2 * W],
                                      float w2) {
    const uint32_t W2 = (uint32_t)(w2 * 65536.0f);
    all = W2 >= 65536u;
    const uint32_t k = (W2 - 32768u) & 0xffffu;
    k2 = k | (k << 16);
#pragma unroll
    for (int q = 0; q < W; q++) {
      c2[q] = ((uint32_t)(int32_t)(cth[2 * q] * 65536.0f) & 0xffffu) |
              ((uint32_t)(int32_t)(cth[2 * q + 1] * 65536.0f) << 16);
      t2[q] = ((uint32_t)(int32_t)(tws[2 * q] * 65536.0f) & 0xffffu) |
              ((uint32_t)(int32_t)(tws[2 * q + 1] * 65536.0f) << 16);
    }
  }
  __device__ __forceinline__ void apply(uint32_t (&w)[W]) const {
#pragma unroll
    for (int q = 0; q < W; q++) {
      const u16x2 x = __builtin_bit_cast(u16x2, w[q]);
      const u16x2 t = (u16x2)(x << (unsigned short)1) - __builtin_bit_cast(u16x2, c2[q]);
      const s16x2 sgn = __builtin_bit_cast(s16x2, __builtin_bit_cast(uint32_t, t) ^ 0x80008000u);
      const s16x2 d = __builtin_elementwise_sub_sat(sgn, __builtin_bit_cast(s16x2, k2));
      const u16x2 m = all ? (u16x2)(0xffff) : (u16x2)(d >> (short)15);
      w[q] = __builtin_bit_cast(uint32_t, (u16x2)(x + (__builtin_bit_cast(u16x2, t2[q]) & m)));
    }
  }
};

// Storage formats with a lazy wrap (phases wrapped only at the twists).
constexpr bool lazy_storage(int st) {
  return st == COSM_STORE_FP32 || st == COSM_STORE_FP16 || st == COSM_STORE_BF16 ||
         st == COSM_STORE_FP16_PK;
}

// The twist on one row.  LAZY (phases wrapped only at the twists): the row is
// wrapped first, so the window test is that of the wrapped form, and the
// twisted value x + twist is left unwrapped (it is at most the twist past the
// wrapped range; the host's drift bound counts it).
template <int ST, int W, bool LAZY>
__device__ __forceinline__ void twist_row(const TwistOps<ST, W> &op, uint32_t (&w)[W]) {
  if constexpr (LAZY) {
    static_assert(lazy_storage(ST), "the lazy wrap is a floating-point form");
    using F = Fmt<ST>;
    constexpr int RW = W * F::kPerWord;
    float x[RW];
    F::template unpack<W>(w, x);
#pragma unroll
    for (int k = 0; k < RW; k++) {
      const float y = F::wrap(x[k]);
      x[k] = in_windows(y, op.c[k], op.win2) ? y + op.t[k] : y;
    }
    F::template pack<W>(x, w);
  } else {
    op.apply(w);
  }
}

// The twist on the W words of one row.  FIX16: packed 16-bit integers; with
// t = (2x - c) mod 1 turn in 16-bit lanes, a lane is in the windows iff
// t < 2w: t is moved to signed range (top bit flipped) and compared with
// 2w - 1/2 turn by a saturating subtraction, whose sign gives the mask.
// FIX32: the same test on 32-bit integers.  Other formats: unpack, twist_values,
// pack.
template <int ST, int W>
__device__ __forceinline__ void twist_words(uint32_t (&w)[W],
                                            const float (&c)[W * Fmt<ST>::kPerWord],
                                            const float (&tws)[W * Fmt<ST>::kPerWord],
                                            float win2) {
  TwistOps<ST, W> op;
  op.set(c, tws, win2);
  op.apply(w);
}

// Eq. (6) on every replica of one edge of the last class, followed by the
// twist of both endpoints: their phases are final for the sweep once the
// update is done, so the twist needs no pass of its own for them.  The twist
// sees the stored (rounded) phases, as a pass of its own would.
template <int ST, int W, bool LAZY = false, bool RD = false>
__device__ __forceinline__ void edge_rows_twist(uint32_t *lds, uint32_t bu, uint32_t bv, float aJ,
                                                const TwistOps<ST, W> &op, float pm = 0.0f) {
  uint32_t wu[W], wv[W];
  lds_load_at<W>(lds, bu, wu);
  lds_load_at<W>(lds, bv, wv);
  update_words<ST, W, LAZY, RD>(wu, wv, aJ, pm);
  twist_row<ST, W, LAZY>(op, wu);
  twist_row<ST, W, LAZY>(op, wv);
  lds_store_at<W>(lds, bu, wu);
  lds_store_at<W>(lds, bv, wv);
}

// The twist of one row that no edge of the last class touches.
template <int ST, int W, bool LAZY = false>
__device__ __forceinline__ void row_twist(uint32_t *lds, uint32_t b, const TwistOps<ST, W> &op) {
  uint32_t w[W];
  lds_load_at<W>(lds, b, w);
  twist_row<ST, W, LAZY>(op, w);
  lds_store_at<W>(lds, b, w);
}

// ---------------------------------------------------------------------------
// Block reductions (wave64 shuffles, then one LDS slot per wave).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *scratch /* >= 16 */) {
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

// Eq. (6) on one edge in nsets replica sets that lie set_bytes apart in LDS.
// The sets are disjoint, so the rows of four sets are read before any is
// written back, which lets the LDS latency of one set overlap the arithmetic
// of the others.
template <int ST, int W, bool LAZY = false, bool RD = false>
__device__ __forceinline__ void edge_rows_sets(uint32_t *lds, uint32_t bu, uint32_t bv,
                                               uint32_t set_bytes, int nsets, float aJ,
                                               float pm = 0.0f) {
  int k = 0;
  for (; k + 4 <= nsets; k += 4) {
    uint32_t wu[4][W], wv[4][W];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      lds_load_at<W>(lds, bu + (uint32_t)(k + q) * set_bytes, wu[q]);
      lds_load_at<W>(lds, bv + (uint32_t)(k + q) * set_bytes, wv[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) update_words<ST, W, LAZY, RD>(wu[q], wv[q], aJ, pm);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      lds_store_at<W>(lds, bu + (uint32_t)(k + q) * set_bytes, wu[q]);
      lds_store_at<W>(lds, bv + (uint32_t)(k + q) * set_bytes, wv[q]);
    }
  }
  for (; k < nsets; k++)
    edge_rows<ST, W, LAZY, RD>(lds, bu + (uint32_t)k * set_bytes, bv + (uint32_t)k * set_bytes,
                               aJ, pm);
}

// One workgroup's pass over the classes of one sweep with the lane schedule
// streamed from memory: slot j of thread t is desc[j * nth + t]; Ks[c] (in LDS)
// is the number of slots of class c; a barrier follows every non-empty class.
// Two descriptors are in flight: A holds slot j and B slot j + 1, and each is
// refilled right after use, so a wait only ever covers the descriptor needed
// next.  edge(d) applies Eq. (6) for descriptor d.
template <typename EdgeFn, typename LastFn, typename TailFn>
__device__ __forceinline__ void stream_classes(const EdgeDesc *desc_any, const int32_t *Ks, int C,
                                               int total, EdgeDesc &A, EdgeDesc &B, int &j,
                                               EdgeFn edge, LastFn last, TailFn tail,
                                               bool fuse_now) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const gptr<EdgeDesc> desc = as_global(desc_any) + tid;
  // slot x <= total + 1: the schedule repeats its first slots after the last,
  // so the prefetch of the next sweep's first slots needs no wrap
  auto at = [&](int x) {
    const gptr<EdgeDesc> p = desc + (uint32_t)(x * nth);
    return EdgeDesc{p->slots, p->J};
  };
  auto run = [&](int kc, auto &&fn) {
    int k = 0;
    for (; k + 2 <= kc; k += 2, j += 2) {
      if (A.slots != kEmptySlot) fn(A);
      A = at(j + 2);
      if (B.slots != kEmptySlot) fn(B);
      B = at(j + 3);
    }
    if (k < kc) {
      if (A.slots != kEmptySlot) fn(A);
      A = B;
      B = at(j + 2);
      j += 1;
    }
  };
  for (int c = 0; c < C - 1; c++) {
    const int kc = __builtin_amdgcn_readfirstlane(Ks[c]);
    run(kc, edge);
    if (kc > 0) __syncthreads();
  }
  const int kl = __builtin_amdgcn_readfirstlane(Ks[C - 1]);
  if (fuse_now) {  // the last class with its twist, and the rows it leaves out
    run(kl, last);
    tail();
    __syncthreads();
  } else {
    run(kl, edge);
    if (kl > 0) __syncthreads();
  }
  j -= total;  // exactly one pass over the slots: keep j in [0, total)
}

template <typename EdgeFn>
__device__ __forceinline__ void stream_classes(const EdgeDesc *desc_any, const int32_t *Ks, int C,
                                               int total, EdgeDesc &A, EdgeDesc &B, int &j,
                                               EdgeFn edge) {
  stream_classes(desc_any, Ks, C, total, A, B, j, edge, edge, [] {}, false);
}

// Arguments of the readout of one instance (phases [n][R]).
struct ReadoutArgs {
  const void *phases;
  const int32_t *eu, *ev, *J, *h;
  uint16_t *code_global;  // [R][n] bisector codes in device memory, or null: in LDS
  int8_t *spins;
  int64_t *H, *cut;
  int32_t *best_p;
  int32_t n, R, B, grid;
  int64_t m;
};

// Readout, Algorithm 1 binarization, of replica r by one workgroup.  Bisector p
// is beta_p (increasing, beta_0 = 0); spin i is +1 on [beta_p, beta_p + 1/2).
// With x in [0,1): s_i(0) = +1 iff x < 1/2, and spin i flips exactly once, at
// q_i = #{p : beta_p <= y_i}, y_i = x_i mod 1/2.  An edge's term -J s_u s_v thus
// changes sign at min(q_u, q_v) and back at max(q_u, q_v): a difference array
// over p gives every H_p in O(n + m + B).  sm64: dynamic LDS of
// readout_lds_bytes(n, B) bytes (readout_lds_bytes(0, B) when the codes live
// in device memory, for n too large for LDS).
template <int ST>
__device__ void readout_block(const ReadoutArgs &a, int r, int64_t *sm64) {
  using F = Fmt<ST>;
  int64_t *red = sm64;            // 16
  int64_t *bins = sm64 + 16;      // B + 1
  float *beta = reinterpret_cast<float *>(bins + a.B + 1);  // B
  uint16_t *code = a.code_global != nullptr ? a.code_global + (size_t)r * a.n
                                             : reinterpret_cast<uint16_t *>(beta + a.B);  // n
  const int tid = threadIdx.x, nth = blockDim.x;
  const int B = a.B;
  int64_t &s_best = red[14];
  int64_t &s_bp = red[15];

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
  const int bp = (int)s_bp;
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

}  // namespace
}  // namespace cosm
