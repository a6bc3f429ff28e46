// sweep_reg.hip -- the register-owner form of the LDS-resident sweep
// (k_sweep_reg) and its launchers, in a translation unit of their own.
#include <hip/hip_runtime.h>

#include <string>

#include "device_common.hpp"
#include "internal.hpp"
#include "lds_args.hpp"

namespace cosm {
namespace {

// ---------------------------------------------------------------------------
// The register-owner form of the LDS sweep: thread t keeps K vertices of an
// independent set in registers (RW replicas each, as W words) and applies
// every edge incident to them, reading and writing only the other endpoint's
// LDS row; edges between two LDS rows take one pair-form slot per class.  The
// classes (at most CM) run in order with a barrier after each, as in
// k_sweep_lds (CLASSES > 0: exactly that many, else a.C); the schedule is held
// in registers; lanes without an edge use dummy rows with J = 0.  The twist visits the LDS rows (all threads) and the
// register rows (their owner), after the last class.
// ---------------------------------------------------------------------------
template <int ST, int W, int K, int CM, int CLASSES, bool FUSE, bool RD>
__global__ void __launch_bounds__(1024) k_sweep_reg(const LdsArgs a) {
  static_assert(!FUSE || CLASSES == CM, "the fused twist needs the exact class count");
  static_assert(!RD || ST == COSM_STORE_FP32, "the parity step is an FP32 grid form");
  extern __shared__ uint32_t lds[];
  using F = Fmt<ST>;
  constexpr int RW = W * F::kPerWord;
  constexpr uint32_t ROWB = 4 * W;
  const int tid = threadIdx.x, nth = blockDim.x;
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
  float *theta_buf = reinterpret_cast<float *>(lds + (size_t)(a.n_rows + kDummyRows) * W);
  // HBM -> register rows
  uint32_t reg[K][W];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int32_t v = a.reg_vertex[k * nth + tid];
    float x[RW];
#pragma unroll
    for (int q = 0; q < RW; q++)
      x[q] = (v >= 0 && q < nvalid) ? F::load_elem(a.phases, (size_t)v * a.R + r0 + q) : 0.0f;
    F::template pack<W>(x, reg[k]);
  }
  // the schedule: [C][K + 1][nth]; a register slot keeps its row's byte offset
  // (a multiple of 4) with the role flag in bit 0
  uint32_t row[CM][K], fuv[CM];
  float jr[CM][K], jf[CM];
#pragma unroll
  for (int c = 0; c < CM; c++) {
    const bool on = c < a.C;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const EdgeDesc d = on ? a.desc[(size_t)(c * (K + 1) + k) * nth + tid] : EdgeDesc{0u, 0.0f};
      row[c][k] = (d.slots & 0xffffu) * ROWB | ((d.slots >> 16) & 1u);
      jr[c][k] = d.J;
    }
    const EdgeDesc d = on ? a.desc[(size_t)(c * (K + 1) + K) * nth + tid] : EdgeDesc{0u, 0.0f};
    fuv[c] = d.slots;  // u | v << 16 (rows)
    jf[c] = d.J;
  }
  // the pair slot's edges sit in the first lanes: a wave with none of them in
  // a class skips that slot (its other lanes hold no-op dummy edges)
  uint32_t wave_free = 0;
#pragma unroll
  for (int c = 0; c < CM; c++)
    if (__ballot(a.reg_free && jf[c] != 0.0f) != 0ull) wave_free |= 1u << c;
  __syncthreads();

  SweepSchedule sc = a.sch;
  const uint32_t nsw = (uint32_t)a.nsw;
  uint32_t t = (uint32_t)a.t0;
  uint32_t tw = 0;
  ScheduleChunk chunk;
  // RD: every operation of the sweeps is exact (the grid schedule)
  float pm = 0.0f;
  if constexpr (RD) pm = f32_round_down();
  for (uint32_t it = 0; it < nsw; it++) {
    t++;
    if ((it & 63u) == 0u) chunk.fill(sc, t);
    float alpha, twist;
    chunk.get(it & 63u, alpha, twist);
    const float alpha_s = alpha * F::kStepScale;
    // FUSE: on a twist sweep the last class twists every LDS row as it updates
    // it (the schedule touches each exactly once there) and the owners twist
    // the register rows after it
    bool fuse_now = false;
    TwistOps<ST, W> tops;
    if constexpr (FUSE) {
      fuse_now = chunk.twist_at(it & 63u);
      if (fuse_now) {
        const int slot = (int)(tw % (uint32_t)kThetaChunk);
        if (slot == 0) {
          theta_fill(theta_buf, nullptr, kThetaChunk, RW, t, sc.period, a.rid0 + (uint32_t)r0,
                     a.k0, a.k1, sc.win, sc.tshift, sc.tscale);
          __syncthreads();
        }
        tw++;
        float cth[RW], tws[RW];
#pragma unroll
        for (int k = 0; k < RW; k++) {
          cth[k] = theta_buf[slot * RW + k];
          tws[k] = twist;
        }
        tops.set(cth, tws, sc.win2);
      }
    }
#pragma unroll
    for (int c = 0; c < CM; c++) {
      if (c < CLASSES || (CLASSES == 0 && c < a.C)) {
        const bool last_twist = FUSE && c == CM - 1 && fuse_now;
        const bool fon = __builtin_amdgcn_readfirstlane((wave_free >> c) & 1u) != 0u;
        uint32_t w[K][W], pu[W], pv[W];
#pragma unroll
        for (int k = 0; k < K; k++) lds_load_at<W>(lds, row[c][k] & ~1u, w[k]);
        if (fon) {
          lds_load_at<W>(lds, (fuv[c] & 0xffffu) * ROWB, pu);
          lds_load_at<W>(lds, (fuv[c] >> 16) * ROWB, pv);
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
          update_reg_words<ST, W, RD>(reg[k], w[k], alpha_s * jr[c][k], row[c][k] & 1u, pm);
          if (last_twist) tops.apply(w[k]);
          lds_store_at<W>(lds, row[c][k] & ~1u, w[k]);
        }
        if (fon) {
          update_words<ST, W, false, RD>(pu, pv, alpha_s * jf[c], pm);
          if (last_twist) {
            tops.apply(pu);
            tops.apply(pv);
          }
          lds_store_at<W>(lds, (fuv[c] & 0xffffu) * ROWB, pu);
          lds_store_at<W>(lds, (fuv[c] >> 16) * ROWB, pv);
        }
        __syncthreads();
      }
    }
    if constexpr (FUSE) {
      if (fuse_now) {
#pragma unroll
        for (int k = 0; k < K; k++) tops.apply(reg[k]);
      }
    } else if (chunk.twist_at(it & 63u)) {
      const int slot = (int)(tw % (uint32_t)kThetaChunk);
      if (slot == 0) {
        theta_fill(theta_buf, nullptr, kThetaChunk, RW, t, sc.period, a.rid0 + (uint32_t)r0,
                   a.k0, a.k1, sc.win, sc.tshift, sc.tscale);
        __syncthreads();
      }
      tw++;
      float cth[RW], tws[RW];
#pragma unroll
      for (int k = 0; k < RW; k++) {
        cth[k] = theta_buf[slot * RW + k];
        tws[k] = twist;
      }
      TwistOps<ST, W> op;
      op.set(cth, tws, sc.win2);
#pragma unroll
      for (int k = 0; k < K; k++) op.apply(reg[k]);
      for (int s0 = tid; s0 < a.n_rows; s0 += 4 * nth) {
        uint32_t w[4][W];
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (s0 + q * nth < a.n_rows) lds_load<W>(lds, s0 + q * nth, w[q]);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          if (s0 + q * nth < a.n_rows) {
            op.apply(w[q]);
            lds_store<W>(lds, s0 + q * nth, w[q]);
          }
        }
      }
      __syncthreads();
    }
  }
  if constexpr (RD) f32_round_nearest();

  // register rows and LDS rows -> HBM
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int32_t v = a.reg_vertex[k * nth + tid];
    if (v < 0) continue;
    float x[RW];
    F::template unpack<W>(reg[k], x);
#pragma unroll
    for (int q = 0; q < RW; q++)
      if (q < nvalid) F::store_elem(a.phases, (size_t)v * a.R + r0 + q, x[q]);
  }
  for (int s = tid; s < a.n_rows; s += nth) {
    const int32_t v = a.slot_vertex[s];
    if (v < 0) continue;
    uint32_t w[W];
    lds_load<W>(lds, s, w);
    float x[RW];
    F::template unpack<W>(w, x);
#pragma unroll
    for (int k = 0; k < RW; k++)
      if (k < nvalid) F::store_elem(a.phases, (size_t)v * a.R + r0 + k, x[k]);
  }
}

int launch_check(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    return set_error(COSM_EDEVICE, std::string(what) + ": " + hipGetErrorString(err));
  return COSM_OK;
}

template <int ST, int W, int K, int CM, int CLASSES, bool FUSE, bool RD>
int launch_reg_k(cosm_state *s, const LdsArgs &a) {
  const size_t lds = s->shape.lds_bytes;
  (void)hipFuncSetAttribute((const void *)k_sweep_reg<ST, W, K, CM, CLASSES, FUSE, RD>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_sweep_reg<ST, W, K, CM, CLASSES, FUSE, RD>), dim3(s->shape.blocks),
                     dim3(s->shape.threads), lds, s->stream, a);
  return launch_check("k_sweep_reg");
}

// FP32 on the grid schedule: the parity step
template <int ST, int W, int K, int CM, int CLASSES = 0, bool FUSE = false>
int launch_reg(cosm_state *s, const LdsArgs &a) {
  if constexpr (ST == COSM_STORE_FP32) {
    if (exact_grid_fp32(*s)) return launch_reg_k<ST, W, K, CM, CLASSES, FUSE, true>(s, a);
  }
  return launch_reg_k<ST, W, K, CM, CLASSES, FUSE, false>(s, a);
}

// The register-owner form exists for the formats whose update is exact for
// any input (FP32, and the fixed-point formats), with up to 8 classes (4 and
// 2 register rows per thread) or 4 classes (4 rows).
template <int ST, int W>
int launch_reg_w(cosm_state *s, const LdsArgs &a) {
  if constexpr (ST == COSM_STORE_FP32 || ST == COSM_STORE_FIX32 || ST == COSM_STORE_FIX16) {
    const int K = s->lds.reg_k;
    if (lds_twist_fused(*s)) {
      if (K == 1) return launch_reg<ST, W, 1, 4, 4, true>(s, a);
      if (K == 2) return launch_reg<ST, W, 2, 4, 4, true>(s, a);
      if (K == 4) return launch_reg<ST, W, 4, 4, 4, true>(s, a);
    } else if (a.C == 4) {
      if (K == 1) return launch_reg<ST, W, 1, 4, 4>(s, a);
      if (K == 2) return launch_reg<ST, W, 2, 4, 4>(s, a);
      if (K == 4) return launch_reg<ST, W, 4, 4, 4>(s, a);
    } else if (a.C < 4) {
      if (K == 1) return launch_reg<ST, W, 1, 4>(s, a);
      if (K == 2) return launch_reg<ST, W, 2, 4>(s, a);
      if (K == 4) return launch_reg<ST, W, 4, 4>(s, a);
    } else if (a.C <= 8) {
      if (K == 1) return launch_reg<ST, W, 1, 8>(s, a);
      if (K == 2) return launch_reg<ST, W, 2, 8>(s, a);
    }
    return set_error(COSM_EINVAL, "register form: unsupported register count or classes");
  } else {
    (void)s;
    (void)a;
    return set_error(COSM_EINVAL, "register form: unsupported storage");
  }
}

}  // namespace

int launch_sweeps_reg(cosm_state *s, const LdsArgs &a, int W) {
  switch (s->p.storage) {
    case COSM_STORE_FP32:
      if (W == 4) return launch_reg_w<COSM_STORE_FP32, 4>(s, a);
      if (W == 2) return launch_reg_w<COSM_STORE_FP32, 2>(s, a);
      if (W == 1) return launch_reg_w<COSM_STORE_FP32, 1>(s, a);
      break;
    case COSM_STORE_FIX32:
      if (W == 4) return launch_reg_w<COSM_STORE_FIX32, 4>(s, a);
      if (W == 2) return launch_reg_w<COSM_STORE_FIX32, 2>(s, a);
      if (W == 1) return launch_reg_w<COSM_STORE_FIX32, 1>(s, a);
      break;
    case COSM_STORE_FIX16:
      if (W == 4) return launch_reg_w<COSM_STORE_FIX16, 4>(s, a);
      if (W == 2) return launch_reg_w<COSM_STORE_FIX16, 2>(s, a);
      if (W == 1) return launch_reg_w<COSM_STORE_FIX16, 1>(s, a);
      break;
    default:
      return set_error(COSM_EINVAL, "register form: unsupported storage");
  }
  return set_error(COSM_EINVAL, "unsupported replicas per workgroup");
}

}  // namespace cosm
