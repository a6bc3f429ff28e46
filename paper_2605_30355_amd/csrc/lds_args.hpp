// lds_args.hpp -- the arguments of the LDS-resident sweep kernels of
// kernels.hip (the pair form) and sweep_reg.hip (the register-owner form),
// and the launcher of the latter.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace cosm {

struct LdsArgs {
  void *phases;
  const EdgeDesc *desc;       // [total_slots * nth] lane schedule
  const int32_t *Kc;          // [C] slots per thread of each class
  const int32_t *slot_vertex; // [n_rows]
  const int32_t *h_slot;      // [n_rows] bias field per slot, or null (no fields)
  int32_t R, n_rows, C, total_slots;
  int64_t t0, nsw;
  SweepSchedule sch;
  uint32_t k0, k1, rid0;
  uint32_t bar_mask;          // register-resident schedule: barrier after slot j
  // fused form: the twist runs inside the last class's sub-sweep, with fuse_k
  // rows per thread (after the repeated slots in desc) that no edge of that
  // class touches
  int32_t fuse_k;
  // register-owner form: [K][nth] register vertices, and whether the slot of
  // edges between two LDS rows is in use
  const int32_t *reg_vertex;
  int32_t reg_free;
};

// The register-owner form's sweeps for the state's storage and W words per
// row (sweep_reg.hip); COSM_EINVAL for a storage, register count or class
// count that has no kernel.
int launch_sweeps_reg(cosm_state *s, const LdsArgs &a, int W);

}  // namespace cosm
