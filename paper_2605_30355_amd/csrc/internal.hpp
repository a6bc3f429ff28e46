// internal.hpp -- declarations shared by the host side of libcosm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cosm.h"

namespace cosm {

// ---- errors ------------------------------------------------------------------
// Every entry point returns a status; set_error records the message for
// cosm_last_error() on the calling thread.
int set_error(int status, const std::string &msg);
void clear_error();

#define COSM_HIP_CHECK(expr)                                                              \
  do {                                                                                    \
    hipError_t err_ = (expr);                                                             \
    if (err_ != hipSuccess)                                                               \
      return ::cosm::set_error(COSM_EDEVICE, std::string(#expr) + ": " +                  \
                                                 hipGetErrorString(err_));                \
  } while (0)

// ---- graph checks and colourings (graph.cpp) --------------------------------------
// EINVAL / EDUP with a message, or COSM_OK.  Fills degree[n] when non-null.
int validate_graph(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                   std::vector<int32_t> *degree);
// ECOLOR unless colour[] is a proper colouring with classes 0..C-1.
int validate_colouring(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                       const int32_t *colour, int32_t C);
int32_t colour_greedy(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                      int32_t *colour);
int32_t colour_misra_gries(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                           int32_t *colour);
void equalise_classes(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, int32_t C,
                      int32_t *colour);
// Misra-Gries, then Kempe-chain moves towards Delta colours; returns C.
int32_t colour_minimum(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                       int32_t *colour);
// Returns C, or a negative status for a non-lattice edge.
int32_t colour_torus(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, int32_t Lx,
                     int32_t Ly, int32_t *colour);

// ---- phase and schedule encoding ----------------------------------------------------
// Phases are turns.  The grid quantum is 2^-23 turn; step sizes live on the
// 2^-22 grid so that half a step stays on the 2^-23 grid.
constexpr double kTwo23 = 8388608.0;
constexpr double kTwo22 = 4194304.0;

// Scalars a sweep kernel needs to evaluate the schedule of sweep t on the device.
struct Schedule {
  int32_t grid;          // COSM_SCHED_GRID ?
  int64_t S;             // schedule length
  // grid: alpha_units(t) = floor((a0 * (S - t + 1) + S/2) / S), units of aunit
  int64_t a0_units;
  int32_t twist_num2;    // 2 * dwt_ratio (grid)
  // continuous
  float alpha0_turns;
  float dwt_ratio;
  int32_t dwt_period;    // 0: never
  float window2;         // 2 * window width in turns (membership threshold)
  float window;          // window width in turns
  // grid units: alpha = q * aunit, twist = twist_num2 * q * tunit; reference
  // angles (w >> tshift) * tscale and initial phases (w >> ishift) * iscale
  // from a 32-bit draw w (2^-23 grid; 2^-16 for FIX16; 24-bit continuous init)
  float aunit, tunit, tscale, iscale;
  int32_t tshift, ishift;
};

// EINVAL unless every field of *p is in range.
int check_params_public(const cosm_params *p);
// Validates the schedule parameters against the couplings and fills *sc.
int make_schedule(const cosm_params &p, int32_t max_abs_J, Schedule *sc);

// ---- the device-side problem description -----------------------------------------
// Per-class edge descriptors for the LDS kernel: 32-bit word of LDS slots
// (slot_u | slot_v << 16) and the coupling as a float.
struct EdgeDesc {
  uint32_t slots;
  float J;
};
constexpr uint32_t kEmptySlot = 0xffffffffu;  // masked lane

// Lane schedule of the LDS-resident sweep (schedule.cpp).  Entry (j, t) of
// desc is thread t's edge in its j-th slot; slots run class by class, K[c]
// per class, and a workgroup barrier follows the last slot of every class.
struct LdsSchedule {
  int32_t G = 0;                   // lanes per LDS cycle for the row width
  int32_t n_rows = 0;              // LDS rows (slots)
  int32_t nth = 0;                 // threads per workgroup
  int32_t total_slots = 0;
  int64_t pad_entries = 0;         // masked lanes added by the schedule
  std::vector<int32_t> slot_vertex;  // [n_rows] vertex of each slot
  std::vector<int32_t> K;          // [C] slots per thread for each class
  std::vector<int32_t> padded;     // [C] padded list length of each class
  // [(total_slots + kStreamRepeat + fuse_k) * nth]: the slots, the first
  // kStreamRepeat slots again (mod total_slots), then the rows below
  std::vector<EdgeDesc> desc;
  // Rows that no edge of the last class touches, fuse_k per thread, stored in
  // desc after the repeated slots (slots = row, kEmptySlot for none).  They let
  // the twist run inside the last class's sub-sweep; fuse is false when they
  // would need more than kFuseRowsMax per thread (beyond that a pass of its own
  // with four rows in flight is faster).
  bool fuse = false;
  int32_t fuse_k = 0;
  bool dummy_pairs = false;  // masked lanes carry dummy-row no-op edges
  // Register-owner form (reg_k > 0): an independent set of vertices lives in
  // registers, reg_k per thread (reg_vertex [reg_k][nth], -1 for none); every
  // edge with an endpoint there is updated by that endpoint's thread, touching
  // LDS for the other endpoint only.  desc is [C][reg_k + 1][nth]: per class
  // the reg_k register slots (row of the LDS endpoint | flip << 16, where flip
  // = the register vertex is the edge's v), then one slot of an edge between
  // two LDS rows (the pair form's encoding), used when reg_free is 1.  Lanes
  // without an edge carry a dummy row with J = 0.  Rows: slot_vertex, -1 for
  // padding; n_rows is a multiple of 64 and the dummy rows follow it.
  // Streamed word form (stream = true; schedules longer than the register-
  // resident ones, no bias fields): the schedule again as two 32-bit words per
  // lane and slot in sdesc, (u_off | Jneg << 31, v_off), where u_off / v_off
  // are the LDS byte offsets of the rows (row * 4 W) and Jneg the sign bit of
  // J; masked lanes hold dummy-row pairs (J = 0).  Class c keeps its K[c]
  // slots, padded to an even number (an added slot holds dummy pairs and is
  // never run), stotal slots in all, then kWordRepeat repeated slots, then the
  // rows outside the last class as (row_off, 0).  For odd K[c] the last slot
  // holds entries in its first last_lanes[c] lanes only (later waves skip it;
  // for even K[c] last_lanes[c] = nth: the final pair runs on every wave).
  // With junit every |J| equals jscale; otherwise sjmag holds |J| per entry of
  // the slots and the repeated slots.
  bool stream = false;
  bool junit = true;
  float jscale = 1.0f;
  int32_t stotal = 0;
  std::vector<uint32_t> sdesc;
  std::vector<float> sjmag;
  std::vector<int32_t> last_lanes;
  // Streamed register-owner form (rstream = true; the large graphs): reg_k
  // (8, 10, 12 or 16) register rows per thread as above, with the schedule
  // streamed from memory instead of held in registers.  Only the classes in
  // which at least half of the register set has an edge have register slots
  // (register classes); a vertex with an edge in another class stays in LDS.
  // rs_words [register classes][reg_k][nth][2]: per register slot (row byte
  // offset of the LDS endpoint | flip << 31, J as a float, 0 for a lane
  // without an edge there, whose row is then a dummy row); rs_pwords
  // [C][kRStreamPairs][nth][2]: up to kRStreamPairs slots of edges between two
  // LDS rows per class (u row offset | J << 18, v row offset; |J| < 2^13),
  // dummy-row pairs with J = 0 where a lane has none; rs_act [C][nth / 64]:
  // per class and wave, bit 0 set in a register class and bit 1 + p when pair
  // slot p holds an edge in some lane of the wave (a wave skips the others).
  // Row offsets are below 2^18 bytes.
  bool rstream = false;
  std::vector<uint32_t> rs_words;
  std::vector<uint32_t> rs_pwords;
  std::vector<uint32_t> rs_act;
  int32_t reg_k = 0;
  int32_t reg_free = 0;
  std::vector<int32_t> reg_vertex;
  int64_t reg_set = 0;          // size of the independent set before any cut to K nth
  int64_t reg_edges = 0;        // edges with an endpoint in registers
  int64_t reg_conflicts = 0;    // lane groups whose rows share a bank (extra LDS cycles)
};
constexpr int32_t kRegKMax = 4;
// Streamed register-owner form: register rows per thread (one of 8, 12, 16),
// pair slots per class, classes.
constexpr int32_t kRStreamKMax = 16;
constexpr int32_t kRStreamPairs = 4;
constexpr int32_t kRStreamClassesMax = 32;
constexpr int32_t kRegClassesMax = 8;
constexpr int32_t kRegRowsSlack = 4096;  // slot_vertex capacity beyond n
constexpr int32_t kRegisterSlotsMax = 16;  // schedules this short stay in registers
constexpr int32_t kFuseRowsMax = 4;
constexpr int32_t kStreamRepeat = 3;
// Streamed word form: every class is padded to a multiple of kWordGroup
// slots (the sweep kernel runs them in pairs); kWordRepeat slots repeat after
// the last, for the words fetched two slots ahead.
constexpr int32_t kWordGroup = 2;
constexpr int32_t kWordRepeat = 2;

struct DeviceBuffers {
  void *phases = nullptr;       // [n][R] float or 16-bit, replica-major
  EdgeDesc *desc = nullptr;     // LDS-form descriptors, grouped by class
  int32_t *class_off = nullptr; // [2C + 1]: slots per class, then (streamed form) last_lanes
  float *jmag = nullptr;        // streamed word form: |J| per schedule entry (non-uniform |J|)
  int32_t *slot_vertex = nullptr; // [n_slots] vertex held by each LDS slot
  int32_t *reg_vertex = nullptr;  // [kRStreamKMax * 1024] register-owner forms
  uint32_t *rs_words = nullptr;   // streamed register-owner form: its three tables
  uint32_t *rs_pwords = nullptr;
  uint32_t *rs_act = nullptr;
  int32_t *h_slot = nullptr;    // [n_slots] bias field of the vertex in each slot (with h)
  int32_t *eu = nullptr;        // [m] (original ids)
  int32_t *ev = nullptr;
  int32_t *J = nullptr;
  int32_t *h = nullptr;         // [n] or null
  int32_t *peu = nullptr;       // [m] edges grouped by class, original ids (plain / HBM forms)
  int32_t *pev = nullptr;
  float *pJ = nullptr;
  int8_t *spins = nullptr;      // [R][n]
  uint16_t *codes = nullptr;    // [R][n] readout codes when n is too large for LDS, else null
  int64_t *H = nullptr;         // [R]
  int64_t *cut = nullptr;       // [R]
  int32_t *best_p = nullptr;    // [R]
  // full-gradient form: incidence lists and a second phase buffer
  int32_t *inc_off = nullptr;   // [n+1]
  uint32_t *inc_nbr = nullptr;  // [2m] neighbour | (1u << 31 when the vertex is the edge's u)
  float *inc_J = nullptr;       // [2m]
  void *phases_alt = nullptr;   // [n][R]
  // optimal-bisector readout: sort keys and values [R][n] (twice), segment
  // offsets [R + 1], the sort's temporary storage
  uint32_t *opt_keys = nullptr, *opt_keys2 = nullptr, *opt_vals = nullptr, *opt_vals2 = nullptr;
  int32_t *opt_off = nullptr;
  void *opt_temp = nullptr;
};

struct KernelShape {
  int32_t residency = COSM_RES_LDS;
  int32_t rw = 1;          // replicas per workgroup (LDS form)
  int32_t threads = 256;
  int32_t blocks = 1;
  int32_t lds_bytes = 0;
};

}  // namespace cosm

// The state behind the opaque handle.
struct cosm_state {
  int32_t n = 0, C = 0, R = 0;
  int64_t m = 0;
  cosm_params p{};
  uint64_t seed = 0;
  int64_t rid0 = 0;   // global index of replica 0
  int64_t t = 0;      // sweeps done
  hipStream_t stream = nullptr;
  bool own_memory = false;
  void *base = nullptr;
  size_t base_bytes = 0;
  cosm::DeviceBuffers d;
  cosm::KernelShape shape;
  cosm::Schedule sched{};
  int32_t n_slots = 0;
  int32_t max_class = 0;
  cosm::LdsSchedule lds;  // resolved lane schedule of the LDS form
  std::vector<int32_t> lds_widths;  // row widths (words) that fit, for the autotuner
  bool has_h = false;
  int64_t sumJ = 0;                 // sum of J over the edges
  int64_t wdeg_max = 0;             // largest sum of |J| (and |h|) at one vertex
  size_t opt_temp_bytes = 0;        // segmented sort workspace (optimal readout)
  std::vector<int32_t> h_eu, h_ev, h_J, h_h, h_colour;
  std::vector<int32_t> h_slot;       // h of the vertex in each LDS slot (host copy)
  std::vector<int32_t> class_sizes;  // edges per class
  std::vector<int32_t> class_begin;  // offset of each class in the grouped edge arrays
  // timing
  bool timing = false;
  int64_t launches = 0;
  double kernel_ms = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // device whose static scratch array holds the buffers (cosm_init_static), or -1
  int32_t static_dev = -1;
};

namespace cosm {
// ---- state creation (api.cpp) ------------------------------------------------------
// cosm_init with the buffers in device_workspace (or, when it is null, one
// hipMalloc of the library's).  static_dev >= 0: the workspace is that
// device's static scratch array; the shape is then chosen without the timed
// autotuner and no HIP event is created, so the call allocates nothing.
int init_state(cosm_state **out, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
               const int32_t *J, const int32_t *h, const int32_t *colour, int32_t num_colours,
               const cosm_params *p, uint64_t seed, int32_t replicas, void *hip_stream,
               void *device_workspace, size_t workspace_bytes, int32_t static_dev);
// Releases the static scratch array of a device held by a state (static_scratch.hip).
void release_static_scratch(int32_t dev);

// ---- kernel launchers (kernels.hip) -------------------------------------------------
int launch_init(cosm_state *s);
int launch_sweeps(cosm_state *s, int64_t n_sweeps);
// Whether the LDS sweep of s runs the twist inside the last class's sub-sweep
// (the launchers pick the fused kernel forms by this test).
bool lds_twist_fused(const cosm_state &s);
// Whether the sweeps of s keep phases unwrapped between twists: FP32 in the
// streamed LDS forms on the grid schedule (exact), FP16 / BF16 / FP16_PK in every form
// (lazy16) -- in both cases only while no phase can drift by 1/2 turn from its
// wrapped range between two twists (sweep_stream.hip, kernels.hip).
bool lds_lazy_wrap(const cosm_state &s);
bool lazy16(const cosm_state &s);
// Whether every phase operation of the sweeps of s is exact in FP32 (FP32
// storage on the grid schedule: phases on the 2^-23 turn grid, steps and twists
// on the 2^-22 grid, |alpha J| below a turn): the LDS kernels then take the
// step's sign from the parity of floor(2(x_u - x_v)) under round-toward-minus-
// infinity (step_by_parity, kernels.hip, sweep_stream.hip, batch.hip).
bool exact_grid_fp32(const cosm_state &s);
// The same for the streamed pair form, which also takes the parity step for
// FP16 and BF16 storage on the grid (their values are on the same grid; the
// conversions that round them on store keep rounding to nearest even).
bool grid_parity_step(const cosm_state &s);
// That drift bound in turns: the largest twist plus period x the largest step
// x the largest sum of |J| and |h| at one vertex.
double wrap_drift_turns(const cosm_state &s);
int launch_readout(cosm_state *s);
// Optimal-bisector readout (readout_opt.hip); h must be absent.
int launch_readout_optimal(cosm_state *s);
size_t opt_readout_temp_bytes(int32_t n, int32_t R);
constexpr int32_t kOptReadoutMaxN = 32768;  // difference array of n + 1 ints in LDS
int launch_energy(cosm_state *s);  // spins already in s->d.spins
// Convert between the storage format and FP32 turns in [0, 1), both [n][R].
int launch_to_turns(cosm_state *s, float *turns_dev);
int launch_from_turns(cosm_state *s, const float *turns_dev);
int lds_capacity_bytes();
// dummy_pairs: masked lanes of a register-resident schedule get conflict-free
// no-op edges between dummy rows (only for the single-instance sweep kernel,
// whose LDS holds the dummy rows).
// allow_stream: long schedules without bias fields take the streamed word
// form (needs dummy_pairs); false keeps the classic streamed schedule.
int build_lds_schedule(const cosm_state &s, int32_t W, int32_t nth_request, LdsSchedule *out,
                       bool dummy_pairs = false, bool allow_stream = true);
// The streamed word form's sweep (sweep_stream.hip), for states whose schedule
// has it (lds.stream).
int launch_sweeps_stream(cosm_state *s, int64_t n_sweeps);
// Register-owner schedule (see LdsSchedule) for rows of W words, K register
// vertices per thread and nth_request threads (0: as many as the register
// vertices need).  COSM_ERANGE when the form does not apply (more than
// kRegClassesMax classes, bias fields, more edges outside the register set
// than one slot per class holds, too many rows).
int build_reg_schedule(const cosm_state &s, int32_t W, int32_t K, int32_t nth_request,
                       LdsSchedule *out);
// The streamed register-owner schedule (reg_k = 8, 12 or 16 register rows per
// thread, the fewest that hold the independent set, at most kRStreamKMax).
int build_rstream_schedule(const cosm_state &s, int32_t W, int32_t nth_request,
                           LdsSchedule *out);
// The LDS bytes of the streamed register-owner sweep for a schedule.
size_t rstream_lds_bytes(const LdsSchedule &L, int W, int32_t C);
// Whether the streamed register-owner kernel exists for this storage, row
// width and register count (sweep_rstream.hip).
bool rstream_shape_supported(int32_t storage, int32_t W, int32_t K);
int launch_sweeps_rstream(cosm_state *s, int64_t n_sweeps);
// Whether the register form applies (storage, classes, fields, update), a
// register schedule checked against the LDS capacity, and the fewest register
// rows per thread that give one for row width W.
bool reg_form_supported(const cosm_state &s);
int reg_schedule_for(const cosm_state &s, int32_t W, int32_t K, int32_t nth, LdsSchedule *out);
int pick_reg_schedule(cosm_state *s, int32_t W, int32_t nth);
// The streamed register-owner schedule checked against the kernels that exist
// and the LDS capacity.
int rstream_schedule_for(const cosm_state &s, int32_t W, int32_t nth, LdsSchedule *out);
// Measure candidate LDS shapes (row widths in words) and keep the fastest.
int autotune_lds_shape(cosm_state *s, const std::vector<int32_t> &widths);
// Uploads the bias field in LDS-slot order (no-op without bias fields).
int upload_h_slot(cosm_state *s);
// Uploads s->lds (the schedule in the kernel's encoding, the slots per class,
// the slot map, the register rows and the slot-ordered fields); synchronises.
int upload_lds_schedule(cosm_state *s);
// Reference angles of the dual window twist are drawn kThetaChunk twists at a
// time into an LDS table of kThetaChunk x (at most 8) floats, followed by a
// table of the same size for the twist directions (bias fields).
constexpr int kThetaChunk = 32;
constexpr int kThetaFloats = kThetaChunk * 8;

// Rows after the n_rows vertex rows that masked lanes of the single-instance
// sweep read and write instead of branching around their update (J = 0).
constexpr int kDummyRows = 64;
// LDS bytes of the sweep kernel: the vertex and dummy rows, the table of
// reference angles and the slot count of each of the C classes.
inline size_t lds_sweep_bytes(int32_t n_rows, int W, int32_t C) {
  return (size_t)(n_rows + kDummyRows) * W * 4 + (size_t)2 * kThetaFloats * 4 + (size_t)C * 8;
}

size_t readout_lds_bytes(int32_t n, int32_t B);
// The readout keeps its per-vertex codes in LDS up to this many bytes.
constexpr size_t kReadoutLdsLimit = 163840;
}  // namespace cosm
