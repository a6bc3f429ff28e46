// batch.hip -- many instances of uneven sizes in one persistent sweep launch.
//
// A batch holds several instances ("graphs"), each with its own couplings,
// colouring, parameters, seed and replica count.  cosm_batch_run enqueues, for
// the listed graphs, phase init, their whole schedule of sweeps and the
// readout as three kernels:
//   k_batch_init     grid-stride over every phase of every listed graph;
//   k_batch_sweeps   persistent: each workgroup pops work items (graph, first
//                    replica, number of replica sets) from a device counter
//                    until the list is empty; a small graph packs several
//                    replica sets into one workgroup's LDS so that every item
//                    carries a similar amount of work;
//   k_batch_readout  grid-stride over (graph, replica).
// Kernel arguments only point at device tables that the host rewrites before
// each run, so the three launches are captured once into a hipGraph and
// replayed for every run.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "device_common.hpp"
#include "internal.hpp"

namespace cosm {
namespace {

constexpr int kBatchThreads = 1024;
// Dynamic LDS of the persistent kernel: rows, reference angles and slot counts,
// then 256 bytes of control words at the end.
constexpr int kLdsBudget = 163840;
constexpr int kMaxSetReplicas = 256;  // replica sets x replicas per set, per item

// One graph as the batch kernels see it.
struct GraphDev {
  void *phases;               // [n][R]
  const EdgeDesc *desc;       // lane schedule for kBatchThreads threads
  const int32_t *Kc;          // [C]
  const int32_t *slot_vertex; // [n]
  int32_t n, R, C, total_slots, W;
  int64_t S;                  // sweeps per trial
  SweepSchedule sch;          // at t0 = 0
  uint32_t k0, k1, rid0;
  ReadoutArgs ro;
  int32_t grid;
  int32_t lazy;               // 16-bit float phases wrapped at the twists only
  uint32_t ishift;            // initial phases: (draw >> ishift) * iscale
  float iscale;
};

struct Item {
  int32_t graph, r0, nsets, pad;
};

// Per-run table: counts and prefix sums that the fixed-grid kernels read.
struct RunDesc {
  int32_t n_items;
  int32_t n_run;              // graphs in this run
  int64_t total_phases;       // sum of n * R over the run's graphs
  int32_t total_replicas;     // sum of R
  int32_t counter;            // work-item counter of k_batch_sweeps
};

__global__ void k_batch_reset(RunDesc *rd) {
  if (threadIdx.x == 0 && blockIdx.x == 0) rd->counter = 0;
}

// run_graphs[k]: graph index of the k-th graph of the run; phase_prefix and
// rep_prefix: exclusive prefix sums over the run (length n_run + 1).
template <int ST>
__global__ void __launch_bounds__(256) k_batch_init(const GraphDev *graphs, const RunDesc *rd,
                                                    const int32_t *run_graphs,
                                                    const int64_t *phase_prefix) {
  using F = Fmt<ST>;
  const int64_t total = rd->total_phases;
  const int32_t nr = rd->n_run;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nr - 1;  // last k with phase_prefix[k] <= idx
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (phase_prefix[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    const GraphDev &g = graphs[run_graphs[lo]];
    const int64_t loc = idx - phase_prefix[lo];
    const int32_t i = (int32_t)(loc / g.R), r = (int32_t)(loc % g.R);
    const uint32_t w = philox_first_word((uint32_t)i, 0u, g.rid0 + (uint32_t)r, kTagInit, g.k0, g.k1);
    const float x = (float)(w >> g.ishift) * g.iscale;
    F::store_elem(g.phases, (size_t)loc, F::from_turn(x));
  }
}

// All sweeps of one work item: nsets sets of RW replicas, set k in the LDS rows
// [k * n, (k + 1) * n).  Lane schedule streamed one slot ahead.  RD: every
// graph of the run is FP32 on the grid schedule, so every operation of the
// sweeps is exact and the step's sign comes from the parity form under
// round-toward-minus-infinity.
template <int ST, int W, bool RD>
__device__ void item_sweeps(uint32_t *lds, const GraphDev &g, const Item &it) {
  using F = Fmt<ST>;
  static_assert(!RD || ST == COSM_STORE_FP32, "the parity step is an FP32 grid form");
  // FP16 / BF16 / FP16_PK: wrapped at the twists only when the graph's drift bound holds
  // (g.lazy, set by the host).  (FP32 on the grid could be too, exactly, but a
  // second FP32 sweep path in this kernel made the mixed stream 5 % slower.)
  constexpr bool kLazyOk =
      ST == COSM_STORE_FP16 || ST == COSM_STORE_BF16 || ST == COSM_STORE_FP16_PK;
  constexpr int RW = W * F::kPerWord;
  constexpr uint32_t ROWB = 4 * W;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nsets = it.nsets;
  const uint32_t set_bytes = (uint32_t)g.n * ROWB;
  const int nreps = nsets * RW;
  // reference angles of nch twists for the nreps replicas, then slots per class
  float *theta_buf = reinterpret_cast<float *>(lds + (size_t)nsets * g.n * W);  // [nch][nreps]
  int32_t *Ks = reinterpret_cast<int32_t *>(theta_buf + 2 * kMaxSetReplicas);  // [C]
  const int nch = max(1, min(kThetaChunk, 2 * kMaxSetReplicas / nreps));
  int tw = 0;
  for (int c = tid; c < g.C; c += nth) Ks[c] = as_global(g.Kc)[c];

  for (int s = tid; s < g.n * nsets; s += nth) {
    const int k = s / g.n, slot = s - k * g.n;
    const int32_t rb = it.r0 + k * RW;
    const int32_t nvalid = min(RW, g.R - rb);
    const size_t base = (size_t)as_global(g.slot_vertex)[slot] * g.R + rb;
    float v[RW];
#pragma unroll
    for (int q = 0; q < RW; q++) v[q] = (q < nvalid) ? F::load_elem(g.phases, base + q) : 0.0f;
    uint32_t w[W];
    F::template pack<W>(v, w);
    lds_store<W>(lds, s, w);
  }
  EdgeDesc dA{kEmptySlot, 0.0f}, dB{kEmptySlot, 0.0f};
  int jslot = 0;
  if (g.total_slots > 0) {
    const gptr<EdgeDesc> d0 = as_global(g.desc) + tid;
    const gptr<EdgeDesc> d1 = as_global(g.desc) + (size_t)(1 % g.total_slots) * nth + tid;
    dA = EdgeDesc{d0->slots, d0->J};
    dB = EdgeDesc{d1->slots, d1->J};
  }
  SweepSchedule sc = g.sch;
  __syncthreads();

  const uint32_t S = (uint32_t)g.S;  // at most 2^31 sweeps
  ScheduleChunk chunk;
  float pm = 0.0f;  // RD: 1.5 * 2^23 from the switch, the parity fma's addend
  if constexpr (RD) pm = f32_round_down();
  for (uint32_t t = 1; t - 1 < S; t++) {
    if (((t - 1) & 63u) == 0u) chunk.fill(sc, t);
    float alpha, twist;
    chunk.get((t - 1) & 63u, alpha, twist);
    const float alpha_s = alpha * F::kStepScale;
    if (g.total_slots > 0) {
      if (kLazyOk && g.lazy) {
        stream_classes(g.desc, Ks, g.C, g.total_slots, dA, dB, jslot, [&](const EdgeDesc &d) {
          edge_rows_sets<ST, W, kLazyOk>(lds, (d.slots & 0xffffu) * ROWB, (d.slots >> 16) * ROWB,
                                         set_bytes, nsets, alpha_s * d.J);
        });
      } else {
        stream_classes(g.desc, Ks, g.C, g.total_slots, dA, dB, jslot, [&](const EdgeDesc &d) {
          edge_rows_sets<ST, W, false, RD>(lds, (d.slots & 0xffffu) * ROWB,
                                           (d.slots >> 16) * ROWB, set_bytes, nsets,
                                           alpha_s * d.J, pm);
        });
      }
    }
    if (sc.period > 0 && ++sc.phase == sc.period) {
      sc.phase = 0;
      const int slot = tw % nch;
      if (slot == 0) {
        theta_fill(theta_buf, nullptr, nch, nreps, t, sc.period, g.rid0 + (uint32_t)it.r0, g.k0,
                   g.k1, sc.win, sc.tshift, sc.tscale);
        __syncthreads();
      }
      tw++;
      // set by set (no per-row division), two rows per thread in flight
      for (int k = 0; k < nsets; k++) {
        const float *cth = theta_buf + slot * nreps + k * RW;
        float ck[RW], tws[RW];
#pragma unroll
        for (int r = 0; r < RW; r++) {
          ck[r] = cth[r];
          tws[r] = twist;
        }
        TwistOps<ST, W> op;
        op.set(ck, tws, sc.win2);
        uint32_t *set = lds + (size_t)k * g.n * W;
        for (int s0 = tid; s0 < g.n; s0 += 2 * nth) {
          uint32_t w[2][W];
#pragma unroll
          for (int q = 0; q < 2; q++)
            if (s0 + q * nth < g.n) lds_load<W>(set, s0 + q * nth, w[q]);
#pragma unroll
          for (int q = 0; q < 2; q++) {
            if (s0 + q * nth < g.n) {
              if (kLazyOk && g.lazy) twist_row<ST, W, kLazyOk>(op, w[q]);
              else op.apply(w[q]);
              lds_store<W>(set, s0 + q * nth, w[q]);
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if constexpr (RD) f32_round_nearest();

  for (int s = tid; s < g.n * nsets; s += nth) {
    const int k = s / g.n, slot = s - k * g.n;
    const int32_t rb = it.r0 + k * RW;
    const int32_t nvalid = min(RW, g.R - rb);
    const size_t base = (size_t)as_global(g.slot_vertex)[slot] * g.R + rb;
    uint32_t w[W];
    lds_load<W>(lds, s, w);
    float v[RW];
    F::template unpack<W>(w, v);
#pragma unroll
    for (int q = 0; q < RW; q++)
      if (q < nvalid) F::store_elem(g.phases, base + q, kLazyOk && g.lazy ? F::wrap(v[q]) : v[q]);
  }
}

template <int ST, bool RD>
__global__ void __launch_bounds__(kBatchThreads) k_batch_sweeps(const GraphDev *__restrict__ graphs,
                                                                const Item *__restrict__ items,
                                                                RunDesc *rd) {
  // no static LDS here: it would shift the dynamic rows off their 16-byte alignment
  extern __shared__ __align__(16) uint32_t lds[];
  int32_t &s_item = *reinterpret_cast<int32_t *>(lds + (kLdsBudget - 16) / 4);
  const int32_t n_items = rd->n_items;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(&rd->counter, 1);
    __syncthreads();
    // the same for every lane: keep it (and everything loaded through it) scalar
    const int32_t k = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (k >= n_items) break;  // every wave of the workgroup leaves together
    const Item it = items[k];
    const GraphDev g = graphs[it.graph];  // by value: its fields stay in registers
    if (g.W == 4) item_sweeps<ST, 4, RD>(lds, g, it);
    else if (g.W == 2) item_sweeps<ST, 2, RD>(lds, g, it);
    else item_sweeps<ST, 1, RD>(lds, g, it);
    __syncthreads();
  }
}

template <int ST>
__global__ void __launch_bounds__(256) k_batch_readout(const GraphDev *graphs, const RunDesc *rd,
                                                       const int32_t *run_graphs,
                                                       const int32_t *rep_prefix) {
  extern __shared__ int64_t sm64[];
  const int32_t total = rd->total_replicas, nr = rd->n_run;
  for (int32_t b = blockIdx.x; b < total; b += gridDim.x) {
    int32_t lo = 0, hi = nr - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (rep_prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const GraphDev &g = graphs[run_graphs[lo]];
    readout_block<ST>(g.ro, b - rep_prefix[lo], sm64);
    __syncthreads();
  }
}

int check_launch(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    return set_error(COSM_EDEVICE, std::string(what) + ": " + hipGetErrorString(err));
  return COSM_OK;
}

}  // namespace
}  // namespace cosm

using namespace cosm;

// Host side of a batch graph.
struct BatchGraphHost {
  cosm_state meta;          // sizes, host copies of the instance, parameters, schedule
  void *mem = nullptr;      // one hipMalloc holding every buffer below
  GraphDev dev{};
  int32_t sets_max = 1;     // replica sets that fit one workgroup's LDS
  int32_t tuned = 0;        // 1: the row width was chosen by timed probes (2: from the cache)
  float probe_ms = 0.0f;    // the chosen width's probe time
};

struct cosm_batch {
  hipStream_t stream = nullptr;
  int32_t storage = COSM_STORE_FP32;
  int32_t max_graphs = 0, max_n = 0, max_items = 0, max_bisectors = 0;
  bool own_stream = false;
  size_t lds_budget = 0, readout_lds = 0;
  int32_t cus = 256;
  std::vector<BatchGraphHost *> graphs;
  GraphDev *d_graphs = nullptr;
  Item *d_items = nullptr;
  RunDesc *d_run = nullptr;
  int32_t *d_run_graphs = nullptr, *d_rep_prefix = nullptr;
  int64_t *d_phase_prefix = nullptr;
  // the captured run, one per sweep variant (1: every graph FP32 on the grid)
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int32_t run_rd = 0;       // the variant of the prepared run
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool graphs_dirty = true;
};

namespace {

template <int ST>
void enqueue_run(cosm_batch *b) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->stream, b->d_run);
  hipLaunchKernelGGL((k_batch_init<ST>), dim3(2048), dim3(256), 0, b->stream, b->d_graphs,
                     b->d_run, b->d_run_graphs, b->d_phase_prefix);
  if constexpr (ST == COSM_STORE_FP32) {
    if (b->run_rd)
      hipLaunchKernelGGL((k_batch_sweeps<ST, true>), dim3(b->cus), dim3(kBatchThreads),
                         (size_t)kLdsBudget, b->stream, b->d_graphs, b->d_items, b->d_run);
    else
      hipLaunchKernelGGL((k_batch_sweeps<ST, false>), dim3(b->cus), dim3(kBatchThreads),
                         (size_t)kLdsBudget, b->stream, b->d_graphs, b->d_items, b->d_run);
  } else {
    hipLaunchKernelGGL((k_batch_sweeps<ST, false>), dim3(b->cus), dim3(kBatchThreads),
                       (size_t)kLdsBudget, b->stream, b->d_graphs, b->d_items, b->d_run);
  }
  hipLaunchKernelGGL((k_batch_readout<ST>), dim3(4096), dim3(256), b->readout_lds, b->stream,
                     b->d_graphs, b->d_run, b->d_run_graphs, b->d_rep_prefix);
}

template <int ST>
void set_attrs(cosm_batch *b) {
  (void)hipFuncSetAttribute((const void *)k_batch_sweeps<ST, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
  if constexpr (ST == COSM_STORE_FP32)
    (void)hipFuncSetAttribute((const void *)k_batch_sweeps<ST, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
  (void)hipFuncSetAttribute((const void *)k_batch_readout<ST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->readout_lds);
}

// The run's tables (work items, per-graph descriptors and prefix sums), on
// the device and synchronised, for the graphs ids (valid ids of b->graphs).
int prepare_run(cosm_batch *b, const std::vector<int32_t> &ids, bool fill = true) {
  const int32_t count = (int32_t)ids.size();
  // the sweep variant: the parity form when every graph is FP32 on the grid
  b->run_rd = b->storage == COSM_STORE_FP32 ? 1 : 0;
  for (int32_t id : ids)
    if (!b->graphs[(size_t)id]->dev.grid) b->run_rd = 0;
  // work items: split every graph's replicas into items of up to sets_max sets,
  // shrinking the sets (fill) while the run would leave CUs without an item
  std::vector<int32_t> sets(ids.size());
  for (size_t k = 0; k < ids.size(); k++) sets[k] = b->graphs[(size_t)ids[k]]->sets_max;
  const int32_t pw = (b->storage == COSM_STORE_FP32 || b->storage == COSM_STORE_FIX32) ? 1 : 2;
  auto count_items = [&]() {
    int64_t total = 0;
    for (size_t k = 0; k < ids.size(); k++) {
      const GraphDev &d = b->graphs[(size_t)ids[k]]->dev;
      const int32_t rw = d.W * pw;
      total += (d.R + rw * sets[k] - 1) / (rw * sets[k]);
    }
    return total;
  };
  while (fill && count_items() < 2 * (int64_t)b->cus) {
    bool shrunk = false;
    for (auto &v : sets)
      if (v > 1) {
        v = (v + 1) / 2;
        shrunk = true;
      }
    if (!shrunk) break;
  }
  std::vector<Item> items;
  std::vector<double> cost;
  for (size_t k = 0; k < ids.size(); k++) {
    const GraphDev &d = b->graphs[(size_t)ids[k]]->dev;
    const int32_t rw = d.W * pw;
    for (int32_t r0 = 0; r0 < d.R; r0 += rw * sets[k]) {
      const int32_t ns = std::min(sets[k], (d.R - r0 + rw - 1) / rw);
      items.push_back(Item{ids[k], r0, ns, 0});
      cost.push_back((double)ns * (double)(b->graphs[(size_t)ids[k]]->meta.m + d.n) * (double)d.S);
    }
  }
  if ((int64_t)items.size() > b->max_items) {
    // grow the item table; the captured graph points at the old one, so drop it
    COSM_HIP_CHECK(hipStreamSynchronize(b->stream));
    const int32_t cap = (int32_t)std::min<int64_t>((int64_t)items.size() * 2, 1 << 28);
    Item *fresh = nullptr;
    if (hipMalloc(&fresh, sizeof(Item) * (size_t)cap) != hipSuccess)
      return set_error(COSM_ENOMEM, "hipMalloc of the work-item table failed");
    (void)hipFree(b->d_items);
    b->d_items = fresh;
    b->max_items = cap;
    for (int v = 0; v < 2; v++) {
      if (b->exec[v]) (void)hipGraphExecDestroy(b->exec[v]);
      if (b->graph[v]) (void)hipGraphDestroy(b->graph[v]);
      b->exec[v] = nullptr;
      b->graph[v] = nullptr;
    }
  }
  // largest items first (longest-processing-time order)
  std::vector<size_t> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return cost[a] > cost[c]; });
  std::vector<Item> sorted;
  for (size_t k : order) sorted.push_back(items[k]);
  RunDesc rd{};
  rd.n_items = (int32_t)sorted.size();
  rd.n_run = count;
  std::vector<int64_t> phase_prefix((size_t)count + 1, 0);
  std::vector<int32_t> rep_prefix((size_t)count + 1, 0);
  for (int32_t k = 0; k < count; k++) {
    const GraphDev &d = b->graphs[(size_t)ids[(size_t)k]]->dev;
    phase_prefix[(size_t)k + 1] = phase_prefix[(size_t)k] + (int64_t)d.n * d.R;
    rep_prefix[(size_t)k + 1] = rep_prefix[(size_t)k] + d.R;
  }
  rd.total_phases = phase_prefix[(size_t)count];
  rd.total_replicas = rep_prefix[(size_t)count];
  std::vector<GraphDev> gd;
  for (BatchGraphHost *g : b->graphs) gd.push_back(g->dev);
  int rc = COSM_OK;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (rc == COSM_OK && bytes &&
        hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
      rc = set_error(COSM_EDEVICE, "hipMemcpyAsync");
  };
  up(b->d_graphs, gd.data(), gd.size() * sizeof(GraphDev));
  up(b->d_items, sorted.data(), sorted.size() * sizeof(Item));
  up(b->d_run, &rd, sizeof rd);
  up(b->d_run_graphs, ids.data(), ids.size() * 4);
  up(b->d_rep_prefix, rep_prefix.data(), rep_prefix.size() * 4);
  up(b->d_phase_prefix, phase_prefix.data(), phase_prefix.size() * 8);
  if (rc) return rc;
  // the host tables above are read by the copies: wait before they go out of scope
  COSM_HIP_CHECK(hipStreamSynchronize(b->stream));
  return COSM_OK;
}

int launch_run(cosm_batch *b) {
  switch (b->storage) {
    case COSM_STORE_FP32: enqueue_run<COSM_STORE_FP32>(b); break;
    case COSM_STORE_FP16: enqueue_run<COSM_STORE_FP16>(b); break;
    case COSM_STORE_FP16_PK: enqueue_run<COSM_STORE_FP16_PK>(b); break;
    case COSM_STORE_BF16: enqueue_run<COSM_STORE_BF16>(b); break;
    case COSM_STORE_FIX16: enqueue_run<COSM_STORE_FIX16>(b); break;
    default: enqueue_run<COSM_STORE_FIX32>(b); break;
  }
  return check_launch("batch run");
}

// The row width of a graph by measurement.  Each candidate's lane schedule is
// installed (install(k)) and a probe is timed with events through the run
// path: one work item of the graph as a full batch lays it out (as many
// replica sets as fit, never shrunk to fill the chip), up to 128 sweeps.  A
// busy batch keeps every CU on one such item at a time, so the time per
// replica of that item is the graph's cost per replica in the batch; the
// width with the least is kept.  (Timing the graph alone with all its
// replicas would instead favour the narrow rows that spread a lone graph over
// more CUs.)  The choice is cached by the instance's signature (sizes,
// storage, replicas, sweeps and an FNV-1a hash of the edge list and
// colouring), so later graphs with the same signature skip the probes.  The
// probe overwrites only the graph's own first replicas' phases and results,
// which every run initialises afresh.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, std::pair<int32_t, float>> g_tune_cache;  // width, probe ms

template <typename Install>
int tune_batch_graph(cosm_batch *b, BatchGraphHost *g, const std::vector<int32_t> &widths,
                     Install install) {
  const cosm_state &s = g->meta;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint32_t v) {
    for (int q = 0; q < 4; q++) h = (h ^ ((v >> (8 * q)) & 0xffu)) * 1099511628211ull;
  };
  for (int64_t k = 0; k < s.m; k++) {
    mix((uint32_t)s.h_eu[(size_t)k]);
    mix((uint32_t)s.h_ev[(size_t)k]);
    mix((uint32_t)s.h_colour[(size_t)k]);
  }
  const std::vector<int64_t> key{s.n, s.m, s.C, s.R, b->storage, s.p.sweeps_per_trial, (int64_t)h};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end())
      for (size_t k = 0; k < widths.size(); k++)
        if (widths[k] == it->second.first) {
          install(k);
          g->tuned = 2;
          g->probe_ms = it->second.second;
          return COSM_OK;
        }
  }
  COSM_HIP_CHECK(hipStreamSynchronize(b->stream));
  const int64_t full_S = g->dev.S;
  const int32_t full_R = g->dev.R;
  const int32_t pw = (b->storage == COSM_STORE_FP32 || b->storage == COSM_STORE_FIX32) ? 1 : 2;
  g->dev.S = std::min<int64_t>(full_S, 128);
  const int32_t gid = (int32_t)b->graphs.size();
  b->graphs.push_back(g);  // (for the probes only)
  int rc = COSM_OK;
  float best_ms = 0.0f;
  double best_per_replica = 0.0;
  size_t best = 0;
  for (size_t k = 0; k < widths.size() && rc == COSM_OK; k++) {
    install(k);
    // one full work item: the first replicas only
    g->dev.R = std::min<int32_t>(full_R, g->dev.W * pw * g->sets_max);
    g->dev.ro.R = g->dev.R;
    rc = prepare_run(b, {gid}, false);
    float ms = 0.0f, ms_min = 0.0f;
    for (int rep = 0; rep < 3 && rc == COSM_OK; rep++) {  // a warm-up, then two timed probes
      if (hipEventRecord(b->e0, b->stream) != hipSuccess) rc = set_error(COSM_EDEVICE, "event");
      if (rc == COSM_OK) rc = launch_run(b);
      if (rc == COSM_OK && (hipEventRecord(b->e1, b->stream) != hipSuccess ||
                            hipEventSynchronize(b->e1) != hipSuccess))
        rc = set_error(COSM_EDEVICE, "event");
      if (rc == COSM_OK) (void)hipEventElapsedTime(&ms, b->e0, b->e1);
      if (rep == 1 || (rep == 2 && ms < ms_min)) ms_min = ms;
    }
    const double per_replica = (double)ms_min / (double)g->dev.R;
    if (rc == COSM_OK && (k == 0 || per_replica < best_per_replica)) {
      best_per_replica = per_replica;
      best_ms = ms_min;
      best = k;
    }
  }
  b->graphs.pop_back();
  g->dev.S = full_S;
  g->dev.R = full_R;
  g->dev.ro.R = full_R;
  if (rc) return rc;
  install(best);
  g->tuned = 1;
  g->probe_ms = best_ms;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = {widths[best], best_ms};
  return COSM_OK;
}

}  // namespace

extern "C" {

int cosm_batch_create(cosm_batch **out, int32_t storage, int32_t max_graphs, int32_t max_n,
                      int32_t max_bisectors, void *hip_stream) {
  clear_error();
  if (out == nullptr) return set_error(COSM_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (storage < COSM_STORE_FP32 || storage > COSM_STORE_FP16_PK) return set_error(COSM_EINVAL, "bad storage");
  if (max_graphs < 1 || max_n < 1 || max_n > 65536 || max_bisectors < 1 || max_bisectors > 32767)
    return set_error(COSM_EINVAL, "bad batch limits");
  cosm_batch *b = new cosm_batch();
  // a graph cannot be captured on the legacy default stream: use a stream of our own then
  b->stream = static_cast<hipStream_t>(hip_stream);
  if (b->stream == nullptr) {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return set_error(COSM_EDEVICE, "hipStreamCreate");
    }
    b->own_stream = true;
  }
  b->max_bisectors = max_bisectors;
  b->storage = storage;
  b->max_graphs = max_graphs;
  b->max_n = max_n;
  if (lds_capacity_bytes() < kLdsBudget) {
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return set_error(COSM_EDEVICE, "the device offers less LDS per workgroup than the batch kernel uses");
  }
  b->lds_budget = kLdsBudget - 256;  // data; the last 256 bytes hold control words
  b->readout_lds = readout_lds_bytes(max_n, max_bisectors);
  if (b->readout_lds > b->lds_budget) {
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return set_error(COSM_ERANGE, "max_n too large for the readout");
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    b->cus = cus;
  b->max_items = 64 * b->cus + 16 * max_graphs;
  int rc = COSM_OK;
  auto alloc = [&](void **p, size_t bytes) {
    if (rc == COSM_OK && hipMalloc(p, bytes) != hipSuccess) rc = set_error(COSM_ENOMEM, "hipMalloc");
  };
  alloc((void **)&b->d_graphs, sizeof(GraphDev) * max_graphs);
  alloc((void **)&b->d_items, sizeof(Item) * b->max_items);
  alloc((void **)&b->d_run, sizeof(RunDesc));
  alloc((void **)&b->d_run_graphs, sizeof(int32_t) * max_graphs);
  alloc((void **)&b->d_rep_prefix, sizeof(int32_t) * (max_graphs + 1));
  alloc((void **)&b->d_phase_prefix, sizeof(int64_t) * (max_graphs + 1));
  if (rc == COSM_OK && (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess))
    rc = set_error(COSM_EDEVICE, "hipEventCreate");
  if (rc) {
    cosm_batch_destroy(b);
    return rc;
  }
  switch (storage) {
    case COSM_STORE_FP32: set_attrs<COSM_STORE_FP32>(b); break;
    case COSM_STORE_FP16: set_attrs<COSM_STORE_FP16>(b); break;
    case COSM_STORE_FP16_PK: set_attrs<COSM_STORE_FP16_PK>(b); break;
    case COSM_STORE_BF16: set_attrs<COSM_STORE_BF16>(b); break;
    case COSM_STORE_FIX16: set_attrs<COSM_STORE_FIX16>(b); break;
    default: set_attrs<COSM_STORE_FIX32>(b); break;
  }
  *out = b;
  return COSM_OK;
}

int cosm_batch_destroy(cosm_batch *b) {
  clear_error();
  if (b == nullptr) return COSM_OK;
  (void)hipStreamSynchronize(b->stream);
  for (int v = 0; v < 2; v++) {
    if (b->exec[v]) (void)hipGraphExecDestroy(b->exec[v]);
    if (b->graph[v]) (void)hipGraphDestroy(b->graph[v]);
  }
  for (BatchGraphHost *g : b->graphs) {
    if (g->mem) (void)hipFree(g->mem);
    delete g;
  }
  (void)hipFree(b->d_graphs);
  (void)hipFree(b->d_items);
  (void)hipFree(b->d_run);
  (void)hipFree(b->d_run_graphs);
  (void)hipFree(b->d_rep_prefix);
  (void)hipFree(b->d_phase_prefix);
  if (b->e0) (void)hipEventDestroy(b->e0);
  if (b->e1) (void)hipEventDestroy(b->e1);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return COSM_OK;
}

int cosm_batch_add_graph(cosm_batch *b, int32_t n, int64_t m, const int32_t *eu,
                         const int32_t *ev, const int32_t *J, const int32_t *colour,
                         int32_t num_colours, const cosm_params *p, uint64_t seed,
                         int32_t replicas, int32_t *graph_id_out) {
  clear_error();
  if (b == nullptr || p == nullptr || graph_id_out == nullptr)
    return set_error(COSM_EINVAL, "NULL argument");
  if ((int32_t)b->graphs.size() >= b->max_graphs) return set_error(COSM_ERANGE, "batch is full");
  if (n > b->max_n) return set_error(COSM_ERANGE, "graph larger than the batch's max_n");
  if (replicas < 1) return set_error(COSM_EINVAL, "replicas must be >= 1");
  if (p->storage != b->storage) return set_error(COSM_EINVAL, "storage differs from the batch's");
  if (p->update != COSM_UPDATE_SCS) return set_error(COSM_EINVAL, "batches run the SCS update only");
  if (p->n_bisectors > b->max_bisectors) return set_error(COSM_ERANGE, "more bisectors than the batch's limit");
  if (int rc = check_params_public(p)) return rc;
  if (m > 0 && J == nullptr) return set_error(COSM_EINVAL, "J must not be NULL");
  if (int rc = validate_graph(n, m, eu, ev, nullptr)) return rc;
  if (int rc = validate_colouring(n, m, eu, ev, colour, num_colours)) return rc;
  int32_t max_abs_J = 0;
  for (int64_t k = 0; k < m; k++) max_abs_J = std::max(max_abs_J, std::abs(J[k]));
  BatchGraphHost *g = new BatchGraphHost();
  cosm_state &s = g->meta;
  s.n = n;
  s.m = m;
  s.C = num_colours;
  s.R = replicas;
  s.p = *p;
  s.seed = seed;
  s.h_eu.assign(eu, eu + m);
  s.h_ev.assign(ev, ev + m);
  s.h_J.assign(J, J + m);
  s.h_colour.assign(colour, colour + m);
  s.n_slots = n;
  {
    std::vector<int64_t> wdeg((size_t)n, 0);
    for (int64_t k = 0; k < m; k++) {
      wdeg[(size_t)eu[k]] += std::abs((int64_t)J[k]);
      wdeg[(size_t)ev[k]] += std::abs((int64_t)J[k]);
    }
    for (int64_t w : wdeg) s.wdeg_max = std::max(s.wdeg_max, w);
  }
  int rc = make_schedule(s.p, max_abs_J, &s.sched);
  // Row widths: those that leave room for at least one replica set (a
  // requested replicas_per_wg picks one); each gets its lane schedule.  With
  // more than one, the shape is chosen by timed probes (below).
  const int32_t pw = (b->storage == COSM_STORE_FP32 || b->storage == COSM_STORE_FIX32) ? 1 : 2;
  std::vector<int32_t> widths;
  for (int32_t w : {4, 2, 1}) {
    if ((size_t)n * w * 4 + 2 * kMaxSetReplicas * 4 + (size_t)num_colours * 4 > b->lds_budget) continue;
    if (p->replicas_per_wg > 0 && p->replicas_per_wg != w * pw) continue;
    widths.push_back(w);
  }
  if (rc == COSM_OK && widths.empty())
    rc = set_error(COSM_ERANGE, p->replicas_per_wg > 0
                                    ? "requested replicas per set do not fit one workgroup's LDS"
                                    : "graph does not fit one workgroup's LDS");
  std::vector<LdsSchedule> scheds(widths.size());
  size_t desc_max = 0;
  for (size_t k = 0; k < widths.size() && rc == COSM_OK; k++) {
    rc = build_lds_schedule(s, widths[k], kBatchThreads, &scheds[k]);
    desc_max = std::max(desc_max, scheds[k].desc.size());
  }
  if (rc) {
    delete g;
    return rc;
  }
  int32_t W = widths[0];
  s.lds = scheds[0];
  auto sets_for = [&](int32_t w) {
    return (int32_t)std::max<size_t>(
        1, std::min<size_t>((b->lds_budget - 2 * kMaxSetReplicas * 4 - (size_t)num_colours * 4) /
                                ((size_t)n * w * 4),
                            (size_t)kMaxSetReplicas / (size_t)(w * pw)));
  };
  g->sets_max = sets_for(W);
  // device memory: phases, schedule, K, slot map, edges, spins, H, cut, best_p
  const size_t nr = (size_t)n * replicas, sb = pw == 1 ? 4 : 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    return at;
  };
  const size_t o_ph = take(nr * sb), o_desc = take(desc_max * sizeof(EdgeDesc)),
               o_K = take((size_t)num_colours * 4), o_sv = take((size_t)n * 4),
               o_eu = take((size_t)m * 4), o_ev = take((size_t)m * 4), o_J = take((size_t)m * 4),
               o_sp = take(nr), o_H = take((size_t)replicas * 8), o_cut = take((size_t)replicas * 8),
               o_bp = take((size_t)replicas * 4);
  if (hipMalloc(&g->mem, off) != hipSuccess) {
    delete g;
    return set_error(COSM_ENOMEM, "hipMalloc of a batch graph failed");
  }
  char *base = static_cast<char *>(g->mem);
  auto up = [&](size_t o, const void *src, size_t bytes) {
    if (rc == COSM_OK && bytes && hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      rc = set_error(COSM_EDEVICE, "hipMemcpy");
  };
  up(o_eu, eu, (size_t)m * 4);
  up(o_ev, ev, (size_t)m * 4);
  up(o_J, J, (size_t)m * 4);
  GraphDev &d = g->dev;
  d.phases = base + o_ph;
  d.desc = reinterpret_cast<const EdgeDesc *>(base + o_desc);
  d.Kc = reinterpret_cast<const int32_t *>(base + o_K);
  d.slot_vertex = reinterpret_cast<const int32_t *>(base + o_sv);
  d.n = n;
  d.R = replicas;
  d.C = num_colours;
  d.total_slots = s.lds.total_slots;
  d.W = W;
  d.S = s.p.sweeps_per_trial;
  const Schedule &sc = s.sched;
  d.sch = make_sweep_schedule(sc, 0);
  d.k0 = (uint32_t)(seed & 0xffffffffu);
  d.k1 = (uint32_t)(seed >> 32);
  d.rid0 = 0;
  d.grid = sc.grid;
  d.lazy = lazy16(s) ? 1 : 0;
  d.ishift = (uint32_t)sc.ishift;
  d.iscale = sc.iscale;
  ReadoutArgs &ro = d.ro;
  ro.phases = d.phases;
  ro.eu = reinterpret_cast<const int32_t *>(base + o_eu);
  ro.ev = reinterpret_cast<const int32_t *>(base + o_ev);
  ro.J = reinterpret_cast<const int32_t *>(base + o_J);
  ro.h = nullptr;
  ro.code_global = nullptr;  // the batch keeps readout codes in LDS (max_n bounded)
  ro.spins = reinterpret_cast<int8_t *>(base + o_sp);
  ro.H = reinterpret_cast<int64_t *>(base + o_H);
  ro.cut = reinterpret_cast<int64_t *>(base + o_cut);
  ro.best_p = reinterpret_cast<int32_t *>(base + o_bp);
  ro.n = n;
  ro.R = replicas;
  ro.B = s.p.n_bisectors;
  ro.grid = sc.grid;
  ro.m = m;
  // the lane schedule of candidate k: its descriptors, slot counts and slot
  // map on the device, its width and replica sets in the descriptor
  auto install = [&](size_t k) {
    s.lds = scheds[k];
    W = widths[k];
    d.W = W;
    d.total_slots = s.lds.total_slots;
    g->sets_max = sets_for(W);
    up(o_desc, s.lds.desc.data(), s.lds.desc.size() * sizeof(EdgeDesc));
    up(o_K, s.lds.K.data(), s.lds.K.size() * 4);
    up(o_sv, s.lds.slot_vertex.data(), s.lds.slot_vertex.size() * 4);
  };
  install(0);
  if (rc == COSM_OK && widths.size() > 1) {
    const int rt = tune_batch_graph(b, g, widths, install);
    if (rc == COSM_OK) rc = rt;  // (a failed upload inside install set rc itself)
  }
  if (rc) {
    (void)hipFree(g->mem);
    delete g;
    return rc;
  }
  *graph_id_out = (int32_t)b->graphs.size();
  b->graphs.push_back(g);
  b->graphs_dirty = true;
  return COSM_OK;
}

int cosm_batch_graph_shape(const cosm_batch *b, int32_t graph_id, int32_t *replicas_per_set,
                           int32_t *sets_per_item, int32_t *tuned, double *probe_ms,
                           int32_t *lazy_wrap) {
  clear_error();
  if (b == nullptr || graph_id < 0 || graph_id >= (int32_t)b->graphs.size())
    return set_error(COSM_EINVAL, "bad graph id");
  const BatchGraphHost *g = b->graphs[(size_t)graph_id];
  const int32_t pw = (b->storage == COSM_STORE_FP32 || b->storage == COSM_STORE_FIX32) ? 1 : 2;
  if (replicas_per_set) *replicas_per_set = g->dev.W * pw;
  if (sets_per_item) *sets_per_item = g->sets_max;
  if (tuned) *tuned = g->tuned;
  if (probe_ms) *probe_ms = g->probe_ms;
  if (lazy_wrap) *lazy_wrap = g->dev.lazy;
  return COSM_OK;
}

int cosm_batch_set_seed(cosm_batch *b, int32_t graph_id, uint64_t seed, int64_t replica_offset) {
  clear_error();
  if (b == nullptr || graph_id < 0 || graph_id >= (int32_t)b->graphs.size())
    return set_error(COSM_EINVAL, "bad graph id");
  BatchGraphHost *g = b->graphs[(size_t)graph_id];
  if (replica_offset < 0 || replica_offset + g->dev.R > ((int64_t)1 << 32))
    return set_error(COSM_ERANGE, "replica indices must stay below 2^32");
  g->dev.k0 = (uint32_t)(seed & 0xffffffffu);
  g->dev.k1 = (uint32_t)(seed >> 32);
  g->dev.rid0 = (uint32_t)replica_offset;
  b->graphs_dirty = true;
  return COSM_OK;
}

int cosm_batch_run(cosm_batch *b, const int32_t *graph_ids, int32_t count) {
  clear_error();
  if (b == nullptr || graph_ids == nullptr || count < 1) return set_error(COSM_EINVAL, "bad run");
  if (count > b->max_graphs) return set_error(COSM_ERANGE, "too many graphs in one run");
  std::vector<int32_t> ids(graph_ids, graph_ids + count);
  for (int32_t id : ids)
    if (id < 0 || id >= (int32_t)b->graphs.size()) return set_error(COSM_EINVAL, "bad graph id");
  if (int rc = prepare_run(b, ids)) return rc;
  const int v = b->run_rd;
  if (b->exec[v] == nullptr) {
    COSM_HIP_CHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    switch (b->storage) {
      case COSM_STORE_FP32: enqueue_run<COSM_STORE_FP32>(b); break;
      case COSM_STORE_FP16: enqueue_run<COSM_STORE_FP16>(b); break;
      case COSM_STORE_FP16_PK: enqueue_run<COSM_STORE_FP16_PK>(b); break;
      case COSM_STORE_BF16: enqueue_run<COSM_STORE_BF16>(b); break;
      case COSM_STORE_FIX16: enqueue_run<COSM_STORE_FIX16>(b); break;
      default: enqueue_run<COSM_STORE_FIX32>(b); break;
    }
    COSM_HIP_CHECK(hipStreamEndCapture(b->stream, &b->graph[v]));
    COSM_HIP_CHECK(hipGraphInstantiate(&b->exec[v], b->graph[v], nullptr, nullptr, 0));
  }
  COSM_HIP_CHECK(hipEventRecord(b->e0, b->stream));
  COSM_HIP_CHECK(hipGraphLaunch(b->exec[v], b->stream));
  COSM_HIP_CHECK(hipEventRecord(b->e1, b->stream));
  return check_launch("cosm_batch_run");
}

int cosm_batch_wait(cosm_batch *b, double *device_ms_out) {
  clear_error();
  if (b == nullptr) return set_error(COSM_EINVAL, "batch must not be NULL");
  COSM_HIP_CHECK(hipEventSynchronize(b->e1));
  if (device_ms_out) {
    float ms = 0.0f;
    COSM_HIP_CHECK(hipEventElapsedTime(&ms, b->e0, b->e1));
    *device_ms_out = ms;
  }
  return COSM_OK;
}

int cosm_batch_poll(cosm_batch *b, int32_t *done_out) {
  clear_error();
  if (b == nullptr || done_out == nullptr)
    return set_error(COSM_EINVAL, "batch and done_out must not be NULL");
  hipError_t q = hipEventQuery(b->e1);
  if (q == hipErrorNotReady) {
    *done_out = 0;
    return COSM_OK;
  }
  COSM_HIP_CHECK(q);
  *done_out = 1;
  return COSM_OK;
}

int cosm_batch_results(cosm_batch *b, int32_t graph_id, int64_t *H_out, int64_t *cut_out,
                       int8_t *spins_out) {
  clear_error();
  if (b == nullptr || graph_id < 0 || graph_id >= (int32_t)b->graphs.size())
    return set_error(COSM_EINVAL, "bad graph id");
  const GraphDev &d = b->graphs[(size_t)graph_id]->dev;
  if (H_out)
    COSM_HIP_CHECK(hipMemcpyAsync(H_out, d.ro.H, (size_t)d.R * 8, hipMemcpyDeviceToHost, b->stream));
  if (cut_out)
    COSM_HIP_CHECK(hipMemcpyAsync(cut_out, d.ro.cut, (size_t)d.R * 8, hipMemcpyDeviceToHost, b->stream));
  if (spins_out)
    COSM_HIP_CHECK(hipMemcpyAsync(spins_out, d.ro.spins, (size_t)d.R * d.n, hipMemcpyDeviceToHost,
                                  b->stream));
  COSM_HIP_CHECK(hipStreamSynchronize(b->stream));
  return COSM_OK;
}

}  // extern "C"
