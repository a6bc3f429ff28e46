/*
 * cosm.h -- C ABI of libcosm, an MI355X (gfx950) implementation of the sweep of
 * Cosm ("Collective Switched Motion for Fast and Accurate Sparse Ising
 * Optimization", Zick, Shukla, Marakov).
 *
 * The problem (Eq. (1)): spins s_i in {-1,+1}, i < n; sparse couplings J on m
 * undirected edges (u_k, v_k); optional bias h.  H(s) = -sum_k J_k s_u s_v -
 * sum_i h_i s_i.  The Max-Cut form (Appendix A, Eq. (14)) uses w = -J, so
 * cut(s) = sum over edges with s_u != s_v of (-J_k).
 *
 * The method (Algorithm 1): a proper edge colouring splits the edges into C
 * matchings (Eqs. (9)-(11)); every replica keeps one phase per spin on the
 * circle; a sweep applies the pair update of Eq. (6) to every edge of class 0,
 * then class 1, ..., class C-1 (Eqs. (12)-(13)); every dwt_period sweeps the
 * dual window twist rotates the phases inside two opposing windows centred at
 * a random angle (Sec. II-D); the step size ramps linearly from alpha0 to 0,
 * constant within a sweep (Sec. II-B, Appendix B); after the last sweep the
 * phases are cut by B equally spaced bisectors and the lowest-energy spin
 * vector is kept.
 *
 * Conventions for every function:
 *   - Return value: COSM_OK (0) or a negative COSM_E* status; no exception or
 *     abort crosses the ABI.  cosm_last_error() gives a message for the last
 *     failing call on the calling thread.
 *   - Host pointers are read during the call only; the caller keeps ownership
 *     and may free them afterwards.  Output arrays are caller-allocated.
 *   - A cosm_state is owned by the library, released by cosm_destroy, and must
 *     not be used from two host threads at once.  Separate states are
 *     independent.
 *   - Every GPU operation of a state is enqueued on the hip stream given to
 *     cosm_init.  Functions that return host values synchronise that stream.
 *   - Phases live on the device as turns in [0, 1) (1 turn = 360 degrees).
 */
#ifndef COSM_H
#define COSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
enum {
  COSM_OK = 0,
  COSM_EINVAL = -1,  /* bad argument: NULL, out of range, self-loop, bad spin value */
  COSM_EDUP = -2,    /* duplicate undirected edge */
  COSM_ECOLOR = -3,  /* colouring is not proper or does not cover every edge */
  COSM_ERANGE = -4,  /* request exceeds a limit (sweeps past S, LDS capacity, sizes) */
  COSM_ENOMEM = -5,  /* device or host allocation failed, or workspace too small */
  COSM_EDEVICE = -6, /* HIP runtime error */
  COSM_ESTATE = -7   /* call not valid in the state's current condition */
};

/* ---- enumerations ---------------------------------------------------------- */
enum { COSM_COLOR_GREEDY = 0, COSM_COLOR_MISRA_GRIES = 1, COSM_COLOR_TORUS = 2,
       COSM_COLOR_BALANCED = 3, COSM_COLOR_MINIMUM = 4 };
/* Class-order flag, ORed into the method of cosm_build_partitions: the labels of
 * the largest class and of the last one are swapped, so that the class applied
 * last covers the most vertices (the sweep then folds the twist into it,
 * dropping a pass).  The order is part of the dynamics (Sec. V-A); the flag is
 * deterministic and the returned colouring records it. */
enum { COSM_ORDER_LARGEST_LAST = 0x100 };
/* Phase storage.  FP32: x in [0, 1) turn.  FP16 / BF16: the centred value
 * y = x - 1/2, FP32 arithmetic, rounded on every store.  FP16_PK: FP16 storage
 * as FP16, Eq. (6) in FP16 arithmetic (packed, two replicas per instruction):
 * e = y_u - y_v, the sign of the coupling from round(2e - 1/2) being even (an
 * exact half-turn difference counts as positive), the step alpha J and both
 * updates each rounded to FP16; its twist computes in FP32.  FIX16: x in 16-bit fixed
 * point (units of 2^-16 turn), wrapping by integer overflow; needs the GRID
 * schedule, which it runs on the 2^-16 turn grid (steps on 2^-15, initial
 * phases and twist angles the top 16 bits of the same draws), so trajectories
 * are exact; the window must be a multiple of 2^-16 turn.  FIX32: x in 32-bit
 * fixed point (units of 2^-32 turn), wrapping by integer overflow; needs the
 * GRID schedule, on the same 2^-23 turn grid as FP32, and gives the FP32
 * trajectory bit for bit with integer instead of floating-point arithmetic
 * (phases set from outside are rounded to 2^-32 turn). */
enum { COSM_STORE_FP32 = 0, COSM_STORE_FP16 = 1, COSM_STORE_BF16 = 2, COSM_STORE_FIX16 = 3,
       COSM_STORE_FIX32 = 4, COSM_STORE_FP16_PK = 5 };
/* Where a replica's phases live during a sweep.  LDS: a workgroup holds whole
 * replicas in LDS for all sweeps of a call.  HBM: phases stay in device memory,
 * one launch per colour class.  PLAIN: one replica per launch, one launch per
 * colour class (the unbatched baseline). */
enum { COSM_RES_AUTO = 0, COSM_RES_LDS = 1, COSM_RES_HBM = 2, COSM_RES_PLAIN = 3 };
/* GRID: every phase, step and angle is a multiple of 2^-23 turn (2^-16 with
 * FIX16 storage), so sweeps are exact; the window must be a multiple of 2^-22
 * turn.  CONTINUOUS: the literal ramp alpha0 (S - t + 1) / S in FP32. */
enum { COSM_SCHED_GRID = 0, COSM_SCHED_CONTINUOUS = 1 };
/* Layout of the LDS form.  PAIR: every edge update reads and writes both
 * endpoint rows in LDS.  REGISTER: an independent set of vertices stays in
 * registers, a few per thread; each edge with an endpoint there is applied by
 * that endpoint's thread, which touches LDS only for the other endpoint (the
 * even tori: every edge), the remaining edges as in PAIR.  The same updates in
 * the same class order: trajectories are identical.  REGISTER needs FP32,
 * FIX32 or FIX16 storage, at most 8 classes, no bias fields, and few enough
 * edges outside the register set (COSM_ERANGE otherwise when requested).
 * REGISTER moves far fewer LDS bytes but needs more vector and scalar
 * instructions per update (the u / v roles of each edge, the dummy lanes of
 * vertices without an edge in a class): it wins where LDS traffic dominates
 * (the large even tori) and loses on the 3-regular benchmark graph.  AUTO:
 * when the shape is autotuned both layouts are timed and the faster kept;
 * otherwise PAIR. */
enum {
  COSM_LDS_FORM_AUTO = 0,
  COSM_LDS_FORM_PAIR = 1,
  COSM_LDS_FORM_REGISTER = 2,
  COSM_LDS_FORM_REGISTER_STREAM = 3 /* register owners with a streamed schedule: FP32, no bias
                                       fields, up to 32 classes (the large graphs) */
};
/* SCS: Eqs. (12)-(13), classes one after another.  FULL_GRADIENT: Eq. (8), all
 * edges read the same state (the "without SCS" variant of Table VII). */
enum { COSM_UPDATE_SCS = 0, COSM_UPDATE_FULL_GRADIENT = 1 };
/* Readout rule (Algorithm 1, binarization).  BISECTORS: B equally spaced
 * bisectors.  OPTIMAL: the best of all distinct bisectors (every position where
 * some spin changes side), the alternative the paper cites from Burer et al.:
 * lowest H, smallest angle on ties; per replica a segmented sort of the n
 * values x_i mod 180 and an O(n + m) difference array.  OPTIMAL needs h = NULL,
 * n <= 32768 and n * replicas < 2^31 (EINVAL / ERANGE at cosm_init); its
 * device workspace grows by about 16 n R bytes. */
enum { COSM_READOUT_BISECTORS = 0, COSM_READOUT_OPTIMAL = 1 };
enum { COSM_UNIT_TURNS = 0, COSM_UNIT_DEGREES = 1, COSM_UNIT_RADIANS = 2 };

/* ---- parameters (Tables IX-XI) --------------------------------------------- */
typedef struct {
  double alpha0_deg;        /* initial step size, degrees (14 in Table IX) */
  double dwt_ratio;         /* twist = dwt_ratio * alpha_t (Table X: 0.5 / 1.0 / 1.5) */
  int32_t dwt_period;       /* twist after sweeps t with t % period == 0; 0 = never */
  double dwt_window_deg;    /* width of each of the two windows (90 in Table IX) */
  int32_t n_bisectors;      /* B (100 in Table IX); forced to 1 when h is given */
  int64_t sweeps_per_trial; /* S: the schedule length */
  int32_t schedule;         /* COSM_SCHED_* */
  int32_t storage;          /* COSM_STORE_*: phase storage (FIX16: integer arithmetic) */
  int32_t residency;        /* COSM_RES_* */
  int32_t replicas_per_wg;  /* LDS form: replicas per workgroup; 0 = autotune */
  int32_t threads_per_wg;   /* LDS form: threads per workgroup; 0 = autotune */
  int32_t update;           /* COSM_UPDATE_* */
  int32_t readout;          /* COSM_READOUT_* */
  int32_t lds_form;         /* COSM_LDS_FORM_*: layout of the LDS form (AUTO: measured) */
} cosm_params;

/* Fill *p with Table IX/X defaults: alpha0 14, ratio 0.5, period 3, window 90,
 * B 100, S 1000, GRID, FP32, AUTO, autotuned shape, SCS, BISECTORS. */
void cosm_default_params(cosm_params *p);

typedef struct cosm_state cosm_state;

/* ---- partitions (Sec. II-B, Eqs. (9)-(11)) -------------------------------- */
/* Proper edge colouring of the graph with n vertices and m edges (eu[k], ev[k]).
 *   method GREEDY: edges in input order, each gets the lowest colour free at
 *     both endpoints (Sec. II-B); at most 2*Delta - 1 colours.
 *   method MISRA_GRIES: Misra-Gries fan/path recolouring; at most Delta + 1.
 *   method TORUS: the regular lattice pattern (Sec. II-B); method_args =
 *     {Lx, Ly}, vertex (r, c) = r*Lx + c; every edge must join lattice
 *     neighbours.  Horizontal edges with even / odd left column get colours 0 /
 *     1, vertical edges with even / odd upper row 2 / 3; with an odd side the
 *     wrap-around edges of that direction get their own colour (4 horizontal,
 *     5 vertical), the remaining colours are renumbered to stay contiguous.
 *   method BALANCED: Misra-Gries, then class sizes equalised (largest minus
 *     smallest <= 1 where Kempe swaps allow) by recolouring alternating
 *     two-colour paths; same number of colours.  Appendix B notes that
 *     colourings which balance the edges per colour are admissible.
 *   method MINIMUM: Misra-Gries, then the edges of colour Delta moved into
 *     Delta colours by alternating-path swaps when that succeeds (a minimum
 *     colouring, as the paper's greedy heuristic reached on its non-lattice
 *     graphs, Sec. III-B); Delta + 1 colours otherwise (class-2 graphs); then
 *     equalised as BALANCED.  Deterministic for a given input.
 * method may carry COSM_ORDER_LARGEST_LAST.
 * colour_out[m] (caller-owned) receives the class of every edge; class indices
 * are also the order in which a sweep applies them.  *num_colours_out = C.
 * Errors: EINVAL (NULL, n < 1, endpoint out of range, self-loop, TORUS edge that
 * is not a lattice edge), EDUP (repeated undirected edge). */
int cosm_build_partitions(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                          int32_t method, const int32_t *method_args, int32_t *colour_out,
                          int32_t *num_colours_out);

/* ---- state ------------------------------------------------------------------ */
/* Device bytes cosm_init needs when the caller supplies the workspace. */
int cosm_workspace_bytes(int32_t n, int64_t m, int32_t num_colours, int32_t replicas,
                         const cosm_params *p, size_t *bytes_out);

/* Create a solver state: validates the graph and the colouring, copies them to
 * the device, picks (or takes from p) the sweep kernel's shape, and draws the
 * initial phases of replicas 0..replicas-1 (Algorithm 1, "Set x_i random"):
 * Philox4x32-10 with key = seed, counter (i, 0, replica, "INIT").
 *   J: Ising couplings (Eq. (1) sign), m entries.  h: n entries or NULL (h = 0).
 *     With h the sweep couples every x_i with h_i != 0 to a fixed virtual
 *     spin at phase 0 (coupling h_i), applied by Eq. (6) as one more
 *     conflict-free sub-sweep after the C classes; each twist then rotates in
 *     a direction drawn per (replica, twist) from word 1 of the reference
 *     angle's Philox draw; the readout uses the single semicircle centred at
 *     0 (B is forced to 1).  The paper leaves h out of the dynamics (Eq. (7));
 *     this is the library's reading.  |alpha0 * h_i| is bounded like |J|.
 *   colour / num_colours: as returned by cosm_build_partitions or any proper
 *     colouring; classes are applied in index order.
 *   hip_stream: a hipStream_t or NULL for the default stream.
 *   device_workspace / workspace_bytes: device memory the state uses for all its
 *     buffers (at least cosm_workspace_bytes), owned by the caller, kept alive
 *     until cosm_destroy; NULL makes the library allocate its own.
 * Errors: EINVAL, EDUP, ECOLOR (not a proper colouring), ERANGE (alpha0*|J|,
 * dwt_ratio*alpha0 or the window not below a full turn; GRID with 2*dwt_ratio
 * not an integer or a window off the 2^-23 turn grid; forced LDS residency that
 * does not fit), ENOMEM, EDEVICE. */
int cosm_init(cosm_state **out, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
              const int32_t *J, const int32_t *h, const int32_t *colour, int32_t num_colours,
              const cosm_params *p, uint64_t seed, int32_t replicas, void *hip_stream,
              void *device_workspace, size_t workspace_bytes);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops with a fixed memory footprint, harnesses that forbid
 * hipMalloc): cosm_init with every device buffer of the state placed in a
 * static array the library holds on each GPU (32 MiB per device, kept until
 * the process ends) instead of hipMalloc or a caller workspace.  Arguments and
 * results are those of cosm_init.  The call allocates nothing: no hipMalloc,
 * no HIP event, and the kernel shape is chosen without the timed autotuner
 * (replicas_per_wg / threads_per_wg = 0 take the untimed default).
 * One such state may live per device at a time: the array is shared, so a
 * second cosm_init_static on the same device fails with ESTATE until the first
 * state is cosm_destroy'ed; states made this way on different devices are
 * independent.  The array keeps whatever the last state left in it; every
 * buffer is written before it is read.  Errors: those of cosm_init, ERANGE when
 * cosm_workspace_bytes exceeds 32 MiB, ESTATE as above.  Later calls on the
 * state behave as for cosm_init (cosm_get_phases / cosm_set_phases still
 * allocate a staging buffer; cosm_set_timing creates its events). */
int cosm_init_static(cosm_state **out, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                     const int32_t *J, const int32_t *h, const int32_t *colour,
                     int32_t num_colours, const cosm_params *p, uint64_t seed, int32_t replicas,
                     void *hip_stream);

/* Release the state and everything the library allocated for it. */
int cosm_destroy(cosm_state *s);

/* Redraw the initial phases (sweep counter back to 0) for replicas with global
 * indices replica_offset .. replica_offset+R-1 under a new seed.  Used to run
 * successive trial batches. */
int cosm_reset(cosm_state *s, uint64_t seed, int64_t replica_offset);

/* ---- the sweep (Algorithm 1, main loop) ----------------------------------- */
/* Run sweeps t+1 .. t+n_sweeps on every replica (t = sweeps already done),
 * asynchronously on the state's stream.  ERANGE if t + n_sweeps > S. */
int cosm_sweep(cosm_state *s, int64_t n_sweeps);

/* ---- readout and energy (Algorithm 1 binarization; Eq. (1); Eq. (14)) ---- */
/* spins == NULL: binarize the current phases of every replica (B bisectors
 * beta_p = p/(2B) turn rounded to the grid, +1 on [beta_p, beta_p + 1/2),
 * lowest H kept, lowest p on ties; with h a single semicircle centred at 0).
 * spins != NULL: [R][n] int8 in {-1,+1} supplied by the caller; its energies.
 * spins_out ([R][n] int8) may be NULL; H_out and cut_out ([R] int64) must not.
 * Synchronises the stream.  EINVAL on a spin outside {-1,+1}. */
int cosm_energy(cosm_state *s, const int8_t *spins, int8_t *spins_out, int64_t *H_out,
                int64_t *cut_out);

/* ---- trials and time to target (Appendix A, Eqs. (15)-(17)) --------------- */
typedef struct {
  int64_t trials;      /* replicas run */
  int64_t successes;   /* replicas whose final H <= target */
  double ps;           /* successes / trials */
  double ps_lo, ps_hi; /* Wilson 95% interval of ps */
  double r99;          /* Eq. (15); 1 for ps = 1, +inf for ps = 0 */
  double t_trial_s;    /* batch wall time / replicas, init to readout inclusive */
  double ttt_s;        /* Eq. (17): t_trial * R99 */
  double stt_sweeps;   /* Eq. (16): S * R99 */
  int64_t best_H;      /* lowest H seen */
  int64_t best_cut;    /* its cut */
} cosm_tts_result;

/* Run batches of R independent trials (each: cosm_reset with the next replica
 * offset, S sweeps, readout) until max_trials replicas have run, or after the
 * first batch with a hit when stop_at_first_hit != 0.  best_spins ([n] int8)
 * may be NULL.  Leaves the state holding the last batch. */
int cosm_solve_to_target(cosm_state *s, int64_t target_H, int64_t max_trials,
                         int32_t stop_at_first_hit, cosm_tts_result *out, int8_t *best_spins);

/* ---- many instances in one persistent launch ------------------------------- */
/* A batch holds instances of uneven sizes (each with its own couplings,
 * colouring, parameters, seed and replica count) and runs whole trials of any
 * subset of them with one persistent sweep launch: work items (instance, first
 * replica, replica sets) are taken from a device counter by one workgroup per
 * CU; a small instance packs several replica sets into one workgroup's LDS.
 * Init, sweeps and readout are captured once into a hipGraph and replayed by
 * every run.  Trajectories are the same as cosm_init / cosm_sweep / cosm_energy
 * with the same seed and replica offset.  Storage is fixed per batch; the SCS
 * update only; no bias fields. */
typedef struct cosm_batch cosm_batch;
/* max_graphs: instances the batch can hold; max_n: largest instance (<= 65536);
 * max_bisectors: largest B; hip_stream: NULL makes the batch use a stream of its
 * own (a graph cannot be captured on the legacy default stream).  ERANGE if a
 * readout of max_n spins does not fit in LDS. */
int cosm_batch_create(cosm_batch **out, int32_t storage, int32_t max_graphs, int32_t max_n,
                      int32_t max_bisectors, void *hip_stream);
int cosm_batch_destroy(cosm_batch *b);
/* Add an instance (arguments as cosm_init; p->storage must match the batch).
 * Uploads it, builds its lane schedule, and returns its id (0, 1, ...).  The
 * replicas per set (row width) are p->replicas_per_wg when given, else the
 * width with the least time per replica among those that fit, measured by
 * short probe runs of one full work item of the instance (as many replica
 * sets as fit one workgroup, up to 128 sweeps; the stream is synchronised;
 * results are cached per process by the instance's sizes, storage, replicas,
 * sweeps and a hash of its edges and colouring). */
int cosm_batch_add_graph(cosm_batch *b, int32_t n, int64_t m, const int32_t *eu,
                         const int32_t *ev, const int32_t *J, const int32_t *colour,
                         int32_t num_colours, const cosm_params *p, uint64_t seed,
                         int32_t replicas, int32_t *graph_id_out);
/* The shape an instance runs in: replicas per set, sets per work item, and
 * how it was chosen (tuned: 0 one width fits or was requested, 1 timed probes,
 * 2 the probe cache) with the chosen width's probe time (ms, one work item;
 * 0 when not probed), and lazy_wrap: 1 when its phases are wrapped at the
 * twists only (FP16 / BF16 / FP16_PK within the drift bound of cosm_info.lazy_wrap).
 * Any output pointer may be NULL. */
int cosm_batch_graph_shape(const cosm_batch *b, int32_t graph_id, int32_t *replicas_per_set,
                           int32_t *sets_per_item, int32_t *tuned, double *probe_ms,
                           int32_t *lazy_wrap);
/* Seed and global index of replica 0 used by the next run of that instance. */
int cosm_batch_set_seed(cosm_batch *b, int32_t graph_id, uint64_t seed, int64_t replica_offset);
/* Enqueue one whole trial (init, S sweeps, readout) of every listed instance.
 * Asynchronous; host tables are copied before returning. */
int cosm_batch_run(cosm_batch *b, const int32_t *graph_ids, int32_t count);
/* Wait for the last run; *device_ms_out (may be NULL) = its device time. */
int cosm_batch_wait(cosm_batch *b, double *device_ms_out);
/* Non-blocking check of the last run: *done_out = 1 once its work (init,
 * sweeps, readout) has finished on the device, else 0.  Never waits, so a
 * serving loop can keep submitting to other batches; 1 before any run. */
int cosm_batch_poll(cosm_batch *b, int32_t *done_out);
/* Results of an instance's last run: H, cut ([R] int64) and spins ([R][n]); any
 * output may be NULL.  Synchronises the batch's stream. */
int cosm_batch_results(cosm_batch *b, int32_t graph_id, int64_t *H_out, int64_t *cut_out,
                       int8_t *spins_out);

/* ---- phase access ------------------------------------------------------------ */
/* Copy the phases out as [R][n] doubles in the given unit (COSM_UNIT_*); turns
 * and degrees are exact.  Synchronises the stream. */
int cosm_get_phases(cosm_state *s, int32_t unit, double *out);
/* Overwrite the phases from [R][n] doubles in the given unit (wrapped into one
 * turn, rounded to the storage format) and set the sweep counter to t. */
int cosm_set_phases(cosm_state *s, int32_t unit, const double *in, int64_t t);

/* ---- QUBO inputs -------------------------------------------------------------- */
/* Map the QUBO  min E(x) = sum_k qv[k] x_{qi[k]} x_{qj[k]},  x in {0,1}^n, to the
 * Ising form of Eq. (1) with s = 2x - 1:  4 E(x) = H(s) + *offset_out, where
 * J_uv = -(sum of qv over off-diagonal terms on {u, v}, either order),
 * h_i = -(sum of qv over off-diagonal terms touching i) - 2 (sum of qv[k] with
 * qi = qj = i).  Repeated terms add up; pairs whose J sums to 0 are dropped.
 * Outputs (caller-owned): eu_out, ev_out, J_out with room for nnz edges,
 * sorted by (u, v) with u < v, *m_out edges written; h_out[n]; *offset_out.
 * Pass the result to cosm_init with h = h_out (a state with h reads out with
 * the single semicircle; minimising H minimises E).  Host only.
 * EINVAL (n < 1, NULL, index out of range), ERANGE (a sum overflows int32). */
int cosm_qubo_to_ising(int32_t n, int64_t nnz, const int32_t *qi, const int32_t *qj,
                       const int32_t *qv, int32_t *eu_out, int32_t *ev_out, int32_t *J_out,
                       int64_t *m_out, int32_t *h_out, int64_t *offset_out);

/* ---- introspection ---------------------------------------------------------- */
typedef struct {
  int32_t n, num_colours, replicas;
  int64_t m, sweeps_done;
  int32_t residency;       /* resolved COSM_RES_* */
  int32_t storage;
  int32_t replicas_per_wg; /* resolved */
  int32_t threads_per_wg;  /* resolved */
  int32_t workgroups;
  int32_t lds_bytes;       /* dynamic LDS per workgroup */
  int32_t max_class_edges;
  int64_t sweep_launches;  /* sweep kernels launched so far */
  double sweep_kernel_ms;  /* their summed duration (HIP events), when timing is on */
  int32_t lds_form;        /* resolved COSM_LDS_FORM_* (0 outside the LDS form) */
  int32_t register_rows;   /* REGISTER: register vertices per thread */
  int32_t twist_fused;     /* 1: the LDS sweep applies the twist inside the last class's
                              sub-sweep (same result as a pass after the classes) */
  int32_t register_vertices; /* REGISTER: vertices whose phases stay in registers */
  int64_t register_edges;  /* REGISTER: edges with an endpoint in registers (one LDS row
                              read and written per update instead of two) */
  int32_t streamed;        /* 1: the LDS sweep streams its lane schedule from memory, two
                              slots in flight per wave (long schedules: the large graphs) */
  int32_t lazy_wrap;       /* 1: phases are wrapped only at the twists, not after every
                              update, because no phase can drift by 1/2 turn from its
                              wrapped range between two twists (twist + period x alpha0 x
                              largest sum of |J| and |h| at a vertex < 1/2 turn): FP32 in
                              the streamed LDS forms on the grid schedule (the result is
                              the same bit for bit), FP16 / BF16 / FP16_PK in every form (the
                              centred value y then lies in (-1, 1) between twists) */
} cosm_info;
int cosm_get_info(const cosm_state *s, cosm_info *out);

/* Time every sweep kernel with HIP events on the state's stream (on != 0). */
int cosm_set_timing(cosm_state *s, int32_t on);

/* LDS bandwidth ceiling of the current device for the sweep's access mix,
 * measured with the library's own kernel: every lane reads two rows of
 * row_words (1, 2 or 4) 32-bit words, adds one to each word and writes both
 * back (2 reads + 2 writes, as per edge of a sweep, without the arithmetic), rows
 * of consecutive lanes in distinct banks, blocks_per_cu (1 or 2) workgroups of
 * 768 threads per compute unit, no barriers.  Writes the aggregate LDS bytes
 * (reads + writes) per second over all compute units, in GB/s, to *gbs_out.
 * Runs on hip_stream (NULL: the default stream) and synchronises it.
 * EINVAL for other row_words / blocks_per_cu, EDEVICE on a HIP error. */
int cosm_lds_probe(int32_t row_words, int32_t blocks_per_cu, void *hip_stream, double *gbs_out);

const char *cosm_last_error(void);
const char *cosm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* COSM_H */
