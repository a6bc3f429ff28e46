/*
 * cosm_oracle.h -- plain FP64 CPU oracle for the Cosm sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this code.  The product
 * library (libcosm.so) never links it, and this code includes no header and
 * shares no source with the product.
 *
 * The oracle follows the paper "Cosm: Collective Switched Motion for Fast and
 * Accurate Sparse Ising Optimization" (Zick, Shukla, Marakov):
 *   - Ising energy, Eq. (1); Max-Cut form and w = -J, Appendix A, Eq. (14);
 *   - circular variables in degrees on [0, 360) with non-negative mod, Sec. II-A;
 *   - relaxed coupling v and objective f, Eqs. (2), (3), (7) (diagnostic);
 *   - biased sign and pair contributions, Eqs. (4)-(6);
 *   - sequential conflict-free search over a proper edge colouring,
 *     Eqs. (9)-(13), Sec. II-C;
 *   - dual window twist, Sec. II-D and Algorithm 1;
 *   - linear step-size ramp alpha0 -> 0, updated once per sweep (Sec. II-B,
 *     Appendix B);
 *   - binarization by equally spaced bisectors over a semicircle (Algorithm 1,
 *     Appendix B);
 *   - R99 / STT / TTT, Appendix A, Eqs. (15)-(17);
 *   - greedy edge colouring "lowest colour available, looping over the edges"
 *     (Sec. II-B).
 * Readings where the paper is silent are listed with each function.
 *
 * Phase unit: degrees, FP64.  "Grid" schedule: every phase, step and angle is a
 * multiple of q = 360 * 2^-23 degrees, so every operation below is exact in
 * FP64 (and, scaled to turns, in FP32).  "Grid16" is the same construction on
 * q16 = 360 * 2^-16 degrees (steps on 2 q16), for phases held in 16-bit fixed
 * point; bisectors stay on the q grid.
 */
#ifndef COSM_ORACLE_H
#define COSM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SCHED_GRID = 0, ORC_SCHED_CONTINUOUS = 1, ORC_SCHED_GRID16 = 2 };
enum { ORC_UPDATE_SCS = 0, ORC_UPDATE_FULL_GRADIENT = 1 };

/* Counter words that separate the random streams (last Philox counter word). */
#define ORC_TAG_INIT 0x494E4954u /* "INIT" */
#define ORC_TAG_DWT  0x44575420u /* "DWT " */

typedef struct {
  int32_t n;            /* number of spins */
  int64_t m;            /* number of edges */
  const int32_t *eu;    /* [m] first endpoint (the "i" of Eq. (6)) */
  const int32_t *ev;    /* [m] second endpoint (the "j" of Eq. (6)) */
  const int32_t *J;     /* [m] Ising coupling, Eq. (1) sign */
  const int32_t *h;     /* [n] bias field or NULL */
  const int32_t *colour;/* [m] class of each edge, 0..C-1; classes run in index order */
  int32_t C;            /* number of classes */
} orc_problem;

typedef struct {
  double alpha0_deg;     /* initial step size, degrees */
  double dwt_ratio;      /* twist = ratio * alpha_t */
  int32_t dwt_period;    /* twist when sweep % period == 0; 0 disables the twist */
  double dwt_window_deg; /* width of each of the two windows, degrees */
  int32_t n_bisectors;   /* B */
  int64_t sweeps;        /* S, length of the schedule */
  int32_t schedule;      /* ORC_SCHED_* */
  int32_t update;        /* ORC_UPDATE_* */
} orc_params;

/* Philox4x32-10, Salmon et al., "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Greedy edge colouring: edges in input order, each takes the lowest colour not
 * yet used at either endpoint.  Returns the number of colours, or -1 on a
 * self-loop / out-of-range endpoint. */
int32_t orc_greedy_colouring(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                             int32_t *colour);

/* 1 if colour[] is a proper edge colouring with classes 0..C-1 (each class a
 * matching, every edge coloured), else 0. */
int32_t orc_is_proper_colouring(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                                const int32_t *colour, int32_t C);

/* Step size of sweep t (1-based), degrees. */
double orc_alpha(const orc_params *p, int64_t t);

/* Bisector angle beta_p (0 <= p < B), degrees. */
double orc_bisector(const orc_params *p, int32_t schedule, int32_t idx);

/* Random initial phases for replicas rid0 .. rid0+R-1; x is [R][n], degrees. */
void orc_init_phases(int32_t n, uint64_t seed, int64_t rid0, int32_t R, int32_t schedule,
                     double *x);

/* DWT reference angle for (sweep t, replica rid), degrees (q grid). */
double orc_theta_ref(uint64_t seed, int64_t t, int64_t rid);
/* The same draw on the schedule's grid: the top 16 bits for ORC_SCHED_GRID16. */
double orc_theta_ref_sched(uint64_t seed, int64_t t, int64_t rid, int32_t schedule);

/* Twist direction (+1 / -1) for (sweep t, replica rid), used only with bias
 * fields; word 1 of the reference angle's Philox draw. */
int32_t orc_twist_direction(uint64_t seed, int64_t t, int64_t rid);

/* Run sweeps t_from+1 .. t_from+n_sweeps for R replicas (rows of x, [R][n]).
 * If margin is not NULL, margin[r] receives the smallest distance (degrees) of
 * any sign decision, window edge or wrap point from its threshold during the
 * first diag_sweeps of these sweeps (near-tie diagnostic).  n_threads <= 0
 * uses the OpenMP default.  Returns 0, or -1 on bad arguments. */
int32_t orc_sweeps(const orc_problem *pb, const orc_params *p, uint64_t seed, int64_t rid0,
                   int32_t R, int64_t t_from, int64_t n_sweeps, double *x, double *margin,
                   int64_t diag_sweeps, int32_t n_threads);

/* Energy, Eq. (1), and cut, Eq. (14) with w = -J, for spins [R][n] in {-1,+1}. */
void orc_energy(const orc_problem *pb, int32_t R, const int8_t *spins, int64_t *H, int64_t *cut);

/* Relaxed coupling v of Eq. (2) for two phases in degrees: 1 at equal phases,
 * -1 diametrically opposite, linear in the shorter angular distance between. */
double orc_coupling_v(double xi, double xj);

/* Relaxed objective f(x) of Eq. (7) for x [R][n] (degrees) into f [R]: the sum
 * of the pair energies -J v of Eq. (3); with bias fields each h_i adds the pair
 * term of a coupling h_i to a fixed spin at phase 0 (the reading the sweep
 * uses).  At phases restricted to {0, 180} f equals H of Eq. (1). */
void orc_relaxed_objective(const orc_problem *pb, int32_t R, const double *x, double *f);

/* Binarize x ([R][n], degrees) by B bisectors, keeping the lowest-H one (lowest
 * index on ties); with h present a single semicircle centred at 0.
 * spins [R][n] (may be NULL), H [R], cut [R], best_p [R] (may be NULL). */
void orc_readout(const orc_problem *pb, const orc_params *p, int32_t R, const double *x,
                 int8_t *spins, int64_t *H, int64_t *cut, int32_t *best_p);

/* Optimal-bisector binarization: every distinct x_i mod 180 tried as the
 * bisector by brute force, lowest H kept, smallest angle on ties; h must be
 * NULL.  spins [R][n] (may be NULL), H [R], cut [R], beta_out [R] (may be
 * NULL, degrees).  Returns 0, or -1 with bias fields. */
int32_t orc_readout_optimal(const orc_problem *pb, int32_t R, const double *x, int8_t *spins,
                            int64_t *H, int64_t *cut, double *beta_out);

/* Exhaustive ground state for n <= 26.  Returns 0 or -1 if n is too large. */
int32_t orc_brute_force_ground_state(const orc_problem *pb, int8_t *best_spins, int64_t *H);

/* R99 of Eq. (15); returns 1 for P_s = 1 and +inf for P_s = 0. */
double orc_r99(double ps);

#ifdef __cplusplus
}
#endif
#endif
