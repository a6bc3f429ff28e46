/*
 * cosm_oracle.c -- plain FP64 CPU oracle for the Cosm sweep.
 *
 * TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg are the only users.  Shares no code with the product.
 *
 * Every function is written for clarity, not speed: phases are doubles in
 * degrees, the paper's unit, and each step of the method is a direct
 * transcription of the equation it cites (see cosm_oracle.h for the list).
 *
 * Parity pins: Philox known-answer vectors; closed-form ground states;
 * energy/cut identity (Appendix A) and the G70 worked example; printed R99
 * values of Tables II and VI; dynamical invariants (sum of phases conserved by
 * sub-sweeps, |dx| = alpha|J|, gauge symmetry, window measure); the circular
 * conflict trap of Figs. 2 and 4.  The whole long-run trajectory has no
 * printed reference in the paper: parity unpinned beyond those invariants.
 */
#include "cosm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                         */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) { /* key schedule: the key is bumped before every round but the first */
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t philox_word0(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[0];
}

/* ------------------------------------------------------------------------ */
/* Modular helpers, Sec. II-A: x in [0, 360), "mod returns a non-negative     */
/* remainder".                                                               */
/* ------------------------------------------------------------------------ */
static double mod_pos(double y, double period) {
  double r = y - period * floor(y / period);
  if (r >= period) r -= period; /* rounding can land exactly on the period */
  if (r < 0.0) r += period;
  return r;
}

/* Minimum angular difference in [-180, 180), from the mod form of Eq. (2). */
static double wrapped_difference(double d) { return mod_pos(d + 180.0, 360.0) - 180.0; }

/* Biased sign of Eq. (4): +1 for a non-negative argument. */
static int sgn_b(double a) { return a >= 0.0 ? 1 : -1; }

/* ------------------------------------------------------------------------ */
/* Edge colouring, Sec. II-B ("loops over the edges and assigns the lowest    */
/* color number available").                                                 */
/* ------------------------------------------------------------------------ */
int32_t orc_greedy_colouring(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                             int32_t *colour) {
  /* used[v] lists the colours already present at vertex v. */
  int32_t **used = (int32_t **)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t *));
  int32_t *cnt = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int32_t *cap = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int32_t C = 0;
  for (int64_t k = 0; k < m; k++) {
    int32_t u = eu[k], v = ev[k];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) { C = -1; break; }
    int32_t c = 0;
    for (;;) { /* lowest colour used at neither endpoint */
      int taken = 0;
      for (int32_t a = 0; a < cnt[u] && !taken; a++) taken = (used[u][a] == c);
      for (int32_t a = 0; a < cnt[v] && !taken; a++) taken = (used[v][a] == c);
      if (!taken) break;
      c++;
    }
    colour[k] = c;
    if (c + 1 > C) C = c + 1;
    int32_t ends[2] = {u, v};
    for (int e = 0; e < 2; e++) {
      int32_t w = ends[e];
      if (cnt[w] == cap[w]) {
        cap[w] = cap[w] ? 2 * cap[w] : 4;
        used[w] = (int32_t *)realloc(used[w], (size_t)cap[w] * sizeof(int32_t));
      }
      used[w][cnt[w]++] = c;
    }
  }
  for (int32_t i = 0; i < n; i++) free(used[i]);
  free(used); free(cnt); free(cap);
  return C;
}

int32_t orc_is_proper_colouring(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                                const int32_t *colour, int32_t C) {
  if (C < 0) return 0;
  /* seen[c*n + v] = 1 once some class-c edge touches v (Eqs. (9)-(10): each class a matching) */
  size_t cells = (size_t)(C > 0 ? C : 1) * (size_t)(n > 0 ? n : 1);
  unsigned char *seen = (unsigned char *)calloc(cells, 1);
  int ok = 1;
  for (int64_t k = 0; k < m && ok; k++) {
    int32_t c = colour[k], u = eu[k], v = ev[k];
    if (c < 0 || c >= C || u < 0 || v < 0 || u >= n || v >= n || u == v) { ok = 0; break; }
    if (seen[(size_t)c * n + u] || seen[(size_t)c * n + v]) { ok = 0; break; }
    seen[(size_t)c * n + u] = 1;
    seen[(size_t)c * n + v] = 1;
  }
  free(seen);
  return ok;
}

/* ------------------------------------------------------------------------ */
/* Schedules and angles.                                                     */
/* ------------------------------------------------------------------------ */
/* Grid quantum: q = 360 * 2^-23 degrees.  Steps use 2q so that half a step is
 * still on the grid. */
static const double TWO_POW_23 = 8388608.0;
static const double TWO_POW_22 = 4194304.0;
static const double TWO_POW_16 = 65536.0;
static const double TWO_POW_15 = 32768.0;

/* The 16-bit grid (ORC_SCHED_GRID16): phases and angles are multiples of
 * 360 * 2^-16 degrees and steps of 360 * 2^-15, the same construction one
 * level coarser, so that phases fit 16-bit fixed point exactly. */
static double step_units_per_turn(int32_t schedule) {
  return schedule == ORC_SCHED_GRID16 ? TWO_POW_15 : TWO_POW_22;
}

static int64_t alpha0_grid_units(const orc_params *p) {
  /* alpha0 in step units (360 * 2^-22 or 2^-15 degrees), nearest integer */
  return (int64_t)floor(p->alpha0_deg / 360.0 * step_units_per_turn(p->schedule) + 0.5);
}

/* Linear ramp alpha0 -> 0, constant within a sweep (Sec. II-B, Appendix B):
 * sweep t (1-based) uses alpha0 * (S - t + 1) / S, so the value after the last
 * update is 0.  Grid schedule: the same ramp rounded to the 2q grid with
 * integer arithmetic. */
double orc_alpha(const orc_params *p, int64_t t) {
  int64_t S = p->sweeps;
  if (p->schedule != ORC_SCHED_CONTINUOUS) {
    int64_t a0 = alpha0_grid_units(p);
    int64_t units = (a0 * (S - t + 1) + S / 2) / S;
    return (double)units * 360.0 / step_units_per_turn(p->schedule);
  }
  return p->alpha0_deg * (double)(S - t + 1) / (double)S;
}

/* Bisector p of B, equally spaced over a semicircle starting at 0 (Appendix B:
 * 100 bisectors spaced by 1.8 degrees).  Grid schedule: rounded half-up to q. */
double orc_bisector(const orc_params *p, int32_t schedule, int32_t idx) {
  int64_t B = p->n_bisectors;
  if (schedule != ORC_SCHED_CONTINUOUS) {
    int64_t units = ((int64_t)idx * (int64_t)TWO_POW_23 + B) / (2 * B);
    return (double)units * 360.0 / TWO_POW_23;
  }
  return 180.0 * (double)idx / (double)B;
}

/* Algorithm 1, "Set x_i random": uniform on [0, 360) from Philox word 0 of
 * counter (i, 0, rid, INIT).  Grid: the top 23 bits; continuous: the top 24. */
void orc_init_phases(int32_t n, uint64_t seed, int64_t rid0, int32_t R, int32_t schedule,
                     double *x) {
  for (int32_t r = 0; r < R; r++) {
    uint32_t rid = (uint32_t)(rid0 + r);
    for (int32_t i = 0; i < n; i++) {
      uint32_t w = philox_word0(seed, (uint32_t)i, 0u, rid, ORC_TAG_INIT);
      double v;
      if (schedule == ORC_SCHED_GRID)
        v = (double)(w >> 9) * 360.0 / TWO_POW_23;
      else if (schedule == ORC_SCHED_GRID16)
        v = (double)(w >> 16) * 360.0 / TWO_POW_16;
      else
        v = (double)(w >> 8) * 360.0 / (2.0 * TWO_POW_23);
      x[(size_t)r * n + i] = v;
    }
  }
}

/* DWT reference angle (Algorithm 1, "Select random reference angle"): one per
 * (sweep, replica), uniform on the grid, Philox counter (0, t, rid, DWT). */
double orc_theta_ref(uint64_t seed, int64_t t, int64_t rid) {
  uint32_t w = philox_word0(seed, 0u, (uint32_t)t, (uint32_t)rid, ORC_TAG_DWT);
  return (double)(w >> 9) * 360.0 / TWO_POW_23;
}

double orc_theta_ref_sched(uint64_t seed, int64_t t, int64_t rid, int32_t schedule) {
  if (schedule != ORC_SCHED_GRID16) return orc_theta_ref(seed, t, rid);
  uint32_t w = philox_word0(seed, 0u, (uint32_t)t, (uint32_t)rid, ORC_TAG_DWT);
  return (double)(w >> 16) * 360.0 / TWO_POW_16;
}

/* Direction of the twist.  Without bias fields one direction suffices
 * (Sec. II-D) and it is always +.  With bias fields the rotation sense matters,
 * so each twist event draws it: -1 when the top bit of word 1 of the same
 * Philox draw as theta is set, else +1 (a reading; the paper gives no rule). */
int32_t orc_twist_direction(uint64_t seed, int64_t t, int64_t rid) {
  uint32_t ctr[4] = {0u, (uint32_t)t, (uint32_t)rid, ORC_TAG_DWT};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return (out[1] >> 31) ? -1 : 1;
}

/* ------------------------------------------------------------------------ */
/* One replica's sweeps.                                                      */
/* ------------------------------------------------------------------------ */
static double dmin(double a, double b) { return a < b ? a : b; }

/* Distance of a wrapped difference from the sign thresholds 0 and -180/180. */
static double decision_margin(double dw) {
  return dmin(fabs(dw), dmin(fabs(dw + 180.0), fabs(dw - 180.0)));
}

/* class_start[c] .. class_start[c+1]-1 index class_edges[], the edges of
 * class c in input order. */
static void run_replica(const orc_problem *pb, const orc_params *p, uint64_t seed, int64_t rid,
                        int64_t t_from, int64_t n_sweeps, double *x, double *margin,
                        int64_t diag_sweeps, const int64_t *class_start,
                        const int64_t *class_edges) {
  const int32_t n = pb->n;
  double min_margin = 1e300;
  double *acc = NULL; /* full-gradient accumulator */
  if (p->update == ORC_UPDATE_FULL_GRADIENT) acc = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));

  for (int64_t t = t_from + 1; t <= t_from + n_sweeps; t++) {
    const double alpha = orc_alpha(p, t);
    const int diag = margin != NULL && (t - t_from) <= diag_sweeps;

    if (p->update == ORC_UPDATE_SCS) {
      /* Eqs. (12)-(13): the classes are applied one after another, c = 0..C-1;
       * within a class the edges are disjoint, so their order is immaterial. */
      for (int32_t c = 0; c < pb->C; c++) {
        for (int64_t e = class_start[c]; e < class_start[c + 1]; e++) {
          const int64_t k = class_edges[e];
          const int32_t i = pb->eu[k], j = pb->ev[k];
          /* Eq. (4) on the minimum angular difference (Fig. 1 caption) */
          const double dw = wrapped_difference(x[i] - x[j]);
          const int s = sgn_b(dw);
          if (diag) min_margin = dmin(min_margin, decision_margin(dw));
          /* Eq. (6) */
          const double dxi = -alpha * (double)pb->J[k] * (double)s;
          const double dxj = +alpha * (double)pb->J[k] * (double)s;
          x[i] = mod_pos(x[i] + dxi, 360.0);
          x[j] = mod_pos(x[j] + dxj, 360.0);
        }
      }
      /* Bias fields (a reading; the paper leaves h out of the dynamics,
       * Eq. (7)): h_i couples x_i to a fixed virtual spin at phase 0 with
       * coupling h_i, applied by Eq. (6) as one more conflict-free sub-sweep
       * after the C classes; the virtual spin does not move. */
      if (pb->h != NULL) {
        for (int32_t i = 0; i < n; i++) {
          if (pb->h[i] == 0) continue;
          const double dw = wrapped_difference(x[i] - 0.0);
          const int s = sgn_b(dw);
          if (diag) min_margin = dmin(min_margin, decision_margin(dw));
          x[i] = mod_pos(x[i] - alpha * (double)pb->h[i] * (double)s, 360.0);
        }
      }
    } else {
      /* Eq. (8): every edge reads x_t, contributions are summed per variable. */
      for (int32_t i = 0; i < n; i++) acc[i] = 0.0;
      for (int64_t k = 0; k < pb->m; k++) {
        const int32_t i = pb->eu[k], j = pb->ev[k];
        const double dw = wrapped_difference(x[i] - x[j]);
        const int s = sgn_b(dw);
        if (diag) min_margin = dmin(min_margin, decision_margin(dw));
        acc[i] += -alpha * (double)pb->J[k] * (double)s;
        acc[j] += +alpha * (double)pb->J[k] * (double)s;
      }
      /* the virtual spin at phase 0 is one more neighbour (coupling h_i) */
      if (pb->h != NULL) {
        for (int32_t i = 0; i < n; i++) {
          if (pb->h[i] == 0) continue;
          const double dw = wrapped_difference(x[i] - 0.0);
          if (diag) min_margin = dmin(min_margin, decision_margin(dw));
          acc[i] += -alpha * (double)pb->h[i] * (double)sgn_b(dw);
        }
      }
      for (int32_t i = 0; i < n; i++) x[i] = mod_pos(x[i] + acc[i], 360.0);
    }

    /* Dual window twist, Algorithm 1 and Sec. II-D: two opposing windows of
     * width w centred at theta and theta + 180; members (tested on the
     * pre-twist phases) rotate by ratio * alpha_t, in the + direction without
     * bias fields and in a drawn direction with them. */
    if (p->dwt_period > 0 && t % p->dwt_period == 0) {
      const double theta = orc_theta_ref_sched(seed, t, rid, p->schedule);
      const double w = p->dwt_window_deg;
      const double dir = pb->h != NULL ? (double)orc_twist_direction(seed, t, rid) : 1.0;
      const double twist = dir * p->dwt_ratio * alpha;
      for (int32_t i = 0; i < n; i++) {
        const double pos = mod_pos(x[i] - theta + 0.5 * w, 180.0);
        if (diag) min_margin = dmin(min_margin, dmin(pos, dmin(fabs(pos - w), 180.0 - pos)));
        if (pos < w) x[i] = mod_pos(x[i] + twist, 360.0);
      }
    }
  }
  free(acc);
  if (margin != NULL) *margin = min_margin;
}

int32_t orc_sweeps(const orc_problem *pb, const orc_params *p, uint64_t seed, int64_t rid0,
                   int32_t R, int64_t t_from, int64_t n_sweeps, double *x, double *margin,
                   int64_t diag_sweeps, int32_t n_threads) {
  if (pb == NULL || p == NULL || x == NULL || R < 0 || t_from < 0 || n_sweeps < 0) return -1;
  if (t_from + n_sweeps > p->sweeps) return -1;
  if (p->n_bisectors <= 0 || p->sweeps <= 0) return -1;
  for (int64_t k = 0; k < pb->m; k++)
    if (pb->colour[k] < 0 || pb->colour[k] >= pb->C) return -1;
  /* Group the edges by class (stable). */
  int64_t *class_start = (int64_t *)calloc((size_t)pb->C + 1, sizeof(int64_t));
  int64_t *class_edges = (int64_t *)malloc((size_t)(pb->m > 0 ? pb->m : 1) * sizeof(int64_t));
  int64_t *fill = (int64_t *)calloc((size_t)pb->C + 1, sizeof(int64_t));
  for (int64_t k = 0; k < pb->m; k++) class_start[pb->colour[k] + 1]++;
  for (int32_t c = 0; c < pb->C; c++) class_start[c + 1] += class_start[c];
  for (int64_t k = 0; k < pb->m; k++) {
    const int32_t c = pb->colour[k];
    class_edges[class_start[c] + fill[c]++] = k;
  }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int32_t r = 0; r < R; r++) {
    run_replica(pb, p, seed, rid0 + r, t_from, n_sweeps, x + (size_t)r * pb->n,
                margin ? margin + r : NULL, diag_sweeps, class_start, class_edges);
  }
  (void)n_threads;
  free(class_start);
  free(class_edges);
  free(fill);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Energy and cut, Eq. (1) and Eq. (14) with w = -J.                          */
/* ------------------------------------------------------------------------ */
static void energy_one(const orc_problem *pb, const int8_t *s, int64_t *H, int64_t *cut) {
  int64_t e = 0, c = 0;
  for (int64_t k = 0; k < pb->m; k++) {
    const int32_t i = pb->eu[k], j = pb->ev[k];
    e -= (int64_t)pb->J[k] * (int64_t)s[i] * (int64_t)s[j];
    if (s[i] != s[j]) c += -(int64_t)pb->J[k]; /* weight w = -J on every cut edge */
  }
  if (pb->h != NULL)
    for (int32_t i = 0; i < pb->n; i++) e -= (int64_t)pb->h[i] * (int64_t)s[i];
  *H = e;
  *cut = c;
}

void orc_energy(const orc_problem *pb, int32_t R, const int8_t *spins, int64_t *H, int64_t *cut) {
  for (int32_t r = 0; r < R; r++)
    energy_one(pb, spins + (size_t)r * pb->n, H + r, cut + r);
}

/* ------------------------------------------------------------------------ */
/* Relaxed coupling and objective, Eqs. (2), (3) and (7) (a diagnostic: the    */
/* sweep itself only evaluates the sign of Eq. (4)).                          */
/* ------------------------------------------------------------------------ */
double orc_coupling_v(double xi, double xj) {
  return 1.0 - fabs(wrapped_difference(xi - xj)) / 90.0;
}

void orc_relaxed_objective(const orc_problem *pb, int32_t R, const double *x, double *f) {
  for (int32_t r = 0; r < R; r++) {
    const double *xr = x + (size_t)r * pb->n;
    double acc = 0.0;
    for (int64_t k = 0; k < pb->m; k++)
      acc -= (double)pb->J[k] * orc_coupling_v(xr[pb->eu[k]], xr[pb->ev[k]]);
    /* bias fields: the same pair term against a fixed spin at phase 0 */
    if (pb->h != NULL)
      for (int32_t i = 0; i < pb->n; i++) acc -= (double)pb->h[i] * orc_coupling_v(xr[i], 0.0);
    f[r] = acc;
  }
}

/* ------------------------------------------------------------------------ */
/* Binarization, Algorithm 1 (final loop) and Appendix B.                      */
/* ------------------------------------------------------------------------ */
void orc_readout(const orc_problem *pb, const orc_params *p, int32_t R, const double *x,
                 int8_t *spins, int64_t *H, int64_t *cut, int32_t *best_p) {
  const int32_t n = pb->n;
  int8_t *cand = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
  int8_t *best = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
  for (int32_t r = 0; r < R; r++) {
    const double *xr = x + (size_t)r * n;
    int64_t bestH = 0, bestCut = 0;
    int32_t bp = -1;
    if (pb->h != NULL) {
      /* With bias fields the semicircles are fixed (Sec. II-B): the half centred
       * at 0 degrees is +1. */
      for (int32_t i = 0; i < n; i++) best[i] = mod_pos(xr[i] + 90.0, 360.0) < 180.0 ? 1 : -1;
      energy_one(pb, best, &bestH, &bestCut);
      bp = 0;
    } else {
      for (int32_t q = 0; q < p->n_bisectors; q++) {
        const double beta = orc_bisector(p, p->schedule, q);
        for (int32_t i = 0; i < n; i++)
          cand[i] = mod_pos(xr[i] - beta, 360.0) < 180.0 ? 1 : -1; /* +1 on [beta, beta+180) */
        int64_t e, c;
        energy_one(pb, cand, &e, &c);
        if (bp < 0 || e < bestH) { /* strict: the lowest index wins ties */
          bestH = e;
          bestCut = c;
          bp = q;
          memcpy(best, cand, (size_t)n);
        }
      }
    }
    H[r] = bestH;
    cut[r] = bestCut;
    if (best_p) best_p[r] = bp;
    if (spins) memcpy(spins + (size_t)r * n, best, (size_t)n);
  }
  free(cand);
  free(best);
}

/* ------------------------------------------------------------------------ */
/* Optimal bisector (the exact best line through the origin, as in the         */
/* Burer-Monteiro-Zhang rank-2 rounding the paper cites for its binarization): */
/* the spins are constant while the bisector angle beta stays between two      */
/* consecutive values of x_i mod 180, so every distinct value b of x_i mod 180 */
/* is tried as beta (+1 on [b, b + 180)), by brute force; the lowest H wins,   */
/* the smallest b on ties.  h must be NULL (with fields the semicircle is      */
/* fixed).  beta_out[R] (may be NULL) receives the chosen angle, degrees.      */
/* ------------------------------------------------------------------------ */
int32_t orc_readout_optimal(const orc_problem *pb, int32_t R, const double *x, int8_t *spins,
                            int64_t *H, int64_t *cut, double *beta_out) {
  if (pb->h != NULL) return -1;
  const int32_t n = pb->n;
  int8_t *cand = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
  int8_t *best = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
  for (int32_t r = 0; r < R; r++) {
    const double *xr = x + (size_t)r * n;
    int64_t bestH = 0, bestCut = 0;
    double bestB = 0.0;
    int found = 0;
    for (int32_t a = 0; a < n; a++) {
      const double b = mod_pos(xr[a], 180.0);
      for (int32_t i = 0; i < n; i++) cand[i] = mod_pos(xr[i] - b, 360.0) < 180.0 ? 1 : -1;
      int64_t e, c;
      energy_one(pb, cand, &e, &c);
      if (!found || e < bestH || (e == bestH && b < bestB)) {
        found = 1;
        bestH = e;
        bestCut = c;
        bestB = b;
        memcpy(best, cand, (size_t)n);
      }
    }
    if (!found) { /* n = 0 cannot happen (n >= 1) */
      bestH = 0;
      bestCut = 0;
    }
    H[r] = bestH;
    cut[r] = bestCut;
    if (beta_out) beta_out[r] = bestB;
    if (spins) memcpy(spins + (size_t)r * n, best, (size_t)n);
  }
  free(cand);
  free(best);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive ground state (pins only).                                       */
/* ------------------------------------------------------------------------ */
int32_t orc_brute_force_ground_state(const orc_problem *pb, int8_t *best_spins, int64_t *H) {
  const int32_t n = pb->n;
  if (n <= 0 || n > 26) return -1;
  int8_t *s = (int8_t *)malloc((size_t)n);
  int64_t best = 0;
  int have = 0;
  for (uint64_t code = 0; code < ((uint64_t)1 << n); code++) {
    for (int32_t i = 0; i < n; i++) s[i] = ((code >> i) & 1u) ? -1 : 1;
    int64_t e, c;
    energy_one(pb, s, &e, &c);
    if (!have || e < best) {
      best = e;
      have = 1;
      if (best_spins) memcpy(best_spins, s, (size_t)n);
    }
  }
  free(s);
  *H = best;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Appendix A, Eq. (15).                                                      */
/* ------------------------------------------------------------------------ */
double orc_r99(double ps) {
  if (ps >= 1.0) return 1.0;
  if (ps <= 0.0) return INFINITY;
  return log(1.0 - 0.99) / log(1.0 - ps);
}
