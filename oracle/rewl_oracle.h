/*
 * rewl_oracle.h -- plain CPU reference for replica-exchange Wang-Landau (REWL).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product path never does.  It shares no code, header or table
 * with the GPU library.
 *
 * Method: Vogel, Li, Wuest, Landau, "Scalable replica-exchange framework for
 * Wang-Landau sampling" (arXiv:1407.5140), Sec. II.A (WL walker, windows,
 * Eq. (1) exchange, multiple walkers per window, merge, termination) and
 * Sec. II.B (concatenation).  The readings taken where the paper is silent are
 * stated next to each step in rewl_oracle.c.
 */
#ifndef REWL_ORACLE_H
#define REWL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem statement (same field meaning as the product's configuration). */
typedef struct {
    int32_t model;              /* 0 = Ising (s = +-1, J = 1), 1 = q-state Potts      */
    int32_t q;                  /* Potts states (>= 3); ignored for Ising             */
    int32_t L;                  /* periodic L x L lattice                             */
    int32_t n_windows;          /* h                                                  */
    int32_t overlap_num;        /* o = overlap_num / overlap_den                      */
    int32_t overlap_den;
    int32_t walkers_per_window; /* m, a power of two                                  */
    int32_t flat_num;           /* flatness parameter, see flat_rule                  */
    int32_t flat_den;
    int32_t lnf_k0;             /* initial ln f = 2^-k0                               */
    int32_t lnf_kfinal;         /* window converged once k >= kfinal                  */
    int32_t exchange_enabled;   /* 1 = replica exchange on                            */
    int64_t exchange_interval;  /* flip attempts per walker between exchanges         */
    uint64_t seed;              /* Philox key                                         */
    int32_t flat_rule;          /* 0: min H >= num/den mean H (Sec. II.A);
                                   1: H(E) >= (num/den)/sqrt(ln f) for all E, Eq. (8)   */
    int32_t reserved;
    const int32_t* window_lo;   /* optional explicit windows (inclusive global bins,     */
    const int32_t* window_hi;   /* n_windows each); NULL: the equal-width partition      */
} orc_config;

typedef struct orc_sim orc_sim;

/* --- building blocks, exposed so that tests can pin each one ------------- */
void     orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int      orc_accept(double delta, uint64_t u53);          /* exact u53 < 2^53 e^delta  */
int32_t  orc_n_bins(const orc_config* c);                 /* W                          */
int      orc_layout(const orc_config* c, int32_t* lo, int32_t* hi);  /* 0 on success   */
void     orc_mask_rule(const orc_config* c, uint8_t* mask);          /* W entries       */
int64_t  orc_energy(const orc_config* c, const uint8_t* spins);      /* E of a lattice  */

/* --- simulation ----------------------------------------------------------- */
/* mask: W entries (1 = energy level occurs) or NULL for the closed-form rule.
 * init_lng: W entries of a starting ln g (warm start) or NULL for ln g = 0.
 * Returns NULL and sets *status < 0 on invalid input.                          */
orc_sim* orc_create(const orc_config* c, const uint8_t* mask, const double* init_lng,
                    int* status);
void     orc_destroy(orc_sim* s);
/* Run up to n_intervals exchange intervals; stops early once every window has
 * converged.  Returns 1 if all windows are done, 0 otherwise, < 0 on error.     */
int      orc_run(orc_sim* s, int64_t n_intervals, int n_threads);

int64_t  orc_interval(const orc_sim* s);                  /* completed intervals t     */
int32_t  orc_window_bins(const orc_sim* s);               /* bins per window (w+1)     */
/* State, slot-major (slot = a*m + r):
 *   spins  [S*N]   Ising 1 = up, 0 = down; Potts 0..q-1
 *   bins   [S]     global energy bin of the slot's configuration
 *   H      [S*WB]  histogram over the window's bins (WB = w+1)
 *   lng    [S*WB]  the walker's ln g over its window
 *   flat   [S]     latched flatness flag
 *   k      [h], done [h]
 *   swaps  [S]     1 if the slot's configuration was exchanged in the last
 *                  interval, 0 if an exchange was attempted and rejected,
 *                  -1 if no exchange involved the slot                          */
void     orc_get_state(const orc_sim* s, uint8_t* spins, int32_t* bins, int64_t* H,
                       double* lng, uint8_t* flat, int32_t* k, uint8_t* done,
                       int8_t* swaps);
/* Merged ln g of one window (valid once the window has merged at least once;
 * before that it is walker 0's estimate).                                      */
void     orc_window_lng(const orc_sim* s, int32_t window, double* out);
/* Replace the ln g table of every walker of one window (WB entries). */
void     orc_set_window_lng(orc_sim* s, int32_t window, const double* tab);
/* Counters: attempts made, exchange proposals and acceptances per window pair. */
void     orc_stats(const orc_sim* s, int64_t* attempts, int64_t* ex_prop, int64_t* ex_acc);
int      orc_init_attempts_max(const orc_sim* s);         /* longest init drive        */
/* Replicas (Sec. IV.A, fig:wanderlogs): rid[S] = replica held by each slot
 * (replica r starts in slot r; it follows its configuration through accepted
 * exchanges); round_trips[S] by replica = completed visits window 0 -> window
 * h-1 -> window 0 (starting in window 0 counts as the first visit).  NULL ok.   */
void     orc_replicas(const orc_sim* s, int32_t* rid, int32_t* round_trips);
/* Replace every walker's counts H[S*WB] and ln g lng[S*WB] (either may be NULL),
 * e.g. to start from counts past 2^32.                                          */
void     orc_set_tables(orc_sim* s, const int64_t* H, const double* lng);
/* Test hook: plant a mistake in the exchange rule (0 = none, 1 = always accept,
 * 2 = sign of the log ratio flipped, 3 = walker j's factor dropped).            */
void     orc_test_exchange_mutation(int mode);

/* --- post-processing (Sec. II.B) ----------------------------------------- */
/* pieces: h*WB, piece a covers global bins lo[a]..hi[a].  Output: W entries of
 * ln g normalised to sum_E g(E) = q^N (Ising q = 2), -inf where mask is 0.
 * join[a] receives the join bin between pieces a and a+1.  Returns 0 or < 0.  */
int      orc_concat(const orc_config* c, const uint8_t* mask, const double* pieces,
                    double* out, int32_t* join);

/* --- n independent runs (Sec. II.B error analysis) ----------------------- */
/* Which run's piece each draw of a resample takes: picks[(r*h + a)*n + j] for
 * r = 0..R, window a < h, draw j < n.  Resample 0 is the ensemble itself (draw j
 * takes run j); resample r >= 1 draws with repetition: run floor(x0 * n / 2^32)
 * with x0 the first word of Philox4x32-10 at counter (r, j, a, 4) under key
 * (seed low word, seed high word).  Returns 0, or -1 for n < 1, h < 1, R < 0.  */
int      orc_boot_picks(uint64_t seed, int32_t R, int32_t h, int32_t n, int32_t* picks);

#ifdef __cplusplus
}
#endif
#endif
