/*
 * rewl.h -- C ABI of the MI355X replica-exchange Wang-Landau library (librewl.so).
 *
 * Method: T. Vogel, Y. W. Li, T. Wuest, D. P. Landau, "Scalable replica-exchange
 * framework for Wang-Landau sampling", arXiv:1407.5140.  Section references below
 * are to that paper.
 *
 * Conventions
 *  - Every call returns a rewl_status; no exception crosses the ABI.  On failure
 *    rewl_last_error() returns a thread-local description.
 *  - The library owns all device memory it allocates.  Host pointers are owned by
 *    the caller and only read or written during the call.
 *  - All device work is ordered on the HIP stream given at creation (NULL = the
 *    default stream).  Calls that return host data synchronise that stream.
 *  - A handle holds a batch of one or more independent REWL instances that
 *    advance together, one exchange interval per step.  Instance indices are
 *    0-based positions in the configuration array given at creation.
 *  - Energy bins: Ising E = -sum s_i s_j, bin (E + 2N)/4 in [0, N];
 *    Potts E = -sum delta(q_i, q_j) (Eq. (2)), bin E + 2N in [0, 2N].
 *  - A handle must not be used from two threads at once.
 */
#ifndef REWL_H
#define REWL_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    REWL_OK = 0,
    REWL_E_INVALID = -1,      /* bad argument or configuration                     */
    REWL_E_EMPTY_WINDOW = -2, /* a window holds no energy level that occurs         */
    REWL_E_NOMEM = -3,        /* device or host allocation failed                  */
    REWL_E_DEVICE = -4,       /* a HIP call failed                                  */
    REWL_E_OVERFLOW = -5,     /* the exact-FP64 budget would overflow, or a walker's
                                 counts since its last merge (64-bit, no ceiling of
                                 their own) spread too far for one interval: every
                                 count of an occurring level of its window must lie
                                 within 2^31 below and 2^31 - X above the count of
                                 the level it sits at (H >= 2^31 of a level means
                                 ~10^12 attempts of one walker without a merge); the
                                 handle's state is then undefined                   */
    REWL_E_INIT_STUCK = -6,   /* a walker could not be driven into its window       */
    REWL_E_STATE = -7         /* call not valid in the handle's current state       */
} rewl_status;

/* The problem statement of Sec. II.A and IV (model, lattice, windows h with
 * overlap o, m walkers per window, flatness, ln f schedule, exchange interval). */
typedef struct {
    int32_t model;              /* 0 = 2D Ising (J = 1), 1 = q-state Potts, Eq. (2)      */
    int32_t q;                  /* Potts states, 3..255 (ignored for Ising)             */
    int32_t L;                  /* periodic L x L; Ising: even, 4..128; Potts: 4..255    */
    int32_t n_windows;          /* h >= 1                                               */
    int32_t overlap_num;        /* overlap o = num/den with the next lower window, 0<=o<1 */
    int32_t overlap_den;
    int32_t walkers_per_window; /* m: a power of two, 1..1024                            */
    int32_t flat_num;           /* flatness parameter num/den, see flat_rule             */
    int32_t flat_den;
    int32_t lnf_k0;             /* initial ln f = 2^-k0 (Sec. II.A uses ln f = 1: k0=0)  */
    int32_t lnf_kfinal;         /* window converged once k >= kfinal (ln f <= 2^-kfinal) */
    int32_t exchange_enabled;   /* 1: replica exchange (Eq. (1)); 0: independent windows */
    int64_t exchange_interval;  /* flip attempts per walker between exchange steps       */
    uint64_t seed;              /* Philox4x32-10 key                                     */
    int32_t flat_rule;          /* REWL_FLAT_MEAN or REWL_FLAT_VISITS (below)            */
    int32_t reserved;           /* must be 0                                             */
    const int32_t* window_lo;   /* optional explicit windows, host arrays of n_windows   */
    const int32_t* window_hi;   /* inclusive global bins (NULL, NULL: the equal-width
                                   partition of rewl_layout).  Unequal widths let windows
                                   that converge slowly be narrower (Sec. V).  Rules:
                                   lo[0] = 0, hi[h-1] = W-1, hi[a] - lo[a] >= 1, both
                                   ascending strictly, lo[a+1] <= hi[a] (overlap); read
                                   only during the call that takes the config.          */
} rewl_config;

/* Flatness rules, tested per walker over the levels of its window that occur;
 * a window merges once all m walkers have passed (latched):
 *  REWL_FLAT_MEAN   min H >= (flat_num/flat_den) * mean H, 0 <= num <= den (Sec. II.A,
 *                   80 %: 4/5);
 *  REWL_FLAT_VISITS H(E) >= a / sqrt(ln f) for every E, a = flat_num/flat_den
 *                   (Eq. (8), the Zhou-Bhatt criterion applied to all m walkers);
 *                   with ln f = 2^-k it is decided exactly as H^2 den^2 >= num^2 2^k;
 *                   0 <= num, 1 <= den, both <= 2^20.                                */
enum { REWL_FLAT_MEAN = 0, REWL_FLAT_VISITS = 1 };

/* Sweep variants.  LANE: one walker per lane, draws precomputed for the whole
 * interval by a separate kernel (suits batches of many thousands of walkers).
 * WAVE: one walker per wave, the chain on wave-uniform values, the lanes draw
 * the next 64 attempts (suits few walkers; falls back to LANE where one walker's
 * wave tables do not fit the LDS).  AUTO: WAVE for a batch of at most 8192
 * walkers in all, LANE above that.  Both give bit-identical results.            */
enum { REWL_SWEEP_AUTO = 0, REWL_SWEEP_LANE = 1, REWL_SWEEP_WAVE = 2 };

/* Where the WAVE sweep keeps a walker's counts while it runs.  LDS: a 32-bit copy
 * beside the walker's site map and lattice.  DEVICE: the 64-bit counts in device
 * memory, read when the walker's 64-bin register window of ln g is loaded and
 * written when it moves (a few times per thousand attempts), so LDS holds only the
 * window's base table, the site maps and the lattices, and more walkers fit a
 * block on large lattices.  AUTO: chosen with the site-map size (rewl_tune
 * map_log2) and the walkers per block so that as many of the instance's walkers
 * as possible are resident on the GPU at once; on a tie the larger site map, then
 * LDS.  Both give bit-identical results; the LANE sweep always uses LDS.         */
enum { REWL_TABLE_AUTO = 0, REWL_TABLE_LDS = 1, REWL_TABLE_DEVICE = 2 };

/* Optional tuning of a batch (NULL = library choice). */
typedef struct {
    int32_t walkers_per_block;  /* LANE: walkers per LDS tile (power of two <= 64);
                                   WAVE: walkers (waves) per block (<= 8); 0 = auto   */
    int32_t use_graph;          /* 1: replay the interval as a captured HIP graph        */
    int32_t poll_every;         /* intervals between host checks of the done flags      */
    int32_t sweep_kind;         /* REWL_SWEEP_*, applied to every instance that allows it */
    int32_t lds_target_kb;      /* LANE: cap on a tile's LDS (sets walkers per block and
                                   so blocks per CU); 0 = the device limit               */
    int32_t autotune;           /* 1: time candidate variants, LDS targets, the
                                   persistent lane sweep, table placements and site-map
                                   sizes on the real batch for two intervals at
                                   creation, keep the fastest                          */
    int32_t guard_band_log2;    /* guard band of the fast acceptance test, 2^v:
                                   0 = 2^-40 (the default); -40..-2 widen it.  Every
                                   decision stays exact either way; a wider band only
                                   sends more of them to the exact slow path (used by
                                   the tests to exercise that path).                  */
    int32_t table_placement;    /* REWL_TABLE_* (WAVE sweep)                             */
    int32_t persistent;         /* LANE sweep: 1 = a grid of as many blocks as the GPU
                                   holds at once, each taking tiles (longest first) from
                                   a device-side queue until none is left; 0 = one
                                   block per tile, handed out by the hardware          */
    int32_t map_log2;           /* WAVE sweep: at most 2^map_log2 site-map entries per
                                   walker (6..12); 0 = auto.  The map marks which
                                   attempts of a 64-attempt chunk lie in one another's
                                   neighbourhoods; a lattice with more sites than
                                   entries shares an entry between the sites equal
                                   modulo the entry count, which only marks extra
                                   attempts for re-evaluation (results stay
                                   bit-identical) but frees LDS for more resident
                                   walkers.  Auto takes the largest map among 2^12 ..
                                   2^9 entries that keeps the most walkers resident,
                                   with the placement above.                            */
} rewl_tune;

typedef struct rewl_handle rewl_handle;

/* Pure host: global bin count W, bins per window WB (the widest window: every
 * per-window table has WB entries, index = global bin - lo), and the window
 * bounds lo[h], hi[h] (inclusive global bins): the explicit windows of the
 * config if it has them, else Sec. II.A's partition: equal widths, overlap >= o
 * up to one bin, first window starts at bin 0, last ends at W-1.  lo/hi may be
 * NULL.  Returns REWL_E_INVALID for a bad configuration.                          */
rewl_status rewl_layout(const rewl_config* cfg, int32_t* n_bins, int32_t* window_bins,
                        int32_t* lo, int32_t* hi);

/* Pure host: windows of unequal width with equal total difficulty (Sec. V:
 * windows that converge at a similar pace).  rho[W] > 0 is a per-bin
 * difficulty density (for instance from a pilot run: sqrt(time per ln f halving)
 * of a window spread over its bins); with C the cumulative sum of rho, window a
 * covers C in [a s, a s + l], l = C_total / (1 + (h-1)(1-o)), s = l (1-o), o the
 * config's overlap, then each window is widened as needed to at least 2 bins and
 * an overlap of at least 8 bins (enough for the Sec. II.B joins).  lo[h], hi[h]
 * receive inclusive global bins valid as the config's explicit windows.          */
rewl_status rewl_balanced_layout(const rewl_config* cfg, const double* rho, int32_t* lo, int32_t* hi);

/* Pure host: the WAVE sweep's plan for an instance of cfg alone, as the library
 * makes it at creation from the device's LDS bytes per block, CU count and the
 * waves of the sweep kernel a CU holds (hipDeviceGetAttribute / the occupancy
 * API): walkers per block, count placement (REWL_TABLE_LDS / _DEVICE), site-map
 * entries per walker and LDS bytes per block.  The plan keeps the most walkers
 * resident at once (fewest rounds of blocks over the CUs); on a tie the larger
 * map, then LDS; counts asked for in LDS that do not fit go to device memory.
 * tune may be NULL (library choices); its walkers_per_block, table_placement and
 * map_log2 apply.  Returns REWL_E_INVALID for a bad argument or when one
 * walker's tables do not fit.  Output pointers may be NULL.                       */
rewl_status rewl_wave_plan(const rewl_config* cfg, const rewl_tune* tune, int32_t lds_per_block, int32_t n_cu,
                           int32_t waves_per_cu, int32_t* walkers_per_block, int32_t* placement,
                           int32_t* map_entries, size_t* lds_bytes);

/* Pure host: a difficulty density for rewl_balanced_layout from a model of the
 * single-spin-flip walk near the ground levels, where a walker spends most
 * attempts on rejected moves (the slow end windows that Sec. V proposes to
 * narrow).  Near a ground level a configuration holds a dilute set of flipped
 * spins, so only about one attempt in kappa is an accepted move:
 *   Ising: kappa = 1 + N / (d + 2), d = bins to the nearer end (both the ferro-
 *          and the antiferromagnetic ground level; a flip costs two bins);
 *   Potts: kappa = 1 + 18 N / (b + 4), b = bins above the ground level (a flip
 *          back to the surrounding state is 1 of N sites times 1 of q - 1 states);
 * with d and b capped at N/5, where the dilute picture ends.  A window's cost is
 * modelled as width^2 kappa, so rho[b] = sqrt(kappa) (W entries) makes windows of
 * equal rho-mass equally costly.                                                 */
rewl_status rewl_tilt_density(const rewl_config* cfg, double* rho);

/* Pure host: mask[W] = 1 where the energy level occurs on the periodic lattice. */
rewl_status rewl_mask(const rewl_config* cfg, uint8_t* mask);

/* Create a batch of n >= 1 instances on `hip_stream` (a hipStream_t or NULL).
 * Validates every configuration before allocating; allocates device state,
 * and drives every walker into its window (start configurations are ground
 * states).  *out receives the handle.                                          */
rewl_status rewl_batch_create(const rewl_config* cfgs, int32_t n, void* hip_stream,
                              const rewl_tune* tune, rewl_handle** out);
/* Single-instance form of rewl_batch_create. */
rewl_status rewl_create(const rewl_config* cfg, void* hip_stream, rewl_handle** out);

/* Warm start: replace every window's ln g by lng[W] (host array, global bins)
 * before the first interval.  Values must be finite multiples of 2^-20 with
 * |value| < 2^30 (keeps every later FP64 step exact).  REWL_E_STATE after run. */
rewl_status rewl_set_initial_lng(rewl_handle* h, int32_t instance, const double* lng);

/* Advance every unfinished instance by up to max_intervals exchange intervals
 * (Sec. II.A: X attempts per walker, flatness/merge, exchange).  Stops early
 * once every instance has converged.  *all_done (may be NULL) = 1 when every
 * window of every instance has reached lnf_kfinal.  Resumable.                */
rewl_status rewl_run(rewl_handle* h, int64_t max_intervals, int32_t* all_done);

/* Run exactly n intervals with no host polling in between (timing helper). */
rewl_status rewl_run_exact(rewl_handle* h, int64_t n);

/* ln g of one window over its WB bins (index = global bin - lo): the table the
 * window's walkers share since its last merge (Sec. II.A "merge and average");
 * for a converged window this is its result, before the first merge it is the
 * starting table (zero or the warm start).                                      */
rewl_status rewl_get_window_lng(rewl_handle* h, int32_t instance, int32_t window, double* out);

/* Sec. II.B concatenation of the h pieces into ln g over all W bins (-inf where
 * a level does not occur), normalised to sum_E g(E) = q^N (Ising: 2^N).  join
 * (h-1 entries, may be NULL) receives the join bins.  Runs on the device.      */
rewl_status rewl_concat(rewl_handle* h, int32_t instance, double* out_lng, int32_t* join);

/* rewl_concat for callers that cannot allocate device memory (code that must not
 * call hipMalloc: graph-capturing or tight serving loops, harnesses that forbid
 * it).  Same inputs, outputs and result as rewl_concat; its device staging lives
 * in a fixed 256 KiB array of device memory that each GPU holds from library
 * load until the process ends, so the call makes no allocation.  Limit: 8 W +
 * 12 h bytes (plus alignment) must fit 256 KiB, e.g. W <= 32 000 bins for a
 * few hundred windows (every Ising lattice up to L = 128, Potts up to L = 126);
 * larger instances get REWL_E_INVALID before any device work.  The array is
 * shared by every call on one GPU: calls from threads of one process are
 * serialised by the library; calls that overlapped on one GPU would race.  The
 * handle's device must be the current device (REWL_E_INVALID otherwise).       */
rewl_status rewl_concat_noalloc(rewl_handle* h, int32_t instance, double* out_lng, int32_t* join);

/* Error analysis over n independent runs (Sec. II.B).  runs[0..n) are instances
 * of the handle with equal model, q, L and windows (normally differing only in
 * seed); each supplies one piece per window, its rewl_get_window_lng table.
 *   Row 0 of out_lng: the mean global ln g.  For every window, the bin-wise
 *   mean of the n runs' pieces (summed in run order, then divided by n), then
 *   the concatenation of rewl_concat.
 *   Rows 1..R: bootstrap resamples.  For every window, n pieces drawn with
 *   repetition, then the same mean and concatenation.  Draw j of window a in
 *   resample r takes run runs[floor(x0 * n / 2^32)], x0 the first word of
 *   Philox4x32-10 at counter (r, j, a, 4) under key (seed low word, seed high).
 * The mean is taken over ln g; each run's additive constant only shifts a mean
 * piece, which the joining removes.  out_lng: (R+1) x W host doubles, row-major;
 * join (may be NULL): (R+1) x (h-1) host ints.  1 <= n <= 4096, 0 <= R <= 65534,
 * device tables up to 16 GiB per call (about (R+1)(h WB + W) doubles).
 * REWL_E_STATE if some overlap of some row has no valid join point (every row
 * is still written).  Runs on the device; returns with the stream synchronised. */
rewl_status rewl_ensemble(rewl_handle* h, const int32_t* runs, int32_t n, int32_t R, uint64_t seed,
                          double* out_lng, int32_t* join);

/* Canonical averages from densities of states (k_B = J = 1), as used for the
 * specific heat of the Potts study (Sec. IV.A).  For every row s < S of lng
 * (S x W host doubles over the bins of `model` on the L x L lattice, the
 * convention above; -inf marks a level that does not occur) and every
 * temperature T[t] > 0, with Z = sum_E g(E) e^{-E/T}:
 *   u = <E> / N,  c = <(E - <E>)^2> / (N T^2),  f = -T ln Z / N.
 * u, c, f: S x nT host doubles, row-major, each may be NULL.  Terms below
 * e^-745 of the largest are zero (double precision).  REWL_E_INVALID for NaN or
 * +inf in lng, a row without an occurring level, T <= 0, S outside 1..65535.
 * Runs on the device (library-owned buffers, the null stream).                */
rewl_status rewl_thermo(int32_t model, int32_t L, const double* lng, int32_t S, const double* T,
                        int32_t nT, double* u, double* c, double* f);

/* Full state of one instance for inspection (S = h*m slots, slot = a*m + r):
 *   spins[S*N] (Ising 1 = up; Potts 0..q-1), bins[S], H[S*WB] (each walker's
 *   counts since its window's last merge: 64-bit, no ceiling below 2^53),
 *   lng[S*WB] (each walker's ln g), flat[S], k[h], done[h], swaps[S] (1
 *   exchanged in the last interval, 0 proposed and rejected, -1 not proposed),
 *   *t = completed intervals.  Any pointer may be NULL.                         */
rewl_status rewl_get_state(rewl_handle* h, int32_t instance, uint8_t* spins, int32_t* bins,
                           int64_t* H, double* lng, uint8_t* flat, int32_t* k, uint8_t* done,
                           int8_t* swaps, int64_t* t);

typedef struct {
    int64_t intervals;          /* completed intervals                                 */
    int64_t attempts;           /* flip attempts made (all walkers)                    */
    int32_t windows_done;
    int32_t min_k;              /* smallest ln f exponent over windows                 */
    double sweep_ms;            /* summed device time of the sweep launches (events)   */
    double interval_ms;         /* summed device time of whole intervals (events)      */
    int64_t round_trips;        /* completed replica round trips, all replicas          */
    int64_t slow_decisions;     /* acceptance decisions (moves and exchanges) that fell
                                   inside the guard band and were taken exactly by the
                                   slow path                                            */
} rewl_stats;

/* Counters of one instance.  Each may be NULL:
 *   ex_prop, ex_acc (h entries): proposed and accepted exchanges per window pair
 *     (a, a+1) (Eq. (1));
 *   k (h entries): each window's current ln f exponent, ln f = 2^-k;
 *   round_trips (S = h*m entries, by replica): completed round trips of each
 *     replica over the energy range, the diagnostic of Sec. IV.A
 *     (fig:wanderlogs).  A replica is a configuration, identified by the slot it
 *     started in (replica r starts in slot r = a*m + w); it moves one window per
 *     accepted exchange.  A round trip is a visit to window 0, then to window
 *     h-1, then to window 0 again (a replica starting in window 0 has made the
 *     first visit); none are counted for h = 1.                                  */
rewl_status rewl_get_stats(rewl_handle* h, int32_t instance, rewl_stats* out, int64_t* ex_prop,
                           int64_t* ex_acc, int32_t* k, int32_t* round_trips);

/* Enable (1) or disable (0) per-launch event timing of the sweep kernel. */
rewl_status rewl_set_timing(rewl_handle* h, int32_t on);

/* Checkpoint: *len receives the byte size; with buf != NULL the state of all
 * instances is written to buf (len bytes).  Restore requires a handle created
 * from the same configurations.  Philox is counter-based, so a restored run
 * continues bit for bit.                                                        */
rewl_status rewl_checkpoint(rewl_handle* h, void* buf, size_t* len);
rewl_status rewl_restore(rewl_handle* h, const void* buf, size_t len);

void rewl_destroy(rewl_handle* h);
const char* rewl_last_error(void);

/* The tuning in effect (after autotuning, the winner). */
rewl_status rewl_get_tune(rewl_handle* h, rewl_tune* out);

/* Number of instances, and for one instance the sweep variant chosen
 * (REWL_SWEEP_LANE / _WAVE), walkers per block, LDS bytes per block, the count
 * table's placement (REWL_TABLE_LDS / _DEVICE) and the WAVE sweep's site-map
 * entries per walker (0 for LANE).  Any pointer may be NULL.                     */
rewl_status rewl_info(rewl_handle* h, int32_t instance, int32_t* n_instances, int32_t* sweep_kind,
                      int32_t* walkers_per_block, size_t* lds_bytes, int32_t* table_placement,
                      int32_t* map_entries);

/* Diagnostics (run on the device, used by the tests):
 * the full acceptance predicate u53 < 2^53 exp(delta) for n pairs: out[i] =
 * 1/0 decided by the fast test, 3/2 accepted/rejected by the exact slow path;
 * Philox4x32-10 blocks: in[6 n] = (ctr0..3, key0, key1), out[4 n].               */
rewl_status rewl_probe_accept(const double* delta, const uint64_t* u53, int32_t n, int32_t* out);
rewl_status rewl_probe_philox(const uint32_t* in, int32_t n, uint32_t* out);

#ifdef __cplusplus
}
#endif
#endif
