/*
 * rewl_oracle.c -- plain, slow CPU reference for replica-exchange Wang-Landau.
 *
 * TEST INFRASTRUCTURE ONLY (see rewl_oracle.h).  Written for readability:
 * every walker keeps its own ln g(E) and H(E) literally, every step follows
 * the order in which the paper describes it, nothing is blocked or fused.
 *
 * Paper: arXiv:1407.5140, Sec. II.A and II.B; Potts Hamiltonian Eq. (2).
 * Readings where the paper is silent (numbered as in the design notes):
 *   R1  energy levels that never occur are excluded from flatness tests;
 *   R2  window widths: ceil width, floor starts, last window ends at the top;
 *   R3  start configurations: ground state, then a distance-non-increasing
 *       drive into the window;
 *   R4  random numbers: Philox4x32-10, counter = (t*X + j, slot, stream tag);
 *   R5  a move leaving the window is rejected and the current bin updated;
 *   R6  the acceptance test is the exact real comparison u53 < 2^53 e^delta;
 *   R7  interval order: sweep, flatness/merge, stop test, exchange;
 *   R8  flatness is tested once per exchange interval;
 *   R9  a walker that passed the test stays flat (latched) and keeps
 *       updating at the same ln f until its whole window merges;
 *   R10 the merge is the arithmetic mean of ln g (exact for m = 2^j);
 *       afterwards the window's table is shifted by the integer part of its
 *       minimum over occurring levels (a per-window constant, exact);
 *   R11 converged windows keep walking with frozen ln g and keep exchanging;
 *   R12 pairing between neighbour windows: r <-> (r + c) mod m, c random;
 *   R13 no WL update on exchange;
 *   R14 concatenation stencil step clamp(overlap/8, 1, 10), ties to low E,
 *       each join searched above the previous one so that pieces stay in order;
 *   R29 replica round trips (Sec. IV.A, fig:wanderlogs): a replica is a
 *       configuration; it moves one window per accepted exchange; a round trip
 *       is a visit to window 0, then to window h-1, then to window 0 again.
 */
#include "rewl_oracle.h"

#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11.  Ten rounds of the 4x32 S-box with two 32x32   */
/* multiplications per round and a Weyl key schedule.                       */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random words for (64-bit counter T, slot, stream tag). */
static void draw(const uint32_t key[2], uint64_t T, uint32_t slot, uint32_t tag, uint32_t x[4])
{
    uint32_t ctr[4] = {(uint32_t)T, (uint32_t)(T >> 32), slot, tag};
    orc_philox4x32_10(ctr, key, x);
}

enum { TAG_FLIP = 0, TAG_EXCHANGE = 1, TAG_INIT = 2, TAG_PARTNER = 3, TAG_BOOT = 4 };

/* ------------------------------------------------------------------------ */
/* Acceptance (Sec. II.A: states are sampled with weight 1/g(E)):           */
/* accept iff u53 < 2^53 * exp(delta), delta = ln g(E_old) - ln g(E_new),   */
/* decided as an exact real comparison (R6).  exp(delta) is irrational for */
/* rational delta != 0, so ties cannot occur.                               */
/* ------------------------------------------------------------------------ */
int orc_accept(double delta, uint64_t u53)
{
    if (delta >= 0.0) return 1;         /* exp(delta) >= 1 > u53 / 2^53        */
    if (u53 == 0) return 1;             /* 0 < exp(delta) always               */
    /* libm exp is within a few units in the last place: at scale 2^53 the    */
    /* estimate y is within +-2 of 2^53 e^delta, so a margin of 8 decides.     */
    double y = ldexp(exp(delta), 53);
    double u = (double)u53;             /* exact, u53 < 2^53                   */
    if (u < y - 8.0) return 1;
    if (u > y + 8.0) return 0;
    /* near tie: 113-bit arithmetic, error ~2^-59 at this scale               */
    __float128 yq = ldexpq(expq((__float128)delta), 53);
    return (__float128)u53 < yq;
}

/* ------------------------------------------------------------------------ */
/* Model: Ising E = -sum s_i s_j (J = 1); Potts E = -sum delta(q_i, q_j),   */
/* Eq. (2), both on the periodic L x L lattice with N = L^2 sites.          */
/* Energy bins: Ising (E + 2N)/4 in 0..N; Potts E + 2N in 0..2N.            */
/* ------------------------------------------------------------------------ */
int32_t orc_n_bins(const orc_config* c)
{
    int32_t N = c->L * c->L;
    return c->model == 0 ? N + 1 : 2 * N + 1;
}

static int64_t bin_of(const orc_config* c, int64_t E)
{
    int64_t N = (int64_t)c->L * c->L;
    return c->model == 0 ? (E + 2 * N) / 4 : E + 2 * N;
}

int64_t orc_energy(const orc_config* c, const uint8_t* spins)
{
    int L = c->L;
    int64_t E = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            int i = y * L + x;
            int r = y * L + (x + 1) % L;
            int d = ((y + 1) % L) * L + x;
            if (c->model == 0) {
                int si = spins[i] ? 1 : -1, sr = spins[r] ? 1 : -1, sd = spins[d] ? 1 : -1;
                E -= si * sr + si * sd;
            } else {
                E -= (spins[i] == spins[r]) + (spins[i] == spins[d]);
            }
        }
    return E;
}

/* R1: levels that never occur on the periodic lattice.  Ising (even L):   */
/* E = -2N+4 and 2N-4 (bins 1 and N-1).  Potts (q >= 3, L >= 4): one, two, */
/* three or five broken bonds (bins 1, 2, 3, 5).                            */
void orc_mask_rule(const orc_config* c, uint8_t* mask)
{
    int32_t W = orc_n_bins(c), N = c->L * c->L;
    for (int b = 0; b < W; ++b) mask[b] = 1;
    if (c->model == 0) {
        mask[1] = 0;
        mask[N - 1] = 0;
    } else {
        mask[1] = mask[2] = mask[3] = mask[5] = 0;
    }
}

/* R2: h windows of equal width w (in bin steps) over S = W-1 steps, each   */
/* sharing a fraction >= o with its lower neighbour (Sec. II.A; the Potts  */
/* example of Sec. IV.A has width 1000, shift 250 and 77..1277 windows).   */
int orc_layout(const orc_config* c, int32_t* lo, int32_t* hi)
{
    int64_t S = orc_n_bins(c) - 1;
    int64_t h = c->n_windows, num = c->overlap_num, den = c->overlap_den;
    if (c->window_lo || c->window_hi) {
        /* explicit windows (unequal widths, Sec. V): each at least 2 bins, both  */
        /* ends ascending, covering [0, S], each overlapping the next             */
        if (!c->window_lo || !c->window_hi || h < 1) return -1;
        for (int64_t a = 0; a < h; ++a) {
            lo[a] = c->window_lo[a];
            hi[a] = c->window_hi[a];
            if (lo[a] < 0 || hi[a] > S || hi[a] - lo[a] < 1) return -1;
            if (a > 0 && (lo[a] <= lo[a - 1] || hi[a] <= hi[a - 1] || lo[a] > hi[a - 1])) return -1;
        }
        return (lo[0] == 0 && hi[h - 1] == S) ? 0 : -1;
    }
    if (h < 1 || den < 1 || num < 0 || num >= den) return -1;
    if (h == 1) {
        lo[0] = 0;
        hi[0] = (int32_t)S;
        return 0;
    }
    int64_t D = den + (h - 1) * (den - num);
    int64_t w = (S * den + D - 1) / D;
    if (w > S) w = S;
    for (int64_t a = 0; a < h; ++a) {
        lo[a] = (int32_t)(a * (S - w) / (h - 1));
        hi[a] = (int32_t)(lo[a] + w);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Simulation state                                                         */
/* ------------------------------------------------------------------------ */
struct orc_sim {
    orc_config c;
    int N, W, h, m, S, WB, log2m;
    int32_t *lo, *hi, *nreach;
    uint8_t* mask;
    int16_t* spins;   /* S*N: Ising +-1, Potts 0..q-1 */
    int64_t* E;       /* S    */
    int64_t* H;       /* S*WB */
    double* lng;      /* S*WB */
    uint8_t* flat;    /* S    */
    int32_t* k;       /* h    */
    uint8_t* done;    /* h    */
    int8_t* swaps;    /* S    */
    int64_t t, attempts;
    int64_t *ex_prop, *ex_acc;
    int32_t* rid;     /* S: replica held by each slot                         */
    int8_t* rt_state; /* S, by replica: 0 window 0 not yet visited, 1 visited,  */
                      /*    2 window h-1 reached after the last visit to 0      */
    int32_t* rt_count;/* S, by replica: completed round trips                  */
    int all_done, init_max, error;
    uint32_t key[2];
};

/* Test hook: planted mistakes in the exchange rule, so that the tests can show */
/* that their checks of Eq. (1) fail on a wrong rule.  0 = Eq. (1) as written;  */
/* 1 = accept every proposal whose energies fit both windows; 2 = the sign of   */
/* the log ratio flipped; 3 = walker j's factor dropped.  Never set otherwise.  */
static int g_exchange_mutation = 0;
void orc_test_exchange_mutation(int mode) { g_exchange_mutation = mode; }

static int ilog2_exact(int v)
{
    int j = 0;
    while ((1 << j) < v) ++j;
    return (1 << j) == v ? j : -1;
}

/* Energy change of the proposed move at `site`; for Potts also the new value. */
static int64_t delta_energy(const orc_sim* s, const int16_t* sp, int site, const uint32_t x[4],
                            int* newval)
{
    int L = s->c.L, xx = site % L, yy = site / L;
    int nb[4] = {yy * L + (xx + 1) % L, yy * L + (xx + L - 1) % L,
                 ((yy + 1) % L) * L + xx, ((yy + L - 1) % L) * L + xx};
    if (s->c.model == 0) {
        int sum = sp[nb[0]] + sp[nb[1]] + sp[nb[2]] + sp[nb[3]];
        *newval = -sp[site];
        return 2 * (int64_t)sp[site] * sum;
    }
    int q = s->c.q, old = sp[site];
    int nv = (old + 1 + (int)(((uint64_t)x[1] * (uint64_t)(q - 1)) >> 32)) % q;
    int n_old = 0, n_new = 0;
    for (int d = 0; d < 4; ++d) {
        n_old += sp[nb[d]] == old;
        n_new += sp[nb[d]] == nv;
    }
    *newval = nv;
    return (int64_t)n_old - n_new;
}

static int64_t dist_to(int64_t b, int64_t lo, int64_t hi)
{
    if (b < lo) return lo - b;
    if (b > hi) return b - hi;
    return 0;
}

/* R3: start from a ground state (Ising: all up, or the checkerboard for a  */
/* window in the upper half of the range; Potts: all 0) and drive into the  */
/* window: a proposal is taken iff it does not increase the distance of the */
/* energy bin to the window.  Returns attempts used, or -1 when stuck.      */
static int64_t init_slot(orc_sim* s, int slot)
{
    int N = s->N, L = s->c.L, a = slot / s->m;
    int16_t* sp = s->spins + (size_t)slot * N;
    int upper = (int64_t)s->lo[a] + s->hi[a] > (int64_t)(s->W - 1);
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            if (s->c.model == 0)
                sp[y * L + x] = (upper && ((x + y) & 1)) ? -1 : 1;
            else
                sp[y * L + x] = 0;
        }
    uint8_t* tmp = malloc(N);
    for (int i = 0; i < N; ++i) tmp[i] = s->c.model == 0 ? (sp[i] > 0) : (uint8_t)sp[i];
    int64_t E = orc_energy(&s->c, tmp);
    free(tmp);
    int64_t b = bin_of(&s->c, E), lo = s->lo[a], hi = s->hi[a];
    int64_t j = 0, cap = 1000 * (int64_t)N;
    while (b < lo || b > hi) {
        if (j >= cap) return -1;
        uint32_t x[4];
        draw(s->key, (uint64_t)j, (uint32_t)slot, TAG_INIT, x);
        int site = (int)(((uint64_t)x[0] * (uint64_t)N) >> 32), nv;
        int64_t dE = delta_energy(s, sp, site, x, &nv);
        int64_t nb = bin_of(&s->c, E + dE);
        if (dist_to(nb, lo, hi) <= dist_to(b, lo, hi)) {
            sp[site] = (int16_t)nv;
            E += dE;
            b = nb;
        }
        ++j;
    }
    s->E[slot] = E;
    return j;
}

orc_sim* orc_create(const orc_config* c, const uint8_t* mask, const double* init_lng,
                    int* status)
{
    *status = -1;
    if (c->model != 0 && c->model != 1) return NULL;
    if (c->L < 3 || (c->model == 0 && (c->L % 2 || c->L < 4))) return NULL;
    if (c->model == 1 && c->q < 3) return NULL;
    if (c->L > 1024) return NULL;
    if (c->walkers_per_window < 1 || ilog2_exact(c->walkers_per_window) < 0) return NULL;
    if (c->flat_rule == 0 && (c->flat_den < 1 || c->flat_num < 0 || c->flat_num > c->flat_den)) return NULL;
    if (c->flat_rule == 1 && (c->flat_den < 1 || c->flat_den > (1 << 20) || c->flat_num < 0 ||
                              c->flat_num > (1 << 20))) return NULL;
    if (c->flat_rule != 0 && c->flat_rule != 1) return NULL;
    if (c->lnf_k0 < 0 || c->lnf_kfinal <= c->lnf_k0 || c->lnf_kfinal > 40) return NULL;
    if (c->exchange_interval < 1) return NULL;
    if (mask == NULL && c->model == 1 && c->L < 4) return NULL;

    orc_sim* s = calloc(1, sizeof(orc_sim));
    s->c = *c;
    s->N = c->L * c->L;
    s->W = orc_n_bins(c);
    s->h = c->n_windows;
    s->m = c->walkers_per_window;
    s->log2m = ilog2_exact(s->m);
    s->S = s->h * s->m;
    s->lo = calloc(s->h, sizeof(int32_t));
    s->hi = calloc(s->h, sizeof(int32_t));
    s->nreach = calloc(s->h, sizeof(int32_t));
    if (orc_layout(c, s->lo, s->hi) != 0) {
        orc_destroy(s);
        return NULL;
    }
    s->WB = 0;                          /* table length: the widest window */
    for (int a = 0; a < s->h; ++a)
        if (s->hi[a] - s->lo[a] + 1 > s->WB) s->WB = s->hi[a] - s->lo[a] + 1;
    s->mask = malloc(s->W);
    if (mask)
        memcpy(s->mask, mask, s->W);
    else
        orc_mask_rule(c, s->mask);
    for (int a = 0; a < s->h; ++a) {
        for (int b = s->lo[a]; b <= s->hi[a]; ++b) s->nreach[a] += s->mask[b];
        if (s->nreach[a] < 1) {
            *status = -2;
            orc_destroy(s);
            return NULL;
        }
    }
    s->key[0] = (uint32_t)c->seed;
    s->key[1] = (uint32_t)(c->seed >> 32);
    s->spins = calloc((size_t)s->S * s->N, sizeof(int16_t));
    s->E = calloc(s->S, sizeof(int64_t));
    s->H = calloc((size_t)s->S * s->WB, sizeof(int64_t));
    s->lng = calloc((size_t)s->S * s->WB, sizeof(double));
    s->flat = calloc(s->S, 1);
    s->k = calloc(s->h, sizeof(int32_t));
    s->done = calloc(s->h, 1);
    s->swaps = malloc(s->S);
    memset(s->swaps, -1, s->S);
    s->ex_prop = calloc(s->h, sizeof(int64_t));
    s->ex_acc = calloc(s->h, sizeof(int64_t));
    s->rid = malloc(s->S * sizeof(int32_t));
    s->rt_state = malloc(s->S);
    s->rt_count = calloc(s->S, sizeof(int32_t));
    for (int sl = 0; sl < s->S; ++sl) {
        s->rid[sl] = sl;                           /* replica r starts in slot r */
        s->rt_state[sl] = (sl / s->m == 0) ? 1 : 0;
    }
    for (int a = 0; a < s->h; ++a) s->k[a] = c->lnf_k0;
    for (int sl = 0; sl < s->S; ++sl) {
        int a = sl / s->m;
        for (int b = 0; b < s->WB; ++b)
            s->lng[(size_t)sl * s->WB + b] =
                (init_lng && s->lo[a] + b <= s->hi[a]) ? init_lng[s->lo[a] + b] : 0.0;
    }
    int stuck = 0, imax = 0;
    /* walkers are independent: each drives only its own lattice */
#pragma omp parallel for schedule(dynamic, 16) reduction(| : stuck) reduction(max : imax)
    for (int sl = 0; sl < s->S; ++sl) {
        int64_t used = init_slot(s, sl);
        if (used < 0) stuck = 1;
        else if (used > imax) imax = (int)used;
    }
    s->init_max = imax;
    if (stuck) {
        *status = -6;
        orc_destroy(s);
        return NULL;
    }
    *status = 0;
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->lo); free(s->hi); free(s->nreach); free(s->mask); free(s->spins);
    free(s->E); free(s->H); free(s->lng); free(s->flat); free(s->k); free(s->done);
    free(s->swaps); free(s->ex_prop); free(s->ex_acc);
    free(s->rid); free(s->rt_state); free(s->rt_count);
    free(s);
}

/* One walker's share of an interval: X single-site attempts, each followed */
/* by the WL update at the state the walker then resides in (Sec. II.A).    */
static void sweep_slot(orc_sim* s, int slot)
{
    int a = slot / s->m, N = s->N;
    int64_t X = s->c.exchange_interval, lo = s->lo[a], hi = s->hi[a];
    int16_t* sp = s->spins + (size_t)slot * N;
    int64_t* H = s->H + (size_t)slot * s->WB;
    double* lng = s->lng + (size_t)slot * s->WB;
    int update = !s->done[a];
    double lnf = ldexp(1.0, -s->k[a]);
    int64_t E = s->E[slot], b = bin_of(&s->c, E);
    for (int64_t j = 0; j < X; ++j) {
        uint32_t x[4];
        draw(s->key, (uint64_t)(s->t * X + j), (uint32_t)slot, TAG_FLIP, x);
        int site = (int)(((uint64_t)x[0] * (uint64_t)N) >> 32), nv;
        int64_t dE = delta_energy(s, sp, site, x, &nv);
        int64_t nb = bin_of(&s->c, E + dE);
        if (nb >= lo && nb <= hi) {             /* R5: leaving the window is rejected */
            double delta = lng[b - lo] - lng[nb - lo];
            uint64_t u53 = (((uint64_t)x[3] << 32) | x[2]) >> 11;
            if (orc_accept(delta, u53)) {
                sp[site] = (int16_t)nv;
                E += dE;
                b = nb;
            }
        }
        if (update) {
            H[b - lo] += 1;
            lng[b - lo] += lnf;
        }
    }
    s->E[slot] = E;
}

/* Flatness of one walker over the levels of its window that occur.         */
/* Rule 0 (Sec. II.A): no H(E) below flat_num/flat_den of the mean, in the   */
/* integer form den*min*n >= num*sum.  Rule 1 (Eq. (8)): every H(E) at least */
/* a/sqrt(ln f) with a = num/den and ln f = 2^-k, i.e. min^2 den^2 >=        */
/* num^2 2^k, evaluated in 128-bit integers.                                 */
static int is_flat(const orc_sim* s, int slot)
{
    int a = slot / s->m;
    const int64_t* H = s->H + (size_t)slot * s->WB;
    int64_t mn = -1, sum = 0, n = 0;
    for (int b = s->lo[a]; b <= s->hi[a]; ++b) {
        if (!s->mask[b]) continue;
        int64_t v = H[b - s->lo[a]];
        if (mn < 0 || v < mn) mn = v;
        sum += v;
        ++n;
    }
    typedef unsigned __int128 u128;
    if (s->c.flat_rule == 1) {
        /* min*den < 2^84 here; its square may not fit 128 bits, but num^2 2^k  */
        /* < 2^81, so min*den >= 2^41 decides the test by itself                */
        u128 x = (u128)mn * (u128)s->c.flat_den;
        u128 rhs = ((u128)s->c.flat_num * (u128)s->c.flat_num) << s->k[a];
        if (x >= ((u128)1 << 41)) return 1;
        return x * x >= rhs;
    }
    return (u128)s->c.flat_den * (u128)mn * (u128)n >= (u128)s->c.flat_num * (u128)sum;
}

/* Merge (Sec. II.A): the m walkers of a window average their estimators,  */
/* reset H and proceed together with ln f halved.                           */
static int merge_window(orc_sim* s, int a)
{
    int m = s->m, WB = s->WB;
    double* mean = malloc(WB * sizeof(double));
    for (int b = 0; b < WB; ++b) {
        __float128 acc = 0;
        for (int r = 0; r < m; ++r) acc += (__float128)s->lng[(size_t)(a * m + r) * WB + b];
        __float128 mq = acc / m;
        mean[b] = (double)mq;
        if ((__float128)mean[b] != mq) { free(mean); return -5; }   /* budget exceeded */
    }
    double mn = INFINITY;
    for (int b = 0; b <= s->hi[a] - s->lo[a]; ++b)
        if (s->mask[s->lo[a] + b] && mean[b] < mn) mn = mean[b];
    double shift = floor(mn);
    for (int b = 0; b < WB; ++b) {
        __float128 exact = (__float128)mean[b] - (__float128)shift;
        mean[b] = mean[b] - shift;
        if ((__float128)mean[b] != exact) { free(mean); return -5; }
    }
    for (int r = 0; r < m; ++r) {
        int sl = a * m + r;
        memcpy(s->lng + (size_t)sl * WB, mean, WB * sizeof(double));
        memset(s->H + (size_t)sl * WB, 0, WB * sizeof(int64_t));
        s->flat[sl] = 0;
    }
    free(mean);
    s->k[a] += 1;
    if (s->k[a] >= s->c.lnf_kfinal) s->done[a] = 1;
    return 0;
}

/* Replica exchange (Sec. II.A, Eq. (1)): neighbouring windows (a, a+1) with */
/* a = t mod 2 alternate, walker r of a pairs with walker (r+c) mod m of a+1. */
static void exchange(orc_sim* s)
{
    int m = s->m, h = s->h, N = s->N, WB = s->WB;
    memset(s->swaps, -1, s->S);
    if (!s->c.exchange_enabled) return;
    int16_t* tmp = malloc(N * sizeof(int16_t));
    for (int a = (int)(s->t & 1); a + 1 < h; a += 2) {
        uint32_t xc[4];
        draw(s->key, (uint64_t)s->t, (uint32_t)a, TAG_PARTNER, xc);
        int c = (int)(((uint64_t)xc[0] * (uint64_t)m) >> 32);
        for (int r = 0; r < m; ++r) {
            int i = a * m + r, j = (a + 1) * m + (r + c) % m;
            int64_t bi = bin_of(&s->c, s->E[i]), bj = bin_of(&s->c, s->E[j]);
            int ok = 0;
            s->ex_prop[a] += 1;
            if (bj >= s->lo[a] && bj <= s->hi[a] && bi >= s->lo[a + 1] && bi <= s->hi[a + 1]) {
                const double* gi = s->lng + (size_t)i * WB;
                const double* gj = s->lng + (size_t)j * WB;
                double delta = (gi[bi - s->lo[a]] - gi[bj - s->lo[a]]) +
                               (gj[bj - s->lo[a + 1]] - gj[bi - s->lo[a + 1]]);
                if (g_exchange_mutation == 2) delta = -delta;
                if (g_exchange_mutation == 3) delta = gi[bi - s->lo[a]] - gi[bj - s->lo[a]];
                uint32_t x[4];
                draw(s->key, (uint64_t)s->t, (uint32_t)i, TAG_EXCHANGE, x);
                uint64_t u53 = (((uint64_t)x[3] << 32) | x[2]) >> 11;
                ok = g_exchange_mutation == 1 ? 1 : orc_accept(delta, u53);
            }
            if (ok) {
                memcpy(tmp, s->spins + (size_t)i * N, N * sizeof(int16_t));
                memcpy(s->spins + (size_t)i * N, s->spins + (size_t)j * N, N * sizeof(int16_t));
                memcpy(s->spins + (size_t)j * N, tmp, N * sizeof(int16_t));
                int64_t e = s->E[i];
                s->E[i] = s->E[j];
                s->E[j] = e;
                s->ex_acc[a] += 1;
                /* R29: the replica from slot i went up to window a+1, the one  */
                /* from slot j came down to window a                            */
                int up = s->rid[i], down = s->rid[j];
                s->rid[i] = down;
                s->rid[j] = up;
                if (a + 1 == h - 1 && s->rt_state[up] == 1) s->rt_state[up] = 2;
                if (a == 0) {
                    if (s->rt_state[down] == 2) s->rt_count[down] += 1;
                    s->rt_state[down] = 1;
                }
            }
            s->swaps[i] = (int8_t)ok;
            s->swaps[j] = (int8_t)ok;
        }
    }
    free(tmp);
}

int orc_run(orc_sim* s, int64_t n_intervals, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int64_t it = 0; it < n_intervals && !s->all_done; ++it) {
        /* 1. every walker makes X attempts (independent between sync points) */
#pragma omp parallel for schedule(dynamic, 1)
        for (int sl = 0; sl < s->S; ++sl) sweep_slot(s, sl);
        s->attempts += (int64_t)s->S * s->c.exchange_interval;
        /* 2. flatness per walker, merge per window                           */
        for (int a = 0; a < s->h; ++a) {
            if (s->done[a]) continue;
            int all = 1;
            for (int r = 0; r < s->m; ++r) {
                int sl = a * s->m + r;
                if (!s->flat[sl] && is_flat(s, sl)) s->flat[sl] = 1;
                all &= s->flat[sl];
            }
            if (all) {
                int st = merge_window(s, a);
                if (st) { s->error = st; return st; }
            }
        }
        /* 3. stop once every window has converged                            */
        int done = 1;
        for (int a = 0; a < s->h; ++a) done &= s->done[a];
        if (done) {
            s->all_done = 1;
            memset(s->swaps, -1, s->S);
            s->t += 1;
            break;
        }
        /* 4. replica exchange between neighbouring windows                   */
        exchange(s);
        s->t += 1;
    }
    return s->all_done;
}

int64_t orc_interval(const orc_sim* s) { return s->t; }
int32_t orc_window_bins(const orc_sim* s) { return s->WB; }
int orc_init_attempts_max(const orc_sim* s) { return s->init_max; }

void orc_get_state(const orc_sim* s, uint8_t* spins, int32_t* bins, int64_t* H, double* lng,
                   uint8_t* flat, int32_t* k, uint8_t* done, int8_t* swaps)
{
    size_t SN = (size_t)s->S * s->N, SW = (size_t)s->S * s->WB;
    if (spins)
        for (size_t i = 0; i < SN; ++i)
            spins[i] = s->c.model == 0 ? (uint8_t)(s->spins[i] > 0) : (uint8_t)s->spins[i];
    if (bins)
        for (int i = 0; i < s->S; ++i) bins[i] = (int32_t)bin_of(&s->c, s->E[i]);
    if (H) memcpy(H, s->H, SW * sizeof(int64_t));
    if (lng) memcpy(lng, s->lng, SW * sizeof(double));
    if (flat) memcpy(flat, s->flat, s->S);
    if (k) memcpy(k, s->k, s->h * sizeof(int32_t));
    if (done) memcpy(done, s->done, s->h);
    if (swaps) memcpy(swaps, s->swaps, s->S);
}

void orc_set_window_lng(orc_sim* s, int32_t window, const double* tab)
{
    for (int r = 0; r < s->m; ++r)
        memcpy(s->lng + (size_t)(window * s->m + r) * s->WB, tab, s->WB * sizeof(double));
}

void orc_window_lng(const orc_sim* s, int32_t window, double* out)
{
    memcpy(out, s->lng + (size_t)window * s->m * s->WB, s->WB * sizeof(double));
}

void orc_stats(const orc_sim* s, int64_t* attempts, int64_t* ex_prop, int64_t* ex_acc)
{
    if (attempts) *attempts = s->attempts;
    if (ex_prop) memcpy(ex_prop, s->ex_prop, s->h * sizeof(int64_t));
    if (ex_acc) memcpy(ex_acc, s->ex_acc, s->h * sizeof(int64_t));
}

void orc_replicas(const orc_sim* s, int32_t* rid, int32_t* round_trips)
{
    if (rid) memcpy(rid, s->rid, s->S * sizeof(int32_t));
    if (round_trips) memcpy(round_trips, s->rt_count, s->S * sizeof(int32_t));
}

void orc_set_tables(orc_sim* s, const int64_t* H, const double* lng)
{
    size_t SW = (size_t)s->S * s->WB;
    if (H) memcpy(s->H, H, SW * sizeof(int64_t));
    if (lng) memcpy(s->lng, lng, SW * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Concatenation (Sec. II.B): in each overlap, take the 5-point derivative  */
/* of ln g of both pieces (step delta up to 10), join where the two inverse */
/* microcanonical temperatures agree best, and cut the overhanging tails.   */
/* ------------------------------------------------------------------------ */
static double stencil(const double* f, int b, int d)
{
    double num = ((f[b - 2 * d] - 8.0 * f[b - d]) + 8.0 * f[b + d]) - f[b + 2 * d];
    return num / (12.0 * d);
}

int orc_concat(const orc_config* c, const uint8_t* mask, const double* pieces, double* out,
               int32_t* join)
{
    int h = c->n_windows, W = orc_n_bins(c);
    int32_t* lo = malloc(h * sizeof(int32_t));
    int32_t* hi = malloc(h * sizeof(int32_t));
    if (orc_layout(c, lo, hi) != 0) { free(lo); free(hi); return -1; }
    int WB = 0;
    for (int a = 0; a < h; ++a)
        if (hi[a] - lo[a] + 1 > WB) WB = hi[a] - lo[a] + 1;
    double* shift = calloc(h, sizeof(double));
    int rc = 0;
    for (int a = 0; a + 1 < h; ++a) {
        const double* fa = pieces + (size_t)a * WB;       /* index: bin - lo[a]   */
        const double* fb = pieces + (size_t)(a + 1) * WB; /* index: bin - lo[a+1] */
        int ov = hi[a] - lo[a + 1] + 1;
        int d = ov / 8;
        if (d < 1) d = 1;
        if (d > 10) d = 10;
        int best = -1;
        double best_diff = 0.0;
        /* joins ascend: the search starts above the previous join point */
        int first = lo[a + 1] + 2 * d;
        if (a > 0 && join[a - 1] + 1 > first) first = join[a - 1] + 1;
        for (int b = first; b + 2 * d <= hi[a]; ++b) {
            if (!mask[b] || !mask[b - d] || !mask[b + d] || !mask[b - 2 * d] || !mask[b + 2 * d])
                continue;
            double ba = stencil(fa, b - lo[a], d);
            double bb = stencil(fb, b - lo[a + 1], d);
            double diff = fabs(ba - bb);
            if (best < 0 || diff < best_diff) {
                best = b;
                best_diff = diff;
            }
        }
        if (best < 0) { rc = -2; break; }
        join[a] = best;
        shift[a + 1] = shift[a] + (fa[best - lo[a]] - fb[best - lo[a + 1]]);
    }
    if (rc == 0) {
        int a = 0;
        for (int b = 0; b < W; ++b) {
            while (a + 1 < h && b > join[a]) ++a;
            out[b] = pieces[(size_t)a * WB + (b - lo[a])] + shift[a];
        }
        /* normalise: sum over occurring levels of g(E) = q^N (Ising: 2^N) */
        double mx = -INFINITY;
        for (int b = 0; b < W; ++b)
            if (mask[b] && out[b] > mx) mx = out[b];
        double acc = 0.0;
        for (int b = 0; b < W; ++b)
            if (mask[b]) acc += exp(out[b] - mx);
        double lse = mx + log(acc);
        double N = (double)c->L * c->L;
        double target = N * log(c->model == 0 ? 2.0 : (double)c->q);
        for (int b = 0; b < W; ++b) out[b] = mask[b] ? out[b] + (target - lse) : -INFINITY;
    }
    free(lo); free(hi); free(shift);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Bootstrap over n independent runs (Sec. II.B, error analysis): each       */
/* resample takes, for every window on its own, n of the runs' pieces with   */
/* repetition.  The draws are Philox words like every other random number   */
/* of the method (counter = resample, draw, window, stream tag).             */
/* ------------------------------------------------------------------------ */
int orc_boot_picks(uint64_t seed, int32_t R, int32_t h, int32_t n, int32_t* picks)
{
    if (n < 1 || h < 1 || R < 0) return -1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int32_t r = 0; r <= R; ++r)
        for (int32_t a = 0; a < h; ++a)
            for (int32_t j = 0; j < n; ++j) {
                int32_t* p = picks + ((size_t)r * h + a) * n + j;
                if (r == 0) {
                    *p = j;
                    continue;
                }
                uint32_t ctr[4] = {(uint32_t)r, (uint32_t)j, (uint32_t)a, TAG_BOOT}, x[4];
                orc_philox4x32_10(ctr, key, x);
                *p = (int32_t)(((uint64_t)x[0] * (uint64_t)n) >> 32);
            }
    return 0;
}
