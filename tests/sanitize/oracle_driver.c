/* Drives the C oracle through every entry point under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py builds and runs it). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/rewl_oracle.h"

static int run_case(orc_config c, int intervals)
{
    int st = 0;
    orc_sim* s = orc_create(&c, NULL, NULL, &st);
    if (!s) { fprintf(stderr, "create failed %d\n", st); return 1; }
    orc_run(s, intervals, 2);
    int32_t W = orc_n_bins(&c), WB = orc_window_bins(s);
    int S = c.n_windows * c.walkers_per_window, N = c.L * c.L;
    uint8_t* spins = malloc((size_t)S * N);
    int32_t* bins = malloc(S * sizeof(int32_t));
    int64_t* H = malloc((size_t)S * WB * sizeof(int64_t));
    double* lng = malloc((size_t)S * WB * sizeof(double));
    uint8_t* flat = malloc(S);
    int32_t* k = malloc(c.n_windows * sizeof(int32_t));
    uint8_t* done = malloc(c.n_windows);
    int8_t* swaps = malloc(S);
    orc_get_state(s, spins, bins, H, lng, flat, k, done, swaps);
    int32_t* rid = malloc(S * sizeof(int32_t));
    int32_t* rt = malloc(S * sizeof(int32_t));
    orc_replicas(s, rid, rt);
    int64_t att, *ep = malloc(c.n_windows * 8), *ea = malloc(c.n_windows * 8);
    orc_stats(s, &att, ep, ea);
    orc_set_tables(s, H, lng);
    double* pieces = malloc((size_t)c.n_windows * WB * sizeof(double));
    for (int a = 0; a < c.n_windows; ++a) orc_window_lng(s, a, pieces + (size_t)a * WB);
    orc_set_window_lng(s, 0, pieces);
    uint8_t* mask = malloc(W);
    orc_mask_rule(&c, mask);
    double* out = malloc(W * sizeof(double));
    int32_t* join = malloc((c.n_windows > 1 ? c.n_windows - 1 : 1) * sizeof(int32_t));
    int rc = orc_concat(&c, mask, pieces, out, join);
    orc_run(s, 5, 1);
    int32_t* picks = malloc((size_t)3 * c.n_windows * 4 * sizeof(int32_t));
    orc_boot_picks(7, 2, c.n_windows, 4, picks);
    printf("L=%d model=%d t=%lld rc=%d E=%lld\n", c.L, c.model, (long long)orc_interval(s), rc,
           (long long)orc_energy(&c, spins));
    free(spins); free(bins); free(H); free(lng); free(flat); free(k); free(done); free(swaps);
    free(rid); free(rt); free(ep); free(ea); free(pieces); free(mask); free(out); free(join); free(picks);
    orc_destroy(s);
    return 0;
}

int main(void)
{
    orc_config a = {0, 2, 8, 4, 3, 4, 2, 4, 5, 0, 12, 1, 500, 1, 0, 0, NULL, NULL};
    orc_config b = {1, 3, 5, 3, 3, 4, 4, 4, 5, 0, 10, 1, 300, 2, 0, 0, NULL, NULL};
    orc_config c = {1, 10, 8, 4, 3, 4, 2, 1, 1, 0, 10, 1, 300, 3, 1, 0, NULL, NULL};
    int32_t lo[3] = {0, 30, 80}, hi[3] = {50, 110, 128};
    orc_config d = {1, 10, 8, 3, 3, 4, 2, 4, 5, 0, 10, 1, 300, 4, 0, 0, lo, hi};
    int fails = run_case(a, 60) + run_case(b, 60) + run_case(c, 40) + run_case(d, 40);
    for (int i = 0; i < 2000; ++i) {
        const uint64_t u = ((uint64_t)i * 0x9E3779B97F4A7C15ull) >> 11;
        (void)orc_accept(-ldexp((double)i, -8), u);
    }
    return fails;
}
