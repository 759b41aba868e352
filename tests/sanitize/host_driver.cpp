// Drives the pure-host entry points of librewl (layout, masks, unequal windows,
// validation) under AddressSanitizer and UndefinedBehaviorSanitizer; no call here
// touches a GPU (tests/test_sanitizers.py builds the library's host half with
// the sanitizers and runs this).
#include <cstdio>
#include <vector>

#include "../../include/rewl.h"

int main()
{
    int fails = 0;
    for (int model = 0; model < 2; ++model)
        for (int L : {4, 8, 16, 33, 64}) {
            if (model == 0 && (L % 2)) continue;
            for (int h : {1, 3, 8}) {
                rewl_config c{};
                c.model = model; c.q = 10; c.L = L; c.n_windows = h; c.overlap_num = 3; c.overlap_den = 4;
                c.walkers_per_window = 4; c.flat_num = 4; c.flat_den = 5; c.lnf_k0 = 0; c.lnf_kfinal = 20;
                c.exchange_enabled = 1; c.exchange_interval = 1000; c.seed = 1;
                int32_t W = 0, WB = 0;
                std::vector<int32_t> lo(h), hi(h);
                if (rewl_layout(&c, &W, &WB, lo.data(), hi.data()) != REWL_OK) { ++fails; continue; }
                std::vector<uint8_t> mask(W);
                fails += rewl_mask(&c, mask.data()) != REWL_OK;
                std::vector<double> rho(W);
                fails += rewl_tilt_density(&c, rho.data()) != REWL_OK;
                std::vector<int32_t> blo(h), bhi(h);
                const rewl_status s = rewl_balanced_layout(&c, rho.data(), blo.data(), bhi.data());
                if (s == REWL_OK) {
                    c.window_lo = blo.data();
                    c.window_hi = bhi.data();
                    fails += rewl_layout(&c, &W, &WB, lo.data(), hi.data()) != REWL_OK;
                }
            }
        }
    // invalid configurations are rejected before anything is allocated
    rewl_config bad{};
    bad.model = 0; bad.L = 7; bad.n_windows = 1; bad.overlap_den = 4; bad.walkers_per_window = 3;
    bad.flat_den = 5; bad.lnf_kfinal = 20; bad.exchange_interval = 10;
    int32_t W;
    fails += rewl_layout(&bad, &W, nullptr, nullptr, nullptr) != REWL_E_INVALID;
    fails += rewl_last_error()[0] == 0;
    std::printf("host entry points checked, %d failures\n", fails);
    return fails;
}
