// rewl_api.hip -- host side of librewl: validation, layout, device state,
// the interval launch sequence (plain or as a replayed HIP graph) and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rewl.h"
#include "rewl_kernels.hip"
#include "ensemble_kernels.hip"

using namespace rewl;

namespace {

thread_local std::string g_err;

rewl_status fail(rewl_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(REWL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

int ilog2_exact(int64_t v)
{
    int j = 0;
    while ((int64_t(1) << j) < v) ++j;
    return (int64_t(1) << j) == v ? j : -1;
}

int64_t n_bins_of(const rewl_config& c)
{
    const int64_t N = (int64_t)c.L * c.L;
    return c.model == 0 ? N + 1 : 2 * N + 1;
}

// Sec. II.A partition: h windows of equal width w over S = W-1 bin steps, each
// sharing at least a fraction o of its width with the next lower window (up to
// one bin lost to integer starts); width w = ceil(S den / (den + (h-1)(den-num))),
// start a = floor(a (S - w) / (h - 1)).  This reproduces the Potts example of
// Sec. IV.A: width 1000, shift 250, 77/317/717/1277 windows for L = 100..400.
bool layout_of(const rewl_config& c, std::vector<int32_t>& lo, std::vector<int32_t>& hi)
{
    const int64_t S = n_bins_of(c) - 1, h = c.n_windows, num = c.overlap_num, den = c.overlap_den;
    if (c.window_lo || c.window_hi) {
        if (!c.window_lo || !c.window_hi || h < 1) return false;
        lo.assign(c.window_lo, c.window_lo + h);
        hi.assign(c.window_hi, c.window_hi + h);
        for (int64_t a = 0; a < h; ++a) {
            if (lo[a] < 0 || hi[a] > S || hi[a] - lo[a] < 1) return false;
            if (a > 0 && (lo[a] <= lo[a - 1] || hi[a] <= hi[a - 1] || lo[a] > hi[a - 1])) return false;
        }
        return lo[0] == 0 && hi[h - 1] == S;
    }
    if (h < 1 || den < 1 || num < 0 || num >= den) return false;
    lo.assign(h, 0);
    hi.assign(h, 0);
    if (h == 1) {
        hi[0] = (int32_t)S;
        return true;
    }
    const int64_t D = den + (h - 1) * (den - num);
    int64_t w = (S * den + D - 1) / D;
    if (w > S) w = S;
    for (int64_t a = 0; a < h; ++a) {
        lo[a] = (int32_t)(a * (S - w) / (h - 1));
        hi[a] = (int32_t)(lo[a] + w);
    }
    return true;
}

// Levels that never occur on the periodic lattice: Ising (even L) E = -2N+4 and
// 2N-4; Potts (q >= 3, L >= 4) one, two, three or five broken bonds.
void mask_of(const rewl_config& c, std::vector<uint8_t>& mask)
{
    const int64_t W = n_bins_of(c), N = (int64_t)c.L * c.L;
    mask.assign(W, 1);
    if (c.model == 0) {
        mask[1] = 0;
        mask[N - 1] = 0;
    } else {
        mask[1] = mask[2] = mask[3] = mask[5] = 0;
    }
}

rewl_status validate(const rewl_config& c)
{
    if (c.model != 0 && c.model != 1) return fail(REWL_E_INVALID, "model must be 0 (Ising) or 1 (Potts)");
    if (c.model == 0 && (c.L < 4 || c.L > 128 || c.L % 2))
        return fail(REWL_E_INVALID, "Ising needs an even L in [4, 128]");
    if (c.model == 1 && (c.L < 4 || c.L > 255)) return fail(REWL_E_INVALID, "Potts needs L in [4, 255]");
    if (c.model == 1 && (c.q < 3 || c.q > 255)) return fail(REWL_E_INVALID, "Potts needs q in [3, 255]");
    if (c.n_windows < 1) return fail(REWL_E_INVALID, "n_windows must be >= 1");
    if (c.overlap_den < 1 || c.overlap_num < 0 || c.overlap_num >= c.overlap_den)
        return fail(REWL_E_INVALID, "overlap must be num/den in [0, 1)");
    if (c.walkers_per_window < 1 || c.walkers_per_window > 1024 || ilog2_exact(c.walkers_per_window) < 0)
        return fail(REWL_E_INVALID, "walkers_per_window must be a power of two in [1, 1024]");
    if (c.flat_rule != REWL_FLAT_MEAN && c.flat_rule != REWL_FLAT_VISITS)
        return fail(REWL_E_INVALID, "flat_rule must be REWL_FLAT_MEAN or REWL_FLAT_VISITS");
    if (c.reserved != 0) return fail(REWL_E_INVALID, "reserved must be 0");
    if (c.flat_rule == REWL_FLAT_MEAN && (c.flat_den < 1 || c.flat_num < 0 || c.flat_num > c.flat_den))
        return fail(REWL_E_INVALID, "flatness must be num/den in [0, 1]");
    if (c.flat_rule == REWL_FLAT_VISITS &&
        (c.flat_den < 1 || c.flat_num < 0 || c.flat_den > (1 << 20) || c.flat_num > (1 << 20)))
        return fail(REWL_E_INVALID, "Eq. (8) needs a = num/den with 0 <= num, 1 <= den, both <= 2^20");
    if (c.lnf_k0 < 0 || c.lnf_kfinal <= c.lnf_k0 || c.lnf_kfinal > 40)
        return fail(REWL_E_INVALID, "need 0 <= lnf_k0 < lnf_kfinal <= 40");
    if (c.exchange_interval < 1 || c.exchange_interval > (int64_t(1) << 31))
        return fail(REWL_E_INVALID, "exchange_interval must be in [1, 2^31]");
    if (c.exchange_enabled != 0 && c.exchange_enabled != 1)
        return fail(REWL_E_INVALID, "exchange_enabled must be 0 or 1");
    std::vector<int32_t> lo, hi;
    if (!layout_of(c, lo, hi)) return fail(REWL_E_INVALID, "bad layout");
    if (hi[0] - lo[0] < 1) return fail(REWL_E_INVALID, "windows narrower than two bins");
    if ((int64_t)c.n_windows * c.walkers_per_window > (int64_t(1) << 24))
        return fail(REWL_E_INVALID, "too many walkers");
    std::vector<uint8_t> mask;
    mask_of(c, mask);
    for (int a = 0; a < c.n_windows; ++a) {
        int n = 0;
        for (int b = lo[a]; b <= hi[a]; ++b) n += mask[b];
        if (n < 1) return fail(REWL_E_EMPTY_WINDOW, "window " + std::to_string(a) + " is empty");
    }
    return REWL_OK;
}

struct HostInst {
    rewl_config cfg;
    int N, W, h, m, S, WB, log2m, wpr, wpb, kind, placement, mapn;
    size_t lds;
    std::vector<int32_t> lo, hi, nreach;
    std::vector<uint8_t> mask;
    Inst dev;
};

}  // namespace

struct rewl_handle {
    int device = 0;             // the device current at creation (owns every buffer)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n = 0;
    std::vector<HostInst> inst;
    std::vector<void*> allocs;
    Inst* d_insts = nullptr;
    Tile* d_tiles = nullptr;
    int ntiles = 0;
    int32_t* d_queue = nullptr; // tile queue of the persistent lane sweep
    int persist_grid = 0;       // its blocks: as many as the GPU holds at once
    Tile* d_wtiles = nullptr;
    int nwtiles = 0;
    int wave_threads = 64;
    size_t max_lds_wave = 0;
    int2* d_merge = nullptr;
    int nmerge = 0;
    int32_t* d_rng_start = nullptr;
    int rng_grid = 0;
    int32_t* d_exch_start = nullptr;
    int exch_threads = 0;
    int32_t* d_slot_start = nullptr;
    int slot_threads = 0;
    size_t max_lds = 0;
    InstCtr* d_ctr = nullptr;
    InstCtr* h_ctr = nullptr;   // pinned
    bool started = false;
    rewl_tune tune{};
    hipGraphExec_t gexec = nullptr;
    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double sweep_ms = 0.0, interval_ms = 0.0;

    template <class T>
    rewl_status alloc(T** p, size_t count)
    {
        void* q = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&q, count * sizeof(T));
        if (e != hipSuccess) return fail(REWL_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = (T*)q;
        return REWL_OK;
    }
};

namespace {

// The wave sweep's plan for one instance: walkers per block, count placement and
// site-map size.  Among the candidate maps (largest first) and placements (LDS
// first), the one that keeps the most of the instance's S walkers resident at
// once (fewest rounds of blocks over n_cu CUs, from the LDS per block and the
// waves a CU holds) wins; on a tie the earlier candidate.  Counts asked for in
// LDS that do not fit there go to device memory.  False when nothing fits.
struct WavePlan { int G, mapn; bool hg; size_t lds; };

bool plan_wave(int model, int L, int N, int WB, int m, int64_t S, const rewl_tune& tune, int lds_limit,
               int n_cu, int wave_cap, WavePlan* out)
{
    const int want = tune.walkers_per_block > 0 ? tune.walkers_per_block : 4;
    int G0 = 1;
    while (G0 * 2 <= std::min(want, std::min(8, m))) G0 *= 2;
    std::vector<bool> places;
    if (tune.table_placement != REWL_TABLE_DEVICE) places.push_back(false);
    if (tune.table_placement != REWL_TABLE_LDS) places.push_back(true);
    std::vector<int> maps;
    if (tune.map_log2 > 0) maps.push_back(wave_map_entries(N, tune.map_log2));
    else
        for (int lg = 12; lg >= 9; --lg) {
            const int mn = wave_map_entries(N, lg);
            if (maps.empty() || mn < maps.back()) maps.push_back(mn);
        }
    WavePlan best{0, 0, false, 0};
    int64_t best_rounds = INT64_MAX;
    auto search = [&](const std::vector<bool>& pl) {
        for (int mapn : maps)
            for (bool hg : pl) {
                int G = G0;
                while (G > 1 && wave_lds_bytes(model, L, WB, G, hg, mapn) > (size_t)lds_limit) G /= 2;
                const size_t lds = wave_lds_bytes(model, L, WB, G, hg, mapn);
                if (lds > (size_t)lds_limit) continue;
                const int64_t per_cu =
                    std::max<int64_t>(1, std::min<int64_t>((int64_t)lds_limit / (int64_t)lds, wave_cap / G));
                const int64_t resident = per_cu * G * std::max(n_cu, 1);
                const int64_t rounds = (S + resident - 1) / resident;
                if (rounds < best_rounds) {
                    best_rounds = rounds;
                    best = WavePlan{G, mapn, hg, lds};
                }
            }
    };
    search(places);
    if (best.G == 0) search({true});
    *out = best;
    return best.G > 0;
}

rewl_status enqueue_interval(rewl_handle* H, bool time_it)
{
    if (time_it) HIP_TRY(hipEventRecord(H->ev[0], H->stream));
    if (H->rng_grid > 0)
        hipLaunchKernelGGL(k_rng, dim3(H->rng_grid), dim3(256), 0, H->stream, H->d_insts,
                           H->d_rng_start, H->n);
    if (time_it) HIP_TRY(hipEventRecord(H->ev[1], H->stream));
    if (H->ntiles > 0 && H->tune.persistent)
        hipLaunchKernelGGL(k_sweep_persist, dim3(H->persist_grid), dim3(64), H->max_lds, H->stream, H->d_insts,
                           H->d_tiles, H->ntiles, H->d_queue);
    else if (H->ntiles > 0)
        hipLaunchKernelGGL(k_sweep, dim3(H->ntiles), dim3(64), H->max_lds, H->stream, H->d_insts,
                           H->d_tiles, H->ntiles);
    if (H->nwtiles > 0)
        hipLaunchKernelGGL(k_sweep_wave, dim3(H->nwtiles), dim3(H->wave_threads), H->max_lds_wave,
                           H->stream, H->d_insts, H->d_wtiles, H->nwtiles);
    if (time_it) HIP_TRY(hipEventRecord(H->ev[2], H->stream));
    hipLaunchKernelGGL(k_merge, dim3(H->nmerge), dim3(256), 0, H->stream, H->d_insts, H->d_merge);
    if (H->exch_threads > 0)
        hipLaunchKernelGGL(k_exchange, dim3((H->exch_threads + 3) / 4), dim3(256), 0, H->stream,
                           H->d_insts, H->d_exch_start, H->n);
    hipLaunchKernelGGL(k_advance, dim3((H->n + 63) / 64), dim3(64), 0, H->stream, H->d_insts, H->n,
                       H->d_queue);
    if (time_it) HIP_TRY(hipEventRecord(H->ev[3], H->stream));
    HIP_TRY(hipGetLastError());
    return REWL_OK;
}

rewl_status step(rewl_handle* H)
{
    if (H->tune.use_graph && !H->timing) {
        if (!H->gexec) {
            hipGraph_t g;
            HIP_TRY(hipStreamBeginCapture(H->stream, hipStreamCaptureModeThreadLocal));
            rewl_status s = enqueue_interval(H, false);
            hipError_t e = hipStreamEndCapture(H->stream, &g);
            if (s != REWL_OK) return s;
            HIP_TRY(e);
            HIP_TRY(hipGraphInstantiate(&H->gexec, g, nullptr, nullptr, 0));
            HIP_TRY(hipGraphDestroy(g));
        }
        HIP_TRY(hipGraphLaunch(H->gexec, H->stream));
        return REWL_OK;
    }
    rewl_status s = enqueue_interval(H, H->timing);
    if (s != REWL_OK) return s;
    if (H->timing) {
        HIP_TRY(hipEventSynchronize(H->ev[3]));
        float ms = 0.f, ms2 = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, H->ev[1], H->ev[2]));
        HIP_TRY(hipEventElapsedTime(&ms2, H->ev[0], H->ev[3]));
        H->sweep_ms += ms;
        H->interval_ms += ms2;
    }
    return REWL_OK;
}

rewl_status sync_flags(rewl_handle* H, bool* all_done)
{
    HIP_TRY(hipMemcpyAsync(H->h_ctr, H->d_ctr, sizeof(InstCtr) * H->n, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    bool all = true;
    for (int i = 0; i < H->n; ++i) {
        const InstCtr& c = H->h_ctr[i];
        if (c.err & kErrInitStuck) return fail(REWL_E_INIT_STUCK, "instance " + std::to_string(i) + ": walker stuck outside its window");
        if (c.err & kErrOverflow) return fail(REWL_E_OVERFLOW, "instance " + std::to_string(i) + ": a walker's counts spread over more than 2^32 - X since the last merge");
        if (c.err & kErrExactness) return fail(REWL_E_OVERFLOW, "instance " + std::to_string(i) + ": ln g outside the exact FP64 budget");
        all = all && c.all_done;
    }
    if (all_done) *all_done = all;
    return REWL_OK;
}

rewl_status check_inst(rewl_handle* H, int32_t i)
{
    if (!H) return fail(REWL_E_INVALID, "null handle");
    if (i < 0 || i >= H->n) return fail(REWL_E_INVALID, "instance index out of range");
    return REWL_OK;
}

}  // namespace

// ---- checkpoint: per instance the arrays below, in this order
namespace {
struct Span {
    void* dev;
    size_t bytes;
};
std::vector<Span> spans_of(rewl_handle* H, int i)
{
    HostInst& hi = H->inst[i];
    Inst& d = hi.dev;
    const size_t S = hi.S, h = hi.h, WB = hi.WB;
    std::vector<Span> v;
    if (d.model == 0) v.push_back({d.lat, (size_t)hi.cfg.L * hi.wpr * S * 8});
    else v.push_back({d.plat, (size_t)hi.N * S});
    v.push_back({d.bin, S * 4});
    v.push_back({d.H, h * WB * hi.m * 8});
    v.push_back({d.base, h * WB * 8});
    v.push_back({d.k, h * 4});
    v.push_back({d.done, h * 4});
    v.push_back({d.flat, S});
    v.push_back({d.swaps, S});
    v.push_back({d.ex_prop, h * 8});
    v.push_back({d.ex_acc, h * 8});
    v.push_back({d.merges, h * 4});
    v.push_back({d.rid, S * 4});
    v.push_back({d.rt_state, S});
    v.push_back({d.rt_count, S * 4});
    v.push_back({d.ctr, sizeof(InstCtr)});
    return v;
}
}  // namespace

namespace {
// device buffer released on every return path
struct DevBuf {
    void* p = nullptr;
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes < 8 ? 8 : bytes); }
    ~DevBuf() { if (p) (void)hipFree(p); }
    template <class T> T* as() const { return (T*)p; }
};
constexpr size_t kEnsembleMaxBytes = size_t(16) << 30;
}  // namespace

extern "C" {

const char* rewl_last_error(void) { return g_err.c_str(); }

rewl_status rewl_layout(const rewl_config* cfg, int32_t* n_bins, int32_t* window_bins, int32_t* lo,
                        int32_t* hi)
{
    if (!cfg) return fail(REWL_E_INVALID, "null config");
    rewl_status s = validate(*cfg);
    if (s != REWL_OK) return s;
    std::vector<int32_t> l, u;
    layout_of(*cfg, l, u);
    if (n_bins) *n_bins = (int32_t)n_bins_of(*cfg);
    if (window_bins) {
        int32_t wb = 0;
        for (size_t a = 0; a < l.size(); ++a) wb = std::max(wb, u[a] - l[a] + 1);
        *window_bins = wb;
    }
    if (lo) std::copy(l.begin(), l.end(), lo);
    if (hi) std::copy(u.begin(), u.end(), hi);
    return REWL_OK;
}

rewl_status rewl_wave_plan(const rewl_config* cfg, const rewl_tune* tune, int32_t lds_per_block, int32_t n_cu,
                           int32_t waves_per_cu, int32_t* walkers_per_block, int32_t* placement,
                           int32_t* map_entries, size_t* lds_bytes)
{
    if (!cfg) return fail(REWL_E_INVALID, "null config");
    rewl_status s = validate(*cfg);
    if (s != REWL_OK) return s;
    if (lds_per_block < 1 || n_cu < 1 || waves_per_cu < 1)
        return fail(REWL_E_INVALID, "lds_per_block, n_cu and waves_per_cu must be positive");
    rewl_tune t{};
    if (tune) t = *tune;
    if (t.table_placement < REWL_TABLE_AUTO || t.table_placement > REWL_TABLE_DEVICE)
        return fail(REWL_E_INVALID, "table_placement must be REWL_TABLE_AUTO, _LDS or _DEVICE");
    if (t.map_log2 != 0 && (t.map_log2 < 6 || t.map_log2 > 12))
        return fail(REWL_E_INVALID, "map_log2 must be 0 (auto) or in [6, 12]");
    std::vector<int32_t> l, u;
    layout_of(*cfg, l, u);
    int WB = 0;
    for (size_t a = 0; a < l.size(); ++a) WB = std::max(WB, u[a] - l[a] + 1);
    const int N = cfg->L * cfg->L, m = cfg->walkers_per_window;
    WavePlan p;
    if (!plan_wave(cfg->model, cfg->L, N, WB, m, (int64_t)cfg->n_windows * m, t, lds_per_block, n_cu,
                   waves_per_cu, &p))
        return fail(REWL_E_INVALID, "one walker's wave tables exceed the LDS per block");
    if (walkers_per_block) *walkers_per_block = p.G;
    if (placement) *placement = p.hg ? REWL_TABLE_DEVICE : REWL_TABLE_LDS;
    if (map_entries) *map_entries = p.mapn;
    if (lds_bytes) *lds_bytes = p.lds;
    return REWL_OK;
}

rewl_status rewl_tilt_density(const rewl_config* cfg, double* rho)
{
    if (!cfg || !rho) return fail(REWL_E_INVALID, "null argument");
    rewl_config c = *cfg;
    c.window_lo = c.window_hi = nullptr;
    rewl_status st = validate(c);
    if (st != REWL_OK) return st;
    const double N = (double)c.L * c.L, cap = N / 5.0;
    const int W = c.model == 0 ? c.L * c.L + 1 : 2 * c.L * c.L + 1;
    for (int b = 0; b < W; ++b) {
        double kappa;
        if (c.model == 0) {
            const double d = std::min({(double)b, (double)(W - 1 - b), cap});
            kappa = 1.0 + N / (d + 2.0);
        } else {
            kappa = 1.0 + 18.0 * N / (std::min((double)b, cap) + 4.0);
        }
        rho[b] = std::sqrt(kappa);
    }
    return REWL_OK;
}

rewl_status rewl_balanced_layout(const rewl_config* cfg, const double* rho, int32_t* lo, int32_t* hi)
{
    if (!cfg || !rho || !lo || !hi) return fail(REWL_E_INVALID, "null argument");
    rewl_config c = *cfg;
    c.window_lo = c.window_hi = nullptr;
    rewl_status st = validate(c);
    if (st != REWL_OK) return st;
    const int64_t W = n_bins_of(c), h = c.n_windows;
    std::vector<double> C(W);
    double acc = 0.0;
    for (int64_t b = 0; b < W; ++b) {
        if (!(rho[b] > 0.0) || !std::isfinite(rho[b])) return fail(REWL_E_INVALID, "rho must be finite and > 0");
        acc += rho[b];
        C[b] = acc;                                   // C[b] = sum of rho over bins <= b
    }
    std::vector<int32_t> l(h), u(h);
    if (h == 1) {
        l[0] = 0;
        u[0] = (int32_t)(W - 1);
    } else {
        const double o = (double)c.overlap_num / c.overlap_den;
        const double span = acc / (1.0 + (double)(h - 1) * (1.0 - o)), step = span * (1.0 - o);
        auto first_at = [&](double v) {               // first bin whose cumulative sum reaches v
            return (int32_t)(std::lower_bound(C.begin(), C.end(), v) - C.begin());
        };
        for (int64_t a = 0; a < h; ++a) {
            l[a] = a == 0 ? 0 : std::min<int32_t>(first_at(a * step), (int32_t)(W - 1));
            u[a] = a == h - 1 ? (int32_t)(W - 1) : std::min<int32_t>(first_at(a * step + span), (int32_t)(W - 1));
        }
        // minimum sizes: 2 bins per window, 8 bins of overlap, both ends ascending
        const int32_t kMinOverlap = 8;
        for (int64_t a = 0; a < h; ++a) {
            if (a > 0) l[a] = std::max(l[a], l[a - 1] + 1);
            u[a] = std::max(u[a], l[a] + 1);
            if (a > 0) u[a] = std::max(u[a], u[a - 1] + 1);
        }
        for (int64_t a = 0; a + 1 < h; ++a)
            if (u[a] - l[a + 1] + 1 < kMinOverlap) {
                const int32_t need = kMinOverlap - (u[a] - l[a + 1] + 1);
                const int32_t down = std::min<int32_t>(need / 2 + need % 2, l[a + 1] - l[a] - 1);
                l[a + 1] -= std::max(down, 0);
                u[a] = std::min<int32_t>(u[a] + (need - std::max(down, 0)), (int32_t)(W - 1));
            }
        for (int64_t a = 1; a < h; ++a) u[a] = std::max(u[a], u[a - 1] + 1);
        u[h - 1] = (int32_t)(W - 1);
    }
    c.window_lo = l.data();
    c.window_hi = u.data();
    st = validate(c);
    if (st != REWL_OK) return fail(st, "no valid unequal layout for these sizes: " + std::string(rewl_last_error()));
    std::copy(l.begin(), l.end(), lo);
    std::copy(u.begin(), u.end(), hi);
    return REWL_OK;
}

rewl_status rewl_mask(const rewl_config* cfg, uint8_t* mask)
{
    if (!cfg || !mask) return fail(REWL_E_INVALID, "null argument");
    rewl_status s = validate(*cfg);
    if (s != REWL_OK) return s;
    std::vector<uint8_t> m;
    mask_of(*cfg, m);
    std::copy(m.begin(), m.end(), mask);
    return REWL_OK;
}

void rewl_destroy(rewl_handle* H)
{
    if (!H) return;
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    if (H->gexec) (void)hipGraphExecDestroy(H->gexec);
    for (hipEvent_t e : H->ev)
        if (e) (void)hipEventDestroy(e);
    for (void* p : H->allocs) (void)hipFree(p);
    if (H->h_ctr) (void)hipHostFree(H->h_ctr);
    if (H->own_stream && H->stream) (void)hipStreamDestroy(H->stream);
    delete H;
}

static rewl_status create_impl(const rewl_config* cfgs, int32_t n, void* hip_stream,
                               const rewl_tune* tune, rewl_handle** out)
{
    if (!cfgs || !out || n < 1) return fail(REWL_E_INVALID, "need n >= 1 configurations");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        rewl_status s = validate(cfgs[i]);
        if (s != REWL_OK) return fail(s, "instance " + std::to_string(i) + ": " + g_err);
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int lds_limit = 0, n_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (lds_limit <= 0) lds_limit = 65536;
    if (n_cu <= 0) n_cu = 1;
    // waves of the wave sweep a CU holds at once as far as registers allow
    // (one-wave blocks without LDS)
    int wave_cap = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&wave_cap, (const void*)k_sweep_wave, 64, 0));
    if (wave_cap <= 0) wave_cap = 1;

    if (tune && tune->guard_band_log2 != 0 && (tune->guard_band_log2 < -40 || tune->guard_band_log2 > -2))
        return fail(REWL_E_INVALID, "guard_band_log2 must be 0 (2^-40) or in [-40, -2]");
    if (tune && (tune->table_placement < REWL_TABLE_AUTO || tune->table_placement > REWL_TABLE_DEVICE))
        return fail(REWL_E_INVALID, "table_placement must be REWL_TABLE_AUTO, _LDS or _DEVICE");
    if (tune && tune->persistent != 0 && tune->persistent != 1)
        return fail(REWL_E_INVALID, "persistent must be 0 or 1");
    if (tune && tune->map_log2 != 0 && (tune->map_log2 < 6 || tune->map_log2 > 12))
        return fail(REWL_E_INVALID, "map_log2 must be 0 (auto) or in [6, 12]");
    rewl_handle* H = new rewl_handle();
    H->device = dev;
    if (tune) H->tune = *tune;
    if (H->tune.poll_every <= 0) H->tune.poll_every = 8;
    const double band = H->tune.guard_band_log2 ? std::ldexp(1.0, H->tune.guard_band_log2) : kBand;
    H->n = n;
    H->inst.resize(n);
    std::vector<Inst> devs(n);
    std::vector<Tile> tiles, wtiles;
    std::vector<int2> merges;
    std::vector<int32_t> rng_start(1, 0), exch_start(1, 0), slot_start(1, 0);
    auto bail = [&](rewl_status s) {
        rewl_destroy(H);
        return s;
    };
    if (hip_stream) {
        H->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreate(&H->stream);
        if (e != hipSuccess) return bail(fail(REWL_E_DEVICE, "hipStreamCreate failed"));
        H->own_stream = true;
    }
    for (int k = 0; k < 4; ++k)
        if (hipEventCreate(&H->ev[k]) != hipSuccess) return bail(fail(REWL_E_DEVICE, "hipEventCreate failed"));

    for (int i = 0; i < n; ++i) {
        HostInst& hi = H->inst[i];
        hi.cfg = cfgs[i];
        const rewl_config& c = hi.cfg;
        hi.N = c.L * c.L;
        hi.W = (int)n_bins_of(c);
        hi.h = c.n_windows;
        hi.m = c.walkers_per_window;
        hi.S = hi.h * hi.m;
        hi.log2m = ilog2_exact(hi.m);
        hi.wpr = c.model == 0 ? (c.L + 63) / 64 : 1;
        layout_of(c, hi.lo, hi.hi);
        mask_of(c, hi.mask);
        hi.WB = 0;                                          // the widest window
        for (int a = 0; a < hi.h; ++a) hi.WB = std::max(hi.WB, hi.hi[a] - hi.lo[a] + 1);
        hi.nreach.assign(hi.h, 0);
        for (int a = 0; a < hi.h; ++a)
            for (int b = hi.lo[a]; b <= hi.hi[a]; ++b) hi.nreach[a] += hi.mask[b];
        // sweep variant.  The lane variant serves a wave of walkers with ~74
        // instructions per wave-attempt; the wave variant serves one walker with
        // ~27 per attempt (chunked evaluation and runs).  With few walkers per
        // SIMD the chain latency sets the rate and the wave variant wins (about
        // 2.4x on Ising L=64 with 1024 walkers and on Potts q=10 L=32 with 4096);
        // with tens of thousands of walkers the lane variant's width wins (the
        // 64-instance batch).  The wave variant takes any lattice whose walker
        // tables fit the LDS with the smallest site map the choice below may
        // take, or with the one asked for.
        const bool wave_ok =
            wave_lds_bytes(c.model, c.L, hi.WB, 1, true,
                           wave_map_entries(hi.N, H->tune.map_log2 > 0 ? H->tune.map_log2 : 9)) <=
            (size_t)lds_limit;
        int64_t total_walkers = 0;
        for (int u = 0; u < n; ++u) total_walkers += (int64_t)cfgs[u].n_windows * cfgs[u].walkers_per_window;
        hi.kind = REWL_SWEEP_LANE;
        if (wave_ok && (H->tune.sweep_kind == REWL_SWEEP_WAVE ||
                        (H->tune.sweep_kind == REWL_SWEEP_AUTO && total_walkers <= 8192)))
            hi.kind = REWL_SWEEP_WAVE;
        hi.placement = REWL_TABLE_LDS;
        if (hi.kind == REWL_SWEEP_LANE) {
            int want = H->tune.walkers_per_block > 0 ? H->tune.walkers_per_block : 64;
            int wpb = 1;
            while (wpb * 2 <= std::min(want, std::min(64, hi.m))) wpb *= 2;
            size_t cap = (size_t)lds_limit;
            if (H->tune.lds_target_kb > 0) cap = std::min(cap, (size_t)H->tune.lds_target_kb * 1024);
            while (wpb > 1 && sweep_lds_bytes(c.model, c.L, hi.wpr, hi.WB, wpb) > cap) wpb /= 2;
            hi.wpb = wpb;
            hi.lds = sweep_lds_bytes(c.model, c.L, hi.wpr, hi.WB, wpb);
            H->max_lds = std::max(H->max_lds, hi.lds);
        } else {
            WavePlan best;
            if (!plan_wave(c.model, c.L, hi.N, hi.WB, hi.m, hi.S, H->tune, lds_limit, n_cu, wave_cap, &best))
                return bail(fail(REWL_E_INVALID, "instance " + std::to_string(i) + ": one walker's tables exceed LDS"));
            hi.placement = best.hg ? REWL_TABLE_DEVICE : REWL_TABLE_LDS;
            hi.wpb = best.G;
            hi.mapn = best.mapn;
            hi.lds = best.lds;
            H->max_lds_wave = std::max(H->max_lds_wave, hi.lds);
            H->wave_threads = std::max(H->wave_threads, 64 * best.G);
        }
        if (hi.lds > (size_t)lds_limit)
            return bail(fail(REWL_E_INVALID, "instance " + std::to_string(i) + ": one walker's tables exceed LDS"));

        Inst& d = hi.dev;
        std::memset(&d, 0, sizeof(d));
        d.model = c.model; d.q = c.model ? c.q : 2; d.L = c.L; d.N = hi.N; d.W = hi.W; d.h = hi.h;
        d.m = hi.m; d.S = hi.S; d.WB = hi.WB; d.log2m = hi.log2m; d.flat_num = c.flat_num;
        d.flat_den = c.flat_den; d.flat_rule = c.flat_rule; d.kfinal = c.lnf_kfinal; d.exch = c.exchange_enabled; d.wpr = hi.wpr;
        d.X = c.exchange_interval; d.k0 = (uint32_t)c.seed; d.k1 = (uint32_t)(c.seed >> 32);
        d.band = band;
        d.hglobal = hi.placement == REWL_TABLE_DEVICE ? 1 : 0;
        d.mapn = hi.kind == REWL_SWEEP_WAVE ? hi.mapn : 0;
        d.XP = (c.exchange_interval + 31) / 32 * 32;   // two draw chunks of 16
        if ((uint64_t)d.XP * hi.S >= (uint64_t(1) << 32))
            return bail(fail(REWL_E_INVALID, "instance " + std::to_string(i) + ": walkers x interval exceeds 2^32 draws"));
        const size_t S = hi.S, h = hi.h, WB = hi.WB;
        rewl_status s = REWL_OK;
        if (c.model == 0) s = H->alloc(&d.lat, (size_t)c.L * hi.wpr * S);
        else s = H->alloc(&d.plat, (size_t)hi.N * S);
        if (s == REWL_OK) s = H->alloc(&d.bin, S);
        if (s == REWL_OK) s = H->alloc(&d.H, h * WB * hi.m);
        if (s == REWL_OK) s = H->alloc(&d.base, h * WB);
        if (s == REWL_OK) s = H->alloc(&d.lo, h);
        if (s == REWL_OK) s = H->alloc(&d.hi, h);
        if (s == REWL_OK) s = H->alloc(&d.nreach, h);
        if (s == REWL_OK) s = H->alloc(&d.mask, hi.W);
        if (s == REWL_OK) s = H->alloc(&d.k, h);
        if (s == REWL_OK) s = H->alloc(&d.done, h);
        if (s == REWL_OK) s = H->alloc(&d.flat, S);
        if (s == REWL_OK) s = H->alloc(&d.swaps, S);
        const size_t ndraw = hi.kind == REWL_SWEEP_LANE ? (size_t)d.XP * S : 1;
        if (s == REWL_OK) s = H->alloc(&d.rpack, ndraw);
        if (s == REWL_OK) s = H->alloc(&d.rv, ndraw);
        if (s == REWL_OK) s = H->alloc(&d.ex_prop, h);
        if (s == REWL_OK) s = H->alloc(&d.ex_acc, h);
        if (s == REWL_OK) s = H->alloc(&d.merges, h);
        if (s == REWL_OK) s = H->alloc(&d.rid, S);
        if (s == REWL_OK) s = H->alloc(&d.rt_state, S);
        if (s == REWL_OK) s = H->alloc(&d.rt_count, S);
        if (s != REWL_OK) return bail(s);

        std::vector<int32_t> kinit(h, c.lnf_k0), zeros(h, 0);
        std::vector<int32_t> merges0(h, -1), rid0(S);
        std::vector<int8_t> rts0(S);
        for (size_t sl = 0; sl < S; ++sl) {
            rid0[sl] = (int32_t)sl;                            // replica r starts in slot r
            rts0[sl] = sl / hi.m == 0 ? 1 : 0;                 // starting in window 0 counts as a visit
        }
        hipStream_t st = H->stream;
        bool ok = true;
        ok &= hipMemcpyAsync(d.lo, hi.lo.data(), h * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.hi, hi.hi.data(), h * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.nreach, hi.nreach.data(), h * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.mask, hi.mask.data(), hi.W, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.k, kinit.data(), h * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.merges, merges0.data(), h * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.rid, rid0.data(), S * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemcpyAsync(d.rt_state, rts0.data(), S, hipMemcpyHostToDevice, st) == hipSuccess;
        ok &= hipMemsetAsync(d.rt_count, 0, S * 4, st) == hipSuccess;
        ok &= hipMemsetAsync(d.done, 0, h * 4, st) == hipSuccess;
        ok &= hipMemsetAsync(d.H, 0, h * WB * hi.m * 8, st) == hipSuccess;
        ok &= hipMemsetAsync(d.base, 0, h * WB * 8, st) == hipSuccess;
        ok &= hipMemsetAsync(d.flat, 0, S, st) == hipSuccess;
        ok &= hipMemsetAsync(d.swaps, 0xff, S, st) == hipSuccess;
        ok &= hipMemsetAsync(d.ex_prop, 0, h * 8, st) == hipSuccess;
        ok &= hipMemsetAsync(d.ex_acc, 0, h * 8, st) == hipSuccess;
        ok &= hipStreamSynchronize(st) == hipSuccess;   // host vectors above are locals
        if (!ok) return bail(fail(REWL_E_DEVICE, "initial upload failed"));

        for (int a = 0; a < hi.h; ++a) {
            merges.push_back(make_int2(i, a));
            for (int r0 = 0; r0 < hi.m; r0 += hi.wpb)
                (hi.kind == REWL_SWEEP_LANE ? tiles : wtiles).push_back({i, a, r0, hi.wpb});
        }
        const int64_t work = c.exchange_interval * (int64_t)S;
        const int64_t nb = hi.kind != REWL_SWEEP_LANE
                               ? 0
                               : std::min<int64_t>(std::max<int64_t>((work + 2047) / 2048, 1), 16384);
        rng_start.push_back(rng_start.back() + (int32_t)nb);
        exch_start.push_back(exch_start.back() + ((c.exchange_enabled && hi.h > 1) ? (hi.h - 1) * hi.m : 0));
        slot_start.push_back(slot_start.back() + hi.S);
    }
    rewl_status s = H->alloc(&H->d_ctr, n);
    if (s != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_queue, 1)) != REWL_OK) return bail(s);
    if (hipMemsetAsync(H->d_queue, 0, 4, H->stream) != hipSuccess)
        return bail(fail(REWL_E_DEVICE, "memset failed"));
    if (hipHostMalloc((void**)&H->h_ctr, sizeof(InstCtr) * n, hipHostMallocDefault) != hipSuccess)
        return bail(fail(REWL_E_NOMEM, "hipHostMalloc failed"));
    if (hipMemsetAsync(H->d_ctr, 0, sizeof(InstCtr) * n, H->stream) != hipSuccess)
        return bail(fail(REWL_E_DEVICE, "memset failed"));
    for (int i = 0; i < n; ++i) {
        H->inst[i].dev.ctr = H->d_ctr + i;
        devs[i] = H->inst[i].dev;
    }
    // lane tiles longest first (Potts before Ising, larger lattices first): the
    // persistent sweep hands them out in this order, the plain launch in block order
    std::stable_sort(tiles.begin(), tiles.end(), [&](const Tile& x, const Tile& y) {
        const HostInst &a = H->inst[x.inst], &b = H->inst[y.inst];
        if (a.cfg.model != b.cfg.model) return a.cfg.model > b.cfg.model;
        return a.N > b.N;
    });
    H->ntiles = (int)tiles.size();
    H->nwtiles = (int)wtiles.size();
    H->nmerge = (int)merges.size();
    H->rng_grid = rng_start.back();
    H->exch_threads = exch_start.back();
    H->slot_threads = slot_start.back();
    if ((s = H->alloc(&H->d_insts, n)) != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_tiles, tiles.size())) != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_wtiles, wtiles.size())) != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_merge, merges.size())) != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_rng_start, rng_start.size())) != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_exch_start, exch_start.size())) != REWL_OK) return bail(s);
    if ((s = H->alloc(&H->d_slot_start, slot_start.size())) != REWL_OK) return bail(s);
    bool ok = true;
    hipStream_t st = H->stream;
    ok &= hipMemcpyAsync(H->d_insts, devs.data(), sizeof(Inst) * n, hipMemcpyHostToDevice, st) == hipSuccess;
    if (!tiles.empty())
        ok &= hipMemcpyAsync(H->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    if (!wtiles.empty())
        ok &= hipMemcpyAsync(H->d_wtiles, wtiles.data(), sizeof(Tile) * wtiles.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipMemcpyAsync(H->d_merge, merges.data(), sizeof(int2) * merges.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipMemcpyAsync(H->d_rng_start, rng_start.data(), 4 * rng_start.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipMemcpyAsync(H->d_exch_start, exch_start.data(), 4 * exch_start.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipMemcpyAsync(H->d_slot_start, slot_start.data(), 4 * slot_start.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipStreamSynchronize(st) == hipSuccess;
    if (!ok) return bail(fail(REWL_E_DEVICE, "descriptor upload failed"));
    if (hipFuncSetAttribute((const void*)k_sweep, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)std::max<size_t>(H->max_lds, 1)) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_sweep_persist, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)std::max<size_t>(H->max_lds, 1)) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_sweep_wave, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)std::max<size_t>(H->max_lds_wave, 1)) != hipSuccess)
        return bail(fail(REWL_E_DEVICE, "cannot raise the dynamic LDS limit"));

    if (H->ntiles > 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_sweep_persist, 64,
                                                         std::max<size_t>(H->max_lds, 1)) != hipSuccess)
            return bail(fail(REWL_E_DEVICE, "occupancy query failed"));
        H->persist_grid = std::max(1, std::min(H->ntiles, std::max(per_cu, 1) * n_cu));
    }
    hipLaunchKernelGGL(k_init, dim3((H->slot_threads + 127) / 128), dim3(128), 0, st, H->d_insts,
                       H->d_slot_start, n);
    if (hipGetLastError() != hipSuccess) return bail(fail(REWL_E_DEVICE, "init launch failed"));
    s = sync_flags(H, nullptr);
    if (s != REWL_OK) return bail(s);
    *out = H;
    return REWL_OK;
}

// Autotuner: build the batch with each candidate tuning, time two intervals of
// the real workload (state and draws are those of the run itself), keep the
// fastest.  Every candidate computes bit-identical results; only speed differs.
static rewl_status autotune(const rewl_config* cfgs, int32_t n, void* hip_stream,
                            const rewl_tune& base, rewl_tune* best)
{
    std::vector<rewl_tune> cand;
    const bool all_wave = true;         // the wave variant runs every supported lattice
    for (int kb : {40, 53, 80, 0})
        for (int persist : {0, 1}) {
            rewl_tune t = base;
            t.table_placement = REWL_TABLE_AUTO;
            t.sweep_kind = REWL_SWEEP_LANE;
            t.walkers_per_block = 0;
            t.lds_target_kb = kb;
            t.persistent = persist;
            t.autotune = 0;
            cand.push_back(t);
        }
    // wave variant: the library's own choice of walkers per block, placement and
    // site map (largest map that keeps the most walkers resident), the same with
    // the full map, and fixed walkers per block and placements
    struct WaveCand { int g, pl, map_log2; };
    const WaveCand wave_cands[] = {{0, REWL_TABLE_AUTO, 0}, {0, REWL_TABLE_AUTO, 12},
                                   {1, REWL_TABLE_LDS, 12},  {1, REWL_TABLE_DEVICE, 12},
                                   {4, REWL_TABLE_LDS, 12},  {4, REWL_TABLE_DEVICE, 12}};
    if (all_wave)
        for (const WaveCand& w : wave_cands) {
            rewl_tune t = base;
            t.sweep_kind = REWL_SWEEP_WAVE;
            t.walkers_per_block = w.g;
            t.lds_target_kb = 0;
            t.persistent = 0;
            t.table_placement = w.pl;
            t.map_log2 = w.map_log2;
            t.autotune = 0;
            cand.push_back(t);
        }
    double best_ms = 1e300;
    *best = cand[0];
    for (const rewl_tune& t : cand) {
        rewl_handle* h = nullptr;
        rewl_status s = create_impl(cfgs, n, hip_stream, &t, &h);
        if (s != REWL_OK) continue;                      // e.g. out of memory: skip
        h->timing = true;
        s = rewl_run_exact(h, 2);
        const double ms = h->interval_ms;
        rewl_destroy(h);
        if (s == REWL_OK && ms < best_ms) {
            best_ms = ms;
            *best = t;
        }
    }
    return best_ms < 1e300 ? REWL_OK : fail(REWL_E_DEVICE, "autotune: no candidate ran");
}

rewl_status rewl_batch_create(const rewl_config* cfgs, int32_t n, void* hip_stream,
                              const rewl_tune* tune, rewl_handle** out)
{
    if (tune && tune->autotune) {
        for (int i = 0; i < n && cfgs; ++i) {
            rewl_status s = validate(cfgs[i]);
            if (s != REWL_OK) return s;
        }
        rewl_tune best;
        rewl_status s = autotune(cfgs, n, hip_stream, *tune, &best);
        if (s != REWL_OK) return s;
        return create_impl(cfgs, n, hip_stream, &best, out);
    }
    return create_impl(cfgs, n, hip_stream, tune, out);
}

rewl_status rewl_get_tune(rewl_handle* H, rewl_tune* out)
{
    if (!H || !out) return fail(REWL_E_INVALID, "null argument");
    *out = H->tune;
    return REWL_OK;
}

rewl_status rewl_create(const rewl_config* cfg, void* hip_stream, rewl_handle** out)
{
    return create_impl(cfg, 1, hip_stream, nullptr, out);
}

rewl_status rewl_set_initial_lng(rewl_handle* H, int32_t i, const double* lng)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    if (!lng) return fail(REWL_E_INVALID, "null table");
    if (H->started) return fail(REWL_E_STATE, "warm start must precede the first interval");
    HostInst& hi = H->inst[i];
    for (int b = 0; b < hi.W; ++b) {
        const double v = lng[b];
        if (!std::isfinite(v) || std::fabs(v) >= 0x1p30 || std::ldexp(v, 20) != std::nearbyint(std::ldexp(v, 20)))
            return fail(REWL_E_INVALID, "warm-start values must be finite multiples of 2^-20 below 2^30");
    }
    std::vector<double> tab((size_t)hi.h * hi.WB);
    for (int a = 0; a < hi.h; ++a)
        for (int b = 0; b < hi.WB; ++b)
            tab[(size_t)a * hi.WB + b] = hi.lo[a] + b <= hi.hi[a] ? lng[hi.lo[a] + b] : 0.0;
    HIP_TRY(hipMemcpyAsync(hi.dev.base, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    return REWL_OK;
}

rewl_status rewl_run(rewl_handle* H, int64_t max_intervals, int32_t* all_done)
{
    if (!H) return fail(REWL_E_INVALID, "null handle");
    if (max_intervals < 0) return fail(REWL_E_INVALID, "negative interval count");
    bool all = false;
    rewl_status s = sync_flags(H, &all);
    if (s != REWL_OK) return s;
    int64_t left = max_intervals;
    while (!all && left > 0) {
        const int64_t chunk = std::min<int64_t>(left, H->tune.poll_every);
        for (int64_t c = 0; c < chunk; ++c)
            if ((s = step(H)) != REWL_OK) return s;
        H->started = true;
        left -= chunk;
        if ((s = sync_flags(H, &all)) != REWL_OK) return s;
    }
    if (all_done) *all_done = all ? 1 : 0;
    return REWL_OK;
}

rewl_status rewl_run_exact(rewl_handle* H, int64_t n)
{
    if (!H) return fail(REWL_E_INVALID, "null handle");
    rewl_status s;
    for (int64_t c = 0; c < n; ++c)
        if ((s = step(H)) != REWL_OK) return s;
    if (n > 0) H->started = true;
    return sync_flags(H, nullptr);
}

rewl_status rewl_set_timing(rewl_handle* H, int32_t on)
{
    if (!H) return fail(REWL_E_INVALID, "null handle");
    H->timing = on != 0;
    return REWL_OK;
}

rewl_status rewl_info(rewl_handle* H, int32_t i, int32_t* n_instances, int32_t* kind, int32_t* wpb,
                      size_t* lds, int32_t* placement, int32_t* map_entries)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    if (n_instances) *n_instances = H->n;
    if (kind) *kind = H->inst[i].kind;
    if (wpb) *wpb = H->inst[i].wpb;
    if (lds) *lds = H->inst[i].lds;
    if (placement) *placement = H->inst[i].placement;
    if (map_entries) *map_entries = H->inst[i].kind == REWL_SWEEP_WAVE ? H->inst[i].mapn : 0;
    return REWL_OK;
}

rewl_status rewl_get_window_lng(rewl_handle* H, int32_t i, int32_t a, double* out)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    HostInst& hi = H->inst[i];
    if (a < 0 || a >= hi.h || !out) return fail(REWL_E_INVALID, "bad window or null output");
    HIP_TRY(hipMemcpyAsync(out, hi.dev.base + (size_t)a * hi.WB, hi.WB * 8, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    return REWL_OK;
}

rewl_status rewl_get_state(rewl_handle* H, int32_t i, uint8_t* spins, int32_t* bins, int64_t* Hout,
                           double* lng, uint8_t* flat, int32_t* k, uint8_t* done, int8_t* swaps,
                           int64_t* t)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    HostInst& hi = H->inst[i];
    const Inst& d = hi.dev;
    const size_t S = hi.S, h = hi.h, WB = hi.WB, m = hi.m;
    hipStream_t st = H->stream;
    std::vector<int32_t> kk(h), dd(h);
    HIP_TRY(hipMemcpyAsync(kk.data(), d.k, h * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(dd.data(), d.done, h * 4, hipMemcpyDeviceToHost, st));
    std::vector<uint64_t> Hd;
    std::vector<double> base;
    if (Hout || lng) {
        Hd.resize(h * WB * m);
        base.resize(h * WB);
        HIP_TRY(hipMemcpyAsync(Hd.data(), d.H, Hd.size() * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(base.data(), d.base, base.size() * 8, hipMemcpyDeviceToHost, st));
    }
    std::vector<uint64_t> lat;
    std::vector<uint8_t> plat;
    if (spins) {
        if (d.model == 0) {
            lat.resize((size_t)hi.cfg.L * hi.wpr * S);
            HIP_TRY(hipMemcpyAsync(lat.data(), d.lat, lat.size() * 8, hipMemcpyDeviceToHost, st));
        } else {
            plat.resize((size_t)hi.N * S);
            HIP_TRY(hipMemcpyAsync(plat.data(), d.plat, plat.size(), hipMemcpyDeviceToHost, st));
        }
    }
    if (bins) HIP_TRY(hipMemcpyAsync(bins, d.bin, S * 4, hipMemcpyDeviceToHost, st));
    if (flat) HIP_TRY(hipMemcpyAsync(flat, d.flat, S, hipMemcpyDeviceToHost, st));
    if (swaps) HIP_TRY(hipMemcpyAsync(swaps, d.swaps, S, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(H->h_ctr, H->d_ctr, sizeof(InstCtr) * H->n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (k) std::copy(kk.begin(), kk.end(), k);
    if (done)
        for (size_t a = 0; a < h; ++a) done[a] = (uint8_t)dd[a];
    if (t) *t = H->h_ctr[i].t;
    const int L = hi.cfg.L, N = hi.N;
    if (spins) {
        for (size_t sl = 0; sl < S; ++sl)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    uint8_t v;
                    if (d.model == 0)
                        v = (uint8_t)((lat[sl * L * hi.wpr + y * hi.wpr + (x >> 6)] >> (x & 63)) & 1u);
                    else
                        v = plat[sl * N + y * L + x];
                    spins[sl * N + y * L + x] = v;
                }
    }
    if (Hout || lng) {
        for (size_t sl = 0; sl < S; ++sl) {
            const size_t a = sl / m;
            const double scale = std::ldexp(1.0, -kk[a]);
            for (size_t b = 0; b < WB; ++b) {
                const uint64_t hv = Hd[sl * WB + b];
                if (Hout) Hout[sl * WB + b] = (int64_t)hv;
                if (lng) lng[sl * WB + b] = std::fma((double)hv, scale, base[a * WB + b]);
            }
        }
    }
    return REWL_OK;
}

rewl_status rewl_get_stats(rewl_handle* H, int32_t i, rewl_stats* out, int64_t* ex_prop, int64_t* ex_acc,
                           int32_t* k, int32_t* round_trips)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    HostInst& hi = H->inst[i];
    std::vector<int32_t> kk(hi.h), rt(hi.S);
    HIP_TRY(hipMemcpyAsync(kk.data(), hi.dev.k, hi.h * 4, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipMemcpyAsync(rt.data(), hi.dev.rt_count, (size_t)hi.S * 4, hipMemcpyDeviceToHost, H->stream));
    if (ex_prop) HIP_TRY(hipMemcpyAsync(ex_prop, hi.dev.ex_prop, hi.h * 8, hipMemcpyDeviceToHost, H->stream));
    if (ex_acc) HIP_TRY(hipMemcpyAsync(ex_acc, hi.dev.ex_acc, hi.h * 8, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipMemcpyAsync(H->h_ctr, H->d_ctr, sizeof(InstCtr) * H->n, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    if (k) std::copy(kk.begin(), kk.end(), k);
    if (round_trips) std::copy(rt.begin(), rt.end(), round_trips);
    if (out) {
        const InstCtr& c = H->h_ctr[i];
        out->intervals = c.t;
        out->attempts = c.t * hi.cfg.exchange_interval * (int64_t)hi.S;
        out->windows_done = c.n_done;
        out->min_k = *std::min_element(kk.begin(), kk.end());
        out->sweep_ms = H->sweep_ms;
        out->interval_ms = H->interval_ms;
        int64_t tot = 0;
        for (int32_t v : rt) tot += v;
        out->round_trips = tot;
        out->slow_decisions = c.slow;
    }
    return REWL_OK;
}

rewl_status rewl_concat(rewl_handle* H, int32_t i, double* out_lng, int32_t* join)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    if (!out_lng) return fail(REWL_E_INVALID, "null output");
    HostInst& hi = H->inst[i];
    int32_t status = 0;
    DevBuf d_out, d_shift, d_join, d_status;       // released (after the device is idle) on every return
    HIP_TRY(d_out.alloc((size_t)hi.W * 8));
    HIP_TRY(d_shift.alloc((size_t)hi.h * 8));
    HIP_TRY(d_join.alloc((size_t)std::max(hi.h - 1, 1) * 4));
    HIP_TRY(d_status.alloc(4));
    hipLaunchKernelGGL(k_concat, dim3(1), dim3(256), 0, H->stream, H->d_insts, i, hi.dev.base,
                       d_out.as<double>(), d_join.as<int32_t>(), d_shift.as<double>(), d_status.as<int32_t>());
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out_lng, d_out.p, (size_t)hi.W * 8, hipMemcpyDeviceToHost, H->stream);
    if (e == hipSuccess && join && hi.h > 1)
        e = hipMemcpyAsync(join, d_join.p, (size_t)(hi.h - 1) * 4, hipMemcpyDeviceToHost, H->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&status, d_status.p, 4, hipMemcpyDeviceToHost, H->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(H->stream);
    if (e != hipSuccess) return fail(REWL_E_DEVICE, std::string("concat: ") + hipGetErrorString(e));
    if (status != 0) return fail(REWL_E_STATE, "no valid join point in some overlap");
    return REWL_OK;
}

// ---- concatenation without allocation.  Its device staging (the joined row,
// the pieces' shifts, the join bins and a status word) lives in `scratch`, a
// fixed array in device memory: every GPU the library runs on holds its own
// copy from load until the process ends.  Host code never uses the array's name
// as a device address; the address is looked up once per device.
constexpr size_t kScratchBytes = size_t(256) << 10;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                 // guards the lookup table and serialises calls
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev` (current), looked up on first use.
rewl_status scratch_ptr(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(REWL_E_DEVICE, "device index out of range");
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(REWL_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return REWL_OK;
}
}  // namespace

rewl_status rewl_concat_noalloc(rewl_handle* H, int32_t i, double* out_lng, int32_t* join)
{
    rewl_status s = check_inst(H, i);
    if (s != REWL_OK) return s;
    if (!out_lng) return fail(REWL_E_INVALID, "null output");
    const HostInst& hi = H->inst[i];
    const size_t nj = (size_t)std::max(hi.h - 1, 1);
    const size_t off_shift = ((size_t)hi.W * 8 + 255) & ~size_t(255);
    const size_t off_join = off_shift + (((size_t)hi.h * 8 + 255) & ~size_t(255));
    const size_t off_status = off_join + ((nj * 4 + 255) & ~size_t(255));
    if (off_status + 4 > kScratchBytes)
        return fail(REWL_E_INVALID, "rewl_concat_noalloc: " + std::to_string(hi.W) + " bins and " +
                                        std::to_string(hi.h) + " windows need " + std::to_string(off_status + 4) +
                                        " bytes of staging, above its fixed " + std::to_string(kScratchBytes) +
                                        " (use rewl_concat)");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != H->device) return fail(REWL_E_INVALID, "the handle's device is not the current device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    char* base = nullptr;
    if ((s = scratch_ptr(dev, (void**)&base)) != REWL_OK) return s;
    double* d_out = (double*)base;
    double* d_shift = (double*)(base + off_shift);
    int32_t* d_join = (int32_t*)(base + off_join);
    int32_t* d_status = (int32_t*)(base + off_status);
    int32_t status = 0;
    // k_concat writes every entry it later reads (status and shift[0] first)
    hipLaunchKernelGGL(k_concat, dim3(1), dim3(256), 0, H->stream, H->d_insts, i, hi.dev.base, d_out, d_join,
                       d_shift, d_status);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out_lng, d_out, (size_t)hi.W * 8, hipMemcpyDeviceToHost, H->stream));
    if (join && hi.h > 1)
        HIP_TRY(hipMemcpyAsync(join, d_join, (size_t)(hi.h - 1) * 4, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipMemcpyAsync(&status, d_status, 4, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    if (status != 0) return fail(REWL_E_STATE, "no valid join point in some overlap");
    return REWL_OK;
}

rewl_status rewl_ensemble(rewl_handle* H, const int32_t* runs, int32_t n, int32_t R, uint64_t seed,
                          double* out_lng, int32_t* join)
{
    if (!H || !runs || !out_lng) return fail(REWL_E_INVALID, "null argument");
    if (n < 1 || n > 4096) return fail(REWL_E_INVALID, "n must be 1..4096");
    if (R < 0 || R > 65534) return fail(REWL_E_INVALID, "R must be 0..65534");
    for (int j = 0; j < n; ++j) {
        rewl_status s = check_inst(H, runs[j]);
        if (s != REWL_OK) return s;
    }
    const HostInst& h0 = H->inst[runs[0]];
    for (int j = 1; j < n; ++j) {
        const HostInst& hj = H->inst[runs[j]];
        if (hj.cfg.model != h0.cfg.model || hj.cfg.L != h0.cfg.L || hj.dev.q != h0.dev.q ||
            hj.lo != h0.lo || hj.hi != h0.hi || hj.WB != h0.WB)
            return fail(REWL_E_INVALID, "runs " + std::to_string(runs[0]) + " and " +
                                            std::to_string(runs[j]) + " differ in model, lattice or windows");
    }
    const int h = h0.h, WB = h0.WB, W = h0.W, nj = std::max(h - 1, 1);
    const size_t rows = (size_t)R + 1;
    const size_t mean_b = rows * h * WB * 8, out_b = rows * W * 8;
    if (mean_b + out_b + rows * (nj * 4 + h * 8 + 4) > kEnsembleMaxBytes)
        return fail(REWL_E_INVALID, "ensemble tables exceed 16 GiB: use fewer resamples per call");
    std::vector<const double*> ptrs(n);
    for (int j = 0; j < n; ++j) ptrs[j] = H->inst[runs[j]].dev.base;
    // host staging first: on an early return the device buffers are released
    // (hipFree waits for the device) before these go out of scope
    std::vector<int32_t> status(rows), jall(join && h > 1 ? rows * nj : 0);
    DevBuf d_ptrs, d_mean, d_out, d_join, d_shift, d_status;
    HIP_TRY(d_ptrs.alloc(n * sizeof(double*)));
    HIP_TRY(d_mean.alloc(mean_b));
    HIP_TRY(d_out.alloc(out_b));
    HIP_TRY(d_join.alloc(rows * nj * 4));
    HIP_TRY(d_shift.alloc(rows * h * 8));
    HIP_TRY(d_status.alloc(rows * 4));
    HIP_TRY(hipMemcpyAsync(d_ptrs.p, ptrs.data(), n * sizeof(double*), hipMemcpyHostToDevice, H->stream));
    hipLaunchKernelGGL(k_boot_mean, dim3(h, (unsigned)rows), dim3(256), n * sizeof(double*), H->stream,
                       d_ptrs.as<const double*>(), n, h, WB, (uint32_t)seed, (uint32_t)(seed >> 32),
                       d_mean.as<double>());
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_concat, dim3((unsigned)rows), dim3(256), 0, H->stream, H->d_insts, runs[0],
                       d_mean.as<double>(), d_out.as<double>(), d_join.as<int32_t>(),
                       d_shift.as<double>(), d_status.as<int32_t>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out_lng, d_out.p, out_b, hipMemcpyDeviceToHost, H->stream));
    if (join && h > 1)
        HIP_TRY(hipMemcpyAsync(jall.data(), d_join.p, rows * nj * 4, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipMemcpyAsync(status.data(), d_status.p, rows * 4, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    if (join && h > 1) std::memcpy(join, jall.data(), rows * nj * 4);
    for (size_t r = 0; r < rows; ++r)
        if (status[r] != 0)
            return fail(REWL_E_STATE, "row " + std::to_string(r) + ": no valid join point in some overlap");
    return REWL_OK;
}

rewl_status rewl_thermo(int32_t model, int32_t L, const double* lng, int32_t S, const double* T,
                        int32_t nT, double* u, double* c, double* f)
{
    if (!lng || !T) return fail(REWL_E_INVALID, "null argument");
    if (model != 0 && model != 1) return fail(REWL_E_INVALID, "model must be 0 (Ising) or 1 (Potts)");
    if (L < 2 || L > 4096) return fail(REWL_E_INVALID, "L must be 2..4096");
    if (S < 1 || S > 65535 || nT < 1) return fail(REWL_E_INVALID, "need 1 <= S <= 65535 rows and nT >= 1");
    const int N = L * L, W = model == 0 ? N + 1 : 2 * N + 1;
    for (int t = 0; t < nT; ++t)
        if (!(T[t] > 0.0) || !std::isfinite(T[t])) return fail(REWL_E_INVALID, "temperatures must be finite and > 0");
    for (int s = 0; s < S; ++s) {
        bool any = false;
        for (int b = 0; b < W; ++b) {
            const double v = lng[(size_t)s * W + b];
            if (std::isnan(v) || v == HUGE_VAL)
                return fail(REWL_E_INVALID, "row " + std::to_string(s) + ": ln g holds NaN or +inf");
            any |= v != -HUGE_VAL;
        }
        if (!any) return fail(REWL_E_INVALID, "row " + std::to_string(s) + ": no energy level occurs");
    }
    const size_t in_b = (size_t)S * W * 8, out_b = (size_t)S * nT * 8;
    DevBuf d_lng, d_T, d_u, d_c, d_f;
    HIP_TRY(d_lng.alloc(in_b));
    HIP_TRY(d_T.alloc((size_t)nT * 8));
    if (u) HIP_TRY(d_u.alloc(out_b));
    if (c) HIP_TRY(d_c.alloc(out_b));
    if (f) HIP_TRY(d_f.alloc(out_b));
    HIP_TRY(hipMemcpy(d_lng.p, lng, in_b, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_T.p, T, (size_t)nT * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_thermo, dim3((nT + kThermoT - 1) / kThermoT, S), dim3(64), 0, 0,
                       d_lng.as<double>(), W, model, N, d_T.as<double>(), nT, d_u.as<double>(),
                       d_c.as<double>(), d_f.as<double>());
    HIP_TRY(hipGetLastError());
    if (u) HIP_TRY(hipMemcpy(u, d_u.p, out_b, hipMemcpyDeviceToHost));
    if (c) HIP_TRY(hipMemcpy(c, d_c.p, out_b, hipMemcpyDeviceToHost));
    if (f) HIP_TRY(hipMemcpy(f, d_f.p, out_b, hipMemcpyDeviceToHost));
    HIP_TRY(hipStreamSynchronize(nullptr));
    return REWL_OK;
}

rewl_status rewl_checkpoint(rewl_handle* H, void* buf, size_t* len)
{
    if (!H || !len) return fail(REWL_E_INVALID, "null argument");
    size_t total = 16;
    for (int i = 0; i < H->n; ++i)
        for (const Span& sp : spans_of(H, i)) total += sp.bytes;
    if (!buf) {
        *len = total;
        return REWL_OK;
    }
    if (*len < total) return fail(REWL_E_INVALID, "checkpoint buffer too small");
    char* p = (char*)buf;
    const uint64_t magic = 0x4c57455232ull, count = (uint64_t)H->n;
    std::memcpy(p, &magic, 8);
    std::memcpy(p + 8, &count, 8);
    p += 16;
    for (int i = 0; i < H->n; ++i)
        for (const Span& sp : spans_of(H, i)) {
            HIP_TRY(hipMemcpyAsync(p, sp.dev, sp.bytes, hipMemcpyDeviceToHost, H->stream));
            p += sp.bytes;
        }
    HIP_TRY(hipStreamSynchronize(H->stream));
    *len = total;
    return REWL_OK;
}

rewl_status rewl_restore(rewl_handle* H, const void* buf, size_t len)
{
    if (!H || !buf) return fail(REWL_E_INVALID, "null argument");
    size_t total = 16;
    for (int i = 0; i < H->n; ++i)
        for (const Span& sp : spans_of(H, i)) total += sp.bytes;
    uint64_t magic = 0, count = 0;
    if (len != total) return fail(REWL_E_INVALID, "checkpoint size does not match this handle");
    std::memcpy(&magic, buf, 8);
    std::memcpy(&count, (const char*)buf + 8, 8);
    if (magic != 0x4c57455232ull || count != (uint64_t)H->n) return fail(REWL_E_INVALID, "not a checkpoint of this batch");
    const char* p = (const char*)buf + 16;
    for (int i = 0; i < H->n; ++i)
        for (const Span& sp : spans_of(H, i)) {
            HIP_TRY(hipMemcpyAsync(sp.dev, p, sp.bytes, hipMemcpyHostToDevice, H->stream));
            p += sp.bytes;
        }
    HIP_TRY(hipStreamSynchronize(H->stream));
    H->started = true;
    return REWL_OK;
}

rewl_status rewl_probe_accept(const double* delta, const uint64_t* u53, int32_t n, int32_t* out)
{
    if (!delta || !u53 || !out || n < 0) return fail(REWL_E_INVALID, "bad arguments");
    if (n == 0) return REWL_OK;
    double* dd = nullptr;
    uint64_t* du = nullptr;
    int32_t* dout = nullptr;
    HIP_TRY(hipMalloc(&dd, n * 8));
    HIP_TRY(hipMalloc(&du, n * 8));
    HIP_TRY(hipMalloc(&dout, n * 4));
    hipError_t e = hipMemcpy(dd, delta, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(du, u53, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_accept_probe, dim3((n + 255) / 256), dim3(256), 0, 0, dd, du, n, dout);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, n * 4, hipMemcpyDeviceToHost);
    (void)hipFree(dd);
    (void)hipFree(du);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(REWL_E_DEVICE, hipGetErrorString(e));
    return REWL_OK;
}

rewl_status rewl_probe_philox(const uint32_t* in, int32_t n, uint32_t* out)
{
    if (!in || !out || n < 0) return fail(REWL_E_INVALID, "bad arguments");
    if (n == 0) return REWL_OK;
    uint32_t *din = nullptr, *dout = nullptr;
    HIP_TRY(hipMalloc(&din, (size_t)n * 24));
    HIP_TRY(hipMalloc(&dout, (size_t)n * 16));
    hipError_t e = hipMemcpy(din, in, (size_t)n * 24, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_philox_probe, dim3((n + 255) / 256), dim3(256), 0, 0, din, n, dout);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost);
    (void)hipFree(din);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(REWL_E_DEVICE, hipGetErrorString(e));
    return REWL_OK;
}

}  // extern "C"
