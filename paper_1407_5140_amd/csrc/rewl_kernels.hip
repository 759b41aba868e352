// rewl_kernels.hip -- the REWL hot path on gfx950.
//
// One interval of replica-exchange Wang-Landau (arXiv:1407.5140 Sec. II.A):
//   k_rng      Philox draws of every flip attempt of the interval (whole GPU)
//   k_sweep    X single-site attempts per walker, one walker per lane, the
//              walker's lattice and histogram and its window's ln g base in LDS,
//              flatness test of every walker in the epilogue
//   k_merge    per window: when all m walkers are flat, average ln g, reset H,
//              halve ln f, detect convergence
//   k_exchange Eq. (1) between neighbouring windows, alternating pairings
//   k_advance  interval counter and termination bookkeeping
// All interval state lives in device memory, so an interval is a fixed
// sequence of launches that can be captured once and replayed.
#include "rewl_device.hpp"

namespace rewl {

// --------------------------------------------------------------------- RNG
// For instance i, walker row `slot` holds the interval's X draws contiguously
// (row stride XP = X rounded up to the sweep's chunk pair): entry slot*XP + j
// has site = floor(x0 N / 2^32), row = site / L, col = site % L, and
//   Ising pack = row | col<<8 | row_up<<16 | row_down<<24 (periodic rows),
//   Potts pack = row | col<<8 | off<<16, off = floor(x1 (q-1) / 2^32),
// and the acceptance threshold of u53 (threshold_of).  Consecutive threads take
// consecutive j (coalesced stores).
__global__ void __launch_bounds__(256) k_rng(const Inst* __restrict__ insts,
                                             const int32_t* __restrict__ block_start, int n_inst)
{
    int lo = 0, hi = n_inst - 1;
    const int b = blockIdx.x;
    while (lo < hi) {                          // instance owning this block
        int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const Inst& I = insts[lo];
    if (I.ctr->all_done) return;
    const uint32_t X = (uint32_t)I.X, XP = (uint32_t)I.XP;
    const uint32_t n = X * (uint32_t)I.S;      // < 2^32, checked at creation
    const uint32_t nthreads = (uint32_t)(block_start[lo + 1] - block_start[lo]) * blockDim.x;
    const uint64_t T0 = (uint64_t)I.ctr->t * (uint64_t)X;
    const uint32_t N = I.N, L = I.L, qm1 = I.q - 1;
    const float rL = 1.0f / (float)L;
    // element e = slot X + j, walked with stride nthreads = sq X + sr: the
    // division happens once per thread, then slot and j advance by adds
    const uint32_t e0 = (uint32_t)(b - block_start[lo]) * blockDim.x + threadIdx.x;
    const uint32_t sq = nthreads / X, sr = nthreads - sq * X;
    uint32_t slot = e0 / X, j = e0 - slot * X;
    for (uint64_t e = e0; e < n; e += nthreads) {
        const u32x4 x = draw(I.k0, I.k1, T0 + j, slot, kTagFlip);
        const uint32_t site = (uint32_t)(((uint64_t)x.x * N) >> 32);
        // row = site / L: site < 2^24 is exact in FP32, the product's rounding
        // puts the estimate at most one off, corrected below
        uint32_t row = (uint32_t)((float)site * rL);
        int32_t col = (int32_t)site - (int32_t)(row * L);
        if (col < 0) { --row; col += (int32_t)L; }
        else if (col >= (int32_t)L) { ++row; col -= (int32_t)L; }
        uint32_t pack;
        if (I.model) {
            pack = row | ((uint32_t)col << 8) | ((uint32_t)(((uint64_t)x.y * qm1) >> 32) << 16);
        } else {
            const uint32_t ru = row == 0 ? L - 1 : row - 1, rd = row == L - 1 ? 0 : row + 1;
            pack = row | ((uint32_t)col << 8) | (ru << 16) | (rd << 24);
        }
        const size_t idx = (size_t)slot * XP + j;
        I.rpack[idx] = pack;
        I.rv[idx] = threshold_of(u53_of(x), I.band);
        slot += sq;
        j += sr;
        if (j >= X) { j -= X; ++slot; }
    }
}

// ------------------------------------------------------------------- sweep
// LDS of one tile of nw walkers of window a:
//   base [kPad + WB + kPad]         window ln g base, +inf in the pads
//   H    [(kPad + WB + kPad) << lnw] per-walker counts, bin-major (lane minor)
//   lat  Ising [L*wpr << lnw] u64 words / Potts [N << lnw] bytes
// A move changes the bin by at most 2 (Ising) or 4 (Potts), so a proposal
// outside the window lands in a pad, sees ln g = +inf and is rejected.
constexpr int kPad = 4;

__host__ __device__ inline size_t sweep_lds_bytes(int model, int L, int wpr, int WB, int nw)
{
    const size_t nb = (size_t)WB + 2 * kPad;
    size_t s = nb * 8 + nb * nw * 4;
    s = (s + 7) & ~size_t(7);
    s += model == 0 ? (size_t)L * wpr * nw * 8 : (size_t)L * L * nw;
    return s;
}

// Exact acceptance for the lanes whose fast test fell inside the guard band:
// re-draw the attempt's u53 from its Philox counter and decide exactly.
__device__ __noinline__ bool slow_decide(const Inst& I, uint64_t T, uint32_t slot, double delta)
{
    return accept_slow(delta, u53_of(draw(I.k0, I.k1, T, slot, kTagFlip)));
}

// Native vectors for the draw chunks, loaded from the global address space
// (plain vector loads rather than flat addressing).
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ T gload(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}

// Lane l's value of a wave-uniform lane index l (v_readlane).
__device__ __forceinline__ uint32_t rl(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t rl64(uint64_t v, int l)
{
    return ((uint64_t)rl((uint32_t)(v >> 32), l) << 32) | rl((uint32_t)v, l);
}
__device__ __forceinline__ double rld(double v, int l)
{
    return __builtin_bit_cast(double, rl64(__builtin_bit_cast(uint64_t, v), l));
}

template <int MODEL, int WPR>
__device__ void sweep_tile(const Inst& I, const Tile& tile, char* smem)
{
    const int a = tile.window, nw = tile.nw, lane = threadIdx.x;
    const int WB = I.WB, L = I.L, N = I.N;
    const int slot0 = a * I.m + tile.r0;
    const int lo = I.lo[a];
    const int nbins = WB + 2 * kPad;
    double* lbase = (double*)smem;                               // index kPad + bin
    uint32_t* lH = (uint32_t*)(lbase + nbins);                   // index (kPad + bin) << lnw | lane
    char* latp = smem + ((nbins * 8 + (size_t)nbins * nw * 4 + 7) & ~size_t(7));
    const int nthr = blockDim.x;
    const int lnw = __builtin_ctz(nw);                           // nw is a power of two

    // ---- stage the window table, the tile's histograms and lattices in LDS.
    //      A walker's counts enter LDS relative to an offset cw of its own (kept by
    //      lane l for walker l): every decision of the sweep compares two ln g
    //      values of one walker, so a per-walker constant cancels, and the 32-bit
    //      LDS entries only need to hold the counts' spread around the offset.
    //      cw = H(current bin) - 2^31 when that count is past 2^31, else 0 (so
    //      counts below 2^31 enter as they are).  Levels that never occur carry
    //      the sentinel 0xffffffff (never visited, excluded from the flatness
    //      minimum, written back as 0).
    // bins b >= width (a window narrower than WB) are outside the window: +inf
    // table (moves there are rejected) and the never-visited sentinel
    const int width = I.hi[a] - lo + 1;
    for (int i = lane; i < nbins; i += nthr) {
        const int b = i - kPad;
        lbase[i] = (b >= 0 && b < width) ? I.base[(size_t)a * WB + b] : __builtin_inf();
    }
    uint64_t cw = 0;
    if (lane < nw) {
        const uint64_t hc0 = I.H[(size_t)(slot0 + lane) * WB + (I.bin[slot0 + lane] - lo)];
        cw = hc0 > (1ull << 31) ? hc0 - (1ull << 31) : 0ull;
    }
    // counts must lie in [cw, cw + 2^32 - 1 - X) so that this interval's X
    // updates stay below the sentinel; otherwise the run reports an overflow
    const uint64_t span = 0xffffffffull - (uint64_t)I.X;
    // global H is walker-major: H[slot][bin]; consecutive threads take consecutive bins
    bool bad = false;
    for (int l = 0; l < nw; ++l) {
        const uint64_t cl = rl64(cw, l);
        for (int i = lane; i < nbins; i += nthr) {
            const int b = i - kPad;
            uint32_t hv = 0;
            if (b >= 0 && b < WB) {
                hv = 0xffffffffu;
                if (b < width && I.mask[lo + b]) {
                    const uint64_t v = I.H[(size_t)(slot0 + l) * WB + b] - cl;   // wraps if below cl
                    bad |= v >= span;
                    hv = (uint32_t)v;
                }
            }
            lH[(i << lnw) + l] = hv;
        }
    }
    if (bad) atomicOr(&I.ctr->err, kErrOverflow);
    // lattices are walker-major too: lat[slot][word] / plat[slot][site]
    if (MODEL == 0) {
        uint64_t* lat = (uint64_t*)latp;
        const int nwords = L * WPR;
        for (int l = 0; l < nw; ++l)
            for (int w = lane; w < nwords; w += nthr) lat[(w << lnw) + l] = I.lat[(size_t)(slot0 + l) * nwords + w];
    } else {
        uint8_t* lat = (uint8_t*)latp;
        for (int l = 0; l < nw; ++l)
            for (int w = lane; w < N; w += nthr) lat[(w << lnw) + l] = I.plat[(size_t)(slot0 + l) * N + w];
    }
    __syncthreads();

    const int k = I.k[a];
    const uint32_t inc = I.done[a] == 0 ? 1u : 0u;               // converged: frozen
    const double scale = __builtin_ldexp(1.0, -k);
    const int64_t X = I.X;
    const uint64_t T0 = (uint64_t)I.ctr->t * (uint64_t)X;

    if (lane < nw) {
        const int slot = slot0 + lane;
        int b = I.bin[slot] - lo + kPad;                         // padded bin index
        uint32_t hc = lH[(b << lnw) + lane];
        double lngc = __builtin_fma((double)hc, scale, lbase[b]);
        const double incv = inc ? scale : 0.0;
        const double band2 = 2.0 * I.band;

        // one flip attempt with the precomputed draw (pk, vb) of attempt j;
        // lH always holds the walker's current counts, including bin b
        auto attempt = [&](uint32_t pk, double vb, int64_t j) {
            int nb;
            int waddr;                                           // LDS index of the flipped word/byte
            uint64_t wnew = 0;
            uint8_t pnew = 0;
            if (MODEL == 0) {
                const uint64_t* lat = (const uint64_t*)latp;
                const int r = pk & 0xff, c = (pk >> 8) & 0xff;
                const int ru = (pk >> 16) & 0xff, rd = pk >> 24;
                if (WPR == 1) {
                    const int cl = c == 0 ? L - 1 : c - 1, cr = c == L - 1 ? 0 : c + 1;
                    waddr = (r << lnw) + lane;
                    const uint64_t w = lat[waddr];
                    const uint64_t wu = lat[(ru << lnw) + lane];
                    const uint64_t wd = lat[(rd << lnw) + lane];
                    const uint32_t sp = (uint32_t)(w >> c) & 1u;
                    const uint32_t ones = ((uint32_t)(wu >> c) & 1u) + ((uint32_t)(wd >> c) & 1u) +
                                          ((uint32_t)(w >> cl) & 1u) + ((uint32_t)(w >> cr) & 1u);
                    // aligned neighbours al: dE = 4 al - 8, bin change al - 2
                    nb = b + (sp ? (int)ones : 4 - (int)ones) - 2;
                    wnew = w ^ (1ull << c);
                } else {
                    const int cl = c == 0 ? L - 1 : c - 1, cr = c == L - 1 ? 0 : c + 1;
                    auto spin = [&](int rr, int cc) -> uint32_t {
                        return (uint32_t)(lat[((rr * WPR + (cc >> 6)) << lnw) + lane] >> (cc & 63)) & 1u;
                    };
                    waddr = ((r * WPR + (c >> 6)) << lnw) + lane;
                    const uint64_t w = lat[waddr];
                    const uint32_t sp = (uint32_t)(w >> (c & 63)) & 1u;
                    const uint32_t ones = spin(ru, c) + spin(rd, c) + spin(r, cl) + spin(r, cr);
                    nb = b + (sp ? (int)ones : 4 - (int)ones) - 2;
                    wnew = w ^ (1ull << (c & 63));
                }
            } else {
                const uint8_t* lat = (const uint8_t*)latp;
                const int r = pk & 0xff, c = (pk >> 8) & 0xff;
                const int site = (int)__umul24((uint32_t)r, (uint32_t)L) + c;
                const int up = r == 0 ? site + N - L : site - L;
                const int dn = r == L - 1 ? site - N + L : site + L;
                const int lf = c == 0 ? site + L - 1 : site - 1;
                const int rt = c == L - 1 ? site - L + 1 : site + 1;
                waddr = (site << lnw) + lane;
                const int s0 = lat[waddr];
                const int n0 = lat[(up << lnw) + lane];
                const int n1 = lat[(dn << lnw) + lane];
                const int n2 = lat[(lf << lnw) + lane];
                const int n3 = lat[(rt << lnw) + lane];
                int nv = s0 + 1 + (int)(pk >> 16);
                nv = nv >= I.q ? nv - I.q : nv;
                pnew = (uint8_t)nv;
                const int nold = (n0 == s0) + (n1 == s0) + (n2 == s0) + (n3 == s0);
                const int nnew = (n0 == nv) + (n1 == nv) + (n2 == nv) + (n3 == nv);
                nb = b + nold - nnew;                            // dE = n(old) - n(new)
            }
            const double bn = lbase[nb];
            const uint32_t hn = lH[(nb << lnw) + lane];
            const double lngn = __builtin_fma((double)hn, scale, bn);   // +inf in a pad
            const double delta = lngc - lngn;                    // exact (or -inf)
            // delta > vb accepts for certain; below vb - 2 band rejects for certain
            bool f = delta > vb;
            const bool band = !f && delta >= vb - band2;
            if (__builtin_expect(__any(band), 0)) {
                if (band) {
                    f = slow_decide(I, T0 + (uint64_t)j, (uint32_t)slot, delta);
                    atomicAdd((unsigned long long*)&I.ctr->slow, 1ull);
                }
            }
            if (f) {
                if (MODEL == 0) ((uint64_t*)latp)[waddr] = wnew;
                else ((uint8_t*)latp)[waddr] = pnew;
            }
            b = f ? nb : b;
            hc = (f ? hn : hc) + inc;
            lH[(b << lnw) + lane] = hc;
            lngc = (f ? lngn : lngc) + incv;                     // exact: base + 2^-k H
        };

        // the walker's draws arrive in register chunks of kChunk attempts; the
        // next chunk's vector loads are in flight while this one is walked
        constexpr int kChunk = 16;
        const v4u* pkp = (const v4u*)(I.rpack + (size_t)slot * I.XP);
        const v2d* vp = (const v2d*)(I.rv + (size_t)slot * I.XP);
        v4u PA[kChunk / 4], PB[kChunk / 4];
        v2d VA[kChunk / 2], VB[kChunk / 2];
        auto load = [&](v4u* P, v2d* V, int64_t j0) {
#pragma unroll
            for (int i = 0; i < kChunk / 4; ++i) P[i] = gload(pkp + j0 / 4 + i);
#pragma unroll
            for (int i = 0; i < kChunk / 2; ++i) V[i] = gload(vp + j0 / 2 + i);
        };
        auto walk = [&](const v4u* P, const v2d* V, int64_t j0, bool check) {
#pragma unroll
            for (int i = 0; i < kChunk; ++i) {
                if (!check || j0 + i < X) {
                    const v4u q4 = P[i / 4];
                    const uint32_t pk = (i & 3) == 0 ? q4.x : (i & 3) == 1 ? q4.y : (i & 3) == 2 ? q4.z : q4.w;
                    const double vb = (i & 1) ? V[i / 2].y : V[i / 2].x;
                    attempt(pk, vb, j0 + i);
                }
            }
        };
        // XP is a multiple of 2 kChunk, so every chunk load below stays inside the row
        load(PA, VA, 0);
        for (int64_t j0 = 0; j0 < X; j0 += 2 * kChunk) {
            load(PB, VB, j0 + kChunk);
            if (j0 + 2 * kChunk <= X) {
                walk(PA, VA, j0, false);
                if (j0 + 2 * kChunk < X) load(PA, VA, j0 + 2 * kChunk);
                walk(PB, VB, j0 + kChunk, false);
            } else {
                walk(PA, VA, j0, true);
                walk(PB, VB, j0 + kChunk, true);
            }
        }
        I.bin[slot] = b - kPad + lo;
        I.swaps[slot] = -1;
    }
    __syncthreads();

    // ---- write back (absolute counts: the walker's offset added back)
    for (int l = 0; l < nw; ++l) {
        const uint64_t cl = rl64(cw, l);
        for (int bb = lane; bb < WB; bb += nthr) {
            const uint32_t hv = lH[((bb + kPad) << lnw) + l];
            I.H[(size_t)(slot0 + l) * WB + bb] = hv == 0xffffffffu ? 0ull : (uint64_t)hv + cl;
        }
    }
    if (MODEL == 0) {
        const uint64_t* lat = (const uint64_t*)latp;
        const int nwords = L * WPR;
        for (int l = 0; l < nw; ++l)
            for (int w = lane; w < nwords; w += nthr) I.lat[(size_t)(slot0 + l) * nwords + w] = lat[(w << lnw) + l];
    } else {
        const uint8_t* lat = (const uint8_t*)latp;
        for (int l = 0; l < nw; ++l)
            for (int w = lane; w < N; w += nthr) I.plat[(size_t)(slot0 + l) * N + w] = lat[(w << lnw) + l];
    }

    // ---- flatness of each walker (Sec. II.A, or Eq. (8)) over the levels of the
    //      window that occur; latched until the window merges
    if (inc && lane < nw) {
        uint32_t mn = 0xffffffffu;
        uint64_t sum = 0;
        for (int bb = kPad; bb < WB + kPad; ++bb) {
            const uint32_t v = lH[(bb << lnw) + lane];
            mn = v < mn ? v : mn;                                // the sentinel never wins the min
            sum += v == 0xffffffffu ? 0u : v;
        }
        const int slot = slot0 + lane;
        const int64_t n = I.nreach[a];
        if (walker_flat(I, (uint64_t)mn + cw, sum + (uint64_t)n * cw, n, k)) I.flat[slot] = 1;
    }
}

__device__ __forceinline__ void sweep_one_tile(const Inst* __restrict__ insts, const Tile& tile, char* smem)
{
    const Inst& I = insts[tile.inst];
    if (I.ctr->all_done) return;
    if (I.model == 0) {
        if (I.wpr == 1) sweep_tile<0, 1>(I, tile, smem);
        else sweep_tile<0, 2>(I, tile, smem);
    } else {
        sweep_tile<1, 1>(I, tile, smem);
    }
}

__global__ void __launch_bounds__(64) k_sweep(const Inst* __restrict__ insts,
                                              const Tile* __restrict__ tiles, int ntiles)
{
    extern __shared__ __align__(16) char smem[];
    sweep_one_tile(insts, tiles[blockIdx.x], smem);
}

// Persistent form: a grid sized to the blocks the GPU holds at once; each block
// takes the next tile from a queue counter until the tiles run out (the tiles
// are ordered longest-first by the host).  The counter is reset by k_advance at
// the end of the interval, so the launch sequence needs no memset.
__global__ void __launch_bounds__(64) k_sweep_persist(const Inst* __restrict__ insts,
                                                      const Tile* __restrict__ tiles, int ntiles,
                                                      int32_t* __restrict__ queue)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int t = next;
        __syncthreads();
        if (t >= ntiles) break;             // block-uniform: every wave of the grid ends here
        sweep_one_tile(insts, tiles[t], smem);
        __syncthreads();                    // the tile's LDS is free before the next one is staged
    }
}

// -------------------------------------------------------------- wave sweep
// One wave per walker, for workloads with few walkers: the walker's Markov
// chain runs on wave-uniform (scalar) values, and the 64 lanes draw the Philox
// numbers of the next 64 attempts in parallel (no draw buffer).
// LDS: the window's base table (shared by the block's walkers, all of one
// window), then per wave its counts (LDS placement only), then per wave its site
// map, then per wave its lattice (Potts one byte per site, Ising wpr 64-bit words
// per row).  The site map holds one 64-bit attempt mask per entry: one entry per
// site, or M = 2^j < N entries shared by the sites equal modulo M, which only
// adds attempts to the out-of-date sets, never removes one (so a smaller map
// trades extra re-evaluations for LDS).
constexpr int kWaveMapMax = 4096;
// site-map entries per walker for a lattice of N sites and a cap of 2^map_log2
// entries (0: 2^12)
__host__ __device__ inline int wave_map_entries(int N, int map_log2 = 0)
{
    const int cap = 1 << (map_log2 > 0 ? map_log2 : 12);
    return N <= cap ? N : cap;
}
__host__ __device__ inline size_t wave_lds_bytes(int model, int L, int WB, int G, bool hglobal, int mapn)
{
    const size_t nb = (size_t)WB + 2 * kPad, N = (size_t)L * L;
    size_t s = nb * 8 + (hglobal ? 0 : (size_t)G * nb * 4);
    s = (s + 7) & ~size_t(7);
    s += (size_t)G * mapn * 8;
    s += model == 1 ? (size_t)G * N : (size_t)G * L * ((L + 63) / 64) * 8;
    return s;
}

__device__ __forceinline__ uint32_t shfl32(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

// Bin change of flipping Ising spin (r, c): rows w (row r), wu (r-1), wd (r+1).
__device__ __forceinline__ int ising_d(uint64_t w, uint64_t wu, uint64_t wd, int c, int L)
{
    const int cl = c == 0 ? L - 1 : c - 1, cr = c == L - 1 ? 0 : c + 1;
    const uint32_t sp = (uint32_t)(w >> c) & 1u;
    const uint32_t ones = ((uint32_t)(wu >> c) & 1u) + ((uint32_t)(wd >> c) & 1u) +
                          ((uint32_t)(w >> cl) & 1u) + ((uint32_t)(w >> cr) & 1u);
    return (sp ? (int)ones : 4 - (int)ones) - 2;
}

// Bin change of flipping Ising spin (r, c) on rows of wpr 64-bit words.
__device__ __forceinline__ int ising_d_words(const uint64_t* rows, int wpr, int r, int ru, int rd, int c,
                                             int L)
{
    if (wpr == 1) return ising_d(rows[r], rows[ru], rows[rd], c, L);
    auto spin = [&](int rr, int cc) -> uint32_t {
        return (uint32_t)(rows[rr * wpr + (cc >> 6)] >> (cc & 63)) & 1u;
    };
    const int cl = c == 0 ? L - 1 : c - 1, cr = c == L - 1 ? 0 : c + 1;
    const uint32_t sp = spin(r, c);
    const uint32_t ones = spin(ru, c) + spin(rd, c) + spin(r, cl) + spin(r, cr);
    return (sp ? (int)ones : 4 - (int)ones) - 2;
}

// Wave variant: one walker per wave.
// * The walker's ln g over 64 consecutive bins lives in registers, one bin per
//   lane, so that no table memory is on the dependent chain; the window moves
//   when the walker comes within four bins of its edge.
// * Per chunk of 64 attempts the lanes draw the numbers and evaluate every
//   attempt's bin change d on the lattice.  A per-site bit map in LDS gives each
//   attempt the earlier attempts of the chunk whose site lies in its
//   neighbourhood (P); an attempt is out of date once one of those has flipped.
// * The chain advances a run at a time.  From attempt i on, every lane j >= i
//   evaluates its attempt as if the walker were still in its bin, with ln g
//   raised by the (j - i) updates of the attempts in between: that holds while
//   those attempts were rejected or were accepted with d = 0 (a move within the
//   bin, always accepted).  The run ends at the first accepted move with d != 0,
//   or before the first attempt that a flip of the run made out of date.
// WIDE: Ising rows of several 64-bit words (L > 64); the narrow form keeps one
// word per row.
// HG: the walker's counts stay in device memory (the 64-bit H array) instead of
// an LDS copy: they are touched only when the register window is loaded or
// stored and by the flatness test, so LDS then holds only the window's base table,
// the site maps and the lattices, and more walkers fit a block.  Both placements
// compute identical results.
template <int MODEL, bool WIDE, bool HG>
__device__ void sweep_wave(const Inst& I, const Tile& tile, char* smem)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int G = tile.nw;
    const int a = tile.window, WB = I.WB, L = I.L, N = I.N;
    const int nbins = WB + 2 * kPad;
    const int lo = I.lo[a];
    double* lbase = (double*)smem;
    // bins b >= width (a window narrower than WB) lie outside the window
    const int width = I.hi[a] - lo + 1;
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) {
        const int b = i - kPad;
        lbase[i] = (b >= 0 && b < width) ? I.base[(size_t)a * WB + b] : __builtin_inf();
    }
    const bool active = wave < G;
    const int r = tile.r0 + wave, slot = a * I.m + r;
    uint32_t* lH = (uint32_t*)(lbase + nbins) + (size_t)wave * nbins;           // LDS placement only
    uint64_t* gH = I.H + (size_t)slot * WB;                                      // the walker's counts
    const int M = I.mapn;                                     // site-map entries
    // site -> map entry: the site itself when every site has one, else site mod M
    const uint32_t mmask = M >= N ? 0xffffffffu : (uint32_t)(M - 1);
    const int wpr = WIDE ? I.wpr : 1;                         // Ising words per row
    const size_t off_map = ((size_t)nbins * 8 + (HG ? 0 : (size_t)G * nbins * 4) + 7) & ~size_t(7);
    uint64_t* lmap = (uint64_t*)(smem + off_map) + (size_t)wave * M;
    uint8_t* llat = (uint8_t*)(smem + off_map + (size_t)G * M * 8) + (size_t)wave * N;
    uint64_t* lrow = (uint64_t*)(smem + off_map + (size_t)G * M * 8) + (size_t)wave * L * wpr;
    auto ent = [&](int site) { return (int)((uint32_t)site & mmask); };
    // the walker's counts relative to an offset of its own (a per-walker constant
    // cancels from every decision), chosen and checked as in sweep_tile
    uint64_t cw = 0;
    if (active && !HG) {
        const uint64_t hc0 = I.H[(size_t)slot * WB + (I.bin[slot] - lo)];
        cw = hc0 > (1ull << 31) ? hc0 - (1ull << 31) : 0ull;
        const uint64_t span = 0xffffffffull - (uint64_t)I.X;
        bool bad = false;
        for (int i = lane; i < nbins; i += 64) {
            const int b = i - kPad;
            uint32_t hv = 0;
            if (b >= 0 && b < WB) {
                hv = 0xffffffffu;
                if (b < width && I.mask[lo + b]) {
                    const uint64_t v = I.H[(size_t)slot * WB + b] - cw;
                    bad |= v >= span;
                    hv = (uint32_t)v;
                }
            }
            lH[i] = hv;
        }
        if (bad) atomicOr(&I.ctr->err, kErrOverflow);
    }
    if (active) {
        for (int i = lane; i < M; i += 64) lmap[i] = 0;
        if (MODEL == 0) {
            for (int i = lane; i < L * wpr; i += 64) lrow[i] = I.lat[(size_t)slot * L * wpr + i];
        } else {
            for (int i = lane; i < N; i += 64) llat[i] = I.plat[(size_t)slot * N + i];
        }
    }
    __syncthreads();
    if (!active) return;

    const int k = I.k[a];
    const uint32_t inc = I.done[a] == 0 ? 1u : 0u;
    const double scale = __builtin_ldexp(1.0, -k);
    const double incv = inc ? scale : 0.0;
    const int64_t X = I.X;
    const uint64_t T0 = (uint64_t)I.ctr->t * (uint64_t)X;
    const uint32_t q = (uint32_t)I.q, qm1 = q - 1;
    const double band = I.band;
    const int b = __builtin_amdgcn_readfirstlane(I.bin[slot] - lo + kPad);

    // register window of the walker's table: lane l holds ln g of bin b0 + l
    // (+inf beyond the table).  Every value is a multiple of 2^-(k + log2 m)
    // below 2^21, so every step here is exact; the counts are recovered as
    // H = (ln g - base) 2^k when the window moves.
    const int b0max = nbins > 64 ? nbins - 64 : 0;
    int b0 = b - 32 < 0 ? 0 : (b - 32 > b0max ? b0max : b - 32);
    int idx = b - b0;                     // the walker's bin, as a lane of the window
    const double unscale = __builtin_ldexp(1.0, k);
    double gl;
    // with HG the table entries are absolute counts (below 2^53: exact in FP64)
    auto occurs = [&](int i) { return i >= kPad && i < kPad + width && I.mask[lo + i - kPad]; };
    auto load_window = [&]() {
        const int i = b0 + lane;
        if (HG) {
            // the window's entries may have been stored by other lanes of this wave
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            gl = i < nbins ? (occurs(i) ? __builtin_fma((double)gH[i - kPad], scale, lbase[i]) : lbase[i])
                           : __builtin_inf();
        } else {
            gl = i < nbins ? __builtin_fma((double)lH[i], scale, lbase[i]) : __builtin_inf();
        }
    };
    auto store_window = [&]() {
        const int i = b0 + lane;
        // pads and levels that do not occur are never visited: leave them
        if (HG) {
            if (occurs(i)) gH[i - kPad] = (uint64_t)((gl - lbase[i]) * unscale);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        } else if (i >= kPad && i < kPad + WB && lH[i] != 0xffffffffu) {
            lH[i] = (uint32_t)((gl - lbase[i]) * unscale);
        }
    };
    load_window();
    // B + j incv is the walker's ln g at its current bin before attempt j of the
    // chunk.  The register window's entry for that bin is left stale while the
    // walker stays there (only attempts with d != 0 read the window) and is
    // written when the walker leaves the bin or the window is stored.
    double B = rld(gl, idx);
    const double laneinc = (double)lane * incv;

    for (int64_t j0 = 0; j0 < X; j0 += 64) {
        const int n = (int)((X - j0) < 64 ? (X - j0) : 64);
        // ---- lanes: draws and sites of the chunk's attempts
        const u32x4 x = draw(I.k0, I.k1, T0 + (uint64_t)(j0 + lane), (uint32_t)slot, kTagFlip);
        const int site = (int)(((uint64_t)x.x * (uint32_t)N) >> 32);
        const int rr = site / L, cc = site - rr * L;
        const int ru = rr == 0 ? L - 1 : rr - 1, rd = rr == L - 1 ? 0 : rr + 1;
        const int cl = cc == 0 ? L - 1 : cc - 1, cr = cc == L - 1 ? 0 : cc + 1;
        const int s_up = ru * L + cc, s_dn = rd * L + cc, s_lf = rr * L + cl, s_rt = rr * L + cr;
        const uint32_t off = MODEL == 0 ? 0u : (uint32_t)(((uint64_t)x.y * qm1) >> 32);
        int d;                            // bin change of this lane's attempt
        uint32_t nv = 0;                  // Potts: proposed state
        auto evaluate = [&]() {           // on the lattice as it stands
            if (MODEL == 0) {
                d = ising_d_words(lrow, wpr, rr, ru, rd, cc, L);
            } else {
                const uint32_t s0 = llat[site];
                const uint32_t n0 = llat[s_up], n1 = llat[s_dn], n2 = llat[s_lf], n3 = llat[s_rt];
                nv = s0 + 1u + off;
                nv = nv >= q ? nv - q : nv;
                const int nold = (n0 == s0) + (n1 == s0) + (n2 == s0) + (n3 == s0);
                const int nnew = (n0 == nv) + (n1 == nv) + (n2 == nv) + (n3 == nv);
                d = nold - nnew;
            }
        };
        evaluate();
        const double vbl = threshold_of(u53_of(x), band);
        const double vbl2 = vbl - 2.0 * band;     // below it a reject is certain
        // attempts of the chunk at this attempt's site or one of its neighbours.
        // Neighbourhoods are symmetric, so the later ones among them (qm) are
        // exactly the attempts whose evaluation a flip of this one makes out of
        // date, and the earlier ones (pm) those whose flip makes this one out of
        // date.  (Sites sharing a map entry only add attempts to either set.)
        const uint64_t lanebit = 1ull << lane;
        if (lane < n) atomicOr((unsigned long long*)&lmap[ent(site)], lanebit);
        const uint64_t nbh = lmap[ent(site)] | lmap[ent(s_up)] | lmap[ent(s_dn)] | lmap[ent(s_lf)] |
                             lmap[ent(s_rt)];
        if (lane < n) lmap[ent(site)] = 0;
        const uint64_t pm = nbh & (lanebit - 1);
        const uint64_t qm = nbh & ~(lanebit | (lanebit - 1));
        const uint64_t live = n == 64 ? ~0ull : ((1ull << n) - 1);
        uint64_t* const fword = lrow + (WIDE ? rr * wpr + (cc >> 6) : rr);   // Ising: the flip's word
        const uint64_t fbit = 1ull << (cc & 63);
        // zall: moves within the bin (d = 0, always accepted); stale: attempts that
        // are out of date by the time the chain reaches them -- an earlier d = 0
        // move since the last evaluation lies in the neighbourhood (fixed at the
        // evaluation), or an accepted move with d != 0 since then (added per move)
        uint64_t zall, nzl, stale;
        int d4;                           // byte offset of the candidate bin's lane from idx
        auto classify = [&](int i0) {
            d4 = d << 2;
            zall = __builtin_amdgcn_ballot_w64(d == 0) & live;
            nzl = ~zall & live;
            stale = __builtin_amdgcn_ballot_w64((pm & zall & (~0ull << i0)) != 0) & live;
        };
        classify(0);

        // flips decided but not yet applied to the lattice (d = 0 moves and
        // accepted moves); they are applied together before the lattice is read
        // again (a re-evaluation, the next chunk)
        uint64_t pend = 0;
        auto apply = [&]() {
            if (pend) {
                if (__builtin_amdgcn_inverse_ballot_w64(pend)) {
                    if (MODEL == 0) atomicXor((unsigned long long*)fword, fbit);
                    else llat[site] = (uint8_t)nv;
                }
                pend = 0;
            }
        };

        // the run loop; it leaves at the end of the chunk, and to move the
        // register window when a move brings the walker within four bins of its
        // edge (then it continues at attempt i)
        int i = 0;
        for (;;) {
            const uint64_t run = ~0ull << i;              // every mask below is within live
            const double t = B + laneinc;                 // ln g of the bin, exact
            const int pos4 = d4 + (idx << 2);
            const double gp = __builtin_bit_cast(
                double, ((uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(
                             pos4, (int)(uint32_t)(__builtin_bit_cast(uint64_t, gl) >> 32))
                         << 32) |
                            (uint32_t)__builtin_amdgcn_ds_bpermute(pos4, (int)(uint32_t)__builtin_bit_cast(uint64_t, gl)));
            const double dl = t - gp;                     // ln g now - ln g of the candidate, exact
            const uint64_t gt = __builtin_amdgcn_ballot_w64(dl > vbl);
            const uint64_t ge = __builtin_amdgcn_ballot_w64(dl >= vbl2);    // holds gt
            const uint64_t nzr = nzl & run;               // attempts with d != 0 from i on
            const uint64_t acc = gt & nzr;
            const uint64_t stop = acc | (stale & run);
            uint64_t sbit = stop & (~stop + 1);           // the first stop, or 0
            uint64_t below = sbit - 1;                    // lanes below it (all if none)
            // accepted and out of date counts as out of date: re-evaluated first
            uint64_t mv = sbit & acc & ~stale;            // the accepted move, or 0
            // attempts inside the guard band are decided exactly, in order
            uint64_t amb = ge & ~gt & nzr & below;
            if (__builtin_expect(amb != 0, 0)) {
                do {
                    const int kk = (int)__builtin_ctzll(amb);
                    amb &= amb - 1;
                    if (lane == 0) atomicAdd((unsigned long long*)&I.ctr->slow, 1ull);
                    if (__builtin_amdgcn_readfirstlane(
                            slow_decide(I, T0 + (uint64_t)j0 + (uint64_t)kk, (uint32_t)slot, rld(dl, kk)) ? 1 : 0)) {
                        sbit = mv = 1ull << kk;
                        below = sbit - 1;
                        break;
                    }
                } while (amb);
            }
            // attempts i..js-1 were rejected or moved within the bin; the d = 0
            // moves among them and an accepted move at js flip
            pend |= (zall & run & below) | mv;
            if (__builtin_expect(mv != 0, 1)) {
                const int js = (int)__builtin_ctzll(mv);
                // the old bin after attempts up to js - 1 is t at lane js; the
                // differences below are exact (multiples of 2^-k, small)
                const double tjs = rld(t, js);
                const double jsinc = tjs - B;             // js incv
                if (lane == idx) gl = tjs;
                idx += __builtin_amdgcn_readlane(d, js);
                stale |= rl64(qm, js);
                // the new bin's entry lacks attempt js's update, so B = entry - js incv
                B = rld(gl, idx) - jsinc;
                i = js + 1;
                if (__builtin_expect((unsigned)(idx - 4) > 55u, 0)) {   // idx < 4 or idx > 59
                    // store the window with the bin's current value (B + i incv),
                    // reload it around the walker; the entry may stay current
                    if (lane == idx) gl = B + (double)i * incv;
                    store_window();
                    const int bb = b0 + idx;
                    b0 = bb - 32 < 0 ? 0 : (bb - 32 > b0max ? b0max : bb - 32);
                    idx = bb - b0;
                    load_window();
                }
                if (i >= n) break;
            } else {
                if (!stop) break;
                i = (int)__builtin_ctzll(stop);           // attempt i is out of date
                apply();
                evaluate();
                classify(i);
            }
        }
        apply();
        B += (double)n * incv;
    }
    if (lane == idx) gl = B;
    store_window();

    // ---- write back (HG: the window's store above is the write back)
    if (!HG)
        for (int i = lane; i < WB; i += 64) {
            const uint32_t hv = lH[i + kPad];
            gH[i] = hv == 0xffffffffu ? 0ull : (uint64_t)hv + cw;
        }
    else
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (MODEL == 0) {
        for (int i = lane; i < L * wpr; i += 64) I.lat[(size_t)slot * L * wpr + i] = lrow[i];
    } else {
        for (int i = lane; i < N; i += 64) I.plat[(size_t)slot * N + i] = llat[i];
    }
    if (lane == 0) {
        I.bin[slot] = b0 + idx - kPad + lo;
        I.swaps[slot] = -1;
    }
    // ---- flatness (Sec. II.A): wave-wide min and sum of the walker's counts
    if (inc) {
        // minimum and sum of the counts over the levels that occur (relative to cw
        // with LDS placement, absolute with HG)
        uint64_t mn = ~0ull, sum = 0;
        for (int i = lane + kPad; i < WB + kPad; i += 64) {
            if (HG) {
                if (!occurs(i)) continue;
                const uint64_t v = gH[i - kPad];
                mn = v < mn ? v : mn;
                sum += v;
            } else {
                const uint32_t v = lH[i];
                if (v == 0xffffffffu) continue;
                mn = v < mn ? v : mn;
                sum += v;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t m2 = shfl_xor_u64(mn, off), s2 = shfl_xor_u64(sum, off);
            mn = m2 < mn ? m2 : mn;
            sum += s2;
        }
        if (lane == 0) {
            const int64_t n = I.nreach[a];
            if (walker_flat(I, mn + cw, sum + (uint64_t)n * cw, n, k)) I.flat[slot] = 1;
        }
    }
}

__global__ void __launch_bounds__(512) k_sweep_wave(const Inst* __restrict__ insts,
                                                    const Tile* __restrict__ tiles, int ntiles)
{
    extern __shared__ __align__(16) char smem[];
    const Tile tile = tiles[blockIdx.x];
    const Inst& I = insts[tile.inst];
    if (I.ctr->all_done) return;
    const bool wide = I.wpr > 1;
    if (I.hglobal) {
        if (I.model == 0) {
            if (wide) sweep_wave<0, true, true>(I, tile, smem);
            else sweep_wave<0, false, true>(I, tile, smem);
        } else {
            sweep_wave<1, false, true>(I, tile, smem);
        }
    } else {
        if (I.model == 0) {
            if (wide) sweep_wave<0, true, false>(I, tile, smem);
            else sweep_wave<0, false, false>(I, tile, smem);
        } else {
            sweep_wave<1, false, false>(I, tile, smem);
        }
    }
}

// ------------------------------------------------------------------- merge
// One block per (instance, window).  When all m walkers are flat:
// ln g := mean_w ln g_w = base + 2^-(k + log2 m) sum_w H_w (exact), then the
// table is shifted by the integer part of its minimum over occurring levels.
__global__ void __launch_bounds__(256) k_merge(const Inst* __restrict__ insts,
                                               const int2* __restrict__ items)
{
    __shared__ double red[256];
    __shared__ int okflag, skip;
    const int2 it = items[blockIdx.x];
    const Inst& I = insts[it.x];
    const int a = it.y, tid = threadIdx.x;
    if (tid == 0) skip = I.ctr->all_done || I.done[a];   // one read, block-uniform
    __syncthreads();
    if (skip) return;
    int ok = 1;
    for (int r = tid; r < I.m; r += blockDim.x) ok &= I.flat[a * I.m + r];
    ok = __syncthreads_and(ok);
    if (!ok) return;
    const int WB = I.WB, m = I.m, k = I.k[a], lo = I.lo[a];
    const int sh = k + I.log2m;
    double* base = I.base + (size_t)a * WB;
    uint64_t* H = I.H + (size_t)a * m * WB;                    // the window's walkers, H[r][bin]
    double mn = __builtin_inf(), mx = 0.0;
    bool big = false;
    for (int b = tid; b < WB; b += blockDim.x) {
        uint64_t s = 0;
        for (int r = 0; r < m; ++r) s += H[(size_t)r * WB + b];
        big |= s >= (1ull << 53);                             // (double)s would round
        const double nb = base[b] + __builtin_ldexp((double)s, -sh);
        base[b] = nb;
        if (b <= I.hi[a] - lo && I.mask[lo + b]) mn = nb < mn ? nb : mn;
        mx = fabs(nb) > mx ? fabs(nb) : mx;
    }
    red[tid] = mn;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) red[tid] = red[tid + st] < red[tid] ? red[tid + st] : red[tid];
        __syncthreads();
    }
    const double shift = floor(red[0]);
    __syncthreads();
    red[tid] = mx;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) red[tid] = red[tid + st] > red[tid] ? red[tid + st] : red[tid];
        __syncthreads();
    }
    // values are multiples of 2^-sh, or of 2^-20 after a warm start: exact below 2^(52 - that)
    if (tid == 0) okflag = red[0] < __builtin_ldexp(1.0, 52 - (sh > 20 ? sh : 20));
    __syncthreads();
    if (__syncthreads_or(big) && tid == 0) okflag = 0;
    for (int b = tid; b < WB; b += blockDim.x) base[b] = base[b] - shift;
    for (size_t i = tid; i < (size_t)WB * m; i += blockDim.x) H[i] = 0ull;
    for (int r = tid; r < m; r += blockDim.x) I.flat[a * m + r] = 0;
    if (tid == 0) {
        if (!okflag) atomicOr(&I.ctr->err, kErrExactness);
        I.k[a] = k + 1;
        I.merges[a] = (int32_t)I.ctr->t;
        if (k + 1 >= I.kfinal) {
            I.done[a] = 1;
            const int nd = atomicAdd(&I.ctr->n_done, 1) + 1;
            if (nd == I.h) I.ctr->all_done = 1;
        }
    }
}

// ---------------------------------------------------------------- exchange
// Thread per (instance, window a < h-1, walker r); pairs with a = t (mod 2)
// are active.  Walker r of window a meets walker (r + c) mod m of window a+1,
// c drawn once per (t, a).  Eq. (1) in log form, decided exactly; on accept the
// two configurations (lattice and energy) change places, ln g and H stay.
__global__ void __launch_bounds__(256) k_exchange(const Inst* __restrict__ insts,
                                                  const int32_t* __restrict__ pair_start,
                                                  int n_inst)
{
    // one wave per proposing walker: every lane takes the same decision from the
    // same values, then the lanes swap the two configurations together
    const int lane = threadIdx.x & 63;
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (gw >= pair_start[n_inst]) return;
    int lo_i = 0, hi_i = n_inst - 1;
    while (lo_i < hi_i) {
        int mid = (lo_i + hi_i + 1) >> 1;
        if (pair_start[mid] <= gw) lo_i = mid;
        else hi_i = mid - 1;
    }
    const Inst& I = insts[lo_i];
    if (!I.exch || I.ctr->all_done) return;
    const int local = gw - pair_start[lo_i];
    const int m = I.m, a = local / m, r = local - a * m;
    const int64_t t = I.ctr->t;
    if ((a & 1) != (int)(t & 1)) return;
    const u32x4 xc = draw(I.k0, I.k1, (uint64_t)t, (uint32_t)a, kTagPartner);
    const int c = (int)(((uint64_t)xc.x * (uint64_t)m) >> 32);
    const int rj = (r + c) & (m - 1);
    const int i = a * m + r, j = (a + 1) * m + rj;
    const int bi = I.bin[i], bj = I.bin[j];
    const int loa = I.lo[a], hia = I.hi[a], lob = I.lo[a + 1], hib = I.hi[a + 1];
    bool acc = false;
    if (bj >= loa && bj <= hia && bi >= lob && bi <= hib) {
        const int WB = I.WB;
        const double sa = __builtin_ldexp(1.0, -I.k[a]);
        const double sb = __builtin_ldexp(1.0, -I.k[a + 1]);
        const double* ba = I.base + (size_t)a * WB;
        const double* bb = I.base + (size_t)(a + 1) * WB;
        const uint64_t* Hi = I.H + (size_t)i * WB;
        const uint64_t* Hj = I.H + (size_t)j * WB;
        auto gi = [&](int bin) { return __builtin_fma((double)Hi[bin - loa], sa, ba[bin - loa]); };
        auto gj = [&](int bin) { return __builtin_fma((double)Hj[bin - lob], sb, bb[bin - lob]); };
        const double delta = (gi(bi) - gi(bj)) + (gj(bj) - gj(bi));
        const uint64_t u53 = u53_of(draw(I.k0, I.k1, (uint64_t)t, (uint32_t)i, kTagExchange));
        const int f = decide_fast(delta, threshold_of(u53, I.band), I.band);
        if (f == 2) {
            acc = accept_slow(delta, u53);
            if (lane == 0) atomicAdd((unsigned long long*)&I.ctr->slow, 1ull);
        } else {
            acc = f == 1;
        }
    }
    if (acc) {
        if (I.model == 0) {
            const int nwords = I.L * I.wpr;
            uint64_t* pi = I.lat + (size_t)i * nwords;
            uint64_t* pj = I.lat + (size_t)j * nwords;
            for (int w = lane; w < nwords; w += 64) {
                const uint64_t x = pi[w];
                pi[w] = pj[w];
                pj[w] = x;
            }
        } else {
            uint8_t* pi = I.plat + (size_t)i * I.N;
            uint8_t* pj = I.plat + (size_t)j * I.N;
            if ((I.N & 15) == 0) {                  // rows of 16-byte words (slots are N apart)
                uint4* qi = (uint4*)pi;
                uint4* qj = (uint4*)pj;
                for (int w = lane; w < (I.N >> 4); w += 64) {
                    const uint4 x = qi[w];
                    qi[w] = qj[w];
                    qj[w] = x;
                }
            } else {
                for (int w = lane; w < I.N; w += 64) {
                    const uint8_t x = pi[w];
                    pi[w] = pj[w];
                    pj[w] = x;
                }
            }
        }
    }
    if (lane == 0) {
        if (acc) {
            I.bin[i] = bj;
            I.bin[j] = bi;
            // replicas follow their configurations; a round trip is window 0,
            // then window h-1, then window 0 again (each replica takes part in
            // one proposal per interval, so these updates do not race)
            const int up = I.rid[i], down = I.rid[j];      // up: window a -> a+1
            I.rid[i] = down;
            I.rid[j] = up;
            if (a + 1 == I.h - 1 && I.rt_state[up] == 1) I.rt_state[up] = 2;
            if (a == 0) {
                if (I.rt_state[down] == 2) I.rt_count[down] += 1;
                I.rt_state[down] = 1;
            }
            atomicAdd((unsigned long long*)&I.ex_acc[a], 1ull);
        }
        atomicAdd((unsigned long long*)&I.ex_prop[a], 1ull);
        I.swaps[i] = acc ? 1 : 0;
        I.swaps[j] = acc ? 1 : 0;
    }
}

// ----------------------------------------------------------------- advance
__global__ void k_advance(const Inst* __restrict__ insts, int n_inst, int32_t* __restrict__ queue)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *queue = 0;                 // the persistent sweep's tile queue
    if (i >= n_inst) return;
    InstCtr* c = insts[i].ctr;
    if (!c->stopped) {
        c->t += 1;
        if (c->all_done) c->stopped = 1;
    }
    c->queue = 0;
}

// -------------------------------------------------------------------- init
// Thread per slot.  Start from a ground state (Ising: all up, or the
// checkerboard for a window in the upper half; Potts: all 0) and take every
// proposal that does not increase the distance of the energy bin to the window.
__device__ int lattice_bin(const Inst& I, int slot)
{
    const int L = I.L;
    int broken = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const int xr = x + 1 == L ? 0 : x + 1, yd = y + 1 == L ? 0 : y + 1;
            if (I.model == 0) {
                auto sp = [&](int yy, int xx) {
                    return (int)(I.lat[(size_t)slot * L * I.wpr + yy * I.wpr + (xx >> 6)] >> (xx & 63)) & 1;
                };
                broken += (sp(y, x) != sp(y, xr)) + (sp(y, x) != sp(yd, x));
            } else {
                auto sp = [&](int yy, int xx) { return (int)I.plat[(size_t)slot * I.N + yy * L + xx]; };
                broken += (sp(y, x) != sp(y, xr)) + (sp(y, x) != sp(yd, x));
            }
        }
    return I.model == 0 ? broken / 2 : broken;
}

__global__ void k_init(const Inst* __restrict__ insts, const int32_t* __restrict__ thread_start,
                       int n_inst)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= thread_start[n_inst]) return;
    int lo_i = 0, hi_i = n_inst - 1;
    while (lo_i < hi_i) {
        int mid = (lo_i + hi_i + 1) >> 1;
        if (thread_start[mid] <= gid) lo_i = mid;
        else hi_i = mid - 1;
    }
    const Inst& I = insts[lo_i];
    const int slot = gid - thread_start[lo_i];
    const int a = slot / I.m, L = I.L, N = I.N;
    const int wlo = I.lo[a], whi = I.hi[a];
    const bool upper = wlo + whi > I.W - 1;
    if (I.model == 0) {
        for (int y = 0; y < L; ++y)
            for (int wi = 0; wi < I.wpr; ++wi) {
                uint64_t word = 0;
                for (int xb = 0; xb < 64; ++xb) {
                    const int x = wi * 64 + xb;
                    if (x >= L) break;
                    const bool up = upper ? ((x + y) & 1) == 0 : true;
                    word |= (uint64_t)up << xb;
                }
                I.lat[(size_t)slot * L * I.wpr + y * I.wpr + wi] = word;
            }
    } else {
        for (int s = 0; s < N; ++s) I.plat[(size_t)slot * N + s] = 0;
    }
    int b = lattice_bin(I, slot);
    auto dist = [&](int bb) { return bb < wlo ? wlo - bb : (bb > whi ? bb - whi : 0); };
    const int64_t cap = 1000 * (int64_t)N;
    for (int64_t j = 0; b < wlo || b > whi; ++j) {
        if (j >= cap) {
            atomicOr(&I.ctr->err, kErrInitStuck);
            return;
        }
        const u32x4 x = draw(I.k0, I.k1, (uint64_t)j, (uint32_t)slot, kTagInit);
        const int site = (int)(((uint64_t)x.x * (uint64_t)N) >> 32);
        const int r = site / L, c = site - r * L;
        const int ru = r == 0 ? L - 1 : r - 1, rd = r == L - 1 ? 0 : r + 1;
        const int cl = c == 0 ? L - 1 : c - 1, cr = c == L - 1 ? 0 : c + 1;
        int nb;
        int nv = 0;
        if (I.model == 0) {
            auto sp = [&](int yy, int xx) {
                return (int)(I.lat[(size_t)slot * L * I.wpr + yy * I.wpr + (xx >> 6)] >> (xx & 63)) & 1;
            };
            const int s = sp(r, c);
            const int ones = sp(ru, c) + sp(rd, c) + sp(r, cl) + sp(r, cr);
            const int al = s ? ones : 4 - ones;
            nb = b + al - 2;
        } else {
            auto sp = [&](int yy, int xx) { return (int)I.plat[(size_t)slot * N + yy * L + xx]; };
            const int s = sp(r, c);
            nv = s + 1 + (int)(((uint64_t)x.y * (uint64_t)(I.q - 1)) >> 32);
            nv = nv >= I.q ? nv - I.q : nv;
            const int n[4] = {sp(ru, c), sp(rd, c), sp(r, cl), sp(r, cr)};
            int nold = 0, nnew = 0;
            for (int d = 0; d < 4; ++d) {
                nold += n[d] == s;
                nnew += n[d] == nv;
            }
            nb = b + nold - nnew;
        }
        if (dist(nb) <= dist(b)) {
            if (I.model == 0) {
                uint64_t* p = I.lat + (size_t)slot * L * I.wpr + r * I.wpr + (c >> 6);
                *p ^= 1ull << (c & 63);
            } else {
                I.plat[(size_t)slot * N + site] = (uint8_t)nv;
            }
            b = nb;
        }
    }
    I.bin[slot] = b;
}

// ------------------------------------------------------------ concatenate
// Sec. II.B: per overlap, 5-point derivative of both pieces with step d,
// join where they agree best (ties to the lower bin, joins ascending), shift
// the pieces, cut the tails, normalise to sum g = q^N.  One block per set of
// pieces: block r joins pieces[r][h][WB] into out[r][W] (join[r][max(h-1,1)],
// shift[r][h], status[r]); all sets share the windows of instance `inst`.
__global__ void __launch_bounds__(256) k_concat(const Inst* __restrict__ insts, int inst,
                                                const double* __restrict__ pieces,
                                                double* __restrict__ out,
                                                int32_t* __restrict__ join, double* __restrict__ shift,
                                                int32_t* __restrict__ status)
{
    __shared__ double rd[256];
    __shared__ int rb[256];
    const Inst& I = insts[inst];
    const int h = I.h, WB = I.WB, W = I.W, tid = threadIdx.x;
    const size_t set = blockIdx.x;
    pieces += set * h * WB;
    out += set * W;
    join += set * (h > 1 ? h - 1 : 1);
    shift += set * h;
    status += set;
    if (tid == 0) {
        shift[0] = 0.0;
        *status = 0;
    }
    __syncthreads();
    for (int a = 0; a + 1 < h; ++a) {
        const double* fa = pieces + (size_t)a * WB;
        const double* fb = pieces + (size_t)(a + 1) * WB;
        const int loa = I.lo[a], lob = I.lo[a + 1], hia = I.hi[a];
        const int ov = hia - lob + 1;
        int d = ov / 8;
        d = d < 1 ? 1 : (d > 10 ? 10 : d);
        int first = lob + 2 * d;
        if (a > 0 && join[a - 1] + 1 > first) first = join[a - 1] + 1;
        double best = __builtin_inf();
        int bestb = -1;
        for (int b = first + tid; b + 2 * d <= hia; b += blockDim.x) {
            const uint8_t* mk = I.mask;
            if (!mk[b] || !mk[b - d] || !mk[b + d] || !mk[b - 2 * d] || !mk[b + 2 * d]) continue;
            const int ia = b - loa, ib = b - lob;
            const double na = ((fa[ia - 2 * d] - 8.0 * fa[ia - d]) + 8.0 * fa[ia + d]) - fa[ia + 2 * d];
            const double nbv = ((fb[ib - 2 * d] - 8.0 * fb[ib - d]) + 8.0 * fb[ib + d]) - fb[ib + 2 * d];
            const double diff = fabs(na / (12.0 * d) - nbv / (12.0 * d));
            if (bestb < 0 || diff < best) {
                best = diff;
                bestb = b;
            }
        }
        rd[tid] = best;
        rb[tid] = bestb;
        __syncthreads();
        for (int st = blockDim.x / 2; st > 0; st >>= 1) {
            if (tid < st) {
                const double d2 = rd[tid + st];
                const int b2 = rb[tid + st];
                if (b2 >= 0 && (rb[tid] < 0 || d2 < rd[tid] || (d2 == rd[tid] && b2 < rb[tid]))) {
                    rd[tid] = d2;
                    rb[tid] = b2;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            const int bs = rb[0];
            if (bs < 0) {                      // no valid join: report, keep indices inside
                *status = -2;
                join[a] = first < lob ? lob : (first > hia ? hia : first);
                shift[a + 1] = shift[a];
            } else {
                join[a] = bs;
                shift[a + 1] = shift[a] + (fa[bs - loa] - fb[bs - lob]);
            }
        }
        __syncthreads();
    }
    // assemble
    double mx = -__builtin_inf();
    for (int b = tid; b < W; b += blockDim.x) {
        int a = 0;
        while (a + 1 < h && b > join[a]) ++a;
        const double v = pieces[(size_t)a * WB + (b - I.lo[a])] + shift[a];
        out[b] = v;
        if (I.mask[b] && v > mx) mx = v;
    }
    rd[tid] = mx;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) rd[tid] = rd[tid + st] > rd[tid] ? rd[tid + st] : rd[tid];
        __syncthreads();
    }
    const double gmax = rd[0];
    __syncthreads();
    double acc = 0.0;
    for (int b = tid; b < W; b += blockDim.x)
        if (I.mask[b]) acc += exp(out[b] - gmax);
    rd[tid] = acc;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) rd[tid] += rd[tid + st];
        __syncthreads();
    }
    const double lse = gmax + log(rd[0]);
    const double target = (double)I.N * log(I.model == 0 ? 2.0 : (double)I.q);
    __syncthreads();
    for (int b = tid; b < W; b += blockDim.x)
        out[b] = I.mask[b] ? out[b] + (target - lse) : -__builtin_inf();
}

// ------------------------------------------------------ predicate probe
// Evaluates the full acceptance predicate (fast test against log(u53 2^-53)
// with the guard band, exact slow path inside it) on caller-given inputs.
__global__ void k_accept_probe(const double* __restrict__ delta, const uint64_t* __restrict__ u53,
                               int n, int32_t* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int f = decide_fast(delta[i], threshold_of(u53[i], kBand), kBand);
        out[i] = f == 2 ? (accept_slow(delta[i], u53[i]) ? 3 : 2) : f;
    }
}

__global__ void k_philox_probe(const uint32_t* __restrict__ in, int n, uint32_t* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint32_t* c = in + 6 * i;
        const u32x4 x = philox10(c[0], c[1], c[2], c[3], c[4], c[5]);
        out[4 * i + 0] = x.x;
        out[4 * i + 1] = x.y;
        out[4 * i + 2] = x.z;
        out[4 * i + 3] = x.w;
    }
}

}  // namespace rewl
