// rewl_device.hpp -- device-side building blocks of the REWL library (gfx950).
//
// * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
// * Double-double arithmetic and exp, used only for near-tie acceptance decisions.
// * The exact acceptance predicate  u53 < 2^53 * exp(delta)  of the Wang-Landau
//   move (arXiv:1407.5140 Sec. II.A: states are weighted by 1/g(E)) and of the
//   replica exchange, Eq. (1), in its log form.
// * Per-instance descriptors shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

// ---------------------------------------------------------------- Philox
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Stream tags of the counter's fourth word.
enum : uint32_t { kTagFlip = 0, kTagExchange = 1, kTagInit = 2, kTagPartner = 3 };

__device__ __forceinline__ u32x4 draw(uint32_t k0, uint32_t k1, uint64_t T, uint32_t slot,
                                      uint32_t tag)
{
    return philox10((uint32_t)T, (uint32_t)(T >> 32), slot, tag, k0, k1);
}

__device__ __forceinline__ uint64_t u53_of(const u32x4& x)
{
    return ((((uint64_t)x.w) << 32) | x.z) >> 11;
}

// ---------------------------------------------------------- double-double
// Error-free transformations (Dekker / Knuth) and a double-double exp built
// from argument reduction by ln 2 and a Taylor series, accurate to ~2^-100.
// Contraction must stay off here: fusing a rounded product into a following
// add (a*b + c -> fma) destroys the exact error terms these rely on.
#pragma clang fp contract(off)
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b)
{
    double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_div_d(dd a, double b)
{
    double q1 = a.hi / b;
    dd p = two_prod(q1, b);
    dd r = two_sum(a.hi, -p.hi);
    r.lo += a.lo - p.lo;
    double q2 = (r.hi + r.lo) / b;
    return quick_two_sum(q1, q2);
}

// exp(x) for |x| < 700 as a double-double: x = n ln2 + r, |r| <= ln2/2,
// exp(r) = sum_k r^k / k! (27 terms reach 2^-106 at |r| = 0.35), times 2^n.
__device__ inline dd dd_exp(double x)
{
    const dd ln2 = {0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56};
    double n = __builtin_rint(x / ln2.hi);
    dd nl = dd_mul({n, 0.0}, ln2);
    dd r = dd_add({x, 0.0}, {-nl.hi, -nl.lo});
    dd p = {1.0, 0.0};
    for (int k = 27; k >= 1; --k) p = dd_add({1.0, 0.0}, dd_div_d(dd_mul(p, r), (double)k));
    int e = (int)n;
    return {__builtin_ldexp(p.hi, e), __builtin_ldexp(p.lo, e)};
}

// Exact decision of u53 < 2^53 exp(delta) for delta < 0, u53 >= 1, used when
// the fast comparison is inside its guard band.  exp(delta) is irrational for
// rational delta != 0, so there is no tie; the double-double error (~2^-100
// relative) could only matter within 2^-47 of an integer at this scale.
__device__ inline bool accept_slow(double delta, uint64_t u53)
{
    if (delta >= 0.0) return true;
    if (u53 == 0) return true;
    if (delta < -40.0) return false;            // 2^53 e^-40 < 1 <= u53
    dd y = dd_exp(delta);
    y.hi = __builtin_ldexp(y.hi, 53);
    y.lo = __builtin_ldexp(y.lo, 53);
    double u = (double)u53;                      // exact, u53 < 2^53
    double diff = u - y.hi;                      // exact: u and y.hi within a factor 2
    return diff < y.lo;
}

// Guard band of the fast comparison: the device log is within a few ulp
// (|log u| <= 36.8, ulp <= 7.2e-15); 2^-40 leaves a margin above 100 ulp.  A
// handle may widen it (every decision stays exact: only more of them go to the
// slow path), which is how the slow path is exercised under test.
constexpr double kBand = 0x1p-40;

// Threshold of the fast test for a draw u53: vb = log(u53 2^-53) + band, or
// -DBL_MAX for u53 = 0 (every finite delta accepts, an out-of-window move with
// delta = -inf does not).  accept  <=>  delta > log(u53 2^-53)  exactly; the
// fast test decides whenever delta is outside [vb - 2 band, vb].
__device__ __forceinline__ double threshold_of(uint64_t u53, double band)
{
    return u53 == 0 ? -0x1.fffffffffffffp+1023 : log(__builtin_ldexp((double)u53, -53)) + band;
}

// 1 accept, 0 reject, 2 undecided (decide with accept_slow).
__device__ __forceinline__ int decide_fast(double delta, double vb, double band)
{
    return delta > vb ? 1 : (delta >= vb - 2.0 * band ? 2 : 0);
}

// ---------------------------------------------------------- descriptors
enum : int32_t { kErrOverflow = 1, kErrInitStuck = 2, kErrExactness = 4 };

// Device counters of one instance (one cache line each would be overkill).
struct InstCtr {
    int64_t t;          // completed intervals
    int64_t slow;       // acceptance decisions taken by the exact slow path
    int32_t all_done;   // every window converged
    int32_t stopped;    // the interval that finished the run has been counted
    int32_t n_done;     // converged windows
    int32_t err;        // sticky error flags
    int32_t queue;      // sweep tile queue head
    int32_t pad;
};

struct Inst {
    // problem
    int32_t model, q, L, N, W, h, m, S, WB, log2m;
    int32_t flat_num, flat_den, kfinal, exch, wpr, flat_rule;
    int64_t X;
    int64_t XP;         // row stride of the draw buffers: X rounded up to 32
    uint32_t k0, k1;
    // device arrays
    uint64_t* lat;      // Ising: [S][L*wpr] words, bit x of row y's word = spin up
    uint8_t* plat;      // Potts: [S][N] bytes
    int32_t* bin;       // [S]   global energy bin of the slot's configuration
    uint64_t* H;        // [S][WB] (slot = a*m + r): walker-major counts since the
                        //         window's last merge
    double* base;       // [h][WB] window ln g base: ln g_w = base + 2^-k H_w
    int32_t* lo;        // [h]
    int32_t* hi;        // [h]
    int32_t* nreach;    // [h]   occurring levels inside the window
    uint8_t* mask;      // [W]
    int32_t* k;         // [h]   ln f = 2^-k
    int32_t* done;      // [h]
    uint8_t* flat;      // [S]   latched flatness
    int8_t* swaps;      // [S]   last interval: 1 swapped, 0 rejected, -1 none
    uint32_t* rpack;    // [S][XP] Ising: row | col<<8 | row_up<<16 | row_down<<24;
                        //         Potts: row | col<<8 | proposal offset<<16
    double* rv;         // [S][XP] threshold log(u53 2^-53) + band
    int64_t* ex_prop;   // [h]
    int64_t* ex_acc;    // [h]
    int32_t* merges;    // [h] interval of each window's last merge
    int32_t* rid;       // [S] replica (configuration) held by each slot
    int8_t* rt_state;   // [S] per replica: 0 not yet in window 0, 1 in or last at
                        //     window 0, 2 reached window h-1 since
    int32_t* rt_count;  // [S] per replica: completed round trips 0 -> h-1 -> 0
    double band;        // guard band of the fast acceptance test
    int32_t hglobal;    // wave sweep: counts read from device memory, not an LDS copy
    int32_t mapn;       // wave sweep: site-map entries per walker (N, or a power of two below N)
    InstCtr* ctr;
};

// Flatness of one walker from the minimum and sum of its counts over the n
// levels of its window that occur.  Rule 0 (Sec. II.A): min >= num/den of the
// mean, decided as den min n >= num sum.  Rule 1 (Eq. (8)): min >= (num/den) /
// sqrt(ln f), ln f = 2^-k, decided as (min den)^2 >= num^2 2^k.  Both exactly
// in 128-bit integers (num, den <= 2^31, n <= 2^17, k <= 40).
__device__ __forceinline__ bool walker_flat(const Inst& I, uint64_t mn, uint64_t sum, int64_t n, int k)
{
    typedef unsigned __int128 u128;
    if (I.flat_rule == 1) {
        const u128 x = (u128)mn * (uint64_t)I.flat_den;                 // < 2^84
        const u128 rhs = (u128)((uint64_t)I.flat_num * (uint64_t)I.flat_num) << k;  // < 2^81
        if (x >= ((u128)1 << 41)) return true;                          // x^2 >= 2^82 > rhs
        return x * x >= rhs;
    }
    return (u128)mn * (uint64_t)I.flat_den * (uint64_t)n >= (u128)sum * (uint64_t)I.flat_num;
}

// 64-bit lane exchange through two 32-bit shuffles.
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask);
    return ((uint64_t)hi << 32) | lo;
}

// A sweep tile: nw consecutive walkers of one window of one instance.
struct Tile {
    int32_t inst, window, r0, nw;
};

}  // namespace rewl
