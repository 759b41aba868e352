// Kernels of the n-run error analysis and of the canonical averages:
//   k_boot_mean  the bin-wise mean of n runs' pieces per window, for the
//                ensemble itself and for bootstrap resamples (Sec. II.B)
//   k_thermo     u, c and f per spin from a density of states over a grid of
//                temperatures (the specific-heat analysis of Sec. IV.A)
// The joining of the mean pieces is k_concat, one block per resample.
#pragma once
#include "rewl_device.hpp"

namespace rewl {

enum : uint32_t { kTagBoot = 4 };

// Grid (h, R + 1), 256 threads, n pointers of dynamic LDS.  runs[i] points at
// run i's window tables [h][WB]; mean receives [R + 1][h][WB].  Resample 0
// takes run j for draw j; resample r >= 1 takes run floor(x0 n / 2^32) for
// draw j of window a, x0 the first Philox word at counter (r, j, a, kTagBoot).
// The sum runs in draw order and is then divided by n.
__global__ void __launch_bounds__(256) k_boot_mean(const double* const* __restrict__ runs, int n,
                                                   int h, int WB, uint32_t k0, uint32_t k1,
                                                   double* __restrict__ mean)
{
    extern __shared__ const double* piece[];   // draw j -> the picked run's table of window a
    const int a = blockIdx.x, r = blockIdx.y;
    const size_t off = (size_t)a * WB;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int p = j;
        if (r > 0) {
            const u32x4 x = philox10((uint32_t)r, (uint32_t)j, (uint32_t)a, kTagBoot, k0, k1);
            p = (int)(((uint64_t)x.x * (uint64_t)n) >> 32);
        }
        piece[j] = runs[p] + off;
    }
    __syncthreads();
    double* o = mean + ((size_t)r * h + a) * WB;
    for (int b = threadIdx.x; b < WB; b += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += piece[j][b];
        o[b] = acc / (double)n;
    }
}

// ------------------------------------------------------------------ thermo
// One wave per (row s, tile of kThermoT temperatures).  Pass 1 finds, per
// temperature, the largest exponent x(E) = ln g(E) - E / T and the lowest bin
// where it occurs (energy Em); pass 2 sums w = e^{x - max} (terms below
// e^-745.2 are zero in double precision and are skipped), w (E - Em) and
// w (E - Em)^2.  Then <E> = Em + S1/Z, the variance S2/Z - (S1/Z)^2 (centred
// at the most probable energy, so the difference loses little), and
// ln Z = max + ln sum w.
constexpr int kThermoT = 8;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(64) k_thermo(const double* __restrict__ lng, int W, int model, int N,
                                               const double* __restrict__ T, int nT,
                                               double* __restrict__ u, double* __restrict__ c,
                                               double* __restrict__ f)
{
    const int lane = threadIdx.x, s = blockIdx.y, t0 = blockIdx.x * kThermoT;
    const int nt = nT - t0 < kThermoT ? nT - t0 : kThermoT;
    const double* row = lng + (size_t)s * W;
    const double twoN = 2.0 * N;
    double beta[kThermoT], mx[kThermoT];
    int arg[kThermoT];
#pragma unroll
    for (int i = 0; i < kThermoT; ++i) {
        beta[i] = 1.0 / T[t0 + (i < nt ? i : nt - 1)];
        mx[i] = -__builtin_inf();
        arg[i] = W;
    }
    for (int b = lane; b < W; b += 64) {
        const double v = row[b];
        if (!(v > -__builtin_inf())) continue;
        const double E = model == 0 ? 4.0 * b - twoN : (double)b - twoN;
#pragma unroll
        for (int i = 0; i < kThermoT; ++i) {
            const double x = v - beta[i] * E;
            if (x > mx[i]) {
                mx[i] = x;
                arg[i] = b;
            }
        }
    }
    // wave max with the lowest bin on ties
#pragma unroll
    for (int i = 0; i < kThermoT; ++i) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double m2 = __shfl_xor(mx[i], o, 64);
            const int a2 = __shfl_xor(arg[i], o, 64);
            if (m2 > mx[i] || (m2 == mx[i] && a2 < arg[i])) {
                mx[i] = m2;
                arg[i] = a2;
            }
        }
    }
    double Em[kThermoT], Z[kThermoT], S1[kThermoT], S2[kThermoT];
#pragma unroll
    for (int i = 0; i < kThermoT; ++i) {
        Em[i] = model == 0 ? 4.0 * arg[i] - twoN : (double)arg[i] - twoN;
        Z[i] = S1[i] = S2[i] = 0.0;
    }
    for (int b = lane; b < W; b += 64) {
        const double v = row[b];
        if (!(v > -__builtin_inf())) continue;
        const double E = model == 0 ? 4.0 * b - twoN : (double)b - twoN;
#pragma unroll
        for (int i = 0; i < kThermoT; ++i) {
            const double d = (v - beta[i] * E) - mx[i];
            if (d >= -745.2) {
                const double w = exp(d), e = E - Em[i], we = w * e;
                Z[i] += w;
                S1[i] += we;
                S2[i] += we * e;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kThermoT; ++i) {
        Z[i] = wave_sum(Z[i]);
        S1[i] = wave_sum(S1[i]);
        S2[i] = wave_sum(S2[i]);
    }
    if (lane < nt) {
        double zz = 0, s1 = 0, s2 = 0, em = 0, m = 0;
#pragma unroll
        for (int i = 0; i < kThermoT; ++i)
            if (i == lane) {
                zz = Z[i]; s1 = S1[i]; s2 = S2[i]; em = Em[i]; m = mx[i];
            }
        const double t = T[t0 + lane], mean = s1 / zz;
        const size_t o = (size_t)s * nT + t0 + lane;
        if (u) u[o] = (em + mean) / N;
        if (c) c[o] = (s2 / zz - mean * mean) / ((double)N * t * t);
        if (f) f[o] = -t * (m + log(zz)) / N;
    }
}

}  // namespace rewl
