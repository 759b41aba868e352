// mlp.hip -- a small MLP that learns ln g(E)/N, trained and evaluated on gfx950.
//
// Network: x = (E/N, 1/L, q) -> `layers` hidden layers of width H with the erf
// GELU -> one linear output (ln g / N).  Weights are kept in FP32 (master copy,
// Adam moments) and in BF16 for the matrix cores; every H x H product is a
// BF16 MFMA GEMM (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.  The first
// layer (K = 3) and the output layer (N = 1) are plain FP32 kernels.
//
// Flat parameter order: W1[in][H], b1[H], then for each further hidden layer
// W[H][H], b[H], then w_out[H], b_out[1] (row-major, W[i][j]: input i -> unit j).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rewl_mlp.h"

namespace {

thread_local std::string g_mlp_err;

rewl_status mfail(rewl_status s, const std::string& m)
{
    g_mlp_err = m;
    return s;
}

#define MLP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return mfail(REWL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu(float a)
{
    return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float a)
{
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) +
           a * 0.39894228040143268f * expf(-0.5f * a * a);
}

// ---------------------------------------------------------------- GEMM
// C = op(A) op(B) on the matrix cores: A(i,k) = A[i*lda + k] (ta = 0) or
// A[k*lda + i] (ta = 1); B(k,j) = B[k*ldb + j] (tb = 0) or B[j*ldb + k] (tb = 1);
// BF16 operands, FP32 accumulation.  A block of 4 waves computes a 64 x 64 tile
// of C, one 32 x 32 quarter per wave, with K staged through LDS 32 at a time:
// A as [i][k] and B as [j][k], so that each lane's 8 consecutive k are one
// 16-byte read.  M and N are multiples of 64, K / gridDim.z a multiple of 32.
// With gridDim.z > 1 (split K; plain stores only) split z writes its FP32 partial
// product to C + z*M*N and k_splitk_sum adds the splits in order.
// Operand layout of v_mfma_f32_32x32x16_bf16: lane l supplies A row l%32 and B
// column l%32 with k = 8*(l/32) .. +7; its 16 accumulators hold
// C(8*(r/4) + 4*(l/32) + r%4, l%32), r = 0..15.
enum Epi : int {
    kEpiStore = 0,        // C = acc (FP32)
    kEpiBiasGelu = 1,     // pre = acc + bias[j] (FP32 out), act = gelu(pre) (BF16 out)
    kEpiGeluGrad = 2,     // d = acc * gelu'(pre) (FP32 and BF16 out)
};
constexpr int kBM = 64, kBN = 64, kBK = 32, kLdsRow = kBK + 8;   // +8: spread the banks

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm(const __bf16* __restrict__ A, int lda, int ta,
                                              const __bf16* __restrict__ B, int ldb, int tb,
                                              int M, int N, int K, int epi,
                                              float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias,
                                              const float* __restrict__ pre,
                                              __bf16* __restrict__ out16)
{
    __shared__ __align__(16) __bf16 As[kBM * kLdsRow];
    __shared__ __align__(16) __bf16 Bs[kBN * kLdsRow];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int i0 = blockIdx.y * kBM, j0 = blockIdx.x * kBN;
    const int kspan = K / (int)gridDim.z, kbeg = (int)blockIdx.z * kspan, kend = kbeg + kspan;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int li = lane & 31, kg = (lane >> 5) * 8;
    f32x16 acc = {};
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        // stage: every thread moves 8 consecutive elements of A and of B
        if (ta == 0) {
            const int r = t >> 2, c = (t & 3) * 8;
            *(u32x4*)&As[r * kLdsRow + c] = *(const u32x4*)&A[(size_t)(i0 + r) * lda + k0 + c];
        } else {
            const int kk = t >> 3, c = (t & 7) * 8;
            u32x4 v = *(const u32x4*)&A[(size_t)(k0 + kk) * lda + i0 + c];
            const __bf16* e = (const __bf16*)&v;
#pragma unroll
            for (int u = 0; u < 8; ++u) As[(c + u) * kLdsRow + kk] = e[u];
        }
        if (tb == 1) {
            const int r = t >> 2, c = (t & 3) * 8;
            *(u32x4*)&Bs[r * kLdsRow + c] = *(const u32x4*)&B[(size_t)(j0 + r) * ldb + k0 + c];
        } else {
            const int kk = t >> 3, c = (t & 7) * 8;
            u32x4 v = *(const u32x4*)&B[(size_t)(k0 + kk) * ldb + j0 + c];
            const __bf16* e = (const __bf16*)&v;
#pragma unroll
            for (int u = 0; u < 8; ++u) Bs[(c + u) * kLdsRow + kk] = e[u];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 16) {
            const bf16x8 av = *(const bf16x8*)&As[(wi + li) * kLdsRow + ks + kg];
            const bf16x8 bv = *(const bf16x8*)&Bs[(wj + li) * kLdsRow + ks + kg];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = j0 + wj + li;
        const float v = acc[r];
        if (gridDim.z > 1) {
            C[(size_t)blockIdx.z * M * N + (size_t)i * N + j] = v;
            continue;
        }
        const size_t o = (size_t)i * ldc + j;
        if (epi == kEpiStore) {
            C[o] = v;
        } else if (epi == kEpiBiasGelu) {
            const float p = v + bias[j];
            C[o] = p;
            out16[o] = (__bf16)gelu(p);
        } else {
            const float d = v * gelu_grad(pre[o]);
            C[o] = d;
            out16[o] = (__bf16)d;
        }
    }
}

// out[e] = sum over splits z (in order) of part[z*n + e]
__global__ void k_splitk_sum(const float* __restrict__ part, int S, int n, float* __restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(size_t)z * n + e];
    out[e] = s;
}

// Weighted column sums over the batch, in two passes with a fixed order:
// part[z][k][j] = sum over rows r of chunk z of w_k(r) Mx[r][j], where w_k(r) =
// W[r*ldw + k] for k < nw and 1 for k = nw when `ones`; then k_colsum_final adds
// the chunks.  Gradients of the output layer, of the biases and of the first layer.
constexpr int kColK = 17;   // nw + ones <= in_dim + 1 <= 17
template <class T>
__global__ void k_colsum_part(const T* __restrict__ Mx, int ldm, int Bn, int H,
                              const float* __restrict__ W, int ldw, int nw, int ones, int rows,
                              float* __restrict__ part)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, z = blockIdx.y;
    if (j >= H) return;
    const int K = nw + ones, r0 = z * rows, r1 = r0 + rows < Bn ? r0 + rows : Bn;
    float acc[kColK];
#pragma unroll
    for (int k = 0; k < kColK; ++k) acc[k] = 0.f;
    for (int r = r0; r < r1; ++r) {
        const float v = (float)Mx[(size_t)r * ldm + j];
#pragma unroll
        for (int k = 0; k < kColK; ++k)
            if (k < nw) acc[k] += W[(size_t)r * ldw + k] * v;
        if (ones) {
#pragma unroll
            for (int k = 0; k < kColK; ++k)
                if (k == nw) acc[k] += v;
        }
    }
#pragma unroll
    for (int k = 0; k < kColK; ++k)
        if (k < K) part[((size_t)z * K + k) * H + j] = acc[k];
}

// out[e] = sum over chunks z of part[z*KH + e]: 16 threads per output, each over
// every 16th chunk, then the 16 sums added pairwise in a fixed order (deterministic)
__global__ void __launch_bounds__(256) k_colsum_final(const float* __restrict__ part, int Z, int KH,
                                                      float* __restrict__ out)
{
    __shared__ float red[16][17];
    const int t = threadIdx.x, c = t & 15, g = t >> 4;
    const int e = blockIdx.x * 16 + c;
    float s = 0.f;
    if (e < KH)
        for (int z = g; z < Z; z += 16) s += part[(size_t)z * KH + e];
    red[g][c] = s;
    __syncthreads();
    for (int w = 8; w > 0; w >>= 1) {
        if (g < w) red[g][c] += red[g + w][c];
        __syncthreads();
    }
    if (g == 0 && e < KH) out[e] = red[0][c];
}

// first layer: pre = x W1 + b1 (K = in_dim), act = gelu(pre) in BF16
__global__ void k_layer_in(const float* __restrict__ x, int in_dim, const float* __restrict__ W,
                           const float* __restrict__ b, int H, int B, float* __restrict__ pre,
                           __bf16* __restrict__ act)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * H) return;
    const int r = idx / H, j = idx - r * H;
    float s = b[j];
    for (int i = 0; i < in_dim; ++i) s += x[r * in_dim + i] * W[i * H + j];
    pre[idx] = s;
    act[idx] = (__bf16)gelu(s);
}

// output layer y = act . w + b0 (FP32), one wave per row, fixed reduction order
__global__ void __launch_bounds__(256) k_layer_out(const __bf16* __restrict__ act,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ b0, int H, int B,
                                                   float* __restrict__ y)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= B) return;
    float s = 0.f;
    for (int j = lane; j < H; j += 64) s += (float)act[(size_t)row * H + j] * w[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) y[row] = s + b0[0];
}

// loss pieces: dy = 2 (y - t) / B for rows < nvalid, 0 for padding; loss sum
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ t, int B, int nvalid,
                       float* __restrict__ dy, float* __restrict__ loss)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    float d = 0.f;
    if (r < nvalid) {
        d = y[r] - t[r];
        atomicAdd(loss, d * d / (float)nvalid);
        d = 2.f * d / (float)nvalid;
    }
    dy[r] = d;
}

// back through the output layer: d_pre = dy[r] w[j] gelu'(pre), grads of w_out, b_out
__global__ void k_back_out(const float* __restrict__ dy, const float* __restrict__ w,
                           const float* __restrict__ pre, int H, int B, float* __restrict__ dpre,
                           __bf16* __restrict__ dpre16)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * H) return;
    const int r = idx / H, j = idx - r * H;
    const float d = dy[r] * w[j] * gelu_grad(pre[idx]);
    dpre[idx] = d;
    dpre16[idx] = (__bf16)d;
}

// Adam (Kingma & Ba) on the FP32 master weights, BF16 copies refreshed
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, __bf16* __restrict__ p16, const int* __restrict__ map16)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    const int o = map16[i];
    if (o >= 0) p16[o] = (__bf16)pi;
}

__global__ void k_to_bf16(const float* __restrict__ a, __bf16* __restrict__ b, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (__bf16)a[i];
}

// gather a minibatch: rows idx = floor(u * n) from a counter-based hash
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ Y, int in_dim,
                         int n, int B, uint64_t step, uint32_t seed, float* __restrict__ xb,
                         float* __restrict__ yb)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    // splitmix64 of (seed, step, r): any fixed hash serves, only the sample order depends on it
    uint64_t z = ((uint64_t)seed << 32) ^ (step * 0x9E3779B97F4A7C15ull) ^ (uint64_t)r * 0xD1B54A32D192ED03ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int k = (int)(((z >> 32) * (uint64_t)n) >> 32);
    for (int i = 0; i < in_dim; ++i) xb[r * in_dim + i] = X[(size_t)k * in_dim + i];
    yb[r] = Y[k];
}

}  // namespace

struct mlp_handle {
    mlp_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int H = 0, nl = 0, P = 0, Bmax = 0;
    std::vector<int> off_W, off_b;     // offsets into the flat parameter vector
    int off_wout = 0, off_bout = 0, n16 = 0;
    std::vector<int> off16;            // BF16 copy offsets of the H x H matrices
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    __bf16* p16 = nullptr;
    int* map16 = nullptr;
    std::vector<float*> pre;           // [nl] B x H pre-activations (FP32)
    std::vector<__bf16*> act;          // [nl] B x H activations (BF16)
    float *dpre = nullptr, *dtmp = nullptr, *y = nullptr, *dy = nullptr, *loss = nullptr;
    __bf16 *d16a = nullptr, *d16b = nullptr;
    float *xb = nullptr, *yb = nullptr;
    float* kpart = nullptr;            // split-K partial products [Smax][H][H]
    int Smax = 1;
    float* cpart = nullptr;            // column-sum partials [Zmax][kColK][H]
    int crow = 64;                     // rows per column-sum chunk
    float *dx = nullptr, *dt = nullptr;   // training rows of the last mlp_fit call
    int64_t data_cap = 0;
    int64_t steps = 0;
    std::vector<void*> allocs;
    template <class T>
    rewl_status alloc(T** q, size_t n)
    {
        void* r = nullptr;
        if (hipMalloc(&r, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
            return mfail(REWL_E_NOMEM, "hipMalloc failed");
        allocs.push_back(r);
        *q = (T*)r;
        return REWL_OK;
    }
};

namespace {

inline dim3 grid1(int n, int b = 256) { return dim3((n + b - 1) / b); }

// C = op(A) op(B) with the handle's split-K buffer when K is long
void gemm(mlp_handle* h, const __bf16* A, int lda, int ta, const __bf16* B, int ldb, int tb, int M, int N,
          int K, int epi, float* C, int ldc, const float* bias, const float* pre, __bf16* out16)
{
    int S = 1;
    if (epi == kEpiStore && M * N <= h->H * h->H)
        while (S < h->Smax && K % (2 * S * kBK) == 0 && K / (2 * S) >= 256) S *= 2;
    hipLaunchKernelGGL(k_gemm, dim3(N / kBN, M / kBM, S), dim3(256), 0, h->stream, A, lda, ta, B, ldb, tb,
                       M, N, K, epi, S > 1 ? h->kpart : C, ldc, bias, pre, out16);
    if (S > 1)
        hipLaunchKernelGGL(k_splitk_sum, grid1(M * N), dim3(256), 0, h->stream, h->kpart, S, M * N, C);
}

// out[k][j] = sum_r w_k(r) Mx[r][j] over B rows (see k_colsum_part)
template <class T>
void colsum(mlp_handle* h, const T* Mx, int ldm, int B, int H, const float* W, int ldw, int nw, int ones,
            float* out)
{
    const int Z = (B + h->crow - 1) / h->crow, K = nw + ones;
    hipLaunchKernelGGL(k_colsum_part<T>, dim3((H + 63) / 64, Z), dim3(64), 0, h->stream, Mx, ldm, B, H, W, ldw,
                       nw, ones, h->crow, h->cpart);
    hipLaunchKernelGGL(k_colsum_final, dim3((K * H + 15) / 16), dim3(256), 0, h->stream, h->cpart, Z, K * H, out);
}

// forward pass of B rows (B a multiple of 64) already in xb; y written
void forward(mlp_handle* h, const float* x, int B)
{
    const int H = h->H;
    hipLaunchKernelGGL(k_layer_in, grid1(B * H), dim3(256), 0, h->stream, x, h->cfg.in_dim,
                       h->p + h->off_W[0], h->p + h->off_b[0], H, B, h->pre[0], h->act[0]);
    for (int l = 1; l < h->nl; ++l)
        gemm(h, h->act[l - 1], H, 0, h->p16 + h->off16[l], H, 0, B, H, H, kEpiBiasGelu, h->pre[l], H,
             h->p + h->off_b[l], nullptr, h->act[l]);
    hipLaunchKernelGGL(k_layer_out, dim3((B + 3) / 4), dim3(256), 0, h->stream, h->act[h->nl - 1],
                       h->p + h->off_wout, h->p + h->off_bout, H, B, h->y);
}

// backward after forward(); gradients into h->g (loss value in h->loss)
void backward(mlp_handle* h, const float* x, const float* t, int B, int nvalid)
{
    const int H = h->H, nl = h->nl;
    (void)hipMemsetAsync(h->loss, 0, sizeof(float), h->stream);
    hipLaunchKernelGGL(k_loss, grid1(B), dim3(256), 0, h->stream, h->y, t, B, nvalid, h->dy, h->loss);
    // output layer: w_out gradient = act^T dy, b_out gradient = sum dy
    colsum(h, h->act[nl - 1], H, B, H, h->dy, 1, 1, 0, h->g + h->off_wout);
    colsum(h, h->dy, 1, B, 1, (const float*)nullptr, 0, 0, 1, h->g + h->off_bout);
    hipLaunchKernelGGL(k_back_out, grid1(B * H), dim3(256), 0, h->stream, h->dy, h->p + h->off_wout,
                       h->pre[nl - 1], H, B, h->dpre, h->d16a);
    __bf16* dcur = h->d16a;
    __bf16* dnext = h->d16b;
    for (int l = nl - 1; l >= 1; --l) {
        // dW_l = act_{l-1}^T d_l  (K = B), db_l = column sums of d_l
        gemm(h, h->act[l - 1], H, 1, dcur, H, 0, H, H, B, kEpiStore, h->g + h->off_W[l], H, nullptr, nullptr,
             nullptr);
        colsum(h, h->dpre, H, B, H, (const float*)nullptr, 0, 0, 1, h->g + h->off_b[l]);
        // d_{l-1} = (d_l W_l^T) * gelu'(pre_{l-1})
        gemm(h, dcur, H, 0, h->p16 + h->off16[l], H, 1, B, H, H, kEpiGeluGrad, h->dtmp, H, nullptr,
             h->pre[l - 1], dnext);
        std::swap(h->dpre, h->dtmp);
        std::swap(dcur, dnext);
    }
    // first layer: W1 gradient rows = x_i^T d_0, then b1 = column sums (contiguous in g)
    colsum(h, h->dpre, H, B, H, x, h->cfg.in_dim, h->cfg.in_dim, 1, h->g + h->off_W[0]);
}

}  // namespace

extern "C" {

const char* mlp_last_error(void) { return g_mlp_err.c_str(); }

void mlp_destroy(mlp_handle* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void* q : h->allocs) (void)hipFree(q);
    if (h->dx) (void)hipFree(h->dx);
    if (h->dt) (void)hipFree(h->dt);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

rewl_status mlp_create(const mlp_config* c, void* hip_stream, mlp_handle** out)
{
    if (!c || !out) return mfail(REWL_E_INVALID, "null argument");
    *out = nullptr;
    if (c->in_dim < 1 || c->in_dim > 16 || c->hidden < 64 || c->hidden % 64 || c->hidden > 4096 ||
        c->layers < 1 || c->layers > 16 || c->max_batch < 1 || c->max_batch > (1 << 20))
        return mfail(REWL_E_INVALID, "need 1<=in_dim<=16, hidden a multiple of 64 up to 4096, 1<=layers<=16, "
                                     "1<=max_batch<=2^20");
    mlp_handle* h = new mlp_handle();
    h->cfg = *c;
    h->H = c->hidden;
    h->nl = c->layers;
    h->Bmax = (c->max_batch + 63) / 64 * 64;
    const int H = h->H;
    int off = 0;
    h->off_W.push_back(off);
    off += c->in_dim * H;
    h->off_b.push_back(off);
    off += H;
    h->off16.push_back(-1);
    for (int l = 1; l < h->nl; ++l) {
        h->off_W.push_back(off);
        h->off16.push_back(h->n16);
        h->n16 += H * H;
        off += H * H;
        h->off_b.push_back(off);
        off += H;
    }
    h->off_wout = off;
    off += H;
    h->off_bout = off;
    off += 1;
    h->P = off;
    auto bail = [&](rewl_status s) {
        mlp_destroy(h);
        return s;
    };
    if (hip_stream) h->stream = (hipStream_t)hip_stream;
    else {
        if (hipStreamCreate(&h->stream) != hipSuccess) return bail(mfail(REWL_E_DEVICE, "hipStreamCreate"));
        h->own_stream = true;
    }
    rewl_status s = REWL_OK;
    const size_t BH = (size_t)h->Bmax * H;
    if (s == REWL_OK) s = h->alloc(&h->p, h->P);
    if (s == REWL_OK) s = h->alloc(&h->g, h->P);
    if (s == REWL_OK) s = h->alloc(&h->m, h->P);
    if (s == REWL_OK) s = h->alloc(&h->v, h->P);
    if (s == REWL_OK) s = h->alloc(&h->p16, h->n16);
    if (s == REWL_OK) s = h->alloc(&h->map16, h->P);
    h->pre.assign(h->nl, nullptr);
    h->act.assign(h->nl, nullptr);
    for (int l = 0; l < h->nl && s == REWL_OK; ++l) {
        s = h->alloc(&h->pre[l], BH);
        if (s == REWL_OK) s = h->alloc(&h->act[l], BH);
    }
    if (s == REWL_OK) s = h->alloc(&h->dpre, BH);
    if (s == REWL_OK) s = h->alloc(&h->dtmp, BH);
    if (s == REWL_OK) s = h->alloc(&h->d16a, BH);
    if (s == REWL_OK) s = h->alloc(&h->d16b, BH);
    if (s == REWL_OK) s = h->alloc(&h->y, h->Bmax);
    if (s == REWL_OK) s = h->alloc(&h->dy, h->Bmax);
    if (s == REWL_OK) s = h->alloc(&h->loss, 1);
    if (s == REWL_OK) s = h->alloc(&h->xb, (size_t)h->Bmax * c->in_dim);
    if (s == REWL_OK) s = h->alloc(&h->yb, h->Bmax);
    // split-K partials: at most 16 splits and 64 MiB
    while (h->Smax < 16 && (size_t)2 * h->Smax * H * H * 4 <= ((size_t)64 << 20)) h->Smax *= 2;
    if (s == REWL_OK && h->Smax > 1) s = h->alloc(&h->kpart, (size_t)h->Smax * H * H);
    h->crow = std::max(16, h->Bmax / 1024);
    if (s == REWL_OK) s = h->alloc(&h->cpart, (size_t)((h->Bmax + h->crow - 1) / h->crow) * kColK * H);
    if (s != REWL_OK) return bail(s);
    // initial weights: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a fixed hash, biases 0
    std::vector<float> p0(h->P, 0.f);
    std::vector<int> map(h->P, -1);
    uint64_t z = c->seed * 0x9E3779B97F4A7C15ull + 1;
    auto uni = [&]() {
        z += 0x9E3779B97F4A7C15ull;
        uint64_t r = z;
        r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
        r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
        r ^= r >> 31;
        return (float)((r >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;
    };
    for (int i = 0; i < c->in_dim * H; ++i) p0[i] = uni() / std::sqrt((float)c->in_dim);
    for (int l = 1; l < h->nl; ++l)
        for (int i = 0; i < H * H; ++i) {
            p0[h->off_W[l] + i] = uni() / std::sqrt((float)H);
            map[h->off_W[l] + i] = h->off16[l] + i;
        }
    for (int j = 0; j < H; ++j) p0[h->off_wout + j] = uni() / std::sqrt((float)H);
    if (hipMemcpy(h->p, p0.data(), h->P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->map16, map.data(), h->P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->m, 0, h->P * 4) != hipSuccess || hipMemset(h->v, 0, h->P * 4) != hipSuccess)
        return bail(mfail(REWL_E_DEVICE, "initial upload failed"));
    for (int l = 1; l < h->nl; ++l)
        hipLaunchKernelGGL(k_to_bf16, grid1(H * H), dim3(256), 0, h->stream, h->p + h->off_W[l],
                           h->p16 + h->off16[l], H * H);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(mfail(REWL_E_DEVICE, "init failed"));
    *out = h;
    return REWL_OK;
}

rewl_status mlp_n_params(const mlp_handle* h, int64_t* n)
{
    if (!h || !n) return mfail(REWL_E_INVALID, "null argument");
    *n = h->P;
    return REWL_OK;
}

rewl_status mlp_get_params(const mlp_handle* h, float* host, size_t n)
{
    if (!h || !host || n != (size_t)h->P) return mfail(REWL_E_INVALID, "need n = parameter count");
    MLP_TRY(hipMemcpyAsync(host, h->p, n * 4, hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return REWL_OK;
}

rewl_status mlp_set_params(mlp_handle* h, const float* host, size_t n)
{
    if (!h || !host || n != (size_t)h->P) return mfail(REWL_E_INVALID, "need n = parameter count");
    MLP_TRY(hipMemcpyAsync(h->p, host, n * 4, hipMemcpyHostToDevice, h->stream));
    for (int l = 1; l < h->nl; ++l)
        hipLaunchKernelGGL(k_to_bf16, grid1(h->H * h->H), dim3(256), 0, h->stream, h->p + h->off_W[l],
                           h->p16 + h->off16[l], h->H * h->H);
    MLP_TRY(hipStreamSynchronize(h->stream));
    return REWL_OK;
}

// Forward over host rows x[B][in_dim] -> y[B], in chunks of max_batch rows.
rewl_status mlp_infer(mlp_handle* h, const float* x, float* y, int32_t B)
{
    if (!h || (B > 0 && (!x || !y)) || B < 0) return mfail(REWL_E_INVALID, "bad arguments");
    const int in = h->cfg.in_dim;
    for (int r0 = 0; r0 < B; r0 += h->Bmax) {
        const int nb = std::min(h->Bmax, B - r0);
        const int Bp = (nb + 63) / 64 * 64;
        MLP_TRY(hipMemsetAsync(h->xb, 0, (size_t)Bp * in * 4, h->stream));
        MLP_TRY(hipMemcpyAsync(h->xb, x + (size_t)r0 * in, (size_t)nb * in * 4, hipMemcpyHostToDevice, h->stream));
        forward(h, h->xb, Bp);
        MLP_TRY(hipMemcpyAsync(y + r0, h->y, nb * 4, hipMemcpyDeviceToHost, h->stream));
        MLP_TRY(hipStreamSynchronize(h->stream));
    }
    MLP_TRY(hipGetLastError());
    return REWL_OK;
}

// Loss and gradient of the flat parameter vector on host rows.
rewl_status mlp_grad(mlp_handle* h, const float* x, const float* t, int32_t B, float* grad_host, float* loss)
{
    if (!h || !x || !t || B < 1 || B > h->Bmax) return mfail(REWL_E_INVALID, "need 1 <= B <= max_batch");
    const int in = h->cfg.in_dim, Bp = (B + 63) / 64 * 64;
    MLP_TRY(hipMemsetAsync(h->xb, 0, (size_t)Bp * in * 4, h->stream));
    MLP_TRY(hipMemsetAsync(h->yb, 0, (size_t)Bp * 4, h->stream));
    MLP_TRY(hipMemcpyAsync(h->xb, x, (size_t)B * in * 4, hipMemcpyHostToDevice, h->stream));
    MLP_TRY(hipMemcpyAsync(h->yb, t, (size_t)B * 4, hipMemcpyHostToDevice, h->stream));
    forward(h, h->xb, Bp);
    backward(h, h->xb, h->yb, Bp, B);
    MLP_TRY(hipGetLastError());
    if (grad_host) MLP_TRY(hipMemcpyAsync(grad_host, h->g, h->P * 4, hipMemcpyDeviceToHost, h->stream));
    if (loss) MLP_TRY(hipMemcpyAsync(loss, h->loss, 4, hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return REWL_OK;
}

// `steps` Adam steps on minibatches of B rows sampled from n host rows (the
// rows are uploaded once per call into a device buffer the handle keeps).
rewl_status mlp_fit(mlp_handle* h, const float* x, const float* t, int64_t n, int32_t B, int64_t steps,
                    float lr, uint32_t seed, float* last_loss)
{
    if (!h || !x || !t || n < 1 || n > INT32_MAX || B < 64 || B > h->Bmax || B % 64 || steps < 0)
        return mfail(REWL_E_INVALID, "need 1 <= n < 2^31 rows, B a multiple of 64 in [64, max_batch]");
    const int in = h->cfg.in_dim;
    if (n > h->data_cap) {
        if (h->dx) (void)hipFree(h->dx);
        if (h->dt) (void)hipFree(h->dt);
        h->dx = h->dt = nullptr;
        h->data_cap = 0;
        MLP_TRY(hipMalloc(&h->dx, (size_t)n * in * 4));
        MLP_TRY(hipMalloc(&h->dt, (size_t)n * 4));
        h->data_cap = n;
    }
    MLP_TRY(hipMemcpyAsync(h->dx, x, (size_t)n * in * 4, hipMemcpyHostToDevice, h->stream));
    MLP_TRY(hipMemcpyAsync(h->dt, t, (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t s = 0; s < steps; ++s) {
        hipLaunchKernelGGL(k_gather, grid1(B), dim3(256), 0, h->stream, h->dx, h->dt, in, (int)n, B,
                           (uint64_t)h->steps, seed, h->xb, h->yb);
        forward(h, h->xb, B);
        backward(h, h->xb, h->yb, B, B);
        h->steps += 1;
        const float c1 = 1.f - std::pow(b1, (float)h->steps), c2 = 1.f - std::pow(b2, (float)h->steps);
        hipLaunchKernelGGL(k_adam, grid1(h->P), dim3(256), 0, h->stream, h->p, h->g, h->m, h->v, h->P,
                           lr, b1, b2, eps, c1, c2, h->p16, h->map16);
    }
    MLP_TRY(hipGetLastError());
    if (last_loss) MLP_TRY(hipMemcpyAsync(last_loss, h->loss, 4, hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return REWL_OK;
}

// Warm-start table for a model: ln g(E) = N * net(E/N, 1/L, q) at every bin,
// rounded to a multiple of 2^-16 (keeps the REWL arithmetic exact).
rewl_status mlp_warm_table(mlp_handle* h, int32_t model, int32_t q, int32_t L, double* lng_host)
{
    if (!h || !lng_host || L < 2 || L > 4096 || (model != 0 && model != 1))
        return mfail(REWL_E_INVALID, "bad arguments");
    if (h->cfg.in_dim != 3) return mfail(REWL_E_INVALID, "warm tables need in_dim = 3");
    const int N = L * L, W = model == 0 ? N + 1 : 2 * N + 1;
    std::vector<float> xh((size_t)W * 3), yh(W);
    for (int b = 0; b < W; ++b) {
        const double E = model == 0 ? 4.0 * b - 2.0 * N : (double)b - 2.0 * N;
        xh[3 * b + 0] = (float)(E / N);
        xh[3 * b + 1] = (float)(1.0 / L);
        xh[3 * b + 2] = (float)(model == 0 ? 2 : q);
    }
    rewl_status s = mlp_infer(h, xh.data(), yh.data(), W);
    if (s != REWL_OK) return s;
    for (int b = 0; b < W; ++b) lng_host[b] = std::nearbyint((double)yh[b] * N * 65536.0) / 65536.0;
    return REWL_OK;
}

// Diagnostic: the BF16 MFMA GEMM on host data, C = A B (A: M x K, B: K x N).
rewl_status mlp_probe_gemm(const float* A, const float* B, int32_t M, int32_t N, int32_t K, float* C)
{
    if (!A || !B || !C || M < 64 || N < 64 || K < 32 || M % 64 || N % 64 || K % 32)
        return mfail(REWL_E_INVALID, "M, N multiples of 64, K of 32");
    std::vector<__bf16> a16((size_t)M * K), b16((size_t)K * N);
    for (size_t i = 0; i < a16.size(); ++i) a16[i] = (__bf16)A[i];
    for (size_t i = 0; i < b16.size(); ++i) b16[i] = (__bf16)B[i];
    __bf16 *da = nullptr, *db = nullptr;
    float* dc = nullptr;
    MLP_TRY(hipMalloc(&da, a16.size() * 2));
    MLP_TRY(hipMalloc(&db, b16.size() * 2));
    MLP_TRY(hipMalloc(&dc, (size_t)M * N * 4));
    hipError_t e = hipMemcpy(da, a16.data(), a16.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(db, b16.data(), b16.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gemm, dim3(N / kBN, M / kBM, 1), dim3(256), 0, 0, da, K, 0, db, N, 0, M, N, K,
                           (int)kEpiStore, dc, N, (const float*)nullptr, (const float*)nullptr,
                           (__bf16*)nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(C, dc, (size_t)M * N * 4, hipMemcpyDeviceToHost);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dc);
    if (e != hipSuccess) return mfail(REWL_E_DEVICE, hipGetErrorString(e));
    return REWL_OK;
}

}  // extern "C"
