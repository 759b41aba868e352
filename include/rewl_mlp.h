/*
 * rewl_mlp.h -- C ABI of the density-of-states network in librewl.so.
 *
 * A multilayer perceptron learns s = ln g(E) / N as a function of
 * x = (E/N, 1/L, q) from densities of states that REWL (Sec. II) produced for
 * smaller systems, and supplies the starting ln g of a larger run, which then
 * begins its ln f schedule at 2^-k0 with k0 > 0 instead of ln f = 1 (the
 * schedule of Sec. II.A).  Plain flat-start REWL stays available unchanged.
 *
 * Network: in_dim inputs -> `layers` hidden layers of `hidden` units with the
 * erf form of GELU, a(z) = z * (1 + erf(z / sqrt 2)) / 2 -> one linear output.
 * Loss: mean squared error over the rows of a batch.  Optimiser: Adam
 * (Kingma & Ba, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments).
 *
 * Precision: master weights, Adam moments, biases, the first and the output
 * layer in FP32; every hidden x hidden product (forward, input gradient and
 * weight gradient) runs on the matrix cores with BF16 operands (weights,
 * activations, back-propagated errors rounded to BF16) and FP32 accumulation.
 *
 * Flat parameter vector (FP32), in this order: W1[in_dim][hidden], b1[hidden];
 * for each further hidden layer W[hidden][hidden], b[hidden]; then
 * w_out[hidden], b_out.  W[i][j] connects input i to unit j (row-major).
 *
 * Conventions are those of rewl.h: every call returns a rewl_status, the
 * thread-local mlp_last_error() describes a failure, the library owns the
 * device memory it allocates and work is ordered on the stream given at
 * creation.  Rows, targets and results cross as host arrays: the library stages
 * them through its own device buffers (the data sets are small: tens of
 * thousands of rows), and every call returns with its stream synchronised.
 */
#ifndef REWL_MLP_H
#define REWL_MLP_H
#include "rewl.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t in_dim;     /* inputs per row, 1..16 (3 for the (E/N, 1/L, q) encoding)        */
    int32_t hidden;     /* units per hidden layer: a multiple of 64, 64..4096              */
    int32_t layers;     /* hidden layers, 1..16                                            */
    int32_t max_batch;  /* largest batch a call may use, 1..2^20 (rounded up to a multiple of 64) */
    uint64_t seed;      /* initial weights: uniform in +-1/sqrt(fan_in), biases zero       */
} mlp_config;

typedef struct mlp_handle mlp_handle;

/* Allocate a network on `hip_stream` (a hipStream_t or NULL for a private one). */
rewl_status mlp_create(const mlp_config* cfg, void* hip_stream, mlp_handle** out);
void mlp_destroy(mlp_handle* h);
const char* mlp_last_error(void);

/* *n = length of the flat parameter vector. */
rewl_status mlp_n_params(const mlp_handle* h, int64_t* n);

/* Copy the FP32 parameters out / in (host arrays of exactly n entries).  Setting
 * parameters refreshes the BF16 copies and leaves the Adam moments untouched. */
rewl_status mlp_get_params(const mlp_handle* h, float* host, size_t n);
rewl_status mlp_set_params(mlp_handle* h, const float* host, size_t n);

/* Forward pass: y[r] = net(x[r][0..in_dim)) for r < B (host arrays x[B][in_dim],
 * y[B]; any B >= 0, processed in chunks of max_batch rows). */
rewl_status mlp_infer(mlp_handle* h, const float* x, float* y, int32_t B);

/* Loss (1/B) sum_r (net(x_r) - t_r)^2 and its gradient with respect to the flat
 * parameter vector, for 1 <= B <= max_batch host rows x[B][in_dim], t[B].
 * grad (n_params entries) and loss may be NULL.  Does not change the parameters. */
rewl_status mlp_grad(mlp_handle* h, const float* x, const float* t, int32_t B, float* grad,
                     float* loss);

/* `steps` Adam steps with learning rate lr, each on B rows (a multiple of 64,
 * <= max_batch) drawn with replacement from the n host rows x[n][in_dim], t[n]
 * (1 <= n < 2^31, uploaded once per call) by a hash of (seed, handle's step
 * count).  *last_loss (may be NULL) receives the last step's batch loss. */
rewl_status mlp_fit(mlp_handle* h, const float* x, const float* t, int64_t n, int32_t B,
                    int64_t steps, float lr, uint32_t seed, float* last_loss);

/* Warm-start table of a model (in_dim must be 3): for every global energy bin of
 * the bin convention of rewl.h (model 0 Ising: W = N + 1, E = 4b - 2N; model 1
 * Potts: W = 2N + 1, E = b - 2N), lng_host[b] = N * net(E/N, 1/L, q) rounded to
 * the nearest multiple of 2^-16 (q = 2 encodes Ising; 2 <= L <= 4096).  The
 * table is a valid argument of rewl_set_initial_lng. */
rewl_status mlp_warm_table(mlp_handle* h, int32_t model, int32_t q, int32_t L, double* lng_host);

/* Diagnostic: C = A B on the matrix cores with BF16-rounded operands and FP32
 * accumulation; host arrays, A[M][K], B[K][N], C[M][N]; M, N multiples of 64,
 * K a multiple of 32. */
rewl_status mlp_probe_gemm(const float* A, const float* B, int32_t M, int32_t N, int32_t K, float* C);

#ifdef __cplusplus
}
#endif
#endif
