/*
 * sph_mlp.h - C ABI of the learned body-wrench surrogate (arXiv 2511.15908,
 * Sec. 3.3: the haptic device needs force updates near 1 kHz while the SPH step
 * runs slower; the paper bridges the gap with a rolling average of the last
 * wrenches; this library adds a small multilayer perceptron that predicts the
 * wrench between SPH updates from the grabbed body's state, its recent wrenches
 * and the fluid density around it (density field of Sec. 3.4)).
 *
 * Network: x (n_in <= 256 raw features, standardised, zero-padded to K_0 =
 *   128 columns, or 256 when n_in > 128)
 *   -> L hidden layers of H units (GELU, erf form) -> n_out <= 16 outputs
 *   (standardised targets; de-standardised on output).  With residual_from
 *   = k > 0 the output is y = x[k-1 .. k-2+n_out] + destandardised network
 *   output, and targets, normaliser and loss refer to y - x[k-1 ..].
 * Precision: GEMM operands (weights, activations, output gradients) in BF16,
 * accumulation in FP32 on the matrix cores; master weights, biases, Adam
 * moments, pre-activations and the loss in FP32 (loss sum in FP64).
 * Training: mean squared error over the n_out standardised outputs, Adam
 * (Kingma and Ba, with bias correction).
 *
 * Parameter layout (FP32, flat, mlp_param_count() floats), layer l = 0..L:
 *   W_l [N_l][K_l] row-major (row = output unit), then b_l [N_l];
 *   K_0 = 128 (n_in <= 128) or 256, K_l = H (l > 0); N_l = H (l < L), N_L = 16.
 * Rows n_out..15 of W_L and entries n_out..15 of b_L are forced to zero.
 *
 * Device arrays (X, Y, out) are caller-owned device memory; host arrays are
 * copied before the call returns.  All device work is enqueued on the stream
 * given to mlp_init.  Every call returns an mlp_status and never aborts; after
 * a device error the context only accepts mlp_destroy.  One context per thread.
 */
#ifndef SPH_MLP_H_
#define SPH_MLP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_ABI_VERSION 1

typedef enum {
    MLP_OK = 0,
    MLP_ERR_ARG = 1,        /* bad argument; nothing enqueued */
    MLP_ERR_WORKSPACE = 2,  /* workspace missing, too small or misaligned */
    MLP_ERR_DEVICE = 3,     /* HIP error; text in mlp_last_error */
    MLP_ERR_STATE = 4,      /* context unusable after an earlier device error */
    MLP_ERR_NONFINITE = 5   /* loss or a normaliser statistic is not finite */
} mlp_status;

typedef struct {
    uint32_t abi_version;   /* MLP_ABI_VERSION */
    uint32_t n_in;          /* raw input features, 1..256 */
    uint32_t n_out;         /* outputs, 1..16 */
    uint32_t hidden;        /* H: 64, 128, 192 or 256 */
    uint32_t layers;        /* L hidden layers, 1..4 */
    uint32_t max_batch;     /* most rows per mlp_forward / training call, 1..65536 */
    float beta1, beta2, eps; /* Adam constants (0.9, 0.999, 1e-8 typical) */
    uint32_t residual_from; /* 0: the outputs are the network's; k > 0: raw input columns
                               k-1 .. k-2+n_out are added to them (the network learns the
                               change from those inputs); k-1+n_out <= n_in */
    uint32_t reserved[6];   /* must be zero */
} mlp_config;

typedef struct mlp_ctx mlp_ctx;

/* Bytes of device workspace for cfg (256-byte aligned base required). */
mlp_status mlp_workspace_size(const mlp_config *cfg, size_t *bytes);
/* Create a context over the caller's workspace (borrowed until mlp_destroy).
 * Parameters start at zero and the normaliser at identity; call
 * mlp_set_params with the caller's initial weights (the random draw is the
 * caller's). */
mlp_status mlp_init(const mlp_config *cfg, void *d_workspace, size_t ws_bytes, void *hip_stream,
                    mlp_ctx **out);
size_t mlp_param_count(const mlp_ctx *ctx);

/* FP32 master parameters in the layout above (host array of mlp_param_count()
 * floats).  Resets the Adam moments and step count.  mlp_get_params
 * synchronises. */
mlp_status mlp_set_params(mlp_ctx *ctx, const float *params, size_t n);
mlp_status mlp_get_params(mlp_ctx *ctx, float *params, size_t n);

/* Standardisation x' = (x - mu_x) / sd_x, y' = (y - mu_y) / sd_y.
 * mlp_fit_normalizer computes mean and population standard deviation of each
 * column of the m x n_in raw inputs X and m x n_out raw targets Y (device,
 * row-major) on the device (FP64 sums); a column whose deviation is below
 * 1e-12 (or zero) gets sd = 1.  With residual_from the target statistics are
 * those of Y minus the residual input columns.  mlp_set_normalizer / mlp_get_normalizer move
 * the four host vectors (n_in, n_in, n_out, n_out floats). */
mlp_status mlp_fit_normalizer(mlp_ctx *ctx, const float *X, const float *Y, uint32_t m);
mlp_status mlp_set_normalizer(mlp_ctx *ctx, const float *mu_x, const float *sd_x, const float *mu_y,
                              const float *sd_y);
mlp_status mlp_get_normalizer(mlp_ctx *ctx, float *mu_x, float *sd_x, float *mu_y, float *sd_y);

/*
 * Plain SPH as the fallback: the device loop of Sec. 3.3 holds the
 * simulator's last wrench between its updates; the network refines that hold
 * only on inputs like those it was trained on, and elsewhere the loop keeps
 * the simulator's own wrench.  mlp_fit_normalizer also
 * records the minimum lo_j and maximum hi_j of every input column of X;
 * mlp_set_input_range sets them from host arrays (n_in floats each, finite,
 * lo <= hi) and mlp_get_input_range reads them back.  mlp_set_guard(margin)
 * with margin >= 0 turns the guard on: with w_j = hi_j - lo_j and, in FP32,
 * a_j = lo_j - margin w_j, b_j = hi_j + margin w_j, a row whose input fails
 * a_j <= x_j <= b_j in some column (NaN included) gets the residual base
 * instead of the network's output: out_j = x[residual_from - 1 + j], for the
 * wrench surrogate the last SPH wrench (zero-order hold).  mlp_forward and
 * both haptic-tick calls apply it; training and mlp_gradients never do.
 * margin < 0 turns it off (the default).  Errors: MLP_ERR_ARG
 * for a model without residual_from or a bad range, MLP_ERR_STATE when no
 * range was fitted or set.  mlp_guard_count: out[0] rows checked by guarded
 * calls since init, out[1] rows that fell back (synchronises).
 */
mlp_status mlp_set_input_range(mlp_ctx *ctx, const float *lo, const float *hi);
mlp_status mlp_get_input_range(mlp_ctx *ctx, float *lo, float *hi);
mlp_status mlp_set_guard(mlp_ctx *ctx, float margin);
mlp_status mlp_guard_count(mlp_ctx *ctx, uint64_t out[2]);

/* Batched inference: out [m][n_out] (raw units) from X [m][n_in] (raw), m <= max_batch. */
mlp_status mlp_forward(mlp_ctx *ctx, const float *X, uint32_t m, float *out);

/* Gradient of the loss L = 1/(m n_out) sum_{rows, j < n_out} (out'_j - y'_j)^2 on
 * standardised values, for X [m][n_in], Y [m][n_out] (raw, device); written to
 * the host array grad (mlp_param_count() floats, parameter layout) together
 * with the loss; synchronises.  The parameters are not changed. */
mlp_status mlp_gradients(mlp_ctx *ctx, const float *X, const float *Y, uint32_t m, float *grad, double *loss);

/* One Adam step with the given host gradient (parameter layout). */
mlp_status mlp_adam_step(mlp_ctx *ctx, const float *grad, size_t n, float lr);

/* One training step on a batch: forward, loss, backward, Adam with rate lr.
 * The batch loss is kept on the device; mlp_last_loss synchronises and returns
 * it (MLP_ERR_NONFINITE if it is not finite). */
mlp_status mlp_train_step(mlp_ctx *ctx, const float *X, const float *Y, uint32_t m, float lr);
mlp_status mlp_last_loss(mlp_ctx *ctx, double *loss);

/* One sample at haptic rate: a single workgroup runs the whole chain
 * (standardise, L+1 GEMVs with GELU, de-standardise).  x: n_in raw floats,
 * y: n_out floats.  mlp_predict_one takes host arrays and synchronises
 * (end-to-end latency of one haptic tick); mlp_predict_one_device takes
 * device arrays and only enqueues. */
mlp_status mlp_predict_one(mlp_ctx *ctx, const float *x, float *y);
mlp_status mlp_predict_one_device(mlp_ctx *ctx, const float *x, float *y);

/* Stand-alone product C[M][N] = sum_k A(m,k) B(k,n) of the training
 * kernels' tile engine (BF16 operands, FP32 accumulation and result), enqueued on
 * hip_stream.  A(m,k) = A[m*lda + k] (a_layout 0) or A[k*lda + m] (1);
 * B(k,n) = B[n*ldb + k] (b_layout 0) or B[k*ldb + n] (1).  Operands are BF16
 * bit patterns in device memory, 16-byte aligned with lda, ldb multiples of 8;
 * C is FP32 with row stride ldc >= N. */
mlp_status mlp_gemm_bf16(void *hip_stream, int a_layout, int b_layout, const uint16_t *A, uint32_t lda,
                         const uint16_t *B, uint32_t ldb, uint32_t M, uint32_t N, uint32_t K, float *C, uint32_t ldc);

/* Release the context (not the workspace).  NULL is accepted. */
mlp_status mlp_destroy(mlp_ctx *ctx);
const char *mlp_last_error(const mlp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SPH_MLP_H_ */
