// Internal interface between the surrogate-MLP kernels (k_mlp.hip) and the C
// ABI (mlp_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlpk {

constexpr uint32_t kInMax = 256;  // most raw inputs
// padded input width: 128 columns for up to 128 inputs, else 256
__host__ __device__ constexpr uint32_t k0_of(uint32_t n_in) { return n_in <= 128u ? 128u : 256u; }
constexpr uint32_t kOutPad = 16;  // padded output width
constexpr uint32_t kTile = 64;    // GEMM output tile (rows and columns)
constexpr uint32_t kTileK = 32;   // GEMM contraction step (one MFMA 16x16x32)

// Operand element (r, k) of a GEMM operand sits at p[r * ld + k] (K-contiguous)
// or at p[k * ld + r] (row-contiguous); r runs over the rows of C (operand A)
// or its columns (operand B).
enum Layout : int { LD_K = 0, LD_R = 1 };
// What the GEMM does with its FP32 tile:
//  EPI_GELU     z = acc + bias -> Z (FP32), H = bf16(GELU(z))
//  EPI_LINEAR   C = acc + bias (FP32)
//  EPI_BWD_GELU H = bf16(acc * GELU'(Z))
//  EPI_PARTIAL  C[blockIdx.z] = acc (split-K partial sums)
enum Epi : int { EPI_GELU = 0, EPI_LINEAR = 1, EPI_BWD_GELU = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
    const uint16_t *A;
    uint32_t lda;
    const uint16_t *B;
    uint32_t ldb;
    uint32_t M, N, K;    // C is M x N, contraction over K
    uint32_t k_split;    // contraction elements per blockIdx.z (multiple of kTileK)
    const float *bias;
    float *Z;
    uint32_t ldz;
    uint16_t *H;
    uint32_t ldh;
    float *C;
    uint32_t ldc;
};

bool launch_gemm(hipStream_t s, int a_layout, int b_layout, int epi, const GemmArgs &g, uint32_t splits);
void launch_splitk_reduce(hipStream_t s, const float *partials, uint32_t splits, uint32_t count, float *out);
void launch_standardize(hipStream_t s, const float *X, uint32_t m, uint32_t n_in, const float *mu,
                        const float *sd, uint16_t *Xb);
// Residual input columns added to the outputs: X[r * ldx + col0 + j] (X null: none).
struct Residual {
    const float *X;
    uint32_t ldx, col0;
};
void launch_loss(hipStream_t s, const float *out, const float *Y, uint32_t m, uint32_t n_out, const float *mu,
                 const float *sd, const Residual &res, uint16_t *dout, double *partials, uint32_t nblk, double *loss);
uint32_t loss_blocks(uint32_t m);
// db = column sums of dz (m rows); part: scratch of ceil(m / 128) * n floats.
void launch_bias_grad(hipStream_t s, const uint16_t *dz, uint32_t m, uint32_t n, uint32_t ld, float *db,
                      float *part);
void launch_adam(hipStream_t s, float *w, float *m1, float *m2, const float *g, uint16_t *wb, uint32_t count,
                 float lr, float beta1, float beta2, float eps, float bc1, float bc2);
void launch_to_bf16(hipStream_t s, const float *w, uint16_t *wb, uint32_t count);
// flags (null: none): rows whose output is the residual base alone.
void launch_destandardize(hipStream_t s, const float *out, uint32_t m, uint32_t n_out, const float *mu,
                          const float *sd, const Residual &res, const uint8_t *flags, float *Y);
// lo, hi (null: not wanted): column minimum and maximum of X.
void launch_fit_normalizer(hipStream_t s, const float *X, uint32_t m, uint32_t cols, const Residual &res, float *mu,
                           float *sd, float *lo, float *hi);
// Training-range guard: a row falls back when some column j fails
// a[j] <= x_j <= b[j] (NaN included); count (device) adds the rows that did.
struct Guard {
    const float *a, *b;          // null: guard off
    unsigned long long *count;
};
void launch_guard_rows(hipStream_t s, const float *X, uint32_t m, uint32_t n_in, const Guard &g, uint8_t *flags);
void launch_fill_f32(hipStream_t s, float *p, float v, uint32_t count);

struct PredictArgs {
    const float *x;      // n_in raw features
    float *y;            // n_out raw outputs
    const uint16_t *wb;  // BF16 parameters (parameter layout)
    const float *w;      // FP32 parameters (biases are read from here)
    const float *mu_x, *sd_x, *mu_y, *sd_y;
    uint32_t n_in, k0, n_out, hidden, layers;   // k0: padded input width
    int32_t res_col0;    // first residual input column, or -1
    Guard guard;         // out of the training range: y = residual base
};
void launch_predict_one(hipStream_t s, const PredictArgs &a);

}  // namespace mlpk
