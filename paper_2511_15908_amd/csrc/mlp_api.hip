// C ABI of the wrench-surrogate MLP (include/sph_mlp.h): validation,
// workspace carving, and the sequences of kernels of a forward pass, a
// gradient pass, an Adam step and a haptic tick.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sph_mlp.h"
#include "mlp_internal.h"

using namespace mlpk;

struct mlp_ctx {
    mlp_config cfg{};
    hipStream_t stream = nullptr;
    uint32_t H = 0, L = 0, B = 0;
    size_t P = 0;                       // parameter count
    std::vector<size_t> off;            // parameter offset of W_l
    std::vector<uint32_t> Nl, Kl;
    // device buffers
    float *w = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    uint16_t *wb = nullptr;
    float *mu_x = nullptr, *sd_x = nullptr, *mu_y = nullptr, *sd_y = nullptr;
    uint16_t *xb = nullptr;
    std::vector<float *> Z;
    std::vector<uint16_t *> Hact;
    float *out = nullptr;
    uint16_t *dout = nullptr, *dz[2] = {nullptr, nullptr};
    float *partials = nullptr;
    uint32_t max_splits = 1;
    double *loss_part = nullptr, *loss = nullptr;
    float *px = nullptr, *py = nullptr;
    // training-range guard (plain-SPH fallback)
    float *xlo = nullptr, *xhi = nullptr;        // device: fitted column range
    float *ga = nullptr, *gb = nullptr;          // device: guard bounds a_j, b_j
    uint8_t *gflags = nullptr;                   // [max_batch] rows that fell back
    unsigned long long *gcount = nullptr;        // rows that fell back
    std::vector<float> lo, hi;                   // host copy of the range (empty: none)
    float margin = -1.0f;                        // < 0: guard off
    uint64_t guarded_rows = 0;
    uint64_t t = 0;                     // Adam steps taken
    bool dead = false;
    std::string last_error;
};

namespace {

constexpr uint32_t kSplitRows = 256;    // batch rows per split-K slice
constexpr uint32_t kMaxSplits = 64;

struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T) + 16;
        return p;
    }
};

mlp_status validate(const mlp_config *c, std::string &why)
{
    if (!c) {
        why = "null config";
        return MLP_ERR_ARG;
    }
    if (c->abi_version != MLP_ABI_VERSION) {
        why = "abi_version mismatch";
        return MLP_ERR_ARG;
    }
    for (uint32_t r : c->reserved)
        if (r) {
            why = "reserved fields must be zero";
            return MLP_ERR_ARG;
        }
    if (c->n_in < 1 || c->n_in > kInMax || c->n_out < 1 || c->n_out > kOutPad) {
        why = "n_in must be 1..256 and n_out 1..16";
        return MLP_ERR_ARG;
    }
    if (c->hidden < 64 || c->hidden > 256 || c->hidden % 64) {
        why = "hidden must be 64, 128, 192 or 256";
        return MLP_ERR_ARG;
    }
    if (c->layers < 1 || c->layers > 4) {
        why = "layers must be 1..4";
        return MLP_ERR_ARG;
    }
    if (c->max_batch < 1 || c->max_batch > 65536) {
        why = "max_batch must be 1..65536";
        return MLP_ERR_ARG;
    }
    if (c->residual_from && c->residual_from - 1u + c->n_out > c->n_in) {
        why = "residual columns must lie inside the inputs";
        return MLP_ERR_ARG;
    }
    if (!(c->beta1 >= 0.f && c->beta1 < 1.f) || !(c->beta2 >= 0.f && c->beta2 < 1.f) || !(c->eps > 0.f) ||
        !isfinite(c->eps)) {
        why = "Adam constants: 0 <= beta < 1, eps > 0";
        return MLP_ERR_ARG;
    }
    return MLP_OK;
}

void layout(mlp_ctx *c)
{
    c->H = c->cfg.hidden;
    c->L = c->cfg.layers;
    c->B = c->cfg.max_batch;
    c->off.clear();
    c->Nl.clear();
    c->Kl.clear();
    size_t o = 0;
    for (uint32_t l = 0; l <= c->L; ++l) {
        const uint32_t K = l == 0 ? k0_of(c->cfg.n_in) : c->H, N = l == c->L ? kOutPad : c->H;
        c->off.push_back(o);
        c->Nl.push_back(N);
        c->Kl.push_back(K);
        o += (size_t)N * K + N;
    }
    c->P = o;
    c->max_splits = (c->B + kSplitRows - 1) / kSplitRows;
    if (c->max_splits > kMaxSplits) c->max_splits = kMaxSplits;
    if (c->max_splits < 1) c->max_splits = 1;
}

size_t carve(mlp_ctx *c, char *base)
{
    Carve cv{base};
    const size_t P = c->P, B = c->B, H = c->H;
    c->w = cv.take<float>(P);
    c->m1 = cv.take<float>(P);
    c->m2 = cv.take<float>(P);
    c->grad = cv.take<float>(P);
    c->wb = cv.take<uint16_t>(P);
    c->mu_x = cv.take<float>(kInMax);
    c->sd_x = cv.take<float>(kInMax);
    c->mu_y = cv.take<float>(kOutPad);
    c->sd_y = cv.take<float>(kOutPad);
    c->xb = cv.take<uint16_t>(B * k0_of(c->cfg.n_in));
    c->Z.assign(c->L, nullptr);
    c->Hact.assign(c->L, nullptr);
    for (uint32_t l = 0; l < c->L; ++l) {
        c->Z[l] = cv.take<float>(B * H);
        c->Hact[l] = cv.take<uint16_t>(B * H);
    }
    c->out = cv.take<float>(B * kOutPad);
    c->dout = cv.take<uint16_t>(B * kOutPad);
    c->dz[0] = cv.take<uint16_t>(B * H);
    c->dz[1] = cv.take<uint16_t>(B * H);
    size_t maxwk = 0;
    for (uint32_t l = 0; l <= c->L; ++l) maxwk = std::max(maxwk, (size_t)c->Nl[l] * c->Kl[l]);
    // split-K partials of the weight gradients, later the bias-gradient row
    // slices (128 rows each) of the same layer
    const size_t bias_part = (size_t)((c->B + 127) / 128) * std::max<uint32_t>(c->H, 16u);
    c->partials = cv.take<float>(std::max((size_t)c->max_splits * maxwk, bias_part));
    c->loss_part = cv.take<double>(loss_blocks(c->B));
    c->loss = cv.take<double>(1);
    c->px = cv.take<float>(kInMax);
    c->py = cv.take<float>(kOutPad);
    c->xlo = cv.take<float>(kInMax);
    c->xhi = cv.take<float>(kInMax);
    c->ga = cv.take<float>(kInMax);
    c->gb = cv.take<float>(kInMax);
    c->gflags = cv.take<uint8_t>(B);
    c->gcount = cv.take<unsigned long long>(1);
    return cv.off;
}

mlp_status dev_fail(mlp_ctx *c, hipError_t e, const char *what)
{
    c->dead = true;
    c->last_error = std::string(what) + ": " + hipGetErrorString(e);
    return MLP_ERR_DEVICE;
}

#define MLPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return dev_fail(ctx, e_, #call); \
    } while (0)

mlp_status arg_fail(mlp_ctx *c, const char *why)
{
    c->last_error = why;
    return MLP_ERR_ARG;
}

// Refresh the BF16 copy of the master parameters.
void refresh_bf16(mlp_ctx *c) { launch_to_bf16(c->stream, c->w, c->wb, (uint32_t)c->P); }

void forward(mlp_ctx *c, const float *X, uint32_t m)
{
    hipStream_t s = c->stream;
    launch_standardize(s, X, m, c->cfg.n_in, c->mu_x, c->sd_x, c->xb);
    const uint16_t *a = c->xb;
    uint32_t lda = k0_of(c->cfg.n_in);
    for (uint32_t l = 0; l <= c->L; ++l) {
        GemmArgs g{};
        g.A = a;
        g.lda = lda;
        g.B = c->wb + c->off[l];
        g.ldb = c->Kl[l];
        g.M = m;
        g.N = c->Nl[l];
        g.K = c->Kl[l];
        g.k_split = g.K;
        g.bias = c->w + c->off[l] + (size_t)c->Nl[l] * c->Kl[l];
        if (l < c->L) {
            g.Z = c->Z[l];
            g.ldz = c->H;
            g.H = c->Hact[l];
            g.ldh = c->H;
            launch_gemm(s, LD_K, LD_K, EPI_GELU, g, 1);
            a = c->Hact[l];
            lda = c->H;
        } else {
            g.C = c->out;
            g.ldc = kOutPad;
            launch_gemm(s, LD_K, LD_K, EPI_LINEAR, g, 1);
        }
    }
}

Residual residual(const mlp_ctx *c, const float *X)
{
    Residual r{nullptr, 0, 0};
    if (c->cfg.residual_from) {
        r.X = X;
        r.ldx = c->cfg.n_in;
        r.col0 = c->cfg.residual_from - 1u;
    }
    return r;
}

// Loss and gradient into c->grad (forward must have run on the same rows X).
void backward(mlp_ctx *c, const float *X, const float *Y, uint32_t m)
{
    hipStream_t s = c->stream;
    launch_loss(s, c->out, Y, m, c->cfg.n_out, c->mu_y, c->sd_y, residual(c, X), c->dout, c->loss_part,
                loss_blocks(m), c->loss);
    uint32_t splits = (m + kSplitRows - 1) / kSplitRows;
    if (splits > c->max_splits) splits = c->max_splits;
    uint32_t ks = (m + splits - 1) / splits;
    ks = (ks + kTileK - 1) / kTileK * kTileK;
    splits = (m + ks - 1) / ks;
    const uint16_t *dz = c->dout;
    uint32_t ldd = kOutPad;
    int cur = 0;
    for (int l = (int)c->L; l >= 0; --l) {
        const uint32_t N = c->Nl[l], K = c->Kl[l];
        const uint16_t *aprev = l == 0 ? c->xb : c->Hact[l - 1];
        // dW_l = dz^T a_{l-1}: rows N, columns K, contraction over the batch
        GemmArgs g{};
        g.A = dz;
        g.lda = ldd;
        g.B = aprev;
        g.ldb = K;
        g.M = N;
        g.N = K;
        g.K = m;
        g.k_split = ks;
        g.C = c->partials;
        g.ldc = K;
        launch_gemm(s, LD_R, LD_R, EPI_PARTIAL, g, splits);
        launch_splitk_reduce(s, c->partials, splits, N * K, c->grad + c->off[l]);
        // the split-K partials are consumed: their buffer holds the bias partials
        launch_bias_grad(s, dz, m, N, ldd, c->grad + c->off[l] + (size_t)N * K, c->partials);
        if (l > 0) {
            // dz_{l-1} = (dz W_l) * GELU'(z_{l-1})
            GemmArgs h{};
            h.A = dz;
            h.lda = ldd;
            h.B = c->wb + c->off[l];
            h.ldb = K;
            h.M = m;
            h.N = K;
            h.K = N;
            h.k_split = N;
            h.Z = c->Z[l - 1];
            h.ldz = c->H;
            h.H = c->dz[cur];
            h.ldh = c->H;
            launch_gemm(s, LD_K, LD_R, EPI_BWD_GELU, h, 1);
            dz = c->dz[cur];
            ldd = c->H;
            cur ^= 1;
        }
    }
}

mlp_status adam(mlp_ctx *c, float lr)
{
    c->t += 1;
    const double bc1 = 1.0 - pow((double)c->cfg.beta1, (double)c->t);
    const double bc2 = 1.0 - pow((double)c->cfg.beta2, (double)c->t);
    launch_adam(c->stream, c->w, c->m1, c->m2, c->grad, c->wb, (uint32_t)c->P, lr, c->cfg.beta1, c->cfg.beta2,
                c->cfg.eps, (float)bc1, (float)bc2);
    MLPCHK(c, hipGetLastError());
    return MLP_OK;
}

mlp_status check_batch(mlp_ctx *c, const void *X, uint32_t m)
{
    if (m < 1 || m > c->B) return arg_fail(c, "m must be 1..max_batch");
    if (!X || ((uintptr_t)X & 3u)) return arg_fail(c, "null or misaligned device array");
    return MLP_OK;
}

}  // namespace

extern "C" {

// Guard bounds a_j = lo_j - margin w_j, b_j = hi_j + margin w_j in FP32 (one
// rounding per operation, no fused multiply-add), uploaded when the guard is on.
static mlp_status upload_guard(mlp_ctx *c)
{
    if (c->margin < 0.0f || c->lo.empty()) return MLP_OK;
    const uint32_t n = c->cfg.n_in;
    std::vector<float> a(n), b(n);
    for (uint32_t j = 0; j < n; ++j) {
        const float w = c->hi[j] - c->lo[j];
        const float mw = c->margin * w;
        a[j] = c->lo[j] - mw;
        b[j] = c->hi[j] + mw;
    }
    MLPCHK(c, hipMemcpyAsync(c->ga, a.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipMemcpyAsync(c->gb, b.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

static Guard guard_of(const mlp_ctx *c)
{
    return c->margin >= 0.0f ? Guard{c->ga, c->gb, c->gcount} : Guard{nullptr, nullptr, nullptr};
}

mlp_status mlp_workspace_size(const mlp_config *cfg, size_t *bytes)
{
    std::string why;
    if (!bytes) return MLP_ERR_ARG;
    const mlp_status st = validate(cfg, why);
    if (st != MLP_OK) return st;
    mlp_ctx tmp;
    tmp.cfg = *cfg;
    layout(&tmp);
    *bytes = carve(&tmp, nullptr);
    return MLP_OK;
}

mlp_status mlp_init(const mlp_config *cfg, void *d_workspace, size_t ws_bytes, void *hip_stream, mlp_ctx **out)
{
    if (!out) return MLP_ERR_ARG;
    *out = nullptr;
    std::string why;
    const mlp_status st = validate(cfg, why);
    if (st != MLP_OK) return st;
    mlp_ctx *c = new mlp_ctx;
    c->cfg = *cfg;
    c->stream = (hipStream_t)hip_stream;
    layout(c);
    const size_t need = carve(c, nullptr);
    if (!d_workspace || ws_bytes < need || ((uintptr_t)d_workspace & 255u)) {
        delete c;
        return MLP_ERR_WORKSPACE;
    }
    carve(c, (char *)d_workspace);
    hipStream_t s = c->stream;
    launch_fill_f32(s, c->w, 0.f, (uint32_t)c->P);
    launch_fill_f32(s, c->m1, 0.f, (uint32_t)c->P);
    launch_fill_f32(s, c->m2, 0.f, (uint32_t)c->P);
    launch_fill_f32(s, c->grad, 0.f, (uint32_t)c->P);
    launch_fill_f32(s, c->mu_x, 0.f, kInMax);
    launch_fill_f32(s, c->sd_x, 1.f, kInMax);
    launch_fill_f32(s, c->mu_y, 0.f, kOutPad);
    launch_fill_f32(s, c->sd_y, 1.f, kOutPad);
    launch_fill_f32(s, reinterpret_cast<float *>(c->gcount), 0.f, 2);
    refresh_bf16(c);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete c;
        return MLP_ERR_DEVICE;
    }
    *out = c;
    return MLP_OK;
}

size_t mlp_param_count(const mlp_ctx *ctx) { return ctx ? ctx->P : 0; }

mlp_status mlp_set_params(mlp_ctx *c, const float *params, size_t n)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!params || n != c->P) return arg_fail(c, "params must hold mlp_param_count() floats");
    std::vector<float> p(params, params + n);
    for (float v : p)
        if (!isfinite(v)) return arg_fail(c, "non-finite parameter");
    // padded output rows carry nothing
    const uint32_t L = c->L, K = c->Kl[L];
    for (uint32_t r = c->cfg.n_out; r < kOutPad; ++r) {
        for (uint32_t k = 0; k < K; ++k) p[c->off[L] + (size_t)r * K + k] = 0.f;
        p[c->off[L] + (size_t)kOutPad * K + r] = 0.f;
    }
    MLPCHK(c, hipMemcpyAsync(c->w, p.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    launch_fill_f32(c->stream, c->m1, 0.f, (uint32_t)c->P);
    launch_fill_f32(c->stream, c->m2, 0.f, (uint32_t)c->P);
    refresh_bf16(c);
    c->t = 0;
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

mlp_status mlp_get_params(mlp_ctx *c, float *params, size_t n)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!params || n != c->P) return arg_fail(c, "params must hold mlp_param_count() floats");
    MLPCHK(c, hipMemcpyAsync(params, c->w, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

mlp_status mlp_fit_normalizer(mlp_ctx *c, const float *X, const float *Y, uint32_t m)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (m < 1 || !X || !Y) return arg_fail(c, "m >= 1 and device arrays required");
    launch_fit_normalizer(c->stream, X, m, c->cfg.n_in, Residual{nullptr, 0, 0}, c->mu_x, c->sd_x, c->xlo, c->xhi);
    launch_fit_normalizer(c->stream, Y, m, c->cfg.n_out, residual(c, X), c->mu_y, c->sd_y, nullptr, nullptr);
    MLPCHK(c, hipGetLastError());
    std::vector<float> a(kInMax), b(kInMax), d(kOutPad), e(kOutPad), lo(c->cfg.n_in), hi(c->cfg.n_in);
    MLPCHK(c, hipMemcpyAsync(lo.data(), c->xlo, c->cfg.n_in * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(hi.data(), c->xhi, c->cfg.n_in * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(a.data(), c->mu_x, kInMax * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(b.data(), c->sd_x, kInMax * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(d.data(), c->mu_y, kOutPad * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(e.data(), c->sd_y, kOutPad * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    for (uint32_t i = 0; i < c->cfg.n_in; ++i)
        if (!isfinite(a[i]) || !isfinite(b[i])) return MLP_ERR_NONFINITE;
    for (uint32_t i = 0; i < c->cfg.n_out; ++i)
        if (!isfinite(d[i]) || !isfinite(e[i])) return MLP_ERR_NONFINITE;
    for (uint32_t i = 0; i < c->cfg.n_in; ++i)
        if (!isfinite(lo[i]) || !isfinite(hi[i])) return MLP_ERR_NONFINITE;
    c->lo = lo;
    c->hi = hi;
    return upload_guard(c);
}

mlp_status mlp_set_normalizer(mlp_ctx *c, const float *mu_x, const float *sd_x, const float *mu_y, const float *sd_y)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!mu_x || !sd_x || !mu_y || !sd_y) return arg_fail(c, "null normaliser array");
    const uint32_t ni = c->cfg.n_in, no = c->cfg.n_out;
    for (uint32_t i = 0; i < ni; ++i)
        if (!isfinite(mu_x[i]) || !(sd_x[i] > 0.f) || !isfinite(sd_x[i])) return arg_fail(c, "bad input statistic");
    for (uint32_t i = 0; i < no; ++i)
        if (!isfinite(mu_y[i]) || !(sd_y[i] > 0.f) || !isfinite(sd_y[i])) return arg_fail(c, "bad output statistic");
    MLPCHK(c, hipMemcpyAsync(c->mu_x, mu_x, ni * 4, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipMemcpyAsync(c->sd_x, sd_x, ni * 4, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipMemcpyAsync(c->mu_y, mu_y, no * 4, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipMemcpyAsync(c->sd_y, sd_y, no * 4, hipMemcpyHostToDevice, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

mlp_status mlp_get_normalizer(mlp_ctx *c, float *mu_x, float *sd_x, float *mu_y, float *sd_y)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!mu_x || !sd_x || !mu_y || !sd_y) return arg_fail(c, "null normaliser array");
    const uint32_t ni = c->cfg.n_in, no = c->cfg.n_out;
    MLPCHK(c, hipMemcpyAsync(mu_x, c->mu_x, ni * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(sd_x, c->sd_x, ni * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(mu_y, c->mu_y, no * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipMemcpyAsync(sd_y, c->sd_y, no * 4, hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

mlp_status mlp_forward(mlp_ctx *c, const float *X, uint32_t m, float *out)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    mlp_status st = check_batch(c, X, m);
    if (st != MLP_OK) return st;
    if (!out) return arg_fail(c, "null output");
    forward(c, X, m);
    const Guard g = guard_of(c);
    if (g.a) {
        launch_guard_rows(c->stream, X, m, c->cfg.n_in, g, c->gflags);
        c->guarded_rows += m;
    }
    launch_destandardize(c->stream, c->out, m, c->cfg.n_out, c->mu_y, c->sd_y, residual(c, X),
                         g.a ? c->gflags : nullptr, out);
    MLPCHK(c, hipGetLastError());
    return MLP_OK;
}

mlp_status mlp_set_input_range(mlp_ctx *c, const float *lo, const float *hi)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!lo || !hi) return arg_fail(c, "null range array");
    const uint32_t n = c->cfg.n_in;
    for (uint32_t j = 0; j < n; ++j)
        if (!isfinite(lo[j]) || !isfinite(hi[j]) || !(lo[j] <= hi[j])) return arg_fail(c, "bad input range");
    c->lo.assign(lo, lo + n);
    c->hi.assign(hi, hi + n);
    return upload_guard(c);
}

mlp_status mlp_get_input_range(mlp_ctx *c, float *lo, float *hi)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!lo || !hi) return arg_fail(c, "null range array");
    if (c->lo.empty()) return MLP_ERR_STATE;
    std::copy(c->lo.begin(), c->lo.end(), lo);
    std::copy(c->hi.begin(), c->hi.end(), hi);
    return MLP_OK;
}

mlp_status mlp_set_guard(mlp_ctx *c, float margin)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (isnan(margin) || isinf(margin)) return arg_fail(c, "margin must be finite");
    if (margin < 0.0f) {
        c->margin = -1.0f;
        return MLP_OK;
    }
    if (!c->cfg.residual_from) return arg_fail(c, "the guard's fallback is the residual base: set residual_from");
    if (c->lo.empty()) return MLP_ERR_STATE;
    c->margin = margin;
    return upload_guard(c);
}

mlp_status mlp_guard_count(mlp_ctx *c, uint64_t out[2])
{
    if (!c || !out) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    unsigned long long n = 0;
    MLPCHK(c, hipMemcpyAsync(&n, c->gcount, sizeof(n), hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = c->guarded_rows;
    out[1] = (uint64_t)n;
    return MLP_OK;
}

mlp_status mlp_gradients(mlp_ctx *c, const float *X, const float *Y, uint32_t m, float *grad, double *loss)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    mlp_status st = check_batch(c, X, m);
    if (st != MLP_OK) return st;
    if (!Y || !grad) return arg_fail(c, "null array");
    forward(c, X, m);
    backward(c, X, Y, m);
    MLPCHK(c, hipGetLastError());
    MLPCHK(c, hipMemcpyAsync(grad, c->grad, c->P * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    double l = 0.0;
    MLPCHK(c, hipMemcpyAsync(&l, c->loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = l;
    return isfinite(l) ? MLP_OK : MLP_ERR_NONFINITE;
}

mlp_status mlp_adam_step(mlp_ctx *c, const float *grad, size_t n, float lr)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!grad || n != c->P || !(lr >= 0.f) || !isfinite(lr)) return arg_fail(c, "bad gradient or rate");
    MLPCHK(c, hipMemcpyAsync(c->grad, grad, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    const mlp_status st = adam(c, lr);
    if (st != MLP_OK) return st;
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

mlp_status mlp_train_step(mlp_ctx *c, const float *X, const float *Y, uint32_t m, float lr)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    mlp_status st = check_batch(c, X, m);
    if (st != MLP_OK) return st;
    if (!Y || !(lr >= 0.f) || !isfinite(lr)) return arg_fail(c, "null targets or bad rate");
    forward(c, X, m);
    backward(c, X, Y, m);
    return adam(c, lr);
}

mlp_status mlp_last_loss(mlp_ctx *c, double *loss)
{
    if (!c || !loss) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    MLPCHK(c, hipMemcpyAsync(loss, c->loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return isfinite(*loss) ? MLP_OK : MLP_ERR_NONFINITE;
}

static PredictArgs predict_args(mlp_ctx *c, const float *x, float *y)
{
    PredictArgs a{};
    a.x = x;
    a.y = y;
    a.wb = c->wb;
    a.w = c->w;
    a.mu_x = c->mu_x;
    a.sd_x = c->sd_x;
    a.mu_y = c->mu_y;
    a.sd_y = c->sd_y;
    a.n_in = c->cfg.n_in;
    a.k0 = k0_of(c->cfg.n_in);
    a.n_out = c->cfg.n_out;
    a.hidden = c->H;
    a.layers = c->L;
    a.res_col0 = c->cfg.residual_from ? (int32_t)c->cfg.residual_from - 1 : -1;
    a.guard = guard_of(c);
    if (a.guard.a) c->guarded_rows += 1;
    return a;
}

mlp_status mlp_predict_one_device(mlp_ctx *c, const float *x, float *y)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!x || !y) return arg_fail(c, "null array");
    launch_predict_one(c->stream, predict_args(c, x, y));
    MLPCHK(c, hipGetLastError());
    return MLP_OK;
}

mlp_status mlp_predict_one(mlp_ctx *c, const float *x, float *y)
{
    if (!c) return MLP_ERR_ARG;
    if (c->dead) return MLP_ERR_STATE;
    if (!x || !y) return arg_fail(c, "null array");
    MLPCHK(c, hipMemcpyAsync(c->px, x, c->cfg.n_in * sizeof(float), hipMemcpyHostToDevice, c->stream));
    launch_predict_one(c->stream, predict_args(c, c->px, c->py));
    MLPCHK(c, hipGetLastError());
    MLPCHK(c, hipMemcpyAsync(y, c->py, c->cfg.n_out * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    MLPCHK(c, hipStreamSynchronize(c->stream));
    return MLP_OK;
}

mlp_status mlp_gemm_bf16(void *hip_stream, int a_layout, int b_layout, const uint16_t *A, uint32_t lda,
                         const uint16_t *B, uint32_t ldb, uint32_t M, uint32_t N, uint32_t K, float *C, uint32_t ldc)
{
    if ((a_layout != 0 && a_layout != 1) || (b_layout != 0 && b_layout != 1) || !A || !B || !C) return MLP_ERR_ARG;
    if (lda % 8 || ldb % 8 || ((uintptr_t)A & 15u) || ((uintptr_t)B & 15u) || ldc < N) return MLP_ERR_ARG;
    if ((a_layout == LD_K ? lda < K : lda < M) || (b_layout == LD_K ? ldb < K : ldb < N)) return MLP_ERR_ARG;
    GemmArgs g{};
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.k_split = (K + kTileK - 1) / kTileK * kTileK;
    if (!g.k_split) g.k_split = kTileK;
    g.C = C;
    g.ldc = ldc;
    if (!launch_gemm((hipStream_t)hip_stream, a_layout, b_layout, EPI_PARTIAL, g, 1)) return MLP_ERR_ARG;
    return hipGetLastError() == hipSuccess ? MLP_OK : MLP_ERR_DEVICE;
}

mlp_status mlp_destroy(mlp_ctx *c)
{
    if (!c) return MLP_OK;
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return MLP_OK;
}

const char *mlp_last_error(const mlp_ctx *c) { return c ? c->last_error.c_str() : "null context"; }

}  // extern "C"
