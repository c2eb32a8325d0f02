// surrogate.cpp -- host runtime of the learned coarse step (rod_surrogate.h):
// parameter layout, MLP workspace, forward / gradient / Adam drivers.
#include "rod_surrogate.h"
#include "mlp_internal.h"
#include "rod_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

namespace {

int sfail(int code, const std::string &msg) { return rodk::set_error(code, msg); }

#define SHIPCHK(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return sfail(e_ == hipErrorOutOfMemory ? ROD_ENOMEM : ROD_EDEVICE,               \
                         std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

constexpr int NL = 4;
constexpr int KDIM[NL] = {ROD_SURROGATE_INPUTS, 256, 256, 256};
constexpr int NDIM[NL] = {256, 256, 256, ROD_SURROGATE_OUTPUTS};   // external
constexpr int NPAD[NL] = {256, 256, 256, 16};                        // internal
constexpr int NOUT_LD = 16;

struct Layout {
    int64_t w[NL], b[NL], total;
};

Layout internal_layout()
{
    Layout L{};
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        L.w[l] = o;
        o += (int64_t)KDIM[l] * NPAD[l];
        L.b[l] = o;
        o += NPAD[l];
    }
    L.total = o;
    return L;
}

}  // namespace

struct rod_surrogate {
    int k = 32;
    int max_rows = 65536;
    Layout lay{};
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;   // FP32, internal layout
    __bf16 *wb = nullptr;                                           // BF16 weights (internal layout)
    int64_t adam_t = 0;
    // workspace (max_rows rows)
    float *Z[3] = {nullptr, nullptr, nullptr};
    __bf16 *Ab[3] = {nullptr, nullptr, nullptr};
    float *Y = nullptr, *dY = nullptr, *dZa = nullptr, *dZb = nullptr;
    float *partial = nullptr, *loss = nullptr;
};

namespace {

int refresh_bf16(rod_surrogate *s, hipStream_t st)
{
    hipError_t e = mlpk::to_bf16(s->w, s->wb, s->lay.total, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("to_bf16: ") + hipGetErrorString(e));
    return ROD_OK;
}

// Forward over rows [0, M) of x (M <= max_rows), keeping Z and BF16 activations.
int forward_chunk(rod_surrogate *s, const __bf16 *x, int M, hipStream_t st)
{
    const __bf16 *in = x;
    for (int l = 0; l < NL; ++l) {
        mlpk::GemmArgs a{};
        a.A = in;
        a.lda = KDIM[l];
        a.B = s->wb + s->lay.w[l];
        a.ldb = NPAD[l];
        a.M = M;
        a.N = NPAD[l];
        a.K = KDIM[l];
        a.bias = s->w + s->lay.b[l];
        hipError_t e;
        if (l < NL - 1) {
            a.C = s->Z[l];
            a.act = s->Ab[l];
            a.ldc = NPAD[l];
            e = mlpk::gemm_forward(a, mlpk::EPI_BIAS_SILU, st);
            in = s->Ab[l];
        } else {
            a.C = s->Y;
            a.ldc = NOUT_LD;
            e = mlpk::gemm_forward(a, mlpk::EPI_BIAS, st);
        }
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("forward gemm: ") + hipGetErrorString(e));
    }
    return ROD_OK;
}

// Loss and gradients (internal layout, into s->g) for one chunk.
int gradient_chunk(rod_surrogate *s, const __bf16 *x, const float *t, const float *mask, int M,
                   hipStream_t st)
{
    int rc = forward_chunk(s, x, M, st);
    if (rc) return rc;
    hipError_t e = mlpk::mse_grad(s->Y, t, mask, s->dY, s->partial, M, ROD_SURROGATE_OUTPUTS, NOUT_LD, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("mse_grad: ") + hipGetErrorString(e));
    // loss = sum(mask * e^2) / (M * 12): masked entries still count in the mean
    e = mlpk::sum_partials(s->partial, mlpk::mse_partials(M, NOUT_LD), 1.0f / (float)(M * ROD_SURROGATE_OUTPUTS),
                           s->loss, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("loss: ") + hipGetErrorString(e));
    const float *dZ = s->dY;
    int ldz = NOUT_LD;
    float *bufs[2] = {s->dZa, s->dZb};
    for (int l = NL - 1; l >= 0; --l) {
        // dW_l = A_{l-1}^T dZ_l ; db_l = colsum(dZ_l)
        mlpk::GemmArgs a{};
        a.A = l > 0 ? (const void *)s->Ab[l - 1] : (const void *)x;
        a.lda = KDIM[l];
        a.B = dZ;
        a.ldb = ldz;
        a.M = KDIM[l];
        a.N = NPAD[l];
        a.K = M;
        a.C = s->g + s->lay.w[l];
        a.ldc = NPAD[l];
        e = mlpk::gemm_backward_weight(a, st);
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("dW gemm: ") + hipGetErrorString(e));
        e = mlpk::colsum(dZ, M, NPAD[l], ldz, s->g + s->lay.b[l], st);
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("db: ") + hipGetErrorString(e));
        if (l == 0) break;
        // dZ_{l-1} = (dZ_l W_l^T) * silu'(Z_{l-1})
        mlpk::GemmArgs b{};
        b.A = dZ;
        b.lda = ldz;
        b.B = s->wb + s->lay.w[l];
        b.ldb = NPAD[l];
        b.M = M;
        b.N = KDIM[l];
        b.K = NPAD[l];
        float *out = bufs[l & 1];
        b.C = out;
        b.ldc = KDIM[l];
        b.zsave = s->Z[l - 1];
        e = mlpk::gemm_backward_data(b, mlpk::EPI_DSILU, st);
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("dA gemm: ") + hipGetErrorString(e));
        dZ = out;
        ldz = KDIM[l];
    }
    return ROD_OK;
}

void internal_to_external(const rod_surrogate *s, const std::vector<float> &in, float *out)
{
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        for (int k = 0; k < KDIM[l]; ++k)
            for (int n = 0; n < NDIM[l]; ++n) out[o++] = in[s->lay.w[l] + (int64_t)k * NPAD[l] + n];
        for (int n = 0; n < NDIM[l]; ++n) out[o++] = in[s->lay.b[l] + n];
    }
}

void external_to_internal(const rod_surrogate *s, const float *in, std::vector<float> &out)
{
    out.assign(s->lay.total, 0.0f);
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        for (int k = 0; k < KDIM[l]; ++k)
            for (int n = 0; n < NDIM[l]; ++n) out[s->lay.w[l] + (int64_t)k * NPAD[l] + n] = in[o++];
        for (int n = 0; n < NDIM[l]; ++n) out[s->lay.b[l] + n] = in[o++];
    }
}

}  // namespace

extern "C" {

int rod_surrogate_create(const rod_surrogate_desc *d, rod_surrogate **out)
{
    if (!d || !out) return sfail(ROD_EINVAL, "desc or out is NULL");
    *out = nullptr;
    if (d->k_substeps <= 0) return sfail(ROD_EINVAL, "k_substeps must be > 0");
    if (d->max_rows < 0 || d->max_rows % 64) return sfail(ROD_EINVAL, "max_rows must be 0 or a positive multiple of 64");
    auto *s = new (std::nothrow) rod_surrogate();
    if (!s) return sfail(ROD_ENOMEM, "host allocation failed");
    s->k = d->k_substeps;
    s->max_rows = d->max_rows ? d->max_rows : 65536;
    s->lay = internal_layout();
    const int64_t P = s->lay.total;
    const size_t R = (size_t)s->max_rows;
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    alloc((void **)&s->w, P * 4);
    alloc((void **)&s->m, P * 4);
    alloc((void **)&s->v, P * 4);
    alloc((void **)&s->g, P * 4);
    alloc((void **)&s->wb, P * 2);
    for (int l = 0; l < 3; ++l) {
        alloc((void **)&s->Z[l], R * 256 * 4);
        alloc((void **)&s->Ab[l], R * 256 * 2);
    }
    alloc((void **)&s->Y, R * NOUT_LD * 4);
    alloc((void **)&s->dY, R * NOUT_LD * 4);
    alloc((void **)&s->dZa, R * 256 * 4);
    alloc((void **)&s->dZb, R * 256 * 4);
    alloc((void **)&s->partial, (size_t)mlpk::mse_partials(s->max_rows, NOUT_LD) * 4);
    alloc((void **)&s->loss, 4);
    if (e != hipSuccess) {
        rod_surrogate_destroy(s);
        return sfail(e == hipErrorOutOfMemory ? ROD_ENOMEM : ROD_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    // initialisation (same rule as the oracle's; the draws are this library's own)
    std::vector<float> ext(ROD_SURROGATE_PARAMS, 0.0f);
    std::mt19937_64 rng(d->seed);
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        const double a = std::sqrt(6.0 / KDIM[l]);
        std::uniform_real_distribution<double> U(-a, a);
        for (int64_t i = 0; i < (int64_t)KDIM[l] * NDIM[l]; ++i) ext[o++] = (float)U(rng);
        o += NDIM[l];
    }
    int rc = rod_surrogate_set_params(s, ext.data());
    if (rc) {
        rod_surrogate_destroy(s);
        return rc;
    }
    *out = s;
    return ROD_OK;
}

void rod_surrogate_destroy(rod_surrogate *s)
{
    if (!s) return;
    (void)hipFree(s->w);
    (void)hipFree(s->m);
    (void)hipFree(s->v);
    (void)hipFree(s->g);
    (void)hipFree(s->wb);
    for (int l = 0; l < 3; ++l) {
        (void)hipFree(s->Z[l]);
        (void)hipFree(s->Ab[l]);
    }
    (void)hipFree(s->Y);
    (void)hipFree(s->dY);
    (void)hipFree(s->dZa);
    (void)hipFree(s->dZb);
    (void)hipFree(s->partial);
    (void)hipFree(s->loss);
    delete s;
}

int rod_surrogate_set_params(rod_surrogate *s, const float *params)
{
    if (!s || !params) return sfail(ROD_EINVAL, "handle or params is NULL");
    std::vector<float> in;
    external_to_internal(s, params, in);
    SHIPCHK(hipMemcpy(s->w, in.data(), in.size() * 4, hipMemcpyHostToDevice));
    SHIPCHK(hipMemset(s->m, 0, in.size() * 4));
    SHIPCHK(hipMemset(s->v, 0, in.size() * 4));
    SHIPCHK(hipMemset(s->g, 0, in.size() * 4));
    s->adam_t = 0;
    int rc = refresh_bf16(s, nullptr);
    if (rc) return rc;
    SHIPCHK(hipDeviceSynchronize());
    return ROD_OK;
}

int rod_surrogate_get_params(rod_surrogate *s, float *params)
{
    if (!s || !params) return sfail(ROD_EINVAL, "handle or params is NULL");
    std::vector<float> in(s->lay.total);
    SHIPCHK(hipDeviceSynchronize());
    SHIPCHK(hipMemcpy(in.data(), s->w, in.size() * 4, hipMemcpyDeviceToHost));
    internal_to_external(s, in, params);
    return ROD_OK;
}

int rod_surrogate_forward(rod_surrogate *s, const void *x, int64_t M, float *y, void *stream)
{
    if (!s || !x || !y) return sfail(ROD_EINVAL, "NULL argument");
    if (M < 0) return sfail(ROD_EINVAL, "M must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    for (int64_t r0 = 0; r0 < M; r0 += s->max_rows) {
        const int rows = (int)std::min<int64_t>(s->max_rows, M - r0);
        int rc = forward_chunk(s, (const __bf16 *)x + r0 * ROD_SURROGATE_INPUTS, rows, st);
        if (rc) return rc;
        SHIPCHK(hipMemcpy2DAsync(y + r0 * ROD_SURROGATE_OUTPUTS, ROD_SURROGATE_OUTPUTS * 4, s->Y, NOUT_LD * 4,
                                 ROD_SURROGATE_OUTPUTS * 4, rows, hipMemcpyDeviceToDevice, st));
    }
    return ROD_OK;
}

int rod_surrogate_gradients(rod_surrogate *s, const void *x, const float *t, const float *mask, int64_t M,
                            float *grads, float *loss, void *stream)
{
    if (!s || !x || !t || !grads) return sfail(ROD_EINVAL, "NULL argument");
    if (M <= 0 || M > s->max_rows || M % 32) return sfail(ROD_EINVAL, "M must be in (0, max_rows], a multiple of 32");
    hipStream_t st = (hipStream_t)stream;
    int rc = gradient_chunk(s, (const __bf16 *)x, t, mask, (int)M, st);
    if (rc) return rc;
    std::vector<float> gi(s->lay.total);
    SHIPCHK(hipMemcpyAsync(gi.data(), s->g, gi.size() * 4, hipMemcpyDeviceToHost, st));
    float l = 0;
    SHIPCHK(hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, st));
    SHIPCHK(hipStreamSynchronize(st));
    internal_to_external(s, gi, grads);
    if (loss) *loss = l;
    return ROD_OK;
}

int rod_surrogate_train_step(rod_surrogate *s, const void *x, const float *t, const float *mask, int64_t M,
                             float lr, float *loss, void *stream)
{
    if (!s || !x || !t) return sfail(ROD_EINVAL, "NULL argument");
    if (M <= 0 || M > s->max_rows || M % 32) return sfail(ROD_EINVAL, "M must be in (0, max_rows], a multiple of 32");
    if (!(lr >= 0.0f)) return sfail(ROD_EINVAL, "lr must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    int rc = gradient_chunk(s, (const __bf16 *)x, t, mask, (int)M, st);
    if (rc) return rc;
    s->adam_t += 1;
    hipError_t e = mlpk::adam(s->w, s->m, s->v, s->g, s->lay.total, lr, 0.9f, 0.999f, 1e-8f, s->adam_t, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("adam: ") + hipGetErrorString(e));
    rc = refresh_bf16(s, st);
    if (rc) return rc;
    if (loss) {
        SHIPCHK(hipMemcpyAsync(loss, s->loss, 4, hipMemcpyDeviceToHost, st));
        SHIPCHK(hipStreamSynchronize(st));
    }
    return ROD_OK;
}

}  // extern "C"
