// surrogate.cpp -- host runtime of the learned coarse step (rod_surrogate.h):
// parameter layout, MLP workspace, forward / gradient / Adam drivers.
#include "rod_surrogate.h"
#include "mlp_internal.h"
#include "rod_internal.h"
#include "surrogate_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
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
    // standardisation (device and host copies)
    float *norm = nullptr;                   // mu_x[96] sd_x[96] mu_t[12] sd_t[12]
    std::vector<float> norm_h;
    // per-batch window context
    const rod_batch *ctx_batch = nullptr;
    int64_t ctx_rods = -1;
    int64_t n_windows = 0, n_elems = 0;
    int32_t *win_rod = nullptr, *elem_rod = nullptr;
    int64_t *win_first = nullptr, *elem_first = nullptr;
    float *rodf = nullptr, *disp = nullptr;
    void *saved = nullptr;                   // state copy for targets / the judge
    size_t saved_bytes = 0;
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


// ------------------------------------------------------------------ windows

void free_ctx(rod_surrogate *s)
{
    (void)hipFree(s->win_rod);
    (void)hipFree(s->elem_rod);
    (void)hipFree(s->win_first);
    (void)hipFree(s->elem_first);
    (void)hipFree(s->rodf);
    (void)hipFree(s->disp);
    (void)hipFree(s->saved);
    s->win_rod = s->elem_rod = nullptr;
    s->win_first = s->elem_first = nullptr;
    s->rodf = s->disp = nullptr;
    s->saved = nullptr;
    s->saved_bytes = 0;
    s->ctx_batch = nullptr;
    s->ctx_rods = -1;
}

// Window and element maps, per-rod feature constants and scratch for batch b.
int ensure_ctx(rod_surrogate *s, rod_batch *b, rodk::BatchView &v)
{
    int rc = rodk::batch_view(b, &v);
    if (rc) return rc;
    if (v.precision != ROD_F32) return sfail(ROD_EUNSUPPORTED, "the learned coarse step runs on FP32 batches");
    if (s->ctx_batch == b && s->ctx_rods == v.n_rods) return ROD_OK;
    free_ctx(s);
    const int R = v.n_rods;
    std::vector<int32_t> wr, er;
    std::vector<int64_t> wf(R), ef(R);
    std::vector<float> rf((size_t)R * surk::NRF);
    int64_t w = 0, e = 0;
    for (int r = 0; r < R; ++r) {
        const int n = v.n[r];
        wf[r] = w;
        ef[r] = e;
        for (int i = 0; i <= n; ++i) wr.push_back(r);
        for (int i = 0; i < n; ++i) er.push_back(r);
        w += n + 1;
        e += n;
        const double A = M_PI * v.radius[r] * v.radius[r], I = M_PI * std::pow(v.radius[r], 4) / 4.0;
        float *f = &rf[(size_t)r * surk::NRF];
        f[surk::RF_LOGE] = (float)std::log10(v.youngs[r] / 1e6);
        f[surk::RF_RADIUS] = (float)v.radius[r];
        f[surk::RF_SQRT_RHOA_EI] = (float)std::sqrt(v.density[r] * A / (v.youngs[r] * I));
        f[surk::RF_ALPHA] = (float)v.shear_coeff[r];
        f[surk::RF_CLAMP0] = (float)v.bc_start[r];
        f[surk::RF_AMP] = (float)(v.couple_amp[3 * r] / (double)surk::AMP_SCALE);
        f[surk::RF_FREQ] = (float)v.couple_freq[r];
        f[surk::RF_PHASE] = (float)v.couple_phase[r];
    }
    s->n_windows = w;
    s->n_elems = e;
    hipError_t err = hipSuccess;
    auto up = [&](void **p, const void *src, size_t bytes) {
        if (err == hipSuccess) err = hipMalloc(p, bytes);
        if (err == hipSuccess && src) err = hipMemcpy(*p, src, bytes, hipMemcpyHostToDevice);
    };
    up((void **)&s->win_rod, wr.data(), wr.size() * 4);
    up((void **)&s->elem_rod, er.data(), er.size() * 4);
    up((void **)&s->win_first, wf.data(), wf.size() * 8);
    up((void **)&s->elem_first, ef.data(), ef.size() * 8);
    up((void **)&s->rodf, rf.data(), rf.size() * 4);
    up((void **)&s->disp, nullptr, (size_t)w * 3 * 4);
    s->saved_bytes = v.state_bytes + v.tail_bytes;
    up(&s->saved, nullptr, s->saved_bytes);
    if (err != hipSuccess) {
        free_ctx(s);
        return sfail(err == hipErrorOutOfMemory ? ROD_ENOMEM : ROD_EDEVICE, std::string("window context: ") + hipGetErrorString(err));
    }
    s->ctx_batch = b;
    s->ctx_rods = R;
    return ROD_OK;
}

surk::WinArgs win_args(const rod_surrogate *s, const rodk::BatchView &v)
{
    surk::WinArgs a{};
    a.B = v.f32;
    a.win_rod = s->win_rod;
    a.win_first = s->win_first;
    a.rodf = s->rodf;
    a.n_windows = s->n_windows;
    a.tau = (float)(s->k * v.dt);
    a.time = v.time;
    return a;
}

// A copy of the batch's state (and tail) in s->saved, seen as a DevBatch.
rodk::DevBatch<float> saved_batch(const rod_surrogate *s, const rodk::BatchView &v)
{
    rodk::DevBatch<float> d = v.f32;
    d.state = (float *)s->saved;
    d.tail = (float *)((char *)s->saved + v.state_bytes);
    return d;
}

int save_state(rod_surrogate *s, const rodk::BatchView &v, hipStream_t st)
{
    SHIPCHK(hipMemcpyAsync(s->saved, v.f32.state, v.state_bytes, hipMemcpyDeviceToDevice, st));
    SHIPCHK(hipMemcpyAsync((char *)s->saved + v.state_bytes, v.f32.tail, v.tail_bytes, hipMemcpyDeviceToDevice, st));
    return ROD_OK;
}

// Forward and loss only (no backward), for validation.
int loss_chunk(rod_surrogate *s, const __bf16 *x, const float *t, const float *mask, int M, hipStream_t st)
{
    int rc = forward_chunk(s, x, M, st);
    if (rc) return rc;
    hipError_t e = mlpk::mse_grad(s->Y, t, mask, s->dY, s->partial, M, ROD_SURROGATE_OUTPUTS, NOUT_LD, st);
    if (e == hipSuccess)
        e = mlpk::sum_partials(s->partial, mlpk::mse_partials(M, NOUT_LD), 1.0f / (float)(M * ROD_SURROGATE_OUTPUTS),
                               s->loss, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("loss: ") + hipGetErrorString(e));
    return ROD_OK;
}

int upload_norm(rod_surrogate *s)
{
    SHIPCHK(hipMemcpy(s->norm, s->norm_h.data(), s->norm_h.size() * 4, hipMemcpyHostToDevice));
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
    alloc((void **)&s->norm, (2 * ROD_SURROGATE_INPUTS + 2 * ROD_SURROGATE_OUTPUTS) * 4);
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
    if (!rc) {
        s->norm_h.assign(2 * ROD_SURROGATE_INPUTS + 2 * ROD_SURROGATE_OUTPUTS, 0.0f);
        for (int i = 0; i < ROD_SURROGATE_INPUTS; ++i) s->norm_h[ROD_SURROGATE_INPUTS + i] = 1.0f;
        for (int i = 0; i < ROD_SURROGATE_OUTPUTS; ++i)
            s->norm_h[2 * ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS + i] = 1.0f;
        rc = upload_norm(s);
    }
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
    (void)hipFree(s->norm);
    free_ctx(s);
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


int rod_surrogate_features(rod_surrogate *s, rod_batch *b, float *features, void *stream)
{
    if (!s || !b || !features) return sfail(ROD_EINVAL, "NULL argument");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    hipError_t e = surk::features(win_args(s, v), features, nullptr, nullptr, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("features: ") + hipGetErrorString(e));
    return ROD_OK;
}

int rod_surrogate_collect(rod_surrogate *s, rod_batch *b, float *features, float *targets, float *mask, void *stream)
{
    if (!s || !b || !features || !targets || !mask) return sfail(ROD_EINVAL, "NULL argument");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = surk::features(win_args(s, v), features, nullptr, nullptr, nullptr, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("features: ") + hipGetErrorString(e));
    if ((rc = save_state(s, v, st))) return rc;
    if ((rc = rod_step(b, s->k, stream))) return rc;
    rodk::BatchView v1;
    if ((rc = rodk::batch_view(b, &v1))) return rc;
    e = surk::targets(win_args(s, v1), saved_batch(s, v), targets, mask, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("targets: ") + hipGetErrorString(e));
    return ROD_OK;
}

int rod_surrogate_apply(rod_surrogate *s, rod_batch *b, const float *deltas, void *stream)
{
    if (!s || !b || !deltas) return sfail(ROD_EINVAL, "NULL argument");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = surk::apply(win_args(s, v), deltas, ROD_SURROGATE_OUTPUTS, nullptr, nullptr, nullptr, s->disp,
                               s->elem_rod, s->elem_first, s->n_elems, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("apply: ") + hipGetErrorString(e));
    return rodk::batch_advance_clock(b, s->k, st);
}

int rod_surrogate_set_normalization(rod_surrogate *s, const float *mu_x, const float *sd_x, const float *mu_t,
                                    const float *sd_t)
{
    if (!s || !mu_x || !sd_x || !mu_t || !sd_t) return sfail(ROD_EINVAL, "NULL argument");
    for (int i = 0; i < ROD_SURROGATE_INPUTS; ++i)
        if (!(sd_x[i] > 0) || !std::isfinite(mu_x[i])) return sfail(ROD_EINVAL, "sd_x must be > 0, mu_x finite");
    for (int i = 0; i < ROD_SURROGATE_OUTPUTS; ++i)
        if (!(sd_t[i] > 0) || !std::isfinite(mu_t[i])) return sfail(ROD_EINVAL, "sd_t must be > 0, mu_t finite");
    std::copy(mu_x, mu_x + ROD_SURROGATE_INPUTS, s->norm_h.begin());
    std::copy(sd_x, sd_x + ROD_SURROGATE_INPUTS, s->norm_h.begin() + ROD_SURROGATE_INPUTS);
    std::copy(mu_t, mu_t + ROD_SURROGATE_OUTPUTS, s->norm_h.begin() + 2 * ROD_SURROGATE_INPUTS);
    std::copy(sd_t, sd_t + ROD_SURROGATE_OUTPUTS, s->norm_h.begin() + 2 * ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS);
    return upload_norm(s);
}

int rod_surrogate_get_normalization(rod_surrogate *s, float *mu_x, float *sd_x, float *mu_t, float *sd_t)
{
    if (!s) return sfail(ROD_EINVAL, "NULL argument");
    const float *h = s->norm_h.data();
    if (mu_x) std::copy(h, h + ROD_SURROGATE_INPUTS, mu_x);
    if (sd_x) std::copy(h + ROD_SURROGATE_INPUTS, h + 2 * ROD_SURROGATE_INPUTS, sd_x);
    if (mu_t) std::copy(h + 2 * ROD_SURROGATE_INPUTS, h + 2 * ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS, mu_t);
    if (sd_t) std::copy(h + 2 * ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS, h + s->norm_h.size(), sd_t);
    return ROD_OK;
}

int rod_surrogate_train(rod_surrogate *s, rod_batch *b, const rod_train_desc *d, float *epoch_loss, float *val_loss,
                        void *stream)
{
    if (!s || !b || !d) return sfail(ROD_EINVAL, "NULL argument");
    if (d->warmup_steps < 0 || d->n_samples < 1 || d->sample_stride < s->k || d->epochs < 1 || d->batch_rows <= 0
        || d->batch_rows % 64 || d->batch_rows > s->max_rows || !(d->lr > 0) || !(d->lr_min >= 0)
        || !(d->val_fraction >= 0 && d->val_fraction < 1))
        return sfail(ROD_EINVAL, "invalid training descriptor");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t W = s->n_windows;
    const int64_t N = W * d->n_samples;
    // ---- data: plain trajectories
    float *F = nullptr, *T = nullptr, *Mk = nullptr;
    double *stats = nullptr;
    __bf16 *xb = nullptr;
    float *tb = nullptr, *mb = nullptr, *lhist = nullptr;
    int64_t *idx = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(F); (void)hipFree(T); (void)hipFree(Mk); (void)hipFree(stats);
        (void)hipFree(xb); (void)hipFree(tb); (void)hipFree(mb); (void)hipFree(idx); (void)hipFree(lhist);
    };
    const int B = d->batch_rows;
    const int64_t n_val = (int64_t)std::llround(d->val_fraction * (double)N);
    const int64_t n_tr = ((N - n_val) / B) * B;
    const int64_t steps_per_epoch = n_tr / B;
    const int64_t total_steps = steps_per_epoch * d->epochs;
    if (steps_per_epoch < 1) return sfail(ROD_EINVAL, "fewer training windows than one minibatch");
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    alloc((void **)&F, (size_t)N * ROD_SURROGATE_INPUTS * 4);
    alloc((void **)&T, (size_t)N * ROD_SURROGATE_OUTPUTS * 4);
    alloc((void **)&Mk, (size_t)N * ROD_SURROGATE_OUTPUTS * 4);
    alloc((void **)&stats, 3 * (ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS) * 8);
    alloc((void **)&xb, (size_t)B * ROD_SURROGATE_INPUTS * 2);
    alloc((void **)&tb, (size_t)B * ROD_SURROGATE_OUTPUTS * 4);
    alloc((void **)&mb, (size_t)B * ROD_SURROGATE_OUTPUTS * 4);
    alloc((void **)&idx, (size_t)std::max<int64_t>(N, 1) * 8);
    alloc((void **)&lhist, (size_t)std::max<int64_t>(total_steps, 1) * 4);
    if (e != hipSuccess) {
        cleanup();
        return sfail(e == hipErrorOutOfMemory ? ROD_ENOMEM : ROD_EDEVICE, std::string("training buffers: ") + hipGetErrorString(e));
    }
#define TRY(x)                \
    do {                      \
        int rc_ = (x);        \
        if (rc_) {            \
            cleanup();        \
            return rc_;       \
        }                     \
    } while (0)
#define TRYH(x)                                                                                   \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) {                                                                   \
            cleanup();                                                                            \
            return sfail(ROD_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));            \
        }                                                                                         \
    } while (0)
    if (d->warmup_steps > 0) TRY(rod_step(b, d->warmup_steps, stream));
    for (int i = 0; i < d->n_samples; ++i) {
        TRY(rod_surrogate_collect(s, b, F + (size_t)i * W * ROD_SURROGATE_INPUTS,
                                  T + (size_t)i * W * ROD_SURROGATE_OUTPUTS, Mk + (size_t)i * W * ROD_SURROGATE_OUTPUTS,
                                  stream));
        if (i + 1 < d->n_samples && d->sample_stride > s->k) TRY(rod_step(b, d->sample_stride - s->k, stream));
    }
    // ---- standardisation from the whole data set
    TRYH(surk::colstats(F, nullptr, N, ROD_SURROGATE_INPUTS, stats, st));
    TRYH(surk::colstats(T, Mk, N, ROD_SURROGATE_OUTPUTS, stats + 3 * ROD_SURROGATE_INPUTS, st));
    std::vector<double> hs(3 * (ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS));
    TRYH(hipMemcpyAsync(hs.data(), stats, hs.size() * 8, hipMemcpyDeviceToHost, st));
    TRYH(hipStreamSynchronize(st));
    std::vector<float> mu(ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS), sd(mu.size());
    for (size_t j = 0; j < mu.size(); ++j) {
        const double c = hs[3 * j], sm = hs[3 * j + 1], sq = hs[3 * j + 2];
        const double m = c > 0 ? sm / c : 0.0;
        const double var = c > 0 ? std::max(0.0, sq / c - m * m) : 0.0;
        double sdv = std::sqrt(var);
        if (!(sdv > 1e-6 * std::max(1.0, std::fabs(m)))) sdv = 1.0;   // constant column
        mu[j] = (float)m;
        sd[j] = (float)sdv;
    }
    TRY(rod_surrogate_set_normalization(s, mu.data(), sd.data(), mu.data() + ROD_SURROGATE_INPUTS,
                                        sd.data() + ROD_SURROGATE_INPUTS));
    const float *mux = s->norm, *sdx = s->norm + ROD_SURROGATE_INPUTS;
    const float *mut = s->norm + 2 * ROD_SURROGATE_INPUTS, *sdt = mut + ROD_SURROGATE_OUTPUTS;
    // ---- split and train
    std::mt19937_64 rng(d->seed);
    std::vector<int64_t> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<int64_t> val(perm.begin(), perm.begin() + n_val), tr(perm.begin() + n_val, perm.end());
    int64_t step = 0;
    for (int ep = 0; ep < d->epochs; ++ep) {
        std::shuffle(tr.begin(), tr.end(), rng);
        TRYH(hipMemcpyAsync(idx, tr.data(), n_tr * 8, hipMemcpyHostToDevice, st));
        for (int64_t bi = 0; bi < steps_per_epoch; ++bi, ++step) {
            TRYH(surk::gather_rows(F, T, Mk, idx + bi * B, B, mux, sdx, mut, sdt, xb, tb, mb, st));
            TRY(gradient_chunk(s, xb, tb, mb, B, st));
            const double ph = total_steps > 1 ? (double)step / (double)(total_steps - 1) : 1.0;
            const float lr = (float)(d->lr_min + 0.5 * (d->lr - d->lr_min) * (1.0 + std::cos(M_PI * ph)));
            s->adam_t += 1;
            TRYH(mlpk::adam(s->w, s->m, s->v, s->g, s->lay.total, lr, 0.9f, 0.999f, 1e-8f, s->adam_t, st));
            TRY(refresh_bf16(s, st));
            TRYH(hipMemcpyAsync(lhist + step, s->loss, 4, hipMemcpyDeviceToDevice, st));
        }
        TRYH(hipStreamSynchronize(st));   // the host index buffer is reused next epoch
    }
    std::vector<float> lh(total_steps);
    TRYH(hipMemcpyAsync(lh.data(), lhist, total_steps * 4, hipMemcpyDeviceToHost, st));
    // ---- validation
    double vsum = 0.0;
    int64_t vrows = 0;
    if (n_val >= B) {
        TRYH(hipMemcpyAsync(idx, val.data(), n_val * 8, hipMemcpyHostToDevice, st));
        for (int64_t v0 = 0; v0 + B <= n_val; v0 += B) {
            TRYH(surk::gather_rows(F, T, Mk, idx + v0, B, mux, sdx, mut, sdt, xb, tb, mb, st));
            TRY(loss_chunk(s, xb, tb, mb, B, st));
            float l = 0;
            TRYH(hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, st));
            TRYH(hipStreamSynchronize(st));
            vsum += (double)l * B;
            vrows += B;
        }
    }
    TRYH(hipStreamSynchronize(st));
    if (epoch_loss)
        for (int ep = 0; ep < d->epochs; ++ep) {
            double acc = 0;
            for (int64_t i = 0; i < steps_per_epoch; ++i) acc += lh[ep * steps_per_epoch + i];
            epoch_loss[ep] = (float)(acc / steps_per_epoch);
        }
    if (val_loss) *val_loss = vrows ? (float)(vsum / vrows) : NAN;
#undef TRY
#undef TRYH
    cleanup();
    return ROD_OK;
}

}  // extern "C"
