// surrogate.cpp -- host runtime of the learned coarse step (rod_surrogate.h):
// parameter layout, MLP workspace, forward / gradient / Adam routines, training, the coarse step and its judge.
#include "rod_surrogate.h"
#include "mlp_internal.h"
#include "rod_internal.h"
#include "surrogate_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
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
constexpr int64_t SPLIT_FLOATS = 512 * 64 * 64 + 256 * 256;   // split-reduction partials of the dW GEMMs

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
    __bf16 *frag = nullptr;                                         // BF16 weights as inference fragments
    bool frag_stale = true;                                         // wb changed since frag was packed
    int64_t adam_t = 0;
    // workspace (max_rows rows)
    float *Z[3] = {nullptr, nullptr, nullptr};
    __bf16 *Ab[3] = {nullptr, nullptr, nullptr};
    float *Y = nullptr, *dY = nullptr, *dZa = nullptr, *dZb = nullptr;
    float *partial = nullptr, *loss = nullptr;
    float *splitw = nullptr;                 // dW split-reduction partials
    // standardisation (device and host copies)
    float *norm = nullptr;                   // mu_x[96] sd_x[96] mu_t[12] sd_t[12]
    std::vector<float> norm_h;
    // per-batch window context
    const rod_batch *ctx_batch = nullptr;
    int64_t ctx_rods = -1;
    int64_t n_windows = 0, n_elems = 0;
    int n_max = 0;                           // longest rod of the context
    int32_t *win_rod = nullptr, *elem_rod = nullptr;
    int64_t *win_first = nullptr, *elem_first = nullptr;
    float *rodf = nullptr, *disp = nullptr;
    float2 *phase = nullptr;                 // [R] couple phase sin / cos
    void *saved = nullptr;                   // state copy for targets / the judge
    void *saved2 = nullptr;                  // perturbed start state of a noisy sample
    size_t saved_bytes = 0;
    // coarse stepping
    int32_t *plain = nullptr;                // device [R]: 1 = rod on the plain step
    std::vector<int32_t> plain_h;
    int32_t *plain_tiles = nullptr;          // device: tiles holding plain rods
    int n_plain_tiles = 0;
    __bf16 *xall = nullptr;                  // [W][96] standardised features
    float *yall = nullptr;                   // [W][16] network outputs
    rod_batch *judge = nullptr;              // plain re-runs of the sampled rods
    int judge_rods = 0;
    int32_t *jmap = nullptr, *jsel = nullptr;
    float *jerr = nullptr;
    double *jen = nullptr;                   // [2][m][5] energies of the sample and its plain re-run
    int64_t judge_windows_total = 0;
};

namespace {

// BF16 copies of the FP32 weights; the inference fragments are repacked
// lazily, before the next inference (training steps never need them).
int refresh_bf16(rod_surrogate *s, hipStream_t st)
{
    hipError_t e = mlpk::to_bf16(s->w, s->wb, s->lay.total, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("to_bf16: ") + hipGetErrorString(e));
    s->frag_stale = true;
    return ROD_OK;
}

int pack_if_stale(rod_surrogate *s, hipStream_t st)
{
    if (!s->frag_stale) return ROD_OK;
    mlpk::PackArgs p{};
    for (int l = 0; l < NL; ++l) {
        p.w_offset[l] = s->lay.w[l];
        p.ld[l] = NPAD[l];
    }
    hipError_t e = mlpk::pack_fragments(s->wb, p, s->frag, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("pack: ") + hipGetErrorString(e));
    s->frag_stale = false;
    return ROD_OK;
}

// One Adam step of every parameter with the BF16 copies refreshed in the same pass.
int adam_step(rod_surrogate *s, float lr, hipStream_t st)
{
    s->adam_t += 1;
    hipError_t e = mlpk::adam(s->w, s->m, s->v, s->g, s->lay.total, lr, 0.9f, 0.999f, 1e-8f, s->adam_t, s->wb, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("adam: ") + hipGetErrorString(e));
    s->frag_stale = true;
    return ROD_OK;
}

// Fused inference over M rows of standardised BF16 inputs into y ([M][ldy], ldy 16 or 12).
int infer(rod_surrogate *s, const __bf16 *x, int64_t M, float *y, int ldy, hipStream_t st)
{
    int rc = pack_if_stale(s, st);
    if (rc) return rc;
    mlpk::InferArgs a{};
    a.x = x;
    a.M = M;
    a.frag = s->frag;
    for (int l = 0; l < NL; ++l) a.bias[l] = s->w + s->lay.b[l];
    a.y = y;
    a.ldy = ldy;
    hipError_t e = mlpk::mlp_infer(a, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("inference: ") + hipGetErrorString(e));
    return ROD_OK;
}

// Forward over rows [0, M) of x (M <= max_rows), keeping Z and BF16 activations;
// the output rows ([M][16]) go to yout, or to the workspace when NULL.
int forward_chunk(rod_surrogate *s, const __bf16 *x, int M, hipStream_t st, float *yout = nullptr)
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
            a.C = yout ? yout : s->Y;
            a.ldc = NOUT_LD;
            e = mlpk::gemm_forward(a, mlpk::EPI_BIAS, st);
        }
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("forward gemm: ") + hipGetErrorString(e));
    }
    return ROD_OK;
}

// Loss and gradients (internal layout, into s->g) for one chunk.
int gradient_chunk(rod_surrogate *s, const __bf16 *x, const float *t, const float *mask, int M,
                   hipStream_t st, float *loss_out = nullptr)
{
    int rc = forward_chunk(s, x, M, st);
    if (rc) return rc;
    hipError_t e = mlpk::mse_grad(s->Y, t, mask, s->dY, s->partial, M, ROD_SURROGATE_OUTPUTS, NOUT_LD, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("mse_grad: ") + hipGetErrorString(e));
    // loss = sum(mask * e^2) / (M * 12): masked entries still count in the mean
    e = mlpk::sum_partials(s->partial, mlpk::mse_partials(M, NOUT_LD), 1.0f / (float)(M * ROD_SURROGATE_OUTPUTS),
                           loss_out ? loss_out : s->loss, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("loss: ") + hipGetErrorString(e));
    const float *dZ = s->dY;
    int ldz = NOUT_LD;
    float *bufs[2] = {s->dZa, s->dZb};
    for (int l = NL - 1; l >= 0; --l) {
        // [dW_l; db_l] = [A_{l-1}, 1]^T dZ_l: a row of ones appended to A^T gives the
        // column sums of dZ_l, which land right after dW_l (the bias follows the
        // weights in the internal layout)
        mlpk::GemmArgs a{};
        a.A = l > 0 ? (const void *)s->Ab[l - 1] : (const void *)x;
        a.lda = KDIM[l];
        a.B = dZ;
        a.ldb = ldz;
        a.M = KDIM[l] + 1;
        a.ones_row = KDIM[l];
        a.N = NPAD[l];
        a.K = M;
        a.C = s->g + s->lay.w[l];
        a.ldc = NPAD[l];
        e = mlpk::gemm_backward_weight(a, s->splitw, SPLIT_FLOATS, st);
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("dW gemm: ") + hipGetErrorString(e));
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
    (void)hipFree(s->phase);
    s->phase = nullptr;
    (void)hipFree(s->disp);
    (void)hipFree(s->saved);
    (void)hipFree(s->saved2);
    s->saved2 = nullptr;
    (void)hipFree(s->plain);
    (void)hipFree(s->plain_tiles);
    s->plain_tiles = nullptr;
    s->n_plain_tiles = 0;
    (void)hipFree(s->xall);
    (void)hipFree(s->yall);
    (void)hipFree(s->jmap);
    (void)hipFree(s->jsel);
    (void)hipFree(s->jerr);
    (void)hipFree(s->jen);
    s->jen = nullptr;
    if (s->judge) rod_batch_destroy(s->judge);
    s->judge = nullptr;
    s->judge_rods = 0;
    s->plain = nullptr;
    s->xall = nullptr;
    s->yall = nullptr;
    s->jmap = s->jsel = nullptr;
    s->jerr = nullptr;
    s->plain_h.clear();
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
    if (v.extended)
        return sfail(ROD_EUNSUPPORTED, "the learned coarse step has no features for a magnetic couple, gravity or muscle torques");
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
    s->n_max = 0;
    for (int r = 0; r < R; ++r) s->n_max = std::max(s->n_max, (int)v.n[r]);
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
    up((void **)&s->phase, nullptr, (size_t)R * sizeof(float2));
    s->saved_bytes = v.state_bytes + v.tail_bytes;
    up(&s->saved, nullptr, s->saved_bytes);
    s->plain_h.assign(R, 0);
    up((void **)&s->plain, s->plain_h.data(), (size_t)R * 4);
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
    a.phase = s->phase;
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

int save_state(rod_surrogate *s, const rodk::BatchView &v, hipStream_t st, void *to = nullptr)
{
    char *dst = (char *)(to ? to : s->saved);
    SHIPCHK(hipMemcpyAsync(dst, v.f32.state, v.state_bytes, hipMemcpyDeviceToDevice, st));
    SHIPCHK(hipMemcpyAsync(dst + v.state_bytes, v.f32.tail, v.tail_bytes, hipMemcpyDeviceToDevice, st));
    return ROD_OK;
}

int restore_state(rod_surrogate *s, const rodk::BatchView &v, hipStream_t st)
{
    SHIPCHK(hipMemcpyAsync(v.f32.state, s->saved, v.state_bytes, hipMemcpyDeviceToDevice, st));
    SHIPCHK(hipMemcpyAsync(v.f32.tail, (char *)s->saved + v.state_bytes, v.tail_bytes, hipMemcpyDeviceToDevice, st));
    return ROD_OK;
}

int perturb_batch(rod_surrogate *s, const rodk::BatchView &v, const float noise[4], uint64_t seed, hipStream_t st)
{
    hipError_t e = surk::perturb(v.f32, s->elem_rod, s->elem_first, s->n_elems, noise, (float)(s->k * v.dt), seed, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("perturb: ") + hipGetErrorString(e));
    return ROD_OK;
}

// One training sample.  Without noise: features now, k plain steps, targets.
// With noise: the features are taken at a perturbed copy of the state while the
// batch itself steps on from the clean state, so the targets lead from the
// perturbed state back onto the plain trajectory.
int collect_impl(rod_surrogate *s, rod_batch *b, const float *noise, uint64_t seed, float *F, float *T, float *M,
                 hipStream_t st)
{
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    const bool noisy = noise && (noise[0] != 0.f || noise[1] != 0.f || noise[2] != 0.f || noise[3] != 0.f);
    if ((rc = save_state(s, v, st))) return rc;
    if (noisy) {
        if (!s->saved2) SHIPCHK(hipMalloc(&s->saved2, s->saved_bytes));
        if ((rc = perturb_batch(s, v, noise, seed, st))) return rc;
    }
    hipError_t e = surk::features(win_args(s, v), F, nullptr, nullptr, nullptr, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("features: ") + hipGetErrorString(e));
    if (noisy) {
        if ((rc = save_state(s, v, st, s->saved2))) return rc;
        if ((rc = restore_state(s, v, st))) return rc;
    }
    if ((rc = rod_step(b, s->k, st))) return rc;
    rodk::BatchView v1;
    if ((rc = rodk::batch_view(b, &v1))) return rc;
    rodk::DevBatch<float> s0 = saved_batch(s, v);
    if (noisy) s0.state = (float *)s->saved2, s0.tail = (float *)((char *)s->saved2 + v.state_bytes);
    e = surk::targets(win_args(s, v1), s0, T, M, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("targets: ") + hipGetErrorString(e));
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
    // device copy: mu_x, sd_x, mu_t, sd_t, then 1 / sd_x (inputs are standardised by multiplication)
    std::vector<float> d(s->norm_h);
    for (int i = 0; i < ROD_SURROGATE_INPUTS; ++i) d.push_back(1.0f / s->norm_h[ROD_SURROGATE_INPUTS + i]);
    SHIPCHK(hipMemcpy(s->norm, d.data(), d.size() * 4, hipMemcpyHostToDevice));
    return ROD_OK;
}


// A batch of `m` placeholder rods of n elements (straight, unit material) in
// the main batch's tile width: the judge copies real rods into it.
int make_judge(rod_surrogate *s, const rodk::BatchView &v, int m, int n)
{
    if (s->judge && s->judge_rods == m) return ROD_OK;
    if (s->judge) rod_batch_destroy(s->judge);
    s->judge = nullptr;
    (void)hipFree(s->jmap);
    (void)hipFree(s->jsel);
    (void)hipFree(s->jerr);
    (void)hipFree(s->jen);
    s->jmap = s->jsel = nullptr;
    s->jerr = nullptr;
    s->jen = nullptr;
    const int64_t Ne = (int64_t)m * n, Nn = Ne + m;
    std::vector<int32_t> ne(m, n), zero(m, 0);
    std::vector<double> pos(3 * Nn, 0.0), vel(3 * Nn, 0.0), dir(9 * Ne, 0.0), om(3 * Ne, 0.0), one(m, 1.0);
    for (int64_t i = 0, nd = 0; i < m; ++i)
        for (int j = 0; j <= n; ++j, ++nd) pos[3 * nd + 2] = j;
    for (int64_t e = 0; e < Ne; ++e) dir[9 * e] = dir[9 * e + 4] = dir[9 * e + 8] = 1.0;
    rod_batch_desc d{};
    d.n_rods = m;
    d.n_elems = ne.data();
    d.position = pos.data();
    d.velocity = vel.data();
    d.director = dir.data();
    d.omega = om.data();
    d.density = d.youngs = d.shear_modulus = d.radius = d.shear_coeff = one.data();
    d.bc_start = d.bc_end = zero.data();
    d.dt = v.dt;
    d.precision = ROD_F32;
    d.tile_waves = v.waves;
    int rc = rod_batch_create(&d, nullptr, &s->judge);
    if (rc) return rc;
    SHIPCHK(hipMalloc((void **)&s->jmap, (size_t)m * 4));
    SHIPCHK(hipMalloc((void **)&s->jsel, (size_t)m * 4));
    SHIPCHK(hipMalloc((void **)&s->jerr, (size_t)m * 8));
    SHIPCHK(hipMalloc((void **)&s->jen, (size_t)m * 10 * sizeof(double)));
    s->judge_rods = m;
    return ROD_OK;
}

int ensure_step_buffers(rod_surrogate *s)
{
    if (s->xall) return ROD_OK;
    SHIPCHK(hipMalloc((void **)&s->xall, (size_t)s->n_windows * ROD_SURROGATE_INPUTS * 2));
    SHIPCHK(hipMalloc((void **)&s->yall, (size_t)s->n_windows * NOUT_LD * 4));
    return ROD_OK;
}

// Upload the fallback flags and the sorted list of tiles that hold plain rods.
int upload_plain(rod_surrogate *s, const rodk::BatchView &v, hipStream_t st)
{
    const int TL = 64 * v.waves;
    std::vector<int32_t> tiles;
    for (int r = 0; r < v.n_rods; ++r)
        if (s->plain_h[r]) tiles.push_back((int32_t)(v.rod_slot[r] / TL));
    std::sort(tiles.begin(), tiles.end());
    tiles.erase(std::unique(tiles.begin(), tiles.end()), tiles.end());
    if ((int)tiles.size() > s->n_plain_tiles || !s->plain_tiles) {
        (void)hipFree(s->plain_tiles);
        s->plain_tiles = nullptr;
        SHIPCHK(hipMalloc((void **)&s->plain_tiles, std::max<size_t>(tiles.size(), 1) * 4));
    }
    s->n_plain_tiles = (int)tiles.size();
    if (!tiles.empty())
        SHIPCHK(hipMemcpyAsync(s->plain_tiles, tiles.data(), tiles.size() * 4, hipMemcpyHostToDevice, st));
    SHIPCHK(hipMemcpyAsync(s->plain, s->plain_h.data(), s->plain_h.size() * 4, hipMemcpyHostToDevice, st));
    SHIPCHK(hipStreamSynchronize(st));   // the host vectors are reused
    return ROD_OK;
}

// features -> network -> deltas applied to the rods off the plain step; the
// plain ones take k plain steps.  Advances the clock by k.
int coarse_step(rod_surrogate *s, rod_batch *b, const rodk::BatchView &v, int n_plain, hipStream_t st)
{
    if (n_plain == v.n_rods)   // nothing left to predict
        return rodk::batch_step_masked(b, s->k, s->plain, s->plain_tiles, s->n_plain_tiles, st);
    const float *mux = s->norm, *isdx = s->norm + 2 * ROD_SURROGATE_INPUTS + 2 * ROD_SURROGATE_OUTPUTS;
    const float *mut = s->norm + 2 * ROD_SURROGATE_INPUTS, *sdt = mut + ROD_SURROGATE_OUTPUTS;
    hipError_t e = surk::features(win_args(s, v), nullptr, s->xall, mux, isdx, st);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("features: ") + hipGetErrorString(e));
    int rc = infer(s, s->xall, s->n_windows, s->yall, NOUT_LD, st);
    if (rc) return rc;
    if (n_plain > 0) {
        if ((rc = rodk::batch_step_masked(b, s->k, s->plain, s->plain_tiles, s->n_plain_tiles, st))) return rc;
    }
    e = surk::apply(win_args(s, v), s->yall, NOUT_LD, mut, sdt, n_plain > 0 ? s->plain : nullptr, s->disp, s->elem_rod,
                    s->elem_first, s->n_elems, st, s->n_max);
    if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("apply: ") + hipGetErrorString(e));
    if (n_plain == 0 && (rc = rodk::batch_advance_clock(b, s->k, st))) return rc;
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
    alloc((void **)&s->frag, (size_t)mlpk::infer_fragments_bytes());
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
    alloc((void **)&s->splitw, SPLIT_FLOATS * 4);
    alloc((void **)&s->norm, (3 * ROD_SURROGATE_INPUTS + 2 * ROD_SURROGATE_OUTPUTS) * 4);
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
    (void)hipFree(s->frag);
    (void)hipFree(s->splitw);
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
    if ((uintptr_t)x % 16 || (uintptr_t)y % 4) return sfail(ROD_EINVAL, "x must be 16-byte aligned, y 4-byte aligned");
    return infer(s, (const __bf16 *)x, M, y, ROD_SURROGATE_OUTPUTS, (hipStream_t)stream);
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
    rc = adam_step(s, lr, st);
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
    return collect_impl(s, b, nullptr, 0, features, targets, mask, (hipStream_t)stream);
}

int rod_surrogate_collect_noisy(rod_surrogate *s, rod_batch *b, const float *noise, uint64_t seed, float *features,
                                float *targets, float *mask, void *stream)
{
    if (!s || !b || !noise || !features || !targets || !mask) return sfail(ROD_EINVAL, "NULL argument");
    for (int i = 0; i < 4; ++i)
        if (!(noise[i] >= 0) || !std::isfinite(noise[i])) return sfail(ROD_EINVAL, "noise levels must be finite, >= 0");
    return collect_impl(s, b, noise, seed, features, targets, mask, (hipStream_t)stream);
}

int rod_surrogate_perturb(rod_surrogate *s, rod_batch *b, const float *noise, uint64_t seed, void *stream)
{
    if (!s || !b || !noise) return sfail(ROD_EINVAL, "NULL argument");
    for (int i = 0; i < 4; ++i)
        if (!(noise[i] >= 0) || !std::isfinite(noise[i])) return sfail(ROD_EINVAL, "noise levels must be finite, >= 0");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    return perturb_batch(s, v, noise, seed, (hipStream_t)stream);
}

int rod_surrogate_apply(rod_surrogate *s, rod_batch *b, const float *deltas, void *stream)
{
    if (!s || !b || !deltas) return sfail(ROD_EINVAL, "NULL argument");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = surk::apply(win_args(s, v), deltas, ROD_SURROGATE_OUTPUTS, nullptr, nullptr, nullptr, s->disp,
                               s->elem_rod, s->elem_first, s->n_elems, st, s->n_max);
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
        || !(d->val_fraction >= 0 && d->val_fraction < 1) || !(d->noise[0] >= 0) || !(d->noise[1] >= 0)
        || !(d->noise[2] >= 0) || !(d->noise[3] >= 0))
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
        // noise levels cycle through 0, 1/3, 2/3 and 1 times d->noise
        const float f = (float)(i % 4) / 3.0f;
        const float nz[4] = {f * d->noise[0], f * d->noise[1], f * d->noise[2], f * d->noise[3]};
        TRY(collect_impl(s, b, nz, d->seed * 0x100000001B3ull + (uint64_t)i, F + (size_t)i * W * ROD_SURROGATE_INPUTS,
                         T + (size_t)i * W * ROD_SURROGATE_OUTPUTS, Mk + (size_t)i * W * ROD_SURROGATE_OUTPUTS, st));
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
        // constant column (a flag, or variation below FP32 resolution of its mean): unit scale.
        // Targets keep tiny scales: departures from free flight are small by construction.
        if (!(sdv > 1e-6 * std::fabs(m)) || !(sdv > 0)) sdv = 1.0;
        mu[j] = (float)m;
        sd[j] = (float)sdv;
    }
    TRY(rod_surrogate_set_normalization(s, mu.data(), sd.data(), mu.data() + ROD_SURROGATE_INPUTS,
                                        sd.data() + ROD_SURROGATE_INPUTS));
    const float *mux = s->norm, *isdx = s->norm + 2 * ROD_SURROGATE_INPUTS + 2 * ROD_SURROGATE_OUTPUTS;
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
            TRYH(surk::gather_rows(F, T, Mk, idx + bi * B, B, mux, isdx, mut, sdt, xb, tb, mb, st));
            TRY(gradient_chunk(s, xb, tb, mb, B, st, lhist + step));
            const double ph = total_steps > 1 ? (double)step / (double)(total_steps - 1) : 1.0;
            const float lr = (float)(d->lr_min + 0.5 * (d->lr - d->lr_min) * (1.0 + std::cos(M_PI * ph)));
            TRY(adam_step(s, lr, st));
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
            TRYH(surk::gather_rows(F, T, Mk, idx + v0, B, mux, isdx, mut, sdt, xb, tb, mb, st));
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

int rod_surrogate_step(rod_surrogate *s, rod_batch *b, int64_t n_coarse, const rod_judge_desc *j,
                       rod_surrogate_stats *stats, void *stream)
{
    if (!s || !b || !j) return sfail(ROD_EINVAL, "NULL argument");
    if (n_coarse < 0 || j->judge_every <= 0 || !(j->judge_fraction > 0 && j->judge_fraction <= 1)
        || !(j->max_pos_error >= 0) || !(j->max_orth_error >= 0) || !(j->max_energy_error >= 0))
        return sfail(ROD_EINVAL, "invalid judge descriptor");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    const int n = v.n[0];
    for (int r = 1; r < v.n_rods; ++r)
        if (v.n[r] != n) return sfail(ROD_EUNSUPPORTED, "the coarse step needs rods of equal element count");
    if ((rc = ensure_step_buffers(s))) return rc;
    const int m = std::max(1, (int)std::lround(j->judge_fraction * v.n_rods));
    if ((rc = make_judge(s, v, m, n))) return rc;
    rodk::BatchView jv;
    if ((rc = rodk::batch_view(s->judge, &jv))) return rc;
    hipStream_t st = (hipStream_t)stream;
    rod_surrogate_stats out{};
    int n_plain = 0;
    for (int32_t f : s->plain_h) n_plain += f != 0;
    std::vector<int32_t> map;
    std::vector<float> err;
    std::vector<double> en;
    int64_t c = 0;
    while (c < n_coarse) {
        // ---- open a judge window: sample rods still on the coarse step
        std::vector<int32_t> cand;
        for (int r = 0; r < v.n_rods; ++r)
            if (!s->plain_h[r]) cand.push_back(r);
        const int mw = std::min<int>(m, (int)cand.size());
        if (mw > 0) {
            std::mt19937_64 rng(j->seed + 0x9E3779B97F4A7C15ull * (uint64_t)(s->judge_windows_total + 1));
            std::shuffle(cand.begin(), cand.end(), rng);
            map.assign(cand.begin(), cand.begin() + mw);
            std::sort(map.begin(), map.end());
            map.resize(m, map.back());   // unused tail of the judge batch repeats the last rod
            std::vector<int32_t> sel(m, 0);
            std::fill(sel.begin(), sel.begin() + mw, 1);
            SHIPCHK(hipMemcpyAsync(s->jmap, map.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
            SHIPCHK(hipMemcpyAsync(s->jsel, sel.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
            rodk::BatchView cv;
            if ((rc = rodk::batch_view(b, &cv))) return rc;
            hipError_t e = surk::copy_rods(jv.f32, cv.f32, s->jmap, nullptr, m, n, false, false, st);
            if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("judge copy: ") + hipGetErrorString(e));
            if ((rc = rodk::batch_set_time(s->judge, cv.time, st))) return rc;
            SHIPCHK(hipStreamSynchronize(st));   // the host map and selection buffers are reused
        }
        const int64_t steps = std::min<int64_t>(j->judge_every, n_coarse - c);
        for (int64_t i = 0; i < steps; ++i) {
            rodk::BatchView cv;
            if ((rc = rodk::batch_view(b, &cv))) return rc;
            if ((rc = coarse_step(s, b, cv, n_plain, st))) return rc;
        }
        c += steps;
        out.coarse_steps += steps;
        if (mw == 0) continue;
        // ---- close the window: plain re-run of the sample, compare, fall back
        if ((rc = rod_step(s->judge, steps * s->k, stream))) return rc;
        rodk::BatchView cv, jv2;
        if ((rc = rodk::batch_view(b, &cv)) || (rc = rodk::batch_view(s->judge, &jv2))) return rc;
        hipError_t e = surk::judge_errors(cv.f32, jv2.f32, s->jmap, m, s->jerr, st);
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("judge errors: ") + hipGetErrorString(e));
        e = rodk::launch_energy(cv.f32, s->jen, st, s->jmap, m);
        if (e == hipSuccess) e = rodk::launch_energy(jv2.f32, s->jen + 5 * (size_t)m, st);
        if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("judge energies: ") + hipGetErrorString(e));
        err.resize(2 * (size_t)m);
        en.resize(10 * (size_t)m);
        SHIPCHK(hipMemcpyAsync(err.data(), s->jerr, err.size() * 4, hipMemcpyDeviceToHost, st));
        SHIPCHK(hipMemcpyAsync(en.data(), s->jen, en.size() * 8, hipMemcpyDeviceToHost, st));
        SHIPCHK(hipStreamSynchronize(st));
        std::vector<int32_t> fail_sel(m, 0);
        int nf = 0;
        for (int k = 0; k < mw; ++k) {
            const double pe = err[2 * k], oe = err[2 * k + 1];
            // strain energy (shear + bending) against the plain re-run, relative to the
            // re-run's mechanical energy (kinetic + strain)
            const double *a = &en[5 * (size_t)k], *p = &en[5 * ((size_t)m + k)];
            const double du = std::fabs((a[2] + a[3]) - (p[2] + p[3]));
            const double den = p[0] + p[1] + p[2] + p[3];
            const double ue = du == 0.0 ? 0.0 : (den > 0.0 ? du / den : INFINITY);
            out.max_pos_error = std::max(out.max_pos_error, std::isfinite(pe) ? pe : INFINITY);
            out.max_orth_error = std::max(out.max_orth_error, std::isfinite(oe) ? oe : INFINITY);
            out.max_energy_error = std::max(out.max_energy_error, std::isfinite(ue) ? ue : INFINITY);
            if (!(pe <= j->max_pos_error) || !(oe <= j->max_orth_error) || !(ue <= j->max_energy_error)) {
                fail_sel[k] = 1;
                s->plain_h[map[k]] = 1;
                ++nf;
            }
        }
        out.judge_windows += 1;
        out.rods_judged += mw;
        s->judge_windows_total += 1;
        if (nf > 0) {
            SHIPCHK(hipMemcpyAsync(s->jsel, fail_sel.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
            e = surk::copy_rods(jv2.f32, cv.f32, s->jmap, s->jsel, m, n, true, true, st);
            if (e != hipSuccess) return sfail(ROD_EDEVICE, std::string("fallback copy: ") + hipGetErrorString(e));
            rodk::BatchView pv;
            if ((rc = rodk::batch_view(b, &pv)) || (rc = upload_plain(s, pv, st))) return rc;
            out.rods_failed += nf;
            n_plain += nf;
        }
    }
    out.rods_plain = n_plain;
    if (stats) *stats = out;
    return ROD_OK;
}

int rod_surrogate_fallback_flags(rod_surrogate *s, rod_batch *b, int32_t *flags)
{
    if (!s || !b || !flags) return sfail(ROD_EINVAL, "NULL argument");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    std::copy(s->plain_h.begin(), s->plain_h.end(), flags);
    return ROD_OK;
}

int rod_surrogate_reset_fallback(rod_surrogate *s, rod_batch *b)
{
    if (!s || !b) return sfail(ROD_EINVAL, "NULL argument");
    rodk::BatchView v;
    int rc = ensure_ctx(s, b, v);
    if (rc) return rc;
    std::fill(s->plain_h.begin(), s->plain_h.end(), 0);
    return upload_plain(s, v, nullptr);
}

// File: 8-byte magic "RODSURR1", int32 k, int32 parameter count, int32
// normalisation count, int32 zero, then the FP32 parameters (external layout)
// and the normalisation vector (mu_x, sd_x, mu_t, sd_t), little-endian.
static const char kMagic[8] = {'R', 'O', 'D', 'S', 'U', 'R', 'R', '1'};

int rod_surrogate_save(rod_surrogate *s, const char *path)
{
    if (!s || !path) return sfail(ROD_EINVAL, "NULL argument");
    std::vector<float> p(ROD_SURROGATE_PARAMS);
    int rc = rod_surrogate_get_params(s, p.data());
    if (rc) return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f) return sfail(ROD_EINVAL, std::string("cannot open ") + path + " for writing");
    const int32_t hdr[4] = {s->k, ROD_SURROGATE_PARAMS, (int32_t)s->norm_h.size(), 0};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4
              && std::fwrite(p.data(), 4, p.size(), f) == p.size()
              && std::fwrite(s->norm_h.data(), 4, s->norm_h.size(), f) == s->norm_h.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return sfail(ROD_EINVAL, std::string("write failed: ") + path);
    return ROD_OK;
}

int rod_surrogate_load(rod_surrogate *s, const char *path)
{
    if (!s || !path) return sfail(ROD_EINVAL, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return sfail(ROD_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[4];
    std::vector<float> p(ROD_SURROGATE_PARAMS), nm(s->norm_h.size());
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 && std::fread(hdr, 4, 4, f) == 4
              && hdr[1] == ROD_SURROGATE_PARAMS && hdr[2] == (int32_t)nm.size()
              && std::fread(p.data(), 4, p.size(), f) == p.size() && std::fread(nm.data(), 4, nm.size(), f) == nm.size();
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!ok) return sfail(ROD_EINVAL, std::string("not a surrogate file of this network: ") + path);
    if (hdr[0] != s->k)
        return sfail(ROD_EINVAL, "file was trained for k = " + std::to_string(hdr[0]) + ", handle has k = " + std::to_string(s->k));
    for (float x : p)
        if (!std::isfinite(x)) return sfail(ROD_EINVAL, "non-finite parameter in file");
    const float *n = nm.data();
    int rc = rod_surrogate_set_normalization(s, n, n + ROD_SURROGATE_INPUTS, n + 2 * ROD_SURROGATE_INPUTS,
                                             n + 2 * ROD_SURROGATE_INPUTS + ROD_SURROGATE_OUTPUTS);
    if (rc) return rc;
    return rod_surrogate_set_params(s, p.data());
}

}  // extern "C"
