// The learned surrogate: a Fourier-feature MLP over (theta, phi, f) that
// predicts the co-polarised scattered field A_HH, A_VV, trained on sweeps the
// SBR path computes, and the fill of a dense angle-frequency grid in which
// SBR both judges the network on held-out probes and replaces it on every
// tile where it fails.
//
// Parameters are held as float32 master copies (Adam state beside them) and
// as bf16 copies (row-major, and transposed for the hidden layers whose
// input gradient is needed) that the matrix-core kernels read.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <random>

#include "sbr_internal.hpp"

using namespace sbr;

namespace {

struct Bufs {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    ~Bufs() { release(); }
    void release()
    {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
    template <class T>
    int alloc(T **p, size_t n)
    {
        const size_t b = std::max<size_t>(sizeof(T) * n, 256);
        void *q = nullptr;
        if (hipMalloc(&q, b) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SBR_ERR_OOM, "surrogate: device allocation of " + std::to_string(b) + " bytes failed");
        }
        ptrs.push_back(q);
        bytes += static_cast<int64_t>(b);
        *p = static_cast<T *>(q);
        return SBR_OK;
    }
};

constexpr int64_t kPredictRows = int64_t(1) << 18;  // inference chunk
constexpr int64_t kMaxBatch = 65536;

int64_t pad64(int64_t m) { return (m + 63) / 64 * 64; }

}  // namespace

struct sbr_mlp {
    sbr_ctx *ctx = nullptr;
    int device = 0;
    int n_ff = 64, width = 256, depth = 4, act = kActSilu;
    MlpNorm norm{};
    double scale = 1.0;
    // layer l (0..depth): weights [n_out][n_in] at woff[l], bias at boff[l]
    std::vector<int> n_in, n_out;
    std::vector<int64_t> woff, boff, toff;  // toff: transposed copy offset (-1: none)
    int64_t P = 0;
    Bufs keep;                           // parameters and state
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *Bff = nullptr;
    uint16_t *wb = nullptr, *wt = nullptr, *wf = nullptr;  // wf: fragment-major hidden weights (fused inference)
    int64_t *step = nullptr;  // device: Adam steps taken
    int64_t adam_t = 0;       // host mirror of *step
    // workspaces (grown on demand)
    Bufs ws_pred;
    int64_t pred_rows = 0;
    uint16_t *p_h0 = nullptr, *p_ha = nullptr, *p_hb = nullptr;
    Bufs ws_train;
    int64_t train_rows = 0, train_count_cap = 0;
    std::vector<uint16_t *> h, ht;   // h[0..depth], ht[0..depth-1]
    std::vector<float *> z;          // z[1..depth] stored at z[l - 1]
    float *dz[2] = {nullptr, nullptr};
    uint16_t *dzb[2] = {nullptr, nullptr}, *dzbt[2] = {nullptr, nullptr};
    float *tb = nullptr, *dy = nullptr, *part = nullptr, *losses = nullptr;
    float *red = nullptr;  // reduction scratch (split-K slices, column-sum partials)
    int ksplit = 1;
    int32_t *idx = nullptr;
    int64_t idx_cap = 0;
    int64_t loss_cap = 0;
    float *h_losses = nullptr;  // pinned
};

namespace {

RefreshTable refresh_table(const sbr_mlp *M)
{
    RefreshTable t{};
    t.w = M->w;
    t.wb = M->wb;
    t.wt = M->wt;
    t.wf = M->wf;
    t.n_layers = M->depth + 1;
    const bool fused = fused_ok(M->n_ff, M->width, M->depth);
    for (int l = 0; l <= M->depth; ++l) {
        t.rows[l] = M->n_out[l];
        t.cols[l] = M->n_in[l];
        t.frag[l] = fused && l < M->depth;
        t.woff[l] = M->woff[l];
        t.toff[l] = M->toff[l];
    }
    return t;
}

int refresh_bf16(sbr_mlp *M, hipStream_t s) { return launch_refresh(s, refresh_table(M)); }

int ensure_pred(sbr_mlp *M, int64_t rows)
{
    if (M->pred_rows >= rows) return SBR_OK;
    M->ws_pred.release();
    int rc;
    if ((rc = M->ws_pred.alloc(&M->p_h0, static_cast<size_t>(rows) * 2 * M->n_ff)) ||
        (rc = M->ws_pred.alloc(&M->p_ha, static_cast<size_t>(rows) * M->width)) ||
        (rc = M->ws_pred.alloc(&M->p_hb, static_cast<size_t>(rows) * M->width))) {
        M->pred_rows = 0;
        return rc;
    }
    M->pred_rows = rows;
    return SBR_OK;
}

int ensure_train(sbr_mlp *M, int64_t rows)
{
    if (M->train_rows >= rows) return SBR_OK;
    M->ws_train.release();
    M->train_rows = 0;
    const int W = M->width, D = M->depth;
    M->h.assign(D + 1, nullptr);
    M->ht.assign(D, nullptr);
    M->z.assign(D, nullptr);
    int rc;
    for (int l = 0; l <= D; ++l) {
        const int cols = l == 0 ? 2 * M->n_ff : W;
        if ((rc = M->ws_train.alloc(&M->h[l], static_cast<size_t>(rows) * cols))) return rc;
        if (l < D && (rc = M->ws_train.alloc(&M->ht[l], static_cast<size_t>(rows) * cols))) return rc;
        if (l >= 1 && (rc = M->ws_train.alloc(&M->z[l - 1], static_cast<size_t>(rows) * W))) return rc;
    }
    for (int q = 0; q < 2; ++q)
        if ((rc = M->ws_train.alloc(&M->dz[q], static_cast<size_t>(rows) * W)) ||
            (rc = M->ws_train.alloc(&M->dzb[q], static_cast<size_t>(rows) * W)) ||
            (rc = M->ws_train.alloc(&M->dzbt[q], static_cast<size_t>(rows) * W)))
            return rc;
    if ((rc = M->ws_train.alloc(&M->tb, static_cast<size_t>(rows) * 4)) ||
        (rc = M->ws_train.alloc(&M->dy, static_cast<size_t>(rows) * 4)) ||
        (rc = M->ws_train.alloc(&M->part, static_cast<size_t>(rows / 16 + 1))))
        return rc;
    // weight gradients sum over the batch: split it so that each block walks 128..256 rows
    int ks = 1;
    while (ks * 2 <= 32 && rows % (static_cast<int64_t>(ks) * 2 * 16) == 0 && rows / (ks * 2) >= 128) ks *= 2;
    M->ksplit = ks;
    const int64_t kin_max = std::max(W, 2 * M->n_ff);
    const int64_t R = (rows + 63) / 64;
    // the split-K slices of a weight gradient, the column-sum partials of its
    // bias, and the output layer's partials
    const int64_t red = static_cast<int64_t>(ks) * W * kin_max + R * W + R * (4 * W + 4);
    if ((rc = M->ws_train.alloc(&M->red, static_cast<size_t>(red)))) return rc;
    M->train_rows = rows;
    return SBR_OK;
}

// Forward, loss and gradients (into M->g) of the batch of rows idx[0, count)
// of the points and targets (rows padded to a multiple of 64).  The batch's
// summed squared error goes to *loss_slot (device); *bump (nullable) += 1
// first (the step count of a training step).
int batch_grad(sbr_mlp *M, hipStream_t s, const double *pts, const double *targets, const int32_t *idx, int64_t count,
               int64_t rows, float *loss_slot, int64_t *bump)
{
    int rc;
    const int W = M->width, D = M->depth, K0 = 2 * M->n_ff;
    if ((rc = launch_embed_batch(s, pts, targets, idx, count, rows, M->norm, M->Bff, M->n_ff, 1.0 / M->scale, M->h[0],
                                 M->ht[0], M->tb, bump)))
        return rc;
    for (int l = 1; l <= D; ++l) {
        GemmArgs a{};
        a.A = M->h[l - 1];
        a.lda = l == 1 ? K0 : W;
        a.B = M->wb + M->woff[l - 1];
        a.ldb = M->n_in[l - 1];
        a.M = static_cast<int>(rows);
        a.N = W;
        a.K = M->n_in[l - 1];
        a.bias = M->w + M->boff[l - 1];
        a.act = M->act;
        a.zout = M->z[l - 1];
        a.ldz = W;
        a.hout = M->h[l];
        a.ldh = W;
        a.htout = l < D ? M->ht[l] : nullptr;
        a.ldht = rows;
        if ((rc = launch_gemm(s, kEpiHidden, a))) return rc;
    }
    const int64_t nblk = (rows + 15) / 16;
    if ((rc = launch_out(s, M->h[D], W, M->wb + M->woff[D], M->w + M->boff[D], count, rows, 1, 1.0, nullptr, M->tb,
                         M->dy, M->part)))
        return rc;
    OutBackIn ob{};
    ob.dy = M->dy;
    ob.wo = M->wb + M->woff[D];
    ob.width = W;
    ob.Mrows = rows;
    ob.z = M->z[D - 1];
    ob.act = M->act;
    ob.dz = M->dz[0];
    ob.dzb = M->dzb[0];
    ob.dzbt = M->dzbt[0];
    ob.h = M->h[D];
    ob.part = M->part;
    ob.n_part = static_cast<int>(nblk);
    ob.loss = loss_slot;
    // scratch: the split-K slices of a layer's weight gradient, its bias
    // partials, then the output layer's partials (pending while the next
    // layer's slices are written)
    const int64_t R = (rows + 63) / 64;
    const int64_t kin_max = std::max(W, K0);
    float *red_out = M->red + static_cast<int64_t>(M->ksplit) * W * kin_max + R * W;
    SumPair pending{};
    if ((rc = launch_out_backward(s, ob, M->g + M->woff[D], M->g + M->boff[D], red_out, &pending))) return rc;
    int cur = 0;
    for (int l = D; l >= 1; --l) {
        const int kin = M->n_in[l - 1];
        GemmArgs a{};
        a.A = M->dzbt[cur];
        a.lda = rows;
        a.B = M->ht[l - 1];
        a.ldb = rows;
        a.M = W;
        a.N = kin;
        a.K = static_cast<int>(rows);
        a.fout = M->red;
        a.ldf = kin;
        a.ksplit = M->ksplit;
        a.split_stride = static_cast<int64_t>(W) * kin;
        float *colpart = M->red + static_cast<int64_t>(M->ksplit) * W * kin;
        SumPair mine{};
        if ((rc = launch_wgrad_colsum(s, a, M->dz[cur], rows, W, colpart, M->g + M->woff[l - 1],
                                      M->g + M->boff[l - 1], pending, &mine)))
            return rc;
        pending = mine;
        if (l > 1) {
            const int nxt = cur ^ 1;
            GemmArgs b{};
            b.A = M->dzb[cur];
            b.lda = W;
            b.B = M->wt + M->toff[l - 1];
            b.ldb = W;
            b.M = static_cast<int>(rows);
            b.N = kin;
            b.K = W;
            b.act = M->act;
            b.zin = M->z[l - 2];
            b.ldzi = W;
            b.fout = M->dz[nxt];
            b.ldf = W;
            b.hout = M->dzb[nxt];
            b.ldh = W;
            b.htout = M->dzbt[nxt];
            b.ldht = rows;
            // this layer's gradient sums ride along (the product reads none of their buffers)
            if ((rc = launch_gemm_fold(s, kEpiDz, b, pending))) return rc;
            pending = SumPair{};
            cur = nxt;
        }
    }
    return launch_sum_pair(s, pending);  // the first layer's sums
}

int check_pts(const double *pts, int64_t M, const char *fn)
{
    if (!pts) return fail(SBR_ERR_INVALID_ARG, std::string(fn) + ": NULL points");
    if (M < 1 || M > (int64_t(1) << 31)) return fail(SBR_ERR_INVALID_ARG, std::string(fn) + ": M out of range");
    return SBR_OK;
}

}  // namespace

extern "C" int sbr_mlp_create(sbr_ctx *ctx, const sbr_mlp_desc *d, sbr_mlp **out)
{
    if (!ctx || !d || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: NULL argument");
    *out = nullptr;
    if (d->struct_size < sizeof(sbr_mlp_desc)) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: struct_size too small");
    if (d->n_ff < 64 || d->n_ff > 512 || d->n_ff % 64)
        return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: n_ff must be a multiple of 64 in [64, 512]");
    if (d->width < 128 || d->width > 1024 || d->width % 128)
        return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: width must be a multiple of 128 in [128, 1024]");
    if (d->depth < 1 || d->depth > 8) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: depth must be in [1, 8]");
    if (d->act != SBR_ACT_SILU && d->act != SBR_ACT_RELU) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: unknown act");
    for (int c = 0; c < 3; ++c)
        if (!(d->hi[c] > d->lo[c]) || !std::isfinite(d->lo[c]) || !std::isfinite(d->hi[c]))
            return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: input ranges need lo < hi");
    if (!(d->out_scale > 0.0) || !(d->ff_sigma >= 0.0))
        return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_create: out_scale must be positive, ff_sigma non-negative");
    SBR_HIP(hipSetDevice(ctx->device));
    sbr_mlp *M = new (std::nothrow) sbr_mlp();
    if (!M) return fail(SBR_ERR_OOM, "sbr_mlp_create: out of host memory");
    M->ctx = ctx;
    M->device = ctx->device;
    M->n_ff = d->n_ff;
    M->width = d->width;
    M->depth = d->depth;
    M->act = d->act;
    for (int c = 0; c < 3; ++c) {
        M->norm.lo[c] = d->lo[c];
        M->norm.hi[c] = d->hi[c];
    }
    M->scale = d->out_scale;
    for (int l = 0; l <= d->depth; ++l) {
        M->n_in.push_back(l == 0 ? 2 * d->n_ff : d->width);
        M->n_out.push_back(l == d->depth ? 4 : d->width);
    }
    int64_t off = 0, toff = 0;
    for (int l = 0; l <= d->depth; ++l) {
        M->woff.push_back(off);
        off += static_cast<int64_t>(M->n_in[l]) * M->n_out[l];
        M->boff.push_back(off);
        off += M->n_out[l];
        // transposed bf16 copies for the hidden layers that pass a gradient on
        if (l >= 1 && l < d->depth) {
            M->toff.push_back(toff);
            toff += static_cast<int64_t>(M->n_in[l]) * M->n_out[l];
        } else {
            M->toff.push_back(-1);
        }
    }
    M->P = off;
    int rc;
    if ((rc = M->keep.alloc(&M->w, M->P)) || (rc = M->keep.alloc(&M->m, M->P)) || (rc = M->keep.alloc(&M->v, M->P)) ||
        (rc = M->keep.alloc(&M->g, M->P)) || (rc = M->keep.alloc(&M->wb, M->P)) ||
        (rc = M->keep.alloc(&M->wf, M->P)) || (rc = M->keep.alloc(&M->wt, std::max<int64_t>(toff, 1))) || (rc = M->keep.alloc(&M->step, 1)) ||
        (rc = M->keep.alloc(&M->Bff, 3 * static_cast<size_t>(d->n_ff)))) {
        delete M;
        return rc;
    }
    // seeded initialisation: features B ~ N(0, ff_sigma^2); weights
    // N(0, 2 / n_in) (output layer N(0, 1 / n_in)), biases zero
    std::mt19937_64 rng(d->seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<float> hB(3 * static_cast<size_t>(d->n_ff)), hw(M->P, 0.0f);
    for (auto &x : hB) x = static_cast<float>(d->ff_sigma * nd(rng));
    for (int l = 0; l <= d->depth; ++l) {
        const double sd = std::sqrt((l == d->depth ? 1.0 : 2.0) / M->n_in[l]);
        for (int64_t i = 0; i < static_cast<int64_t>(M->n_in[l]) * M->n_out[l]; ++i)
            hw[M->woff[l] + i] = static_cast<float>(sd * nd(rng));
    }
    hipStream_t s = ctx->stream;
    if (hipMemcpy(M->Bff, hB.data(), 4 * hB.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(M->w, hw.data(), 4 * hw.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(M->m, 0, 4 * M->P, s) != hipSuccess || hipMemsetAsync(M->v, 0, 4 * M->P, s) != hipSuccess ||
        hipMemsetAsync(M->g, 0, 4 * M->P, s) != hipSuccess || hipMemsetAsync(M->step, 0, 8, s) != hipSuccess) {
        delete M;
        return fail(SBR_ERR_HIP, "sbr_mlp_create: initial upload failed");
    }
    if ((rc = refresh_bf16(M, s))) {
        delete M;
        return rc;
    }
    *out = M;
    return SBR_OK;
}

extern "C" int sbr_mlp_get_info(const sbr_mlp *M, sbr_mlp_info *out)
{
    if (!M || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_get_info: NULL argument");
    out->n_params = M->P;
    out->n_ff = M->n_ff;
    out->width = M->width;
    out->depth = M->depth;
    out->act = M->act;
    out->out_scale = M->scale;
    out->adam_steps = M->adam_t;
    out->flops_per_point = 2.0 * (static_cast<double>(2 * M->n_ff) * M->width +
                                  static_cast<double>(M->depth - 1) * M->width * M->width + 4.0 * M->width);
    return SBR_OK;
}

extern "C" int sbr_mlp_get_params(const sbr_mlp *M, float *host, int64_t n)
{
    if (!M || !host || n != M->P) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_get_params: bad argument or size");
    SBR_HIP(hipSetDevice(M->device));
    SBR_HIP(hipStreamSynchronize(M->ctx->stream));
    SBR_HIP(hipMemcpy(host, M->w, 4 * M->P, hipMemcpyDeviceToHost));
    return SBR_OK;
}

extern "C" int sbr_mlp_set_params(sbr_mlp *M, const float *host, int64_t n)
{
    if (!M || !host || n != M->P) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_set_params: bad argument or size");
    SBR_HIP(hipSetDevice(M->device));
    hipStream_t s = M->ctx->stream;
    SBR_HIP(hipStreamSynchronize(s));
    SBR_HIP(hipMemcpy(M->w, host, 4 * M->P, hipMemcpyHostToDevice));
    SBR_HIP(hipMemsetAsync(M->m, 0, 4 * M->P, s));
    SBR_HIP(hipMemsetAsync(M->v, 0, 4 * M->P, s));
    SBR_HIP(hipMemsetAsync(M->step, 0, 8, s));
    M->adam_t = 0;
    return refresh_bf16(M, s);
}

extern "C" int sbr_mlp_get_features(const sbr_mlp *M, float *host)
{
    if (!M || !host) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_get_features: NULL argument");
    SBR_HIP(hipSetDevice(M->device));
    SBR_HIP(hipMemcpy(host, M->Bff, 12 * static_cast<size_t>(M->n_ff), hipMemcpyDeviceToHost));
    return SBR_OK;
}

extern "C" int sbr_mlp_set_scale(sbr_mlp *M, double out_scale)
{
    if (!M || !(out_scale > 0.0)) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_set_scale: scale must be positive");
    M->scale = out_scale;
    return SBR_OK;
}

extern "C" int sbr_mlp_predict(sbr_mlp *M, const double *pts, int64_t n, double *A_out)
{
    if (!M || !A_out) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_predict: NULL argument");
    int rc = check_pts(pts, n, "sbr_mlp_predict");
    if (rc) return rc;
    SBR_HIP(hipSetDevice(M->device));
    hipStream_t s = M->ctx->stream;
    if (fused_ok(M->n_ff, M->width, M->depth)) {  // one launch, activations never leave LDS
        FusedArgs f{};
        f.pts = pts;
        f.M = n;
        f.norm = M->norm;
        f.Bff = M->Bff;
        f.n_ff = M->n_ff;
        f.depth = M->depth;
        f.act = M->act;
        for (int l = 0; l < M->depth; ++l) {
            f.wf[l] = M->wf + M->woff[l];
            f.b[l] = M->w + M->boff[l];
        }
        f.wo = M->wb + M->woff[M->depth];
        f.bo = M->w + M->boff[M->depth];
        f.scale = M->scale;
        f.A = A_out;
        return launch_mlp_fused(s, f);
    }
    const int64_t chunk = std::min(kPredictRows, pad64(n));
    if ((rc = ensure_pred(M, chunk))) return rc;
    const int W = M->width, K0 = 2 * M->n_ff;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t cnt = std::min(chunk, n - r0), rows = pad64(cnt);
        if ((rc = launch_embed(s, pts + 3 * r0, cnt, rows, M->norm, M->Bff, M->n_ff, M->p_h0, nullptr))) return rc;
        const uint16_t *in = M->p_h0;
        uint16_t *bufs[2] = {M->p_ha, M->p_hb};
        for (int l = 1; l <= M->depth; ++l) {
            GemmArgs a{};
            a.A = in;
            a.lda = l == 1 ? K0 : W;
            a.B = M->wb + M->woff[l - 1];
            a.ldb = M->n_in[l - 1];
            a.M = static_cast<int>(rows);
            a.N = W;
            a.K = M->n_in[l - 1];
            a.bias = M->w + M->boff[l - 1];
            a.act = M->act;
            a.hout = bufs[l & 1];
            a.ldh = W;
            if ((rc = launch_gemm(s, kEpiHidden, a))) return rc;
            in = bufs[l & 1];
        }
        if ((rc = launch_out(s, in, W, M->wb + M->woff[M->depth], M->w + M->boff[M->depth], cnt, rows, 0, M->scale,
                             A_out + 4 * r0, nullptr, nullptr, nullptr)))
            return rc;
    }
    return SBR_OK;
}

extern "C" int sbr_mlp_gradients(sbr_mlp *M, const double *pts, const double *targets, int64_t n, float *grads,
                                 float *loss)
{
    if (!M || !targets || !grads) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_gradients: NULL argument");
    int rc = check_pts(pts, n, "sbr_mlp_gradients");
    if (rc) return rc;
    if (n > kMaxBatch) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_gradients: at most 65536 points");
    SBR_HIP(hipSetDevice(M->device));
    hipStream_t s = M->ctx->stream;
    const int64_t rows = pad64(n);
    if ((rc = ensure_train(M, rows))) return rc;
    // identity permutation
    std::vector<int32_t> id(n);
    for (int64_t i = 0; i < n; ++i) id[i] = static_cast<int32_t>(i);
    int32_t *didx = nullptr;
    float *dl = nullptr;
    Bufs tmp;
    if ((rc = tmp.alloc(&didx, n)) || (rc = tmp.alloc(&dl, 1))) return rc;
    SBR_HIP(hipMemcpyAsync(didx, id.data(), 4 * n, hipMemcpyHostToDevice, s));
    if ((rc = batch_grad(M, s, pts, targets, didx, n, rows, dl, nullptr))) return rc;
    SBR_HIP(hipMemcpyAsync(grads, M->g, 4 * M->P, hipMemcpyDeviceToDevice, s));
    float hl = 0.f;
    SBR_HIP(hipMemcpyAsync(&hl, dl, 4, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    if (loss) *loss = hl / (4.0f * static_cast<float>(n));
    return SBR_OK;
}

// One epoch of training steps, captured once per call into a HIP graph and
// replayed for every epoch: the shuffled order is uploaded before each
// replay, the Adam step count and the learning-rate schedule live on the
// device.
extern "C" int sbr_mlp_train(sbr_mlp *M, const double *pts, const double *targets, int64_t n,
                             const sbr_train_opts *o, float *loss_per_epoch)
{
    if (!M || !targets || !o) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_train: NULL argument");
    int rc = check_pts(pts, n, "sbr_mlp_train");
    if (rc) return rc;
    if (o->struct_size < sizeof(sbr_train_opts)) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_train: struct_size too small");
    if (o->epochs < 1 || o->batch < 1 || o->batch > kMaxBatch || !(o->lr > 0.0) || o->lr_min < 0.0)
        return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_train: epochs >= 1, batch in [1, 65536], lr > 0 required");
    if (n > 2147483647LL) return fail(SBR_ERR_INVALID_ARG, "sbr_mlp_train: too many points");
    SBR_HIP(hipSetDevice(M->device));
    hipStream_t s = M->ctx->stream;
    const int64_t bsz = std::min<int64_t>(o->batch, n);
    const int64_t rows = pad64(bsz);
    const int64_t steps = (n + bsz - 1) / bsz;
    const int64_t total = static_cast<int64_t>(o->epochs) * steps;
    if ((rc = ensure_train(M, rows))) return rc;
    Bufs tmp;
    int32_t *didx = nullptr, *dperm = nullptr;
    float *dl = nullptr, *dlr = nullptr, *dlall = nullptr;
    const int64_t ep = o->epochs;
    // epochs per group: their orders (at most 2^24 indices) are uploaded in one copy
    const int64_t grp = std::max<int64_t>(1, std::min<int64_t>(ep, (int64_t(1) << 24) / std::max<int64_t>(n, 1)));
    if ((rc = tmp.alloc(&didx, n)) || (rc = tmp.alloc(&dl, steps)) || (rc = tmp.alloc(&dlr, total)) ||
        (rc = tmp.alloc(&dperm, grp * n)) || (rc = tmp.alloc(&dlall, ep * steps)))
        return rc;
    // cosine decay from lr to lr_min over all steps of this call
    std::vector<float> lr(total);
    for (int64_t t = 0; t < total; ++t)
        lr[t] = static_cast<float>(o->lr_min + 0.5 * (o->lr - o->lr_min) *
                                                   (1.0 + std::cos(kPi * static_cast<double>(t) / static_cast<double>(total))));
    SBR_HIP(hipMemcpyAsync(dlr, lr.data(), 4 * total, hipMemcpyHostToDevice, s));
    const int64_t step0 = M->adam_t;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const RefreshTable rt = refresh_table(M);
    // capture one epoch
    hipStream_t cap = nullptr;
    SBR_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return fail(SBR_ERR_HIP, "sbr_mlp_train: graph capture failed to start");
    }
    for (int64_t st = 0; st < steps && rc == SBR_OK; ++st) {
        const int64_t cnt = std::min(bsz, n - st * bsz);
        if ((rc = batch_grad(M, cap, pts, targets, didx + st * bsz, cnt, rows, dl + st, M->step)) ||
            (rc = launch_adam(cap, M->w, M->m, M->v, M->g, M->P, dlr, M->step, step0, b1, b2, eps, rt)))
            break;
    }
    const hipError_t ec = hipStreamEndCapture(cap, &graph);
    if (rc == SBR_OK && (ec != hipSuccess || !graph)) rc = fail(SBR_ERR_HIP, "sbr_mlp_train: graph capture failed");
    if (rc == SBR_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(SBR_ERR_HIP, "sbr_mlp_train: graph instantiation failed");
    // the epochs' orders (the same shuffles as one per epoch, drawn a group
    // at a time) go to the device in one copy per group; the epochs then run
    // back to back, each an on-device copy of its order, a graph replay and a
    // copy of its losses, with one synchronisation per group (before the
    // pinned buffer is refilled) and one at the end
    float *hl = nullptr;
    const size_t host_words = static_cast<size_t>(std::max<int64_t>(grp * n, ep * steps));
    if (rc == SBR_OK &&
        hipHostMalloc(reinterpret_cast<void **>(&hl), 4 * host_words, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        hl = nullptr;
        rc = fail(SBR_ERR_OOM, "sbr_mlp_train: pinned allocation failed");
    }
    std::mt19937_64 rng(o->seed);
    std::vector<int32_t> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = static_cast<int32_t>(i);
    int32_t *hperm = reinterpret_cast<int32_t *>(hl);  // one pinned buffer: the orders, then the losses
    for (int64_t e0 = 0; e0 < ep && rc == SBR_OK; e0 += grp) {
        const int64_t g = std::min(grp, ep - e0);
        if (e0 > 0 && hipStreamSynchronize(s) != hipSuccess) {  // the previous group's upload read hperm
            rc = fail(SBR_ERR_HIP, "sbr_mlp_train: epoch launch failed");
            break;
        }
        for (int64_t e = 0; e < g; ++e) {
            std::shuffle(perm.begin(), perm.end(), rng);
            std::memcpy(hperm + e * n, perm.data(), 4 * n);
        }
        if (hipMemcpyAsync(dperm, hperm, 4 * g * n, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = fail(SBR_ERR_HIP, "sbr_mlp_train: order upload failed");
            break;
        }
        for (int64_t e = 0; e < g && rc == SBR_OK; ++e) {
            if (hipMemcpyAsync(didx, dperm + e * n, 4 * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipGraphLaunch(exec, s) != hipSuccess ||
                hipMemcpyAsync(dlall + (e0 + e) * steps, dl, 4 * steps, hipMemcpyDeviceToDevice, s) != hipSuccess)
                rc = fail(SBR_ERR_HIP, "sbr_mlp_train: epoch launch failed");
        }
    }
    if (rc == SBR_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(SBR_ERR_HIP, "sbr_mlp_train: epoch failed");
    if (rc == SBR_OK && (hipMemcpyAsync(hl, dlall, 4 * ep * steps, hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
        rc = fail(SBR_ERR_HIP, "sbr_mlp_train: loss copy failed");
    if (rc == SBR_OK && loss_per_epoch) {
        for (int64_t e = 0; e < ep; ++e) {
            double sum = 0.0;
            for (int64_t st = 0; st < steps; ++st) sum += hl[e * steps + st];
            loss_per_epoch[e] = static_cast<float>(sum / (4.0 * static_cast<double>(n)));
        }
    }
    (void)hipStreamSynchronize(s);
    if (rc == SBR_OK) M->adam_t += total;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (hl) (void)hipHostFree(hl);
    return rc;
}

extern "C" void sbr_mlp_destroy(sbr_mlp *M)
{
    if (!M) return;
    (void)hipSetDevice(M->device);
    (void)hipDeviceSynchronize();
    delete M;
}

// ---------------------------------------------------------------- grid fill
namespace {

struct HostTimer {
    std::vector<hipEvent_t> ev;
    ~HostTimer()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

int run_batch(sbr_ctx *ctx, const sbr_bvh *bvh, const std::vector<sbr_batch_item> &items, const double *freqs,
              int64_t n_freqs, const sbr_fill_desc *d, double *A, int64_t *rays, sbr_stats *st = nullptr)
{
    sbr_batch_desc bd{};
    bd.struct_size = sizeof(bd);
    bd.items = items.data();
    bd.n_items = static_cast<int64_t>(items.size());
    bd.freqs_hz = freqs;
    bd.n_freqs_total = n_freqs;
    bd.max_bounces = d->max_bounces;
    bd.mode = d->mode;
    bd.flags = (d->flags | SBR_OPT_NO_GRAPH) & ~static_cast<uint32_t>(SBR_OPT_SYNC);
    bd.samples_per_lambda = 0.0;
    bd.eta = d->eta;
    // a short-lived batch: 2^26-ray chunks, so that its records (4 GB at most)
    // are quick to allocate and free (the 2^29 default's 34 GB took ~1 s)
    sbr_tune tune = default_tune();
    tune.chunk_log2 = 26;
    bd.tune = &tune;
    sbr_batch *b = nullptr;
    int rc = sbr_batch_create(ctx, bvh, &bd, &b);
    if (rc) return rc;
    sbr_batch_info bi;
    (void)sbr_batch_get_info(b, &bi);
    *rays += bi.rays;
    rc = sbr_batch_run(b, A, nullptr, st);
    sbr_batch_destroy(b);
    return rc;
}

}  // namespace

extern "C" int sbr_surrogate_fill(sbr_ctx *ctx, const sbr_bvh *bvh, sbr_mlp *M, const sbr_fill_desc *d, double *A_out,
                                  double *tile_err, uint8_t *fallback, sbr_fill_stats *stats)
{
    const auto t_start = std::chrono::steady_clock::now();
    if (!ctx || !bvh || !M || !d || !A_out) return fail(SBR_ERR_INVALID_ARG, "sbr_surrogate_fill: NULL argument");
    if (d->struct_size < sizeof(sbr_fill_desc)) return fail(SBR_ERR_INVALID_ARG, "sbr_surrogate_fill: struct_size too small");
    if (!d->theta_deg || !d->phi_deg || !d->freqs_hz || !d->probe_dir || !d->probe_freq || d->n_angles < 1 ||
        d->n_freq < 1 || d->tile_angles < 1 || d->tile_freqs < 1 || d->probes_per_tile < 1 || !(d->ds > 0.0))
        return fail(SBR_ERR_INVALID_ARG, "sbr_surrogate_fill: empty grid, tiles, probes or spacing");
    const int64_t na = d->n_angles;
    const int nf = d->n_freq;
    const int64_t n_ta = (na + d->tile_angles - 1) / d->tile_angles;
    const int n_tf = (nf + d->tile_freqs - 1) / d->tile_freqs;
    const int ppt = d->probes_per_tile;
    const int64_t np_dir = static_cast<int64_t>(n_tf) * ppt;  // probe frequencies per probe direction
    if (np_dir > 4096) return fail(SBR_ERR_INVALID_ARG, "sbr_surrogate_fill: more than 4096 probe frequencies");
    if (na * nf > (int64_t(1) << 31)) return fail(SBR_ERR_INVALID_ARG, "sbr_surrogate_fill: grid too large");
    SBR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    HostTimer tm;
    tm.ev.assign(5, nullptr);
    for (auto &e : tm.ev) SBR_HIP(hipEventCreate(&e));
    Bufs tmp;
    int rc;
    int64_t rays = 0;
    // 1. the network on every grid point
    double *dth, *dph, *dfr, *pts;
    if ((rc = tmp.alloc(&dth, na)) || (rc = tmp.alloc(&dph, na)) || (rc = tmp.alloc(&dfr, nf)) ||
        (rc = tmp.alloc(&pts, 3 * static_cast<size_t>(na) * nf)))
        return rc;
    SBR_HIP(hipEventRecord(tm.ev[0], s));
    SBR_HIP(hipMemcpyAsync(dth, d->theta_deg, 8 * na, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dph, d->phi_deg, 8 * na, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dfr, d->freqs_hz, 8 * static_cast<size_t>(nf), hipMemcpyHostToDevice, s));
    if ((rc = launch_grid_pts(s, dth, dph, dfr, na, nf, pts)) || (rc = sbr_mlp_predict(M, pts, na * nf, A_out)))
        return rc;
    SBR_HIP(hipEventRecord(tm.ev[1], s));
    // 2. SBR and the network at the probes
    const int64_t n_probe = n_ta * np_dir;
    std::vector<sbr_batch_item> items(n_ta);
    std::vector<double> hpp(3 * static_cast<size_t>(n_probe));
    for (int64_t t = 0; t < n_ta; ++t) {
        items[t] = sbr_batch_item{0, static_cast<int32_t>(np_dir), 0, d->probe_dir[2 * t], d->probe_dir[2 * t + 1], d->ds};
        for (int64_t q = 0; q < np_dir; ++q) {
            hpp[3 * (t * np_dir + q)] = d->probe_dir[2 * t];
            hpp[3 * (t * np_dir + q) + 1] = d->probe_dir[2 * t + 1];
            hpp[3 * (t * np_dir + q) + 2] = d->probe_freq[q];
        }
    }
    double *A_sbr, *A_sur, *ppts, *smax, *derr;
    uint8_t *dflag;
    if ((rc = tmp.alloc(&A_sbr, 8 * static_cast<size_t>(n_probe))) || (rc = tmp.alloc(&A_sur, 4 * static_cast<size_t>(n_probe))) ||
        (rc = tmp.alloc(&ppts, 3 * static_cast<size_t>(n_probe))) || (rc = tmp.alloc(&smax, 1)) ||
        (rc = tmp.alloc(&derr, n_ta * n_tf)) || (rc = tmp.alloc(&dflag, n_ta * n_tf)))
        return rc;
    SBR_HIP(hipMemcpyAsync(ppts, hpp.data(), 8 * hpp.size(), hipMemcpyHostToDevice, s));
    sbr_stats pst{};
    if ((rc = run_batch(ctx, bvh, items, d->probe_freq, np_dir, d, A_sbr, &rays, &pst)) ||
        (rc = sbr_mlp_predict(M, ppts, n_probe, A_sur)))
        return rc;
    SBR_HIP(hipEventRecord(tm.ev[2], s));
    // 3. judge every tile on its probes
    if ((rc = launch_probe_check(s, A_sbr, A_sur, n_ta, n_tf, ppt, smax, d->floor_db, d->tol_db, dflag, derr))) return rc;
    std::vector<uint8_t> hflag(n_ta * n_tf);
    std::vector<double> herr(n_ta * n_tf);
    SBR_HIP(hipMemcpyAsync(hflag.data(), dflag, hflag.size(), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipMemcpyAsync(herr.data(), derr, 8 * herr.size(), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipEventRecord(tm.ev[3], s));
    SBR_HIP(hipStreamSynchronize(s));
    // 4. SBR on every point of the failing tiles.  A direction is traced once
    // per item, so the failing runs of tiles of a direction share one item
    // when the PO of the passing tiles between them costs less than another
    // trace: the probe sweep measured what one trace costs in frequencies of
    // PO (its trace time over its PO time per frequency).  Points of passing
    // tiles inside such an item are computed and dropped (dst = -1).
    const double trace_freqs = pst.ms_po > 0.0 ? static_cast<double>(np_dir) * pst.ms_trace / pst.ms_po : 0.0;
    std::vector<sbr_batch_item> fb;
    std::vector<int64_t> dst;
    int64_t n_fail = 0, n_fb_points = 0;
    for (int64_t t = 0; t < n_ta; ++t) {
        for (int tf = 0; tf < n_tf; ++tf) n_fail += hflag[t * n_tf + tf];
        // runs [b, e) of failing tiles of this tile row, merged across cheap gaps
        std::vector<std::pair<int, int>> runs;
        for (int tf = 0; tf < n_tf;) {
            if (!hflag[t * n_tf + tf]) {
                ++tf;
                continue;
            }
            int e = tf;
            while (e < n_tf && hflag[t * n_tf + e]) ++e;
            if (!runs.empty() && static_cast<double>((tf - runs.back().second) * d->tile_freqs) <= trace_freqs)
                runs.back().second = e;
            else
                runs.emplace_back(tf, e);
            tf = e;
        }
        for (int64_t a = t * d->tile_angles; a < std::min(na, (t + 1) * d->tile_angles); ++a) {
            for (const auto &r : runs) {
                int f0 = r.first * d->tile_freqs;
                const int f1 = std::min(nf, r.second * d->tile_freqs);
                while (f0 < f1) {
                    const int cnt = std::min(4096, f1 - f0);
                    fb.push_back(sbr_batch_item{0, cnt, f0, d->theta_deg[a], d->phi_deg[a], d->ds});
                    for (int f = f0; f < f0 + cnt; ++f) {
                        const bool fails = hflag[t * n_tf + f / d->tile_freqs] != 0;
                        dst.push_back(fails ? a * nf + f : -1);
                        n_fb_points += fails;
                    }
                    f0 += cnt;
                }
            }
        }
    }
    if (!fb.empty()) {
        double *A_fb;
        int64_t *ddst;
        if ((rc = tmp.alloc(&A_fb, 8 * dst.size())) || (rc = tmp.alloc(&ddst, dst.size()))) return rc;
        SBR_HIP(hipMemcpyAsync(ddst, dst.data(), 8 * dst.size(), hipMemcpyHostToDevice, s));
        if ((rc = run_batch(ctx, bvh, fb, d->freqs_hz, nf, d, A_fb, &rays)) ||
            (rc = launch_scatter_copol(s, A_fb, ddst, static_cast<int64_t>(dst.size()), A_out)))
            return rc;
    }
    SBR_HIP(hipEventRecord(tm.ev[4], s));
    SBR_HIP(hipStreamSynchronize(s));
    if (tile_err) std::memcpy(tile_err, herr.data(), 8 * herr.size());
    if (fallback) std::memcpy(fallback, hflag.data(), hflag.size());
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->tiles = n_ta * n_tf;
        stats->fallback_tiles = n_fail;
        stats->points = na * nf;
        stats->fallback_points = n_fb_points;
        stats->probe_points = n_probe;
        float t01 = 0, t12 = 0, t23 = 0, t34 = 0;
        SBR_HIP(hipEventElapsedTime(&t01, tm.ev[0], tm.ev[1]));
        SBR_HIP(hipEventElapsedTime(&t12, tm.ev[1], tm.ev[2]));
        SBR_HIP(hipEventElapsedTime(&t23, tm.ev[2], tm.ev[3]));
        SBR_HIP(hipEventElapsedTime(&t34, tm.ev[3], tm.ev[4]));
        stats->ms_predict = t01;
        stats->ms_probe = t12;
        stats->ms_check = t23;
        stats->ms_fallback = t34;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        stats->sbr_rays = rays;
    }
    return SBR_OK;
}
