// Host driver of the learned proposal network and of the ordered search
// (time to first counterexample, plain order vs learned order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "ibmc_host.h"

struct ibmc_proposer {
    ibmc_ctx *ctx = nullptr;
    ibmc::DevBuf params, grads, mom, vel;   // flat fp32 [kPropParams] (+1 loss slot in grads)
    int step = 0;
};

namespace ibmc {

PropParams prop_views(const ibmc_proposer *p) {
    const float *b = p->params.as<float>();
    PropParams P;
    P.W1 = b;
    P.b1 = b + kPropH * kPropF;
    P.w2 = P.b1 + kPropH;
    P.c = P.w2 + kPropH;
    return P;
}

static PropGrads gviews(const ibmc_proposer *p) {
    float *b = p->grads.as<float>();
    PropGrads G;
    G.gW1 = b;
    G.gb1 = b + kPropH * kPropF;
    G.gw2 = G.gb1 + kPropH;
    G.gc = G.gw2 + kPropH;
    G.loss = G.gc + 1;
    return G;
}

static uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static ibmc_status upload_cand(const int16_t *deltas, int m, PropCand &pc) {
    if (!deltas || m < 1 || m > kMaxDeltas) return fail(IBMC_E_INVALID, "n_deltas %d", m);
    pc.m = m;
    pc.dmax = 0;
    for (int i = 0; i < m; ++i) {
        pc.deltas[i] = deltas[i];
        pc.dmax = std::max(pc.dmax, std::abs((int)deltas[i]));
    }
    return IBMC_OK;
}

// features + scores of one image into device buffers (feat, scores)
static ibmc_status score_image(ibmc_ctx *ctx, const ibmc_proposer *p, const ibmc_mlp *net, const uint8_t *dimage,
                               int rows, int cols, const PropCand &pc, DevBuf &feat, DevBuf &scores, bool want_scores) {
    hipStream_t s = ctx->stream;
    const int64_t N = (int64_t)net->dims[0] * pc.m;
    IBMC_TRY(ctx->prop_scratch.reserve((size_t)(net->qd.H[1] + net->dims[0]) * 4));
    if (want_scores) {
        // clean potentials, then live norms, features and scores in one launch
        IBMC_TRY(scores.reserve((size_t)N * 4));
        HIP_OK(launch_prop_u0(net->qd, dimage, ctx->prop_scratch.as<int32_t>(), s));
        HIP_OK(launch_prop_fused(net->qd, dimage, ctx->prop_scratch.as<int32_t>(), rows, cols, pc, prop_views(p),
                                 scores.as<float>(), s));
        return IBMC_OK;
    }
    IBMC_TRY(feat.reserve((size_t)N * kPropF * 4));
    HIP_OK(launch_prop_features(net->qd, dimage, nullptr, rows, cols, pc, ctx->prop_scratch.as<int32_t>(),
                                ctx->prop_scratch.as<float>() + net->qd.H[1], feat.as<float>(), s));
    return IBMC_OK;
}

static ibmc_status check_net_for_prop(const ibmc_mlp *net, int rows, int cols) {
    if (!net) return fail(IBMC_E_INVALID, "net is null");
    if (net->act != IBMC_ACT_RELU_Q8) return fail(IBMC_E_UNIMPL, "the proposer works on integer networks");
    if (rows < 1 || cols < 1 || rows * cols != net->dims[0])
        return fail(IBMC_E_INVALID, "rows x cols = %d x %d does not match %d pixels", rows, cols, net->dims[0]);
    return IBMC_OK;
}

}  // namespace ibmc

using namespace ibmc;

extern "C" ibmc_status ibmc_proposer_create(ibmc_ctx *ctx, uint64_t seed, ibmc_proposer **out) {
    clear_error();
    if (!ctx || !out) return fail(IBMC_E_INVALID, "null argument");
    HIP_OK(hipSetDevice(ctx->device));
    std::unique_ptr<ibmc_proposer> p(new ibmc_proposer());
    p->ctx = ctx;
    std::vector<float> h(kPropParams, 0.f);
    uint64_t st = seed ^ 0x5eed5eedull;
    auto uni = [&](float a) { return (float)((splitmix(st) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0) * a; };
    const float a1 = std::sqrt(6.f / (kPropF + kPropH)), a2 = std::sqrt(6.f / (kPropH + 1));
    for (int t = 0; t < kPropH * kPropF; ++t) h[t] = uni(a1);
    for (int t = 0; t < kPropH; ++t) h[kPropH * kPropF + kPropH + t] = uni(a2);
    hipStream_t s = ctx->stream;
    IBMC_TRY(p->params.upload(h.data(), h.size() * 4, s));
    std::vector<float> z(kPropParams + 1, 0.f);
    IBMC_TRY(p->grads.upload(z.data(), z.size() * 4, s));
    IBMC_TRY(p->mom.upload(z.data(), kPropParams * 4, s));
    IBMC_TRY(p->vel.upload(z.data(), kPropParams * 4, s));
    HIP_OK(hipStreamSynchronize(s));
    *out = p.release();
    return IBMC_OK;
}

extern "C" void ibmc_proposer_free(ibmc_proposer *p) { delete p; }

extern "C" ibmc_status ibmc_proposer_get(ibmc_proposer *p, float *W1, float *b1, float *w2, float *c) {
    clear_error();
    if (!p) return fail(IBMC_E_INVALID, "null proposer");
    std::vector<float> h(kPropParams);
    HIP_OK(hipMemcpy(h.data(), p->params.p, kPropParams * 4, hipMemcpyDeviceToHost));
    if (W1) memcpy(W1, h.data(), kPropH * kPropF * 4);
    if (b1) memcpy(b1, h.data() + kPropH * kPropF, kPropH * 4);
    if (w2) memcpy(w2, h.data() + kPropH * kPropF + kPropH, kPropH * 4);
    if (c) *c = h[kPropParams - 1];
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_proposer_set(ibmc_proposer *p, const float *W1, const float *b1, const float *w2,
                                         const float *c) {
    clear_error();
    if (!p || !W1 || !b1 || !w2 || !c) return fail(IBMC_E_INVALID, "null argument");
    std::vector<float> h(kPropParams);
    memcpy(h.data(), W1, kPropH * kPropF * 4);
    memcpy(h.data() + kPropH * kPropF, b1, kPropH * 4);
    memcpy(h.data() + kPropH * kPropF + kPropH, w2, kPropH * 4);
    h[kPropParams - 1] = *c;
    HIP_OK(hipMemcpy(p->params.p, h.data(), kPropParams * 4, hipMemcpyHostToDevice));
    std::vector<float> z(kPropParams, 0.f);
    HIP_OK(hipMemcpy(p->mom.p, z.data(), kPropParams * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->vel.p, z.data(), kPropParams * 4, hipMemcpyHostToDevice));
    p->step = 0;
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_proposer_features(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image, int32_t rows,
                                              int32_t cols, const int16_t *deltas, int32_t m, float *features) {
    clear_error();
    if (!ctx || !image || !features) return fail(IBMC_E_INVALID, "null argument");
    IBMC_TRY(check_net_for_prop(net, rows, cols));
    PropCand pc;
    IBMC_TRY(upload_cand(deltas, m, pc));
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf dimg, feat, sc;
    IBMC_TRY(dimg.upload(image, net->dims[0], s));
    IBMC_TRY(score_image(ctx, nullptr, net, dimg.as<uint8_t>(), rows, cols, pc, feat, sc, false));
    HIP_OK(hipMemcpyAsync(features, feat.p, (size_t)net->dims[0] * m * kPropF * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_proposer_score(ibmc_ctx *ctx, const ibmc_proposer *p, const ibmc_mlp *net,
                                           const uint8_t *image, int32_t rows, int32_t cols, const int16_t *deltas,
                                           int32_t m, float *scores) {
    clear_error();
    if (!ctx || !p || !image || !scores) return fail(IBMC_E_INVALID, "null argument");
    IBMC_TRY(check_net_for_prop(net, rows, cols));
    PropCand pc;
    IBMC_TRY(upload_cand(deltas, m, pc));
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf dimg, feat, sc;
    IBMC_TRY(dimg.upload(image, net->dims[0], s));
    IBMC_TRY(score_image(ctx, p, net, dimg.as<uint8_t>(), rows, cols, pc, feat, sc, true));
    HIP_OK(hipMemcpyAsync(scores, sc.p, (size_t)net->dims[0] * m * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_proposer_score_dev(ibmc_ctx *ctx, const ibmc_proposer *p, const ibmc_mlp *net,
                                               const uint8_t *image, int32_t rows, int32_t cols, const int16_t *deltas,
                                               int32_t m, float *scores) {
    clear_error();
    if (!ctx || !p || !image || !scores) return fail(IBMC_E_INVALID, "null argument");
    IBMC_TRY(check_net_for_prop(net, rows, cols));
    PropCand pc;
    IBMC_TRY(upload_cand(deltas, m, pc));
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf feat, sc;
    IBMC_TRY(score_image(ctx, p, net, image, rows, cols, pc, feat, sc, true));
    HIP_OK(hipMemcpyAsync(scores, sc.p, (size_t)net->dims[0] * m * 4, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_proposer_grad(ibmc_ctx *ctx, ibmc_proposer *p, const float *features, const float *labels,
                                          int32_t B, float pos_weight, float *loss, float *gW1, float *gb1, float *gw2,
                                          float *gc) {
    clear_error();
    if (!ctx || !p || !features || !labels || B < 1) return fail(IBMC_E_INVALID, "bad argument");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf df, dl;
    IBMC_TRY(df.upload(features, (size_t)B * kPropF * 4, s));
    IBMC_TRY(dl.upload(labels, (size_t)B * 4, s));
    HIP_OK(launch_fill_u64((unsigned long long *)p->grads.p, (kPropParams + 2) / 2, 0ull, s));
    HIP_OK(launch_prop_train(prop_views(p), df.as<float>(), dl.as<float>(), nullptr, 0, B, 1.f / B, pos_weight, gviews(p),
                             ctx->n_cu, s));
    std::vector<float> h(kPropParams + 1);
    HIP_OK(hipMemcpyAsync(h.data(), p->grads.p, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(launch_fill_u64((unsigned long long *)p->grads.p, (kPropParams + 2) / 2, 0ull, s));
    HIP_OK(hipStreamSynchronize(s));
    if (gW1) memcpy(gW1, h.data(), kPropH * kPropF * 4);
    if (gb1) memcpy(gb1, h.data() + kPropH * kPropF, kPropH * 4);
    if (gw2) memcpy(gw2, h.data() + kPropH * kPropF + kPropH, kPropH * 4);
    if (gc) *gc = h[kPropParams - 1];
    if (loss) *loss = h[kPropParams];
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_proposer_train(ibmc_ctx *ctx, ibmc_proposer *p, const float *features, const float *labels,
                                           int64_t N, const ibmc_train_opts *o, float *losses) {
    clear_error();
    if (!ctx || !p || !features || !labels || N < 1 || !o) return fail(IBMC_E_INVALID, "bad argument");
    if (o->epochs < 0 || o->batch < 1 || !(o->lr > 0.f)) return fail(IBMC_E_INVALID, "bad training options");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf df, dl, didx;
    IBMC_TRY(df.upload(features, (size_t)N * kPropF * 4, s));
    IBMC_TRY(dl.upload(labels, (size_t)N * 4, s));
    IBMC_TRY(didx.reserve((size_t)N * 4));
    int64_t npos = 0;
    for (int64_t t = 0; t < N; ++t) npos += labels[t] > 0.5f;
    float pw = o->pos_weight;
    if (!(pw > 0.f)) pw = npos > 0 ? (float)(N - npos) / (float)npos : 1.f;
    const float b1 = o->beta1 > 0 ? o->beta1 : 0.9f, b2 = o->beta2 > 0 ? o->beta2 : 0.999f;
    const float eps = o->eps > 0 ? o->eps : 1e-8f;
    std::vector<int32_t> idx(N);
    std::mt19937_64 rng(o->seed);
    HIP_OK(launch_fill_u64((unsigned long long *)p->grads.p, (kPropParams + 2) / 2, 0ull, s));
    const int64_t nb = (N + o->batch - 1) / o->batch;
    for (int ep = 0; ep < o->epochs; ++ep) {
        for (int64_t t = 0; t < N; ++t) idx[t] = (int32_t)t;
        std::shuffle(idx.begin(), idx.end(), rng);
        HIP_OK(hipMemcpyAsync(didx.p, idx.data(), (size_t)N * 4, hipMemcpyHostToDevice, s));
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t begin = b * o->batch, cnt = std::min<int64_t>(o->batch, N - begin);
            HIP_OK(launch_prop_train(prop_views(p), df.as<float>(), dl.as<float>(), didx.as<int32_t>(), begin, cnt,
                                     1.f / cnt, pw, gviews(p), ctx->n_cu, s));
            p->step++;
            const float c1 = 1.f - std::pow(b1, (float)p->step), c2 = 1.f - std::pow(b2, (float)p->step);
            HIP_OK(launch_prop_adam(p->params.as<float>(), p->grads.as<float>(), p->mom.as<float>(), p->vel.as<float>(),
                                    kPropParams, o->lr, b1, b2, eps, c1, c2, s));
        }
        float l = 0.f;
        HIP_OK(hipMemcpyAsync(&l, p->grads.as<float>() + kPropParams, 4, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));  // also keeps idx alive until the copy is done
        if (losses) losses[ep] = l / (float)nb;
        HIP_OK(hipMemsetAsync(p->grads.as<float>() + kPropParams, 0, 4, s));
    }
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

static ibmc_status label_or_count(ibmc_ctx *ctx, int32_t n_pixels, int32_t m, const ibmc_cex *recs, int64_t n,
                                  float *labels, bool count);

extern "C" ibmc_status ibmc_label_candidates(ibmc_ctx *ctx, int32_t n_pixels, int32_t m, const ibmc_cex *recs,
                                             int64_t n, float *labels) {
    return label_or_count(ctx, n_pixels, m, recs, n, labels, false);
}

extern "C" ibmc_status ibmc_count_candidates(ibmc_ctx *ctx, int32_t n_pixels, int32_t m, const ibmc_cex *recs,
                                             int64_t n, float *counts) {
    return label_or_count(ctx, n_pixels, m, recs, n, counts, true);
}

static ibmc_status label_or_count(ibmc_ctx *ctx, int32_t n_pixels, int32_t m, const ibmc_cex *recs, int64_t n,
                                  float *labels, bool count) {
    clear_error();
    if (!ctx || n_pixels < 1 || m < 1 || m > kMaxDeltas || n < 0 || !labels || (n > 0 && !recs))
        return fail(IBMC_E_INVALID, "bad argument");
    for (int64_t t = 0; t < n; ++t) {
        if (recs[t].k < 0 || recs[t].k > kMaxK || recs[t].k > n_pixels) return fail(IBMC_E_INVALID, "record k");
        int64_t mk = 1;
        for (int j = 0; j < recs[t].k; ++j) mk *= m;
        if (recs[t].rank < 0 || recs[t].rank >= binom_small(n_pixels, recs[t].k) * mk)
            return fail(IBMC_E_INVALID, "record %lld: rank out of range", (long long)t);
    }
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf dr, dl;
    const int64_t N = (int64_t)n_pixels * m;
    IBMC_TRY(dl.reserve((size_t)N * 4));
    HIP_OK(launch_fill_u64((unsigned long long *)dl.p, (N + 1) / 2, 0ull, s));
    if (n > 0) {
        IBMC_TRY(dr.upload(recs, (size_t)n * sizeof(ibmc_cex), s));
        HIP_OK(launch_label_candidates(n_pixels, m, dr.as<CexRec>(), n, dl.as<float>(), count, s));
    }
    HIP_OK(hipMemcpyAsync(labels, dl.p, (size_t)N * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

// ---------------------------------------------------------------------------
// ordered search
// ---------------------------------------------------------------------------

namespace ibmc {
ibmc_status ordered_search(ibmc_ctx *ctx, const ibmc_mlp *net, const ibmc_proposer *p, const uint8_t *image, int rows,
                           int cols, const int16_t *deltas, int m, const ibmc_check_opts *o, ibmc_check_summary *out,
                           ibmc_cex *cex_buf);
}

extern "C" ibmc_status ibmc_check_property_ranked(ibmc_ctx *ctx, const ibmc_mlp *net, const ibmc_proposer *p,
                                                  const uint8_t *image, int32_t n_pixels, int32_t rows, int32_t cols,
                                                  const int16_t *deltas, int32_t m, const ibmc_check_opts *o,
                                                  ibmc_check_summary *out, ibmc_cex *cex_buf) {
    clear_error();
    if (!ctx || !image || !o || !out) return fail(IBMC_E_INVALID, "null argument");
    IBMC_TRY(check_net_for_prop(net, rows, cols));
    if (n_pixels != net->dims[0]) return fail(IBMC_E_INVALID, "n_pixels %d != %d", n_pixels, net->dims[0]);
    if (o->k_min < 0 || o->k_max > 2 || o->k_max < o->k_min || o->k_step != 1)
        return fail(IBMC_E_INVALID, "ordered search covers levels 0..2 with step 1");
    if (o->cex_capacity > 0 && !cex_buf) return fail(IBMC_E_INVALID, "cex_buf is null");
    if (!deltas || m < 1 || m > kMaxDeltas) return fail(IBMC_E_INVALID, "n_deltas %d", m);
    if (p && (int64_t)n_pixels * m > prop_sort_max())
        return fail(IBMC_E_UNIMPL, "%d candidates exceed the ordering kernel's %d", n_pixels * m, prop_sort_max());
    return ordered_search(ctx, net, p, image, rows, cols, deltas, m, o, out, cex_buf);
}
