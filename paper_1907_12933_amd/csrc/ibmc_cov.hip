// Host driver of the coverage criteria (Sec. III-B): potentials of both
// inputs of every pair, per-pair predicates, OR over pairs, summaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ibmc_host.h"
#include "kernels_covsearch.h"

namespace ibmc {

static CovLayout make_layout(int nl, const int *widths) {
    CovLayout L{};
    L.nl = nl;
    int64_t rows = 0, pairs = 0;
    int all = 0, u = 0;
    for (int l = 0; l < nl; ++l) {
        L.width[l] = widths[l];
        L.uoff[l] = u;
        u += widths[l];
        L.words[l] = (widths[l] + 31) / 32;
    }
    L.U = u;
    for (int l = 0; l < nl; ++l) {
        L.rowoff[l] = rows;
        L.alloff[l] = all;
        L.pairoff[l] = pairs;
        if (l + 1 < nl) {
            rows += (int64_t)widths[l] * L.words[l + 1];
            all += L.words[l + 1];
            pairs += (int64_t)widths[l] * widths[l + 1];
        }
    }
    L.rows_words = rows;
    L.all_words = all;
    L.total_pairs = pairs;
    return L;
}

static ibmc_status params_of(const ibmc_cov_params *p, CovParams &cp, double &P) {
    cp.dist_sq_min = 1;
    cp.ratio_num = 3;
    cp.ratio_den = 2;
    P = 0.8;
    if (p) {
        if (p->dist_sq_min < 0 || p->ratio_num < 0 || p->ratio_den < 0 || p->P < 0)
            return fail(IBMC_E_INVALID, "negative coverage parameter");
        if (p->dist_sq_min) cp.dist_sq_min = p->dist_sq_min;
        if (p->ratio_num) cp.ratio_num = p->ratio_num;
        if (p->ratio_den) cp.ratio_den = p->ratio_den;
        if (p->P > 0) P = p->P;
    }
    return IBMC_OK;
}

// Device state of one coverage evaluation (bitmasks and sums) in ctx scratch.
struct CovRun {
    CovLayout lay;
    CovBits bits;
    CovSums sums;
};

static ibmc_status cov_prepare(ibmc_ctx *ctx, const CovLayout &lay, CovRun &R) {
    hipStream_t s = ctx->stream;
    R.lay = lay;
    const int64_t rows = std::max<int64_t>(lay.rows_words, 1), all = std::max(lay.all_words, 1);
    const int64_t flag_bytes = round_up(std::max(lay.U, 1), 8);
    // one allocation: rows_ss, rows_sv, all_ds, all_dv (uint32), pairs[4], neurons[4] (u64),
    // colmask[4][all] (uint32), condflag[4][flag_bytes]
    const int64_t w32 = 2 * rows + 2 * all + 4 * all;
    const int64_t bytes = w32 * 4 + 64 + 8 * 8 + 4 * flag_bytes + 64;
    IBMC_TRY(ctx->cov_bits.reserve((size_t)bytes));
    char *b = (char *)ctx->cov_bits.p;
    R.bits.rows_ss = (uint32_t *)b;
    R.bits.rows_sv = R.bits.rows_ss + rows;
    R.bits.all_ds = R.bits.rows_sv + rows;
    R.bits.all_dv = R.bits.all_ds + all;
    R.sums.colmask = R.bits.all_dv + all;
    R.sums.colmask_stride = all;
    char *after = (char *)(R.sums.colmask + 4 * all);
    after = (char *)(((uintptr_t)after + 63) & ~(uintptr_t)63);
    R.sums.pairs = (unsigned long long *)after;
    R.sums.neurons = R.sums.pairs + 4;
    R.sums.condflag = (uint8_t *)(R.sums.neurons + 4);
    R.sums.flag_stride = flag_bytes;
    const int64_t used = (char *)(R.sums.condflag + 4 * flag_bytes) - b;
    HIP_OK(launch_fill_u64((unsigned long long *)b, (used + 7) / 8, 0ull, s));
    return IBMC_OK;
}

static ibmc_status cov_finish(ibmc_ctx *ctx, CovRun &R, int first_crit, int n_crit, double P,
                              ibmc_cov_summary *outs, uint64_t *covered_bits, float ms_before) {
    hipStream_t s = ctx->stream;
    HIP_OK(launch_cov_summary(R.lay, R.bits, R.sums, s));
    const int64_t words = (R.lay.total_pairs + 63) / 64;
    if (covered_bits && words > 0) {
        IBMC_TRY(ctx->cov_out.reserve((size_t)words * 8 * n_crit));
        for (int c = 0; c < n_crit; ++c)
            HIP_OK(launch_cov_expand(R.lay, R.bits, first_crit + c, ctx->cov_out.as<uint64_t>() + c * words, words, s));
    }
    HIP_OK(hipEventRecord(ctx->ev1, s));
    unsigned long long h[8];
    HIP_OK(hipMemcpyAsync(h, R.sums.pairs, sizeof(h), hipMemcpyDeviceToHost, s));
    if (covered_bits && words > 0)
        HIP_OK(hipMemcpyAsync(covered_bits, ctx->cov_out.p, (size_t)words * 8 * n_crit, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    for (int c = 0; c < n_crit; ++c) {
        const int crit = first_crit + c;
        ibmc_cov_summary &S = outs[c];
        memset(&S, 0, sizeof(S));
        S.covered_pairs = (int64_t)h[crit];
        S.total_pairs = R.lay.total_pairs;
        S.covered_neurons = (int64_t)h[4 + crit];
        S.total_neurons = R.lay.U;
        S.fraction = R.lay.U ? (double)S.covered_neurons / (double)R.lay.U : 0.0;
        S.literal = S.fraction >= P;
        S.seconds = ms * 1e-3;
    }
    (void)ms_before;
    return IBMC_OK;
}

static ibmc_status coverage_impl(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1, const uint8_t *x2,
                                 int64_t n_pairs, int first_crit, int n_crit, const ibmc_cov_params *params,
                                 ibmc_cov_summary *outs, uint64_t *covered_bits, bool on_device) {
    clear_error();
    if (!ctx || !net || !outs || n_pairs < 0 || (n_pairs > 0 && (!x1 || !x2)))
        return fail(IBMC_E_INVALID, "bad argument");
    if (net->act != IBMC_ACT_RELU_Q8) return fail(IBMC_E_UNIMPL, "coverage runs on integer networks");
    CovParams cp;
    double P;
    IBMC_TRY(params_of(params, cp, P));
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int n = net->dims[0];
    const CovLayout lay = make_layout(net->L, net->dims.data() + 1);
    HIP_OK(hipEventRecord(ctx->ev0, s));
    CovRun R;
    IBMC_TRY(cov_prepare(ctx, lay, R));
    if (n_pairs > 0) {
        const uint8_t *d1 = x1, *d2 = x2;
        if (!on_device) {
            IBMC_TRY(ctx->cov_img.reserve((size_t)2 * n_pairs * n));
            HIP_OK(hipMemcpyAsync(ctx->cov_img.p, x1, (size_t)n_pairs * n, hipMemcpyHostToDevice, s));
            HIP_OK(hipMemcpyAsync(ctx->cov_img.as<uint8_t>() + (size_t)n_pairs * n, x2, (size_t)n_pairs * n,
                                  hipMemcpyHostToDevice, s));
            d1 = ctx->cov_img.as<uint8_t>();
            d2 = d1 + (size_t)n_pairs * n;
        }
        CovPairParams cpp{};
        cpp.net = net->qd;
        cpp.fx = net->fx;
        cpp.lay = lay;
        cpp.cp = cp;
        cpp.bits = R.bits;
        cpp.x1 = d1;
        cpp.x2 = d2;
        cpp.n_pairs = n_pairs;
        HIP_OK(launch_cov_pair(cpp, ctx->n_cu, s));
    }
    if (!on_device) HIP_OK(hipStreamSynchronize(s));  // host images may be released after return
    return cov_finish(ctx, R, first_crit, n_crit, P, outs, covered_bits, 0.f);
}

}  // namespace ibmc

using namespace ibmc;

extern "C" ibmc_status ibmc_coverage(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1, const uint8_t *x2,
                                     int64_t n_pairs, int32_t criterion, const ibmc_cov_params *params,
                                     ibmc_cov_summary *out, uint64_t *covered_bits) {
    if (criterion < 0 || criterion > 3) return fail(IBMC_E_INVALID, "criterion %d", criterion);
    return coverage_impl(ctx, net, x1, x2, n_pairs, criterion, 1, params, out, covered_bits, false);
}

extern "C" ibmc_status ibmc_coverage_dev(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1, const uint8_t *x2,
                                         int64_t n_pairs, int32_t criterion, const ibmc_cov_params *params,
                                         ibmc_cov_summary *out, uint64_t *covered_bits) {
    if (criterion < 0 || criterion > 3) return fail(IBMC_E_INVALID, "criterion %d", criterion);
    return coverage_impl(ctx, net, x1, x2, n_pairs, criterion, 1, params, out, covered_bits, true);
}

extern "C" ibmc_status ibmc_coverage_all_dev(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1,
                                             const uint8_t *x2, int64_t n_pairs, const ibmc_cov_params *params,
                                             ibmc_cov_summary *outs, uint64_t *covered_bits) {
    return coverage_impl(ctx, net, x1, x2, n_pairs, 0, 4, params, outs, covered_bits, true);
}

extern "C" ibmc_status ibmc_coverage_from_potentials(ibmc_ctx *ctx, int32_t n_layers, const int32_t *widths,
                                                     const int64_t *u1, const int64_t *u2, int64_t n_pairs,
                                                     int32_t criterion, const ibmc_cov_params *params,
                                                     ibmc_cov_summary *out, uint64_t *covered_bits) {
    clear_error();
    if (!ctx || !widths || !out || n_pairs < 0 || (n_pairs > 0 && (!u1 || !u2)))
        return fail(IBMC_E_INVALID, "bad argument");
    if (n_layers < 1 || n_layers > IBMC_MAX_LAYERS) return fail(IBMC_E_INVALID, "n_layers %d", n_layers);
    if (criterion < 0 || criterion > 3) return fail(IBMC_E_INVALID, "criterion %d", criterion);
    for (int l = 0; l < n_layers; ++l)
        if (widths[l] < 1 || widths[l] > IBMC_MAX_WIDTH) return fail(IBMC_E_INVALID, "width[%d] = %d", l, widths[l]);
    CovParams cp;
    double P;
    IBMC_TRY(params_of(params, cp, P));
    const CovLayout lay = make_layout(n_layers, widths);
    for (int64_t t = 0; t < n_pairs * lay.U; ++t)
        if (u1[t] >= (1LL << 31) || u1[t] < -(1LL << 31) || u2[t] >= (1LL << 31) || u2[t] < -(1LL << 31))
            return fail(IBMC_E_RANGE, "potential %lld outside int32", (long long)t);
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    HIP_OK(hipEventRecord(ctx->ev0, s));
    CovRun R;
    IBMC_TRY(cov_prepare(ctx, lay, R));
    if (n_pairs > 0) {
        IBMC_TRY(ctx->cov_pots.reserve((size_t)2 * n_pairs * lay.U * 8));
        int64_t *p1 = ctx->cov_pots.as<int64_t>(), *p2 = p1 + (size_t)n_pairs * lay.U;
        HIP_OK(hipMemcpyAsync(p1, u1, (size_t)n_pairs * lay.U * 8, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(p2, u2, (size_t)n_pairs * lay.U * 8, hipMemcpyHostToDevice, s));
        HIP_OK(launch_cov_pred_i64(p1, p2, n_pairs, lay, cp, R.bits, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    return cov_finish(ctx, R, criterion, 1, P, out, covered_bits, 0.f);
}

// ---------------------------------------------------------------------------
// coverage-guided test generation
// ---------------------------------------------------------------------------

extern "C" ibmc_status ibmc_coverage_search(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                            int32_t n_pixels, const int16_t *delta_set, int32_t n_deltas,
                                            int32_t k, int32_t criterion, const ibmc_cov_params *params,
                                            int32_t max_tests, ibmc_cex *tests, int64_t *gains, int32_t *n_tests,
                                            ibmc_cov_summary *out, uint64_t *covered_bits) {
    clear_error();
    if (!ctx || !net || !image || !delta_set || !n_tests || !out || max_tests < 0 || (max_tests > 0 && !tests))
        return fail(IBMC_E_INVALID, "bad argument");
    if (net->act != IBMC_ACT_RELU_Q8) return fail(IBMC_E_UNIMPL, "coverage runs on integer networks");
    if (n_pixels != net->dims[0]) return fail(IBMC_E_INVALID, "n_pixels %d != network input %d", n_pixels, net->dims[0]);
    if (n_deltas < 1 || n_deltas > kMaxDeltas) return fail(IBMC_E_INVALID, "n_deltas %d", n_deltas);
    if (criterion < 0 || criterion > 3) return fail(IBMC_E_INVALID, "criterion %d", criterion);
    const int n = net->dims[0], L = net->L;
    if (k < 1 || k > n || k > kMaxK) return fail(IBMC_E_INVALID, "k %d", k);
    for (int l = 1; l <= L; ++l)
        if (net->dims[l] > 64) return fail(IBMC_E_UNIMPL, "test generation needs non-input layers of <= 64 units");
    const CovLayout lay = make_layout(L, net->dims.data() + 1);
    const int words = (int)((lay.total_pairs + 63) / 64);
    if (words > kCovSearchMaxWords || words < 1)
        return fail(IBMC_E_UNIMPL, "%lld neuron pairs: test generation handles up to %d", (long long)lay.total_pairs,
                    64 * kCovSearchMaxWords);
    __int128 cands = binom_small(n, k);
    for (int t = 0; t < k; ++t) cands *= n_deltas;
    if (cands > ((__int128)1 << 26)) return fail(IBMC_E_UNIMPL, "level %d has more than 2^26 candidates", k);
    const int64_t nc = (int64_t)cands;
    CovParams cp;
    double P;
    IBMC_TRY(params_of(params, cp, P));
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    HIP_OK(hipEventRecord(ctx->ev0, s));
    // the clean image's potentials
    IBMC_TRY(ctx->cov_img.reserve((size_t)(n + 63) / 64 * 64 + (size_t)kMaxDeltas * 2));
    uint8_t *dimg = ctx->cov_img.as<uint8_t>();
    int16_t *ddel = reinterpret_cast<int16_t *>(dimg + ((n + 63) / 64) * 64);
    HIP_OK(hipMemcpyAsync(dimg, image, (size_t)n, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ddel, delta_set, (size_t)n_deltas * 2, hipMemcpyHostToDevice, s));
    const size_t mask_bytes = (size_t)nc * words * 8;
    // [potentials | masks | labels | covered (kCovSearchMaxWords words) | a batch of greedy steps' best
    // keys | their labels], 256-byte aligned parts
    constexpr int kSteps = 16;
    const size_t need = ((size_t)lay.U * 4 + 255) / 256 * 256 + (mask_bytes + 255) / 256 * 256 +
                        ((size_t)nc * 4 + 255) / 256 * 256 + (size_t)(kCovSearchMaxWords + kSteps) * 8 +
                        (size_t)kSteps * 4;
    IBMC_TRY(ctx->cov_pots.reserve(need));
    char *base = ctx->cov_pots.as<char>();
    int32_t *pot0 = reinterpret_cast<int32_t *>(base);
    unsigned long long *masks = reinterpret_cast<unsigned long long *>(base + (((size_t)lay.U * 4 + 255) / 256) * 256);
    int32_t *labels = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(masks) + ((mask_bytes + 255) / 256) * 256);
    unsigned long long *covered =
        reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(labels) + (((size_t)nc * 4 + 255) / 256) * 256);
    unsigned long long *keys = covered + kCovSearchMaxWords;
    int32_t *labs = reinterpret_cast<int32_t *>(keys + kSteps);
    HIP_OK(launch_fwd_pots_q8(net->qd, net->fx, dimg, 1, pot0, lay.U, nullptr, s));
    CovCandParams cpar{};
    cpar.net = net->qd;
    cpar.image = dimg;
    cpar.deltas = ddel;
    cpar.m = n_deltas;
    cpar.k = k;
    cpar.pot0 = pot0;
    cpar.rank0 = 0;
    cpar.n_cand = nc;
    cpar.crit = criterion;
    cpar.words = words;
    cpar.cp = cp;
    cpar.masks = masks;
    cpar.labels = labels;
    HIP_OK(launch_cov_cand(cpar, s));
    HIP_OK(launch_fill_u64(covered, kCovSearchMaxWords, 0ull, s));
    // greedy: the candidate adding the most uncovered pairs (lowest rank on
    // ties), until none adds any or max_tests are taken.  Steps are queued
    // kSteps at a time and their winners read back once per batch; a step
    // after one without a winner finds none either (nothing was added).
    int32_t taken = 0;
    bool done = false;
    std::vector<CexRec> picked;
    std::vector<int64_t> gain_v;
    unsigned long long hk[kSteps];
    int32_t hl[kSteps];
    while (taken < max_tests && !done) {
        const int nb = std::min(kSteps, max_tests - taken);
        HIP_OK(launch_fill_u64(keys, nb, 0ull, s));
        for (int i = 0; i < nb; ++i) {
            HIP_OK(launch_cov_gain(masks, nc, words, covered, keys + i, s));
            HIP_OK(launch_cov_take(masks, words, keys + i, covered, labels, labs + i, s));
        }
        HIP_OK(hipMemcpyAsync(hk, keys, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hl, labs, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        for (int i = 0; i < nb; ++i) {
            if (!hk[i]) {
                done = true;
                break;
            }
            const int64_t c = (int64_t)(((1ull << 40) - 1ull) - (hk[i] & ((1ull << 40) - 1ull)));
            picked.push_back(CexRec{0, k, c, hl[i], 0});
            gain_v.push_back((int64_t)(hk[i] >> 40));
            ++taken;
        }
    }
    std::vector<unsigned long long> cov(words);
    HIP_OK(hipMemcpyAsync(cov.data(), covered, (size_t)words * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipEventRecord(ctx->ev1, s));
    HIP_OK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (taken) memcpy(tests, picked.data(), picked.size() * sizeof(CexRec));
    if (gains && taken) memcpy(gains, gain_v.data(), gain_v.size() * 8);
    *n_tests = taken;
    if (covered_bits) memcpy(covered_bits, cov.data(), (size_t)words * 8);
    // summary: covered pairs, and the neurons (of the non-input layers) in any covered pair
    int64_t pairs = 0, neurons = 0;
    std::vector<char> hit(lay.U, 0);
    int64_t boff = 0;
    for (int l = 0; l + 1 < lay.nl; ++l) {
        const int h0 = lay.width[l], h1 = lay.width[l + 1];
        for (int i = 0; i < h0; ++i)
            for (int j = 0; j < h1; ++j) {
                const int64_t b = boff + (int64_t)i * h1 + j;
                if ((cov[b >> 6] >> (b & 63)) & 1ull) {
                    ++pairs;
                    hit[lay.uoff[l] + i] = 1;
                    hit[lay.uoff[l + 1] + j] = 1;
                }
            }
        boff += (int64_t)h0 * h1;
    }
    for (char h : hit) neurons += h;
    memset(out, 0, sizeof(*out));
    out->covered_pairs = pairs;
    out->total_pairs = lay.total_pairs;
    out->covered_neurons = neurons;
    out->total_neurons = lay.U;
    out->fraction = lay.U ? (double)neurons / lay.U : 0.0;
    out->literal = out->fraction >= P;
    out->seconds = ms * 1e-3;
    return IBMC_OK;
}
