// Host driver of the coverage criteria (Sec. III-B): potentials of both
// inputs of every pair, per-pair predicates, OR over pairs, summaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ibmc_host.h"

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
        IBMC_TRY(ctx->cov_pots.reserve((size_t)2 * n_pairs * lay.U * 4));
        int32_t *p1 = ctx->cov_pots.as<int32_t>(), *p2 = p1 + (size_t)n_pairs * lay.U;
        HIP_OK(launch_fwd_pots_q8(net->qd, net->fx, d1, n_pairs, p1, lay.U, nullptr, s));
        HIP_OK(launch_fwd_pots_q8(net->qd, net->fx, d2, n_pairs, p2, lay.U, nullptr, s));
        HIP_OK(launch_cov_pred_i32(p1, p2, n_pairs, lay, cp, R.bits, s));
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
