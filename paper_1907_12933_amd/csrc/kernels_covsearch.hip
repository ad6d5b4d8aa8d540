// Coverage-guided test generation (the test generation from the covers of
// Sec. III-B that the paper leaves open, Sec. IV-C): every point of one
// level of the delta-set domain is a candidate test x' for the clean image
// x; one wave per candidate computes the potentials of x' (the first layer
// as the rank-k update of x's potentials, Eq. (1), the later layers densely),
// the sign / value / distance changes against x of every non-input layer and
// the neuron pairs (i, j) of adjacent layers that the pair (x, x') covers
// under one criterion, as a bitset in the layout of ibmc_coverage's
// covered_bits.  A greedy loop then picks, one test at a time, the candidate
// covering the most pairs not yet covered (the host queues the steps in
// batches and reads their winners back once per batch).  Networks whose non-input layers
// have at most 64 units (one lane per unit).
#include "kernels_covsearch.h"
#include "enum_common.h"

namespace ibmc {

__global__ void __launch_bounds__(64) cov_cand_kernel(CovCandParams P) {
    __shared__ int act[64];
    __shared__ unsigned long long mask[kCovSearchMaxWords];
    const int lane = threadIdx.x;
    const QNetDev &net = P.net;
    const int L = net.L, n = net.dims[0], m = P.m;
    for (int64_t c = blockIdx.x; c < P.n_cand; c += gridDim.x) {
        // the candidate's pixels and offsets (ascending pixels, digits base m)
        const int64_t rank = P.rank0 + c;
        int64_t mk = 1;
        for (int t = 0; t < P.k; ++t) mk *= m;
        int pix[kMaxK], off[kMaxK];
        lex_unrank_subset(rank / mk, P.k, n, pix);
        int64_t d = rank % mk;
        for (int t = P.k - 1; t >= 0; --t) {
            const int di = (int)(d % m);
            d /= m;
            const int xv = P.image[pix[t]];
            off[t] = clamp_pixel(xv + P.deltas[di]) - xv;
        }
        for (int w = lane; w < P.words; w += 64) mask[w] = 0ull;
        unsigned long long sc[kMaxLayers], vc[kMaxLayers];
        int dc[kMaxLayers];
        int label = 0;
        int uoff = 0;
        for (int l = 1; l <= L; ++l) {
            const int h = net.dims[l];
            int u = 0;
            if (lane < h) {
                if (l == 1) {
                    u = P.pot0[lane];
                    for (int t = 0; t < P.k; ++t) u += off[t] * (int)net.Wd[1][(int64_t)lane * n + pix[t]];
                } else {
                    const int hin = net.dims[l - 1];
                    u = net.bd[l][lane];
                    const int8_t *row = net.Wd[l] + (int64_t)lane * hin;
                    for (int i = 0; i < hin; ++i) u += act[i] * (int)row[i];
                }
            }
            // changes against the clean image's potentials of this layer
            const int a = lane < h ? P.pot0[uoff + lane] : 0;
            const bool sa = a >= 0, sb = u >= 0;   // sign(0) = 1
            const bool s_ch = lane < h && sa != sb;
            const int64_t aa = a < 0 ? -(int64_t)a : a, bb = u < 0 ? -(int64_t)u : u;
            const int64_t mx = aa > bb ? aa : bb, mn = aa > bb ? bb : aa;
            const bool v_ch = lane < h && !s_ch && mx > 0 &&
                              (int64_t)P.cp.ratio_den * mx >= (int64_t)P.cp.ratio_num * mn;
            // squared distance, saturating (as the coverage predicates count it)
            const int64_t dd = (int64_t)a - u;
            const unsigned long long ad = (unsigned long long)(dd < 0 ? -dd : dd);
            unsigned long long d2 = lane < h ? ((ad >> 32) ? ~0ull : ad * ad) : 0ull;
            for (int sh = 32; sh >= 1; sh >>= 1) {
                const unsigned long long o = __shfl_xor(d2, sh), t = d2 + o;
                d2 = t < d2 ? ~0ull : t;
            }
            sc[l - 1] = __ballot(s_ch);
            vc[l - 1] = __ballot(v_ch);
            dc[l - 1] = sc[l - 1] == 0 && d2 >= (unsigned long long)P.cp.dist_sq_min;
            uoff += h;
            // this layer's activations for the next one; the label from the last
            __syncthreads();
            if (l < L) {
                if (lane < h) act[lane] = min(max(u >> net.shift[l - 1], 0), 127);
            } else {
                if (lane < h) act[lane] = u;
            }
            __syncthreads();
            if (l == L && lane == 0) {
                int best = 0;
                for (int j = 1; j < h; ++j) if (act[j] > act[best]) best = j;
                label = best;
            }
        }
        // covered pairs: block l pairs layer l (rows i) with layer l + 1
        int64_t boff = 0;
        for (int l = 1; l < L; ++l) {
            const int h0 = net.dims[l], h1 = net.dims[l + 1];
            const unsigned long long single = (P.crit == 0 || P.crit == 2) ? sc[l - 1] : 0ull;
            const bool one = __popcll(single) == 1;
            const bool dist = (P.crit == 1 || P.crit == 3) && dc[l - 1];
            const unsigned long long pat = (P.crit == 0 || P.crit == 1) ? sc[l] : vc[l];
            // row lane: one sign change at that row (SS / SV), or every row (DS / DV)
            const bool row_on = lane < h0 && pat && ((one && ((single >> lane) & 1ull)) || dist);
            if (row_on) {
                const int64_t b = boff + (int64_t)lane * h1;
                const int w = (int)(b >> 6), sh = (int)(b & 63);
                atomicOr(&mask[w], pat << sh);
                if (sh && sh + h1 > 64) atomicOr(&mask[w + 1], pat >> (64 - sh));
            }
            boff += (int64_t)h0 * h1;
        }
        __syncthreads();
        for (int w = lane; w < P.words; w += 64) P.masks[c * P.words + w] = mask[w];
        if (lane == 0) P.labels[c] = label;
        __syncthreads();
    }
}

// Gain of every candidate (pairs it covers beyond `covered`), reduced to
// the largest gain, lowest candidate index first: key = gain 2^40 + (2^40 -
// 1 - index).
__global__ void __launch_bounds__(256) cov_gain_kernel(const unsigned long long *masks, int64_t n_cand, int words,
                                                       const unsigned long long *covered,
                                                       unsigned long long *best_key) {
    __shared__ unsigned long long cov[kCovSearchMaxWords];
    __shared__ unsigned long long red[4];
    for (int w = threadIdx.x; w < words; w += blockDim.x) cov[w] = covered[w];
    __syncthreads();
    unsigned long long key = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_cand;
         c += (int64_t)gridDim.x * blockDim.x) {
        int gain = 0;
        for (int w = 0; w < words; ++w) gain += __popcll(masks[c * words + w] & ~cov[w]);
        const unsigned long long k =
            ((unsigned long long)gain << 40) | (((1ull << 40) - 1ull) - (unsigned long long)c);
        if (gain > 0 && k > key) key = k;
    }
    for (int sh = 32; sh >= 1; sh >>= 1) {
        const unsigned long long o = __shfl_xor(key, sh);
        key = o > key ? o : key;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = red[0];
        for (int t = 1; t < (int)(blockDim.x >> 6); ++t) b = red[t] > b ? red[t] : b;
        if (b) atomicMax(best_key, b);
    }
}

__global__ void cov_take_kernel(const unsigned long long *masks, int words, const unsigned long long *best_key,
                                unsigned long long *covered, const int32_t *labels, int32_t *label_out) {
    const unsigned long long key = *best_key;
    if (!key) {
        if (threadIdx.x == 0) *label_out = -1;
        return;
    }
    const int64_t c = (int64_t)(((1ull << 40) - 1ull) - (key & ((1ull << 40) - 1ull)));
    for (int w = threadIdx.x; w < words; w += blockDim.x) covered[w] |= masks[c * words + w];
    if (threadIdx.x == 0) *label_out = labels[c];
}

hipError_t launch_cov_cand(const CovCandParams &P, hipStream_t s) {
    if (P.n_cand <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(P.n_cand, 16384);
    hipLaunchKernelGGL(cov_cand_kernel, dim3(grid), dim3(64), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_cov_gain(const unsigned long long *masks, int64_t n_cand, int words,
                           const unsigned long long *covered, unsigned long long *best_key, hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_cand + 255) / 256, 2048));
    hipLaunchKernelGGL(cov_gain_kernel, dim3(grid), dim3(256), 0, s, masks, n_cand, words, covered, best_key);
    return hipGetLastError();
}

hipError_t launch_cov_take(const unsigned long long *masks, int words, const unsigned long long *best_key,
                           unsigned long long *covered, const int32_t *labels, int32_t *label_out, hipStream_t s) {
    hipLaunchKernelGGL(cov_take_kernel, dim3(1), dim3(64), 0, s, masks, words, best_key, covered, labels, label_out);
    return hipGetLastError();
}

}  // namespace ibmc
