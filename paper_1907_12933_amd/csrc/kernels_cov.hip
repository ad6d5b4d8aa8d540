// Coverage kernels (the SS / DS / SV / DV neuron-pair covers; pairs of
// images go through the one-pass kernel of kernels_covpair.hip):
//  1. fwd_pots_q8_kernel: every layer's exact potentials of a batch of
//     images on int8 MFMA (natural K order; activations staged in LDS, the
//     output tiles split over a workgroup's waves), for the forward entry
//     point and the clean image of test generation;
//  2. cov_pred_kernel: per pair of given potentials (int64, from the host),
//     sign / value change masks of every layer as wavefront ballots,
//     sign-change counts by popcount, the layer distance, then the covered
//     rows OR-ed into device bitmasks;
//  3. cov_sum_kernel / cov_expand_kernel: covered pairs, covered neurons and
//     the caller's packed bit layout.
#include "kernels_cov.h"

namespace ibmc {

// ---------------------------------------------------------------------------
// 1. forward potentials
// ---------------------------------------------------------------------------

constexpr int kFwdTile = 16;                  // images per workgroup (one MFMA N-tile)
constexpr int kFwdWaves = 16;                 // waves per workgroup: they split every layer's output tiles
constexpr int kFwdAB = 4;                     // weight tiles loaded ahead of their MFMAs

__device__ __forceinline__ int fwd_requant_byte(int acc_minus_off, int s) {
    // acc - 64 * 2^s -> a - 64 with a = clamp(floor(u / 2^s), 0, 127)
    const int lim = 64 << s;
    const int v = min(max(acc_minus_off, -lim), lim - 1);
    return (v >> s) & 0xff;
}

// One workgroup of kFwdWaves waves per 16 images; wave w computes the
// 16-row output tiles w, w + kFwdWaves, ... of every layer (K-blocks in
// groups of kFwdAB: the group's weight tiles are loaded first, then chained
// through the MFMAs).  LDS: two activation buffers of 16 x 1024 int8 (the
// offset form a - 64; the input layer holds x - 128), and the per-wave label
// candidates.
__global__ void __launch_bounds__(64 * kFwdWaves) fwd_pots_q8_kernel(QNetDev net, FwdExtra fx, const uint8_t *images,
                                                                     int64_t n_images, int32_t *pots,
                                                                     int64_t pot_stride, int32_t *labels) {
    __shared__ __attribute__((aligned(16))) int8_t act[2][kFwdTile][kMaxWidth];
    __shared__ int candv[kFwdWaves][kFwdTile], candi[kFwdWaves][kFwdTile];
    // the wave index as a scalar: the compiler then sees every M-tile
    // condition as wave-uniform (no exec-masked MFMAs, loads run ahead)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j16 = lane & 15, g = lane >> 4;
    const int n = net.dims[0];
    const int K0 = fx.K0;                      // pixels padded to 64
    for (int64_t tile = blockIdx.x; tile * kFwdTile < n_images; tile += gridDim.x) {
        const int64_t img0 = tile * kFwdTile;
        // stage x - 128 (zero padding beyond n and beyond the last image)
        for (int t = threadIdx.x; t < kFwdTile * K0; t += blockDim.x) {
            const int jj = t / K0, pix = t - jj * K0;
            const int64_t img = img0 + jj;
            int8_t v = 0;
            if (img < n_images && pix < n) v = (int8_t)((int)images[img * n + pix] - 128);
            act[0][jj][pix] = v;
        }
        __syncthreads();
        int cur = 0;
        int64_t po = 0;
        const int64_t myimg = img0 + j16;
        int bestv = INT32_MIN, besti = 0x7fffffff;
        for (int l = 1; l <= net.L; ++l) {
            const int KB = (l == 1) ? K0 / 64 : net.H[l - 1] / 64;
            const int MT = net.H[l] / 16;
            const int8_t *tiles = (l == 1) ? net.W1tile : fx.Wn[l];
            const int32_t *init = fx.init[l];
            const bool hidden = l < net.L;
            const int s = hidden ? net.shift[l - 1] : 0;
            const int off = hidden ? (64 << s) : 0;
            const int nout = net.dims[l];
            for (int mt = wave; mt < MT; mt += kFwdWaves) {
                const int4 b = *reinterpret_cast<const int4 *>(init + mt * 16 + g * 4);
                v4i acc = {b.x, b.y, b.z, b.w};
                const v4i *Ap = reinterpret_cast<const v4i *>(tiles) + (int64_t)mt * KB * 64 + lane;
                for (int k0 = 0; k0 < KB; k0 += kFwdAB) {
                    v4i A[kFwdAB];
#pragma unroll
                    for (int z = 0; z < kFwdAB; ++z)
                        if (k0 + z < KB) A[z] = Ap[(k0 + z) * 64];
#pragma unroll
                    for (int z = 0; z < kFwdAB; ++z) {
                        if (k0 + z < KB) {
                            const v4i B = *reinterpret_cast<const v4i *>(&act[cur][j16][(k0 + z) * 64 + g * 16]);
                            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[z], B, acc, 0, 0, 0);
                        }
                    }
                }
                // potentials of neurons 16 mt + 4 g + t for image j16
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int neuron = mt * 16 + g * 4 + t;
                    const int u = acc[t] + off;
                    if (neuron < nout && myimg < n_images) {
                        if (pots) pots[myimg * pot_stride + po + neuron] = u;
                        if (!hidden) {
                            if (u > bestv) { bestv = u; besti = neuron; }
                            else if (u == bestv) besti = min(besti, neuron);
                        }
                    }
                }
                if (hidden) {
                    int packed = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) packed |= fwd_requant_byte(acc[t], s) << (8 * t);
                    *reinterpret_cast<int *>(&act[cur ^ 1][j16][mt * 16 + g * 4]) = packed;
                }
            }
            po += nout;
            __syncthreads();
            cur ^= 1;
        }
        // label: the four lane groups of each image, then the waves
#pragma unroll
        for (int sh = 16; sh <= 32; sh <<= 1) {
            const int ov = __shfl_xor(bestv, sh), oi = __shfl_xor(besti, sh);
            if (ov > bestv) { bestv = ov; besti = oi; }
            else if (ov == bestv) besti = min(besti, oi);
        }
        if (g == 0) {
            candv[wave][j16] = bestv;
            candi[wave][j16] = besti;
        }
        __syncthreads();
        if (wave == 0 && g == 0) {
            for (int w = 1; w < kFwdWaves; ++w) {
                const int ov = candv[w][j16], oi = candi[w][j16];
                if (ov > bestv) { bestv = ov; besti = oi; }
                else if (ov == bestv) besti = min(besti, oi);
            }
            if (labels && myimg < n_images) labels[myimg] = besti;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 2. predicates and pair accumulation
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long sat_add_u64(unsigned long long a, unsigned long long b) {
    const unsigned long long s = a + b;
    return s < a ? ~0ull : s;
}

constexpr int kPredAB = 4;   // 64-neuron chunks whose potentials are loaded ahead of their tests

template <class T>
__global__ void __launch_bounds__(64) cov_pred_kernel(const T *pots1, const T *pots2, int64_t n_pairs,
                                                      CovLayout lay, CovParams cp, CovBits bits) {
    __shared__ uint32_t scm[kMaxLayers][kMaxWidth / 32];
    __shared__ uint32_t vcm[kMaxLayers][kMaxWidth / 32];
    const int lane = threadIdx.x;
    for (int64_t pr = blockIdx.x; pr < n_pairs; pr += gridDim.x) {
        const T *a1 = pots1 + pr * lay.U, *a2 = pots2 + pr * lay.U;
        int nsc[kMaxLayers], istar[kMaxLayers], dc[kMaxLayers];
        for (int l = 0; l < lay.nl; ++l) {
            const int w = lay.width[l];
            const T *x = a1 + lay.uoff[l], *y = a2 + lay.uoff[l];
            int count = 0, first = -1;
            unsigned long long dist = 0;           // this lane's share (saturating sums are associative)
            for (int c1 = 0; c1 < w; c1 += 64 * kPredAB) {
                T xv[kPredAB], yv[kPredAB];
#pragma unroll
                for (int z = 0; z < kPredAB; ++z) {
                    const int i = c1 + 64 * z + lane;
                    xv[z] = i < w ? x[i] : T(0);
                    yv[z] = i < w ? y[i] : T(0);
                }
#pragma unroll
                for (int z = 0; z < kPredAB; ++z) {
                    const int c0 = c1 + 64 * z;
                    if (c0 >= w) break;
                    const int i = c0 + lane;
                    bool sc = false, vc = false;
                    unsigned long long d2 = 0;
                    if (i < w) {
                        const int64_t a = (int64_t)xv[z], b = (int64_t)yv[z];
                        const bool sa = a >= 0, sb = b >= 0;   // sign(0) = 1
                        sc = sa != sb;
                        const int64_t aa = a < 0 ? -a : a, bb = b < 0 ? -b : b;
                        const int64_t mx = aa > bb ? aa : bb, mn = aa > bb ? bb : aa;
                        vc = !sc && mx > 0 && (int64_t)cp.ratio_den * mx >= (int64_t)cp.ratio_num * mn;
                        const int64_t d = a - b;
                        const unsigned long long ad = (unsigned long long)(d < 0 ? -d : d);
                        // |d| < 2^32 for int32 potentials; larger (int64 input) saturates
                        d2 = (ad >> 32) ? ~0ull : ad * ad;
                    }
                    const unsigned long long sm = __ballot(sc), vm = __ballot(vc);
                    if (lane == 0) {
                        scm[l][c0 / 32] = (uint32_t)sm;
                        vcm[l][c0 / 32] = (uint32_t)vm;
                        if (c0 + 32 < kMaxWidth) {
                            scm[l][c0 / 32 + 1] = (uint32_t)(sm >> 32);
                            vcm[l][c0 / 32 + 1] = (uint32_t)(vm >> 32);
                        }
                    }
                    if (sm && first < 0) first = c0 + __ffsll((long long)sm) - 1;
                    count += __popcll(sm);
                    dist = sat_add_u64(dist, d2);
                }
            }
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) dist = sat_add_u64(dist, __shfl_xor(dist, sh));
            nsc[l] = count;
            istar[l] = first;
            dc[l] = count == 0 && dist >= (unsigned long long)cp.dist_sq_min;
        }
        __syncthreads();
        // covered rows: a single sign change at i* (SS / SV) or a distance
        // change of the whole layer (DS / DV, every condition neuron)
        for (int l = 0; l + 1 < lay.nl; ++l) {
            const int W = lay.words[l + 1];
            if (nsc[l] == 1) {
                const int64_t row = lay.rowoff[l] + (int64_t)istar[l] * W;
                for (int t = lane; t < W; t += 64) {
                    const uint32_t s = scm[l + 1][t], v = vcm[l + 1][t];
                    if (s) atomicOr(bits.rows_ss + row + t, s);
                    if (v) atomicOr(bits.rows_sv + row + t, v);
                }
            }
            if (dc[l]) {
                for (int t = lane; t < W; t += 64) {
                    const uint32_t s = scm[l + 1][t], v = vcm[l + 1][t];
                    if (s) atomicOr(bits.all_ds + lay.alloff[l] + t, s);
                    if (v) atomicOr(bits.all_dv + lay.alloff[l] + t, v);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3. summaries and the caller's bit layout
// ---------------------------------------------------------------------------

// grid: (groups of kSumRows rows of block l, criterion).  For SS / SV: per
// row, any bit -> condition neuron covered, OR into the column mask, count
// bits.  For DS / DV the block is "all rows x allrows-mask".  A row holds at
// most kMaxWidth / 32 words, one per lane; each lane ORs its column over the
// group's rows and touches the shared column mask once.
constexpr int kSumRows = 8;
static_assert(kMaxWidth / 32 <= 64, "one mask word per lane");

__global__ void __launch_bounds__(64) cov_sum_kernel(CovLayout lay, CovBits bits, int l, CovSums sums) {
    const int crit = blockIdx.y;   // 0 SS, 1 DS, 2 SV, 3 DV
    const bool per_row = crit == 0 || crit == 2;
    const int W = lay.words[l + 1];
    const int rows = lay.width[l];
    const int lane = threadIdx.x;
    const int r0 = blockIdx.x * kSumRows;
    int cnt = 0;
    uint32_t col = 0;
    for (int rr = 0; rr < kSumRows && r0 + rr < rows; ++rr) {
        const int row = r0 + rr;
        const uint32_t *src = per_row
                                  ? (crit == 0 ? bits.rows_ss : bits.rows_sv) + lay.rowoff[l] + (int64_t)row * W
                                  : (crit == 1 ? bits.all_ds : bits.all_dv) + lay.alloff[l];
        const uint32_t v = lane < W ? src[lane] : 0u;
        cnt += __popc(v);
        col |= v;
        if (__ballot(v != 0) && lane == 0) sums.condflag[(int64_t)crit * sums.flag_stride + lay.uoff[l] + row] = 1;
    }
    if (col && (per_row || blockIdx.x == 0))
        atomicOr(sums.colmask + (int64_t)crit * sums.colmask_stride + lay.alloff[l] + lane, col);
    for (int sh = 32; sh >= 1; sh >>= 1) cnt += __shfl_xor(cnt, sh);
    if (lane == 0 && cnt) atomicAdd(sums.pairs + crit, (unsigned long long)cnt);
}

// Neuron count per criterion: condition flags OR decision bits of the
// previous block's column mask.
__global__ void __launch_bounds__(256) cov_neurons_kernel(CovLayout lay, CovSums sums) {
    const int crit = blockIdx.x;
    int cnt = 0;
    for (int u = threadIdx.x; u < lay.U; u += blockDim.x) {
        int l = 0;
        while (l + 1 < lay.nl && u >= lay.uoff[l + 1]) ++l;
        const int i = u - lay.uoff[l];
        bool cov = sums.condflag[(int64_t)crit * sums.flag_stride + u] != 0;
        if (l > 0) {
            const uint32_t wv = sums.colmask[(int64_t)crit * sums.colmask_stride + lay.alloff[l - 1] + i / 32];
            cov |= (wv >> (i % 32)) & 1u;
        }
        cnt += cov;
    }
    for (int sh = 32; sh >= 1; sh >>= 1) cnt += __shfl_xor(cnt, sh);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(sums.neurons + crit, (unsigned long long)cnt);
}

// The caller's layout: bit off_l + i * h_{l+1} + j, 64 bits per word.
__global__ void __launch_bounds__(256) cov_expand_kernel(CovLayout lay, CovBits bits, int crit, uint64_t *out,
                                                         int64_t n_words) {
    for (int64_t wd = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; wd < n_words;
         wd += (int64_t)gridDim.x * blockDim.x) {
        uint64_t v = 0;
        for (int b = 0; b < 64; ++b) {
            const int64_t t = wd * 64 + b;
            if (t >= lay.total_pairs) break;
            int l = 0;
            while (l + 2 < lay.nl && t >= lay.pairoff[l + 1]) ++l;
            const int64_t r = t - lay.pairoff[l];
            const int hn = lay.width[l + 1];
            const int i = (int)(r / hn), j = (int)(r - (int64_t)i * hn);
            uint32_t w;
            if (crit == 0 || crit == 2)
                w = (crit == 0 ? bits.rows_ss : bits.rows_sv)[lay.rowoff[l] + (int64_t)i * lay.words[l + 1] + j / 32];
            else
                w = (crit == 1 ? bits.all_ds : bits.all_dv)[lay.alloff[l] + j / 32];
            v |= (uint64_t)((w >> (j % 32)) & 1u) << b;
        }
        out[wd] = v;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_fwd_pots_q8(const QNetDev &net, const FwdExtra &fx, const uint8_t *images, int64_t n_images,
                              int32_t *pots, int64_t pot_stride, int32_t *labels, hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    const int64_t tiles = (n_images + kFwdTile - 1) / kFwdTile;
    const int grid = (int)std::min<int64_t>(tiles, 8192);
    hipLaunchKernelGGL(fwd_pots_q8_kernel, dim3(grid), dim3(64 * kFwdWaves), 0, s, net, fx, images, n_images, pots,
                       pot_stride, labels);
    return hipGetLastError();
}

hipError_t launch_cov_pred_i64(const int64_t *p1, const int64_t *p2, int64_t n_pairs, const CovLayout &lay,
                               const CovParams &cp, const CovBits &bits, hipStream_t s) {
    if (n_pairs <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_pairs, 16384);
    hipLaunchKernelGGL(cov_pred_kernel<int64_t>, dim3(grid), dim3(64), 0, s, p1, p2, n_pairs, lay, cp, bits);
    return hipGetLastError();
}

hipError_t launch_cov_summary(const CovLayout &lay, const CovBits &bits, const CovSums &sums, hipStream_t s) {
    for (int l = 0; l + 1 < lay.nl; ++l) {
        hipLaunchKernelGGL(cov_sum_kernel, dim3((lay.width[l] + kSumRows - 1) / kSumRows, 4), dim3(64), 0, s, lay,
                           bits, l, sums);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(cov_neurons_kernel, dim3(4), dim3(256), 0, s, lay, sums);
    return hipGetLastError();
}

hipError_t launch_cov_expand(const CovLayout &lay, const CovBits &bits, int crit, uint64_t *out, int64_t n_words,
                             hipStream_t s) {
    if (n_words <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n_words + 255) / 256, 4096);
    hipLaunchKernelGGL(cov_expand_kernel, dim3(grid), dim3(256), 0, s, lay, bits, crit, out, n_words);
    return hipGetLastError();
}

}  // namespace ibmc
