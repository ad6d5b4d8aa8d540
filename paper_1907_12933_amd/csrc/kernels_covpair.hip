// Pair coverage in one pass (the SS / DS / SV / DV covers of Sec. III-B,
// Eqs. (3)-(6), over input pairs (x1, x2)): a workgroup takes 16 pairs,
// runs both images of every pair through the network on int8 MFMA and tests
// every neuron of every layer on the fly, so that no potential ever goes to
// memory.
//
// Columns of the MFMA B operand: N-tile 0 holds x1 of the 16 pairs, N-tile 1
// x2 of the same pairs, so the accumulators of a pair's
// two images for the same four neurons sit in the same lane.  x2's first
// layer is the rank-r update of x1's (Eq. (1)): u1(x2) = u1(x1) + sum over
// the r pixels where x2 differs of (x2_p - x1_p) W1[:, p], r <= kPairRank
// (else the whole tile runs x2's first layer on the matrix cores too).
//
// Every wave (eight per workgroup) owns up to eight 16-row M-tiles of each
// layer and keeps their accumulators for both N-tiles in registers (each
// weight tile loaded once feeds two MFMAs, each activation fragment read
// from LDS feeds up to eight).  (32 pairs per workgroup, four N-tiles, made
// the compiler spill at 256 registers.)  After a layer: the sign / value changes of every neuron as 4-bit
// nibbles per pair in LDS, the squared distance as per-wave partial sums,
// and (hidden layers) the requantised activations written back over the
// layer's inputs.  At the end every pair's counts, first sign change and
// distance decide its covered rows, which are OR-ed into the device masks
// as the potential-based predicate kernel does (the all-rows masks of DS /
// DV, which every pair with a distance change ORs into the same few words,
// are gathered per tile in LDS and flushed with one atomic per word).
#include <algorithm>

#include "kernels_cov.h"

namespace ibmc {

constexpr int kPairWaves = 8;
constexpr int kPairRank = 16;
constexpr int kPairMaxMt = 8;   // M-tiles per wave (widths <= 1024)

__device__ __forceinline__ unsigned long long sat_add(unsigned long long a, unsigned long long b) {
    const unsigned long long s = a + b;
    return s < a ? ~0ull : s;
}

__device__ __forceinline__ int pair_requant_byte(int acc_minus_off, int s) {
    const int lim = 64 << s;
    const int v = min(max(acc_minus_off, -lim), lim - 1);
    return (v >> s) & 0xff;
}

// One layer's MFMAs when every wave owns exactly NMT M-tiles (mt = wave +
// kPairWaves i): no per-tile conditions, and each K-block's weight tiles are
// loaded one block ahead of their MFMAs (two register sets, the K loop
// unrolled by two).  ncm: N-tiles that take MFMAs (wave-uniform).
template <int NMT, int NC>
__device__ __forceinline__ void pair_layer_mfma(v4i (&acc)[kPairMaxMt][NC], const v4i *tiles, int wave, int KB,
                                                int ncm, const int8_t *act, int RS, int j16, int g, int lane) {
    v4i A0[NMT], A1[NMT];
    auto load = [&](v4i (&A)[NMT], int kb) {
#pragma unroll
        for (int i = 0; i < NMT; ++i) A[i] = tiles[((int64_t)(wave + kPairWaves * i) * KB + kb) * 64 + lane];
    };
    auto step = [&](const v4i (&A)[NMT], int kb) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c < ncm) {
                const v4i B = *reinterpret_cast<const v4i *>(act + (c * 16 + j16) * RS + kb * 64 + g * 16);
#pragma unroll
                for (int i = 0; i < NMT; ++i) acc[i][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[i], B, acc[i][c], 0, 0, 0);
            }
        }
    };
    load(A0, 0);
    for (int kb = 0; kb < KB; kb += 2) {
        if (kb + 1 < KB) load(A1, kb + 1);
        step(A0, kb);
        if (kb + 1 < KB) {
            if (kb + 2 < KB) load(A0, kb + 2);
            step(A1, kb + 1);
        }
    }
}

template <int NX>
__global__ void __launch_bounds__(64 * kPairWaves) cov_pair_kernel(CovPairParams P) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    constexpr int NC = 2 * NX;          // N-tiles
    constexpr int NP = 16 * NX;         // pairs per tile
    const QNetDev &net = P.net;
    const FwdExtra &fx = P.fx;
    const CovLayout &lay = P.lay;
    const int L = net.L, n = net.dims[0];
    const int RS = P.act_stride;        // bytes per activation row
    int8_t *act = reinterpret_cast<int8_t *>(smem);                       // [NC * 16][RS]
    uint8_t *nib = reinterpret_cast<uint8_t *>(smem + P.off_nib);         // [NP][nib_stride]
    unsigned long long *dist = reinterpret_cast<unsigned long long *>(smem + P.off_dist);  // [L][NP][waves]
    int *dlist = reinterpret_cast<int *>(smem + P.off_diff);              // [NP][kPairRank]
    int *dcount = dlist + NP * kPairRank;                                 // [NP]
    int *flags = dcount + NP;                                             // [1]: dense
    // the tile's OR of the all-rows (DS, DV) masks, flushed once per tile
    uint32_t *tds = reinterpret_cast<uint32_t *>(smem + P.off_all);        // [all_words]
    uint32_t *tdv = tds + lay.all_words;                                   // [all_words]
    // the wave index as a scalar: the compiler then sees every M-tile
    // condition as wave-uniform (no exec-masked MFMAs, loads run ahead)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j16 = lane & 15, g = lane >> 4;
    const int K0 = fx.K0;
    for (int64_t tile = blockIdx.x; tile * NP < P.n_pairs; tile += gridDim.x) {
        const int64_t pair0 = tile * NP;
        if (threadIdx.x == 0) flags[0] = 0;
        for (int t = threadIdx.x; t < 2 * lay.all_words; t += blockDim.x) tds[t] = 0u;
        __syncthreads();
        // stage x - 128 of both images (zeros past the last pair and past n):
        // wave w takes rows w, w + waves, ...; lanes take four pixels each
        for (int col = wave; col < NC * 16; col += kPairWaves) {
            const int64_t pg = pair0 + col % NP;
            const uint8_t *src = (col < NP ? P.x1 : P.x2) + pg * n;
            const bool live = pg < P.n_pairs;
            for (int p4 = lane * 4; p4 < K0; p4 += 256) {
                uint32_t w = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int pix = p4 + e;
                    const uint32_t v = (live && pix < n) ? (uint32_t)(uint8_t)((int)src[pix] - 128) : 0u;
                    w |= v << (8 * e);
                }
                *reinterpret_cast<uint32_t *>(act + col * RS + p4) = w;
            }
        }
        // x2 - x1: the changed pixels of each pair (one wave per pair)
        for (int pr = wave; pr < NP; pr += kPairWaves) {
            const int64_t pg = pair0 + pr;
            int cnt = 0;
            if (pg < P.n_pairs) {
                const uint8_t *a = P.x1 + pg * n, *b = P.x2 + pg * n;
                for (int p0 = 0; p0 < n; p0 += 64) {
                    const int p = p0 + lane;
                    const int d = p < n ? (int)b[p] - (int)a[p] : 0;
                    const unsigned long long m = __ballot(d != 0);
                    const int slot = cnt + __popcll(m & ((1ull << lane) - 1ull));
                    if (d != 0 && slot < kPairRank) dlist[pr * kPairRank + slot] = (p << 16) | (d & 0xffff);
                    cnt += __popcll(m);
                }
            }
            if (lane == 0) {
                dcount[pr] = cnt;
                if (cnt > kPairRank) flags[0] = 1;
            }
        }
        __syncthreads();
        const bool dense = flags[0] != 0;
        for (int l = 1; l <= L; ++l) {
            const int KB = (l == 1) ? K0 / 64 : net.H[l - 1] / 64;
            const int MT = net.H[l] / 16;
            const int8_t *tiles = (l == 1) ? net.W1tile : fx.Wn[l];
            const int32_t *init = fx.init[l];
            const bool hidden = l < L;
            const int s = hidden ? net.shift[l - 1] : 0;
            const int off = hidden ? (64 << s) : 0;
            // x2's first layer comes from the rank-r update unless the tile is dense
            const int ncm = (l == 1 && !dense) ? NX : NC;
            v4i acc[kPairMaxMt][NC];
#pragma unroll
            for (int i = 0; i < kPairMaxMt; ++i) {
                const int mt = wave + kPairWaves * i;
                if (mt < MT) {
                    const int4 b = *reinterpret_cast<const int4 *>(init + mt * 16 + g * 4);
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[i][c] = v4i{b.x, b.y, b.z, b.w};
                }
            }
            const int nmt = (MT % kPairWaves == 0) ? MT / kPairWaves : 0;   // M-tiles of every wave
            const v4i *tv = reinterpret_cast<const v4i *>(tiles);
            if (nmt == 8) {
                pair_layer_mfma<8>(acc, tv, wave, KB, ncm, act, RS, j16, g, lane);
            } else if (nmt == 4) {
                pair_layer_mfma<4>(acc, tv, wave, KB, ncm, act, RS, j16, g, lane);
            } else if (nmt == 2) {
                pair_layer_mfma<2>(acc, tv, wave, KB, ncm, act, RS, j16, g, lane);
            } else if (nmt == 1) {
                pair_layer_mfma<1>(acc, tv, wave, KB, ncm, act, RS, j16, g, lane);
            } else if (wave < MT) {
                for (int kb = 0; kb < KB; ++kb) {
                    v4i A[kPairMaxMt];
#pragma unroll
                    for (int i = 0; i < kPairMaxMt; ++i) {
                        const int mt = wave + kPairWaves * i;
                        if (mt < MT) A[i] = reinterpret_cast<const v4i *>(tiles)[((int64_t)mt * KB + kb) * 64 + lane];
                    }
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (c < ncm) {
                            const v4i B = *reinterpret_cast<const v4i *>(act + (c * 16 + j16) * RS + kb * 64 + g * 16);
#pragma unroll
                            for (int i = 0; i < kPairMaxMt; ++i)
                                if (wave + kPairWaves * i < MT)
                                    acc[i][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[i], B, acc[i][c], 0, 0, 0);
                        }
                    }
                }
            }
            {
                if (l == 1 && !dense) {
                    // u1(x2) = u1(x1) + sum (x2_p - x1_p) W1[:, p]; W1T rows are in
                    // sigma order, where neurons 16 mt + 4 g + 0..3 are four
                    // consecutive bytes
#pragma unroll
                    for (int c = 0; c < NX; ++c) {
                        const int pr = c * 16 + j16;
                        const int cnt = dcount[pr];
#pragma unroll
                        for (int i = 0; i < kPairMaxMt; ++i) {
                            const int mt = wave + kPairWaves * i;
                            if (mt < MT) {
                                v4i u = acc[i][c];
                                const int q = sigma64(mt * 16 + g * 4);
                                for (int e = 0; e < cnt; ++e) {
                                    const int ent = dlist[pr * kPairRank + e];
                                    const int p = ent >> 16, d = (int)(short)(ent & 0xffff);
                                    const int w4 = *reinterpret_cast<const int *>(net.W1T + (int64_t)p * net.H[1] + q);
                                    u[0] += d * (int)(int8_t)(w4 & 0xff);
                                    u[1] += d * (int)(int8_t)((w4 >> 8) & 0xff);
                                    u[2] += d * (int)(int8_t)((w4 >> 16) & 0xff);
                                    u[3] += d * (int)(int8_t)(w4 >> 24);
                                }
                                acc[i][c + NX] = u;
                            }
                        }
                    }
                }
            }
            __syncthreads();   // every wave has read this layer's inputs
            // the layer's tests: nibbles of sign / value changes, distance partials
            const int nout = net.dims[l];
            const int nbo = P.nib_off[l];
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                // the squared distance as a 64-bit sum plus a count of its
                // carries (saturated once, after the layer)
                unsigned long long dlo = 0;
                uint32_t dhi = 0;
#pragma unroll
                for (int i = 0; i < kPairMaxMt; ++i) {
                    const int mt = wave + kPairWaves * i;
                    if (mt < MT) {
                        int sn = 0, vn = 0;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int r = mt * 16 + g * 4 + t;
                            if (r < nout) {
                                // potentials fit int32 (the loader's headroom check);
                                // |a - b| < 2^32 is |a| + |b| across a sign change,
                                // else max - min of the magnitudes
                                const int a = acc[i][c][t] + off, b = acc[i][c + NX][t] + off;
                                const bool sc = (a ^ b) < 0;   // the signs differ (sign(0) = 1)
                                const uint32_t aa = a < 0 ? 0u - (uint32_t)a : (uint32_t)a;
                                const uint32_t bb = b < 0 ? 0u - (uint32_t)b : (uint32_t)b;
                                const uint32_t mx = aa > bb ? aa : bb, mn = aa > bb ? bb : aa;
                                const bool vc = !sc && mx > 0 &&
                                                (uint64_t)(uint32_t)P.cp.ratio_den * mx >=
                                                    (uint64_t)(uint32_t)P.cp.ratio_num * mn;
                                const uint32_t ad = sc ? aa + bb : mx - mn;
                                const unsigned long long nl = dlo + (unsigned long long)ad * ad;
                                dhi += nl < dlo;
                                dlo = nl;
                                sn |= (int)sc << t;
                                vn |= (int)vc << t;
                            }
                        }
                        nib[(c * 16 + j16) * P.nib_stride + nbo + mt * 4 + g] = (uint8_t)(sn | (vn << 4));
                    }
                }
                unsigned long long dsum = dhi ? ~0ull : dlo;
                dsum = sat_add(dsum, __shfl_xor(dsum, 16));
                dsum = sat_add(dsum, __shfl_xor(dsum, 32));
                if (g == 0) dist[((l - 1) * NP + c * 16 + j16) * kPairWaves + wave] = dsum;
            }
            if (hidden) {
#pragma unroll
                for (int i = 0; i < kPairMaxMt; ++i) {
                    const int mt = wave + kPairWaves * i;
                    if (mt < MT) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            int packed = 0;
#pragma unroll
                            for (int t = 0; t < 4; ++t) packed |= pair_requant_byte(acc[i][c][t], s) << (8 * t);
                            *reinterpret_cast<int *>(act + (c * 16 + j16) * RS + mt * 16 + g * 4) = packed;
                        }
                    }
                }
            }
            __syncthreads();
        }
        // per pair: counts, first sign change and distance of every layer, then
        // the covered rows (one wave per pair)
        for (int pr = wave; pr < NP; pr += kPairWaves) {
            if (pair0 + pr >= P.n_pairs) continue;
            const uint8_t *nb = nib + pr * P.nib_stride;
            // layer by layer: this layer's count, first sign change and
            // distance; then block l - 1 (rows of layer l - 1, bits of layer l)
            int pcnt = 0, pfirst = 0;
            bool pdc = false;
            for (int l = 0; l < lay.nl; ++l) {
                const int nbytes = net.H[l + 1] / 4, nbo = P.nib_off[l + 1];
                if (l > 0 && (pcnt == 1 || pdc)) {
                    const int W = lay.words[l];
                    for (int t = lane; t < W; t += 64) {
                        uint32_t sw = 0, vw = 0;
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const int b = 8 * t + k;
                            const int v = b < nbytes ? nb[nbo + b] : 0;
                            sw |= (uint32_t)(v & 15) << (4 * k);
                            vw |= (uint32_t)(v >> 4) << (4 * k);
                        }
                        if (pcnt == 1) {
                            const int64_t row = lay.rowoff[l - 1] + (int64_t)pfirst * W;
                            if (sw) atomicOr(P.bits.rows_ss + row + t, sw);
                            if (vw) atomicOr(P.bits.rows_sv + row + t, vw);
                        }
                        if (pdc) {
                            // every pair of the tile ORs the same words: gather in LDS
                            if (sw) atomicOr(tds + lay.alloff[l - 1] + t, sw);
                            if (vw) atomicOr(tdv + lay.alloff[l - 1] + t, vw);
                        }
                    }
                }
                int cnt = 0, first = 0x7fffffff;
                for (int b0 = 0; b0 < nbytes; b0 += 64) {
                    const int b = b0 + lane;
                    const int v = b < nbytes ? (nb[nbo + b] & 15) : 0;
                    cnt += __popc(v);
                    if (v) first = min(first, 4 * b + __ffs(v) - 1);
                }
                unsigned long long dsum = lane < kPairWaves ? dist[(l * NP + pr) * kPairWaves + lane] : 0ull;
#pragma unroll
                for (int sh = 32; sh >= 1; sh >>= 1) {
                    cnt += __shfl_xor(cnt, sh);
                    first = min(first, __shfl_xor(first, sh));
                    dsum = sat_add(dsum, __shfl_xor(dsum, sh));
                }
                pcnt = cnt;
                pfirst = first;
                pdc = cnt == 0 && dsum >= (unsigned long long)P.cp.dist_sq_min;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < lay.all_words; t += blockDim.x) {
            if (tds[t]) atomicOr(P.bits.all_ds + t, tds[t]);
            if (tdv[t]) atomicOr(P.bits.all_dv + t, tdv[t]);
        }
        __syncthreads();
    }
}

static bool cov_pair_plan(const QNetDev &net, const FwdExtra &fx, int nx, CovPairParams &P, size_t &lds) {
    int hmax = fx.K0;
    for (int l = 1; l < net.L; ++l) hmax = std::max(hmax, net.H[l]);
    P.act_stride = hmax + 16;
    int nbo = 0;
    P.nib_off[0] = 0;
    for (int l = 1; l <= net.L; ++l) {
        P.nib_off[l] = nbo;
        nbo += net.H[l] / 4;
    }
    P.nib_off[net.L + 1] = nbo;
    P.nib_stride = (nbo + 3) & ~3;
    const int NP = 16 * nx;
    size_t o = (size_t)2 * NP * P.act_stride;
    o = (o + 15) & ~(size_t)15;
    P.off_nib = (int)o;
    o += (size_t)NP * P.nib_stride;
    o = (o + 15) & ~(size_t)15;
    P.off_dist = (int)o;
    o += (size_t)net.L * NP * kPairWaves * 8;
    P.off_diff = (int)o;
    o += (size_t)NP * kPairRank * 4 + NP * 4 + 16;
    P.off_all = (int)o;
    o += (size_t)2 * std::max(P.lay.all_words, 1) * 4;
    lds = o;
    return lds <= (size_t)160 * 1024;
}

hipError_t launch_cov_pair(CovPairParams P, int n_cu, hipStream_t s) {
    if (P.n_pairs <= 0) return hipSuccess;
    size_t lds = 0;
    if (!cov_pair_plan(P.net, P.fx, 1, P, lds)) return hipErrorInvalidValue;
    const int64_t tiles = (P.n_pairs + 15) / 16;
    const int grid = (int)std::min<int64_t>(tiles, (int64_t)n_cu * 16);
    hipLaunchKernelGGL(cov_pair_kernel<1>, dim3(grid), dim3(64 * kPairWaves), lds, s, P);
    return hipGetLastError();
}

}  // namespace ibmc
