// The enumeration kernel template (instantiated in enum_q8_*.hip).
#pragma once

#include "kernels_q8.h"
#include "enum_common.h"

namespace ibmc {

__device__ __forceinline__ int requant_relu_e(int u, int s) { return min(max(u >> s, 0), 127); }

__device__ __forceinline__ int pack4_e(int a0, int a1, int a2, int a3) {
    return a0 | (a1 << 8) | (a2 << 16) | (a3 << 24);
}

// Base of the current segment: clean first-layer potentials plus the
// prefix's column updates e * W1[:, p], for the sigma positions this lane
// owns (lane, lane + 64, ...), written to the wave's LDS slice.
template <int KB1>
__device__ void build_base(const Cursor &c, const EnumParams &P, const int32_t *u0s,
                           int32_t *base, int lane) {
    const PropDev &pr = P.props[c.prop];
    const int H1 = KB1 * 64;
    int pp[kMaxK], ee[kMaxK];
    int np = 0;
    if (c.mode == SEG_PLAIN) {
        np = c.k - 1;
        for (int j = 0; j < kMaxK; ++j)
            if (j < np) {
                pp[j] = c.pre[j];
                const int xv = pr.image[pp[j]];
                ee[j] = clamp_pixel(xv + pr.deltas[c.dg[j]]) - xv;
            }
    } else if (c.mode == SEG_SHELL) {
        np = 1;
        const int head = P.jobs[c.job].order[c.shell];
        pp[0] = head / c.m;
        const int xv = pr.image[pp[0]];
        ee[0] = clamp_pixel(xv + pr.deltas[head % c.m]) - xv;
    }
#pragma unroll
    for (int r = 0; r < KB1; ++r) {
        const int q = lane + 64 * r;
        int v = u0s[q];
        for (int j = 0; j < kMaxK; ++j)
            if (j < np) v += ee[j] * (int)P.net.W1T[(int64_t)pp[j] * H1 + q];
        base[q] = v;
    }
}

// The enumeration kernel.  L: weight layers (2 or 3); KB1 / KB2: 64-wide
// K-blocks of the first / second hidden layer; NT: 16-point N-tiles per
// chunk; WLDS: weight tiles of layers >= 2 staged in LDS (else read from
// global memory, which the L2 caches).
template <int L, int KB1, int KB2, int NT, bool WLDS>
__global__ void __launch_bounds__(256) enum_q8_kernel(EnumParams P, const int32_t *u0_store,
                                                      int64_t u0_stride, const int32_t *u0_index) {
    constexpr int CH = 16 * NT;
    constexpr int H1 = KB1 * 64;
    constexpr int H2 = KB2 * 64;
    constexpr int MT2 = (L == 3) ? H2 / 16 : 0;          // 16-row tiles of hidden layer 2
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const QNetDev &net = P.net;
    const int HL = net.H[L];                            // padded classes
    const int MTL = HL / 16;
    const int KBL = (L == 3) ? KB2 : KB1;
    // LDS: [tiles of W2 (if L==3)][tiles of W_L][4 waves x H1 ints of base]
    const int64_t w2_bytes = (L == 3) ? (int64_t)MT2 * KB1 * 1024 : 0;
    const int64_t wl_bytes = (int64_t)MTL * KBL * 1024;
    const int8_t *w2s = net.Wt[2];
    const int8_t *wls = net.Wt[L];
    if constexpr (WLDS) {
        int4 *dst = reinterpret_cast<int4 *>(smem);
        const int64_t n2 = w2_bytes / 16, nl = wl_bytes / 16;
        for (int64_t t = threadIdx.x; t < n2; t += blockDim.x)
            dst[t] = reinterpret_cast<const int4 *>(net.Wt[2])[t];
        for (int64_t t = threadIdx.x; t < nl; t += blockDim.x)
            dst[n2 + t] = reinterpret_cast<const int4 *>(net.Wt[L])[t];
        __syncthreads();
        w2s = reinterpret_cast<const int8_t *>(smem);
        wls = reinterpret_cast<const int8_t *>(smem) + w2_bytes;
    }
    const int64_t wbytes = WLDS ? (w2_bytes + wl_bytes) : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j16 = lane & 15, g = lane >> 4;
    int32_t *base = reinterpret_cast<int32_t *>(smem + wbytes) + wave * H1;

    Cursor c;
    c.job = -1;
    bool have = false;
    int64_t cur_chunk = 0, end_chunk = 0;
    int fetches = 0;
    const int s1 = net.shift[0];
    const int s2 = (L == 3) ? net.shift[1] : 0;
    const int ncls = net.dims[L];

    while (true) {
        if (cur_chunk >= end_chunk) {
            unsigned long long start = 0;
            if (lane == 0) start = atomicAdd(P.queue, (unsigned long long)P.batch);
            start = __shfl(start, 0);
            if ((int64_t)start >= P.total_chunks) break;
            if (*P.stop_flag) break;
            if (P.abort_host && (fetches++ & 15) == 0 && *P.abort_host) break;  // host-mapped: poll sparsely
            cur_chunk = (int64_t)start;
            end_chunk = min((int64_t)start + P.batch, P.total_chunks);
            cursor_decode<CH, EnumParams>(c, P, cur_chunk);
            have = false;
        }
        if (!have) {
            const int32_t *u0s = u0_store + (int64_t)u0_index[c.prop] * u0_stride;
            build_base<KB1>(c, P, u0s, base, lane);
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS writes done
            __builtin_amdgcn_wave_barrier();
            have = true;
        }
        const PropDev &pr = P.props[c.prop];
        const int label0 = pr.label0;

        // ---- layer 1: incremental update + requantisation, into B operands
        v4i a1[NT][KB1];
        bool valid[NT];
        int plast[NT], ilast[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t o = c.ch * CH + nt * 16 + j16;
            int p = 0, i = 0, pf = 0, f = 0;
            valid[nt] = last_element(c, P, o, p, i, pf, f);
            if (!valid[nt]) { p = 0; i = 0; }
            plast[nt] = p;
            ilast[nt] = i;
            const int xv = pr.image[p];
            const int e = clamp_pixel(xv + pr.deltas[i]) - xv;
            const int8_t *wcol = net.W1T + (int64_t)p * H1 + g * 16;
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) {
                const int4 wv = *reinterpret_cast<const int4 *>(wcol + kb * 64);
                const int4 *bp = reinterpret_cast<const int4 *>(base + kb * 64 + g * 16);
                const int wd[4] = {wv.x, wv.y, wv.z, wv.w};
                int out[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int4 bv = bp[t];
                    const int w = wd[t];
                    const int u0 = bv.x + e * (int)(int8_t)(w & 0xff);
                    const int u1 = bv.y + e * (int)(int8_t)((w >> 8) & 0xff);
                    const int u2 = bv.z + e * (int)(int8_t)((w >> 16) & 0xff);
                    const int u3 = bv.w + e * (int)(int8_t)((w >> 24) & 0xff);
                    out[t] = pack4_e(requant_relu_e(u0, s1), requant_relu_e(u1, s1), requant_relu_e(u2, s1),
                                   requant_relu_e(u3, s1));
                }
                a1[nt][kb] = v4i{out[0], out[1], out[2], out[3]};
            }
        }

        // ---- hidden layer 2 (L == 3): int8 MFMA, requantise, repack
        v4i a2[NT][(L == 3) ? KB2 : 1];
        if constexpr (L == 3) {
#pragma unroll
            for (int mt = 0; mt < MT2; ++mt) {
                const int4 bias = *reinterpret_cast<const int4 *>(net.bn[2] + mt * 16 + g * 4);
                v4i acc[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb) {
                    const v4i A = *reinterpret_cast<const v4i *>(w2s + ((int64_t)(mt * KB1 + kb) * 64 + lane) * 16);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, a1[nt][kb], acc[nt], 0, 0, 0);
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    a2[nt][mt >> 2][mt & 3] = pack4_e(requant_relu_e(acc[nt][0], s2), requant_relu_e(acc[nt][1], s2),
                                                    requant_relu_e(acc[nt][2], s2), requant_relu_e(acc[nt][3], s2));
            }
        }

        // ---- output layer: int8 MFMA, lowest-index argmax
        int bestv[NT], besti[NT], bestc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) { bestv[nt] = INT32_MIN; besti[nt] = 0x7fffffff; bestc[nt] = 0; }
        for (int mt = 0; mt < MTL; ++mt) {
            const int4 bias = *reinterpret_cast<const int4 *>(net.bn[L] + mt * 16 + g * 4);
            v4i acc[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
#pragma unroll
            for (int kb = 0; kb < ((L == 3) ? KB2 : KB1); ++kb) {
                const v4i A = *reinterpret_cast<const v4i *>(wls + ((int64_t)(mt * KBL + kb) * 64 + lane) * 16);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    if constexpr (L == 3)
                        acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, a2[nt][kb], acc[nt], 0, 0, 0);
                    else
                        acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, a1[nt][kb], acc[nt], 0, 0, 0);
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int cls = mt * 16 + g * 4 + t;
                    const int v = acc[nt][t];
                    if (cls < ncls) {
                        if (v > bestv[nt]) { bestv[nt] = v; besti[nt] = cls; bestc[nt] = 1; }
                        else if (v == bestv[nt]) { bestc[nt] += 1; besti[nt] = min(besti[nt], cls); }
                    }
                }
            }
        }
        // combine the four lane groups holding the same point
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int sh = 16; sh <= 32; sh <<= 1) {
                const int ov = __shfl_xor(bestv[nt], sh);
                const int oi = __shfl_xor(besti[nt], sh);
                const int oc = __shfl_xor(bestc[nt], sh);
                if (ov > bestv[nt]) { bestv[nt] = ov; besti[nt] = oi; bestc[nt] = oc; }
                else if (ov == bestv[nt]) { besti[nt] = min(besti[nt], oi); bestc[nt] += oc; }
            }
        }

        // ---- decisions, ballot, wave-aggregated compaction
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bool mine = valid[nt] && g == 0;
            const bool viol = mine && besti[nt] != label0;
            const bool tie = mine && bestc[nt] > 1;
            const unsigned long long vm = __ballot(viol);
            const unsigned long long tm = __ballot(tie);
            if (tm && lane == 0) atomicAdd(P.slot_ties + c.slot, (unsigned long long)__popcll(tm));
            if (vm) {
                unsigned long long start = 0;
                if (lane == 0) {
                    start = atomicAdd(P.rec_count, (unsigned long long)__popcll(vm));
                    atomicAdd(P.slot_cex + c.slot, (unsigned long long)__popcll(vm));
                    atomicMin(P.first_chunk, (unsigned long long)c.chunk);
                    if (P.hit_host) *P.hit_host = 1;
                    if (P.stop_on_first) *P.stop_flag = 1;
                }
                start = __shfl(start, 0);
                if (viol) {
                    const unsigned long long below = vm & ((1ull << lane) - 1ull);
                    const int64_t idx = (int64_t)start + __popcll(below);
                    if (idx < P.rec_cap) {
                        CexRec r;
                        r.prop = c.prop;
                        r.k = c.k;
                        r.rank = point_rank(c, P, plast[nt], ilast[nt]);
                        r.label = besti[nt];
                        r.reserved = 0;
                        P.recs[idx] = r;
                    }
                }
            }
        }
        // ---- advance
        cur_chunk++;
        if (cur_chunk < end_chunk) {
            if (cursor_next<CH, EnumParams>(c, P)) have = false;
        }
    }
}

#define IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, WLDS_, TAG_)                                   \
    {L_, KB1_, KB2_, NT_, WLDS_, 16 * NT_, "q8_L" #L_ "_kb" #KB1_ "x" #KB2_ "_nt" #NT_ "_" TAG_, \
     reinterpret_cast<const void *>(&enum_q8_kernel<L_, KB1_, KB2_, NT_, WLDS_>)}
#define IBMC_VAR_LDS(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, "lds")
#define IBMC_VAR_L2(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, "l2")

}  // namespace ibmc
