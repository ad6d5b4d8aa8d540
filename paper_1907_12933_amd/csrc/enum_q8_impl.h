// The enumeration kernel template (instantiated in enum_q8_*.hip).
#pragma once

#include "kernels_q8.h"
#include "enum_common.h"

namespace ibmc {

// ---- register-level helpers (gfx950) -------------------------------------

typedef short short2_t __attribute__((ext_vector_type(2)));

// Requantise four accumulators holding u - 64 * 2^s into the packed offset
// activations a - 64 (a = clamp(floor(u / 2^s), 0, 127)): arithmetic shift,
// clamp to [-64, 63], and a byte permute that packs the four low bytes.
// (Plain code on purpose: the compiler then sees every register dependence,
// including the wait states that reading MFMA results requires.)
__device__ __forceinline__ int requant4_offset(v4i acc, int s) {
    int t[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) t[z] = min(max(acc[z] >> s, -64), 63);
    const unsigned lo = __builtin_amdgcn_perm((unsigned)t[1], (unsigned)t[0], 0x0c0c0400u);
    const unsigned hi = __builtin_amdgcn_perm((unsigned)t[3], (unsigned)t[2], 0x04000c0cu);
    return (int)(lo | hi);
}

// Fast hidden epilogue: the accumulator is alpha * u with alpha * 2^s = 256,
// so a = clamp(floor(u / 2^s), 0, 127) is byte 1 of clamp(acc, 0, 32767).
__device__ __forceinline__ int requant4_byte1(v4i acc) {
    int m[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) m[z] = min(max(acc[z], 0), 32767);
    const unsigned lo = __builtin_amdgcn_perm((unsigned)m[1], (unsigned)m[0], 0x0c0c0501u);
    const unsigned hi = __builtin_amdgcn_perm((unsigned)m[3], (unsigned)m[2], 0x05010c0cu);
    return (int)(lo | hi);
}

// a - 64 bytes -> 2 (a - 64) bytes (still int8: [-128, 126]); the bit that
// crosses into the next byte is masked off.
__device__ __forceinline__ int double_bytes(int d) { return (int)(((unsigned)d << 1) & 0xfefefefeu); }

__device__ __forceinline__ int as_int(short2_t v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ short2_t as_s2(int v) { return __builtin_bit_cast(short2_t, v); }

// Base of the current segment: clean first-layer potentials plus the
// prefix's column updates e * W1[:, p].  Every lane computes the values of
// its lane group g for all K-blocks (positions 64 kb + 16 g + b): as packed
// int16 in the scaled window form v = f*u - 16384 (clamped so that adding
// any last-element update cannot overflow) for the packed path, and as
// int32 u - 64 * 2^s into the wave's LDS slice for the general path.
template <int KB1>
__device__ __forceinline__ void build_base(const Cursor &c, const EnumParams &P, const int32_t *u0s, int32_t *base32,
                                           int (&vb)[KB1][8], int lane) {
    const PropDev &pr = P.props[c.prop];
    const int H1 = KB1 * 64;
    const int g = lane >> 4;
    int pp[kMaxK], ee[kMaxK];
    int np = 0;
    if (c.mode == SEG_PLAIN) {
        np = c.k - 1;
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) {
            pp[j] = 0;
            ee[j] = 0;
            if (j < np) {
                pp[j] = c.pre[j];
                const int xv = pr.image[pp[j]];
                ee[j] = clamp_pixel(xv + pr.deltas[c.dg[j]]) - xv;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) { pp[j] = 0; ee[j] = 0; }
        if (c.mode == SEG_SHELL) {
            np = 1;
            const int head = P.jobs[c.job].order[c.shell];
            pp[0] = head / c.m;
            const int xv = pr.image[pp[0]];
            ee[0] = clamp_pixel(xv + pr.deltas[head - pp[0] * c.m]) - xv;
        }
    }
    // u = u0 + sum_j e_j W1[:, p_j] at positions lane + 64 r (coalesced)
    const int off = 64 << P.net.shift[0];
#pragma unroll
    for (int r = 0; r < KB1; ++r) {
        const int q = lane + 64 * r;
        int v = u0s[q];
        for (int j = 0; j < np; ++j) v += ee[j] * (int)P.net.W1T[(int64_t)pp[j] * H1 + q];
        base32[q] = P.packed ? v : v - off;
    }
    if (P.packed) {
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        __builtin_amdgcn_wave_barrier();
        // this lane group's positions 64 kb + 16 g + b as packed int16 v = f u - 16384,
        // clamped so that adding any last-element update cannot overflow
        const int f = P.net.f1;
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            const int4 *src = reinterpret_cast<const int4 *>(base32 + kb * 64 + g * 16);
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                const int4 u = src[t4];
                const int uu[4] = {u.x, u.y, u.z, u.w};
                int h[4];
#pragma unroll
                for (int z = 0; z < 4; ++z) {
                    const int64_t w = (int64_t)uu[z] * f - 16384;
                    h[z] = (int)(w < P.vb_lo ? P.vb_lo : (w > P.vb_hi ? P.vb_hi : w));
                }
                vb[kb][2 * t4] = (h[0] & 0xffff) | (h[1] << 16);
                vb[kb][2 * t4 + 1] = (h[2] & 0xffff) | (h[3] << 16);
            }
        }
    }
}

// The enumeration kernel.  L: weight layers (2 or 3); KB1 / KB2: 64-wide
// K-blocks of the first / second hidden layer; NT: 16-point N-tiles per
// chunk; WLDS: weight tiles of layers >= 2 staged in LDS (else read from
// global memory through the L2).
//
// Activations travel between layers in the offset form a - 64 (int8 in
// [-64, 63]); the offsets are folded into the next layer's bias (bo).
template <int L, int KB1, int KB2, int NT, bool WLDS>
__global__ void __launch_bounds__(256, 2) enum_q8_kernel(EnumParams P, const int32_t *u0_store,
                                                      int64_t u0_stride, const int32_t *u0_index) {
    constexpr int CH = 16 * NT;
    constexpr int H1 = KB1 * 64;
    constexpr int H2 = KB2 * 64;
    constexpr int MT2 = (L == 3) ? H2 / 16 : 0;
    constexpr int KBL = (L == 3) ? KB2 : KB1;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const QNetDev &net = P.net;
    const int MTL = net.H[L] / 16;
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
    int32_t *base32 = reinterpret_cast<int32_t *>(smem + wbytes) + wave * H1;

    Cursor c;
    c.job = -1;
    bool have = false;
    int64_t cur_chunk = 0, end_chunk = 0;
    int fetches = 0;
    const int s1 = net.shift[0];
    const int s2 = (L == 3) ? net.shift[1] : 0;
    const int ncls = net.dims[L];
    // fast hidden epilogue (3-layer nets, shift[1] in {7, 8}): layer 1 emits
    // fast2 * (a1 - 64) (doubled bytes when fast2 == 2), layer 2 emits plain a2
    const bool fast = (L == 3) && net.fast2 != 0;
    const bool dbl1 = fast && net.fast2 == 2;
    const short2_t vlo = {(short)-16384, (short)-16384};
    const short2_t vhi = {(short)16383, (short)16383};
    int vb[KB1][8];

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
            build_base<KB1>(c, P, u0s, base32, vb, lane);
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS writes done
            __builtin_amdgcn_wave_barrier();
            have = true;
        }
        const PropDev &pr = P.props[c.prop];
        const int label0 = pr.label0;

        // ---- layer 1: incremental update, requantisation, B operands
        v4i a1[NT][KB1];
        bool valid[NT];
        int plast[NT], ilast[NT];
        const int obase = (int)c.ch * CH;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int o = obase + nt * 16 + j16;
            int p = 0, i = 0;
            valid[nt] = last_element32(c, P, o, p, i);
            if (!valid[nt]) { p = 0; i = 0; }
            plast[nt] = p;
            ilast[nt] = i;
            const int xv = pr.image[p];
            const int e = clamp_pixel(xv + pr.deltas[i]) - xv;
            if (P.packed) {
                const int16_t *wcol = net.W1T16 + (int64_t)p * H1 + g * 16;
                const short2_t e2 = {(short)e, (short)e};
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb) {
                    const int4 wa = *reinterpret_cast<const int4 *>(wcol + kb * 64);
                    const int4 wb = *reinterpret_cast<const int4 *>(wcol + kb * 64 + 8);
                    const int wv[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
                    int pr2[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        short2_t u = as_s2(vb[kb][t]) + e2 * as_s2(wv[t]);
                        u = __builtin_elementwise_max(u, vlo);
                        u = __builtin_elementwise_min(u, vhi);
                        pr2[t] = as_int(u);
                    }
                    // byte 1 of each 16-bit value is a - 64
                    v4i o = {(int)__builtin_amdgcn_perm(pr2[1], pr2[0], 0x07050301u),
                             (int)__builtin_amdgcn_perm(pr2[3], pr2[2], 0x07050301u),
                             (int)__builtin_amdgcn_perm(pr2[5], pr2[4], 0x07050301u),
                             (int)__builtin_amdgcn_perm(pr2[7], pr2[6], 0x07050301u)};
                    if (L == 3 && dbl1)
                        o = v4i{double_bytes(o[0]), double_bytes(o[1]), double_bytes(o[2]), double_bytes(o[3])};
                    a1[nt][kb] = o;
                }
            } else {
                const int8_t *wcol = net.W1T + (int64_t)p * H1 + g * 16;
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb) {
                    const int4 wv = *reinterpret_cast<const int4 *>(wcol + kb * 64);
                    const int4 *bp = reinterpret_cast<const int4 *>(base32 + kb * 64 + g * 16);
                    const int wd[4] = {wv.x, wv.y, wv.z, wv.w};
                    int out[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int4 bv = bp[t];
                        const int w = wd[t];
                        v4i u = {bv.x + e * (int)(int8_t)(w & 0xff), bv.y + e * (int)(int8_t)((w >> 8) & 0xff),
                                 bv.z + e * (int)(int8_t)((w >> 16) & 0xff), bv.w + e * (int)(int8_t)(w >> 24)};
                        out[t] = requant4_offset(u, s1);
                    }
                    if (L == 3 && dbl1)
                        a1[nt][kb] = v4i{double_bytes(out[0]), double_bytes(out[1]), double_bytes(out[2]),
                                         double_bytes(out[3])};
                    else
                        a1[nt][kb] = v4i{out[0], out[1], out[2], out[3]};
                }
            }
        }

        // ---- hidden layer 2 (L == 3): int8 MFMA, requantise into B operands
        v4i a2[NT][(L == 3) ? KB2 : 1];
        if constexpr (L == 3) {
            // weight tiles of M-tile mt + 1 are loaded while mt computes
            const v4i *wt2 = reinterpret_cast<const v4i *>(w2s) + lane;
            v4i Acur[KB1], Anext[KB1];
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) Acur[kb] = wt2[kb * 64];
            const int4 *bias2 = reinterpret_cast<const int4 *>((fast ? net.bf2 : net.bo[2]) + g * 4);
#pragma unroll
            for (int mt = 0; mt < MT2; ++mt) {
                if (mt + 1 < MT2) {
#pragma unroll
                    for (int kb = 0; kb < KB1; ++kb) Anext[kb] = wt2[((mt + 1) * KB1 + kb) * 64];
                }
                const int4 bias = bias2[mt * 4];
                v4i acc[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Acur[kb], a1[nt][kb], acc[nt], 0, 0, 0);
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    a2[nt][mt >> 2][mt & 3] = fast ? requant4_byte1(acc[nt]) : requant4_offset(acc[nt], s2);
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb) Acur[kb] = Anext[kb];
                __builtin_amdgcn_sched_barrier(0);
            }
        }

        // ---- output layer: int8 MFMA, lowest-index argmax
        int bestv[NT], besti[NT], bestc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) { bestv[nt] = INT32_MIN; besti[nt] = 0x7fffffff; bestc[nt] = 0; }
        for (int mt = 0; mt < MTL; ++mt) {
            const int4 bias = *reinterpret_cast<const int4 *>(((L == 3 && fast) ? net.bn[L] : net.bo[L]) + mt * 16 + g * 4);
            v4i acc[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
#pragma unroll
            for (int kb = 0; kb < KBL; ++kb) {
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
