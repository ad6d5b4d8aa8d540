// The enumeration kernel template (instantiated in enum_q8_*.hip).
#pragma once

#include "kernels_q8.h"
#include "enum_common.h"

namespace ibmc {

// ---- register-level helpers (gfx950) -------------------------------------

typedef short short2_t __attribute__((ext_vector_type(2)));

// Requantise four accumulators: t = clamp(acc >> s, lo, hi), packed as the
// four low bytes.  With (lo, hi) = (-64, 63) and acc = u - 64 * 2^s this is
// the offset activation a - 64 of a = clamp(floor(u / 2^s), 0, 127); with
// (lo, hi) = (0, 127) and acc = u it is a itself.  (Plain code on purpose:
// the compiler then sees every register dependence, including the wait
// states that reading MFMA results requires.)
__device__ __forceinline__ int requant4_clamp(v4i acc, int s, int lo, int hi) {
    int t[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) t[z] = min(max(acc[z] >> s, lo), hi);
    const unsigned l2 = __builtin_amdgcn_perm((unsigned)t[1], (unsigned)t[0], 0x0c0c0400u);
    const unsigned h2 = __builtin_amdgcn_perm((unsigned)t[3], (unsigned)t[2], 0x04000c0cu);
    return (int)(l2 | h2);
}

__device__ __forceinline__ int requant4_offset(v4i acc, int s) { return requant4_clamp(acc, s, -64, 63); }

// Fast hidden epilogue: the accumulator is alpha * u with alpha * 2^s = 256,
// so a = clamp(floor(u / 2^s), 0, 127) is byte 1 of clamp(acc, 0, 32767):
// one med3 per value and no shift.
__device__ __forceinline__ int requant4_byte1(v4i acc) {
    int m[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) m[z] = min(max(acc[z], 0), 32767);
    const unsigned l2 = __builtin_amdgcn_perm((unsigned)m[1], (unsigned)m[0], 0x0c0c0501u);
    const unsigned h2 = __builtin_amdgcn_perm((unsigned)m[3], (unsigned)m[2], 0x05010c0cu);
    return (int)(l2 | h2);
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
                                           int (&vb)[KB1][8], int lane, int ulo, int uhi) {
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
                const int xv = wave_uniform((int)gld(c.img + pp[j]));
                ee[j] = clamp_pixel(xv + wave_uniform((int)gld(c.dl + c.dg[j]))) - xv;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) { pp[j] = 0; ee[j] = 0; }
        if (c.mode == SEG_SHELL) {
            np = 1;
            const int head = wave_uniform(P.jobs[c.job].order[c.shell]);
            pp[0] = head / c.m;
            const int xv = wave_uniform((int)gld(c.img + pp[0]));
            ee[0] = clamp_pixel(xv + wave_uniform((int)gld(c.dl + head - pp[0] * c.m))) - xv;
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
                    // u is first clamped to [ulo, uhi], outside of which the
                    // product clamps to the same bound, so that f u fits in 32 bits
                    const int w = min(max(uu[z], ulo), uhi) * f - 16384;
                    h[z] = min(max(w, P.vb_lo), P.vb_hi);
                }
                vb[kb][2 * t4] = (h[0] & 0xffff) | (h[1] << 16);
                vb[kb][2 * t4 + 1] = (h[2] & 0xffff) | (h[3] << 16);
            }
        }
    }
}

// Lowest-index maximum over one 16-row tile of logits (this lane's four
// rows, classes 16 mt + 4 g + t), combined into (value, index, count).
// CHECK: skip classes >= ncls (else their logits are INT32_MIN, below any
// real logit, which the int32 headroom check keeps above INT32_MIN).
template <bool CHECK>
__device__ __forceinline__ void argmax_tile(v4i acc, int mt, int g, int ncls, int &bv, int &bi, int &bc) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int cls = mt * 16 + g * 4 + t;
        const int v = acc[t];
        if (!CHECK || cls < ncls) {
            if (v > bv) { bv = v; bi = cls; bc = 1; }
            else if (v == bv) { bc += 1; bi = min(bi, cls); }
        }
    }
}

// Combine the four lane groups holding the same point.
__device__ __forceinline__ void argmax_combine(int &bv, int &bi, int &bc) {
#pragma unroll
    for (int sh = 16; sh <= 32; sh <<= 1) {
        const int ov = __shfl_xor(bv, sh);
        const int oi = __shfl_xor(bi, sh);
        const int oc = __shfl_xor(bc, sh);
        if (ov > bv) { bv = ov; bi = oi; bc = oc; }
        else if (ov == bv) { bi = min(bi, oi); bc += oc; }
    }
}

// Record the violations of one 16-point tile (lanes of group 0 carry the
// points): one atomic per wave reserves the slots, lanes write their record.
__device__ __forceinline__ void emit_tile(const EnumParams &P, const Cursor &c, bool viol, int p, int i, int label,
                                          int lane) {
    const unsigned long long vm = __ballot(viol);
    if (!vm) return;
    unsigned long long start = 0;
    if (lane == 0) {
        start = atomicAdd(P.rec_count, (unsigned long long)__popcll(vm));
        atomicAdd(P.slot_cex + c.slot, (unsigned long long)__popcll(vm));
        atomicMin(P.first_chunk, (unsigned long long)c.chunk);
        if (P.hit_host) *P.hit_host = 1;
        if (P.stop_on_first) *P.stop_flag = 1;
    }
    start = wave_uniform(start);  // lane 0's value
    // The rank arithmetic runs for tiles with counterexamples only: passing
    // the level's shape through an empty asm keeps the compiler from hoisting
    // its many uniform conditions into the common path.
    Cursor cl = c;
    cl.k = wave_uniform(c.k);
    cl.n = wave_uniform(c.n);
    cl.m = wave_uniform(c.m);
    cl.mode = wave_uniform(c.mode);
    asm volatile("" : "+s"(cl.k), "+s"(cl.n), "+s"(cl.m), "+s"(cl.mode));
    if (viol) {
        const unsigned long long below = vm & ((1ull << lane) - 1ull);
        const int64_t idx = (int64_t)start + __popcll(below);
        if (idx < P.rec_cap) {
            CexRec r;
            r.prop = c.prop;
            r.k = c.k;
            r.rank = point_rank(cl, P, p, i);
            r.label = label;
            r.reserved = 0;
            P.recs[idx] = r;
        }
    }
}

__device__ __forceinline__ unsigned fold_groups(unsigned long long m) {
    return (unsigned)((m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xffffull);
}

// Loads of one chunk's first layer, issued together before any is used:
// each tile's pixel, delta and weight column slice (packed path: 16 int16 of
// f W1 per K-block in two 16-byte halves; int32 path: 16 int8 of W1, the
// second half then repeats the first).  The path is a uniform select, so that
// no branch separates the loads from each other.
template <int KB1, int NT>
__device__ __forceinline__ void layer1_loads(const Cursor &c, const QNetDev &net, bool packed, const int (&plast)[NT],
                                             const int (&ilast)[NT], int g, int (&ev)[NT], v4i (&wa)[NT][KB1],
                                             v4i (&wb)[NT][KB1]) {
    constexpr int H1 = KB1 * 64;
    const int kstride = packed ? 128 : 64;  // bytes per K-block of a column
    const int boff = packed ? 16 : 0;
    int xv[NT], dv[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        xv[nt] = gld(c.img + plast[nt]);
        dv[nt] = gld(c.dl + ilast[nt]);
        const char *wp = packed ? reinterpret_cast<const char *>(net.W1T16 + plast[nt] * H1 + g * 16)
                                : reinterpret_cast<const char *>(net.W1T + plast[nt] * H1 + g * 16);
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            wa[nt][kb] = gld(reinterpret_cast<const v4i *>(wp + kb * kstride));
            wb[nt][kb] = gld(reinterpret_cast<const v4i *>(wp + kb * kstride + boff));
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) ev[nt] = clamp_pixel(xv[nt] + dv[nt]) - xv[nt];
}

// First layer, packed int16 path: u = base + e W1[:, p] as v = f u - 16384
// in 16-bit halves, clamped to [-16384, 16383], whose byte 1 is a - 64.
template <int KB1, int NT>
__device__ __forceinline__ void layer1_packed(const int (&ev)[NT], const v4i (&wa)[NT][KB1], const v4i (&wb)[NT][KB1],
                                              const int (&vb)[KB1][8], v4i (&a1)[NT][KB1]) {
    const short2_t vlo = {(short)-16384, (short)-16384};
    const short2_t vhi = {(short)16383, (short)16383};
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const short2_t e2 = {(short)ev[nt], (short)ev[nt]};
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            const int wv[8] = {wa[nt][kb][0], wa[nt][kb][1], wa[nt][kb][2], wa[nt][kb][3],
                               wb[nt][kb][0], wb[nt][kb][1], wb[nt][kb][2], wb[nt][kb][3]};
            int pr2[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                short2_t u = as_s2(vb[kb][t]) + e2 * as_s2(wv[t]);
                u = __builtin_elementwise_max(u, vlo);
                u = __builtin_elementwise_min(u, vhi);
                pr2[t] = as_int(u);
            }
            a1[nt][kb] = v4i{(int)__builtin_amdgcn_perm(pr2[1], pr2[0], 0x07050301u),
                             (int)__builtin_amdgcn_perm(pr2[3], pr2[2], 0x07050301u),
                             (int)__builtin_amdgcn_perm(pr2[5], pr2[4], 0x07050301u),
                             (int)__builtin_amdgcn_perm(pr2[7], pr2[6], 0x07050301u)};
        }
    }
}

// First layer, int32 path: u - 64 * 2^s from the wave's LDS base plus
// e W1[:, p], requantised to a - 64.
template <int KB1, int NT>
__device__ __forceinline__ void layer1_int32(const int (&ev)[NT], const v4i (&wa)[NT][KB1], const v4i (&wb)[NT][KB1],
                                             const int32_t *base32, int s1, int g, v4i (&a1)[NT][KB1]) {
    // wb repeats wa on this path; consuming it here keeps its loads beside
    // the others instead of being sunk into the packed path
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) asm volatile("" ::"v"(wb[nt][kb]));
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int e = ev[nt];
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            const int4 *bp = reinterpret_cast<const int4 *>(base32 + kb * 64 + g * 16);
            int out[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int4 bv = bp[t];
                const int w = wa[nt][kb][t];
                v4i u = {bv.x + e * (int)(int8_t)(w & 0xff), bv.y + e * (int)(int8_t)((w >> 8) & 0xff),
                         bv.z + e * (int)(int8_t)((w >> 16) & 0xff), bv.w + e * (int)(int8_t)(w >> 24)};
                out[t] = requant4_offset(u, s1);
            }
            a1[nt][kb] = v4i{out[0], out[1], out[2], out[3]};
        }
    }
}

// The enumeration kernel.  L: weight layers (2 or 3); KB1 / KB2: 64-wide
// K-blocks of the first / second hidden layer; NT: 16-point N-tiles per
// chunk; WLDS: weight tiles of layers >= 2 staged in LDS (else read from
// global memory through the L2); EPI (3-layer nets): 1 for the fast hidden
// epilogue (shift[1] in {7, 8}), 0 for the general one; OUT16: at most 16
// classes (the output layer is one M-tile whose weights stay in registers,
// the second hidden layer streams into it, and decisions are taken from
// ballots against the clean label's logit; else the output layer loops over
// its M-tiles and every point takes the full argmax).
//
// Activations travel between layers in the offset form a - 64 (int8 in
// [-64, 63]); the offsets are folded into the next layer's bias (bo).
template <int L, int KB1, int KB2, int NT, bool WLDS, int EPI, bool OUT16>
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
    // fast hidden epilogue (3-layer nets, shift[1] in {7, 8}): layer 1 emits
    // fast2 * (a1 - 64) (doubled bytes when fast2 == 2), layer 2 emits plain a2
    constexpr bool fast = (L == 3) && EPI == 1;
    const bool dbl1 = fast && net.fast2 == 2;
    // LDS: [weight tiles of layers >= 2 (WLDS)] [layer-2 init] [output init] [per-wave base]
    const int64_t wbytes = WLDS ? (w2_bytes + wl_bytes) : 0;
    const int nb2 = (L == 3) ? H2 : 0;
    const int nbl = net.H[L];
    {
        if constexpr (WLDS) {
            int4 *dst = reinterpret_cast<int4 *>(smem);
            const int64_t n2 = w2_bytes / 16, nl = wl_bytes / 16;
            for (int64_t t = threadIdx.x; t < n2; t += blockDim.x)
                dst[t] = reinterpret_cast<const int4 *>(net.Wt[2])[t];
            for (int64_t t = threadIdx.x; t < nl; t += blockDim.x)
                dst[n2 + t] = reinterpret_cast<const int4 *>(net.Wt[L])[t];
            w2s = reinterpret_cast<const int8_t *>(smem);
            wls = reinterpret_cast<const int8_t *>(smem) + w2_bytes;
        }
        int32_t *bdst = reinterpret_cast<int32_t *>(smem + wbytes);
        if constexpr (L == 3) {
            const int32_t *src2 = fast ? net.bf2 : net.bo[2];
            for (int t = threadIdx.x; t < nb2; t += blockDim.x) bdst[t] = src2[t];
        }
        const int32_t *srcl = fast ? net.bn[L] : net.bo[L];
        for (int t = threadIdx.x; t < nbl; t += blockDim.x) bdst[nb2 + t] = srcl[t];
        __syncthreads();
    }
    const int32_t *b2s = reinterpret_cast<const int32_t *>(smem + wbytes);
    const int32_t *bls = b2s + nb2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j16 = lane & 15, g = lane >> 4;
    int32_t *base32 = reinterpret_cast<int32_t *>(smem + wbytes) + nb2 + nbl + wave * H1;

    // output layer of at most 16 classes: weights and init held in registers
    v4i Wo[OUT16 ? KBL : 1];
    v4i bo4 = v4i{0, 0, 0, 0};
    if constexpr (OUT16) {
#pragma unroll
        for (int kb = 0; kb < KBL; ++kb) Wo[kb] = reinterpret_cast<const v4i *>(wls)[kb * 64 + lane];
        const int4 b = *reinterpret_cast<const int4 *>(bls + g * 4);
        bo4 = v4i{b.x, b.y, b.z, b.w};
        // padding classes start (and, with zero weights, stay) at INT32_MIN
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (g * 4 + t >= net.dims[L]) bo4[t] = INT32_MIN;
    }

    Cursor c;
    c.job = -1;
    bool have = false;
    int64_t cur_chunk = 0, end_chunk = 0;
    int fetches = 0;
    const int s1 = net.shift[0];
    const int s2 = (L == 3) ? net.shift[1] : 0;
    const int ncls = net.dims[L];
    // general epilogue of layer 2: a2 - 64 = clamp(acc >> s2, -64, 63); the
    // bounds live in VGPRs so that the clamp is a single med3
    int lo2 = -64, hi2 = 63;
    asm("" : "+v"(lo2));
    asm("" : "+v"(hi2));
    // 32-bit pre-clamp of first-layer potentials for the packed base
    int ulo = 0, uhi = 0;
    if (P.packed) {
        const int f = net.f1;
        const int a0 = P.vb_lo + 16384, a1v = P.vb_hi + 16384;
        ulo = a0 >= 0 ? a0 / f : -((-a0 + f - 1) / f);   // floor(a0 / f)
        uhi = a1v >= 0 ? (a1v + f - 1) / f : -((-a1v) / f);  // ceil(a1v / f)
    }
    int vb[KB1][8];
    // clean label of the current property and, per lane (OUT16), bit t set
    // when this lane's class 4 g + t has a lower index than the label
    int label0 = -1, cur_prop = -1;
    int lowbits = 0;

    while (true) {
        if (cur_chunk >= end_chunk) {
            unsigned long long start = 0;
            if (lane == 0) start = atomicAdd(P.queue, (unsigned long long)P.batch);
            start = wave_uniform(start);  // lane 0's value
            if ((int64_t)start >= P.total_chunks) break;
            if (wave_uniform(*P.stop_flag)) break;
            // host-mapped: poll sparsely
            if (P.abort_host && (fetches++ & 15) == 0 && wave_uniform(*P.abort_host)) break;
            cur_chunk = (int64_t)start;
            end_chunk = min((int64_t)start + P.batch, P.total_chunks);
            cursor_decode<CH, EnumParams>(c, P, cur_chunk);
            have = false;
        }
        if (!have) {
            const int32_t *u0s = u0_store + (int64_t)wave_uniform(u0_index[c.prop]) * u0_stride;
            build_base<KB1>(c, P, u0s, base32, vb, lane, ulo, uhi);
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS writes done
            __builtin_amdgcn_wave_barrier();
            have = true;
        }
        if (c.prop != cur_prop) {
            cur_prop = c.prop;
            label0 = wave_uniform(P.props[c.prop].label0);
            lowbits = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) lowbits |= (4 * g + t < label0 ? 1 : 0) << t;
        }

        // ---- positions of the chunk's points: last element (p, i)
        bool valid[NT];
        int plast[NT], ilast[NT];
        const int obase = (int)c.ch * CH;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            valid[nt] = last_element32(c, P, obase + nt * 16 + j16, plast[nt], ilast[nt]);

        // ---- layer 1: incremental update, requantisation, B operands.  All
        // loads of the chunk (pixel, delta, weight column) are issued before
        // any of them is used.
        int ev[NT];
        v4i wa[NT][KB1], wb[NT][KB1];
        layer1_loads<KB1, NT>(c, net, P.packed != 0, plast, ilast, g, ev, wa, wb);
        v4i a1[NT][KB1];
        if (P.packed)
            layer1_packed<KB1, NT>(ev, wa, wb, vb, a1);
        else
            layer1_int32<KB1, NT>(ev, wa, wb, base32, s1, g, a1);
        if constexpr (L == 3) {
            if (dbl1) {  // uniform: one branch per chunk
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
                        for (int z = 0; z < 4; ++z) a1[nt][kb][z] = double_bytes(a1[nt][kb][z]);
            }
        }

        // ---- hidden layer 2 (L == 3): int8 MFMA, requantise into B operands;
        // with OUT16 every completed 64-row block of a2 goes straight into the
        // output layer's accumulators
        v4i acco[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acco[nt] = bo4;
        v4i a2[NT][(L == 3 && !OUT16) ? KB2 : 1];
        if constexpr (L == 3) {
            // Software pipeline over the M-tiles: the weight tiles and init of
            // tile mt + 1 are read from LDS while tile mt computes, and the
            // requantisation of tile mt - 1 (VALU) is interleaved with the MFMAs
            // of tile mt, so that the two pipes overlap within one wave.
            const v4i *wt2 = reinterpret_cast<const v4i *>(w2s) + lane;
            v4i Acur[KB1], Anext[KB1];
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) Acur[kb] = wt2[kb * 64];
            const int4 *bias2 = reinterpret_cast<const int4 *>(b2s + g * 4);
            int4 bias = bias2[0], bnext = bias;
            v4i accp[NT];
            v4i blk[NT];  // the a2 block being filled (OUT16)
#pragma unroll
            for (int mt = 0; mt <= MT2; ++mt) {
                if (mt + 1 < MT2) {
#pragma unroll
                    for (int kb = 0; kb < KB1; ++kb) Anext[kb] = wt2[((mt + 1) * KB1 + kb) * 64];
                    bnext = bias2[(mt + 1) * 4];
                }
                v4i acc[NT];
                if (mt < MT2) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
#pragma unroll
                    for (int kb = 0; kb < KB1; ++kb) {
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Acur[kb], a1[nt][kb], acc[nt], 0, 0, 0);
                    }
                }
                if (mt > 0) {
                    const int pm = mt - 1;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        int q = fast ? requant4_byte1(accp[nt]) : requant4_clamp(accp[nt], s2, lo2, hi2);
                        // pin the epilogue here: otherwise it is sunk towards the
                        // output layer, keeping every raw accumulator live
                        asm volatile("" : "+v"(q));
                        if constexpr (OUT16) blk[nt][pm & 3] = q;
                        else a2[nt][pm >> 2][pm & 3] = q;
                    }
                    if constexpr (OUT16) {
                        if ((pm & 3) == 3) {
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt)
                                acco[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Wo[pm >> 2], blk[nt], acco[nt], 0, 0, 0);
                        }
                    }
                    if (mt < MT2) {
                        // the next tile's LDS reads first, then one MFMA and a share of
                        // the epilogue's VALU work, and so on
                        __builtin_amdgcn_sched_group_barrier(0x100, KB1 + 1, 0);
#pragma unroll
                        for (int i = 0; i < KB1 * NT; ++i) {
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x002, ((fast ? 7 : 11) * NT + KB1 * NT - 1) / (KB1 * NT), 0);
                        }
                    }
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) accp[nt] = acc[nt];
#pragma unroll
                for (int kb = 0; kb < KB1; ++kb) Acur[kb] = Anext[kb];
                bias = bnext;
                __builtin_amdgcn_sched_barrier(0);
            }
        } else if constexpr (OUT16) {
#pragma unroll
            for (int kb = 0; kb < KBL; ++kb)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acco[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Wo[kb], a1[nt][kb], acco[nt], 0, 0, 0);
        }

        if constexpr (OUT16) {
            // ---- decisions from ballots against the clean label's logit zL:
            // a point is a counterexample iff some class c has z_c > zL, or
            // z_c == zL with c < label (padding classes sit at INT32_MIN); it is
            // an exact tie iff another class reaches zL.  Tiles with
            // counterexamples take the full argmax.
            const int tL = label0 & 3;
            const unsigned long long rowL = 0xffffull << (16 * (label0 >> 2));
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const v4i z = acco[nt];
                const int zs = tL == 0 ? z[0] : tL == 1 ? z[1] : tL == 2 ? z[2] : z[3];
                const int zL = __shfl(zs, j16 + 16 * (label0 >> 2));
                unsigned long long beat = 0, eqm = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    // z_c beats zL iff z_c > zL - [c < label]
                    beat |= __ballot(z[t] > zL - ((lowbits >> t) & 1));
                    const unsigned long long eq = __ballot(z[t] == zL);
                    eqm |= (t == tL) ? (eq & ~rowL) : eq;
                }
                const unsigned vmask = (unsigned)(__ballot(valid[nt]) & 0xffffull);
                const unsigned viol16 = fold_groups(beat) & vmask;
                const unsigned tie16 = fold_groups(eqm) & vmask & ~viol16;
                unsigned ties = __popc(tie16);
                if (viol16) {
                    int bv = INT32_MIN, bi = 0x7fffffff, bc = 0;
                    argmax_tile<false>(z, 0, g, ncls, bv, bi, bc);
                    argmax_combine(bv, bi, bc);
                    const bool mine = g == 0 && ((viol16 >> j16) & 1u);
                    ties += (unsigned)__popcll(__ballot(mine && bc > 1));
                    emit_tile(P, c, mine, plast[nt], ilast[nt], bi, lane);
                }
                if (ties && lane == 0) atomicAdd(P.slot_ties + c.slot, (unsigned long long)ties);
            }
        } else {
            // ---- general output layer: M-tiles in turn, full lowest-index argmax
            int bestv[NT], besti[NT], bestc[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) { bestv[nt] = INT32_MIN; besti[nt] = 0x7fffffff; bestc[nt] = 0; }
            for (int mt = 0; mt < MTL; ++mt) {
                const int4 bias = *reinterpret_cast<const int4 *>(bls + mt * 16 + g * 4);
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
                for (int nt = 0; nt < NT; ++nt) argmax_tile<true>(acc[nt], mt, g, ncls, bestv[nt], besti[nt], bestc[nt]);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                argmax_combine(bestv[nt], besti[nt], bestc[nt]);
                const bool mine = valid[nt] && g == 0;
                const unsigned long long tm = __ballot(mine && bestc[nt] > 1);
                if (tm && lane == 0) atomicAdd(P.slot_ties + c.slot, (unsigned long long)__popcll(tm));
                emit_tile(P, c, mine && besti[nt] != label0, plast[nt], ilast[nt], besti[nt], lane);
            }
        }

        // ---- advance
        cur_chunk++;
        if (cur_chunk < end_chunk) {
            if (cursor_next<CH, EnumParams>(c, P)) have = false;
        }
    }
}

#define IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, WLDS_, EPI_, O16_, TAG_)                                      \
    {L_, KB1_, KB2_, NT_, WLDS_, EPI_, O16_, 16 * NT_, "q8_L" #L_ "_kb" #KB1_ "x" #KB2_ "_nt" #NT_ "_" TAG_, \
     reinterpret_cast<const void *>(&enum_q8_kernel<L_, KB1_, KB2_, NT_, WLDS_, EPI_, O16_>)}
// instances for at most 16 classes
#define IBMC_VAR_LDS(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, 0, true, "lds")
#define IBMC_VAR_L2(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, 0, true, "l2")
#define IBMC_VAR_LDS_F(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, 1, true, "lds_f")
#define IBMC_VAR_L2_F(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, 1, true, "l2_f")
// instances for any number of classes
#define IBMC_VAR_LDS_G(L_, KB1_, KB2_, NT_, EPI_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, EPI_, false, "lds_g" #EPI_)
#define IBMC_VAR_L2_G(L_, KB1_, KB2_, NT_, EPI_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, EPI_, false, "l2_g" #EPI_)

}  // namespace ibmc
