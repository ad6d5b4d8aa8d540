// Device code of the float (sigmoid variant) enumeration, shared by the
// kernel instances: the per-point forward pass with the incremental first
// layer (Sec. II-A, Eqs. (1)-(2)), the decision against the clean label
// (Sec. III-C) with near ties flagged, and wave-aggregated records.
//
// Both kernel families evaluate a point in one fixed sequence of FP32
// operations, which the eval kernels repeat exactly for listed points:
//   v_j = u0_j; v_j = fma(e_t, W1[p_t][j], v_j) for the prefix pixels in
//   ascending order, then for the last pixel; a_j = sigmoid(v_j);
//   every later layer: total = bias; per block of kF32SumBlock inputs a
//   partial sum accumulated from zero by fma in input order, added to the
//   total; hidden layers apply the sigmoid, the last layer gives the logits.
// e_t = (clamp(x[p_t] + d_t, 0, 255) - x[p_t]) / 256 is exact in FP32.
#pragma once

#include "enum_common.h"
#include "kernels_f32.h"

namespace ibmc {

// Load through the constant address space: a wave-uniform address becomes
// one scalar-cache load for the whole wave (weights, biases and the clean
// potentials are read-only while the kernels run).
template <class T>
__device__ __forceinline__ T cld(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// A pointer the compiler may not treat as loop-invariant: the weight loads
// behind it stay at their use instead of being hoisted out of the chunk loop
// into (spilled) scalar registers.
template <class T>
__device__ __forceinline__ const T *opaque(const T *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// 1 / (1 + e^-u) with the hardware base-2 exponential of -u log2(e) and the
// hardware reciprocal (each about 1 ulp); saturates to 0 and 1 for large |u|.
__device__ __forceinline__ float sigmoid_f32(float u) {
    const float e = __builtin_amdgcn_exp2f(-u * 1.4426950408889634f);
    return __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float eff_delta(int xv, int d) {
    return (float)(clamp_pixel(xv + d) - xv) * (1.0f / 256.0f);
}

// Lowest-index largest logit of the first nc, its value and the margin to the
// runner-up (infinite with one class).
template <int NCP>
__device__ __forceinline__ void decide_f32(const float (&z)[NCP], int nc, int &best, float &top, float &margin) {
    best = 0;
    top = z[0];
#pragma unroll
    for (int j = 1; j < NCP; ++j)
        if (j < nc && z[j] > top) { top = z[j]; best = j; }
    float second = -INFINITY;
#pragma unroll
    for (int j = 0; j < NCP; ++j)
        if (j < nc && j != best) second = fmaxf(second, z[j]);
    margin = top - second;
}

__device__ __forceinline__ unsigned lane_rank(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Counterexample and near-tie records of one wave's points: one atomic per
// wave and kind for the slots, one for the level counter; lanes write their
// own records at base + their rank among the set lanes.
__device__ __forceinline__ void emit_f32(const FEnumParams &P, const Cursor &c, bool viol, bool near, int p, int i,
                                         int best) {
    const int lane = __lane_id();
    const unsigned long long mv = __ballot(viol), mn = __ballot(near);
    if (mv) {
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(P.rec_count, (unsigned long long)__popcll(mv));
            atomicAdd(P.slot_cex + c.slot, (unsigned long long)__popcll(mv));
        }
        base = wave_uniform(base);
        if (viol) {
            const unsigned long long idx = base + lane_rank(mv);
            if ((int64_t)idx < P.rec_cap) {
                DevRec r;
                r.rank = point_rank<FEnumParams>(c, P, p, i);
                r.prop = c.prop;
                r.klab = (c.k << 24) | best;
                P.recs[idx] = r;
            }
        }
    }
    if (mn) {
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(P.tie_count, (unsigned long long)__popcll(mn));
            atomicAdd(P.slot_ties + c.slot, (unsigned long long)__popcll(mn));
        }
        base = wave_uniform(base);
        if (near) {
            const unsigned long long idx = base + lane_rank(mn);
            if ((int64_t)idx < P.tie_cap) {
                DevRec r;
                r.rank = point_rank<FEnumParams>(c, P, p, i);
                r.prop = c.prop;
                r.klab = (c.k << 24) | best;
                P.ties[idx] = r;
            }
        }
    }
}

// Next queue ticket of a persistent wave: the first chunk of a batch of
// P.batch, or -1 when the queue is drained or a stop / abort was requested.
__device__ __forceinline__ int64_t f32_ticket(const FEnumParams &P) {
    unsigned long long t = 0;
    int stop = 0;
    if (__lane_id() == 0) {
        t = atomicAdd(P.queue, (unsigned long long)P.batch);
        stop = *P.stop_flag || (P.abort_host && *P.abort_host);
    }
    const int64_t start = (int64_t)wave_uniform(t);
    if (wave_uniform(stop) || start >= P.total_chunks) return -1;
    return start;
}

// Decode point (k, rank) of a property: ascending pixels and delta indices.
__device__ __forceinline__ void decode_point_dev(int n, int m, int k, int64_t rank, int (&pix)[kMaxK],
                                                 int (&dig)[kMaxK]) {
    int64_t mk = 1;
    for (int j = 0; j < k; ++j) mk *= m;
    lex_unrank_subset_fixed(rank / mk, k, n, pix);
    int64_t d = rank % mk;
#pragma unroll
    for (int j = kMaxK - 1; j >= 0; --j) {
        dig[j] = 0;
        if (j < k) { dig[j] = (int)(d % m); d /= m; }
    }
}

// ---------------------------------------------------------------------------
// one point per lane
// ---------------------------------------------------------------------------

constexpr int kLaneWaves = 4;  // waves per workgroup of the lane kernels

// Logits of the lane's point.  u0: the property's clean first-layer
// potentials [H1]; np prefix elements (pixel pp[t], effective delta ee[t]),
// then the last pixel p with effective delta e.  a2w: this wave's LDS
// columns of the second hidden layer ([H2][64]); each lane touches only its
// own column.
template <int H1, int H2, int NCP>
__device__ __forceinline__ void lane_logits(const FNetDev &net, const float *u0, int np, const int (&pp)[kMaxK],
                                            const float (&ee)[kMaxK], int p, float e, float *a2w, int lane,
                                            float (&z)[NCP]) {
    float a1[H1];
    {
        float v[H1];
#pragma unroll
        for (int j = 0; j < H1; ++j) v[j] = cld(u0 + j);
#pragma unroll
        for (int t = 0; t < kMaxK - 1; ++t) {
            if (t < np) {
                const float *row = net.W1P + (int64_t)pp[t] * H1;
#pragma unroll
                for (int j = 0; j < H1; ++j) v[j] = fmaf(ee[t], cld(row + j), v[j]);
            }
        }
        const float4 *w1 = reinterpret_cast<const float4 *>(net.W1P + (int64_t)p * H1);
#pragma unroll
        for (int j4 = 0; j4 < H1 / 4; ++j4) {
            const float4 w = w1[j4];
            a1[4 * j4 + 0] = sigmoid_f32(fmaf(e, w.x, v[4 * j4 + 0]));
            a1[4 * j4 + 1] = sigmoid_f32(fmaf(e, w.y, v[4 * j4 + 1]));
            a1[4 * j4 + 2] = sigmoid_f32(fmaf(e, w.z, v[4 * j4 + 2]));
            a1[4 * j4 + 3] = sigmoid_f32(fmaf(e, w.w, v[4 * j4 + 3]));
        }
    }
    if constexpr (H2 == 0) {
        const float *W = opaque(net.WP[2]);
        const float *B = opaque(net.bP[2]);
#pragma unroll
        for (int j = 0; j < NCP; ++j) z[j] = cld(B + j);
#pragma unroll
        for (int ib = 0; ib < H1; ib += kF32SumBlock) {
            float part[NCP];
#pragma unroll
            for (int j = 0; j < NCP; ++j) part[j] = 0.0f;
#pragma unroll
            for (int i = ib; i < ib + kF32SumBlock && i < H1; ++i)
#pragma unroll
                for (int j = 0; j < NCP; ++j) part[j] = fmaf(cld(W + i * NCP + j), a1[i], part[j]);
#pragma unroll
            for (int j = 0; j < NCP; ++j) z[j] += part[j];
        }
    } else {
        const float *W2 = opaque(net.WP[2]);
        const float *B2 = opaque(net.bP[2]);
        // second hidden layer, 16 units per step, into this lane's LDS column
#pragma unroll 1
        for (int jb = 0; jb < H2; jb += 16) {
            float tot[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) tot[jj] = cld(B2 + jb + jj);
#pragma unroll
            for (int ib = 0; ib < H1; ib += kF32SumBlock) {
                float part[16];
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) part[jj] = 0.0f;
#pragma unroll
                for (int i = ib; i < ib + kF32SumBlock && i < H1; ++i)
#pragma unroll
                    for (int jj = 0; jj < 16; ++jj) part[jj] = fmaf(cld(W2 + i * H2 + jb + jj), a1[i], part[jj]);
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) tot[jj] += part[jj];
            }
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) a2w[(jb + jj) * 64 + lane] = sigmoid_f32(tot[jj]);
        }
        const float *W3 = opaque(net.WP[3]);
        const float *B3 = opaque(net.bP[3]);
#pragma unroll
        for (int j = 0; j < NCP; ++j) z[j] = cld(B3 + j);
#pragma unroll
        for (int ib = 0; ib < H2; ib += kF32SumBlock) {
            float part[NCP];
#pragma unroll
            for (int j = 0; j < NCP; ++j) part[j] = 0.0f;
#pragma unroll 4
            for (int i = ib; i < ib + (H2 < kF32SumBlock ? H2 : kF32SumBlock); ++i) {
                const float a = a2w[i * 64 + lane];
#pragma unroll
                for (int j = 0; j < NCP; ++j) part[j] = fmaf(cld(W3 + i * NCP + j), a, part[j]);
            }
#pragma unroll
            for (int j = 0; j < NCP; ++j) z[j] += part[j];
        }
    }
}

// Persistent enumeration, one point per lane; chunks of 64 consecutive
// last-element positions of one segment (the prefix is the same for the
// whole wave, so its loads go through the scalar cache).
template <int H1, int H2, int NCP>
__global__ void __launch_bounds__(256) enum_f32_lane_kernel(FEnumParams P) {
    constexpr int CH = kF32LaneChunk;
    __shared__ float a2s[kLaneWaves][H2 > 0 ? H2 : 1][64];
    const int lane = __lane_id();
    float *a2w = &a2s[threadIdx.x >> 6][0][0];
    const int nc = P.net.dims[P.net.L];
    Cursor c;
    int64_t cur = 0, end = 0;
    while (true) {
        if (cur >= end) {
            const int64_t start = f32_ticket(P);
            if (start < 0) break;
            cur = start;
            end = min(start + (int64_t)P.batch, P.total_chunks);
            cursor_decode<CH, FEnumParams>(c, P, cur);
        }
        int pp[kMaxK];
        float ee[kMaxK];
        const int np = c.k - 1;
#pragma unroll
        for (int t = 0; t < kMaxK; ++t) {
            pp[t] = 0;
            ee[t] = 0.0f;
            if (t < np) {
                pp[t] = c.pre[t];
                const int xv = wave_uniform((int)gld(c.img + pp[t]));
                ee[t] = eff_delta(xv, wave_uniform((int)gld(c.dl + c.dg[t])));
            }
        }
        int p = 0, i = 0;
        const bool valid = last_element32<FEnumParams>(c, P, (int)(c.ch * CH) + lane, p, i);
        const float e = eff_delta((int)gld(c.img + p), (int)gld(c.dl + i));
        float z[NCP];
        lane_logits<H1, H2, NCP>(P.net, P.u0f + (int64_t)c.prop * P.u0_stride, np, pp, ee, p, e, a2w, lane, z);
        int best;
        float top, margin;
        decide_f32<NCP>(z, nc, best, top, margin);
        const int label0 = wave_uniform(gld(&P.props[c.prop].label0));
        const bool near = valid && margin <= P.tie_rel * fmaxf(1.0f, fabsf(top));
        const bool viol = valid && best != label0;
        emit_f32(P, c, viol, near, p, i, best);
        cur++;
        if (cur < end) cursor_next<CH, FEnumParams>(c, P);
    }
}

// Listed points (or the clean images of listed properties), one per lane,
// through lane_logits.
template <int H1, int H2, int NCP>
__global__ void __launch_bounds__(256) eval_f32_lane_kernel(F32EvalParams E) {
    __shared__ float a2s[kLaneWaves][H2 > 0 ? H2 : 1][64];
    const int lane = __lane_id();
    float *a2w = &a2s[threadIdx.x >> 6][0][0];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = t < E.n;
    const int64_t tt = ok ? t : 0;
    const int prop = E.prop_of ? E.prop_of[tt] : 0;
    const PropDev &pr = E.props[prop];
    const int k = E.label_props ? 0 : E.ks[tt];
    const int64_t rank = E.label_props ? 0 : E.ranks[tt];
    int pix[kMaxK], dig[kMaxK];
    decode_point_dev(pr.n, pr.m, k, rank, pix, dig);
    int pp[kMaxK];
    float ee[kMaxK];
    const int np = k > 0 ? k - 1 : 0;
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        pp[j] = 0;
        ee[j] = 0.0f;
        if (j < np) {
            pp[j] = pix[j];
            ee[j] = eff_delta(pr.image[pix[j]], pr.deltas[dig[j]]);
        }
    }
    int p = 0;
    float e = 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
        if (k > 0 && j == k - 1) { p = pix[j]; e = eff_delta(pr.image[pix[j]], pr.deltas[dig[j]]); }
    float z[NCP];
    lane_logits<H1, H2, NCP>(E.net, E.u0f + (int64_t)prop * E.u0_stride, np, pp, ee, p, e, a2w, lane, z);
    const int nc = E.net.dims[E.net.L];
    int best;
    float top, margin;
    decide_f32<NCP>(z, nc, best, top, margin);
    if (!ok) return;
    if (E.label_props) {
        E.label_props[prop].label0 = best;
        E.label_props[prop].tie0 = 0;
        return;
    }
    if (E.logits)
#pragma unroll
        for (int j = 0; j < NCP; ++j)
            if (j < nc) E.logits[tt * nc + j] = z[j];
    if (E.labels) E.labels[tt] = best;
    if (E.margins) E.margins[tt] = margin;
}

// A compiled lane instance: L weight layers, padded widths, its kernels.
struct F32LaneVariant {
    int L, h1, h2, ncp;
    const void *enum_fn;
    const void *eval_fn;
};

#define IBMC_F32_LANE(H1, H2, NCP)                                                                 \
    F32LaneVariant { (H2) > 0 ? 3 : 2, H1, H2, NCP,                                                \
                     reinterpret_cast<const void *>(&enum_f32_lane_kernel<H1, H2, NCP>),            \
                     reinterpret_cast<const void *>(&eval_f32_lane_kernel<H1, H2, NCP>) }

// Instance tables (one per source file, to split compilation).
const F32LaneVariant *f32_lane_variants_l2(int *n);
const F32LaneVariant *f32_lane_variants_l3(int *n);

}  // namespace ibmc
