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

// The table sigmoid: knots u_i = -8 + i/16 holding sigma(u_i) in FP32 (tab,
// kLutIntervals + 1 values), linear between knots, the end values outside.
__device__ __forceinline__ float table_sigmoid(float u, const float *tab) {
    const float t = (u + 8.0f) * 16.0f;
    if (!(t > 0.0f)) return tab[0];
    if (t >= (float)kLutIntervals) return tab[kLutIntervals];
    const int i = (int)t;
    const float a = tab[i];
    return fmaf(t - (float)i, tab[i + 1] - a, a);
}

// Hidden-layer activation: the exponential form, or the table (use_tab).
__device__ __forceinline__ float act_f32(float u, bool use_tab, const float *tab) {
    return use_tab ? table_sigmoid(u, tab) : sigmoid_f32(u);
}

// Stage the table sigmoid's knots in LDS (every thread of the block takes
// part; tab: the block's LDS copy).  Returns whether the table is used.
__device__ __forceinline__ bool stage_table(const float *lut, float *tab) {
    if (!lut) return false;
    for (int i = threadIdx.x; i <= kLutIntervals; i += blockDim.x) tab[i] = lut[i];
    __syncthreads();
    return true;
}

// Cross-lane exchange through this wave's LDS: earlier writes complete
// before later reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// Tickets between two reads of the host's abort request by one wave (a read
// of host memory crosses PCIe; one per ticket from every wave saturated it).
constexpr int kAbortPollTickets = 64;

// Next queue ticket of a persistent wave: [start, end) of at most P.batch
// chunks from the wave's current slice q; a drained slice sends the wave to
// the next one (tries counts the slices visited).  Returns -1 when every
// slice is drained or a stop / abort was requested.  The device stop flag is
// read per ticket, the host abort request every kAbortPollTickets tickets
// (polls counts them; never at a wave's first ticket, where every wave of the
// grid would read host memory at once); a wave that sees the abort raises
// the stop flag.
template <class PT>
__device__ __forceinline__ int64_t f32_ticket(const PT &P, int &q, int &tries, int64_t &end, int &polls) {
    while (tries < kF32Queues) {
        const int64_t lo = (int64_t)q * P.slice;
        const int64_t hi = min(lo + P.slice, P.total_chunks);
        unsigned long long t = 0;
        int stop = 0;
        const bool poll_host = P.abort_host && (++polls % kAbortPollTickets) == 0;
        if (__lane_id() == 0) {
            if (lo < hi) t = atomicAdd(P.queue + (int64_t)q * kQueueStride, (unsigned long long)P.batch);
            stop = *P.stop_flag;
            if (poll_host && *P.abort_host) {
                stop = 1;
                *P.stop_flag = 1;
            }
        }
        if (wave_uniform(stop)) return -1;
        const int64_t start = lo + (int64_t)wave_uniform(t);
        if (lo < hi && start < hi) {
            end = min(start + (int64_t)P.batch, hi);
            return start;
        }
        q = q + 1 == kF32Queues ? 0 : q + 1;
        tries++;
    }
    return -1;
}

// The first slice of a wave: waves are spread evenly over the slices.
__device__ __forceinline__ int f32_first_slice() {
    const int w = (int)((blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6));
    return w % kF32Queues;
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

// Layers >= 2 of the lane's point from its first-layer activations a1.
// a2w: this wave's LDS columns ([H2][64] of the second hidden layer, or
// [NCP][64] of the logits with one hidden layer); each lane touches only its
// own column.
template <int H1, int H2, int NCP>
__device__ __forceinline__ void lane_upper(const FNetDev &net, const float (&a1)[H1], float *a2w, int lane,
                                           float (&z)[NCP], bool use_tab, const float *tab) {
    if constexpr (H2 == 0) {
        const float *W = opaque(net.WP[2]);
        const float *B = opaque(net.bP[2]);
        // eight classes per step (eight scalar weights per input in flight),
        // each step's logits parked in this lane's LDS column
#pragma unroll 1
        for (int j0 = 0; j0 < NCP; j0 += 8) {
            float tot[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) tot[j] = cld(B + j0 + j);
#pragma unroll
            for (int ib = 0; ib < H1; ib += kF32SumBlock) {
                float part[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) part[j] = 0.0f;
#pragma unroll
                for (int i = ib; i < ib + kF32SumBlock && i < H1; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) part[j] = fmaf(cld(W + i * NCP + j0 + j), a1[i], part[j]);
#pragma unroll
                for (int j = 0; j < 8; ++j) tot[j] += part[j];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) a2w[(j0 + j) * 64 + lane] = tot[j];
        }
#pragma unroll
        for (int j = 0; j < NCP; ++j) z[j] = a2w[j * 64 + lane];
    } else {
        const float *W2 = opaque(net.WP[2]);
        const float *B2 = opaque(net.bP[2]);
        // second hidden layer, eight units per step, into this lane's LDS column
#pragma unroll 1
        for (int jb = 0; jb < H2; jb += 8) {
            float tot[8];
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) tot[jj] = cld(B2 + jb + jj);
#pragma unroll
            for (int ib = 0; ib < H1; ib += kF32SumBlock) {
                float part[8];
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) part[jj] = 0.0f;
#pragma unroll
                for (int i = ib; i < ib + kF32SumBlock && i < H1; ++i)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) part[jj] = fmaf(cld(W2 + i * H2 + jb + jj), a1[i], part[jj]);
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) tot[jj] += part[jj];
            }
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) a2w[(jb + jj) * 64 + lane] = act_f32(tot[jj], use_tab, tab);
        }
        const float *W3 = opaque(net.WP[3]);
        const float *B3 = opaque(net.bP[3]);
#pragma unroll
        for (int j0 = 0; j0 < NCP; j0 += 8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) z[j0 + j] = cld(B3 + j0 + j);
#pragma unroll
            for (int ib = 0; ib < H2; ib += kF32SumBlock) {
                float part[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) part[j] = 0.0f;
#pragma unroll 4
                for (int i = ib; i < ib + (H2 < kF32SumBlock ? H2 : kF32SumBlock); ++i) {
                    const float a = a2w[i * 64 + lane];
#pragma unroll
                    for (int j = 0; j < 8; ++j) part[j] = fmaf(cld(W3 + i * NCP + j0 + j), a, part[j]);
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) z[j0 + j] += part[j];
            }
        }
    }
}

// First-layer potentials before the last pixel: v_j = u0_j, then one fma
// per prefix element in ascending pixel order.
__device__ __forceinline__ float prefix_potential_rt(const FNetDev &net, int h1p, const float *u0, int np,
                                                     const int (&pp)[kMaxK], const float (&ee)[kMaxK], int j) {
    float v = u0[j];
#pragma unroll
    for (int t = 0; t < kMaxK - 1; ++t)
        if (t < np) v = fmaf(ee[t], net.W1P[(int64_t)pp[t] * h1p + j], v);
    return v;
}

template <int H1>
__device__ __forceinline__ float prefix_potential(const FNetDev &net, const float *u0, int np, const int (&pp)[kMaxK],
                                                  const float (&ee)[kMaxK], int j) {
    return prefix_potential_rt(net, H1, u0, np, pp, ee, j);
}

// The prefix of the cursor's segment: pixels and effective deltas (their
// loads issued together).
__device__ __forceinline__ void segment_prefix(const Cursor &c, int (&pp)[kMaxK], float (&ee)[kMaxK]) {
    const int np = c.k - 1;
    int xs[kMaxK], ds[kMaxK];
#pragma unroll
    for (int t = 0; t < kMaxK; ++t) {
        xs[t] = 0;
        ds[t] = 0;
        if (t < np) { xs[t] = gld(c.img + c.pre[t]); ds[t] = gld(c.dl + c.dg[t]); }
    }
#pragma unroll
    for (int t = 0; t < kMaxK; ++t) {
        pp[t] = t < np ? c.pre[t] : 0;
        ee[t] = t < np ? eff_delta(xs[t], ds[t]) : 0.0f;
    }
}

// Persistent enumeration, one point per lane; chunks of 64 consecutive
// last-element positions of one segment.  Per segment (all prefix pixels
// fixed) the wave computes v_j before the last pixel once into its LDS slot;
// per property it keeps the clean label in a register; a chunk then loads
// only its own pixels, deltas and first-layer rows.
template <int H1, int H2, int NCP, bool TAB>
__global__ void __launch_bounds__(256) enum_f32_lane_kernel(FEnumParams P) {
    constexpr int CH = kF32LaneChunk;
    __shared__ float a2s[kLaneWaves][H2 > 0 ? H2 : NCP][64];
    __shared__ __attribute__((aligned(16))) float bases[kLaneWaves][H1];
    __shared__ float tab[kLutIntervals + 1];
    // TAB is a compile-time switch: a run-time choice inside the unrolled
    // layer loops keeps both activations live and spills the 128-wide ones
    const bool use_tab = TAB && stage_table(P.lut, tab);
    const int lane = __lane_id();
    float *a2w = &a2s[threadIdx.x >> 6][0][0];
    float *base = &bases[threadIdx.x >> 6][0];
    const int nc = P.net.dims[P.net.L];
    Cursor c;
    int64_t cur = 0, end = 0;
    bool seg_new = true;
    int prop_seen = -1, label0 = 0;
    int q = f32_first_slice(), tries = 0, polls = 0;
    while (true) {
        if (cur >= end) {
            const int64_t start = f32_ticket(P, q, tries, end, polls);
            if (start < 0) break;
            cur = start;
            cursor_decode<CH, FEnumParams>(c, P, cur);
            seg_new = true;
        }
        // the lane's point: its loads go out first
        int p = 0, i = 0;
        const bool valid = last_element32<FEnumParams>(c, P, (int)(c.ch * CH) + lane, p, i);
        const int xv = gld(c.img + p), dv = gld(c.dl + i);
        float4 wrow[H1 / 4];
        const float4 *w1 = reinterpret_cast<const float4 *>(P.net.W1P + (int64_t)p * H1);
#pragma unroll
        for (int j4 = 0; j4 < H1 / 4; ++j4) wrow[j4] = w1[j4];
        if (c.prop != prop_seen) {
            prop_seen = c.prop;
            label0 = wave_uniform(gld(&P.props[c.prop].label0));
        }
        if (seg_new) {
            int pp[kMaxK];
            float ee[kMaxK];
            segment_prefix(c, pp, ee);
            const float *u0 = P.u0f + (int64_t)c.prop * P.u0_stride;
#pragma unroll
            for (int j0 = 0; j0 < H1; j0 += 64)
                if (j0 + lane < H1) base[j0 + lane] = prefix_potential<H1>(P.net, u0, c.k - 1, pp, ee, j0 + lane);
            wave_lds_sync();
            seg_new = false;
        }
        const float e = eff_delta(xv, dv);
        float a1[H1];
#pragma unroll
        for (int j4 = 0; j4 < H1 / 4; ++j4) {
            const float4 b = *reinterpret_cast<const float4 *>(base + 4 * j4);
            a1[4 * j4 + 0] = act_f32(fmaf(e, wrow[j4].x, b.x), use_tab, tab);
            a1[4 * j4 + 1] = act_f32(fmaf(e, wrow[j4].y, b.y), use_tab, tab);
            a1[4 * j4 + 2] = act_f32(fmaf(e, wrow[j4].z, b.z), use_tab, tab);
            a1[4 * j4 + 3] = act_f32(fmaf(e, wrow[j4].w, b.w), use_tab, tab);
        }
        float z[NCP];
        lane_upper<H1, H2, NCP>(P.net, a1, a2w, lane, z, use_tab, tab);
        int best;
        float top, margin;
        decide_f32<NCP>(z, nc, best, top, margin);
        bool near = valid && margin <= P.tie_rel * fmaxf(1.0f, fabsf(top));
        bool viol = valid && best != label0;
        if (P.literal) {
            // the threshold literal: the desired (clean) class below V, another above
            float zd = z[0], other = -INFINITY;
#pragma unroll
            for (int j = 0; j < NCP; ++j) {
                if (j == label0) zd = z[j];
                else if (j < nc) other = fmaxf(other, z[j]);
            }
            const float V = P.lit_v;
            viol = valid && zd < V && other > V;
            near = valid && fminf(fabsf(zd - V), fabsf(other - V)) <= P.tie_rel * fmaxf(1.0f, fabsf(V));
        }
        emit_f32(P, c, viol, near, p, i, best);
        cur++;
        if (cur < end) seg_new = cursor_next<CH, FEnumParams>(c, P);
    }
}

// Listed points (or the clean images of listed properties), one per lane,
// in the same sequence of operations.
template <int H1, int H2, int NCP, bool TAB>
__global__ void __launch_bounds__(256) eval_f32_lane_kernel(F32EvalParams E) {
    __shared__ float a2s[kLaneWaves][H2 > 0 ? H2 : NCP][64];
    __shared__ float tab[kLutIntervals + 1];
    const bool use_tab = TAB && stage_table(E.lut, tab);
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
    int p = 0;
    float e = 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        pp[j] = 0;
        ee[j] = 0.0f;
        if (j < np) { pp[j] = pix[j]; ee[j] = eff_delta(pr.image[pix[j]], pr.deltas[dig[j]]); }
        if (k > 0 && j == k - 1) { p = pix[j]; e = eff_delta(pr.image[pix[j]], pr.deltas[dig[j]]); }
    }
    const float *u0 = E.u0f + (int64_t)prop * E.u0_stride;
    const float *w1 = E.net.W1P + (int64_t)p * H1;
    float a1[H1];
#pragma unroll
    for (int j = 0; j < H1; ++j)
        a1[j] = act_f32(fmaf(e, w1[j], prefix_potential<H1>(E.net, u0, np, pp, ee, j)), use_tab, tab);
    float z[NCP];
    lane_upper<H1, H2, NCP>(E.net, a1, a2w, lane, z, use_tab, tab);
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
// enum_fn[t] / eval_fn[t]: the exponential sigmoid (t = 0) or the table (t = 1).
struct F32LaneVariant {
    int L, h1, h2, ncp;
    const void *enum_fn[2];
    const void *eval_fn[2];
};

#define IBMC_F32_LANE(H1, H2, NCP)                                                                 \
    F32LaneVariant { (H2) > 0 ? 3 : 2, H1, H2, NCP,                                                \
                     {reinterpret_cast<const void *>(&enum_f32_lane_kernel<H1, H2, NCP, false>),    \
                      reinterpret_cast<const void *>(&enum_f32_lane_kernel<H1, H2, NCP, true>)},    \
                     {reinterpret_cast<const void *>(&eval_f32_lane_kernel<H1, H2, NCP, false>),    \
                      reinterpret_cast<const void *>(&eval_f32_lane_kernel<H1, H2, NCP, true>)} }

// Instance tables (one per source file, to split compilation).
const F32LaneVariant *f32_lane_variants_l2(int *n);
const F32LaneVariant *f32_lane_variants_l3(int *n);

}  // namespace ibmc
