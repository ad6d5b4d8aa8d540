// Integer enumeration with one point per lane, for small networks (one or
// two hidden layers of at most 64 units, at most 16 classes), where a 16x16
// matrix-core tile would be mostly padding.  Per point: the incremental
// first layer (Sec. II-A, Eq. (1): base + e W1[:, p], then the integer
// requantiser), the later layers as 4-way int8 dot products against weights
// that every lane shares (scalar loads), the lowest-index argmax and the
// decision against the clean label (Sec. III-C).  The domain is either the
// delta set (offsets clamped to [0, 255]) or the L2 ball of Sec. III-C,
// Eq. (9): digits map to offsets -rd..-1, 1..rd, and a point belongs to the
// ball when every pixel stays in [0, 255] and the squared length of its
// offsets is at most r2.
#include "f32_impl.h"
#include "kernels_lane.h"

namespace ibmc {

// Four activations clamp(u >> s, 0, 127) of one 32-bit word of first-layer
// weights (units 4w..4w+3), packed as bytes.
__device__ __forceinline__ int lane_act4(const int32_t *b, int w, int e, int s) {
    int a[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) {
        const int u = b[z] + e * ((w << (24 - 8 * z)) >> 24);
        a[z] = min(max(u >> s, 0), 127);
    }
    return a[0] | (a[1] << 8) | (a[2] << 16) | (a[3] << 24);
}

// Layer of NO outputs (multiple of 8) from NI / 4 packed int8 inputs: eight
// outputs per step, their weight words read through the scalar cache
// (layout [NO / 8][NI / 4][8]).  Hidden layers (REQ) requantise and pack,
// the output layer keeps the int32 logits.
template <int NI, int NO, bool REQ>
__device__ __forceinline__ void lane_layer(const int (&in)[NI / 4], const int32_t *W, const int32_t *B, int s,
                                           int (&out)[REQ ? NO / 4 : NO]) {
#pragma unroll
    for (int st = 0; st < NO / 8; ++st) {
        const int32_t *w = opaque(W + st * (NI / 4) * 8);
        int acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = cld(B + st * 8 + t);
#pragma unroll
        for (int i = 0; i < NI / 4; ++i)
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[t] = __builtin_amdgcn_sdot4(in[i], cld(w + i * 8 + t), acc[t], false);
        if constexpr (REQ) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int a[4];
#pragma unroll
                for (int z = 0; z < 4; ++z) a[z] = min(max(acc[4 * h + z] >> s, 0), 127);
                out[st * 2 + h] = a[0] | (a[1] << 8) | (a[2] << 16) | (a[3] << 24);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) out[st * 8 + t] = acc[t];
        }
    }
}

// Persistent enumeration: chunks of 64 consecutive last-element positions
// of one segment from the sliced queue.  Per segment the wave keeps the
// first-layer potentials before the last pixel in its LDS slot (and, for the
// ball, whether the prefix stays in [0, 255] and its squared length); per
// chunk it tallies counterexamples, exact ties and visited points of the
// level and writes the records with one atomic.
template <int H1, int H2>
__global__ void __launch_bounds__(256) enum_lane_kernel(LaneParams P) {
    constexpr int CH = kLaneChunk;
    constexpr int HL = H2 > 0 ? H2 : H1;
    __shared__ __attribute__((aligned(16))) int32_t bases[kLaneWaves][H1];
    const int lane = __lane_id();
    int32_t *base = &bases[threadIdx.x >> 6][0];
    const int nc = P.net.nc, s1 = P.net.s1, s2 = P.net.s2;
    Cursor c;
    int64_t cur = 0, end = 0;
    bool seg_new = true;
    int prop_seen = -1, label0 = 0, ball = 0, rd = 0, r2 = 0;
    int pre_ok = 1, pre_sq = 0;
    int q = f32_first_slice(), tries = 0, polls = 0;
    int tslot = -1;
    unsigned long long tcex = 0, tties = 0, tpts = 0;
    auto flush = [&]() __attribute__((always_inline)) {
        if (tslot >= 0 && lane == 0) {
            if (tcex) atomicAdd(P.slot_cex + tslot, tcex);
            if (tties) atomicAdd(P.slot_ties + tslot, tties);
            if (tpts) atomicAdd(P.slot_points + tslot, tpts);
        }
        tcex = tties = tpts = 0;
    };
    while (true) {
        if (cur >= end) {
            const int64_t start = f32_ticket(P, q, tries, end, polls);
            if (start < 0) break;
            cur = start;
            cursor_decode<CH, LaneParams>(c, P, cur);
            seg_new = true;
        }
        if (c.slot != tslot) {
            flush();
            tslot = c.slot;
        }
        // the lane's point: its loads go out first
        int p = 0, i = 0;
        bool valid = last_element32<LaneParams>(c, P, (int)(c.ch * CH) + lane, p, i);
        const int xv = gld(c.img + p);
        if (c.prop != prop_seen) {
            prop_seen = c.prop;
            const PropDev &pr = P.props[c.prop];
            label0 = wave_uniform(gld(&pr.label0));
            ball = wave_uniform(gld(&pr.ball));
            rd = wave_uniform(gld(&pr.ball_rd));
            r2 = wave_uniform(gld(&pr.ball_r2));
        }
        const int dv = ball ? ball_offset(i, rd) : (int)gld(c.dl + i);
        v4i wcol[H1 / 16];
        const v4i *w1 = reinterpret_cast<const v4i *>(P.net.W1C + (int64_t)p * H1);
#pragma unroll
        for (int t = 0; t < H1 / 16; ++t) wcol[t] = w1[t];
        if (seg_new) {
            const int np = c.k - 1;
            int pp[kMaxK], ee[kMaxK];
            int ok = 1, sq = 0;
#pragma unroll
            for (int t = 0; t < kMaxK; ++t) {
                pp[t] = 0;
                ee[t] = 0;
                if (t < np) {
                    pp[t] = c.pre[t];
                    const int xs = wave_uniform((int)gld(c.img + pp[t]));
                    if (ball) {
                        const int d = ball_offset(c.dg[t], rd);
                        ok &= (xs + d >= 0 && xs + d <= 255) ? 1 : 0;
                        sq += d * d;
                        ee[t] = d;
                    } else {
                        ee[t] = clamp_pixel(xs + wave_uniform((int)gld(c.dl + c.dg[t]))) - xs;
                    }
                }
            }
            pre_ok = ok;
            pre_sq = sq;
            const int32_t *u0 = P.u0 + (int64_t)c.prop * P.u0_stride;
            for (int j = lane; j < H1; j += 64) {
                const int qj = P.net.q1[j];
                int v = qj >= 0 ? u0[qj] : 0;
#pragma unroll
                for (int t = 0; t < kMaxK - 1; ++t)
                    if (t < np) v += ee[t] * (int)P.net.W1C[(int64_t)pp[t] * H1 + j];
                base[j] = v;
            }
            wave_lds_sync();
            seg_new = false;
        }
        int e;
        if (ball) {
            const int v = xv + dv;
            valid = valid && pre_ok && v >= 0 && v <= 255 && pre_sq + dv * dv <= r2;
            e = dv;
        } else {
            e = clamp_pixel(xv + dv) - xv;
        }
        const unsigned long long vmask = __ballot(valid);
        if (vmask) {
            // first layer from the segment base, requantised and packed
            int a1[H1 / 4];
#pragma unroll
            for (int t = 0; t < H1 / 16; ++t) {
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int4 b = *reinterpret_cast<const int4 *>(base + 16 * t + 4 * w);
                    const int32_t bb[4] = {b.x, b.y, b.z, b.w};
                    a1[4 * t + w] = lane_act4(bb, wcol[t][w], e, s1);
                }
            }
            int z[16];
            if constexpr (H2 > 0) {
                int a2[H2 / 4];
                lane_layer<H1, H2, true>(a1, P.net.W2S, P.net.b2, s2, a2);
                lane_layer<HL, 16, false>(a2, P.net.WOS, P.net.bo, 0, z);
            } else {
                lane_layer<HL, 16, false>(a1, P.net.WOS, P.net.bo, 0, z);
            }
            // lowest-index argmax of the nc logits and how many classes reach it
            int best = 0, top = z[0];
#pragma unroll
            for (int j = 1; j < 16; ++j)
                if (j < nc && z[j] > top) { top = z[j]; best = j; }
            int cnt = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) cnt += (j < nc && z[j] == top) ? 1 : 0;
            bool viol = valid && best != label0;
            bool tie = valid && cnt > 1;
            if (P.literal) {
                // the threshold literal: the desired (clean) class below V,
                // another above; ties: one of the two equals V
                int zd = z[0], other = INT32_MIN;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j == label0) zd = z[j];
                    else if (j < nc) other = max(other, z[j]);
                }
                viol = valid && zd < P.lit_v && other > P.lit_v;
                tie = valid && (zd == P.lit_v || other == P.lit_v);
            }
            const unsigned long long mv = __ballot(viol);
            if (mv) {
                unsigned long long rb = 0;
                if (lane == 0) rb = atomicAdd(P.rec_count, (unsigned long long)__popcll(mv));
                rb = wave_uniform(rb);
                if (viol) {
                    const unsigned long long idx = rb + lane_rank(mv);
                    if ((int64_t)idx < P.rec_cap) {
                        DevRec r;
                        r.rank = point_rank<LaneParams>(c, P, p, i);
                        r.prop = c.prop;
                        r.klab = (c.k << 24) | best;
                        P.recs[idx] = r;
                    }
                }
            }
            tcex += (unsigned long long)__popcll(mv);
            tties += (unsigned long long)__popcll(__ballot(tie));
            tpts += (unsigned long long)__popcll(vmask);
        }
        cur++;
        if (cur < end) seg_new = cursor_next<CH, LaneParams>(c, P);
    }
    flush();
}

struct LaneInst {
    int h1, h2;
    const void *fn;
};

#define IBMC_LANE(H1, H2) LaneInst { H1, H2, reinterpret_cast<const void *>(&enum_lane_kernel<H1, H2>) }

static const LaneInst kLaneInst[] = {
    IBMC_LANE(16, 0),  IBMC_LANE(32, 0),  IBMC_LANE(64, 0),  IBMC_LANE(16, 16), IBMC_LANE(16, 32), IBMC_LANE(16, 64),
    IBMC_LANE(32, 16), IBMC_LANE(32, 32), IBMC_LANE(32, 64), IBMC_LANE(64, 16), IBMC_LANE(64, 32), IBMC_LANE(64, 64),
};

int lane_width(int h) { return h <= 16 ? 16 : h <= 32 ? 32 : h <= 64 ? 64 : 0; }

bool lane_eligible(const int *dims, int L) {
    if (L != 2 && L != 3) return false;
    if (dims[1] < 1 || dims[1] > 64 || dims[L] > 16) return false;
    return L == 2 || (dims[2] >= 1 && dims[2] <= 64);
}

static const LaneInst *find_lane(const LaneNetDev &net) {
    for (const LaneInst &v : kLaneInst)
        if (v.h1 == net.LH1 && v.h2 == net.LH2) return &v;
    return nullptr;
}

int lane_enum_grid(const LaneNetDev &net, int n_cu) {
    const LaneInst *v = net.ok ? find_lane(net) : nullptr;
    if (!v) return 0;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, v->fn, 256, 0) != hipSuccess || occ < 1) return 0;
    return n_cu * occ;
}

hipError_t launch_enum_lane(int grid, const LaneParams &P, hipStream_t s) {
    const LaneInst *v = find_lane(P.net);
    if (!v || grid < 1) return hipErrorInvalidValue;
    void *args[] = {const_cast<LaneParams *>(&P)};
    return hipLaunchKernel(v->fn, dim3(grid), dim3(256), args, 0, s);
}

}  // namespace ibmc
