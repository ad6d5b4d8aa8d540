// Float-network (sigmoid variant) kernels: plain forward and replay (the
// dense reference path, device expf), the clean pass of the enumeration, the
// sixteen-points-per-wave enumeration for wide networks, evaluation of
// listed points with the enumeration arithmetic, and the launchers that pick
// a kernel family per network.
#include "kernels_f32.h"
#include "f32_impl.h"

namespace ibmc {

__device__ __forceinline__ float sigmoidf(float u) { return 1.0f / (1.0f + expf(-u)); }

// Plain forward of one image held in LDS (xs = pixel / 256); one workgroup.
__device__ void dense_forward_f32_block(const FNetDev &net, const float *xs, float *a0, float *a1,
                                        float *pot, float *u0_out, int *label, float *margin,
                                        float *top) {
    const int tid = threadIdx.x;
    const int n = net.dims[0], h1 = net.dims[1];
    for (int j = tid; j < h1; j += blockDim.x) {
        float u = net.bd[1][j];
        for (int i = 0; i < n; ++i) u = fmaf(net.W1T[(int64_t)i * h1 + j], xs[i], u);
        if (pot) pot[j] = u;
        if (u0_out) u0_out[j] = u;
        a0[j] = sigmoidf(u);
    }
    __syncthreads();
    float *in = a0, *out = a1;
    int po = h1;
    for (int l = 2; l <= net.L; ++l) {
        const int nin = net.dims[l - 1], nout = net.dims[l];
        for (int j = tid; j < nout; j += blockDim.x) {
            float u = net.bd[l][j];
            for (int i = 0; i < nin; ++i) u = fmaf(net.WT[l][(int64_t)i * nout + j], in[i], u);
            if (pot) pot[po + j] = u;
            out[j] = (l < net.L) ? sigmoidf(u) : u;
        }
        po += nout;
        __syncthreads();
        float *t = in; in = out; out = t;
    }
    if (tid == 0) {
        const int nc = net.dims[net.L];
        int best = 0;
        for (int j = 1; j < nc; ++j) if (in[j] > in[best]) best = j;
        float second = -INFINITY;
        for (int j = 0; j < nc; ++j) if (j != best && in[j] > second) second = in[j];
        *label = best;
        *margin = in[best] - second;
        *top = in[best];
    }
}

__global__ void __launch_bounds__(256) forward_f32_kernel(FNetDev net, const uint8_t *images, int64_t n_images,
                                                          int32_t *labels, float *pots, int64_t pot_stride) {
    __shared__ float xs[kMaxWidth], a0[kMaxWidth], a1[kMaxWidth];
    __shared__ int lab;
    __shared__ float mg, top;
    for (int64_t img = blockIdx.x; img < n_images; img += gridDim.x) {
        const uint8_t *x = images + img * net.dims[0];
        for (int i = threadIdx.x; i < net.dims[0]; i += blockDim.x) xs[i] = (float)x[i] * (1.0f / 256.0f);
        __syncthreads();
        dense_forward_f32_block(net, xs, a0, a1, pots ? pots + img * pot_stride : nullptr, nullptr, &lab, &mg, &top);
        __syncthreads();
        if (threadIdx.x == 0 && labels) labels[img] = lab;
        __syncthreads();
    }
}

// Clean first-layer potentials of listed properties, padded to HP[1] with
// zeros (the enumeration's u0), one workgroup per property: u_j = b_j +
// sum_i W1[j][i] x_i / 256 by fma in pixel order.
__global__ void __launch_bounds__(256) clean_u0_f32_kernel(FNetDev net, const PropDev *props, const int32_t *prop_ids,
                                                           int32_t n_ids, float *u0_store, int64_t u0_stride) {
    const int n = net.dims[0], h1 = net.dims[1], hp = net.HP[1];
    for (int t = blockIdx.x; t < n_ids; t += gridDim.x) {
        const int pid = prop_ids[t];
        const uint8_t *x = props[pid].image;
        float *out = u0_store + (int64_t)pid * u0_stride;
        for (int j = threadIdx.x; j < hp; j += blockDim.x) {
            float u = 0.0f;
            if (j < h1) {
                u = net.bd[1][j];
                for (int i = 0; i < n; ++i) u = fmaf(net.W1T[(int64_t)i * h1 + j], (float)x[i] * (1.0f / 256.0f), u);
            }
            out[j] = u;
        }
    }
}

__global__ void __launch_bounds__(256) replay_f32_kernel(FNetDev net, const uint8_t *clean, const int16_t *deltas,
                                                         int m, const CexRec *recs, int64_t n_recs, int32_t *labels) {
    __shared__ float xs[kMaxWidth], a0[kMaxWidth], a1[kMaxWidth];
    __shared__ int lab;
    __shared__ float mg, top;
    __shared__ int xi[kMaxWidth];
    const int n = net.dims[0];
    for (int64_t r = blockIdx.x; r < n_recs; r += gridDim.x) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) xi[i] = clean[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            const int k = recs[r].k;
            int64_t mk = 1;
            for (int j = 0; j < k; ++j) mk *= m;
            int p[kMaxK];
            lex_unrank_subset(recs[r].rank / mk, k, n, p);
            int64_t d = recs[r].rank % mk;
            for (int j = k - 1; j >= 0; --j) {
                xi[p[j]] = clamp_pixel(xi[p[j]] + deltas[d % m]);
                d /= m;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = (float)xi[i] * (1.0f / 256.0f);
        __syncthreads();
        dense_forward_f32_block(net, xs, a0, a1, nullptr, nullptr, &lab, &mg, &top);
        __syncthreads();
        if (threadIdx.x == 0) labels[r] = lab;
        __syncthreads();
    }
}



hipError_t launch_forward_f32(const FNetDev &net, const uint8_t *images, int64_t n_images, int32_t *labels,
                              float *pots, int64_t pot_stride, hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_images, 4096);
    hipLaunchKernelGGL(forward_f32_kernel, dim3(grid), dim3(256), 0, s, net, images, n_images, labels, pots,
                       pot_stride);
    return hipGetLastError();
}

hipError_t launch_replay_f32(const FNetDev &net, const uint8_t *clean, const int16_t *deltas, int m,
                             const CexRec *recs, int64_t n_recs, int32_t *labels, hipStream_t s) {
    if (n_recs <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_recs, 8192);
    hipLaunchKernelGGL(replay_f32_kernel, dim3(grid), dim3(256), 0, s, net, clean, deltas, m, recs, n_recs, labels);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sixteen points per wave (wide networks)
// ---------------------------------------------------------------------------

// LDS of one wave: activations of 16 points in two buffers [16][wp], logits
// [16][64], the segment's first-layer potentials before the last pixel [HP1].
__host__ __device__ inline int wide_wp(const FNetDev &net) {
    int wp = 64;
    for (int l = 1; l < net.L; ++l) wp = max(wp, net.HP[l]);
    return wp;
}
static size_t wide_lds_bytes(const FNetDev &net) {
    return (size_t)(2 * 16 * wide_wp(net) + 16 * 64 + net.HP[1]) * 4;
}

// Layers >= 2 of 16 points (lanes = units, 64 at a time) from the
// first-layer activations in act0 [16][wp]; logits to zs [16][64].
__device__ void wide_upper(const FNetDev &net, float *act0, float *act1, float *zs, int wp, int lane) {
    float *in = act0, *out = act1;
    for (int l = 2; l <= net.L; ++l) {
        const int nin = net.HP[l - 1], nout = net.HP[l];
        const float *W = net.WP[l];
        const float *B = net.bP[l];
        const bool last = l == net.L;
        for (int jb = 0; jb < nout; jb += 64) {
            const int j = jb + lane;
            float tot[16];
            const float bj = B[j];
#pragma unroll
            for (int t = 0; t < 16; ++t) tot[t] = bj;
            for (int ib = 0; ib < nin; ib += kF32SumBlock) {
                float part[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) part[t] = 0.0f;
#pragma unroll 2
                for (int i = ib; i < ib + kF32SumBlock; i += 4) {
                    const float w0 = W[(int64_t)(i + 0) * nout + j], w1 = W[(int64_t)(i + 1) * nout + j];
                    const float w2 = W[(int64_t)(i + 2) * nout + j], w3 = W[(int64_t)(i + 3) * nout + j];
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        const float4 a = *reinterpret_cast<const float4 *>(in + t * wp + i);
                        part[t] = fmaf(w0, a.x, part[t]);
                        part[t] = fmaf(w1, a.y, part[t]);
                        part[t] = fmaf(w2, a.z, part[t]);
                        part[t] = fmaf(w3, a.w, part[t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < 16; ++t) tot[t] += part[t];
            }
            if (!last) {
#pragma unroll
                for (int t = 0; t < 16; ++t) out[t * wp + j] = sigmoid_f32(tot[t]);
            } else {
#pragma unroll
                for (int t = 0; t < 16; ++t) zs[t * 64 + j] = tot[t];
            }
        }
        wave_lds_sync();
        float *tmp = in;
        in = out;
        out = tmp;
    }
}

// Decision of point `lane` (< 16) from the logits in zs.
__device__ __forceinline__ void wide_decide(const float *zs, int nc, int lane, int &best, float &top, float &margin) {
    const float *z = zs + (lane & 15) * 64;
    best = 0;
    top = z[0];
    for (int j = 1; j < nc; ++j)
        if (z[j] > top) { top = z[j]; best = j; }
    float second = -INFINITY;
    for (int j = 0; j < nc; ++j)
        if (j != best) second = fmaxf(second, z[j]);
    margin = top - second;
}

__global__ void __launch_bounds__(64) enum_f32_wide_kernel(FEnumParams P) {
    constexpr int CH = kF32WideChunk;
    extern __shared__ __attribute__((aligned(16))) float wlds[];
    const FNetDev &net = P.net;
    const int wp = wide_wp(net), hp1 = net.HP[1], nc = net.dims[net.L];
    float *act0 = wlds, *act1 = wlds + 16 * wp, *zs = wlds + 32 * wp, *base = wlds + 32 * wp + 16 * 64;
    const int lane = __lane_id();
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
        int p = 0, i = 0;
        const bool valid = last_element32<FEnumParams>(c, P, (int)(c.ch * CH) + (lane & 15), p, i) && lane < 16;
        const float e = eff_delta((int)gld(c.img + p), (int)gld(c.dl + i));
        if (c.prop != prop_seen) {
            prop_seen = c.prop;
            label0 = wave_uniform(gld(&P.props[c.prop].label0));
        }
        if (seg_new) {
            // the segment's potentials before the last pixel, each lane its own units
            int pp[kMaxK];
            float ee[kMaxK];
            segment_prefix(c, pp, ee);
            const float *u0 = P.u0f + (int64_t)c.prop * P.u0_stride;
            for (int jb = 0; jb < hp1; jb += 64)
                base[jb + lane] = prefix_potential_rt(net, hp1, u0, c.k - 1, pp, ee, jb + lane);
            seg_new = false;
        }
        // first layer: each point's last pixel on the segment's potentials
        for (int jb = 0; jb < hp1; jb += 64) {
            const int j = jb + lane;
            const float vb = base[j];
#pragma unroll 4
            for (int t = 0; t < 16; ++t) {
                const int pt = __builtin_amdgcn_readlane(p, t);
                const float et = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e), t));
                act0[t * wp + j] = sigmoid_f32(fmaf(et, net.W1P[(int64_t)pt * hp1 + j], vb));
            }
        }
        wave_lds_sync();
        wide_upper(net, act0, act1, zs, wp, lane);
        int best;
        float top, margin;
        wide_decide(zs, nc, lane, best, top, margin);
        wave_lds_sync();   // the logits are read before the next chunk overwrites them
        const bool near = valid && margin <= P.tie_rel * fmaxf(1.0f, fabsf(top));
        const bool viol = valid && best != label0;
        emit_f32(P, c, viol, near, p, i, best);
        cur++;
        if (cur < end) seg_new = cursor_next<CH, FEnumParams>(c, P);
    }
}

// Listed points, sixteen per wave, through the same arithmetic: each point's
// first-layer potentials start from u0 and take its prefix pixels in
// ascending order, then its last pixel.
__global__ void __launch_bounds__(64) eval_f32_wide_kernel(F32EvalParams E) {
    extern __shared__ __attribute__((aligned(16))) float wlds[];
    const FNetDev &net = E.net;
    const int wp = wide_wp(net), hp1 = net.HP[1], nc = net.dims[net.L];
    float *act0 = wlds, *act1 = wlds + 16 * wp, *zs = wlds + 32 * wp;
    const int lane = __lane_id();
    const int64_t t0 = (int64_t)blockIdx.x * 16 + (lane & 15);
    const bool ok = lane < 16 && t0 < E.n;
    const int64_t tt = t0 < E.n ? t0 : 0;
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
    for (int jb = 0; jb < hp1; jb += 64) {
        const int j = jb + lane;
        for (int t = 0; t < 16; ++t) {
            const int pt = __builtin_amdgcn_readlane(prop, t);
            const int npt = __builtin_amdgcn_readlane(np, t);
            int ppt[kMaxK];
            float eet[kMaxK];
#pragma unroll
            for (int q = 0; q < kMaxK; ++q) {
                ppt[q] = __builtin_amdgcn_readlane(pp[q], t);
                eet[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ee[q]), t));
            }
            const float v = prefix_potential_rt(net, hp1, E.u0f + (int64_t)pt * E.u0_stride, npt, ppt, eet, j);
            const int ptl = __builtin_amdgcn_readlane(p, t);
            const float et = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e), t));
            act0[t * wp + j] = sigmoid_f32(fmaf(et, net.W1P[(int64_t)ptl * hp1 + j], v));
        }
    }
    wave_lds_sync();
    wide_upper(net, act0, act1, zs, wp, lane);
    int best;
    float top, margin;
    wide_decide(zs, nc, lane, best, top, margin);
    if (!ok) return;
    if (E.label_props) {
        E.label_props[prop].label0 = best;
        E.label_props[prop].tie0 = 0;
        return;
    }
    if (E.logits)
        for (int j = 0; j < nc; ++j) E.logits[tt * nc + j] = zs[lane * 64 + j];
    if (E.labels) E.labels[tt] = best;
    if (E.margins) E.margins[tt] = margin;
}

// ---------------------------------------------------------------------------
// layouts, dispatch, launchers
// ---------------------------------------------------------------------------

static int lane_class(int h) {
    for (int c : {16, 32, 64, 128})
        if (h <= c) return c;
    return 0;
}

static const F32LaneVariant *find_lane(int L, const int *HP) {
    int n2 = 0, n3 = 0;
    const F32LaneVariant *v2 = f32_lane_variants_l2(&n2), *v3 = f32_lane_variants_l3(&n3);
    if (L == 2)
        for (int i = 0; i < n2; ++i)
            if (v2[i].h1 == HP[1] && v2[i].ncp == HP[2]) return &v2[i];
    if (L == 3)
        for (int i = 0; i < n3; ++i)
            if (v3[i].h1 == HP[1] && v3[i].h2 == HP[2] && v3[i].ncp == HP[3]) return &v3[i];
    return nullptr;
}

bool f32_lane_supported(int L, const int *HP) { return find_lane(L, HP) != nullptr; }

F32Layout f32_layout(int L, const int *dims) {
    F32Layout lay{};
    lay.HP[0] = dims[0];
    bool lane = (L == 2 || L == 3) && dims[L] <= 16;
    for (int l = 1; l < L && lane; ++l) {
        lay.HP[l] = lane_class(dims[l]);
        if (lay.HP[l] == 0) lane = false;
    }
    if (lane) {
        lay.HP[L] = dims[L] <= 8 ? 8 : 16;
        if (!find_lane(L, lay.HP)) lane = false;
    }
    if (lane) {
        lay.kind = F32_LANE;
        return lay;
    }
    lay.kind = F32_WIDE;
    for (int l = 1; l < L; ++l) lay.HP[l] = round_up(dims[l], 64);
    lay.HP[L] = 64;
    return lay;
}

int enum_f32_chunk(const FNetDev &net) { return net.kind == F32_LANE ? kF32LaneChunk : kF32WideChunk; }

int f32_enum_grid(const FNetDev &net, int n_cu, bool table) {
    int occ = 0;
    if (net.kind == F32_LANE) {
        const F32LaneVariant *v = find_lane(net.L, net.HP);
        if (!v || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, v->enum_fn[table ? 1 : 0], 256, 0) != hipSuccess)
            return 0;
        return std::max(occ, 1) * n_cu * kLaneWaves;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, enum_f32_wide_kernel, 64, wide_lds_bytes(net)) !=
        hipSuccess)
        return 0;
    return std::max(occ, 1) * n_cu;
}

hipError_t launch_enum_f32(int grid_waves, const FEnumParams &P, hipStream_t s) {
    if (P.net.kind == F32_LANE) {
        const F32LaneVariant *v = find_lane(P.net.L, P.net.HP);
        if (!v) return hipErrorInvalidValue;
        FEnumParams a = P;
        void *args[] = {&a};
        return hipLaunchKernel(v->enum_fn[P.lut ? 1 : 0], dim3((grid_waves + kLaneWaves - 1) / kLaneWaves), dim3(256), args, 0, s);
    }
    hipLaunchKernelGGL(enum_f32_wide_kernel, dim3(grid_waves), dim3(64), wide_lds_bytes(P.net), s, P);
    return hipGetLastError();
}

hipError_t launch_eval_f32(const F32EvalParams &E, hipStream_t s) {
    if (E.n <= 0) return hipSuccess;
    if (E.net.kind == F32_LANE) {
        const F32LaneVariant *v = find_lane(E.net.L, E.net.HP);
        if (!v) return hipErrorInvalidValue;
        F32EvalParams a = E;
        void *args[] = {&a};
        return hipLaunchKernel(v->eval_fn[E.lut ? 1 : 0], dim3((unsigned)((E.n + 255) / 256)), dim3(256), args, 0, s);
    }
    hipLaunchKernelGGL(eval_f32_wide_kernel, dim3((unsigned)((E.n + 15) / 16)), dim3(64), wide_lds_bytes(E.net), s, E);
    return hipGetLastError();
}

hipError_t launch_clean_f32(const FNetDev &net, PropDev *props, const int32_t *prop_ids, int32_t n_ids,
                            float *u0_store, int64_t u0_stride, hipStream_t s, const float *lut) {
    if (n_ids <= 0) return hipSuccess;
    hipLaunchKernelGGL(clean_u0_f32_kernel, dim3(std::min(n_ids, 4096)), dim3(256), 0, s, net, props, prop_ids, n_ids,
                       u0_store, u0_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the clean label through the enumeration's own arithmetic (a point with
    // no changed pixel), so that a zero perturbation reproduces it exactly
    F32EvalParams E{};
    E.net = net;
    E.props = props;
    E.label_props = props;
    E.prop_of = prop_ids;
    E.n = n_ids;
    E.u0f = u0_store;
    E.u0_stride = (int32_t)u0_stride;
    E.lut = lut;
    if (lut && net.kind != F32_LANE) return hipErrorInvalidValue;
    return launch_eval_f32(E, s);
}

}  // namespace ibmc
