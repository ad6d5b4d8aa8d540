// Float-network (sigmoid variant) kernels: plain forward, clean pass, replay
// and the exhaustive enumeration with an incremental first layer on FP32
// vector FMA.  The sigmoid 1 / (1 + e^-u) calls the device expf.
#include "kernels_f32.h"
#include "enum_common.h"

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

__global__ void __launch_bounds__(256) clean_f32_kernel(FNetDev net, PropDev *props, const int32_t *prop_ids,
                                                        int32_t n_ids, float *u0_store, int64_t u0_stride) {
    __shared__ float xs[kMaxWidth], a0[kMaxWidth], a1[kMaxWidth];
    __shared__ int lab;
    __shared__ float mg, top;
    for (int t = blockIdx.x; t < n_ids; t += gridDim.x) {
        const int pid = prop_ids[t];
        const uint8_t *x = props[pid].image;
        for (int i = threadIdx.x; i < net.dims[0]; i += blockDim.x) xs[i] = (float)x[i] * (1.0f / 256.0f);
        __syncthreads();
        dense_forward_f32_block(net, xs, a0, a1, nullptr, u0_store + (int64_t)pid * u0_stride, &lab, &mg, &top);
        __syncthreads();
        if (threadIdx.x == 0) {
            props[pid].label0 = lab;
            props[pid].tie0 = 0;
        }
        __syncthreads();
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

// Enumeration, one chunk of 16 points per workgroup iteration.  LDS holds the
// segment base (h1 floats) and two activation buffers [16][width].
constexpr int kF32Chunk = 16;
constexpr int kF32MaxWidth = 512;

__global__ void __launch_bounds__(256) enum_f32_kernel(FEnumParams P, const int32_t *u0_index) {
    constexpr int CH = kF32Chunk;
    __shared__ float base[kF32MaxWidth];
    __shared__ __attribute__((aligned(16))) float act[2][CH][kF32MaxWidth];
    __shared__ int s_p[CH], s_i[CH], s_valid[CH];
    __shared__ float s_e[CH];
    __shared__ unsigned long long s_start;
    __shared__ int s_stop;
    const FNetDev &net = P.net;
    const int tid = threadIdx.x;
    const int h1 = net.dims[1];
    Cursor c;
    int64_t cur = 0, end = 0;
    bool have = false;
    while (true) {
        if (cur >= end) {
            if (tid == 0) {
                s_start = atomicAdd(P.queue, (unsigned long long)P.batch);
                s_stop = (*P.stop_flag) || (P.abort_host && *P.abort_host);
            }
            __syncthreads();
            const int64_t start = (int64_t)wave_uniform(s_start);
            const int stop = wave_uniform(s_stop);
            __syncthreads();
            if (start >= P.total_chunks || stop) break;
            cur = start;
            end = min(start + (int64_t)P.batch, P.total_chunks);
            cursor_decode<CH, FEnumParams>(c, P, cur);
            have = false;
        }
        const PropDev &pr = P.props[c.prop];
        if (!have) {
            // base = clean potentials + prefix column updates (e / 256) * W1[:, p]
            const float *u0 = P.u0f + (int64_t)u0_index[c.prop] * P.u0_stride;
            int pp[kMaxK];
            float ee[kMaxK];
            int np = 0;
            if (c.mode == SEG_PLAIN) {
                np = c.k - 1;
                for (int j = 0; j < kMaxK; ++j)
                    if (j < np) {
                        pp[j] = c.pre[j];
                        const int xv = pr.image[pp[j]];
                        ee[j] = (float)(clamp_pixel(xv + pr.deltas[c.dg[j]]) - xv) * (1.0f / 256.0f);
                    }
            }
            for (int j = tid; j < h1; j += blockDim.x) {
                float v = u0[j];
                for (int t = 0; t < kMaxK; ++t)
                    if (t < np) v = fmaf(ee[t], net.W1T[(int64_t)pp[t] * h1 + j], v);
                base[j] = v;
            }
            have = true;
        }
        if (tid < CH) {
            int p = 0, i = 0, pf = 0, f = 0;
            const int64_t o = c.ch * CH + tid;
            const bool v = last_element(c, P, o, p, i, pf, f);
            s_valid[tid] = v;
            s_p[tid] = v ? p : 0;
            s_i[tid] = v ? i : 0;
            const int xv = pr.image[s_p[tid]];
            s_e[tid] = (float)(clamp_pixel(xv + pr.deltas[s_i[tid]]) - xv) * (1.0f / 256.0f);
        }
        __syncthreads();
        // layer 1: incremental update + sigmoid
        for (int j = tid; j < h1; j += blockDim.x) {
            const float b = base[j];
            for (int t = 0; t < CH; ++t)
                act[0][t][j] = sigmoidf(fmaf(s_e[t], net.W1T[(int64_t)s_p[t] * h1 + j], b));
        }
        __syncthreads();
        int cur_buf = 0;
        for (int l = 2; l <= net.L; ++l) {
            const int nin = net.dims[l - 1], nout = net.dims[l];
            const float *WT = net.WT[l];
            for (int j = tid; j < nout; j += blockDim.x) {
                float acc[CH];
                const float b = net.bd[l][j];
#pragma unroll
                for (int t = 0; t < CH; ++t) acc[t] = b;
                // four inputs per step: one 16-byte LDS read per point feeds four
                // FMAs (the products still accumulate in input order)
                int i = 0;
                for (; i + 4 <= nin; i += 4) {
                    const float w0 = WT[(int64_t)(i + 0) * nout + j], w1 = WT[(int64_t)(i + 1) * nout + j];
                    const float w2 = WT[(int64_t)(i + 2) * nout + j], w3 = WT[(int64_t)(i + 3) * nout + j];
#pragma unroll
                    for (int t = 0; t < CH; ++t) {
                        const float4 a = *reinterpret_cast<const float4 *>(&act[cur_buf][t][i]);
                        acc[t] = fmaf(w0, a.x, acc[t]);
                        acc[t] = fmaf(w1, a.y, acc[t]);
                        acc[t] = fmaf(w2, a.z, acc[t]);
                        acc[t] = fmaf(w3, a.w, acc[t]);
                    }
                }
                for (; i < nin; ++i) {
                    const float w = WT[(int64_t)i * nout + j];
#pragma unroll
                    for (int t = 0; t < CH; ++t) acc[t] = fmaf(w, act[cur_buf][t][i], acc[t]);
                }
#pragma unroll
                for (int t = 0; t < CH; ++t) act[cur_buf ^ 1][t][j] = (l < net.L) ? sigmoidf(acc[t]) : acc[t];
            }
            __syncthreads();
            cur_buf ^= 1;
        }
        // decisions: one thread per point
        if (tid < CH && s_valid[tid]) {
            const float *z = act[cur_buf][tid];
            const int nc = net.dims[net.L];
            int best = 0;
            for (int j = 1; j < nc; ++j) if (z[j] > z[best]) best = j;
            float second = -INFINITY;
            for (int j = 0; j < nc; ++j) if (j != best && z[j] > second) second = z[j];
            const float margin = z[best] - second;
            const float scale = fmaxf(1.0f, fabsf(z[best]));
            const bool near = margin <= P.tie_rel * scale;
            const bool viol = best != pr.label0;
            if (near) {
                atomicAdd(P.slot_ties + c.slot, 1ull);
                const unsigned long long idx = atomicAdd(P.tie_count, 1ull);
                if ((int64_t)idx < P.tie_cap) {
                    DevRec r;
                    r.rank = point_rank(c, P, s_p[tid], s_i[tid]);
                    r.prop = c.prop;
                    r.klab = (c.k << 24) | best;
                    P.ties[idx] = r;
                }
            }
            if (viol) {
                atomicAdd(P.slot_cex + c.slot, 1ull);
                const unsigned long long idx = atomicAdd(P.rec_count, 1ull);
                if ((int64_t)idx < P.rec_cap) {
                    DevRec r;
                    r.rank = point_rank(c, P, s_p[tid], s_i[tid]);
                    r.prop = c.prop;
                    r.klab = (c.k << 24) | best;
                    P.recs[idx] = r;
                }
            }
        }
        __syncthreads();
        cur++;
        if (cur < end && cursor_next<CH, FEnumParams>(c, P)) have = false;
    }
}

int enum_f32_chunk() { return kF32Chunk; }

hipError_t launch_forward_f32(const FNetDev &net, const uint8_t *images, int64_t n_images, int32_t *labels,
                              float *pots, int64_t pot_stride, hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_images, 4096);
    hipLaunchKernelGGL(forward_f32_kernel, dim3(grid), dim3(256), 0, s, net, images, n_images, labels, pots,
                       pot_stride);
    return hipGetLastError();
}

hipError_t launch_clean_f32(const FNetDev &net, PropDev *props, const int32_t *prop_ids, int32_t n_ids,
                            float *u0_store, int64_t u0_stride, hipStream_t s) {
    if (n_ids <= 0) return hipSuccess;
    hipLaunchKernelGGL(clean_f32_kernel, dim3(std::min(n_ids, 4096)), dim3(256), 0, s, net, props, prop_ids, n_ids,
                       u0_store, u0_stride);
    return hipGetLastError();
}

hipError_t launch_replay_f32(const FNetDev &net, const uint8_t *clean, const int16_t *deltas, int m,
                             const CexRec *recs, int64_t n_recs, int32_t *labels, hipStream_t s) {
    if (n_recs <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_recs, 8192);
    hipLaunchKernelGGL(replay_f32_kernel, dim3(grid), dim3(256), 0, s, net, clean, deltas, m, recs, n_recs, labels);
    return hipGetLastError();
}

hipError_t launch_enum_f32(int grid, const FEnumParams &P, const int32_t *u0_index, hipStream_t s) {
    hipLaunchKernelGGL(enum_f32_kernel, dim3(grid), dim3(256), 0, s, P, u0_index);
    return hipGetLastError();
}

}  // namespace ibmc
