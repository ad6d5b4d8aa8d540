// Integer-network kernels for gfx950: plain dense forward (clean pass,
// replay, forward), and the exhaustive enumeration of the bounded
// perturbation domain with incremental first layer and int8 MFMA later layers.
#include <vector>

#include "kernels_q8.h"
#include "enum_common.h"

namespace ibmc {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int requant_relu(int u, int s) {
    // floor(u / 2^s) (arithmetic shift), then clamp to [0, 127]
    return min(max(u >> s, 0), 127);
}

__device__ __forceinline__ int pack4(int a0, int a1, int a2, int a3) {
    return a0 | (a1 << 8) | (a2 << 16) | (a3 << 24);
}


// ---------------------------------------------------------------------------
// plain dense forward of one image held in LDS (one workgroup of kFwdThreads)
// ---------------------------------------------------------------------------

constexpr int kFwdThreads = 1024;
constexpr int kFwdSplit = 4;  // every dot product is split over this many threads

__device__ void dense_tail_block(const QNetDev &net, int *act0, int *act1, int (*part)[kMaxWidth], int32_t *pot,
                                 int *label_out, int *tie_out);

// xs: n pixel values; act0/act1: scratch of kMaxWidth ints each; part:
// kFwdSplit x kMaxWidth ints of partial sums.  Every layer's dot products are
// split over the inputs (short dependent chains, coalesced weight reads).
// The transposed first layer is read four neurons per 32-bit load, its
// inputs split as many ways as the partial sums allow (16 for up to 256
// neurons); the row-major later layers are read 16 weights per load when a
// row is a multiple of 16 bytes, split kFwdSplit ways over the row.
// Writes potentials (natural order, layers concatenated) if pot != nullptr,
// layer-1 potentials in sigma order if u0s != nullptr; returns the label
// (thread 0 holds the valid value) and the exact-tie flag.
__device__ void dense_forward_block(const QNetDev &net, const int *xs, int *act0, int *act1,
                                    int (*part)[kMaxWidth], int32_t *pot, int32_t *u0s, int *label_out,
                                    int *tie_out) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n = net.dims[0], H1 = net.H[1];
    int *const pf = &part[0][0];                     // [S1][H1] for the first layer
    // layer 1 through the transposed first layer, sigma order
    const int G1 = H1 / 4;                           // groups of four neurons
    const int S1 = max(1, min(16, kFwdSplit * kMaxWidth / H1));
    const int seg1 = (n + S1 - 1) / S1;
    for (int t = tid; t < G1 * S1; t += nthr) {
        const int grp = t % G1, sp = t / G1;
        const int i0 = sp * seg1, i1 = min(n, i0 + seg1);
        const int *w4 = reinterpret_cast<const int *>(net.W1T) + grp;   // row stride H1 / 4 words
        int u0 = 0, u1 = 0, u2 = 0, u3 = 0;
#pragma unroll 8
        for (int i = i0; i < i1; ++i) {
            const int w = w4[(int64_t)i * G1];
            const int x = xs[i];
            u0 += (int)(int8_t)w * x;
            u1 += (int)(int8_t)(w >> 8) * x;
            u2 += (int)(int8_t)(w >> 16) * x;
            u3 += (w >> 24) * x;
        }
        int *dst = pf + sp * H1 + 4 * grp;
        dst[0] = u0;
        dst[1] = u1;
        dst[2] = u2;
        dst[3] = u3;
    }
    __syncthreads();
    for (int q = tid; q < H1; q += nthr) {
        int u = net.b1s[q];
        for (int sp = 0; sp < S1; ++sp) u += pf[sp * H1 + q];
        const int neuron = sigma64(q);
        if (u0s) u0s[q] = u;
        if (neuron < net.dims[1]) {
            if (pot) pot[neuron] = u;
            act0[neuron] = (net.L > 1) ? requant_relu(u, net.shift[0]) : u;
        }
    }
    __syncthreads();
    dense_tail_block(net, act0, act1, part, pot, label_out, tie_out);
}

// Layers 2..L and the label of one image whose first-layer activations
// (natural order, requantised unless the net has one layer) are in act0.
// act1 and part are scratch as above; pot as above (layers >= 2).
__device__ void dense_tail_block(const QNetDev &net, int *act0, int *act1, int (*part)[kMaxWidth], int32_t *pot,
                                 int *label_out, int *tie_out) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    int *in = act0, *out = act1;
    int po = net.dims[1];
    for (int l = 2; l <= net.L; ++l) {
        const int nin = net.dims[l - 1], nout = net.dims[l];
        const int8_t *W = net.Wd[l];
        const bool wide = (nin % 16) == 0 && (reinterpret_cast<uintptr_t>(W) % 16) == 0;
        // every dot product split sp ways, as many as the block's threads
        // allow (one task each where possible: the loads of a task are issued
        // together, so a layer costs about one memory round trip), at most
        // one 16-weight load per split point and within the partial sums
        const int units = wide ? nin / 16 : nin;
        const int split = max(1, min(min(nthr / nout, units), kFwdSplit * kMaxWidth / nout));
        // split points on 16-weight boundaries when the rows are read 16 at a time
        const int seg = wide ? (units + split - 1) / split * 16 : (nin + split - 1) / split;
        int *const pf = &part[0][0];                     // [split][nout]
        for (int t = tid; t < nout * split; t += nthr) {
            const int j = t / split, sp = t % split;
            const int i0 = sp * seg, i1 = min(nin, i0 + seg);
            const int8_t *row = W + (int64_t)j * nin;
            int u = 0;
            if (wide) {
#pragma unroll 4
                for (int i = i0; i < i1; i += 16) {
                    const int4 w = *reinterpret_cast<const int4 *>(row + i);
                    const int ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        u += (int)(int8_t)ww[c] * in[i + 4 * c] + (int)(int8_t)(ww[c] >> 8) * in[i + 4 * c + 1] +
                             (int)(int8_t)(ww[c] >> 16) * in[i + 4 * c + 2] + (ww[c] >> 24) * in[i + 4 * c + 3];
                    }
                }
            } else {
#pragma unroll 8
                for (int i = i0; i < i1; ++i) u += (int)row[i] * in[i];
            }
            pf[sp * nout + j] = u;
        }
        __syncthreads();
        for (int j = tid; j < nout; j += nthr) {
            int u = net.bd[l][j];
            for (int sp = 0; sp < split; ++sp) u += pf[sp * nout + j];
            if (pot) pot[po + j] = u;
            out[j] = (l < net.L) ? requant_relu(u, net.shift[l - 1]) : u;
        }
        po += nout;
        __syncthreads();
        int *t = in; in = out; out = t;
    }
    if (tid == 0) {
        const int nc = net.dims[net.L];
        int best = 0;
        for (int j = 1; j < nc; ++j) if (in[j] > in[best]) best = j;
        int cnt = 0;
        for (int j = 0; j < nc; ++j) cnt += in[j] == in[best];
        *label_out = best;
        *tie_out = cnt > 1;
    }
}

__global__ void __launch_bounds__(kFwdThreads) forward_q8_kernel(QNetDev net, const uint8_t *images,
                                                                 int64_t n_images, int32_t *labels,
                                                                 int32_t *pots, int64_t pot_stride) {
    __shared__ int xs[kMaxWidth];
    __shared__ int a0[kMaxWidth], a1[kMaxWidth];
    __shared__ int part[kFwdSplit][kMaxWidth];
    __shared__ int lab, tie;
    for (int64_t img = blockIdx.x; img < n_images; img += gridDim.x) {
        const uint8_t *x = images + img * net.dims[0];
        for (int i = threadIdx.x; i < net.dims[0]; i += blockDim.x) xs[i] = x[i];
        __syncthreads();
        dense_forward_block(net, xs, a0, a1, part, pots ? pots + img * pot_stride : nullptr, nullptr, &lab, &tie);
        __syncthreads();
        if (threadIdx.x == 0 && labels) labels[img] = lab;
        __syncthreads();
    }
}

// Clean pass of the properties listed in prop_ids: first-layer potentials in
// sigma order (the base of every incremental update, stored at the property's
// index) and the clean label.  Block b of the grid takes property
// prop_ids[b / S] and the first-layer neurons of slice b % S (S = H1 /
// clean_slice(H1)) over all pixels; the last of a property's S blocks to
// finish (counted in its clean_done, which starts at a multiple of S) runs
// the later layers from the stored potentials and writes the label.  One
// property thus spreads over S compute units instead of one.
__host__ __device__ inline int clean_slice(int H1) { return H1 % 64 == 0 ? 64 : 16; }
constexpr int kCleanThreads = 1024;
// a slice's partial sums, segs x slice = 4 kCleanThreads ints, fit in part
static_assert(4 * kCleanThreads <= kFwdSplit * kMaxWidth, "clean pass partial sums");

__global__ void __launch_bounds__(kCleanThreads) clean_q8_kernel(QNetDev net, PropDev *props,
                                                                 const int32_t *prop_ids, int32_t n_ids,
                                                                 int32_t *u0_store, int64_t u0_stride) {
    __shared__ int a0[kMaxWidth], a1[kMaxWidth];
    __shared__ int part[kFwdSplit][kMaxWidth];
    __shared__ int lab, tie, last;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n = net.dims[0], H1 = net.H[1];
    const int slice = clean_slice(H1), S = H1 / slice;
    const int G = slice / 4;                             // four neurons per 32-bit weight word
    const int segs = nthr / G;                           // pixel segments (segs * slice <= 4 kMaxWidth)
    const int G1 = H1 / 4;
    for (int64_t b = blockIdx.x; b < (int64_t)n_ids * S; b += gridDim.x) {
        const int pid = prop_ids[b / S];
        const int w = (int)(b % S);
        const uint8_t *x = props[pid].image;
        int32_t *u0s = u0_store + (int64_t)pid * u0_stride;
        // partial sums of the slice over this thread's pixel segment
        const int grp = tid % G, sg = tid / G;
        const int seg = (n + segs - 1) / segs;
        const int i0 = sg * seg, i1 = min(n, i0 + seg);
        const int *w4 = reinterpret_cast<const int *>(net.W1T) + w * G + grp;   // row stride G1 words
        int u0 = 0, u1 = 0, u2 = 0, u3 = 0;
#pragma unroll 8
        for (int i = i0; i < i1; ++i) {
            const int wv = w4[(int64_t)i * G1];
            const int xv = x[i];
            u0 += (int)(int8_t)wv * xv;
            u1 += (int)(int8_t)(wv >> 8) * xv;
            u2 += (int)(int8_t)(wv >> 16) * xv;
            u3 += (wv >> 24) * xv;
        }
        int *pf = &part[0][0];                            // [segs][slice]
        pf[sg * slice + 4 * grp + 0] = u0;
        pf[sg * slice + 4 * grp + 1] = u1;
        pf[sg * slice + 4 * grp + 2] = u2;
        pf[sg * slice + 4 * grp + 3] = u3;
        __syncthreads();
        if (tid < slice) {
            const int q = w * slice + tid;
            int u = net.b1s[q];
            for (int t = 0; t < segs; ++t) u += pf[t * slice + tid];
            u0s[q] = u;
        }
        // publish the slice, then count it (release); the block that
        // completes the count sees every slice (acquire)
        __threadfence();
        __syncthreads();
        if (tid == 0) last = (atomicAdd(&props[pid].clean_done, 1) + 1) % S == 0;
        __syncthreads();
        if (last) {
            __threadfence();
            for (int q = tid; q < H1; q += nthr) {
                const int neuron = sigma64(q);
                if (neuron < net.dims[1]) {
                    const int u = u0s[q];
                    a0[neuron] = (net.L > 1) ? requant_relu(u, net.shift[0]) : u;
                }
            }
            __syncthreads();
            dense_tail_block(net, a0, a1, part, nullptr, &lab, &tie);
            __syncthreads();
            if (tid == 0) { props[pid].label0 = lab; props[pid].tie0 = tie; }
        }
        __syncthreads();
    }
}

// Replay: rebuild each perturbed image from its record and run the plain
// forward pass.
__global__ void __launch_bounds__(kFwdThreads) replay_q8_kernel(QNetDev net, const uint8_t *clean,
                                                                const int16_t *deltas, int m,
                                                                const CexRec *recs, int64_t n_recs,
                                                                int32_t *labels) {
    __shared__ int xs[kMaxWidth];
    __shared__ int a0[kMaxWidth], a1[kMaxWidth];
    __shared__ int part[kFwdSplit][kMaxWidth];
    __shared__ int lab, tie;
    __shared__ int pix[kMaxK], dig[kMaxK];
    const int n = net.dims[0];
    for (int64_t r = blockIdx.x; r < n_recs; r += gridDim.x) {
        const int k = recs[r].k;
        if (threadIdx.x == 0) {
            int64_t mk = 1;
            for (int j = 0; j < k; ++j) mk *= m;
            int64_t srank = recs[r].rank / mk, drank = recs[r].rank % mk;
            int p[kMaxK];
            lex_unrank_subset(srank, k, n, p);
            for (int j = k - 1; j >= 0; --j) { dig[j] = (int)(drank % m); drank /= m; }
            for (int j = 0; j < k; ++j) pix[j] = p[j];
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = clean[i];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int j = 0; j < k; ++j) xs[pix[j]] = clamp_pixel(xs[pix[j]] + deltas[dig[j]]);
        __syncthreads();
        dense_forward_block(net, xs, a0, a1, part, nullptr, nullptr, &lab, &tie);
        __syncthreads();
        if (threadIdx.x == 0) labels[r] = lab;
        __syncthreads();
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// enumeration
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// instantiation table (the instances live in enum_q8_*.hip, compiled in parallel)
// ---------------------------------------------------------------------------

const EnumVariant *enum_variants(int *count) {
    static std::vector<EnumVariant> all;
    if (all.empty()) {
        int n = 0;
        const EnumVariant *v = enum_variants_l2(&n);
        all.insert(all.end(), v, v + n);
        v = enum_variants_l3a(&n);
        all.insert(all.end(), v, v + n);
        v = enum_variants_l3b(&n);
        all.insert(all.end(), v, v + n);
        v = enum_variants_l3a_fast(&n);
        all.insert(all.end(), v, v + n);
        v = enum_variants_l3b_fast(&n);
        all.insert(all.end(), v, v + n);
        v = enum_variants_general(&n);
        all.insert(all.end(), v, v + n);
    }
    *count = (int)all.size();
    return all.data();
}

// ---------------------------------------------------------------------------
// host launch wrappers
// ---------------------------------------------------------------------------

hipError_t launch_forward_q8(const QNetDev &net, const uint8_t *images, int64_t n_images,
                             int32_t *labels, int32_t *pots, int64_t pot_stride, hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_images, 4096);
    hipLaunchKernelGGL(forward_q8_kernel, dim3(grid), dim3(kFwdThreads), 0, s, net, images, n_images,
                       labels, pots, pot_stride);
    return hipGetLastError();
}

hipError_t launch_clean_q8(const QNetDev &net, PropDev *props, const int32_t *prop_ids,
                           int32_t n_ids, int32_t *u0_store, int64_t u0_stride, hipStream_t s) {
    if (n_ids <= 0) return hipSuccess;
    if (net.H[1] % 16) return hipErrorInvalidValue;
    const int grid = (int)std::min<int64_t>((int64_t)n_ids * (net.H[1] / clean_slice(net.H[1])), 8192);
    hipLaunchKernelGGL(clean_q8_kernel, dim3(grid), dim3(kCleanThreads), 0, s, net, props, prop_ids, n_ids,
                       u0_store, u0_stride);
    return hipGetLastError();
}

hipError_t launch_replay_q8(const QNetDev &net, const uint8_t *clean, const int16_t *deltas, int m,
                            const CexRec *recs, int64_t n_recs, int32_t *labels, hipStream_t s) {
    if (n_recs <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_recs, 8192);
    hipLaunchKernelGGL(replay_q8_kernel, dim3(grid), dim3(kFwdThreads), 0, s, net, clean, deltas, m, recs,
                       n_recs, labels);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

int64_t enum_lds_bytes(const EnumVariant &v, const QNetDev &net) {
    int64_t w = 0;
    if (v.wlds) {
        if (v.L == 3) w += (int64_t)(net.H[2] / 16) * v.kb1 * 1024;
        const int kbl = (v.L == 3) ? v.kb2 : v.kb1;
        w += (int64_t)(net.H[v.L] / 16) * kbl * 1024;
    }
    const int64_t biases = 4LL * ((v.L == 3 ? (int64_t)v.kb2 * 64 : 0) + net.H[v.L]);
    // per wave (4 per workgroup): one int32 or kSegGroup int16 first-layer
    // bases, and the cursor record
    const int64_t h1 = (int64_t)v.kb1 * 64;
    return w + biases + 4LL * std::max<int64_t>(h1 * 4, (int64_t)kSegGroup * h1 * 2) + 4LL * (int64_t)sizeof(Cursor);
}

hipError_t launch_enum_q8(const EnumVariant &v, int grid, const EnumParams &P,
                          const int32_t *u0_store, int64_t u0_stride, const int32_t *u0_index,
                          hipStream_t s) {
    const int64_t lds = enum_lds_bytes(v, P.net);
    EnumParams Q = P;
    Q.notify = (P.stop_on_first || P.track_first || P.hit_host) ? 1 : 0;
    void *args[] = {&Q, &u0_store, &u0_stride, &u0_index};
    return hipLaunchKernel(v.fn, dim3(grid), dim3(256), args, (size_t)lds, s);
}

}  // namespace ibmc
