// Learned proposal network: candidate features, bf16 MFMA forward (scoring),
// fused forward/backward with the weight gradient on bf16 MFMA, Adam, the
// candidates' order by score (a stable counting rank over the whole chip),
// and candidate labels from counterexample records.
//
// Network: s = w2 . relu(W1 f + b1) + c with f in R^32, hidden 128.
// v_mfma_f32_16x16x32_bf16, orientation out[hidden x samples] = W1 x F^T:
// A = 16 hidden rows x 32 features (8 bf16 per lane), B = 32 features x 16
// samples; the accumulator leaves lane (j + 16 g) with hidden 4g..4g+3 of
// sample j.
#include "kernels_prop.h"

namespace ibmc {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }  // round to nearest even

// ---------------------------------------------------------------------------
// features: clean first-layer potentials (when not given), the live-weighted
// column norm of every pixel, then the candidates' feature rows
// ---------------------------------------------------------------------------

// Clean first-layer potentials of one image in sigma order: 64 neurons per
// workgroup, the inputs split over its four waves.
__global__ void __launch_bounds__(256) prop_u0_kernel(QNetDev net, const uint8_t *image, int32_t *u0) {
    __shared__ int part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = net.dims[0], H1 = net.H[1];
    const int q = blockIdx.x * 64 + lane;
    const int seg = (n + 3) / 4, i0 = wv * seg, i1 = min(n, i0 + seg);
    int u = 0;
    if (q < H1)
        for (int i = i0; i < i1; ++i) u += (int)net.W1T[(int64_t)i * H1 + q] * (int)image[i];
    part[wv][lane] = u;
    __syncthreads();
    if (wv == 0 && q < H1) u0[q] = net.b1s[q] + part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
}

// Sum of |W1[:, p]| over the neurons whose clean potential lies in the
// requantiser's linear window [0, 128 2^s): one wave per pixel.
__global__ void __launch_bounds__(256) prop_live_norm_kernel(QNetDev net, const int32_t *u0, float *nl) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int n = net.dims[0], H1 = net.H[1];
    if (p >= n) return;  // whole waves
    const int top = 128 << net.shift[0];
    int sl = 0;
    for (int q = lane; q < H1; q += 64) {
        const int u = u0[q];
        const int w = net.W1T[(int64_t)p * H1 + q];
        if (sigma64(q) < net.dims[1] && u >= 0 && u < top) sl += w < 0 ? -w : w;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sl += __shfl_xor(sl, off);
    if (lane == 0) nl[p] = (float)sl;
}

// The nine nonzero features of candidate (p, i): position, clean value,
// delta and its clamped effect, the full and L2 column norms over their
// maxima, the live part of the L1 norm on the full norm's scale, a constant.
__device__ __forceinline__ void cand_features(const QNetDev &net, const uint8_t *image, int rows, int cols,
                                              const PropCand &pc, int p, int i, float nlp, float (&f)[9]) {
    const int n = net.dims[0];
    const float M1 = net.pnorm[2 * n], M2 = net.pnorm[2 * n + 1];
    const float rden = rows > 1 ? (float)(rows - 1) : 1.f, cden = cols > 1 ? (float)(cols - 1) : 1.f;
    const float dmax = fmaxf((float)pc.dmax, 1.f);
    const int r = p / cols, c = p - r * cols;
    const int x = image[p];
    const int d = pc.deltas[i];
    const int e = min(max(x + d, 0), 255) - x;
    f[0] = (float)r / rden;
    f[1] = (float)c / cden;
    f[2] = (float)x / 255.f;
    f[3] = (float)d / dmax;
    f[4] = (float)e / dmax;
    f[5] = net.pnorm[p] / M1;
    f[6] = net.pnorm[n + p] / M2;
    f[7] = nlp / M1;
    f[8] = 1.f;
}

// Feature rows [n m][32] of the candidates (p, i) from the live norms nl.
__global__ void __launch_bounds__(256) prop_feat_kernel(QNetDev net, const uint8_t *image, int rows, int cols,
                                                        PropCand pc, const float *nl, float *feat) {
    const int n = net.dims[0], m = pc.m;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * m; t += gridDim.x * blockDim.x) {
        const int p = t / m, i = t - p * m;
        float fv[9];
        cand_features(net, image, rows, cols, pc, p, i, nl[p], fv);
        float *f = feat + (int64_t)t * 32;
#pragma unroll
        for (int z = 0; z < 9; ++z) f[z] = fv[z];
        for (int z = 9; z < 32; ++z) f[z] = 0.f;
    }
}

// ---------------------------------------------------------------------------
// forward scores
// ---------------------------------------------------------------------------

// Stage the bf16 copy of W1 in LDS as A operands: [8 tiles][64 lanes][8 bf16].
__device__ __forceinline__ void stage_w1(const PropParams &P, v8bf *wt) {
    for (int t = threadIdx.x; t < 8 * 64; t += blockDim.x) {
        const int mt = t / 64, ln = t % 64, r = ln & 15, g = ln >> 4;
        v8bf v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = to_bf16(P.W1[(mt * 16 + r) * 32 + g * 8 + e]);
        wt[t] = v;
    }
}

__device__ __forceinline__ v8bf load_feat_bf16(const float *f) {
    const float4 a = *reinterpret_cast<const float4 *>(f), b = *reinterpret_cast<const float4 *>(f + 4);
    v8bf v;
    v[0] = to_bf16(a.x); v[1] = to_bf16(a.y); v[2] = to_bf16(a.z); v[3] = to_bf16(a.w);
    v[4] = to_bf16(b.x); v[5] = to_bf16(b.y); v[6] = to_bf16(b.z); v[7] = to_bf16(b.w);
    return v;
}

__global__ void __launch_bounds__(256) prop_score_kernel(PropParams P, const float *feat, int64_t N, float *scores) {
    __shared__ v8bf wt[8 * 64];
    stage_w1(P, wt);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile * 16 < N; tile += waves) {
        const int64_t s = tile * 16 + j;
        v8bf B;
        if (s < N) B = load_feat_bf16(feat + s * 32 + g * 8);
        else for (int e = 0; e < 8; ++e) B[e] = to_bf16(0.f);
        float part = 0.f;
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[mt * 64 + lane], B, acc, 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int h = mt * 16 + g * 4 + t;
                part += P.w2[h] * fmaxf(acc[t] + P.b1[h], 0.f);
            }
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0 && s < N) scores[s] = part + P.c[0];
    }
}

// Live norms, features and scores of the candidates of 16 pixels per
// workgroup in one launch: each wave sums the live column norms of its
// pixels, then the candidates go through the same bf16 matrix-core forward
// as prop_score_kernel, their features built in registers (bf16 operands
// equal to those of the feature rows prop_feat_kernel writes).
constexpr int kFusedPix = 16;

__global__ void __launch_bounds__(256) prop_fused_kernel(QNetDev net, const uint8_t *image, int rows, int cols,
                                                         PropCand pc, const int32_t *u0, PropParams P, float *scores) {
    __shared__ v8bf wt[8 * 64];
    __shared__ float nls[kFusedPix];
    stage_w1(P, wt);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = net.dims[0], H1 = net.H[1], m = pc.m;
    const int p0 = blockIdx.x * kFusedPix;
    const int top = 128 << net.shift[0];
    for (int pp = wave; pp < kFusedPix; pp += 4) {
        const int p = p0 + pp;
        int sl = 0;
        if (p < n)
            for (int q = lane; q < H1; q += 64) {
                const int u = u0[q];
                const int w = net.W1T[(int64_t)p * H1 + q];
                if (sigma64(q) < net.dims[1] && u >= 0 && u < top) sl += w < 0 ? -w : w;
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sl += __shfl_xor(sl, off);
        if (lane == 0) nls[pp] = (float)sl;
    }
    __syncthreads();
    const int N = min(kFusedPix, n - p0) * m;
    const int j = lane & 15, g = lane >> 4;
    for (int tile = wave; tile * 16 < N; tile += 4) {
        const int t = tile * 16 + j;
        v8bf B;
#pragma unroll
        for (int e = 0; e < 8; ++e) B[e] = to_bf16(0.f);
        if (t < N && g < 2) {
            const int pl = t / m, i = t - pl * m;
            float fv[9];
            cand_features(net, image, rows, cols, pc, p0 + pl, i, nls[pl], fv);
#pragma unroll
            for (int e = 0; e < 8; ++e) B[e] = to_bf16(g * 8 + e < 9 ? fv[g * 8 + e] : 0.f);
        }
        float part = 0.f;
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[mt * 64 + lane], B, acc, 0, 0, 0);
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                const int h = mt * 16 + g * 4 + tt;
                part += P.w2[h] * fmaxf(acc[tt] + P.b1[h], 0.f);
            }
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0 && t < N) scores[(int64_t)p0 * m + t] = part + P.c[0];
    }
}

// ---------------------------------------------------------------------------
// fused forward / backward of one minibatch
// ---------------------------------------------------------------------------

// Each wave takes 32 samples (two 16-sample N-tiles) per iteration.  LDS per
// wave: gh^T as bf16 [128 hidden][32 samples] and the samples' features as
// bf16 [32][32]; then dW1 += GH^T F on MFMA (K = samples).
__global__ void __launch_bounds__(256) prop_train_kernel(PropParams P, const float *feat, const float *labels,
                                                         const int32_t *index, int64_t begin, int64_t count,
                                                         float inv_b, float pw, PropGrads G) {
    __shared__ v8bf wt[8 * 64];
    __shared__ __bf16 ghT[4][128][40];          // [wave][hidden][sample] (+8 pad)
    __shared__ __bf16 fs[4][32][40];            // [wave][sample][feature] (+8 pad)
    __shared__ float hval[4][128][33];          // relu(h) for dw2
    __shared__ float gsv[4][32];
    stage_w1(P, wt);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    v4f dW[8][2];
#pragma unroll
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 2; ++b) dW[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    float gb1_part[2] = {0.f, 0.f}, gw2_part[2] = {0.f, 0.f};  // hidden lane and lane + 64
    float gc_part = 0.f, loss_part = 0.f;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile * 32 < count; tile += waves) {
        // forward of 2 x 16 samples
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int64_t r = tile * 32 + nt * 16 + j;
            const bool ok = r < count;
            const int64_t s = ok ? (index ? index[begin + r] : begin + r) : 0;
            v8bf B;
            if (ok) B = load_feat_bf16(feat + s * 32 + g * 8);
            else for (int e = 0; e < 8; ++e) B[e] = to_bf16(0.f);
#pragma unroll
            for (int e = 0; e < 8; ++e) fs[wave][nt * 16 + j][g * 8 + e] = B[e];
            float part = 0.f;
            float hp[8][4];
#pragma unroll
            for (int mt = 0; mt < 8; ++mt) {
                v4f acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[mt * 64 + lane], B, acc, 0, 0, 0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int h = mt * 16 + g * 4 + t;
                    hp[mt][t] = acc[t] + P.b1[h];
                    const float hr = fmaxf(hp[mt][t], 0.f);
                    hval[wave][h][nt * 16 + j] = hr;
                    part += P.w2[h] * hr;
                }
            }
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            const float sc = part + P.c[0];
            const float y = ok ? labels[s] : 0.f;
            // loss = pw y softplus(-s) + (1 - y) softplus(s); d loss / d s = sig (pw y + 1 - y) - pw y
            const float sig = 1.f / (1.f + expf(-sc));
            const float sp_pos = sc > 0.f ? sc + log1pf(expf(-sc)) : log1pf(expf(sc));
            const float sp_neg = sp_pos - sc;
            const float gs = ok ? (sig * (pw * y + 1.f - y) - pw * y) * inv_b : 0.f;
            if (g == 0 && ok) {
                loss_part += (pw * y * sp_neg + (1.f - y) * sp_pos) * inv_b;
                gc_part += gs;
            }
            if (g == 0) gsv[wave][nt * 16 + j] = gs;
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int h = mt * 16 + g * 4 + t;
                    const float gh = hp[mt][t] > 0.f ? gs * P.w2[h] : 0.f;
                    ghT[wave][h][nt * 16 + j] = to_bf16(gh);
                }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // dW1 (128 x 32) += GH^T (128 x 32 samples) * F (32 samples x 32 features)
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            v8bf A;
#pragma unroll
            for (int e = 0; e < 8; ++e) A[e] = ghT[wave][mt * 16 + j][g * 8 + e];
#pragma unroll
            for (int ntf = 0; ntf < 2; ++ntf) {
                v8bf Bf;
#pragma unroll
                for (int e = 0; e < 8; ++e) Bf[e] = fs[wave][g * 8 + e][ntf * 16 + j];
                dW[mt][ntf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bf, dW[mt][ntf], 0, 0, 0);
            }
        }
        // gb1, gw2 (fp32 sums over the 32 samples; lane owns hidden lane and lane + 64)
#pragma unroll
        for (int z = 0; z < 2; ++z) {
            const int h = lane + 64 * z;
            float sb = 0.f, sw = 0.f;
            for (int q = 0; q < 32; ++q) {
                const float gsq = gsv[wave][q];
                const float hv = hval[wave][h][q];
                sw += gsq * hv;
                sb += hv > 0.f ? gsq * P.w2[h] : 0.f;
            }
            gb1_part[z] += sb;
            gw2_part[z] += sw;
        }
        __builtin_amdgcn_wave_barrier();
    }
    // flush: dW tile (mt, ntf): lane (j + 16 g) holds rows 16 mt + 4 g + t, column 16 ntf + j
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int ntf = 0; ntf < 2; ++ntf)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float v = dW[mt][ntf][t];
                if (v != 0.f) atomicAdd(G.gW1 + (mt * 16 + g * 4 + t) * 32 + ntf * 16 + j, v);
            }
#pragma unroll
    for (int z = 0; z < 2; ++z) {
        if (gb1_part[z] != 0.f) atomicAdd(G.gb1 + lane + 64 * z, gb1_part[z]);
        if (gw2_part[z] != 0.f) atomicAdd(G.gw2 + lane + 64 * z, gw2_part[z]);
    }
    for (int sh = 32; sh >= 1; sh >>= 1) {
        gc_part += __shfl_xor(gc_part, sh);
        loss_part += __shfl_xor(loss_part, sh);
    }
    if (lane == 0) {
        atomicAdd(G.gc, gc_part);
        atomicAdd(G.loss, loss_part);
    }
}

// Adam (Kingma & Ba) on the flat parameter vector; zeroes the gradients.
__global__ void __launch_bounds__(256) prop_adam_kernel(float *theta, float *grad, float *mom, float *vel, int n,
                                                        float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float g = grad[i];
        const float m = b1 * mom[i] + (1.f - b1) * g;
        const float v = b2 * vel[i] + (1.f - b2) * g * g;
        mom[i] = m;
        vel[i] = v;
        theta[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
        grad[i] = 0.f;
    }
}

// ---------------------------------------------------------------------------
// ordering: score descending, ties by candidate index
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned order_key(float s) {
    // monotone float -> uint map, then inverted so that larger scores come
    // first; the order keeps 16 bits (sign, exponent, 7 mantissa bits: the
    // precision of the network's bf16 products), ties go by candidate index
    const unsigned b = __float_as_uint(s);
    const unsigned u = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return (~u) >> 16;
}

// Stable ordering by counting: a candidate's place is the number of
// candidates whose (order key, index) pair is smaller.  The pair is packed as
// key << 14 | index (N <= 16384), so one unsigned compare decides it; every
// workgroup stages all packed keys in LDS (each thread's scores loaded
// kRankLoads at a time, all in flight together: they were just written
// through other XCDs' caches) and places 64 candidates, one per lane, its
// waves splitting the comparisons.  Padding keys (all ones) are larger than
// every packed pair and never counted.
constexpr int kRankWaves = 16;
constexpr int kRankLoads = 8;
constexpr int kRankMax = 16384;

__global__ void __launch_bounds__(64 * kRankWaves) prop_rank_kernel(const float *scores, int N, int32_t *order) {
    extern __shared__ __attribute__((aligned(16))) unsigned pk[];   // N rounded up to 4
    __shared__ int part[kRankWaves][64];
    const int Np = (N + 3) & ~3;
    for (int t0 = threadIdx.x; t0 < Np; t0 += blockDim.x * kRankLoads) {
        float sv[kRankLoads];
#pragma unroll
        for (int u = 0; u < kRankLoads; ++u) {
            const int t = t0 + u * (int)blockDim.x;
            sv[u] = t < N ? scores[t] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kRankLoads; ++u) {
            const int t = t0 + u * (int)blockDim.x;
            if (t < Np) pk[t] = t < N ? (order_key(sv[u]) << 14) | (unsigned)t : 0xffffffffu;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const unsigned ci = i < N ? pk[i] : 0u;
    const int q = Np / 4;
    const int per = (q + kRankWaves - 1) / kRankWaves;
    const int q0 = wave * per, q1 = min(q, q0 + per);
    const uint4 *p4 = reinterpret_cast<const uint4 *>(pk);
    int cnt = 0;
#pragma unroll 4
    for (int j = q0; j < q1; ++j) {
        const uint4 v = p4[j];
        cnt += (v.x < ci) + (v.y < ci) + (v.z < ci) + (v.w < ci);
    }
    part[wave][lane] = cnt;
    __syncthreads();
    if (wave == 0 && i < N) {
        int r = 0;
#pragma unroll
        for (int w = 0; w < kRankWaves; ++w) r += part[w][lane];
        order[r] = i;
    }
}

// ---------------------------------------------------------------------------
// candidate labels: every (pixel, delta) that occurs in a counterexample
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) label_candidates_kernel(int n, int m, const CexRec *recs, int64_t nrec,
                                                               float *labels, int count) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrec;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int k = recs[r].k;
        if (k < 1 || k > kMaxK) continue;
        int64_t mk = 1;
        for (int j = 0; j < k; ++j) mk *= m;
        int p[kMaxK];
        lex_unrank_subset(recs[r].rank / mk, k, n, p);
        int64_t d = recs[r].rank % mk;
        for (int j = k - 1; j >= 0; --j) {
            float *slot = labels + (int64_t)p[j] * m + (int)(d % m);
            if (count) atomicAdd(slot, 1.f);   // exact while a count stays below 2^24
            else *slot = 1.f;
            d /= m;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_prop_features(const QNetDev &net, const uint8_t *image, const int32_t *u0, int rows, int cols,
                                const PropCand &pc, int32_t *u0_scratch, float *nl_scratch, float *feat,
                                hipStream_t s) {
    const int n = net.dims[0];
    if (!u0) {
        hipLaunchKernelGGL(prop_u0_kernel, dim3((net.H[1] + 63) / 64), dim3(256), 0, s, net, image, u0_scratch);
        u0 = u0_scratch;
    }
    hipLaunchKernelGGL(prop_live_norm_kernel, dim3((n + 3) / 4), dim3(256), 0, s, net, u0, nl_scratch);
    const int grid = (int)std::min<int64_t>(((int64_t)n * pc.m + 255) / 256, 1024);
    hipLaunchKernelGGL(prop_feat_kernel, dim3(grid), dim3(256), 0, s, net, image, rows, cols, pc, nl_scratch, feat);
    return hipGetLastError();
}

hipError_t launch_prop_u0(const QNetDev &net, const uint8_t *image, int32_t *u0, hipStream_t s) {
    hipLaunchKernelGGL(prop_u0_kernel, dim3((net.H[1] + 63) / 64), dim3(256), 0, s, net, image, u0);
    return hipGetLastError();
}

hipError_t launch_prop_fused(const QNetDev &net, const uint8_t *image, const int32_t *u0, int rows, int cols,
                             const PropCand &pc, const PropParams &P, float *scores, hipStream_t s) {
    const int n = net.dims[0];
    hipLaunchKernelGGL(prop_fused_kernel, dim3((n + kFusedPix - 1) / kFusedPix), dim3(256), 0, s, net, image, rows,
                       cols, pc, u0, P, scores);
    return hipGetLastError();
}

hipError_t launch_prop_score(const PropParams &P, const float *feat, int64_t N, float *scores, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((N + 63) / 64, 2048);
    hipLaunchKernelGGL(prop_score_kernel, dim3(grid), dim3(256), 0, s, P, feat, N, scores);
    return hipGetLastError();
}

hipError_t launch_prop_train(const PropParams &P, const float *feat, const float *labels, const int32_t *index,
                             int64_t begin, int64_t count, float inv_b, float pw, const PropGrads &G, int n_cu,
                             hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((count + 127) / 128, (int64_t)n_cu * 2);
    hipLaunchKernelGGL(prop_train_kernel, dim3(grid), dim3(256), 0, s, P, feat, labels, index, begin, count, inv_b,
                       pw, G);
    return hipGetLastError();
}

hipError_t launch_prop_adam(float *theta, float *grad, float *mom, float *vel, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(prop_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, theta, grad, mom, vel, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

int prop_sort_max() { return kRankMax; }

hipError_t launch_prop_sort(const float *scores, int N, int32_t *order, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (N > kRankMax) return hipErrorInvalidValue;
    const size_t lds = (size_t)((N + 3) & ~3) * 4;
    hipLaunchKernelGGL(prop_rank_kernel, dim3((N + 63) / 64), dim3(64 * kRankWaves), lds, s, scores, N, order);
    return hipGetLastError();
}

hipError_t launch_label_candidates(int n, int m, const CexRec *recs, int64_t nrec, float *labels, bool count,
                                  hipStream_t s) {
    if (nrec <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((nrec + 255) / 256, 4096);
    hipLaunchKernelGGL(label_candidates_kernel, dim3(grid), dim3(256), 0, s, n, m, recs, nrec, labels, count ? 1 : 0);
    return hipGetLastError();
}

}  // namespace ibmc
