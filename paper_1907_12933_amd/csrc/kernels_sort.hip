// Ordering of counterexample records on the device: records become 64-bit
// keys (property, k, rank packed by significance) with the label as payload,
// sorted by a stable LSD radix sort with 8-bit digits (histogram, scan,
// scatter with wave-ballot ranking), then copied back as keys + labels.
#include "kernels_sort.h"

namespace ibmc {

constexpr int kRsThreads = 256;
constexpr int kRsChunks = 16;                       // 256-key chunks per block tile
constexpr int kRsTile = kRsThreads * kRsChunks;     // 4096 keys per block

__global__ void __launch_bounds__(256) rec_to_key_kernel(const DevRec *recs, int64_t n, int kshift, int pshift,
                                                         uint64_t *keys, uint32_t *vals) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const DevRec r = recs[i];
        const uint64_t k = (uint32_t)r.klab >> 24;
        // sentinels of unused record slots (prop -1) sort last
        keys[i] = r.prop < 0 ? ~0ull : ((uint64_t)r.prop << pshift) | (k << kshift) | (uint64_t)r.rank;
        vals[i] = (uint32_t)r.klab & 0xffffffu;
    }
}

__global__ void __launch_bounds__(256) rs_hist_kernel(const uint64_t *keys, int64_t n, int shift, uint32_t *hist,
                                                      int nblocks) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int c = 0; c < kRsChunks; ++c) {
        const int64_t i = base + c * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xff], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of hist (bin-major, block-minor) in place; one workgroup.
__global__ void __launch_bounds__(1024) rs_scan_kernel(uint32_t *hist, int64_t len) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (len + 1023) / 1024;
    const int64_t b = t * per, e = min(len, b + per);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        const uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(256) rs_scatter_kernel(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                         uint32_t *vout, int64_t n, int shift, const uint32_t *offsets,
                                                         int nblocks) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    base[t] = offsets[(int64_t)t * nblocks + blockIdx.x];
    const int64_t tile = (int64_t)blockIdx.x * kRsTile;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int c = 0; c < kRsChunks; ++c) {
        for (int z = 0; z < 4; ++z) wcnt[w][lane + 64 * z] = 0;
        __syncthreads();
        const int64_t i = tile + c * kRsThreads + t;
        const bool ok = i < n;
        const uint64_t key = ok ? kin[i] : 0;
        const int d = (int)((key >> shift) & 0xff);
        // lanes of this wave holding the same digit
        unsigned long long same = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bm = __ballot(ok && ((d >> bit) & 1));
            same &= ((d >> bit) & 1) ? bm : ~bm;
        }
        const int rank = __popcll(same & below);
        if (ok && (same >> lane) == 1ull) wcnt[w][d] = (uint32_t)__popcll(same);   // last lane of its digit
        __syncthreads();
        if (ok) {
            uint32_t pos = base[d] + rank;
            for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        __syncthreads();
    }
}

ibmc_status_t sort_records_device(const DevRec *recs, int64_t n, int max_prop, int max_k, int64_t max_rank,
                                  SortScratch &S, hipStream_t s, int *key_bits_out) {
    int rbits = 1;
    while (rbits < 63 && ((int64_t)1 << rbits) <= max_rank) ++rbits;
    int kb = 1;
    while ((1 << kb) <= max_k) ++kb;
    int pb = 1;
    while ((1 << pb) <= max_prop) ++pb;
    const int total = rbits + kb + pb;
    *key_bits_out = total;
    if (total > 64 || n > 0xffffffffll) return SORT_UNSUPPORTED;
    if (n == 0) return SORT_OK;
    const int kshift = rbits, pshift = rbits + kb;
    hipLaunchKernelGGL(rec_to_key_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                       recs, n, kshift, pshift, S.k0, S.v0);
    if (hipGetLastError() != hipSuccess) return SORT_HIP_ERROR;
    const int nblocks = (int)((n + kRsTile - 1) / kRsTile);
    uint64_t *ka = S.k0, *kb_ = S.k1;
    uint32_t *va = S.v0, *vb = S.v1;
    for (int shift = 0; shift < total; shift += 8) {
        hipLaunchKernelGGL(rs_hist_kernel, dim3(nblocks), dim3(256), 0, s, ka, n, shift, S.hist, nblocks);
        hipLaunchKernelGGL(rs_scan_kernel, dim3(1), dim3(1024), 0, s, S.hist, (int64_t)256 * nblocks);
        hipLaunchKernelGGL(rs_scatter_kernel, dim3(nblocks), dim3(256), 0, s, ka, va, kb_, vb, n, shift, S.hist,
                           nblocks);
        if (hipGetLastError() != hipSuccess) return SORT_HIP_ERROR;
        std::swap(ka, kb_);
        std::swap(va, vb);
    }
    S.keys_out = ka;
    S.vals_out = va;
    S.kshift = kshift;
    S.pshift = pshift;
    return SORT_OK;
}

size_t sort_scratch_bytes(int64_t n) {
    const int64_t nblocks = (n + kRsTile - 1) / kRsTile;
    return (size_t)n * (8 + 8 + 4 + 4) + (size_t)(256 * std::max<int64_t>(nblocks, 1)) * 4 + 1024;
}

void sort_scratch_carve(void *p, int64_t n, SortScratch &S) {
    char *b = (char *)p;
    S.k0 = (uint64_t *)b;
    S.k1 = S.k0 + n;
    S.v0 = (uint32_t *)(S.k1 + n);
    S.v1 = S.v0 + n;
    S.hist = (uint32_t *)(((uintptr_t)(S.v1 + n) + 255) & ~(uintptr_t)255);
}

}  // namespace ibmc
