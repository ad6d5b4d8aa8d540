// Ordering of counterexample records on the device: records become 64-bit
// keys (property, k, rank packed by significance) with the label as payload,
// sorted by rocPRIM's radix sort over the key bits in use, then unpacked into
// the public record layout without leaving the device.
#include "kernels_sort.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace ibmc {

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

// Sentinels sit at the end of the sorted keys: one lane finds the first.
__global__ void count_valid_kernel(const uint64_t *keys, int64_t m, int64_t *count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t lo = 0, hi = m;  // first index holding a sentinel, in [0, m]
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] == ~0ull) hi = mid; else lo = mid + 1;
    }
    *count = lo;
}

__global__ void __launch_bounds__(256) key_to_rec_kernel(const uint64_t *keys, const uint32_t *vals, int64_t m,
                                                         int kshift, int pshift, CexRec *out) {
    const uint64_t rmask = (kshift >= 64) ? ~0ull : ((1ull << kshift) - 1ull);
    const uint64_t kmask = (1ull << (pshift - kshift)) - 1ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[i];
        if (key == ~0ull) continue;
        CexRec r;
        r.prop = (int32_t)(pshift >= 64 ? 0 : (key >> pshift));
        r.k = (int32_t)((key >> kshift) & kmask);
        r.rank = (int64_t)(key & rmask);
        r.label = (int32_t)vals[i];
        r.reserved = 0;
        out[i] = r;
    }
}

static int key_bits(int max_prop, int max_k, int64_t max_rank, int *kshift, int *pshift) {
    int rbits = 1;
    while (rbits < 63 && ((int64_t)1 << rbits) <= max_rank) ++rbits;
    int kb = 1;
    while ((1 << kb) <= max_k) ++kb;
    int pb = 1;
    while ((1 << pb) <= max_prop) ++pb;
    *kshift = rbits;
    *pshift = rbits + kb;
    return rbits + kb + pb;
}

static size_t radix_tmp_bytes(int64_t n) {
    size_t bytes = 0;
    rocprim::double_buffer<uint64_t> kb(nullptr, nullptr);
    rocprim::double_buffer<uint32_t> vb(nullptr, nullptr);
    (void)rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)std::max<int64_t>(n, 1), 0, 64, 0);
    return bytes;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t sort_scratch_bytes(int64_t n) {
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    return align256(nn * 8) * 2 + align256(nn * 4) * 2 + align256(radix_tmp_bytes(n)) + 256;
}

void sort_scratch_carve(void *p, int64_t n, SortScratch &S) {
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    char *b = (char *)p;
    S.k0 = (uint64_t *)b;
    b += align256(nn * 8);
    S.k1 = (uint64_t *)b;
    b += align256(nn * 8);
    S.v0 = (uint32_t *)b;
    b += align256(nn * 4);
    S.v1 = (uint32_t *)b;
    b += align256(nn * 4);
    S.count = (int64_t *)b;
    b += 256;
    S.tmp = b;
    S.tmp_bytes = radix_tmp_bytes(n);
}

ibmc_status_t sort_records_device(const DevRec *recs, int64_t n, int max_prop, int max_k, int64_t max_rank,
                                  SortScratch &S, hipStream_t s, int *key_bits_out) {
    int kshift = 0, pshift = 0;
    const int total = key_bits(max_prop, max_k, max_rank, &kshift, &pshift);
    *key_bits_out = total;
    if (total > 64 || n > 0xffffffffll) return SORT_UNSUPPORTED;
    S.kshift = kshift;
    S.pshift = pshift;
    S.keys_out = S.k0;
    S.vals_out = S.v0;
    if (n == 0) return SORT_OK;
    hipLaunchKernelGGL(rec_to_key_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                       recs, n, kshift, pshift, S.k0, S.v0);
    if (hipGetLastError() != hipSuccess) return SORT_HIP_ERROR;
    rocprim::double_buffer<uint64_t> kb(S.k0, S.k1);
    rocprim::double_buffer<uint32_t> vb(S.v0, S.v1);
    size_t bytes = S.tmp_bytes;
    if (rocprim::radix_sort_pairs(S.tmp, bytes, kb, vb, (size_t)n, 0, (unsigned)total, s) != hipSuccess)
        return SORT_HIP_ERROR;
    S.keys_out = kb.current();
    S.vals_out = vb.current();
    return SORT_OK;
}

hipError_t sorted_to_records(const SortScratch &S, int64_t m, CexRec *out, hipStream_t s) {
    hipLaunchKernelGGL(count_valid_kernel, dim3(1), dim3(64), 0, s, S.keys_out, m, S.count);
    if (m > 0)
        hipLaunchKernelGGL(key_to_rec_kernel, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 8192)), dim3(256), 0,
                           s, S.keys_out, S.vals_out, m, S.kshift, S.pshift, out);
    return hipGetLastError();
}

}  // namespace ibmc
