// Device ordering of counterexample records: records become 64-bit keys
// (property, level, rank packed by significance) with the label as payload,
// sorted by rocPRIM's radix sort, then written back in the public record
// layout on the device.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

typedef int ibmc_status_t;
enum { SORT_OK = 0, SORT_UNSUPPORTED = 1, SORT_HIP_ERROR = 2 };

struct SortScratch {
    uint64_t *k0, *k1;
    uint32_t *v0, *v1;
    void *tmp;            // radix sort temporary storage
    size_t tmp_bytes;
    int64_t *count;       // valid records among the sorted ones
    uint64_t *keys_out;   // sorted keys (one of k0 / k1)
    uint32_t *vals_out;   // labels in key order
    int kshift, pshift;   // key = prop << pshift | k << kshift | rank
};

size_t sort_scratch_bytes(int64_t n);
void sort_scratch_carve(void *p, int64_t n, SortScratch &S);
// Sort n records by (prop, k, rank); sentinels of unused slots (prop -1)
// sort last.  SORT_UNSUPPORTED when the packed key would need more than 64
// bits (the caller then sorts on the host).
ibmc_status_t sort_records_device(const DevRec *recs, int64_t n, int max_prop, int max_k, int64_t max_rank,
                                  SortScratch &S, hipStream_t s, int *key_bits_out);
// Count the valid records among the first m sorted keys into *S.count, and
// write them in the public layout (ibmc_cex) to out (device memory).
hipError_t sorted_to_records(const SortScratch &S, int64_t m, CexRec *out, hipStream_t s);

}  // namespace ibmc
