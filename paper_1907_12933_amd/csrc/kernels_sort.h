// Device ordering of counterexample records (stable LSD radix sort).
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

typedef int ibmc_status_t;
enum { SORT_OK = 0, SORT_UNSUPPORTED = 1, SORT_HIP_ERROR = 2 };

struct SortScratch {
    uint64_t *k0, *k1;
    uint32_t *v0, *v1;
    uint32_t *hist;
    uint64_t *keys_out;   // sorted keys (one of k0 / k1)
    uint32_t *vals_out;   // labels in key order
    int kshift, pshift;   // key = prop << pshift | k << kshift | rank
};

size_t sort_scratch_bytes(int64_t n);
void sort_scratch_carve(void *p, int64_t n, SortScratch &S);
// Sort n records by (prop, k, rank).  SORT_UNSUPPORTED when the packed key
// would need more than 64 bits (the caller then sorts on the host).
ibmc_status_t sort_records_device(const DevRec *recs, int64_t n, int max_prop, int max_k, int64_t max_rank,
                                  SortScratch &S, hipStream_t s, int *key_bits_out);

}  // namespace ibmc
