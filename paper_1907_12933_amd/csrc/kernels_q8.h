// Launch interface of the integer-network kernels (host side of the library).
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

// One compiled instance of the enumeration kernel.
struct EnumVariant {
    int L, kb1, kb2, nt;
    bool wlds;
    int epi;           // 3-layer nets: 1 = fast hidden epilogue (QNetDev::fast2 != 0), else 0
    bool out16;        // at most 16 classes (one output M-tile); else any number
    int chunk;         // points per chunk (16 * nt)
    const char *name;
    const void *fn;
};

const EnumVariant *enum_variants(int *count);
const EnumVariant *enum_variants_l2(int *count);
const EnumVariant *enum_variants_l3a(int *count);
const EnumVariant *enum_variants_l3b(int *count);
const EnumVariant *enum_variants_l3a_fast(int *count);
const EnumVariant *enum_variants_l3b_fast(int *count);
const EnumVariant *enum_variants_general(int *count);
int64_t enum_lds_bytes(const EnumVariant &v, const QNetDev &net);


hipError_t launch_forward_q8(const QNetDev &net, const uint8_t *images, int64_t n_images,
                             int32_t *labels, int32_t *pots, int64_t pot_stride, hipStream_t s);
hipError_t launch_clean_q8(const QNetDev &net, PropDev *props, const int32_t *prop_ids,
                           int32_t n_ids, int32_t *u0_store, int64_t u0_stride, hipStream_t s);
hipError_t launch_replay_q8(const QNetDev &net, const uint8_t *clean, const int16_t *deltas, int m,
                            const CexRec *recs, int64_t n_recs, int32_t *labels, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_enum_q8(const EnumVariant &v, int grid, const EnumParams &P,
                          const int32_t *u0_store, int64_t u0_stride, const int32_t *u0_index,
                          hipStream_t s);

}  // namespace ibmc
