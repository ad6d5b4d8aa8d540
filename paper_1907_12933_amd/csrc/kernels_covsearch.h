// Launch interface of the coverage-guided test generation kernels.
#pragma once

#include "kernels_cov.h"

namespace ibmc {

constexpr int kCovSearchMaxWords = 64;   // covered-pair bitset of a candidate: at most 4,096 pairs

struct CovCandParams {
    QNetDev net;                       // dense row-major layers (Wd, bd), shifts
    const uint8_t *image;              // the clean image (device)
    const int16_t *deltas;             // the delta set (device)
    int32_t m, k;
    const int32_t *pot0;               // the clean image's potentials, layers 1..L, natural order
    int64_t rank0, n_cand;             // candidates: ranks rank0 .. rank0 + n_cand - 1 of level k
    int32_t crit;                      // 0 SS, 1 DS, 2 SV, 3 DV
    int32_t words;                     // 64-bit words of a candidate's bitset
    CovParams cp;
    unsigned long long *masks;         // [n_cand][words]
    int32_t *labels;                   // [n_cand]
};

hipError_t launch_cov_cand(const CovCandParams &P, hipStream_t s);
hipError_t launch_cov_gain(const unsigned long long *masks, int64_t n_cand, int words,
                           const unsigned long long *covered, unsigned long long *best_key, hipStream_t s);
// ORs the winner's bits into `covered` and writes its label (-1: no winner).
hipError_t launch_cov_take(const unsigned long long *masks, int words, const unsigned long long *best_key,
                           unsigned long long *covered, const int32_t *labels, int32_t *label_out, hipStream_t s);

}  // namespace ibmc
