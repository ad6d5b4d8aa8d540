// Launch interface of the proposal-network kernels.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

constexpr int kPropF = 32;
constexpr int kPropH = 128;
constexpr int kPropParams = kPropH * kPropF + kPropH + kPropH + 1;   // W1, b1, w2, c (flat, in this order)

// Views into the flat fp32 parameter vector.
struct PropParams {
    const float *W1;   // [128][32]
    const float *b1;   // [128]
    const float *w2;   // [128]
    const float *c;    // [1]
};

struct PropGrads {
    float *gW1, *gb1, *gw2, *gc;
    float *loss;
};

// Candidate set of one image: the delta set and its largest magnitude.
struct PropCand {
    int m;
    int dmax;
    int16_t deltas[kMaxDeltas];
};

// Feature rows [n m][32] of one image's candidates.  u0: its clean
// first-layer potentials in sigma order (computed into u0_scratch, H[1]
// ints, when null); nl_scratch: n floats.
hipError_t launch_prop_features(const QNetDev &net, const uint8_t *image, const int32_t *u0, int rows, int cols,
                                const PropCand &pc, int32_t *u0_scratch, float *nl_scratch, float *feat,
                                hipStream_t s);
hipError_t launch_prop_score(const PropParams &P, const float *feat, int64_t N, float *scores, hipStream_t s);
// Scores of an image's candidates [n m] in one launch (live norms, features
// and the forward pass), from its clean first-layer potentials u0 (sigma
// order); equal to launch_prop_features then launch_prop_score.
// Clean first-layer potentials of one image, sigma order, H[1] ints.
hipError_t launch_prop_u0(const QNetDev &net, const uint8_t *image, int32_t *u0, hipStream_t s);
hipError_t launch_prop_fused(const QNetDev &net, const uint8_t *image, const int32_t *u0, int rows, int cols,
                             const PropCand &pc, const PropParams &P, float *scores, hipStream_t s);
hipError_t launch_prop_train(const PropParams &P, const float *feat, const float *labels, const int32_t *index,
                             int64_t begin, int64_t count, float inv_b, float pw, const PropGrads &G, int n_cu,
                             hipStream_t s);
hipError_t launch_prop_adam(float *theta, float *grad, float *mom, float *vel, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2, hipStream_t s);
int prop_sort_max();
hipError_t launch_prop_sort(const float *scores, int N, int32_t *order, hipStream_t s);
// Per candidate (p * m + i): 1 when it occurs in some record (count false),
// or the number of records it occurs in (count true); labels start at 0.
hipError_t launch_label_candidates(int n, int m, const CexRec *recs, int64_t nrec, float *labels, bool count,
                                  hipStream_t s);

}  // namespace ibmc
