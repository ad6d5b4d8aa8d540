// Launch interface of the coverage kernels and of the batched MFMA forward.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

// Extra layout of an integer network for the batched forward: natural-K
// A-operand tiles of layers >= 2 and every layer's accumulator init.
struct FwdExtra {
    int K0;                            // pixels padded to a multiple of 64
    const int8_t *Wn[kMaxLayers + 1];  // l >= 2: [H_l/16][H_{l-1}/64][64][16], natural K
    const int32_t *init[kMaxLayers + 1]; // l >= 1: bias + input-offset fold (+ requant offset), padded
};

// Shapes of the coverage bitmasks.  Layers here are the non-input layers
// (l = 0 .. nl-1); block l pairs layer l (rows i) with layer l+1 (bits j).
struct CovLayout {
    int nl;
    int U;                             // sum of widths
    int width[kMaxLayers];
    int uoff[kMaxLayers];              // offset of layer l in a potential vector
    int words[kMaxLayers];             // ceil(width / 32)
    int64_t rowoff[kMaxLayers];        // block l in the per-row masks (width[l] rows of words[l+1])
    int alloff[kMaxLayers];            // block l in the all-rows / column masks (words[l+1])
    int64_t pairoff[kMaxLayers];       // block l in the caller's packed layout
    int64_t total_pairs;
    int64_t rows_words;                // size of one per-row mask array
    int all_words;                     // size of one all-rows mask array
};

struct CovParams {
    int64_t dist_sq_min;
    int32_t ratio_num, ratio_den;
};

struct CovBits {
    uint32_t *rows_ss, *rows_sv;       // per-row masks (SS, SV)
    uint32_t *all_ds, *all_dv;         // all-rows masks (DS, DV)
};

struct CovSums {
    unsigned long long *pairs;         // [4] covered pairs (SS, DS, SV, DV)
    unsigned long long *neurons;       // [4] covered neurons
    uint8_t *condflag;                 // [4][flag_stride]
    int64_t flag_stride;
    uint32_t *colmask;                 // [4][colmask_stride]
    int64_t colmask_stride;
};

// One pass over input pairs: forward of both images on int8 MFMA (x2's first
// layer as the rank-r update of x1's), the per-neuron tests and the covered
// rows, with no potentials in memory.  x1 / x2: device [n_pairs][dims[0]].
struct CovPairParams {
    QNetDev net;
    FwdExtra fx;
    CovLayout lay;
    CovParams cp;
    CovBits bits;
    const uint8_t *x1, *x2;
    int64_t n_pairs;
    // LDS plan (cov_pair_plan): activation row stride, per-pair nibble
    // offsets of each layer, byte offsets of the regions
    int act_stride, nib_stride, off_nib, off_dist, off_diff, off_all;
    int nib_off[kMaxLayers + 2];
};

hipError_t launch_cov_pair(CovPairParams P, int n_cu, hipStream_t s);

hipError_t launch_fwd_pots_q8(const QNetDev &net, const FwdExtra &fx, const uint8_t *images, int64_t n_images,
                              int32_t *pots, int64_t pot_stride, int32_t *labels, hipStream_t s);
hipError_t launch_cov_pred_i64(const int64_t *p1, const int64_t *p2, int64_t n_pairs, const CovLayout &lay,
                               const CovParams &cp, const CovBits &bits, hipStream_t s);
hipError_t launch_cov_summary(const CovLayout &lay, const CovBits &bits, const CovSums &sums, hipStream_t s);
hipError_t launch_cov_expand(const CovLayout &lay, const CovBits &bits, int crit, uint64_t *out, int64_t n_words,
                             hipStream_t s);

}  // namespace ibmc
