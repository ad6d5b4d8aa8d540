// Internal declarations of the HIP library (host runtime + gfx950 kernels).
//
// Device data layout of an integer network (built once by ibmc_load_mlp):
//
//  * Hidden widths are padded to H_l = roundup(h_l, 64), the class count to
//    H_L = roundup(h_L, 16); padding rows have zero weights and zero bias.
//  * Layers l >= 2 run on v_mfma_i32_16x16x64_i8 in the orientation
//    out[neurons x points] = W_l[neurons x K] * act[K x points]: weights are
//    the A operand (16 rows x 64 K per instruction, 16 bytes per lane), the
//    activations of 16 points are the B operand.  The accumulator of one
//    16-row tile leaves lane (j + 16 g) holding rows 4g..4g+3 of point j.
//    Packing those four requantised values into one dword gives, with no
//    data movement, dword t = (tile % 4) of the next layer's B operand for
//    K-block tile / 4 -- provided the next layer's K index is permuted by
//    sigma below.  So activations stay in registers from layer to layer.
//  * sigma(q): inside each block of 64, storage position q = 16g + 4t + i
//    holds neuron 16t + 4g + i (the two middle base-4 digits swapped; sigma
//    is an involution).  W1T (first layer, transposed [pixel][H1]), its bias
//    and the clean potentials are stored in sigma order, so a lane reads the
//    16 neurons it owns as 16 contiguous values.
//  * A-operand tiles of W_l (l >= 2): [H_l/16][H_{l-1}/64][64 lanes][16 B];
//    lane (r + 16 g), byte b of tile (m, kb) = W_l[16m + r][sigma(64kb + 16g + b)].
//    One wave reads one tile as 1 KB of consecutive 16-byte chunks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ibmc.h"

namespace ibmc {

constexpr int kMaxLayers = IBMC_MAX_LAYERS;
constexpr int kMaxWidth = IBMC_MAX_WIDTH;
constexpr int kMaxClasses = 64;
constexpr int kMaxShift = 24;          // hidden-layer shifts: 64 << s stays inside int32
constexpr int kMaxK = 8;
constexpr int kMaxDeltas = 64;

typedef int v4i __attribute__((ext_vector_type(4)));

__host__ __device__ inline int sigma64(int q) {
    const int blk = q & ~63, g = (q >> 4) & 3, t = (q >> 2) & 3, i = q & 3;
    return blk | (t << 4) | (g << 2) | i;
}

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Integer network as the kernels see it.
struct QNetDev {
    int L;                             // weight layers
    int dims[kMaxLayers + 1];          // true widths
    int H[kMaxLayers + 1];             // padded widths (H[0] = pixels, unpadded)
    int shift[kMaxLayers];             // per hidden layer (index l-1)
    const int8_t *W1T;                 // [n][H1], sigma order
    const int16_t *W1T16;              // [n][H1], sigma order, f1 * W1 (packed first-layer path)
    int f1;                            // 2^(8 - shift[0]) if shift[0] <= 8, else 0
    int maxw1;                         // max |W1|
    const int32_t *bo[kMaxLayers + 1]; // l >= 2: bias with the a - 64 input offset (and the
                                       // hidden requantiser offset) folded in, natural order
    int fast2;                         // 3-layer nets with shift[1] in {7, 8} and int32 room for the
                                       // offset accumulators: alpha = 2^(8 - shift[1]), else 0
    const int32_t *bf2;                // alpha * (b2 + 64 rowsum(W2)) - 32768: layer-2 init for inputs
                                       // alpha (a1 - 64) (fast2 != 0)
    const int32_t *bf3;                // b3 + 128 rowsum(W3): output-layer init for inputs a2 - 128 (fast2 != 0)
    const int32_t *b1s;                // [H1], sigma order
    const int8_t *Wt[kMaxLayers + 1];  // l >= 2: A-operand tiles
    const int32_t *bn[kMaxLayers + 1]; // l >= 2: bias, natural order, padded to H[l]
    const int8_t *W1tile;              // layer-1 A-operand tiles over pixel K-blocks (coverage)
    const int32_t *b1n;                // layer-1 bias, natural order, padded to H1
    const int32_t *rowsum1;            // 128 * sum_i W1[j][i], natural order, padded (x - 128 trick)
    const int8_t *Wd[kMaxLayers + 1];  // l >= 1: dense row-major [dims[l]][dims[l-1]]
    const int32_t *bd[kMaxLayers + 1]; // l >= 1: dense bias [dims[l]]
    const float *pnorm;                // proposer features: sum |W1[:, p]| [n], ||W1[:, p]||_2 [n], their maxima
};

// Float network (sigmoid variant).
struct FNetDev {
    int L;
    int dims[kMaxLayers + 1];
    const float *W1T;                  // [n][h1] transposed first layer
    const float *WT[kMaxLayers + 1];   // l >= 2: transposed [dims[l-1]][dims[l]]
    const float *Wd[kMaxLayers + 1];   // l >= 1: row-major [dims[l]][dims[l-1]]
    const float *bd[kMaxLayers + 1];
    // enumeration layout: widths padded to HP (zero weights and biases in the
    // padding, whose units therefore add exact zeros downstream)
    int kind;                          // F32Kind
    int HP[kMaxLayers + 1];            // HP[0] = pixels
    const float *W1P;                  // [n][HP1] transposed first layer
    const float *WP[kMaxLayers + 1];   // l >= 2: transposed [HP[l-1]][HP[l]]
    const float *bP[kMaxLayers + 1];   // l >= 1: [HP[l]]
};

// One counterexample record, identical to ibmc_cex.
struct CexRec {
    int32_t prop;
    int32_t k;
    int64_t rank;
    int32_t label;
    int32_t reserved;
};
static_assert(sizeof(CexRec) == sizeof(ibmc_cex), "record layout");

// Record as the enumeration kernels write it: 16 bytes, one vector store per
// lane.  klab = k << 24 | new label.  prop -1 marks an unused slot.
struct DevRec {
    int64_t rank;
    int32_t prop;
    int32_t klab;
};
static_assert(sizeof(DevRec) == 16, "device record layout");

// Per-property device data.
struct PropDev {
    const uint8_t *image;  // dims[0] bytes
    const int32_t *u0s;    // clean first-layer potentials, sigma order (integer) / natural (float)
    int32_t label0;        // written by the clean pass
    int32_t m;             // |D|
    int32_t n;             // pixels
    int32_t tie0;          // clean image has an exact top-2 tie (written by the clean pass)
    int32_t clean_done;    // first-layer slices of the integer clean pass finished; 0 when uploaded
    int32_t ball;          // 1: the L2-ball domain (deltas unused), 0: the delta set
    int32_t ball_rd;       // ball: offsets -rd..-1, 1..rd as digits 0..2 rd - 1 (m = 2 rd)
    int32_t ball_r2;       // ball: squared radius
    int16_t deltas[kMaxDeltas];
};

// Offset of digit i in the L2-ball domain's encoding.
__host__ __device__ inline int ball_offset(int i, int rd) { return i < rd ? i - rd : i - rd + 1; }

// Integer network in the compact layouts of the lane-per-point kernels (one
// or two hidden layers of at most 64 units, at most 16 classes): widths
// padded to the instance widths LH1 in {16, 32, 64} and LH2 in {0 (one
// hidden layer), 16, 32, 64}; 16 classes.  Padding units have zero weights
// and biases (activation 0), padding classes are never read.
struct LaneNetDev {
    int ok;                            // the network has these layouts
    int L, n, nc;
    int LH1, LH2;
    int s1, s2;                        // shifts of the hidden layers
    const int8_t *W1C;                 // [n][LH1] first-layer columns, natural unit order
    const int32_t *q1;                 // [LH1] position of unit j in the clean pass's (sigma) order, -1: padding
    const int32_t *W2S;                // L == 3: [LH2 / 8][LH1 / 4][8] words of 4 int8 weights (inputs
                                       // 4w..4w+3 of unit 8s + t)
    const int32_t *b2;                 // L == 3: [LH2]
    const int32_t *WOS;                // [2][LHL / 4][8] output words, LHL the last hidden width
    const int32_t *bo;                 // [16]
};

// Ordering of the last perturbed element inside a segment.
enum SegMode : int32_t {
    SEG_PLAIN = 0,   // last element ranges over (p, i) with p > previous pixel, pixel-major
    SEG_SHELL = 1,   // level 2, shell t: partner candidates order[0..t) (distinct pixel)
    SEG_LIST1 = 2,   // level 1: candidates order[0..n*m)
};

// One (property, level) of a launch.
struct EnumJob {
    int32_t prop;
    int32_t k;
    int32_t slot;          // counter slot of this (property, level)
    int32_t mode;          // SegMode
    int64_t chunk_begin;   // first global chunk of this job
    int64_t chunk_end;
    const int64_t *qcum;   // plain k >= 2: chunks before last-prefix pixel q, [n]
    const int32_t *order;  // shell / list modes: candidate ids (p * m + i) by decreasing score
    const int64_t *shell_cum; // shell mode: chunks before shell t, [n*m + 1]
    int32_t wseg;          // plain k >= 2: segments per group (one chunk covers the same
                           // last-element positions of wseg consecutive segments); else 1
    int32_t pad_;
};

// Segments per group of the integer kernel's packed path.
constexpr int kSegGroup = 4;

struct EnumParams {
    QNetDev net;
    const EnumJob *jobs;
    int32_t n_jobs;
    int32_t batch;                     // chunks per queue ticket once the single chunks are gone
    int64_t total_chunks;
    int64_t single;                    // leading chunks dealt out one at a time, statically: chunk c
                                       // to wave c mod (grid waves) (ordered searches)
    const PropDev *props;
    unsigned long long *queue;         // next queue ticket: ticket t is the batch of chunks from
                                       // single + t * batch
    unsigned long long *rec_count;     // record slots handed out (whole blocks of kRecBlock per wave)
    int64_t rec_cap;                   // record slots in recs: capacity + kRecBlock per wave of the grid
    DevRec *recs;                      // unused slots of a wave's last block hold a sentinel (prop -1)
    unsigned long long *slot_cex;      // per slot counterexamples
    unsigned long long *slot_ties;     // per slot exact top-2 ties
    unsigned long long *first_chunk;   // min chunk index holding a counterexample (ordered searches)
    volatile int32_t *stop_flag;       // device memory: set on the first counterexample if stop_on_first
    volatile int32_t *abort_host;      // host-mapped abort request (nullable), polled every 16th queue
                                       // fetch of a wave, after its first
    volatile int32_t *hit_host;        // host-mapped, set on the first counterexample (nullable;
                                       // needs track_first)
    int32_t stop_on_first;
    int32_t packed;                    // packed int16 first layer (bound checked by the host)
    int32_t vb_lo, vb_hi;              // pre-clamp of the scaled base for the packed path
    int32_t track_first;               // maintain first_chunk (ordered searches)
    int32_t notify;                    // any of stop_on_first, track_first, hit_host (set at launch)
    int64_t resume;                    // queue tickets start at this chunk (a resumed check); chunks
                                       // below it were checked by an earlier call
};

// Record slots a wave of the integer kernel reserves at a time.
constexpr int kRecBlock = 64;

// The float kernels' work queue: the chunk range is cut into kF32Queues
// contiguous slices, each with its own counter on its own 128-byte line, so
// that tickets of small chunks do not serialise on one address.
constexpr int kF32Queues = 32;
constexpr int kQueueStride = 16;   // u64 words between counters

// Float enumeration parameters.
struct FEnumParams {
    FNetDev net;
    const EnumJob *jobs;
    int32_t n_jobs;
    int32_t batch;
    int64_t total_chunks;
    const PropDev *props;
    const float *u0f;                  // clean first-layer potentials per property [prop][h1]
    int32_t u0_stride;
    float tie_rel;
    unsigned long long *queue;         // kF32Queues counters, kQueueStride apart: counter q hands out
                                       // chunks of slice q ([q * slice, (q + 1) * slice)) by offset
    int64_t slice;
    unsigned long long *rec_count;
    int64_t rec_cap;
    DevRec *recs;
    unsigned long long *tie_count;
    int64_t tie_cap;
    DevRec *ties;
    unsigned long long *slot_cex;
    unsigned long long *slot_ties;
    volatile int32_t *stop_flag;
    volatile int32_t *abort_host;
    const float *lut;                  // the table sigmoid's 257 knot values, or null (exponential)
    int32_t literal;                   // the threshold literal instead of the label change
    float lit_v;                       // its reference value V
};

// Knots of the table sigmoid: u = -8 + i / 16, i = 0..kLutIntervals.
constexpr int kLutIntervals = 256;

// Binomial coefficient for the small k used here (exact in int64 for n <= 1024, r <= 8).
__host__ __device__ inline int64_t binom_small(int64_t n, int r) {
    if (r < 0 || n < r) return 0;
    int64_t v = 1;
    for (int t = 1; t <= r; ++t) {
        const int64_t x = n - r + t;  // v * x is divisible by t; split to keep intermediates small
        v = (v / t) * x + ((v % t) * x) / t;
    }
    return v;
}

// Combinatorial number system: the lexicographic rank of a k-subset
// p[0] < ... < p[k-1] of [0, n) is C(n,k) - 1 - sum_j C(n-1-p[j], k-j).
__host__ __device__ inline int64_t lex_rank_subset(const int *p, int k, int n) {
    int64_t s = 0;
    for (int j = 0; j < k; ++j) s += binom_small(n - 1 - p[j], k - j);
    return binom_small(n, k) - 1 - s;
}

// Inverse of lex_rank_subset: write R = C(n,k) - 1 - rank as
// sum_j C(c_j, k-j) with n > c_0 > c_1 > ... >= 0 (greedy), then p_j = n-1-c_j.
__host__ __device__ inline void lex_unrank_subset(int64_t rank, int k, int n, int *p) {
    int64_t R = binom_small(n, k) - 1 - rank;
    int c = n;
    for (int j = 0; j < k; ++j) {
        const int r = k - j;
        int cj = c - 1;
        while (cj >= r && binom_small(cj, r) > R) --cj;  // stops at r-1 at the latest: C(r-1, r) = 0
        R -= binom_small(cj, r);
        p[j] = n - 1 - cj;
        c = cj;
    }
}

}  // namespace ibmc
