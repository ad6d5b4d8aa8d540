// Launch interface of the float (sigmoid) network kernels.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

// Default near-tie threshold of the float path, relative to
// max(1, |largest logit|): when every logit is within eps * max(1, |z64|) of
// its double-precision value, two points of opposite decisions need an FP32
// margin of at most about 2 eps * scale; eps = 1e-5, with a factor of two to
// spare.
constexpr float kDefaultTieRel = 4e-5f;

// Inputs per partial sum of the float layers: each block of products is
// accumulated from zero and then added to the running total (blocked
// summation; its rounding error grows with the block length plus the number
// of blocks instead of with the layer width).
constexpr int kF32SumBlock = 32;

// Enumeration kernel families (chosen per network at load time):
//   one point per lane: hidden widths padded to 16/32/64/128, at most two
//     hidden layers, at most 16 classes; activations in registers (the second
//     hidden layer in the wave's LDS), weights through the scalar cache;
//   sixteen points per wave: every other shape (widths padded to multiples
//     of 64, up to 512); lanes are neurons, the points' activations sit in
//     the wave's LDS.
enum F32Kind : int32_t { F32_LANE = 0, F32_WIDE = 1 };

constexpr int kF32LaneChunk = 64;   // points per chunk (one per lane)
constexpr int kF32WideChunk = 16;   // points per chunk (per wave)
constexpr int kF32MaxWidth = 512;   // widest float layer the kernels accept

// Padded layout of a float network for the enumeration kernels.
struct F32Layout {
    int kind;
    int HP[kMaxLayers + 1];         // HP[0] = pixels
};
// Shape class of a float network (host): kind and padded widths.
F32Layout f32_layout(int L, const int *dims);

// Points given by (k, rank) of one property, evaluated with the enumeration
// kernels' arithmetic.  prop_of: property per point (nullable: all 0).  When
// label_to_props is set the points are k = 0 images of the listed properties
// and their labels are stored as the properties' clean labels.
struct F32EvalParams {
    FNetDev net;
    const PropDev *props;
    PropDev *label_props;           // clean-label mode: write props[prop].label0
    const int32_t *prop_of;         // nullable
    const int32_t *ks;
    const int64_t *ranks;
    int64_t n;
    const float *u0f;               // clean first-layer potentials [prop][u0_stride]
    int32_t u0_stride;
    float *logits;                  // nullable: [n][classes]
    int32_t *labels;                // nullable: [n]
    float *margins;                 // nullable: [n]
    const float *lut;               // the table sigmoid's knots, or null (exponential)
};

hipError_t launch_forward_f32(const FNetDev &net, const uint8_t *images, int64_t n_images,
                              int32_t *labels, float *pots, int64_t pot_stride, hipStream_t s);
hipError_t launch_replay_f32(const FNetDev &net, const uint8_t *clean, const int16_t *deltas, int m,
                             const CexRec *recs, int64_t n_recs, int32_t *labels, hipStream_t s);
// Clean pass of the enumeration: first-layer potentials (padded to HP[1]
// with zeros) of every listed property, then its clean label through the
// enumeration arithmetic.
hipError_t launch_clean_f32(const FNetDev &net, PropDev *props, const int32_t *prop_ids,
                            int32_t n_ids, float *u0_store, int64_t u0_stride, hipStream_t s,
                            const float *lut = nullptr);
hipError_t launch_eval_f32(const F32EvalParams &E, hipStream_t s);
// Persistent enumeration; grid (in waves) from f32_enum_grid.
hipError_t launch_enum_f32(int grid_waves, const FEnumParams &P, hipStream_t s);
// Points per chunk and a grid size (waves) that fills the device.
int enum_f32_chunk(const FNetDev &net);
int f32_enum_grid(const FNetDev &net, int n_cu, bool table);  // table: the table-sigmoid instance
// Whether a compiled lane instance serves this padded shape.
bool f32_lane_supported(int L, const int *HP);

}  // namespace ibmc
