// Launch interface of the training kernels of the float (sigmoid) networks:
// the mean softmax cross-entropy of the logits against the labels and its
// gradient by backpropagation (the networks are trained on labelled
// examples, Sec. II-A; the verifier's counterexamples are added to the
// training set, Sec. VI).
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

constexpr int kTrainThreads = 1024;
constexpr int kTrainMaxTile = 16;          // samples per workgroup
constexpr int kTrainLdsBytes = 64 * 1024;  // LDS of one workgroup

// The flat parameter vector theta: for each layer l = 1..L in turn, W_l
// row-major [dims[l]][dims[l-1]] then b_l [dims[l]].
struct TrainNetDev {
    int L;
    int dims[kMaxLayers + 1];
    int64_t toff[kMaxLayers + 1];   // l >= 1: offset of W_l in theta (b_l follows it)
    int64_t n_params;
    // per-sample LDS layout: activations a_0 .. a_L at aoff[l] (a_L = the
    // logits), units = dims[0] + sum of the other widths; deltas dL/du of
    // layers 1..L at aoff[l] - dims[0] in a block of units - dims[0]
    int aoff[kMaxLayers + 1];
    int units;
};

TrainNetDev train_layout(int L, const int *dims);
// Samples per workgroup: wanted (>= 1) clipped to what LDS holds.
int train_tile(const TrainNetDev &N, int wanted);
size_t train_lds_bytes(const TrainNetDev &N, int tile);

struct TrainGradParams {
    TrainNetDev net;
    const float *theta;
    const uint8_t *images;     // [n_images][dims[0]]
    const int32_t *labels;     // [n_images], each in [0, dims[L])
    const int64_t *order;      // nullable: element e of the pass is image order[e]
    int64_t e0, count;         // this launch: elements e0 .. e0 + count - 1
    int tile;                  // samples per workgroup
    float inv_n;               // 1 / the number of samples the mean runs over
    float *partial;            // [ceil(count / tile)][n_params] per-workgroup gradient sums
    float *partial_loss;       // [ceil(count / tile)] per-workgroup loss sums
};

hipError_t launch_train_grad(const TrainGradParams &P, hipStream_t s);
// grad = (accumulate ? grad : 0) + the sum of the tiles' partials, in tile
// order; *loss_acc += the sum of the tiles' loss sums (in order, double).
hipError_t launch_train_reduce(const float *partial, const float *partial_loss, int tiles, int64_t n_params,
                               float *grad, bool accumulate, double *loss_acc, hipStream_t s);

}  // namespace ibmc
