// Launch interface of the float (sigmoid) network kernels.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

// default near-tie threshold of the float path, relative to max(1, |largest logit|)
constexpr float kDefaultTieRel = 1e-4f;

hipError_t launch_forward_f32(const FNetDev &net, const uint8_t *images, int64_t n_images,
                              int32_t *labels, float *pots, int64_t pot_stride, hipStream_t s);
hipError_t launch_replay_f32(const FNetDev &net, const uint8_t *clean, const int16_t *deltas, int m,
                             const CexRec *recs, int64_t n_recs, int32_t *labels, hipStream_t s);
hipError_t launch_clean_f32(const FNetDev &net, PropDev *props, const int32_t *prop_ids,
                            int32_t n_ids, float *u0_store, int64_t u0_stride, hipStream_t s);
hipError_t launch_enum_f32(int grid, const FEnumParams &P, const int32_t *u0_index, hipStream_t s);
int enum_f32_chunk();

}  // namespace ibmc
