// Launch interface of the integer lane-per-point enumeration kernels: small
// networks (one or two hidden layers of at most 64 units, at most 16
// classes), the delta-set domain and the L2-ball domain.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

constexpr int kLaneChunk = 64;   // points per chunk: one per lane
constexpr const char *kLaneVariantName = "lane";

struct LaneParams {
    LaneNetDev net;
    const EnumJob *jobs;
    int32_t n_jobs;
    int32_t batch;                     // chunks per queue ticket
    int64_t total_chunks;
    const PropDev *props;
    const int32_t *u0;                 // clean first-layer potentials per property, sigma order
    int32_t u0_stride;
    unsigned long long *queue;         // kF32Queues counters, kQueueStride apart (sliced queue)
    int64_t slice;
    unsigned long long *rec_count;
    int64_t rec_cap;
    DevRec *recs;
    unsigned long long *slot_cex;      // per slot: counterexamples
    unsigned long long *slot_ties;     // per slot: exact top-2 logit ties
    unsigned long long *slot_points;   // per slot: points of the domain visited
    volatile int32_t *stop_flag;
    volatile int32_t *abort_host;
    int32_t literal;                   // the threshold literal instead of the label change
    int32_t lit_v;                     // its reference value V
};

// The network has the compact layouts (see LaneNetDev).
bool lane_eligible(const int *dims, int L);
// Instance widths of a hidden layer of h units.
int lane_width(int h);
// Persistent grid of the instance for the network (0: no instance).
int lane_enum_grid(const LaneNetDev &net, int n_cu);
hipError_t launch_enum_lane(int grid, const LaneParams &P, hipStream_t s);

}  // namespace ibmc
