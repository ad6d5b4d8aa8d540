// The check driver: the incremental bound loop of Sec. II-B around the
// safety property of Sec. III-C, over one or many properties.  Builds the
// work plan (jobs of (property, level) and their chunk counts), runs the
// clean pass and the enumeration kernels, gathers counters and records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "ibmc_host.h"

namespace ibmc {

std::string shape_key(const ibmc_mlp *m) {
    std::string s = (m->act == IBMC_ACT_RELU_Q8) ? "q8" : "f32";
    for (int d : m->dims) s += "_" + std::to_string(d);
    if (m->act == IBMC_ACT_RELU_Q8 && m->L == 3 && m->qd.fast2 != 0) s += "_f";
    return s;
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int64_t ipow64(int64_t a, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= a;
    return r;
}

// Chunks of a plain level; qcum receives the chunks before each last-prefix
// pixel q (k >= 2).
// Chunks of one plain level: for each last-prefix pixel q, its segments
// (prefix subsets times prefix deltas) in groups of W, times the chunks of
// one segment's last-element range.  qcum[q]: chunks before q.
static int64_t plan_plain_level(int n, int m, int k, int CH, int W, std::vector<int64_t> &qcum) {
    if (k == 1) return ceil_div((int64_t)n * m, CH);
    qcum.assign(n, 0);
    const int64_t mk1 = ipow64(m, k - 1);
    int64_t acc = 0;
    for (int q = 0; q < n; ++q) {
        qcum[q] = acc;
        if (q >= k - 2 && q <= n - 2)
            acc += ceil_div(binom_small(q, k - 2) * mk1, W) * ceil_div((int64_t)(n - 1 - q) * m, CH);
    }
    return acc;
}

// A kernel instance serves a network when its layer count, hidden widths,
// hidden epilogue form and output width class (at most 16 classes or more)
// agree with it.
static bool variant_matches(const EnumVariant &v, const ibmc_mlp *net) {
    const int L = net->L;
    const int kb2 = (L == 3) ? net->qd.H[2] / 64 : 0;
    const int epi = (L == 3 && net->qd.fast2 != 0) ? 1 : 0;
    const bool out16 = net->qd.H[L] == 16;
    return v.L == L && v.kb1 == net->qd.H[1] / 64 && v.kb2 == kb2 && v.epi == epi && v.out16 == out16;
}

// Variant choice for an integer network: the tuned one if any, else the
// widest point tile whose weights fit the LDS budget.
const EnumVariant *pick_variant(ibmc_ctx *ctx, const ibmc_mlp *net) {
    int nv = 0;
    const EnumVariant *vs = enum_variants(&nv);
    std::string want = net->forced_variant;
    if (want.empty()) {
        auto it = ctx->tuned.find(shape_key(net));
        if (it != ctx->tuned.end()) want = it->second;
    }
    if (!want.empty())
        for (int i = 0; i < nv; ++i)
            if (want == vs[i].name && variant_matches(vs[i], net)) return &vs[i];
    const EnumVariant *best = nullptr;
    for (int i = 0; i < nv; ++i) {
        const EnumVariant &v = vs[i];
        if (!variant_matches(v, net)) continue;
        if (enum_lds_bytes(v, net->qd) > 96 * 1024) continue;
        const int score = (v.wlds ? 100 : 0) + (v.nt == 2 ? 10 : v.nt);
        if (!best || score > (best->wlds ? 100 : 0) + (best->nt == 2 ? 10 : best->nt)) best = &v;
    }
    return best;
}

// The lane kernel serves an integer network when forced or tuned for its
// shape; untuned, it takes the networks with one hidden layer of at most 16
// units, whose 16x16x64 matrix-core tiles are mostly padding.  Wider or
// deeper networks go to the matrix cores by default (on large workloads the
// dot4 path pays about h1 + nc h_last / 4 instructions per point and loses,
// e.g. 64-32-10 at 40 vs 59 G points/s).  Never for resumable calls, which
// only the matrix-core kernel implements (allowed false).
bool use_lane(ibmc_ctx *ctx, const ibmc_mlp *net, bool allowed) {
    if (!allowed || !net->lane.ok) return false;
    std::string want = net->forced_variant;
    if (want.empty()) {
        auto it = ctx->tuned.find(shape_key(net));
        if (it != ctx->tuned.end()) want = it->second;
    }
    if (!want.empty()) return want == kLaneVariantName;
    return net->L == 2 && net->dims[1] <= 16;
}

struct Level {
    int prop;
    int k;
    int slot;
};

struct BatchState {
    std::vector<PropDev> hprops;
    std::vector<int> level_count;             // levels per property
    std::vector<std::vector<int>> level_k;    // k per level per property
    std::vector<int> slot_base;               // first slot of each property
    int n_slots = 0;
};

// Digits per pixel side of the L2-ball domain: min(floor(sqrt(r2)), 255).
static int ball_rd(int64_t r2) {
    int64_t r = 0;
    while (r < 255 && (r + 1) * (r + 1) <= r2) ++r;
    return (int)r;
}

// props: for ball properties (ball_r2[i] >= 0) n_deltas already holds the
// digit count 2 rd and deltas is unused.
static ibmc_status validate_props(const ibmc_property *props, int32_t n_props, const ibmc_check_opts *o,
                                  const int64_t *ball_r2) {
    if (!props || n_props < 1) return fail(IBMC_E_INVALID, "no properties");
    if (!o) return fail(IBMC_E_INVALID, "opts is null");
    if (o->cex_capacity < 0 || o->near_tie_capacity < 0) return fail(IBMC_E_INVALID, "negative capacity");
    for (int i = 0; i < n_props; ++i) {
        const ibmc_property &p = props[i];
        const bool ball = ball_r2 && ball_r2[i] >= 0;
        if (!p.net || !p.image || (!ball && !p.deltas))
            return fail(IBMC_E_INVALID, "property %d: null net/image/deltas", i);
        if (ball) {
            if (ball_r2[i] > ((int64_t)1 << 30))
                return fail(IBMC_E_INVALID, "property %d: radius_sq %lld above 2^30", i, (long long)ball_r2[i]);
            if (p.net->act != IBMC_ACT_RELU_Q8 || !p.net->lane.ok)
                return fail(IBMC_E_UNIMPL, "property %d: the L2-ball domain needs an integer network with 1-2 hidden "
                            "layers of at most 64 units and at most 16 classes", i);
        } else if (p.n_deltas < 1 || p.n_deltas > kMaxDeltas) {
            return fail(IBMC_E_INVALID, "property %d: n_deltas %d outside [1, %d]", i, p.n_deltas, kMaxDeltas);
        }
        const int n = p.net->dims[0];
        if ((int64_t)n * p.n_deltas >= ((int64_t)1 << 24))
            return fail(IBMC_E_UNIMPL, "property %d: pixels * deltas = %lld must be below 2^24", i,
                        (long long)n * p.n_deltas);
        if (p.k_min < 0 || p.k_max < p.k_min || p.k_step < 1)
            return fail(IBMC_E_INVALID, "property %d: bad k range %d..%d step %d", i, p.k_min, p.k_max, p.k_step);
        if (p.k_max > n || p.k_max > kMaxK)
            return fail(IBMC_E_INVALID, "property %d: k_max %d exceeds min(n=%d, %d)", i, p.k_max, n, kMaxK);
        int levels = 0;
        for (int k = p.k_min; k <= p.k_max; k += p.k_step) {
            ++levels;
            // points of the level must fit comfortably in int64
            __int128 pts = (__int128)binom_small(n, k);
            for (int j = 0; j < k; ++j) pts *= std::max(p.n_deltas, 1);
            if (pts > ((__int128)1 << 56)) return fail(IBMC_E_UNIMPL, "property %d: level %d too large", i, k);
        }
        if (levels > IBMC_MAX_LEVELS) return fail(IBMC_E_INVALID, "property %d: %d levels > %d", i, levels, IBMC_MAX_LEVELS);
        if (p.net->act == IBMC_ACT_RELU_Q8 && p.net->L > 3 && p.k_max >= 1)
            return fail(IBMC_E_UNIMPL, "property %d: enumeration supports 2 or 3 weight layers", i);
        if (p.net->act == IBMC_ACT_SIGMOID_F32) {
            for (int l = 1; l <= p.net->L; ++l)
                if (p.net->dims[l] > kF32MaxWidth)
                    return fail(IBMC_E_UNIMPL, "property %d: float layer wider than %d", i, kF32MaxWidth);
        }
    }
    return IBMC_OK;
}


// Sort the first n record slots on the device by (prop, k, rank) and hand
// out the first `keep` records without the sentinels of unused slots (prop
// -1): into `direct` when given (device memory when direct_dev, else host;
// room for keep records), else into outv.  *nout: records handed out.
static ibmc_status fetch_sorted(ibmc_ctx *ctx, const DevRec *drecs, int64_t n, int64_t keep, int max_prop, int max_k,
                                int64_t max_rank, std::vector<CexRec> &outv, CexRec *direct, bool direct_dev,
                                int64_t *nout) {
    hipStream_t s = ctx->stream;
    outv.clear();
    *nout = 0;
    if (n == 0 || keep == 0) return IBMC_OK;
    IBMC_TRY(ctx->sortbuf.reserve(sort_scratch_bytes(n)));
    SortScratch S;
    sort_scratch_carve(ctx->sortbuf.p, n, S);
    int bits = 0;
    const int st = sort_records_device(drecs, n, max_prop, max_k, max_rank, S, s, &bits);
    if (st == SORT_HIP_ERROR) return fail(IBMC_E_HIP, "record sort launch failed");
    if (st == SORT_UNSUPPORTED) {  // keys wider than 64 bits: order on the host
        std::vector<DevRec> raw(n);
        HIP_OK(hipMemcpyAsync(raw.data(), drecs, n * sizeof(DevRec), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        std::vector<CexRec> all;
        all.reserve(n);
        for (const DevRec &d : raw)
            if (d.prop >= 0)
                all.push_back(CexRec{d.prop, (int32_t)((uint32_t)d.klab >> 24), d.rank,
                                     (int32_t)((uint32_t)d.klab & 0xffffffu), 0});
        std::sort(all.begin(), all.end(), [](const CexRec &a, const CexRec &b) {
            if (a.prop != b.prop) return a.prop < b.prop;
            if (a.k != b.k) return a.k < b.k;
            return a.rank < b.rank;
        });
        if ((int64_t)all.size() > keep) all.resize(keep);
        *nout = (int64_t)all.size();
        if (direct && direct_dev) {
            HIP_OK(hipMemcpyAsync(direct, all.data(), all.size() * sizeof(CexRec), hipMemcpyHostToDevice, s));
            HIP_OK(hipStreamSynchronize(s));
        } else if (direct) {
            memcpy(direct, all.data(), all.size() * sizeof(CexRec));
        } else {
            outv.swap(all);
        }
        return IBMC_OK;
    }
    // sentinels sort last (all key bits set); only the first keep slots matter
    const int64_t m = std::min(n, keep);
    CexRec *dout = direct_dev ? direct : nullptr;
    if (!dout) {
        IBMC_TRY(ctx->recout.reserve((size_t)m * sizeof(CexRec)));
        dout = ctx->recout.as<CexRec>();
    }
    HIP_OK(sorted_to_records(S, m, dout, s));
    int64_t valid = 0;
    HIP_OK(hipMemcpyAsync(&valid, S.count, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *nout = valid;
    if (direct_dev) return IBMC_OK;
    CexRec *hout = direct;
    if (!hout) {
        outv.resize(valid);
        hout = outv.data();
    }
    if (valid) {
        HIP_OK(hipMemcpyAsync(hout, dout, valid * sizeof(CexRec), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    return IBMC_OK;
}

// Run the given levels (subset of every property's level list): a clean
// pass and one persistent enumeration launch per network.  All plans are
// uploaded first; with several networks the launches are captured as one HIP
// graph with a parallel branch per network, so networks of uneven size share
// the GPU.  level_sel[prop] = level indices to run.
struct NetPlan {
    const ibmc_mlp *net;
    std::vector<int> ids;
    bool lane = false;      // integer network on the lane-per-point kernel
    const EnumVariant *v = nullptr;
    int64_t total = 0;
    int64_t limit = 0;      // chunks handed out stop here (a budgeted call), else total
    int32_t batch = 1;      // chunks per queue ticket (integer kernels)
    size_t job_off = 0, n_jobs = 0;
    int grid = 0;
    int32_t packed = 0, vb_lo = 0, vb_hi = 0;
};

static ibmc_status run_levels(ibmc_ctx *ctx, const ibmc_property *props, int32_t n_props,
                              const ibmc_check_opts *o, BatchState &B,
                              const std::vector<std::vector<int>> &level_sel, bool images_on_device,
                              std::vector<unsigned long long> &slot_cex, std::vector<unsigned long long> &slot_ties,
                              std::vector<unsigned long long> &slot_points,
                              std::vector<CexRec> &recs, std::vector<CexRec> &ties, int64_t &rec_total,
                              int64_t &tie_total, double &kernel_seconds, int &launches,
                              CexRec *direct_recs = nullptr, CexRec *direct_ties = nullptr, bool direct_dev = false,
                              int64_t resume = 0, int64_t budget = 0, int64_t *next_cursor = nullptr) {
    (void)images_on_device;
    hipStream_t s = ctx->stream;
    std::vector<NetPlan> plans;
    {
        std::map<const ibmc_mlp *, size_t> where;
        for (int i = 0; i < n_props; ++i) {
            if (level_sel[i].empty()) continue;
            auto it = where.find(props[i].net);
            if (it == where.end()) {
                where[props[i].net] = plans.size();
                plans.emplace_back();
                plans.back().net = props[i].net;
                plans.back().ids.push_back(i);
            } else {
                plans[it->second].ids.push_back(i);
            }
        }
    }
    const int NN = (int)plans.size();
    // counters: [1] rec_count, [2] first_chunk, [3] tie_count, [4] stop flag,
    //           [8, 8+NN) per-network queues (integer matrix-core kernels),
    //           then slot_cex[n_slots], slot_ties[n_slots], slot_points[n_slots]
    //           (lane kernels), then per network the sliced queues of the
    //           float and lane kernels: kF32Queues counters, kQueueStride apart
    const int64_t q0 = 8, sc0 = 8 + NN, st0 = sc0 + B.n_slots, sp0 = st0 + B.n_slots;
    const int64_t fq0 = (sp0 + B.n_slots + kQueueStride - 1) / kQueueStride * kQueueStride;
    const int64_t n_ctr = fq0 + (int64_t)NN * kF32Queues * kQueueStride;
    IBMC_TRY(ctx->counters.reserve(n_ctr * 8));
    unsigned long long *ctr = ctx->counters.as<unsigned long long>();
    const int64_t cap = o->cex_capacity, tcap = o->near_tie_capacity;
    IBMC_TRY(ctx->ties.reserve((size_t)std::max<int64_t>(tcap, 1) * sizeof(DevRec)));
    int64_t max_h1 = 64;
    for (auto &pl : plans)
        max_h1 = std::max<int64_t>(max_h1, pl.net->act == IBMC_ACT_RELU_Q8 ? pl.net->qd.H[1] : pl.net->fd.HP[1]);
    IBMC_TRY(ctx->u0.reserve((size_t)n_props * max_h1 * 4));
    std::vector<int32_t> u0_index(n_props), all_ids;
    std::iota(u0_index.begin(), u0_index.end(), 0);
    IBMC_TRY(ctx->u0_index.upload(u0_index.data(), u0_index.size() * 4, s));

    // plans: variants, jobs and chunk prefix sums of every network
    std::vector<EnumJob> jobs;
    std::vector<int64_t> qcum_all;
    std::vector<size_t> qcum_off;
    for (auto &pl : plans) {
        const ibmc_mlp *net = pl.net;
        const bool q8 = net->act == IBMC_ACT_RELU_Q8;
        int CH = q8 ? 0 : enum_f32_chunk(net->fd);
        // an L2-ball property, or the literal, runs on the lane kernel only
        bool need_lane = o->property == IBMC_PROPERTY_LITERAL;
        for (int pid : pl.ids) need_lane |= B.hprops[pid].ball != 0;
        if (q8) pl.lane = need_lane || use_lane(ctx, net, resume == 0 && budget == 0);
        if (pl.lane) {
            CH = kLaneChunk;
        } else if (q8) {
            pl.v = pick_variant(ctx, net);
            if (!pl.v) return fail(IBMC_E_UNIMPL, "no enumeration kernel for network %s", shape_key(net).c_str());
            CH = pl.v->chunk;
        }
        if (q8 && !pl.lane) {
            int maxe = 0;
            for (int pid : pl.ids)
                for (int j = 0; j < props[pid].n_deltas; ++j)
                    maxe = std::max(maxe, std::min(255, std::abs((int)props[pid].deltas[j])));
            const int64_t M2 = (int64_t)net->qd.f1 * maxe * net->qd.maxw1;
            pl.packed = (net->qd.f1 > 0 && M2 <= 8191 && !ctx->force_int32_layer1) ? 1 : 0;
            pl.vb_lo = (int32_t)(-16385 - M2);
            pl.vb_hi = (int32_t)(16384 + M2);
        }
        // segment groups: the packed integer path keeps kSegGroup bases per wave
        const int W = (q8 && !pl.lane && pl.packed) ? kSegGroup : 1;
        pl.job_off = jobs.size();
        for (int pid : pl.ids) {
            const int n = net->dims[0], m = props[pid].n_deltas;
            for (int li : level_sel[pid]) {
                const int k = B.level_k[pid][li];
                if (k == 0) continue;
                std::vector<int64_t> qc;
                const int64_t ch = plan_plain_level(n, m, k, CH, W, qc);
                if (ch == 0) continue;   // an empty level (a ball with no nonzero offset)
                EnumJob J{};
                J.prop = pid;
                J.k = k;
                J.slot = B.slot_base[pid] + li;
                J.mode = SEG_PLAIN;
                J.wseg = W;
                J.chunk_begin = pl.total;
                J.chunk_end = pl.total + ch;
                qcum_off.push_back(k >= 2 ? qcum_all.size() : (size_t)-1);
                if (k >= 2) qcum_all.insert(qcum_all.end(), qc.begin(), qc.end());
                pl.total += ch;
                jobs.push_back(J);
            }
        }
        pl.n_jobs = jobs.size() - pl.job_off;
        if (pl.lane) {
            const int g = lane_enum_grid(net->lane, ctx->n_cu);
            if (g < 1) return fail(IBMC_E_UNIMPL, "no lane kernel for network %s", shape_key(net).c_str());
            pl.grid = (int)std::min<int64_t>(g, std::max<int64_t>(1, pl.total));
        } else if (q8) {
            int occ = 0;
            HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pl.v->fn, 256,
                                                                (size_t)enum_lds_bytes(*pl.v, net->qd)));
            if (occ < 1) return fail(IBMC_E_UNIMPL, "variant %s does not fit", pl.v->name);
            pl.grid = (int)std::min<int64_t>((int64_t)ctx->n_cu * occ, std::max<int64_t>(1, pl.total / 2));
            pl.batch = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, pl.total / ((int64_t)pl.grid * 32)));
        } else {
            const int g = f32_enum_grid(net->fd, ctx->n_cu, o->sigmoid == IBMC_SIGMOID_TABLE);
            if (g < 1) return fail(IBMC_E_UNIMPL, "no float enumeration kernel for network %s", shape_key(net).c_str());
            pl.grid = (int)std::min<int64_t>(g, std::max<int64_t>(1, pl.total));
        }
        pl.limit = budget > 0 ? std::min(pl.total, resume + budget) : pl.total;
        all_ids.insert(all_ids.end(), pl.ids.begin(), pl.ids.end());
    }
    // record slots: the capacity plus one partly used block per wave of the
    // integer kernels (whose unused slots hold sentinels)
    int64_t rec_slots = cap;
    for (auto &pl : plans)
        if (pl.net->act == IBMC_ACT_RELU_Q8 && !pl.lane) rec_slots += (int64_t)pl.grid * 4 * kRecBlock;
    IBMC_TRY(ctx->recs.reserve((size_t)std::max<int64_t>(rec_slots, 1) * sizeof(DevRec)));
    IBMC_TRY(ctx->qcum.reserve(std::max<size_t>(qcum_all.size(), 1) * 8));
    if (!qcum_all.empty())
        HIP_OK(hipMemcpyAsync(ctx->qcum.p, qcum_all.data(), qcum_all.size() * 8, hipMemcpyHostToDevice, s));
    for (size_t j = 0; j < jobs.size(); ++j)
        jobs[j].qcum = (qcum_off[j] == (size_t)-1) ? nullptr : ctx->qcum.as<int64_t>() + qcum_off[j];
    // (no jobs at all: every selected level is k = 0 or empty)
    if (jobs.empty()) IBMC_TRY(ctx->jobs.reserve(sizeof(EnumJob)));
    else IBMC_TRY(ctx->jobs.upload(jobs.data(), jobs.size() * sizeof(EnumJob), s));
    IBMC_TRY(ctx->prop_ids.upload(all_ids.data(), std::max<size_t>(all_ids.size(), 1) * 4, s));
    HIP_OK(hipStreamSynchronize(s));  // host staging vectors may go now

    PropDev *dprops = ctx->props.as<PropDev>();
    // the table sigmoid's knots: sigma(-8 + i/16) rounded to FP32
    const float *lut = nullptr;
    if (o->sigmoid == IBMC_SIGMOID_TABLE) {
        if (!ctx->lut.p) {
            std::vector<float> knots(kLutIntervals + 1);
            for (int i = 0; i <= kLutIntervals; ++i) knots[i] = (float)(1.0 / (1.0 + std::exp(-(-8.0 + i / 16.0))));
            IBMC_TRY(ctx->lut.upload(knots.data(), knots.size() * 4, s));
            HIP_OK(hipStreamSynchronize(s));
        }
        lut = ctx->lut.as<float>();
    }
    const bool literal = o->property == IBMC_PROPERTY_LITERAL;
    // One network: the enumeration launch alone is bracketed by ek0 / ek1
    // (the kernel time reported for rooflines); several: the whole graph.
    const bool time_enum = NN <= 1;
    // the clean pass of a network's properties, and its enumeration launch
    auto launch_clean = [&](const NetPlan &pl, size_t id_off, hipStream_t st) -> ibmc_status {
        const ibmc_mlp *net = pl.net;
        const int32_t *ids = ctx->prop_ids.as<int32_t>() + id_off;
        if (net->act == IBMC_ACT_RELU_Q8)
            HIP_OK(launch_clean_q8(net->qd, dprops, ids, (int32_t)pl.ids.size(), ctx->u0.as<int32_t>(), max_h1, st));
        else
            HIP_OK(launch_clean_f32(net->fd, dprops, ids, (int32_t)pl.ids.size(), ctx->u0.as<float>(), max_h1, st,
                                    lut));
        return IBMC_OK;
    };
    auto launch_net = [&](const NetPlan &pl, hipStream_t st) -> ibmc_status {
        const ibmc_mlp *net = pl.net;
        if (pl.n_jobs == 0 || pl.total == 0) return IBMC_OK;
        const int pi = (int)(&pl - plans.data());
        if (pl.lane) {
            LaneParams P{};
            P.net = net->lane;
            P.jobs = ctx->jobs.as<EnumJob>() + pl.job_off;
            P.n_jobs = (int32_t)pl.n_jobs;
            P.total_chunks = pl.total;
            P.slice = std::max<int64_t>(1, (pl.total + kF32Queues - 1) / kF32Queues);
            const int64_t waves_per_slice = std::max<int64_t>(1, (int64_t)pl.grid * 4 / kF32Queues);
            P.batch = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, P.slice / (waves_per_slice * 8)));
            P.props = dprops;
            P.u0 = ctx->u0.as<int32_t>();
            P.u0_stride = (int32_t)max_h1;
            P.queue = ctr + fq0 + (int64_t)pi * kF32Queues * kQueueStride;
            P.rec_count = ctr + 1;
            P.rec_cap = rec_slots;
            P.recs = ctx->recs.as<DevRec>();
            P.slot_cex = ctr + sc0;
            P.slot_ties = ctr + st0;
            P.slot_points = ctr + sp0;
            P.stop_flag = reinterpret_cast<volatile int32_t *>(ctr + 4);
            P.abort_host = ctx->flags_dev;
            P.literal = literal ? 1 : 0;
            P.lit_v = literal ? (int32_t)o->literal_v : 0;
            if (time_enum) HIP_OK(hipEventRecord(ctx->ek0, st));
            HIP_OK(launch_enum_lane(pl.grid, P, st));
            if (time_enum) HIP_OK(hipEventRecord(ctx->ek1, st));
        } else if (net->act == IBMC_ACT_RELU_Q8) {
            EnumParams P{};
            P.net = net->qd;
            P.jobs = ctx->jobs.as<EnumJob>() + pl.job_off;
            P.n_jobs = (int32_t)pl.n_jobs;
            P.total_chunks = pl.limit;
            P.batch = pl.batch;
            P.resume = resume;
            P.props = dprops;
            P.queue = ctr + q0 + pi;
            P.rec_count = ctr + 1;
            P.first_chunk = ctr + 2;
            P.stop_flag = reinterpret_cast<volatile int32_t *>(ctr + 4);
            P.abort_host = ctx->flags_dev;
            P.hit_host = nullptr;
            P.rec_cap = rec_slots;
            P.recs = ctx->recs.as<DevRec>();
            P.slot_cex = ctr + sc0;
            P.slot_ties = ctr + st0;
            P.stop_on_first = 0;
            P.track_first = 0;
            P.packed = pl.packed;
            P.vb_lo = pl.vb_lo;
            P.vb_hi = pl.vb_hi;
            if (time_enum) HIP_OK(hipEventRecord(ctx->ek0, st));
            HIP_OK(launch_enum_q8(*pl.v, pl.grid, P, ctx->u0.as<int32_t>(), max_h1, ctx->u0_index.as<int32_t>(), st));
            if (time_enum) HIP_OK(hipEventRecord(ctx->ek1, st));
        } else {
            FEnumParams P{};
            P.net = net->fd;
            P.jobs = ctx->jobs.as<EnumJob>() + pl.job_off;
            P.n_jobs = (int32_t)pl.n_jobs;
            P.total_chunks = pl.total;
            // slices of the chunk range, each with its own queue counter;
            // tickets of up to 16 chunks, about 8 per wave of a slice
            P.slice = std::max<int64_t>(1, (pl.total + kF32Queues - 1) / kF32Queues);
            const int64_t waves_per_slice = std::max<int64_t>(1, pl.grid / kF32Queues);
            P.batch = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, P.slice / (waves_per_slice * 8)));
            P.props = dprops;
            P.u0f = ctx->u0.as<float>();
            P.u0_stride = (int32_t)max_h1;
            P.tie_rel = (o->near_tie_rel > 0) ? o->near_tie_rel : kDefaultTieRel;
            P.queue = ctr + fq0 + (int64_t)pi * kF32Queues * kQueueStride;
            P.rec_count = ctr + 1;
            P.rec_cap = rec_slots;
            P.recs = ctx->recs.as<DevRec>();
            P.tie_count = ctr + 3;
            P.tie_cap = tcap;
            P.ties = ctx->ties.as<DevRec>();
            P.slot_cex = ctr + sc0;
            P.slot_ties = ctr + st0;
            P.stop_flag = reinterpret_cast<volatile int32_t *>(ctr + 4);
            P.abort_host = ctx->flags_dev;
            P.lut = lut;
            P.literal = literal ? 1 : 0;
            P.lit_v = (float)o->literal_v;
            if (time_enum) HIP_OK(hipEventRecord(ctx->ek0, st));
            HIP_OK(launch_enum_f32(pl.grid, P, st));
            if (time_enum) HIP_OK(hipEventRecord(ctx->ek1, st));
        }
        return IBMC_OK;
    };

    kernel_seconds = 0.0;
    launches = 0;
    bool timed = false;
    if (!time_enum) HIP_OK(hipEventRecord(ctx->ek0, s));
    if (NN <= 1) {
        HIP_OK(launch_fill_u64(ctr, n_ctr, 0ull, s));
        HIP_OK(launch_fill_u64(ctr + 2, 1, ~0ull, s));
        size_t id_off = 0;
        for (auto &pl : plans) {
            IBMC_TRY(launch_clean(pl, id_off, s));
            IBMC_TRY(launch_net(pl, s));
            id_off += pl.ids.size();
            timed = pl.n_jobs > 0 && pl.total > 0;
        }
    } else {
        // one graph: counters cleared by a kernel (no memset node), then a
        // branch per network on its own stream, joined back into s
        while ((int)ctx->side.size() < NN) {
            hipStream_t ns;
            HIP_OK(hipStreamCreateWithFlags(&ns, hipStreamNonBlocking));
            ctx->side.push_back(ns);
            hipEvent_t ev;
            HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            ctx->side_ev.push_back(ev);
        }
        if (!ctx->fork_ev) HIP_OK(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
        hipStream_t cs = ctx->side[0];  // capture origin: a private stream, never the caller's
        HIP_OK(hipStreamWaitEvent(cs, ctx->ek0, 0));
        // Every value the captured launches read: the plans, the buffers
        // (addresses only: their contents are uploaded before each launch)
        // and the counter layout.  A batch with the same signature replays
        // the graph instantiated for the previous one.
        std::string sig;
        auto put = [&sig](const void *p, size_t n) { sig.append(reinterpret_cast<const char *>(p), n); };
        for (const NetPlan &pl : plans) {
            const size_t nid = pl.ids.size();
            put(&pl.net, sizeof(pl.net));
            put(&pl.lane, sizeof(pl.lane));
            put(&pl.v, sizeof(pl.v));
            put(&pl.total, sizeof(pl.total));
            put(&pl.limit, sizeof(pl.limit));
            put(&pl.batch, sizeof(pl.batch));
            put(&pl.job_off, sizeof(pl.job_off));
            put(&pl.n_jobs, sizeof(pl.n_jobs));
            put(&pl.grid, sizeof(pl.grid));
            put(&pl.packed, sizeof(pl.packed));
            put(&pl.vb_lo, sizeof(pl.vb_lo));
            put(&pl.vb_hi, sizeof(pl.vb_hi));
            put(&nid, sizeof(nid));
        }
        const void *bufs[] = {ctx->jobs.p, ctx->counters.p, ctx->recs.p, ctx->ties.p, ctx->u0.p, ctx->u0_index.p,
                              ctx->prop_ids.p, ctx->props.p, ctx->qcum.p, ctx->flags_dev};
        put(bufs, sizeof(bufs));
        const int64_t scal[] = {n_ctr, rec_slots, tcap, max_h1, resume, sc0, st0, sp0, fq0, (int64_t)NN};
        put(scal, sizeof(scal));
        const float tie_rel = o->near_tie_rel;
        put(&tie_rel, sizeof(tie_rel));
        put(&o->property, sizeof(o->property));
        put(&lut, sizeof(lut));
        put(&o->literal_v, sizeof(o->literal_v));
        if (ctx->graph_exec && sig == ctx->graph_sig) {
            const hipError_t le = hipGraphLaunch(ctx->graph_exec, cs);
            if (le == hipSuccess) {
                HIP_OK(hipEventRecord(ctx->side_ev[0], cs));
                HIP_OK(hipStreamWaitEvent(s, ctx->side_ev[0], 0));
            }
            HIP_OK(hipStreamSynchronize(cs));
            HIP_OK(le);
            ctx->graph_launches++;
            ctx->graph_reuses++;
            goto graph_done;
        }
        HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        ibmc_status cst = IBMC_OK;
        hipError_t ce = launch_fill_u64(ctr, n_ctr, 0ull, cs);
        if (ce == hipSuccess) ce = launch_fill_u64(ctr + 2, 1, ~0ull, cs);
        // every network's clean pass first, on the origin stream: in a branch
        // it would queue behind the other branches' persistent grids, which
        // hold every compute unit until they finish
        size_t id_off = 0;
        for (int i = 0; i < NN && ce == hipSuccess && cst == IBMC_OK; ++i) {
            cst = launch_clean(plans[i], id_off, cs);
            id_off += plans[i].ids.size();
        }
        if (ce == hipSuccess) ce = hipEventRecord(ctx->fork_ev, cs);
        for (int i = 0; i < NN && ce == hipSuccess && cst == IBMC_OK; ++i) {
            hipStream_t bs = (i == 0) ? cs : ctx->side[i];
            if (i > 0) ce = hipStreamWaitEvent(bs, ctx->fork_ev, 0);
            if (ce == hipSuccess) cst = launch_net(plans[i], bs);
            if (i > 0 && ce == hipSuccess && cst == IBMC_OK) {
                ce = hipEventRecord(ctx->side_ev[i], bs);
                if (ce == hipSuccess) ce = hipStreamWaitEvent(cs, ctx->side_ev[i], 0);
            }
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (cst != IBMC_OK) { if (graph) (void)hipGraphDestroy(graph); return cst; }
        HIP_OK(ce);
        HIP_OK(ee);
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_OK(ie);
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = exec;
        ctx->graph_sig.swap(sig);
        const hipError_t le = hipGraphLaunch(exec, cs);
        if (le == hipSuccess) {
            HIP_OK(hipEventRecord(ctx->side_ev[0], cs));
            HIP_OK(hipStreamWaitEvent(s, ctx->side_ev[0], 0));
        }
        HIP_OK(hipStreamSynchronize(cs));
        if (le != hipSuccess) {
            (void)hipGraphExecDestroy(ctx->graph_exec);
            ctx->graph_exec = nullptr;
            ctx->graph_sig.clear();
        }
        HIP_OK(le);
        ctx->graph_launches++;
    }
graph_done:
    if (!time_enum) {
        HIP_OK(hipEventRecord(ctx->ek1, s));
        timed = true;
    }
    float ms = 0.f;
    if (timed) {
        HIP_OK(hipEventSynchronize(ctx->ek1));
        HIP_OK(hipEventElapsedTime(&ms, ctx->ek0, ctx->ek1));
    }
    kernel_seconds = ms * 1e-3;
    launches = timed ? NN : 0;
    // gather
    std::vector<unsigned long long> h(n_ctr);
    HIP_OK(hipMemcpyAsync(h.data(), ctr, n_ctr * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    tie_total = (int64_t)h[3];
    if (next_cursor) {
        // every queue ticket handed out was worked through: chunks below
        // resume + tickets * batch are done
        *next_cursor = -1;
        if (NN == 1 && plans[0].net->act == IBMC_ACT_RELU_Q8 && !plans[0].lane) {
            const NetPlan &pl = plans[0];
            const int64_t done = std::min<int64_t>(pl.limit, resume + (int64_t)h[q0] * pl.batch);
            if (done < pl.total) *next_cursor = done;
        }
    }
    slot_cex.assign(h.begin() + sc0, h.begin() + st0);
    slot_ties.assign(h.begin() + st0, h.begin() + sp0);
    slot_points.assign(h.begin() + sp0, h.begin() + sp0 + B.n_slots);
    // exact total from the level counters; record slots handed out (with the
    // sentinels of partly used blocks) from the record counter
    rec_total = 0;
    for (int i = 0; i < n_props; ++i)
        for (int li : level_sel[i]) rec_total += (int64_t)slot_cex[B.slot_base[i] + li];
    const int64_t nr = std::min((int64_t)h[1], rec_slots), nt = std::min(tie_total, tcap);
    int max_k = 0;
    int64_t max_rank = 0;
    for (const EnumJob &J : jobs) {
        max_k = std::max(max_k, J.k);
        const int pid = J.prop;
        max_rank = std::max(max_rank, binom_small(props[pid].net->dims[0], J.k) * ipow64(props[pid].n_deltas, J.k));
    }
    int64_t nout = 0;
    IBMC_TRY(fetch_sorted(ctx, ctx->recs.as<DevRec>(), nr, cap, n_props - 1, max_k, max_rank, recs, direct_recs,
                          direct_dev, &nout));
    IBMC_TRY(fetch_sorted(ctx, ctx->ties.as<DevRec>(), nt, tcap, n_props - 1, max_k, max_rank, ties, direct_ties,
                          direct_dev, &nout));
    HIP_OK(hipMemcpyAsync(B.hprops.data(), ctx->props.p, n_props * sizeof(PropDev), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (ctx->flags_host[0]) return fail(IBMC_E_ABORTED, "check aborted");
    return IBMC_OK;
}

static bool rec_less(const CexRec &a, const CexRec &b) {
    if (a.prop != b.prop) return a.prop < b.prop;
    if (a.k != b.k) return a.k < b.k;
    return a.rank < b.rank;
}

ibmc_status check_batch_impl(ibmc_ctx *ctx, const ibmc_property *props_in, int32_t n_props, const ibmc_check_opts *o,
                             ibmc_check_summary *outs, ibmc_cex *cex_buf, ibmc_cex *tie_buf, bool images_on_device,
                             const int64_t *ball_r2) {
    clear_error();
    if (!ctx || !outs) return fail(IBMC_E_INVALID, "null ctx / outs");
    if (!props_in || n_props < 1) return fail(IBMC_E_INVALID, "no properties");
    // ball properties: m = 2 rd digits per pixel, no delta table
    std::vector<ibmc_property> pv(props_in, props_in + n_props);
    bool any_ball = false;
    for (int i = 0; i < n_props; ++i)
        if (ball_r2 && ball_r2[i] >= 0) {
            pv[i].n_deltas = 2 * ball_rd(ball_r2[i]);
            pv[i].deltas = nullptr;
            any_ball = true;
        }
    const ibmc_property *props = pv.data();
    IBMC_TRY(validate_props(props, n_props, o, ball_r2));
    if (o->cex_capacity > 0 && !cex_buf) return fail(IBMC_E_INVALID, "cex_buf is null with capacity > 0");
    if (o->near_tie_capacity > 0 && !tie_buf) return fail(IBMC_E_INVALID, "near_tie_buf is null with capacity > 0");
    const bool resumable = o->resume_cursor != 0 || o->chunk_budget != 0;
    if (o->resume_cursor < 0 || o->chunk_budget < 0) return fail(IBMC_E_INVALID, "negative resume cursor or budget");
    // the threshold literal and the table sigmoid: lane-per-point kernels only
    if (o->property != IBMC_PROPERTY_LABEL && o->property != IBMC_PROPERTY_LITERAL)
        return fail(IBMC_E_INVALID, "unknown property %d", o->property);
    if (o->sigmoid != IBMC_SIGMOID_EXP && o->sigmoid != IBMC_SIGMOID_TABLE)
        return fail(IBMC_E_INVALID, "unknown sigmoid %d", o->sigmoid);
    const bool literal = o->property == IBMC_PROPERTY_LITERAL, table = o->sigmoid == IBMC_SIGMOID_TABLE;
    if (literal || table) {
        if (resumable) return fail(IBMC_E_UNIMPL, "resume / budget with the literal or the table sigmoid");
        for (int i = 0; i < n_props; ++i) {
            const ibmc_mlp *net = props[i].net;
            if (net->act == IBMC_ACT_RELU_Q8) {
                if (table) return fail(IBMC_E_INVALID, "property %d: the table sigmoid is for float networks", i);
                if (!net->lane.ok)
                    return fail(IBMC_E_UNIMPL, "property %d: the literal runs on the lane kernel (1-2 hidden layers "
                                "of at most 64 units, at most 16 classes)", i);
                if (o->literal_v != std::floor(o->literal_v) || std::fabs(o->literal_v) > 2147483647.0)
                    return fail(IBMC_E_INVALID, "literal_v %g is not an int32 value (integer network)", o->literal_v);
            } else if (net->fd.kind != F32_LANE) {
                return fail(IBMC_E_UNIMPL, "property %d: the literal and the table sigmoid run on the float lane "
                            "kernel (hidden widths up to 128)", i);
            }
        }
    }
    if (resumable) {
        if (any_ball) return fail(IBMC_E_UNIMPL, "resume / budget with the L2-ball domain");
        if (o->stop_at_first) return fail(IBMC_E_UNIMPL, "resume / budget with stop_at_first");
        for (int i = 0; i < n_props; ++i)
            if (props[i].net != props[0].net || props[i].net->act != IBMC_ACT_RELU_Q8)
                return fail(IBMC_E_UNIMPL, "resume / budget need one integer network per call");
    }
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    ctx->flags_host[0] = 0;
    ctx->flags_host[1] = 0;
    HIP_OK(hipEventRecord(ctx->ev0, s));

    BatchState B;
    B.hprops.resize(n_props);
    B.level_k.resize(n_props);
    B.slot_base.resize(n_props);
    // images to the device
    std::vector<size_t> img_off(n_props, 0);
    size_t img_bytes = 0;
    if (!images_on_device) {
        for (int i = 0; i < n_props; ++i) {
            img_off[i] = img_bytes;
            img_bytes += (size_t)round_up(props[i].net->dims[0], 16);
        }
        IBMC_TRY(ctx->images.reserve(img_bytes));
        std::vector<uint8_t> staging(img_bytes, 0);
        for (int i = 0; i < n_props; ++i) memcpy(staging.data() + img_off[i], props[i].image, props[i].net->dims[0]);
        HIP_OK(hipMemcpyAsync(ctx->images.p, staging.data(), img_bytes, hipMemcpyHostToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    for (int i = 0; i < n_props; ++i) {
        PropDev &d = B.hprops[i];
        memset(&d, 0, sizeof(d));
        d.image = images_on_device ? props[i].image : ctx->images.as<uint8_t>() + img_off[i];
        d.m = props[i].n_deltas;
        d.n = props[i].net->dims[0];
        if (ball_r2 && ball_r2[i] >= 0) {
            d.ball = 1;
            d.ball_rd = ball_rd(ball_r2[i]);
            d.ball_r2 = (int32_t)ball_r2[i];
        } else {
            for (int j = 0; j < d.m; ++j) d.deltas[j] = props[i].deltas[j];
        }
        B.slot_base[i] = B.n_slots;
        for (int k = props[i].k_min; k <= props[i].k_max; k += props[i].k_step) B.level_k[i].push_back(k);
        B.n_slots += (int)B.level_k[i].size();
    }
    IBMC_TRY(ctx->props.upload(B.hprops.data(), B.hprops.size() * sizeof(PropDev), s));

    std::vector<std::vector<int>> done_levels(n_props);
    std::vector<unsigned long long> cex_acc(B.n_slots, 0), ties_acc(B.n_slots, 0), pts_acc(B.n_slots, 0);
    std::vector<CexRec> all_recs, all_ties;
    int64_t rec_total = 0, tie_total = 0;
    double ksec = 0.0;
    int nlaunch = 0;
    std::vector<bool> stopped(n_props, false);
    std::vector<int> next_level(n_props, 0);
    int64_t next_cursor = -1;
    ibmc_status st = IBMC_OK;
    int rounds = 0;
    while (true) {
        std::vector<std::vector<int>> sel(n_props);
        bool any = false;
        for (int i = 0; i < n_props; ++i) {
            if (stopped[i]) continue;
            if (o->stop_at_first) {
                if (next_level[i] < (int)B.level_k[i].size()) { sel[i].push_back(next_level[i]++); any = true; }
            } else {
                for (int li = next_level[i]; li < (int)B.level_k[i].size(); ++li) { sel[i].push_back(li); any = true; }
                next_level[i] = (int)B.level_k[i].size();
            }
        }
        if (!any) break;
        std::vector<unsigned long long> sc, stt, spt;
        std::vector<CexRec> r, t;
        int64_t rt = 0, tt = 0;
        double ks = 0;
        int nl = 0;
        // capacity left for this round
        ibmc_check_opts oo = *o;
        oo.cex_capacity = std::max<int64_t>(0, o->cex_capacity - (int64_t)all_recs.size());
        oo.near_tie_capacity = std::max<int64_t>(0, o->near_tie_capacity - (int64_t)all_ties.size());
        // a single round writes the sorted records straight into the caller's buffers
        const bool direct = !o->stop_at_first;
        st = run_levels(ctx, props, n_props, &oo, B, sel, images_on_device, sc, stt, spt, r, t, rt, tt, ks, nl,
                        direct ? reinterpret_cast<CexRec *>(cex_buf) : nullptr,
                        direct ? reinterpret_cast<CexRec *>(tie_buf) : nullptr, o->records_on_device != 0,
                        o->resume_cursor, o->chunk_budget, &next_cursor);
        rounds++;
        if (st < 0 && st != IBMC_E_ABORTED) return st;
        ksec += ks;
        nlaunch += nl;
        rec_total += rt;
        tie_total += tt;
        all_recs.insert(all_recs.end(), r.begin(), r.end());
        all_ties.insert(all_ties.end(), t.begin(), t.end());
        for (int i = 0; i < n_props; ++i)
            for (int li : sel[i]) {
                const int slot = B.slot_base[i] + li;
                cex_acc[slot] += sc[slot];
                ties_acc[slot] += stt[slot];
                pts_acc[slot] += spt[slot];
                done_levels[i].push_back(li);
                if (o->stop_at_first && sc[slot] > 0) stopped[i] = true;
            }
        if (st == IBMC_E_ABORTED) break;
    }
    HIP_OK(hipEventRecord(ctx->ev1, s));
    HIP_OK(hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_kernel_seconds = ksec;
    ctx->last_kernel_launches = nlaunch;

    if (rounds > 1) {  // every round comes back ordered; rounds interleave properties
        std::sort(all_recs.begin(), all_recs.end(), rec_less);
        std::sort(all_ties.begin(), all_ties.end(), rec_less);
    }
    if (o->stop_at_first) {
        const hipMemcpyKind kind = o->records_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
        if (cex_buf && !all_recs.empty())
            HIP_OK(hipMemcpy(cex_buf, all_recs.data(), all_recs.size() * sizeof(CexRec), kind));
        if (tie_buf && !all_ties.empty())
            HIP_OK(hipMemcpy(tie_buf, all_ties.data(), all_ties.size() * sizeof(CexRec), kind));
    }
    for (int i = 0; i < n_props; ++i) {
        ibmc_check_summary &S = outs[i];
        memset(&S, 0, sizeof(S));
        S.clean_label = B.hprops[i].label0;
        S.first_unsafe_k = -1;
        S.safe_up_to_k = -1;
        S.ttfc_seconds = -1.0;
        S.points_before_first = -1;
        S.seconds = ms * 1e-3;
        S.next_cursor = next_cursor;
        std::vector<int> lv = done_levels[i];
        std::sort(lv.begin(), lv.end());
        S.n_levels = (int32_t)lv.size();
        bool unsafe = false;
        for (size_t t = 0; t < lv.size(); ++t) {
            const int li = lv[t], k = B.level_k[i][li], slot = B.slot_base[i] + li;
            const bool q8 = props[i].net->act == IBMC_ACT_RELU_Q8;
            S.level_k[t] = k;
            // the L2 ball: the points of the level the kernel found inside it
            const bool ball = B.hprops[i].ball != 0;
            int64_t pts = ball ? (k == 0 ? 1 : (int64_t)pts_acc[slot])
                               : binom_small(props[i].net->dims[0], k) * ipow64(props[i].n_deltas, k);
            S.points[t] = pts;
            S.cex[t] = (k == 0) ? 0 : (int64_t)cex_acc[slot];
            S.ties[t] = (k == 0) ? (q8 && !literal ? B.hprops[i].tie0 : 0) : (int64_t)ties_acc[slot];
            S.points_total += pts;
            S.cex_total += S.cex[t];
            if (!q8) S.near_ties_total += S.ties[t];
            if (S.cex[t] > 0 && S.first_unsafe_k < 0) S.first_unsafe_k = k;
            if (S.cex[t] > 0) unsafe = true;
            if (!unsafe) S.safe_up_to_k = k;
        }
    }
    if (st == IBMC_E_ABORTED) return st;
    if (rec_total > o->cex_capacity || tie_total > o->near_tie_capacity) return IBMC_W_TRUNCATED;
    if (next_cursor >= 0) return IBMC_W_PARTIAL;
    return IBMC_OK;
}

}  // namespace ibmc

using namespace ibmc;

extern "C" ibmc_status ibmc_check_batch(ibmc_ctx *ctx, const ibmc_property *props, int32_t n_props,
                                        const ibmc_check_opts *opts, ibmc_check_summary *outs, ibmc_cex *cex_buf,
                                        ibmc_cex *near_tie_buf) {
    return check_batch_impl(ctx, props, n_props, opts, outs, cex_buf, near_tie_buf, false);
}

extern "C" ibmc_status ibmc_check_batch_dev(ibmc_ctx *ctx, const ibmc_property *props, int32_t n_props,
                                            const ibmc_check_opts *opts, ibmc_check_summary *outs, ibmc_cex *cex_buf,
                                            ibmc_cex *near_tie_buf) {
    return check_batch_impl(ctx, props, n_props, opts, outs, cex_buf, near_tie_buf, true);
}

extern "C" ibmc_status ibmc_check_property_dev(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                               int32_t n_pixels, const int16_t *delta_set, int32_t n_deltas,
                                               const ibmc_check_opts *opts, ibmc_check_summary *out, ibmc_cex *cex_buf,
                                               ibmc_cex *near_tie_buf) {
    clear_error();
    if (!net || !opts) return fail(IBMC_E_INVALID, "null net / opts");
    if (n_pixels != net->dims[0]) return fail(IBMC_E_INVALID, "n_pixels %d != network input %d", n_pixels, net->dims[0]);
    ibmc_property p{};
    p.net = net;
    p.image = image;
    p.deltas = delta_set;
    p.n_deltas = n_deltas;
    p.k_min = opts->k_min;
    p.k_max = opts->k_max;
    p.k_step = opts->k_step;
    return check_batch_impl(ctx, &p, 1, opts, out, cex_buf, near_tie_buf, true);
}

extern "C" ibmc_status ibmc_check_property(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image, int32_t n_pixels,
                                           const int16_t *delta_set, int32_t n_deltas, const ibmc_check_opts *opts,
                                           ibmc_check_summary *out, ibmc_cex *cex_buf, ibmc_cex *near_tie_buf) {
    clear_error();
    if (!net || !opts) return fail(IBMC_E_INVALID, "null net / opts");
    if (n_pixels != net->dims[0]) return fail(IBMC_E_INVALID, "n_pixels %d != network input %d", n_pixels, net->dims[0]);
    ibmc_property p{};
    p.net = net;
    p.image = image;
    p.deltas = delta_set;
    p.n_deltas = n_deltas;
    p.k_min = opts->k_min;
    p.k_max = opts->k_max;
    p.k_step = opts->k_step;
    return check_batch_impl(ctx, &p, 1, opts, out, cex_buf, near_tie_buf, false);
}

extern "C" int32_t ibmc_ball_digits(int64_t radius_sq) { return radius_sq < 0 ? 0 : ball_rd(radius_sq); }

extern "C" ibmc_status ibmc_check_ball(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image, int32_t n_pixels,
                                       int64_t radius_sq, const ibmc_check_opts *opts, ibmc_check_summary *out,
                                       ibmc_cex *cex_buf) {
    clear_error();
    if (!net || !opts) return fail(IBMC_E_INVALID, "null net / opts");
    if (n_pixels != net->dims[0]) return fail(IBMC_E_INVALID, "n_pixels %d != network input %d", n_pixels, net->dims[0]);
    if (radius_sq < 0) return fail(IBMC_E_INVALID, "negative radius_sq");
    ibmc_property p{};
    p.net = net;
    p.image = image;
    p.k_min = opts->k_min;
    p.k_max = opts->k_max;
    p.k_step = opts->k_step;
    return check_batch_impl(ctx, &p, 1, opts, out, cex_buf, nullptr, false, &radius_sq);
}

extern "C" ibmc_status ibmc_check_ball_batch(ibmc_ctx *ctx, const ibmc_ball_property *props, int32_t n_props,
                                             const ibmc_check_opts *opts, ibmc_check_summary *outs, ibmc_cex *cex_buf) {
    clear_error();
    if (!props || n_props < 1) return fail(IBMC_E_INVALID, "no properties");
    std::vector<ibmc_property> pv(n_props);
    std::vector<int64_t> r2(n_props);
    for (int i = 0; i < n_props; ++i) {
        if (props[i].radius_sq < 0) return fail(IBMC_E_INVALID, "property %d: negative radius_sq", i);
        pv[i] = ibmc_property{};
        pv[i].net = props[i].net;
        pv[i].image = props[i].image;
        pv[i].k_min = props[i].k_min;
        pv[i].k_max = props[i].k_max;
        pv[i].k_step = props[i].k_step;
        r2[i] = props[i].radius_sq;
    }
    return check_batch_impl(ctx, pv.data(), n_props, opts, outs, cex_buf, nullptr, false, r2.data());
}

extern "C" ibmc_status ibmc_eval_points_f32(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                            const int16_t *delta_set, int32_t n_deltas, const int32_t *ks,
                                            const int64_t *ranks, int64_t n, float *logits, int32_t *labels,
                                            float *margins, int32_t *clean_label) {
    clear_error();
    if (!ctx || !net || !image || !delta_set) return fail(IBMC_E_INVALID, "null ctx / net / image / deltas");
    if (net->act != IBMC_ACT_SIGMOID_F32) return fail(IBMC_E_UNIMPL, "float networks only (integer ones: ibmc_replay)");
    if (n_deltas < 1 || n_deltas > kMaxDeltas) return fail(IBMC_E_INVALID, "n_deltas %d", n_deltas);
    if (n < 0 || (n > 0 && (!ks || !ranks))) return fail(IBMC_E_INVALID, "bad point list");
    const int np = net->dims[0];
    for (int64_t t = 0; t < n; ++t) {
        if (ks[t] < 0 || ks[t] > std::min(np, kMaxK)) return fail(IBMC_E_INVALID, "point %lld: k = %d", (long long)t, ks[t]);
        const int64_t pts = binom_small(np, ks[t]) * ipow64(n_deltas, ks[t]);
        if (ranks[t] < 0 || ranks[t] >= pts)
            return fail(IBMC_E_INVALID, "point %lld: rank %lld outside [0, %lld)", (long long)t, (long long)ranks[t],
                        (long long)pts);
    }
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int hp1 = net->fd.HP[1], nc = net->dims[net->L];
    IBMC_TRY(ctx->images.upload(image, (size_t)np, s));
    PropDev pd;
    memset(&pd, 0, sizeof(pd));
    pd.image = ctx->images.as<uint8_t>();
    pd.m = n_deltas;
    pd.n = np;
    for (int i = 0; i < n_deltas; ++i) pd.deltas[i] = delta_set[i];
    IBMC_TRY(ctx->props.upload(&pd, sizeof(pd), s));
    const int32_t zero = 0;
    IBMC_TRY(ctx->prop_ids.upload(&zero, 4, s));
    IBMC_TRY(ctx->u0.reserve((size_t)hp1 * 4));
    HIP_OK(launch_clean_f32(net->fd, ctx->props.as<PropDev>(), ctx->prop_ids.as<int32_t>(), 1, ctx->u0.as<float>(), hp1,
                            s));
    // point list and outputs in one device buffer
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t o_r = al(nn * 4), o_z = o_r + al(nn * 8), o_l = o_z + al(nn * nc * 4), o_m = o_l + al(nn * 4);
    IBMC_TRY(ctx->recout.reserve(o_m + al(nn * 4)));
    char *B = ctx->recout.as<char>();
    if (n > 0) {
        HIP_OK(hipMemcpyAsync(B, ks, n * 4, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(B + o_r, ranks, n * 8, hipMemcpyHostToDevice, s));
        F32EvalParams E{};
        E.net = net->fd;
        E.props = ctx->props.as<PropDev>();
        E.ks = reinterpret_cast<const int32_t *>(B);
        E.ranks = reinterpret_cast<const int64_t *>(B + o_r);
        E.n = n;
        E.u0f = ctx->u0.as<float>();
        E.u0_stride = hp1;
        E.logits = reinterpret_cast<float *>(B + o_z);
        E.labels = reinterpret_cast<int32_t *>(B + o_l);
        E.margins = reinterpret_cast<float *>(B + o_m);
        HIP_OK(launch_eval_f32(E, s));
        if (logits) HIP_OK(hipMemcpyAsync(logits, B + o_z, (size_t)n * nc * 4, hipMemcpyDeviceToHost, s));
        if (labels) HIP_OK(hipMemcpyAsync(labels, B + o_l, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        if (margins) HIP_OK(hipMemcpyAsync(margins, B + o_m, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    }
    PropDev back;
    HIP_OK(hipMemcpyAsync(&back, ctx->props.p, sizeof(back), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (clean_label) *clean_label = back.label0;
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_set_variant(ibmc_ctx *ctx, const ibmc_mlp *net, const char *variant) {
    clear_error();
    if (!ctx || !net) return fail(IBMC_E_INVALID, "null argument");
    ibmc_mlp *m = const_cast<ibmc_mlp *>(net);
    if (!variant) { m->forced_variant.clear(); return IBMC_OK; }
    if (std::string(variant) == kLaneVariantName) {
        if (!net->lane.ok) return fail(IBMC_E_INVALID, "variant %s does not match the network", variant);
        m->forced_variant = variant;
        return IBMC_OK;
    }
    int nv = 0;
    const EnumVariant *vs = enum_variants(&nv);
    for (int i = 0; i < nv; ++i)
        if (std::string(variant) == vs[i].name) {
            if (!variant_matches(vs[i], net))
                return fail(IBMC_E_INVALID, "variant %s does not match the network", variant);
            m->forced_variant = variant;
            return IBMC_OK;
        }
    return fail(IBMC_E_INVALID, "unknown variant %s", variant);
}

extern "C" ibmc_status ibmc_chosen_variant(ibmc_ctx *ctx, const ibmc_mlp *net, char *out, int64_t cap) {
    clear_error();
    if (!ctx || !net || !out || cap < 1) return fail(IBMC_E_INVALID, "null argument");
    std::string name;
    if (net->act != IBMC_ACT_RELU_Q8) {
        name = "f32";
    } else if (use_lane(ctx, net, true)) {
        name = kLaneVariantName;
    } else {
        const EnumVariant *v = pick_variant(ctx, net);
        if (!v) return fail(IBMC_E_UNIMPL, "no enumeration kernel for network %s", shape_key(net).c_str());
        name = v->name;
    }
    const size_t n = std::min<size_t>(name.size(), (size_t)cap - 1);
    memcpy(out, name.data(), n);
    out[n] = 0;
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_graph_stats(ibmc_ctx *ctx, int64_t *launches, int64_t *reuses) {
    clear_error();
    if (!ctx) return fail(IBMC_E_INVALID, "ctx is null");
    if (launches) *launches = ctx->graph_launches;
    if (reuses) *reuses = ctx->graph_reuses;
    return IBMC_OK;
}

// Tuning table: one "shape key": "variant name" pair per network shape, as
// a flat JSON object.
extern "C" ibmc_status ibmc_tune_save(ibmc_ctx *ctx, const char *path) {
    clear_error();
    if (!ctx || !path) return fail(IBMC_E_INVALID, "null ctx / path");
    FILE *f = fopen(path, "w");
    if (!f) return fail(IBMC_E_INVALID, "cannot write %s", path);
    fprintf(f, "{");
    bool first = true;
    for (const auto &kv : ctx->tuned) {
        fprintf(f, "%s\n  \"%s\": \"%s\"", first ? "" : ",", kv.first.c_str(), kv.second.c_str());
        first = false;
    }
    fprintf(f, "\n}\n");
    const bool ok = fclose(f) == 0;
    return ok ? IBMC_OK : fail(IBMC_E_INVALID, "cannot write %s", path);
}

extern "C" ibmc_status ibmc_tune_load(ibmc_ctx *ctx, const char *path, int32_t *n_loaded) {
    clear_error();
    if (!ctx || !path) return fail(IBMC_E_INVALID, "null ctx / path");
    FILE *f = fopen(path, "r");
    if (!f) return fail(IBMC_E_INVALID, "cannot read %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    // the quoted strings in order: key, value, key, value, ...
    std::vector<std::string> strs;
    for (size_t i = 0; i < text.size(); ++i) {
        if (text[i] != '"') continue;
        const size_t j = text.find('"', i + 1);
        if (j == std::string::npos) return fail(IBMC_E_INVALID, "%s: unterminated string", path);
        strs.push_back(text.substr(i + 1, j - i - 1));
        i = j;
    }
    if (strs.size() % 2) return fail(IBMC_E_INVALID, "%s: a key without a value", path);
    int32_t n = 0;
    for (size_t i = 0; i < strs.size(); i += 2, ++n) ctx->tuned[strs[i]] = strs[i + 1];
    if (n_loaded) *n_loaded = n;
    return IBMC_OK;
}

// ---------------------------------------------------------------------------
// ordered search: the same enumeration visited in plain order or in the
// proposer's order (level 1 by score, level 2 by shells), with the time to
// the first counterexample observed on the host
// ---------------------------------------------------------------------------

namespace ibmc {

ibmc_status ordered_search(ibmc_ctx *ctx, const ibmc_mlp *net, const ibmc_proposer *p, const uint8_t *image, int rows,
                           int cols, const int16_t *deltas, int m, const ibmc_check_opts *o, ibmc_check_summary *out,
                           ibmc_cex *cex_buf) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (o->property != IBMC_PROPERTY_LABEL || o->sigmoid != IBMC_SIGMOID_EXP)
        return fail(IBMC_E_UNIMPL, "the ordered search checks the label property with the exponential sigmoid");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int n = net->dims[0];
    const int64_t N1 = (int64_t)n * m;
    const EnumVariant *v = pick_variant(ctx, net);
    if (!v) return fail(IBMC_E_UNIMPL, "no enumeration kernel for network %s", shape_key(net).c_str());
    const int CH = v->chunk;
    ctx->flags_host[0] = 0;
    ctx->flags_host[1] = 0;
    HIP_OK(hipEventRecord(ctx->ev0, s));
    // property
    PropDev pd;
    memset(&pd, 0, sizeof(pd));
    pd.m = m;
    pd.n = n;
    for (int i = 0; i < m; ++i) pd.deltas[i] = deltas[i];
    IBMC_TRY(ctx->u0.reserve((size_t)net->qd.H[1] * 4));
    std::vector<int32_t> order;
    // jobs: one per level >= 1
    std::vector<int> lv;
    for (int k = o->k_min; k <= o->k_max; ++k) lv.push_back(k);
    std::vector<EnumJob> jobs;
    std::vector<int64_t> qc, scum;
    int64_t total = 0;
    for (size_t li = 0; li < lv.size(); ++li) {
        const int k = lv[li];
        if (k == 0) continue;
        EnumJob J{};
        J.prop = 0;
        J.k = k;
        J.slot = (int)li;
        J.chunk_begin = total;
        J.wseg = 1;  // rank order
        int64_t ch = 0;
        if (!p) {
            J.mode = SEG_PLAIN;
            ch = plan_plain_level(n, m, k, CH, 1, qc);
        } else if (k == 1) {
            J.mode = SEG_LIST1;
            ch = ceil_div(N1, CH);
        } else {
            J.mode = SEG_SHELL;
            // chunks before shell t (shells t >= 1 have t candidates); the
            // table depends on (N1, CH) only and stays on the device
            if (ctx->shell_cum_n != N1 || ctx->shell_cum_ch != CH) {
                scum.assign(N1, 0);
                for (int64_t t = 1; t < N1; ++t) scum[t] = (t >= 2 ? scum[t - 1] + ceil_div(t - 1, CH) : 0);
            }
            int64_t last = 0;  // scum[N1 - 1]
            for (int64_t t = 2; t < N1; ++t) last += ceil_div(t - 1, CH);
            ch = last + ceil_div(N1 - 1, CH);
        }
        J.chunk_end = total + ch;
        total += ch;
        jobs.push_back(J);
    }
    const int n_slots = (int)lv.size();
    const int64_t n_ctr = 8 + 2 * (int64_t)n_slots;
    IBMC_TRY(ctx->counters.reserve(n_ctr * 8));
    unsigned long long *ctr = ctx->counters.as<unsigned long long>();
    HIP_OK(launch_fill_u64(ctr, n_ctr, 0ull, s));
    HIP_OK(launch_fill_u64(ctr + 2, 1, ~0ull, s));
    const int64_t cap = o->cex_capacity;
    // record slots: the capacity plus one partly used block per wave
    int occ = 0;
    const int64_t lds = enum_lds_bytes(*v, net->qd);
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, v->fn, 256, (size_t)lds));
    if (occ < 1) return fail(IBMC_E_UNIMPL, "variant %s does not fit", v->name);
    const int64_t grid = std::min<int64_t>((int64_t)ctx->n_cu * occ, std::max<int64_t>(1, total));
    const int64_t rec_slots = cap + grid * 4 * kRecBlock;
    IBMC_TRY(ctx->recs.reserve((size_t)std::max<int64_t>(rec_slots, 1) * sizeof(DevRec)));
    if (!scum.empty()) {
        IBMC_TRY(ctx->shell_cum.upload(scum.data(), scum.size() * 8, s));
        ctx->shell_cum_n = N1;
        ctx->shell_cum_ch = CH;
    }
    if (p) IBMC_TRY(ctx->order.reserve((size_t)N1 * 4));
    // the per-call inputs in one copy from pinned memory:
    // image | property | property id 0 | u0 index 0 | jobs | plain prefix table
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_pd = al((size_t)n), o_ids = o_pd + al(sizeof(PropDev)), o_u0i = o_ids + 256, o_jobs = o_u0i + 256;
    const size_t o_qc = o_jobs + al(jobs.size() * sizeof(EnumJob)), stage_n = o_qc + qc.size() * 8;
    if (ctx->stage_pending) HIP_OK(hipEventSynchronize(ctx->stage_ev));  // the previous copy has read the staging
    ctx->stage_pending = false;
    if (ctx->stage_host_bytes < stage_n) {
        if (ctx->stage_host) HIP_OK(hipHostFree(ctx->stage_host));
        ctx->stage_host = nullptr;
        ctx->stage_host_bytes = 0;
        const size_t want = std::max<size_t>(stage_n, 64 << 10);
        void *hp = nullptr;
        HIP_OK(hipHostMalloc(&hp, want, hipHostMallocDefault));
        ctx->stage_host = reinterpret_cast<char *>(hp);
        ctx->stage_host_bytes = want;
    }
    IBMC_TRY(ctx->stage_dev.reserve(stage_n));
    char *const SH = ctx->stage_host;
    char *const SD = ctx->stage_dev.as<char>();
    PropDev *const d_props = reinterpret_cast<PropDev *>(SD + o_pd);
    const int32_t *const d_ids = reinterpret_cast<const int32_t *>(SD + o_ids);
    const int32_t *const d_u0i = reinterpret_cast<const int32_t *>(SD + o_u0i);
    pd.image = reinterpret_cast<const uint8_t *>(SD);
    for (auto &J : jobs) {
        J.qcum = (J.mode == SEG_PLAIN && J.k >= 2) ? reinterpret_cast<const int64_t *>(SD + o_qc) : nullptr;
        J.order = p ? ctx->order.as<int32_t>() : nullptr;
        J.shell_cum = (J.mode == SEG_SHELL) ? ctx->shell_cum.as<int64_t>() : nullptr;
    }
    memcpy(SH, image, (size_t)n);
    memcpy(SH + o_pd, &pd, sizeof(pd));
    memset(SH + o_ids, 0, 4);
    memset(SH + o_u0i, 0, 4);
    if (!jobs.empty()) memcpy(SH + o_jobs, jobs.data(), jobs.size() * sizeof(EnumJob));
    if (!qc.empty()) memcpy(SH + o_qc, qc.data(), qc.size() * 8);
    HIP_OK(hipMemcpyAsync(SD, SH, stage_n, hipMemcpyHostToDevice, s));
    HIP_OK(hipEventRecord(ctx->stage_ev, s));
    ctx->stage_pending = true;
    // every upload is done: the clean pass, the proposer's ordering and the
    // enumeration are queued back to back, with no host wait in between
    HIP_OK(launch_clean_q8(net->qd, d_props, d_ids, 1, ctx->u0.as<int32_t>(),
                           net->qd.H[1], s));
    // order of the candidates
    if (p) {
        PropCand pc;
        pc.m = m;
        pc.dmax = 0;
        for (int i = 0; i < m; ++i) { pc.deltas[i] = deltas[i]; pc.dmax = std::max(pc.dmax, std::abs((int)deltas[i])); }
        const PropParams PP = prop_views(p);
        // the context's buffers (no allocation once sized); the clean pass
        // above has left the first-layer potentials in u0: one launch for
        // live norms, features and scores, one for the order
        IBMC_TRY(ctx->prop_scores.reserve((size_t)N1 * 4));
        HIP_OK(launch_prop_fused(net->qd, pd.image, ctx->u0.as<int32_t>(), rows, cols, pc, PP,
                                 ctx->prop_scores.as<float>(), s));
        HIP_OK(launch_prop_sort(ctx->prop_scores.as<float>(), (int)N1, ctx->order.as<int32_t>(), s));
    }
    double ttfc = -1.0;
    int64_t rec_total = 0;
    std::vector<unsigned long long> h(n_ctr);
    if (!jobs.empty() && total > 0) {
        EnumParams P{};
        P.net = net->qd;
        P.jobs = reinterpret_cast<const EnumJob *>(SD + o_jobs);
        P.n_jobs = (int32_t)jobs.size();
        P.total_chunks = total;
        // visit in order: the first four rounds of the grid are single
        // chunks dealt out statically, one per wave and round (the early
        // positions, where a first counterexample usually sits, are visited
        // one chunk at a time without a queue atomic), later queue tickets
        // contiguous batches (the same size rule as the unordered search)
        P.single = std::min<int64_t>(total, grid * 4 * 4);
        P.batch = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, (total - P.single) / (grid * 32)));
        P.props = d_props;
        P.queue = ctr + 0;
        P.rec_count = ctr + 1;
        P.first_chunk = ctr + 2;
        P.stop_flag = reinterpret_cast<volatile int32_t *>(ctr + 4);
        P.abort_host = ctx->flags_dev;
        P.hit_host = ctx->flags_dev + 1;
        P.stop_on_first = o->stop_at_first ? 1 : 0;
        P.rec_cap = rec_slots;
        P.recs = ctx->recs.as<DevRec>();
        P.slot_cex = ctr + 8;
        P.slot_ties = ctr + 8 + n_slots;
        P.track_first = 1;
        int maxe = 0;
        for (int i = 0; i < m; ++i) maxe = std::max(maxe, std::min(255, std::abs((int)deltas[i])));
        const int64_t M2 = (int64_t)net->qd.f1 * maxe * net->qd.maxw1;
        P.packed = (net->qd.f1 > 0 && M2 <= 8191 && !ctx->force_int32_layer1) ? 1 : 0;
        P.vb_lo = (int32_t)(-16385 - M2);
        P.vb_hi = (int32_t)(16384 + M2);
        HIP_OK(hipEventRecord(ctx->ek0, s));
        HIP_OK(launch_enum_q8(*v, (int)grid, P, ctx->u0.as<int32_t>(), net->qd.H[1], d_u0i, s));
        HIP_OK(hipEventRecord(ctx->ek1, s));
        // watch the host-mapped first-hit flag while the kernel runs
        while (true) {
            if (ttfc < 0 && __atomic_load_n(&ctx->flags_host[1], __ATOMIC_ACQUIRE))
                ttfc = std::chrono::duration<double>(clk::now() - t0).count();
            const hipError_t q = hipEventQuery(ctx->ek1);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) HIP_OK(q);
        }
        if (ttfc < 0 && __atomic_load_n(&ctx->flags_host[1], __ATOMIC_ACQUIRE))
            ttfc = std::chrono::duration<double>(clk::now() - t0).count();
        float kms = 0.f;
        HIP_OK(hipEventElapsedTime(&kms, ctx->ek0, ctx->ek1));
        ctx->last_kernel_seconds = kms * 1e-3;
        ctx->last_kernel_launches = 1;
    }
    HIP_OK(hipMemcpyAsync(h.data(), ctr, n_ctr * 8, hipMemcpyDeviceToHost, s));
    PropDev back;
    HIP_OK(hipMemcpyAsync(&back, d_props, sizeof(back), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    rec_total = 0;
    for (int li = 0; li < n_slots; ++li) rec_total += (int64_t)h[8 + li];
    const int64_t nr = std::min((int64_t)h[1], rec_slots);
    std::vector<CexRec> recs;
    int64_t nkept = 0;
    IBMC_TRY(fetch_sorted(ctx, ctx->recs.as<DevRec>(), nr, cap, 0, o->k_max, binom_small(n, 2) * m * m, recs, nullptr,
                          false, &nkept));
    if (p) {
        order.resize(N1);
        HIP_OK(hipMemcpy(order.data(), ctx->order.p, N1 * 4, hipMemcpyDeviceToHost));
    }
    HIP_OK(hipEventRecord(ctx->ev1, s));
    HIP_OK(hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (cex_buf && nkept)
        HIP_OK(hipMemcpy(cex_buf, recs.data(), nkept * sizeof(CexRec),
                         o->records_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));

    // position of every record in the visiting order (hardware independent)
    int64_t first_pos = -1;
    {
        const bool has1 = std::find(lv.begin(), lv.end(), 1) != lv.end();
        const int64_t off2 = has1 ? N1 : 0;
        std::vector<int64_t> pos_of(N1, 0), shell_valid_before, same_pix_before;
        std::vector<std::vector<int32_t>> pix_positions;
        if (p) {
            for (int64_t t = 0; t < N1; ++t) pos_of[order[t]] = t;
            // valid (distinct-pixel) points in shells before t, and per pixel the sorted positions
            pix_positions.assign(n, {});
            shell_valid_before.assign(N1 + 1, 0);
            for (int64_t t = 0; t < N1; ++t) {
                const int px = order[t] / m;
                const int64_t same = (int64_t)pix_positions[px].size();
                shell_valid_before[t + 1] = shell_valid_before[t] + (t - same);
                pix_positions[px].push_back((int32_t)t);
            }
        }
        std::vector<int64_t> rowstart(n + 1, 0);   // plain level 2: points before first pixel q
        for (int q = 0; q < n; ++q) rowstart[q + 1] = rowstart[q] + (int64_t)(n - 1 - q) * m * m;
        // pairs with first pixel below a: the lex index of pair (a, b) is
        // pairs_before[a] + b - a - 1
        std::vector<int64_t> pairs_before(n + 1, 0);
        for (int a = 0; a < n; ++a) pairs_before[a + 1] = pairs_before[a] + (n - 1 - a);
        int first_p0 = -1;
        for (const CexRec &r : recs) {
            int64_t pos = -1;
            int px[2] = {0, 0}, dg[2] = {0, 0};
            int64_t mk = (r.k == 1) ? m : (int64_t)m * m;
            const int64_t sidx = r.rank / mk;  // lex index of the pixel subset
            if (r.k == 1) {
                px[0] = (int)sidx;
            } else {
                px[0] = (int)(std::upper_bound(pairs_before.begin(), pairs_before.end(), sidx) - pairs_before.begin()) - 1;
                px[1] = (int)(sidx - pairs_before[px[0]]) + px[0] + 1;
            }
            int64_t d = r.rank % mk;
            for (int j = r.k - 1; j >= 0; --j) { dg[j] = (int)(d % m); d /= m; }
            // plain order: records come in rank order, level 1 (visited first)
            // before level 2, and within level 2 the visiting order starts with
            // the first pixel, so only the records sharing the first record's
            // first pixel can hold the earliest position
            // level 1 is visited before level 2 (its positions lie below
            // off2) and the records come sorted by (k, rank): once a level-1
            // record has a position, no level-2 record can come earlier
            if (has1 && r.k >= 2 && first_pos >= 0 && first_pos < off2) break;
            if (!p) {
                if (first_pos >= 0 && r.k == 1) continue;
                if (r.k == 2) {
                    if (first_pos >= 0 && first_p0 < 0) break;  // a level-1 record came first
                    if (first_p0 < 0) first_p0 = px[0];
                    else if (px[0] != first_p0) break;
                }
            }
            if (r.k == 1) {
                const int cand = px[0] * m + dg[0];
                pos = p ? pos_of[cand] : cand;
            } else if (!p) {
                pos = off2 + rowstart[px[0]] + (int64_t)dg[0] * (n - 1 - px[0]) * m + (int64_t)(px[1] - px[0] - 1) * m + dg[1];
            } else {
                const int64_t a = pos_of[px[0] * m + dg[0]], b = pos_of[px[1] * m + dg[1]];
                const int64_t t = std::max(a, b), jp = std::min(a, b);
                const int hp = order[t] / m;
                const auto &lst = pix_positions[hp];
                const int64_t same_before_j = std::lower_bound(lst.begin(), lst.end(), (int32_t)jp) - lst.begin();
                pos = off2 + shell_valid_before[t] + (jp - same_before_j);
            }
            if (first_pos < 0 || pos < first_pos) first_pos = pos;
        }
    }
    ibmc_check_summary &S = *out;
    memset(&S, 0, sizeof(S));
    S.next_cursor = -1;
    S.clean_label = back.label0;
    S.first_unsafe_k = -1;
    S.safe_up_to_k = -1;
    S.n_levels = (int32_t)lv.size();
    bool unsafe = false;
    for (size_t li = 0; li < lv.size(); ++li) {
        const int k = lv[li];
        S.level_k[li] = k;
        S.points[li] = binom_small(n, k) * ipow64(m, k);
        S.cex[li] = k == 0 ? 0 : (int64_t)h[8 + li];
        S.ties[li] = k == 0 ? back.tie0 : (int64_t)h[8 + n_slots + li];
        S.points_total += S.points[li];
        S.cex_total += S.cex[li];
        if (S.cex[li] > 0 && S.first_unsafe_k < 0) S.first_unsafe_k = k;
        if (S.cex[li] > 0) unsafe = true;
        if (!unsafe) S.safe_up_to_k = k;
    }
    S.seconds = ms * 1e-3;
    S.ttfc_seconds = ttfc;
    S.points_before_first = first_pos;
    if (rec_total > cap) return IBMC_W_TRUNCATED;
    return IBMC_OK;
}

}  // namespace ibmc

// ---------------------------------------------------------------------------
// autotuner: time every compiled instance that fits the network's shape on a
// synthetic property (seeded image, deltas +-8, +-16, ...) at level k, keep
// the fastest for this shape in the context
// ---------------------------------------------------------------------------

extern "C" ibmc_status ibmc_autotune(ibmc_ctx *ctx, const ibmc_mlp *net, int32_t k, int32_t n_deltas, char *json_out,
                                     int64_t json_cap) {
    clear_error();
    if (!ctx || !net) return fail(IBMC_E_INVALID, "null argument");
    if (net->act != IBMC_ACT_RELU_Q8) return fail(IBMC_E_UNIMPL, "tuning covers integer networks");
    if (k < 1 || k > 3 || n_deltas < 1 || n_deltas > kMaxDeltas) return fail(IBMC_E_INVALID, "k %d / n_deltas %d", k, n_deltas);
    const int n = net->dims[0];
    std::vector<uint8_t> img(n);
    uint64_t st = 0x7475ull;
    for (int i = 0; i < n; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        img[i] = (uint8_t)(st >> 56);
    }
    std::vector<int16_t> D(n_deltas);
    for (int i = 0; i < n_deltas; ++i) D[i] = (int16_t)((i % 2 ? 1 : -1) * 8 * (1 + i / 2));
    int nv = 0;
    const EnumVariant *vs = enum_variants(&nv);
    ibmc_mlp *m = const_cast<ibmc_mlp *>(net);
    const std::string saved = m->forced_variant;
    std::string json = "{\"shape\": \"" + shape_key(net) + "\", \"k\": " + std::to_string(k) + ", \"variants\": [";
    double best_t = 1e30;
    std::string best;
    bool first = true;
    ibmc_check_opts o{};
    o.k_min = k;
    o.k_max = k;
    o.k_step = 1;
    o.cex_capacity = 0;
    // one candidate: the best of three timed checks with it forced
    auto time_candidate = [&](const char *name, int occ) -> ibmc_status {
        m->forced_variant = name;
        ibmc_check_summary S;
        double tmin = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            ibmc_status rc = ibmc_check_property(ctx, net, img.data(), n, D.data(), n_deltas, &o, &S, nullptr, nullptr);
            if (rc < 0 && rc != IBMC_W_TRUNCATED) return rc;
            tmin = std::min(tmin, ctx->last_kernel_seconds);
        }
        const double pps = tmin > 0 ? (double)S.points_total / tmin : 0.0;
        if (!first) json += ", ";
        first = false;
        json += "{\"name\": \"" + std::string(name) + "\", \"kernel_s\": " + std::to_string(tmin) +
                ", \"points_per_s\": " + std::to_string(pps) + ", \"occupancy\": " + std::to_string(occ) + "}";
        if (tmin < best_t) { best_t = tmin; best = name; }
        return IBMC_OK;
    };
    for (int i = 0; i < nv; ++i) {
        const EnumVariant &v = vs[i];
        if (!variant_matches(v, net)) continue;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, v.fn, 256, (size_t)enum_lds_bytes(v, net->qd)) !=
                hipSuccess || occ < 1)
            continue;
        const ibmc_status rc = time_candidate(v.name, occ);
        if (rc < 0) { m->forced_variant = saved; return rc; }
    }
    if (net->lane.ok) {
        const ibmc_status rc = time_candidate(kLaneVariantName, lane_enum_grid(net->lane, ctx->n_cu) / ctx->n_cu);
        if (rc < 0) { m->forced_variant = saved; return rc; }
    }
    m->forced_variant = saved;
    if (best.empty()) return fail(IBMC_E_UNIMPL, "no kernel instance for %s", shape_key(net).c_str());
    ctx->tuned[shape_key(net)] = best;
    json += "], \"best\": \"" + best + "\"}";
    if (json_out && json_cap > 0) {
        const size_t nbytes = std::min<size_t>(json.size(), (size_t)json_cap - 1);
        memcpy(json_out, json.data(), nbytes);
        json_out[nbytes] = 0;
    }
    return IBMC_OK;
}
