// Allocation-free variant of ibmc_check_property for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops).  Every device buffer of the call is carved, in order, from one
// fixed array that the library holds per device for the life of the
// process; nothing is allocated or freed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "ibmc_host.h"

namespace ibmc {

// The fixed scratch of the allocation-free entry point.  Host code never
// passes this name to a kernel or a copy: it uses the device address that
// noalloc_setup looks up per device.
static __device__ __align__(256) uint8_t scratch[IBMC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

ibmc_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(IBMC_E_INVALID, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return IBMC_OK;
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != device) return fail(IBMC_E_INVALID, "scratch lookup needs device %d current (is %d)", device, cur);
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(IBMC_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_ptr[device] = ptr;
    return IBMC_OK;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Upper bound of the bytes one call carves (every buffer the check driver
// reserves for a single property, each 256-byte aligned).
static ibmc_status scratch_need(ibmc_ctx *ctx, const ibmc_mlp *net, int32_t n_deltas, const ibmc_check_opts *o,
                                size_t *need) {
    const int n = net->dims[0];
    int levels = 0;
    for (int k = o->k_min; k <= o->k_max; k += o->k_step) ++levels;
    const int64_t cap = o->cex_capacity, tcap = o->near_tie_capacity;
    int64_t rec_slots = cap;
    int64_t h1 = 64;
    if (net->act == IBMC_ACT_RELU_Q8 && use_lane(ctx, net, o->resume_cursor == 0 && o->chunk_budget == 0)) {
        h1 = std::max<int64_t>(h1, net->qd.H[1]);    // the lane kernel writes records without spare blocks
    } else if (net->act == IBMC_ACT_RELU_Q8) {
        const EnumVariant *v = pick_variant(ctx, net);
        if (!v) return fail(IBMC_E_UNIMPL, "no enumeration kernel for network %s", shape_key(net).c_str());
        int occ = 0;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, v->fn, 256, (size_t)enum_lds_bytes(*v, net->qd)));
        rec_slots += (int64_t)ctx->n_cu * std::max(occ, 1) * 4 * kRecBlock;
        h1 = std::max<int64_t>(h1, net->qd.H[1]);
    } else {
        h1 = std::max<int64_t>(h1, net->dims[1]);
    }
    (void)n_deltas;
    size_t b = 0;
    b += al256((size_t)((n + 15) / 16 * 16));                       // image
    b += al256(sizeof(PropDev));                                     // property
    b += al256((size_t)(8 + 1 + 3 * levels + kQueueStride + kF32Queues * kQueueStride) * 8);  // counters, queues
    b += al256((size_t)std::max<int64_t>(tcap, 1) * sizeof(DevRec)); // near-tie slots
    b += al256((size_t)h1 * 4) + 2 * al256(4);                       // u0, u0 index, property ids
    b += al256((size_t)std::max(levels, 1) * n * 8);                 // prefix tables
    b += al256((size_t)std::max(levels, 1) * sizeof(EnumJob));       // jobs
    b += al256((size_t)std::max<int64_t>(rec_slots, 1) * sizeof(DevRec));
    b += al256(sort_scratch_bytes(rec_slots)) + al256(sort_scratch_bytes(tcap));
    if (!o->records_on_device)
        b += al256((size_t)std::max<int64_t>(cap, 1) * sizeof(CexRec)) + al256((size_t)std::max<int64_t>(tcap, 1) * sizeof(CexRec));
    *need = b;
    return IBMC_OK;
}

}  // namespace ibmc

using namespace ibmc;

extern "C" ibmc_status ibmc_check_property_noalloc(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                                   int32_t n_pixels, const int16_t *delta_set, int32_t n_deltas,
                                                   const ibmc_check_opts *opts, ibmc_check_summary *out,
                                                   ibmc_cex *cex_buf, ibmc_cex *near_tie_buf) {
    clear_error();
    if (!ctx || !net || !opts || !out) return fail(IBMC_E_INVALID, "null ctx / net / opts / out");
    if (n_pixels != net->dims[0]) return fail(IBMC_E_INVALID, "n_pixels %d != network input %d", n_pixels, net->dims[0]);
    if (opts->k_step < 1 || opts->k_max < opts->k_min || opts->cex_capacity < 0 || opts->near_tie_capacity < 0)
        return fail(IBMC_E_INVALID, "bad k range or capacity");
    HIP_OK(hipSetDevice(ctx->device));
    IBMC_TRY(noalloc_setup(ctx->device));
    size_t need = 0;
    IBMC_TRY(scratch_need(ctx, net, n_deltas, opts, &need));
    if (need > (size_t)IBMC_NOALLOC_SCRATCH_BYTES)
        return fail(IBMC_E_INVALID, "this call needs up to %zu bytes of device scratch; the fixed scratch holds %zu "
                    "(lower cex_capacity / near_tie_capacity)", need, (size_t)IBMC_NOALLOC_SCRATCH_BYTES);
    ibmc_property p{};
    p.net = net;
    p.image = image;
    p.deltas = delta_set;
    p.n_deltas = n_deltas;
    p.k_min = opts->k_min;
    p.k_max = opts->k_max;
    p.k_step = opts->k_step;
    // the context's own buffers step aside; empty ones carve the arena
    DevBuf *mine[] = {&ctx->images, &ctx->props, &ctx->jobs, &ctx->qcum, &ctx->u0, &ctx->u0_index,
                      &ctx->prop_ids, &ctx->counters, &ctx->recs, &ctx->ties, &ctx->order, &ctx->u0f,
                      &ctx->sortbuf, &ctx->recout};
    constexpr int NB = sizeof(mine) / sizeof(mine[0]);
    DevBuf saved[NB];
    for (int i = 0; i < NB; ++i) saved[i].swap(*mine[i]);
    ScratchArena arena;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        arena.base = reinterpret_cast<char *>(g_ptr[ctx->device]);
    }
    arena.cap = IBMC_NOALLOC_SCRATCH_BYTES;
    ScratchArena *prev = thread_arena();
    thread_arena() = &arena;
    const ibmc_status st = check_batch_impl(ctx, &p, 1, opts, out, cex_buf, near_tie_buf, false);
    thread_arena() = prev;
    for (int i = 0; i < NB; ++i) {
        mine[i]->release();  // a view into the arena: nothing to free
        mine[i]->swap(saved[i]);
    }
    return st;
}
