// Host-side structures of the library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <utility>
#include <string>
#include <vector>
#include <deque>

#include "ibmc_internal.h"
#include "kernels_q8.h"
#include "kernels_f32.h"
#include "kernels_cov.h"
#include "kernels_prop.h"
#include "kernels_sort.h"
#include "kernels_lane.h"

namespace ibmc {

ibmc_status fail(ibmc_status code, const char *fmt, ...);
const char *last_error();
void clear_error();

#define HIP_OK(expr)                                                                              \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess)                                                                     \
            return ::ibmc::fail(IBMC_E_HIP, "%s:%d %s: %s", __FILE__, __LINE__, #expr,             \
                                hipGetErrorString(_e));                                           \
    } while (0)

#define IBMC_TRY(expr)                                                                            \
    do {                                                                                          \
        ibmc_status _s = (expr);                                                                  \
        if (_s < 0) return _s;                                                                    \
    } while (0)

// A fixed region of device memory that buffers are carved from, in order,
// instead of being allocated (the allocation-free entry point).  While one is
// installed on the calling thread, DevBuf::reserve takes its bytes from it and
// fails with a clear error once the region is used up.
struct ScratchArena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};
ScratchArena *&thread_arena();

// Grow-only device allocation (or a view into the thread's arena).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;   // p points into an arena: never freed here
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), borrowed(o.borrowed) {
        o.p = nullptr;
        o.bytes = 0;
        o.borrowed = false;
    }
    void swap(DevBuf &o) noexcept {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(borrowed, o.borrowed);
    }
    ~DevBuf();
    void release();
    ibmc_status reserve(size_t n);
    ibmc_status upload(const void *src, size_t n, hipStream_t s);
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

}  // namespace ibmc

struct ibmc_ctx {
    int device = 0;
    int n_cu = 0;
    int arch_major = 0, arch_minor = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ek0 = nullptr, ek1 = nullptr;
    int32_t *flags_host = nullptr;   // [0] abort request, [1] first hit
    int32_t *flags_dev = nullptr;    // device view of flags_host
    // scratch of the check driver (grow-only)
    ibmc::DevBuf images, props, jobs, qcum, u0, u0_index, prop_ids, counters, recs, ties, order;
    ibmc::DevBuf u0f, sortbuf;
    ibmc::DevBuf lut;                  // the table sigmoid's knots (built on first use)
    ibmc::DevBuf recout;  // sorted records in the public layout, on their way to a host buffer
    ibmc::DevBuf prop_scratch, prop_feat, prop_scores, shell_cum;  // ranked search
    int64_t shell_cum_n = -1, shell_cum_ch = -1;                   // shell_cum holds this plan
    // a ranked search's per-call inputs, packed in pinned host memory and sent
    // to stage_dev in one copy; stage_ev marks that copy's completion
    char *stage_host = nullptr;
    size_t stage_host_bytes = 0;
    ibmc::DevBuf stage_dev;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    ibmc::DevBuf cov_img, cov_pots, cov_bits, cov_sums, cov_out;
    // tuned kernel variant per network shape key
    std::map<std::string, std::string> tuned;
    std::vector<hipStream_t> side;     // branch streams of captured batch graphs (default priority)
    std::vector<hipEvent_t> side_ev;
    hipEvent_t fork_ev = nullptr;
    int64_t graph_launches = 0;
    // the instantiated graph of the last multi-network batch and the
    // signature of every value its launches were captured with
    hipGraphExec_t graph_exec = nullptr;
    std::string graph_sig;
    int64_t graph_reuses = 0;
    bool force_int32_layer1 = false;   // testing aid: take the general first-layer path
    double last_kernel_seconds = 0.0;
    int last_kernel_launches = 0;
    ~ibmc_ctx();
};

struct ibmc_mlp {
    ibmc_ctx *ctx = nullptr;
    int device = -1;
    int act = 0;
    int L = 0;
    std::vector<int> dims;
    std::vector<int> shift;
    std::vector<std::vector<int8_t>> Wq;
    std::vector<std::vector<int32_t>> bq;
    std::vector<std::vector<float>> Wf;
    std::vector<std::vector<float>> bf;
    std::deque<ibmc::DevBuf> buf;      // device copies (stable addresses)
    ibmc::QNetDev qd;
    ibmc::FwdExtra fx;
    ibmc::FNetDev fd;
    ibmc::LaneNetDev lane{};           // integer nets the lane kernels serve (lane.ok)
    std::string forced_variant;
    ~ibmc_mlp();
};

namespace ibmc {
std::string shape_key(const ibmc_mlp *m);
PropParams prop_views(const ibmc_proposer *p);
const EnumVariant *pick_variant(ibmc_ctx *ctx, const ibmc_mlp *net);
bool use_lane(ibmc_ctx *ctx, const ibmc_mlp *net, bool allowed);
// ball_r2 (nullable): per property the squared radius of the L2-ball domain,
// or -1 for its delta set.
ibmc_status check_batch_impl(ibmc_ctx *ctx, const ibmc_property *props, int32_t n_props, const ibmc_check_opts *o,
                             ibmc_check_summary *outs, ibmc_cex *cex_buf, ibmc_cex *tie_buf, bool images_on_device,
                             const int64_t *ball_r2 = nullptr);
// Looks up, once per device and with that device current, the address of
// the allocation-free entry point's fixed scratch array.
ibmc_status noalloc_setup(int device);
}
