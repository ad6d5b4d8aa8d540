// Host runtime of the library: contexts, network layout, the incremental
// bound driver, record compaction and sorting, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "ibmc_host.h"

namespace ibmc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

ibmc_status fail(ibmc_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char *last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

ScratchArena *&thread_arena() {
    static thread_local ScratchArena *a = nullptr;
    return a;
}

DevBuf::~DevBuf() { release(); }

void DevBuf::release() {
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
}

ibmc_status DevBuf::reserve(size_t n) {
    if (n <= bytes && p) return IBMC_OK;
    if (ScratchArena *a = thread_arena()) {
        // carve the next 256-byte aligned piece; an owned allocation is never
        // held here while an arena is installed (the caller swaps them out)
        if (p && !borrowed) return fail(IBMC_E_INVALID, "owned buffer met while carving fixed scratch");
        const size_t off = (a->used + 255) & ~(size_t)255;
        const size_t want = std::max<size_t>(n, 256);
        if (off > a->cap || want > a->cap - off)
            return fail(IBMC_E_INVALID, "the call needs more than the %zu bytes of fixed device scratch "
                        "(at %zu, %zu more wanted); lower its capacities or use the allocating entry point",
                        a->cap, off, want);
        p = a->base + off;
        bytes = want;
        borrowed = true;
        a->used = off + want;
        return IBMC_OK;
    }
    release();
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return fail(IBMC_E_OOM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    bytes = want;
    return IBMC_OK;
}

ibmc_status DevBuf::upload(const void *src, size_t n, hipStream_t s) {
    ibmc_status st = reserve(n);
    if (st) return st;
    if (n) HIP_OK(hipMemcpyAsync(p, src, n, hipMemcpyHostToDevice, s));
    return IBMC_OK;
}

}  // namespace ibmc

using namespace ibmc;

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

extern "C" const char *ibmc_last_error(void) { return ibmc::last_error(); }

extern "C" ibmc_status ibmc_ctx_create(int32_t device, void *hip_stream, ibmc_ctx **out) {
    clear_error();
    if (!out) return fail(IBMC_E_INVALID, "out is null");
    *out = nullptr;
    int ndev = 0;
    HIP_OK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(IBMC_E_INVALID, "device %d of %d", device, ndev);
    HIP_OK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, device));
    std::unique_ptr<ibmc_ctx> c(new ibmc_ctx());
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->arch_major = prop.major;
    c->arch_minor = prop.minor;
    // testing aid: IBMC_FIRST_LAYER=int32 forces the general (int32) first-layer path
    const char *fl = getenv("IBMC_FIRST_LAYER");
    c->force_int32_layer1 = fl && std::string(fl) == "int32";
    if (hip_stream) {
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        c->own_stream = false;
    } else {
        HIP_OK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    HIP_OK(hipEventCreate(&c->ev0));
    HIP_OK(hipEventCreate(&c->ev1));
    HIP_OK(hipEventCreate(&c->ek0));
    HIP_OK(hipEventCreate(&c->ek1));
    HIP_OK(hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming));
    // coherent (fine-grained) host memory: the device's first-hit store and
    // the host's abort request bypass the GPU caches, so each side sees the
    // other's write while the kernel runs
    void *hm = nullptr;
    HIP_OK(hipHostMalloc(&hm, 64, hipHostMallocMapped | hipHostMallocCoherent));
    c->flags_host = reinterpret_cast<int32_t *>(hm);
    memset(hm, 0, 64);
    void *dm = nullptr;
    HIP_OK(hipHostGetDevicePointer(&dm, hm, 0));
    c->flags_dev = reinterpret_cast<int32_t *>(dm);
    IBMC_TRY(noalloc_setup(device));
    *out = c.release();
    return IBMC_OK;
}

ibmc_ctx::~ibmc_ctx() {
    (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ek0) (void)hipEventDestroy(ek0);
    if (ek1) (void)hipEventDestroy(ek1);
    if (flags_host) (void)hipHostFree(flags_host);
    if (stage_host) (void)hipHostFree(stage_host);
    if (stage_ev) (void)hipEventDestroy(stage_ev);
    for (hipStream_t st : side) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : side_ev) (void)hipEventDestroy(ev);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    (void)hipGetLastError();
}

extern "C" void ibmc_ctx_destroy(ibmc_ctx *ctx) { delete ctx; }

extern "C" ibmc_status ibmc_device_info(ibmc_ctx *ctx, int32_t *n_cu, int32_t *maj, int32_t *min_) {
    clear_error();
    if (!ctx) return fail(IBMC_E_INVALID, "ctx is null");
    if (n_cu) *n_cu = ctx->n_cu;
    if (maj) *maj = ctx->arch_major;
    if (min_) *min_ = ctx->arch_minor;
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_abort(ibmc_ctx *ctx) {
    if (!ctx) return fail(IBMC_E_INVALID, "ctx is null");
    __atomic_store_n(&ctx->flags_host[0], 1, __ATOMIC_SEQ_CST);
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_last_kernel_time(ibmc_ctx *ctx, double *seconds, int32_t *launches) {
    clear_error();
    if (!ctx) return fail(IBMC_E_INVALID, "ctx is null");
    if (seconds) *seconds = ctx->last_kernel_seconds;
    if (launches) *launches = ctx->last_kernel_launches;
    return IBMC_OK;
}

// ---------------------------------------------------------------------------
// networks
// ---------------------------------------------------------------------------

ibmc_mlp::~ibmc_mlp() {
    // the device is kept here, not read from the context, which may be gone
    if (device >= 0) (void)hipSetDevice(device);
    buf.clear();
    (void)hipGetLastError();   // an ignored teardown error must not reach the next launch's check
}

extern "C" void ibmc_free_mlp(ibmc_mlp *net) { delete net; }

// Compact layouts of the lane-per-point kernels (see LaneNetDev), for the
// networks they serve.
static ibmc_status build_lane(ibmc_mlp *m, hipStream_t s) {
    LaneNetDev &ln = m->lane;
    memset(&ln, 0, sizeof(ln));
    const int L = m->L;
    if (!lane_eligible(m->dims.data(), L)) return IBMC_OK;
    const int n = m->dims[0], h1 = m->dims[1], h2 = (L == 3) ? m->dims[2] : 0, nc = m->dims[L];
    ln.L = L;
    ln.n = n;
    ln.nc = nc;
    ln.LH1 = lane_width(h1);
    ln.LH2 = (L == 3) ? lane_width(h2) : 0;
    ln.s1 = m->shift[0];
    ln.s2 = (L == 3) ? m->shift[1] : 0;
    const int H1 = ln.LH1, H2 = ln.LH2, HL = (L == 3) ? H2 : H1, hl = (L == 3) ? h2 : h1;
    std::vector<int8_t> w1c((size_t)n * H1, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < h1; ++j) w1c[(size_t)i * H1 + j] = m->Wq[0][(size_t)j * n + i];
    std::vector<int32_t> q1(H1, -1);
    for (int qpos = 0; qpos < m->qd.H[1]; ++qpos) {
        const int unit = sigma64(qpos);
        if (unit < h1) q1[unit] = qpos;
    }
    // [NO / 8][NI / 4][8] words of four int8 weights of inputs 4w..4w+3
    auto words = [](const std::vector<int8_t> &W, int nout, int nin, int NO, int NI) {
        std::vector<int32_t> out((size_t)NO * NI / 4, 0);
        for (int st = 0; st < NO / 8; ++st)
            for (int w = 0; w < NI / 4; ++w)
                for (int t = 0; t < 8; ++t) {
                    const int o = st * 8 + t;
                    uint32_t v = 0;
                    for (int z = 0; z < 4; ++z) {
                        const int i = 4 * w + z;
                        const int8_t x = (o < nout && i < nin) ? W[(size_t)o * nin + i] : 0;
                        v |= (uint32_t)(uint8_t)x << (8 * z);
                    }
                    out[((size_t)st * (NI / 4) + w) * 8 + t] = (int32_t)v;
                }
        return out;
    };
    auto padded = [](const std::vector<int32_t> &b, int nout, int NO) {
        std::vector<int32_t> out(NO, 0);
        for (int j = 0; j < nout; ++j) out[j] = b[j];
        return out;
    };
    IBMC_TRY(m->buf.emplace_back().upload(w1c.data(), w1c.size(), s));
    ln.W1C = (const int8_t *)m->buf.back().p;
    IBMC_TRY(m->buf.emplace_back().upload(q1.data(), q1.size() * 4, s));
    ln.q1 = (const int32_t *)m->buf.back().p;
    if (L == 3) {
        const std::vector<int32_t> w2 = words(m->Wq[1], h2, h1, H2, H1), b2 = padded(m->bq[1], h2, H2);
        IBMC_TRY(m->buf.emplace_back().upload(w2.data(), w2.size() * 4, s));
        ln.W2S = (const int32_t *)m->buf.back().p;
        IBMC_TRY(m->buf.emplace_back().upload(b2.data(), b2.size() * 4, s));
        ln.b2 = (const int32_t *)m->buf.back().p;
    }
    const std::vector<int32_t> wo = words(m->Wq[L - 1], nc, hl, 16, HL), bo = padded(m->bq[L - 1], nc, 16);
    IBMC_TRY(m->buf.emplace_back().upload(wo.data(), wo.size() * 4, s));
    ln.WOS = (const int32_t *)m->buf.back().p;
    IBMC_TRY(m->buf.emplace_back().upload(bo.data(), bo.size() * 4, s));
    ln.bo = (const int32_t *)m->buf.back().p;
    HIP_OK(hipStreamSynchronize(s));   // the staging vectors go out of scope
    ln.ok = 1;
    return IBMC_OK;
}

static ibmc_status build_q8(ibmc_ctx *ctx, ibmc_mlp *m) {
    const int L = m->L;
    QNetDev &q = m->qd;
    memset(&q, 0, sizeof(q));
    q.L = L;
    for (int l = 0; l <= L; ++l) q.dims[l] = m->dims[l];
    q.H[0] = m->dims[0];
    // hidden widths padded to 64 * 2^j: the kernel instances cover those K-block counts
    for (int l = 1; l < L; ++l) {
        int h = 64;
        while (h < m->dims[l]) h *= 2;
        q.H[l] = h;
    }
    q.H[L] = round_up(m->dims[L], 16);
    for (int l = 0; l < L - 1; ++l) q.shift[l] = m->shift[l];
    const int n = m->dims[0], H1 = q.H[1];
    hipStream_t s = ctx->stream;

    // first layer, transposed, sigma order
    std::vector<int8_t> w1t((size_t)n * H1, 0);
    std::vector<int32_t> b1s(H1, 0), b1n(H1, 0), rs(H1, 0);
    for (int qpos = 0; qpos < H1; ++qpos) {
        const int neuron = sigma64(qpos);
        if (neuron >= m->dims[1]) continue;
        for (int i = 0; i < n; ++i) w1t[(size_t)i * H1 + qpos] = m->Wq[0][(size_t)neuron * n + i];
        b1s[qpos] = m->bq[0][neuron];
    }
    for (int j = 0; j < m->dims[1]; ++j) {
        b1n[j] = m->bq[0][j];
        int64_t sum = 0;
        for (int i = 0; i < n; ++i) sum += m->Wq[0][(size_t)j * n + i];
        rs[j] = (int32_t)(128 * sum);
    }
    IBMC_TRY(m->buf.emplace_back().upload(w1t.data(), w1t.size(), s));
    q.W1T = (const int8_t *)m->buf.back().p;
    // scaled int16 copy for the packed first-layer path: f1 = 2^(8 - shift)
    q.f1 = (L > 1 && m->shift[0] <= 8) ? (1 << (8 - m->shift[0])) : 0;
    q.maxw1 = 0;
    for (int8_t w : m->Wq[0]) q.maxw1 = std::max(q.maxw1, std::abs((int)w));
    {
        std::vector<int16_t> w16(w1t.size());
        for (size_t t = 0; t < w1t.size(); ++t) w16[t] = (int16_t)(w1t[t] * std::max(q.f1, 1));
        IBMC_TRY(m->buf.emplace_back().upload(w16.data(), w16.size() * 2, s));
        q.W1T16 = (const int16_t *)m->buf.back().p;
    }
    IBMC_TRY(m->buf.emplace_back().upload(b1s.data(), b1s.size() * 4, s));
    q.b1s = (const int32_t *)m->buf.back().p;
    // column norms of the first layer for the proposer's features
    {
        std::vector<float> pn((size_t)2 * n + 2, 0.f);
        float M1 = 0.f, M2 = 0.f;
        for (int p = 0; p < n; ++p) {
            int64_t s1 = 0, s2 = 0;
            for (int j = 0; j < m->dims[1]; ++j) {
                const int w = m->Wq[0][(size_t)j * n + p];
                s1 += std::abs(w);
                s2 += (int64_t)w * w;
            }
            pn[p] = (float)s1;
            pn[n + p] = std::sqrt((float)s2);
            M1 = std::max(M1, pn[p]);
            M2 = std::max(M2, pn[n + p]);
        }
        pn[2 * n] = std::max(M1, 1.f);
        pn[2 * n + 1] = std::max(M2, 1.f);
        IBMC_TRY(m->buf.emplace_back().upload(pn.data(), pn.size() * 4, s));
        q.pnorm = (const float *)m->buf.back().p;
    }
    IBMC_TRY(m->buf.emplace_back().upload(b1n.data(), b1n.size() * 4, s));
    q.b1n = (const int32_t *)m->buf.back().p;
    IBMC_TRY(m->buf.emplace_back().upload(rs.data(), rs.size() * 4, s));
    q.rowsum1 = (const int32_t *)m->buf.back().p;

    // layer-1 A-operand tiles over pixel K-blocks (natural pixel order)
    {
        const int KB = (n + 63) / 64;
        std::vector<int8_t> t((size_t)(H1 / 16) * KB * 1024, 0);
        for (int mt = 0; mt < H1 / 16; ++mt)
            for (int kb = 0; kb < KB; ++kb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int b = 0; b < 16; ++b) {
                        const int row = mt * 16 + (lane & 15);
                        const int pix = kb * 64 + (lane >> 4) * 16 + b;
                        if (row < m->dims[1] && pix < n)
                            t[(((size_t)mt * KB + kb) * 64 + lane) * 16 + b] = m->Wq[0][(size_t)row * n + pix];
                    }
        IBMC_TRY(m->buf.emplace_back().upload(t.data(), t.size(), s));
        q.W1tile = (const int8_t *)m->buf.back().p;
    }
    // fast hidden epilogue of 3-layer nets (shift[1] in {7, 8}), where every
    // partial sum of its offset accumulators stays inside int32
    bool fast_ok = L == 3 && (m->shift[1] == 7 || m->shift[1] == 8);
    for (int l = 2; l <= L && fast_ok; ++l) {
        const int nin = m->dims[l - 1], nout = m->dims[l];
        const int64_t alpha = (l == 2) ? (1 << (8 - m->shift[1])) : 1;
        for (int j = 0; j < nout && fast_ok; ++j) {
            int64_t sa = 0;
            for (int i = 0; i < nin; ++i) sa += std::llabs((long long)m->Wq[l - 1][(size_t)j * nin + i]);
            const int64_t bound = alpha * (std::llabs((long long)m->bq[l - 1][j]) + 256 * sa) + 32768;
            if (bound >= (1LL << 31)) fast_ok = false;
        }
    }
    // layers >= 2: A-operand tiles with sigma-permuted K, natural-order bias
    for (int l = 2; l <= L; ++l) {
        const int Hin = q.H[l - 1], Hout = q.H[l], nin = m->dims[l - 1], nout = m->dims[l];
        const int KB = Hin / 64, MT = Hout / 16;
        std::vector<int8_t> t((size_t)MT * KB * 1024, 0);
        for (int mt = 0; mt < MT; ++mt)
            for (int kb = 0; kb < KB; ++kb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int b = 0; b < 16; ++b) {
                        const int row = mt * 16 + (lane & 15);
                        const int col = sigma64(kb * 64 + (lane >> 4) * 16 + b);
                        if (row < nout && col < nin)
                            t[(((size_t)mt * KB + kb) * 64 + lane) * 16 + b] = m->Wq[l - 1][(size_t)row * nin + col];
                    }
        IBMC_TRY(m->buf.emplace_back().upload(t.data(), t.size(), s));
        q.Wt[l] = (const int8_t *)m->buf.back().p;
        std::vector<int32_t> bb(Hout, 0), bo(Hout, 0);
        for (int j = 0; j < nout; ++j) {
            bb[j] = m->bq[l - 1][j];
            // inputs arrive as a - 64: add back 64 * rowsum; hidden outputs are
            // requantised from u - 64 * 2^s
            int64_t rs = 0;
            for (int i = 0; i < nin; ++i) rs += m->Wq[l - 1][(size_t)j * nin + i];
            int64_t v = (int64_t)m->bq[l - 1][j] + 64 * rs;
            if (l < L) v -= (int64_t)64 << m->shift[l - 1];
            bo[j] = (int32_t)v;
        }
        IBMC_TRY(m->buf.emplace_back().upload(bb.data(), bb.size() * 4, s));
        q.bn[l] = (const int32_t *)m->buf.back().p;
        IBMC_TRY(m->buf.emplace_back().upload(bo.data(), bo.size() * 4, s));
        q.bo[l] = (const int32_t *)m->buf.back().p;
        if (l == 2 && fast_ok) {
            // layer 2 fed with alpha (a1 - 64), alpha = 2^(8 - s2): its accumulator is
            // alpha * u2 - 32768, whose saturation to int16 has byte 1 = a2 - 128 once
            // clamped to at most -1
            const int alpha = 1 << (8 - m->shift[1]);
            std::vector<int32_t> bf(Hout, 0);
            for (int j = 0; j < nout; ++j) {
                int64_t rs = 0;
                for (int i = 0; i < nin; ++i) rs += m->Wq[l - 1][(size_t)j * nin + i];
                bf[j] = (int32_t)(alpha * ((int64_t)m->bq[l - 1][j] + 64 * rs) - 32768);
            }
            IBMC_TRY(m->buf.emplace_back().upload(bf.data(), bf.size() * 4, s));
            q.bf2 = (const int32_t *)m->buf.back().p;
            q.fast2 = alpha;
        }
        if (l == L && q.fast2 != 0) {
            // output layer fed with a2 - 128
            std::vector<int32_t> bf(Hout, 0);
            for (int j = 0; j < nout; ++j) {
                int64_t rs = 0;
                for (int i = 0; i < nin; ++i) rs += m->Wq[l - 1][(size_t)j * nin + i];
                bf[j] = (int32_t)((int64_t)m->bq[l - 1][j] + 128 * rs);
            }
            IBMC_TRY(m->buf.emplace_back().upload(bf.data(), bf.size() * 4, s));
            q.bf3 = (const int32_t *)m->buf.back().p;
        }
    }
    // batched forward: natural-K tiles of layers >= 2 and accumulator inits
    {
        FwdExtra &fx = m->fx;
        memset(&fx, 0, sizeof(fx));
        fx.K0 = round_up(n, 64);
        for (int l = 2; l <= L; ++l) {
            const int Hin = q.H[l - 1], Hout = q.H[l], nin = m->dims[l - 1], nout = m->dims[l];
            const int KB = Hin / 64, MT = Hout / 16;
            std::vector<int8_t> t((size_t)MT * KB * 1024, 0);
            for (int mt = 0; mt < MT; ++mt)
                for (int kb = 0; kb < KB; ++kb)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int b = 0; b < 16; ++b) {
                            const int row = mt * 16 + (lane & 15);
                            const int col = kb * 64 + (lane >> 4) * 16 + b;
                            if (row < nout && col < nin)
                                t[(((size_t)mt * KB + kb) * 64 + lane) * 16 + b] = m->Wq[l - 1][(size_t)row * nin + col];
                        }
            IBMC_TRY(m->buf.emplace_back().upload(t.data(), t.size(), s));
            fx.Wn[l] = (const int8_t *)m->buf.back().p;
        }
        for (int l = 1; l <= L; ++l) {
            const int nin = m->dims[l - 1], nout = m->dims[l];
            std::vector<int32_t> init(q.H[l], 0);
            const bool hidden = l < L;
            for (int j = 0; j < q.H[l]; ++j) {
                int64_t v = 0;
                if (j < nout) {
                    int64_t rs = 0;
                    for (int i = 0; i < nin; ++i) rs += m->Wq[l - 1][(size_t)j * nin + i];
                    // layer 1 reads x - 128, later layers a - 64
                    v = (int64_t)m->bq[l - 1][j] + (l == 1 ? 128 : 64) * rs;
                }
                if (hidden) v -= (int64_t)64 << m->shift[l - 1];
                init[j] = (int32_t)v;
            }
            IBMC_TRY(m->buf.emplace_back().upload(init.data(), init.size() * 4, s));
            fx.init[l] = (const int32_t *)m->buf.back().p;
        }
    }
    // dense row-major copies
    for (int l = 1; l <= L; ++l) {
        IBMC_TRY(m->buf.emplace_back().upload(m->Wq[l - 1].data(), m->Wq[l - 1].size(), s));
        q.Wd[l] = (const int8_t *)m->buf.back().p;
        IBMC_TRY(m->buf.emplace_back().upload(m->bq[l - 1].data(), m->bq[l - 1].size() * 4, s));
        q.bd[l] = (const int32_t *)m->buf.back().p;
    }
    IBMC_TRY(build_lane(m, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

static ibmc_status build_f32(ibmc_ctx *ctx, ibmc_mlp *m) {
    FNetDev &f = m->fd;
    memset(&f, 0, sizeof(f));
    f.L = m->L;
    for (int l = 0; l <= m->L; ++l) f.dims[l] = m->dims[l];
    const int n = m->dims[0], h1 = m->dims[1];
    hipStream_t s = ctx->stream;
    std::vector<float> w1t((size_t)n * h1);
    for (int j = 0; j < h1; ++j)
        for (int i = 0; i < n; ++i) w1t[(size_t)i * h1 + j] = m->Wf[0][(size_t)j * n + i];
    IBMC_TRY(m->buf.emplace_back().upload(w1t.data(), w1t.size() * 4, s));
    f.W1T = (const float *)m->buf.back().p;
    for (int l = 2; l <= m->L; ++l) {
        const int nin = m->dims[l - 1], nout = m->dims[l];
        std::vector<float> wt((size_t)nin * nout);
        for (int j = 0; j < nout; ++j)
            for (int i = 0; i < nin; ++i) wt[(size_t)i * nout + j] = m->Wf[l - 1][(size_t)j * nin + i];
        IBMC_TRY(m->buf.emplace_back().upload(wt.data(), wt.size() * 4, s));
        f.WT[l] = (const float *)m->buf.back().p;
    }
    for (int l = 1; l <= m->L; ++l) {
        IBMC_TRY(m->buf.emplace_back().upload(m->Wf[l - 1].data(), m->Wf[l - 1].size() * 4, s));
        f.Wd[l] = (const float *)m->buf.back().p;
        IBMC_TRY(m->buf.emplace_back().upload(m->bf[l - 1].data(), m->bf[l - 1].size() * 4, s));
        f.bd[l] = (const float *)m->buf.back().p;
    }
    // enumeration layout: transposed, zero-padded to the kernel family's widths
    const F32Layout lay = f32_layout(m->L, m->dims.data());
    f.kind = lay.kind;
    for (int l = 0; l <= m->L; ++l) f.HP[l] = lay.HP[l];
    {
        const int hp1 = f.HP[1];
        std::vector<float> w1p((size_t)n * hp1, 0.f);
        for (int j = 0; j < h1; ++j)
            for (int i = 0; i < n; ++i) w1p[(size_t)i * hp1 + j] = m->Wf[0][(size_t)j * n + i];
        IBMC_TRY(m->buf.emplace_back().upload(w1p.data(), w1p.size() * 4, s));
        f.W1P = (const float *)m->buf.back().p;
    }
    for (int l = 1; l <= m->L; ++l) {
        const int nin = m->dims[l - 1], nout = m->dims[l], hin = f.HP[l - 1], hout = f.HP[l];
        if (l >= 2) {
            std::vector<float> wp((size_t)hin * hout, 0.f);
            for (int j = 0; j < nout; ++j)
                for (int i = 0; i < nin; ++i) wp[(size_t)i * hout + j] = m->Wf[l - 1][(size_t)j * nin + i];
            IBMC_TRY(m->buf.emplace_back().upload(wp.data(), wp.size() * 4, s));
            f.WP[l] = (const float *)m->buf.back().p;
        }
        std::vector<float> bp(hout, 0.f);
        for (int j = 0; j < nout; ++j) bp[j] = m->bf[l - 1][j];
        IBMC_TRY(m->buf.emplace_back().upload(bp.data(), bp.size() * 4, s));
        f.bP[l] = (const float *)m->buf.back().p;
    }
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_load_mlp(ibmc_ctx *ctx, const ibmc_mlp_desc *d, ibmc_mlp **out) {
    clear_error();
    if (!ctx || !d || !out) return fail(IBMC_E_INVALID, "null argument");
    *out = nullptr;
    if (d->n_layers < 2 || d->n_layers > IBMC_MAX_LAYERS)
        return fail(IBMC_E_UNIMPL, "n_layers %d outside [2, %d]", d->n_layers, IBMC_MAX_LAYERS);
    if (!d->dims || !d->W || !d->b) return fail(IBMC_E_INVALID, "dims / W / b is null");
    if (d->act != IBMC_ACT_RELU_Q8 && d->act != IBMC_ACT_SIGMOID_F32)
        return fail(IBMC_E_INVALID, "unknown activation %d", d->act);
    const int L = d->n_layers;
    for (int l = 0; l <= L; ++l) {
        if (d->dims[l] < 1) return fail(IBMC_E_INVALID, "dims[%d] = %d", l, d->dims[l]);
        if (d->dims[l] > IBMC_MAX_WIDTH)
            return fail(IBMC_E_UNIMPL, "dims[%d] = %d exceeds %d", l, d->dims[l], IBMC_MAX_WIDTH);
    }
    if (d->dims[L] > kMaxClasses) return fail(IBMC_E_UNIMPL, "%d classes exceed %d", d->dims[L], kMaxClasses);
    for (int l = 0; l < L; ++l)
        if (!d->W[l] || !d->b[l]) return fail(IBMC_E_INVALID, "W[%d] or b[%d] is null", l, l);
    HIP_OK(hipSetDevice(ctx->device));
    std::unique_ptr<ibmc_mlp> m(new ibmc_mlp());
    m->ctx = ctx;
    m->device = ctx->device;
    m->act = d->act;
    m->L = L;
    m->dims.assign(d->dims, d->dims + L + 1);
    if (d->act == IBMC_ACT_RELU_Q8) {
        if (!d->shift) return fail(IBMC_E_INVALID, "shift is null");
        for (int l = 0; l < L - 1; ++l) {
            if (d->shift[l] < 0 || d->shift[l] > kMaxShift)
                return fail(IBMC_E_INVALID, "shift[%d] = %d outside [0, %d]", l, d->shift[l], kMaxShift);
            m->shift.push_back(d->shift[l]);
        }
        for (int l = 0; l < L; ++l) {
            const int nin = d->dims[l], nout = d->dims[l + 1];
            const int8_t *W = (const int8_t *)d->W[l];
            const int32_t *b = (const int32_t *)d->b[l];
            m->Wq.emplace_back(W, W + (size_t)nin * nout);
            m->bq.emplace_back(b, b + nout);
            // int32 headroom of the forms the kernels accumulate in: inputs
            // enter as x - 128 with 128 * rowsum in the init (first layer:
            // every partial sum within |b| + 256 sum|w|), activations as
            // a - 64 with 64 * rowsum in the init (within |b| + 128 sum|w|),
            // and a hidden layer's accumulator is offset by -64 * 2^s
            const int64_t amax = (l == 0) ? 256 : 128;
            const int64_t off = (l < L - 1) ? (64LL << d->shift[l]) : 0;
            for (int j = 0; j < nout; ++j) {
                int64_t s = std::llabs((long long)b[j]) + off;
                for (int i = 0; i < nin; ++i) s += std::llabs((long long)W[(size_t)j * nin + i]) * amax;
                if (s >= (1LL << 31))
                    return fail(IBMC_E_RANGE, "layer %d neuron %d: accumulator bound %lld reaches 2^31", l + 1, j,
                                (long long)s);
            }
        }
        IBMC_TRY(build_q8(ctx, m.get()));
    } else {
        for (int l = 0; l < L; ++l) {
            const int nin = d->dims[l], nout = d->dims[l + 1];
            const float *W = (const float *)d->W[l];
            const float *b = (const float *)d->b[l];
            m->Wf.emplace_back(W, W + (size_t)nin * nout);
            m->bf.emplace_back(b, b + nout);
            for (size_t t = 0; t < m->Wf.back().size(); ++t)
                if (!std::isfinite(m->Wf.back()[t])) return fail(IBMC_E_INVALID, "non-finite weight in layer %d", l + 1);
        }
        IBMC_TRY(build_f32(ctx, m.get()));
    }
    *out = m.release();
    return IBMC_OK;
}

// ---------------------------------------------------------------------------
// decode
// ---------------------------------------------------------------------------

extern "C" ibmc_status ibmc_decode_point(int32_t n, int32_t m, int32_t k, int64_t rank, int32_t *pixels,
                                         int32_t *delta_idx) {
    clear_error();
    if (n < 1 || m < 1 || k < 0 || k > n || k > kMaxK) return fail(IBMC_E_INVALID, "bad n/m/k");
    if (k > 0 && (!pixels || !delta_idx)) return fail(IBMC_E_INVALID, "null output");
    int64_t mk = 1;
    for (int j = 0; j < k; ++j) mk *= m;
    const int64_t total = binom_small(n, k) * mk;
    if (rank < 0 || rank >= total) return fail(IBMC_E_INVALID, "rank %lld outside [0, %lld)", (long long)rank,
                                              (long long)total);
    int p[kMaxK];
    lex_unrank_subset(rank / mk, k, n, p);
    int64_t d = rank % mk;
    for (int j = k - 1; j >= 0; --j) { delta_idx[j] = (int32_t)(d % m); d /= m; }
    for (int j = 0; j < k; ++j) pixels[j] = p[j];
    return IBMC_OK;
}

// ---------------------------------------------------------------------------
// forward and replay
// ---------------------------------------------------------------------------

extern "C" ibmc_status ibmc_forward(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images, int64_t n_images,
                                    void *potentials, int32_t *labels) {
    clear_error();
    if (!ctx || !net || (!images && n_images > 0) || n_images < 0) return fail(IBMC_E_INVALID, "bad argument");
    if (n_images == 0) return IBMC_OK;
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int n = net->dims[0];
    int64_t U = 0;
    for (int l = 1; l <= net->L; ++l) U += net->dims[l];
    DevBuf dimg, dlab, dpot;
    IBMC_TRY(dimg.upload(images, (size_t)n_images * n, s));
    IBMC_TRY(dlab.reserve((size_t)n_images * 4));
    if (potentials) IBMC_TRY(dpot.reserve((size_t)n_images * U * 4));
    if (net->act == IBMC_ACT_RELU_Q8) {
        HIP_OK(launch_fwd_pots_q8(net->qd, net->fx, (const uint8_t *)dimg.p, n_images,
                                  potentials ? (int32_t *)dpot.p : nullptr, U, (int32_t *)dlab.p, s));
    } else {
        HIP_OK(launch_forward_f32(net->fd, (const uint8_t *)dimg.p, n_images, (int32_t *)dlab.p,
                                  potentials ? (float *)dpot.p : nullptr, U, s));
    }
    if (labels) HIP_OK(hipMemcpyAsync(labels, dlab.p, (size_t)n_images * 4, hipMemcpyDeviceToHost, s));
    if (potentials) HIP_OK(hipMemcpyAsync(potentials, dpot.p, (size_t)n_images * U * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_replay(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                   const int16_t *deltas, int32_t m, const ibmc_cex *recs, int64_t n,
                                   int32_t *labels_out) {
    clear_error();
    if (!ctx || !net || !image || !deltas || m < 1 || m > kMaxDeltas || n < 0 || (n > 0 && (!recs || !labels_out)))
        return fail(IBMC_E_INVALID, "bad argument");
    if (n == 0) return IBMC_OK;
    for (int64_t t = 0; t < n; ++t) {
        int64_t mk = 1;
        if (recs[t].k < 0 || recs[t].k > kMaxK || recs[t].k > net->dims[0])
            return fail(IBMC_E_INVALID, "record %lld: k = %d", (long long)t, recs[t].k);
        for (int j = 0; j < recs[t].k; ++j) mk *= m;
        if (recs[t].rank < 0 || recs[t].rank >= binom_small(net->dims[0], recs[t].k) * mk)
            return fail(IBMC_E_INVALID, "record %lld: rank out of range", (long long)t);
    }
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf dimg, dD, drec, dlab;
    IBMC_TRY(dimg.upload(image, net->dims[0], s));
    IBMC_TRY(dD.upload(deltas, (size_t)m * 2, s));
    IBMC_TRY(drec.upload(recs, (size_t)n * sizeof(ibmc_cex), s));
    IBMC_TRY(dlab.reserve((size_t)n * 4));
    if (net->act == IBMC_ACT_RELU_Q8)
        HIP_OK(launch_replay_q8(net->qd, (const uint8_t *)dimg.p, (const int16_t *)dD.p, m, (const CexRec *)drec.p,
                                n, (int32_t *)dlab.p, s));
    else
        HIP_OK(launch_replay_f32(net->fd, (const uint8_t *)dimg.p, (const int16_t *)dD.p, m, (const CexRec *)drec.p,
                                 n, (int32_t *)dlab.p, s));
    HIP_OK(hipMemcpyAsync(labels_out, dlab.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return IBMC_OK;
}
