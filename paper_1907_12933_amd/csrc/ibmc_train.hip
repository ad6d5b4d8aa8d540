// Host driver of the training of the float (sigmoid) networks: the loss and
// gradient of a labelled set, and mini-batch Adam training that returns a
// new network, so that the verifier's counterexamples, labelled with the
// clean image's label, can be added to the training set and the network
// checked again (Sec. VI).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ibmc_host.h"
#include "kernels_prop.h"
#include "kernels_q8.h"
#include "kernels_train.h"

using namespace ibmc;

namespace {

// Workgroups whose partial rows one launch may hold (256 MiB at most).
int64_t tiles_cap(int64_t n_params) {
    return std::max<int64_t>(1, std::min<int64_t>(4096, (256ll << 20) / (4 * n_params)));
}

ibmc_status check_train_args(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images, const int32_t *labels,
                             int64_t n) {
    if (!ctx || !net || !images || !labels || n < 1) return fail(IBMC_E_INVALID, "bad argument");
    if (net->act != IBMC_ACT_SIGMOID_F32) return fail(IBMC_E_UNIMPL, "training needs a float (sigmoid) network");
    if (net->device != ctx->device) return fail(IBMC_E_INVALID, "network lives on another device");
    const int nc = net->dims[net->L];
    for (int64_t t = 0; t < n; ++t)
        if (labels[t] < 0 || labels[t] >= nc)
            return fail(IBMC_E_INVALID, "label %d of sample %lld outside [0, %d)", labels[t], (long long)t, nc);
    return IBMC_OK;
}

std::vector<float> flat_theta(const ibmc_mlp *m) {
    std::vector<float> th;
    for (int l = 0; l < m->L; ++l) {
        th.insert(th.end(), m->Wf[l].begin(), m->Wf[l].end());
        th.insert(th.end(), m->bf[l].begin(), m->bf[l].end());
    }
    return th;
}

// splitmix64 (Steele, Lea, Flood 2014): the sample order of an epoch is a
// Fisher-Yates shuffle driven by splitmix64 of (seed, epoch).
uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void shuffle_epoch(uint64_t seed, int epoch, std::vector<int64_t> &ord) {
    uint64_t st = seed ^ (0xd1b54a32d192ed03ull * (uint64_t)(epoch + 1));
    for (size_t t = 0; t < ord.size(); ++t) ord[t] = (int64_t)t;
    for (size_t t = ord.size(); t > 1; --t) {
        const size_t j = (size_t)(splitmix64(st) % t);
        std::swap(ord[t - 1], ord[j]);
    }
}

// grad (+)= the gradient sum of elements e0 .. e0 + count - 1 of the pass,
// split into launches of at most tiles_cap workgroups; loss_acc += their loss.
ibmc_status grad_pass(const TrainNetDev &N, const float *theta, const uint8_t *images, const int32_t *labels,
                      const int64_t *order, int64_t e0, int64_t count, int tile, float inv_n, DevBuf &partial,
                      DevBuf &partial_loss, float *grad, bool accumulate, double *loss_acc, hipStream_t s) {
    const int64_t cap = tiles_cap(N.n_params);
    for (int64_t done = 0; done < count;) {
        const int64_t c = std::min<int64_t>(count - done, cap * tile);
        TrainGradParams P;
        P.net = N;
        P.theta = theta;
        P.images = images;
        P.labels = labels;
        P.order = order;
        P.e0 = e0 + done;
        P.count = c;
        P.tile = tile;
        P.inv_n = inv_n;
        P.partial = partial.as<float>();
        P.partial_loss = partial_loss.as<float>();
        HIP_OK(launch_train_grad(P, s));
        const int tiles = (int)((c + tile - 1) / tile);
        HIP_OK(launch_train_reduce(P.partial, P.partial_loss, tiles, N.n_params, grad, accumulate || done > 0,
                                   loss_acc, s));
        done += c;
    }
    return IBMC_OK;
}

ibmc_status reserve_partials(const TrainNetDev &N, int64_t count, int tile, DevBuf &partial, DevBuf &partial_loss) {
    const int64_t tiles = std::min<int64_t>(tiles_cap(N.n_params), (count + tile - 1) / tile);
    IBMC_TRY(partial.reserve((size_t)tiles * N.n_params * 4));
    IBMC_TRY(partial_loss.reserve((size_t)tiles * 4));
    return IBMC_OK;
}

}  // namespace

extern "C" ibmc_status ibmc_mlp_loss_grad(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images,
                                          const int32_t *labels, int64_t n, float *grad, double *loss) {
    clear_error();
    IBMC_TRY(check_train_args(ctx, net, images, labels, n));
    if (!grad && !loss) return fail(IBMC_E_INVALID, "grad and loss are both null");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const TrainNetDev N = train_layout(net->L, net->dims.data());
    const std::vector<float> th = flat_theta(net);
    const int tile = train_tile(N, kTrainMaxTile);
    DevBuf dth, dimg, dlab, dgrad, part, ploss, dloss;
    IBMC_TRY(dth.upload(th.data(), th.size() * 4, s));
    IBMC_TRY(dimg.upload(images, (size_t)n * net->dims[0], s));
    IBMC_TRY(dlab.upload(labels, (size_t)n * 4, s));
    IBMC_TRY(dgrad.reserve((size_t)N.n_params * 4));
    IBMC_TRY(dloss.reserve(8));
    IBMC_TRY(reserve_partials(N, n, tile, part, ploss));
    HIP_OK(launch_fill_u64(dloss.as<unsigned long long>(), 1, 0ull, s));
    IBMC_TRY(grad_pass(N, dth.as<float>(), dimg.as<uint8_t>(), dlab.as<int32_t>(), nullptr, 0, n, tile,
                       (float)(1.0 / (double)n), part, ploss, dgrad.as<float>(), false, dloss.as<double>(), s));
    double l = 0.0;
    HIP_OK(hipMemcpyAsync(&l, dloss.p, 8, hipMemcpyDeviceToHost, s));
    if (grad) HIP_OK(hipMemcpyAsync(grad, dgrad.p, (size_t)N.n_params * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (loss) *loss = l / (double)n;
    return IBMC_OK;
}

extern "C" ibmc_status ibmc_fit_mlp(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images, const int32_t *labels,
                                    int64_t n, const ibmc_fit_opts *o, ibmc_mlp **out, float *theta_out,
                                    double *epoch_loss) {
    clear_error();
    IBMC_TRY(check_train_args(ctx, net, images, labels, n));
    if (!o || !out) return fail(IBMC_E_INVALID, "null options or output");
    *out = nullptr;
    if (o->epochs < 1 || o->batch < 1 || !(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) ||
        !(o->beta2 >= 0.f && o->beta2 < 1.f) || !(o->eps >= 0.f))
        return fail(IBMC_E_INVALID, "bad training options");
    if (o->order)
        for (int64_t t = 0; t < (int64_t)o->epochs * n; ++t)
            if (o->order[t] < 0 || o->order[t] >= n)
                return fail(IBMC_E_INVALID, "order[%lld] = %lld outside [0, %lld)", (long long)t,
                            (long long)o->order[t], (long long)n);
    const float b1 = o->beta1 > 0.f ? o->beta1 : 0.9f, b2 = o->beta2 > 0.f ? o->beta2 : 0.999f;
    const float eps = o->eps > 0.f ? o->eps : 1e-8f;
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const TrainNetDev N = train_layout(net->L, net->dims.data());
    const int64_t B = std::min<int64_t>(o->batch, n);
    const int tile = train_tile(N, (int)std::min<int64_t>(kTrainMaxTile, (B + 31) / 32));
    std::vector<float> th = flat_theta(net);
    DevBuf dth, dmom, dvel, dgrad, dimg, dlab, dord, part, ploss, dloss;
    IBMC_TRY(dth.upload(th.data(), th.size() * 4, s));
    IBMC_TRY(dmom.reserve((size_t)N.n_params * 4));
    IBMC_TRY(dvel.reserve((size_t)N.n_params * 4));
    IBMC_TRY(dgrad.reserve((size_t)N.n_params * 4));
    IBMC_TRY(dimg.upload(images, (size_t)n * net->dims[0], s));
    IBMC_TRY(dlab.upload(labels, (size_t)n * 4, s));
    IBMC_TRY(dord.reserve((size_t)n * 8));
    IBMC_TRY(dloss.reserve((size_t)o->epochs * 8));
    IBMC_TRY(reserve_partials(N, B, tile, part, ploss));
    HIP_OK(launch_fill_u64(dmom.as<unsigned long long>(), (N.n_params + 1) / 2, 0ull, s));
    HIP_OK(launch_fill_u64(dvel.as<unsigned long long>(), (N.n_params + 1) / 2, 0ull, s));
    HIP_OK(launch_fill_u64(dloss.as<unsigned long long>(), o->epochs, 0ull, s));
    std::vector<int64_t> ord(n);
    int64_t step = 0;
    for (int ep = 0; ep < o->epochs; ++ep) {
        if (o->order)
            std::copy(o->order + (int64_t)ep * n, o->order + (int64_t)(ep + 1) * n, ord.begin());
        else
            shuffle_epoch(o->seed, ep, ord);
        HIP_OK(hipMemcpyAsync(dord.p, ord.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
        for (int64_t b0 = 0; b0 < n; b0 += B) {
            const int64_t cnt = std::min<int64_t>(B, n - b0);
            IBMC_TRY(grad_pass(N, dth.as<float>(), dimg.as<uint8_t>(), dlab.as<int32_t>(), dord.as<int64_t>(), b0,
                               cnt, tile, (float)(1.0 / (double)cnt), part, ploss, dgrad.as<float>(), false,
                               dloss.as<double>() + ep, s));
            ++step;
            const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
            const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
            HIP_OK(launch_prop_adam(dth.as<float>(), dgrad.as<float>(), dmom.as<float>(), dvel.as<float>(),
                                    (int)N.n_params, o->lr, b1, b2, eps, c1, c2, s));
        }
        HIP_OK(hipStreamSynchronize(s));   // ord is rewritten next epoch
    }
    std::vector<double> el(o->epochs);
    HIP_OK(hipMemcpyAsync(th.data(), dth.p, th.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(el.data(), dloss.p, el.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (float v : th)
        if (!std::isfinite(v)) return fail(IBMC_E_RANGE, "training diverged (non-finite parameter)");
    if (epoch_loss)
        for (int ep = 0; ep < o->epochs; ++ep) epoch_loss[ep] = el[ep] / (double)n;
    if (theta_out) memcpy(theta_out, th.data(), th.size() * 4);
    std::vector<const void *> Wp(net->L), bp(net->L);
    for (int l = 1; l <= net->L; ++l) {
        Wp[l - 1] = th.data() + N.toff[l];
        bp[l - 1] = th.data() + N.toff[l] + (int64_t)N.dims[l] * N.dims[l - 1];
    }
    ibmc_mlp_desc d;
    d.n_layers = net->L;
    d.dims = net->dims.data();
    d.act = IBMC_ACT_SIGMOID_F32;
    d.W = Wp.data();
    d.b = bp.data();
    d.shift = nullptr;
    return ibmc_load_mlp(ctx, &d, out);
}
