// Training kernels of the float (sigmoid) networks: a workgroup takes a tile
// of samples, keeps their activations and deltas in LDS, runs the forward
// pass (a_0 = x / 256, sigmoid hidden layers, linear logits, Eq. (2)), the
// softmax cross-entropy against the label and the backward pass, and writes
// its tile's gradient sum as one row of a partial buffer; a second kernel
// adds the rows in tile order.  No atomics: the gradient of a batch is the
// same on every run.
#include "kernels_train.h"

namespace ibmc {

TrainNetDev train_layout(int L, const int *dims) {
    TrainNetDev N{};
    N.L = L;
    int64_t t = 0;
    int a = dims[0];
    N.dims[0] = dims[0];
    N.aoff[0] = 0;
    for (int l = 1; l <= L; ++l) {
        N.dims[l] = dims[l];
        N.toff[l] = t;
        t += (int64_t)dims[l] * dims[l - 1] + dims[l];
        N.aoff[l] = a;
        a += dims[l];
    }
    N.n_params = t;
    N.units = a;
    return N;
}

size_t train_lds_bytes(const TrainNetDev &N, int tile) {
    return (size_t)tile * (2 * N.units - N.dims[0] + 1) * sizeof(float);
}

int train_tile(const TrainNetDev &N, int wanted) {
    int t = std::max(1, std::min(wanted, kTrainMaxTile));
    while (t > 1 && train_lds_bytes(N, t) > (size_t)kTrainLdsBytes) --t;
    return t;
}

__global__ void __launch_bounds__(kTrainThreads) train_grad_kernel(TrainGradParams P) {
    extern __shared__ float lds[];
    const TrainNetDev &N = P.net;
    const int tid = threadIdx.x, T = P.tile, L = N.L, n = N.dims[0], U = N.units, UD = U - n;
    const int64_t first = (int64_t)blockIdx.x * T;
    const int S = (int)min((int64_t)T, P.count - first);
    float *act = lds;               // [T][U]
    float *del = lds + T * U;       // [T][UD]
    float *loss = del + T * UD;     // [T]
    for (int t = tid; t < S * n; t += kTrainThreads) {
        const int s = t / n, i = t - s * n;
        const int64_t e = P.e0 + first + s;
        const int64_t img = P.order ? P.order[e] : e;
        act[s * U + i] = (float)P.images[img * n + i] * (1.f / 256.f);
    }
    __syncthreads();
    for (int l = 1; l <= L; ++l) {
        const int nin = N.dims[l - 1], nout = N.dims[l];
        const float *W = P.theta + N.toff[l], *b = W + (int64_t)nout * nin;
        for (int t = tid; t < S * nout; t += kTrainThreads) {
            const int s = t / nout, j = t - s * nout;
            const float *a = act + s * U + N.aoff[l - 1];
            const float *w = W + (int64_t)j * nin;
            float u = b[j];
            int i = 0;
            for (; i + 4 <= nin; i += 4) {
                u = fmaf(w[i], a[i], u);
                u = fmaf(w[i + 1], a[i + 1], u);
                u = fmaf(w[i + 2], a[i + 2], u);
                u = fmaf(w[i + 3], a[i + 3], u);
            }
            for (; i < nin; ++i) u = fmaf(w[i], a[i], u);
            act[s * U + N.aoff[l] + j] = (l < L) ? 1.f / (1.f + expf(-u)) : u;
        }
        __syncthreads();
    }
    // softmax cross-entropy of each sample's logits; dL/du of the logits
    const int nc = N.dims[L];
    for (int s = tid; s < S; s += kTrainThreads) {
        const int64_t e = P.e0 + first + s;
        const int y = P.labels[P.order ? P.order[e] : e];
        const float *z = act + s * U + N.aoff[L];
        float zmax = z[0];
        for (int c = 1; c < nc; ++c) zmax = fmaxf(zmax, z[c]);
        float sum = 0.f;
        for (int c = 0; c < nc; ++c) sum += expf(z[c] - zmax);
        loss[s] = logf(sum) - (z[y] - zmax);
        float *d = del + s * UD + N.aoff[L] - n;
        const float inv = 1.f / sum;
        for (int c = 0; c < nc; ++c) d[c] = (expf(z[c] - zmax) * inv - (c == y ? 1.f : 0.f)) * P.inv_n;
    }
    __syncthreads();
    float *out = P.partial + (int64_t)blockIdx.x * N.n_params;
    for (int l = L; l >= 1; --l) {
        const int nin = N.dims[l - 1], nout = N.dims[l];
        const int dl = N.aoff[l] - n, al = N.aoff[l - 1];
        float *g = out + N.toff[l];
        // this tile's sum of dL/du_l a_{l-1}^T and of dL/du_l
        for (int t = tid; t < nout * nin; t += kTrainThreads) {
            const int j = t / nin, i = t - j * nin;
            float acc = 0.f;
            for (int s = 0; s < S; ++s) acc = fmaf(del[s * UD + dl + j], act[s * U + al + i], acc);
            g[t] = acc;
        }
        for (int j = tid; j < nout; j += kTrainThreads) {
            float acc = 0.f;
            for (int s = 0; s < S; ++s) acc += del[s * UD + dl + j];
            g[(int64_t)nout * nin + j] = acc;
        }
        if (l > 1) {
            // dL/du_{l-1} = (W_l^T dL/du_l) a (1 - a)
            const float *W = P.theta + N.toff[l];
            for (int t = tid; t < S * nin; t += kTrainThreads) {
                const int s = t / nin, i = t - s * nin;
                const float *d = del + s * UD + dl;
                float acc = 0.f;
                for (int j = 0; j < nout; ++j) acc = fmaf(W[(int64_t)j * nin + i], d[j], acc);
                const float a = act[s * U + al + i];
                del[s * UD + (al - n) + i] = acc * a * (1.f - a);
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        float acc = 0.f;
        for (int s = 0; s < S; ++s) acc += loss[s];
        P.partial_loss[blockIdx.x] = acc;
    }
}

__global__ void __launch_bounds__(256) train_reduce_kernel(const float *partial, const float *partial_loss, int tiles,
                                                           int64_t n_params, float *grad, int accumulate,
                                                           double *loss_acc) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_params;
         t += (int64_t)gridDim.x * blockDim.x) {
        float acc = accumulate ? grad[t] : 0.f;
        for (int r = 0; r < tiles; ++r) acc += partial[(int64_t)r * n_params + t];
        grad[t] = acc;
    }
    if (loss_acc && blockIdx.x == 0 && threadIdx.x == 0) {
        double acc = 0.0;
        for (int r = 0; r < tiles; ++r) acc += (double)partial_loss[r];
        *loss_acc += acc;
    }
}

hipError_t launch_train_grad(const TrainGradParams &P, hipStream_t s) {
    if (P.count <= 0) return hipSuccess;
    const int64_t tiles = (P.count + P.tile - 1) / P.tile;
    hipLaunchKernelGGL(train_grad_kernel, dim3((unsigned)tiles), dim3(kTrainThreads), train_lds_bytes(P.net, P.tile),
                       s, P);
    return hipGetLastError();
}

hipError_t launch_train_reduce(const float *partial, const float *partial_loss, int tiles, int64_t n_params,
                               float *grad, bool accumulate, double *loss_acc, hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_params + 255) / 256, 4096));
    hipLaunchKernelGGL(train_reduce_kernel, dim3(grid), dim3(256), 0, s, partial, partial_loss, tiles, n_params, grad,
                       accumulate ? 1 : 0, loss_acc);
    return hipGetLastError();
}

}  // namespace ibmc
