// The learned stop network: training samples from search traces, forward /
// backward / Adam kernels (float32), fp16 export, and the in-loop inference
// exposed for testing.
//
// Network: 8 -> 64 -> 64 -> 2 with ReLU.  Loss per sample:
//   softplus(z0) - y_stop z0  +  lam * huber1(z1 - y_beam)
// averaged over the batch.  Parameter vector order: W1 [64][8], b1 [64],
// W2 [64][64], b2 [64], W3 [2][64], b3 [2] (4866 floats).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "mlp_infer.h"
#include "nhq_internal.h"

namespace nhq {
namespace {

constexpr int kP = NHQ_MLP_PARAMS;
constexpr int oW1 = 0, oB1 = 512, oW2 = 576, oB2 = 4672, oW3 = 4736, oB3 = 4864;
constexpr int kChunk = 128;  // samples per workgroup in the gradient kernel

// ---------------------------------------------------------------- samples
__global__ void k_trace_samples(const float *__restrict__ feat, const uint32_t *__restrict__ hop,
                                const uint32_t *__restrict__ hash, const int32_t *__restrict__ count,
                                const uint32_t *__restrict__ final_hash, const uint32_t *__restrict__ counters,
                                const int64_t *__restrict__ off, int64_t nq, int cap, float *__restrict__ X,
                                float *__restrict__ ys, float *__restrict__ yb)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int c = min(count[q], cap);
        // y_beam: the first checkpoint from which every later one already
        // holds the final top-k (the final hop count when the last does not)
        uint32_t first = counters ? counters[2 * q + 1] : 0u;
        for (int t = c - 1; t >= 0 && hash[q * cap + t] == final_hash[q]; --t)
            first = hop[q * cap + t];
        const float target = log2f(fmaxf(1.0f, (float)first));
        for (int t = 0; t < c; ++t) {
            const int64_t o = off[q] + t;
            for (int i = 0; i < 8; ++i)
                X[o * 8 + i] = feat[(q * cap + t) * 8 + i];
            ys[o] = hash[q * cap + t] == final_hash[q] ? 1.0f : 0.0f;
            yb[o] = target;
        }
    }
}

// ---------------------------------------------------------------- gradient
// One workgroup of 256 threads takes a chunk of up to 128 samples: forward
// (one thread per sample), then the weight gradients as sums over the chunk
// in a fixed order.  Writes the chunk's gradient sum and loss sum (each
// sample's terms already divided by the batch size `inv_b`).
__global__ __launch_bounds__(256) void k_mlp_grad_chunk(const float *__restrict__ params,
                                                        const float *__restrict__ X,
                                                        const float *__restrict__ ys,
                                                        const float *__restrict__ yb,
                                                        const int32_t *__restrict__ perm, int64_t n0,
                                                        int64_t n, float inv_b, float lam,
                                                        float *__restrict__ gpart,
                                                        float *__restrict__ lpart,
                                                        float *__restrict__ zout)
{
    extern __shared__ __align__(16) float sm[];
    float *P = sm;                      // [kP]
    float *xs = P + kP + 2;             // [128][8]
    float *h1 = xs + kChunk * 8;        // [128][64] activations, later dA1
    float *h2 = h1 + kChunk * 64;       // [128][64] activations, later dA2
    float *dz = h2 + kChunk * 64;       // [128][2]
    float *ls = dz + kChunk * 2;        // [128]
    const int t = threadIdx.x;
    const int64_t c0 = n0 + (int64_t)blockIdx.x * kChunk;
    const int nc = (int)min<int64_t>(kChunk, n - c0);
    for (int i = t; i < kP; i += 256)
        P[i] = params[i];
    for (int i = t; i < kChunk * 8; i += 256) {
        const int s = i / 8;
        float v = 0.0f;
        if (s < nc) {
            const int64_t g = perm ? perm[c0 + s] : c0 + s;
            v = X[g * 8 + (i % 8)];
        }
        xs[i] = v;
    }
    __syncthreads();
    // forward, one thread per sample
    if (t < kChunk) {
        const int s = t;
        float z0 = P[oB3], z1 = P[oB3 + 1];
        for (int j = 0; j < 64; ++j) {
            float a = P[oB1 + j];
            for (int i = 0; i < 8; ++i)
                a = fmaf(P[oW1 + j * 8 + i], xs[s * 8 + i], a);
            h1[s * 64 + j] = fmaxf(a, 0.0f);
        }
        for (int j = 0; j < 64; ++j) {
            float a = P[oB2 + j];
            for (int i = 0; i < 64; ++i)
                a = fmaf(P[oW2 + j * 64 + i], h1[s * 64 + i], a);
            const float hv = fmaxf(a, 0.0f);
            h2[s * 64 + j] = hv;
            z0 = fmaf(P[oW3 + j], hv, z0);
            z1 = fmaf(P[oW3 + 64 + j], hv, z1);
        }
        float g0 = 0.0f, g1 = 0.0f, l = 0.0f;
        if (s < nc) {
            const int64_t g = perm ? perm[c0 + s] : c0 + s;
            const float y = ys[g], tb = yb[g];
            // softplus(z0) - y z0, computed stably
            const float sp = fmaxf(z0, 0.0f) + log1pf(expf(-fabsf(z0)));
            const float r = z1 - tb, ar = fabsf(r);
            l = (sp - y * z0 + lam * (ar <= 1.0f ? 0.5f * r * r : ar - 0.5f)) * inv_b;
            g0 = (1.0f / (1.0f + expf(-z0)) - y) * inv_b;
            g1 = lam * fminf(fmaxf(r, -1.0f), 1.0f) * inv_b;
            if (zout) {
                zout[(c0 + s) * 2] = z0;
                zout[(c0 + s) * 2 + 1] = z1;
            }
        }
        dz[s * 2] = g0;
        dz[s * 2 + 1] = g1;
        ls[s] = l;
    }
    __syncthreads();
    float *gp = gpart + (int64_t)blockIdx.x * (kP + 1);
    // dW3, db3 (sums over the chunk in sample order)
    if (t < 130) {
        float acc = 0.0f;
        if (t < 128) {
            const int o = t / 64, j = t % 64;
            for (int s = 0; s < kChunk; ++s)
                acc = fmaf(dz[s * 2 + o], h2[s * 64 + j], acc);
            gp[oW3 + t] = acc;
        } else {
            for (int s = 0; s < kChunk; ++s)
                acc += dz[s * 2 + (t - 128)];
            gp[oB3 + (t - 128)] = acc;
        }
    }
    if (t == 255) {
        float acc = 0.0f;
        for (int s = 0; s < kChunk; ++s)
            acc += ls[s];
        lpart[blockIdx.x] = acc;
    }
    __syncthreads();
    // dA2 = (dZ W3) * [h2 > 0], in place of h2
    if (t < kChunk) {
        const int s = t;
        for (int j = 0; j < 64; ++j) {
            const float d = dz[s * 2] * P[oW3 + j] + dz[s * 2 + 1] * P[oW3 + 64 + j];
            h2[s * 64 + j] = h2[s * 64 + j] > 0.0f ? d : 0.0f;
        }
    }
    __syncthreads();
    // dW2 [64][64] and db2
    for (int o = t; o < 64 * 64 + 64; o += 256) {
        float acc = 0.0f;
        if (o < 4096) {
            const int i = o / 64, j = o % 64;
            for (int s = 0; s < kChunk; ++s)
                acc = fmaf(h2[s * 64 + i], h1[s * 64 + j], acc);
            gp[oW2 + o] = acc;
        } else {
            const int i = o - 4096;
            for (int s = 0; s < kChunk; ++s)
                acc += h2[s * 64 + i];
            gp[oB2 + i] = acc;
        }
    }
    __syncthreads();
    // dA1 = (dA2 W2) * [h1 > 0], in place of h1 (entry j is read only for its own mask)
    if (t < kChunk) {
        const int s = t;
        for (int j = 0; j < 64; ++j) {
            float acc = 0.0f;
            for (int i = 0; i < 64; ++i)
                acc = fmaf(h2[s * 64 + i], P[oW2 + i * 64 + j], acc);
            h1[s * 64 + j] = h1[s * 64 + j] > 0.0f ? acc : 0.0f;
        }
    }
    __syncthreads();
    // dW1 [64][8] and db1
    for (int o = t; o < 512 + 64; o += 256) {
        float acc = 0.0f;
        if (o < 512) {
            const int i = o / 8, j = o % 8;
            for (int s = 0; s < kChunk; ++s)
                acc = fmaf(h1[s * 64 + i], xs[s * 8 + j], acc);
            gp[oW1 + o] = acc;
        } else {
            const int i = o - 512;
            for (int s = 0; s < kChunk; ++s)
                acc += h1[s * 64 + i];
            gp[oB1 + i] = acc;
        }
    }
}

// sum the chunk gradients (fixed order) and, when `adam`, take one Adam step
__global__ void k_mlp_reduce(const float *__restrict__ gpart, const float *__restrict__ lpart,
                             int chunks, float *__restrict__ grad, float *__restrict__ loss,
                             float *__restrict__ params, float *__restrict__ mom, int adam,
                             float lr, float bc1, float bc2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kP; i += gridDim.x * blockDim.x) {
        float g = 0.0f;
        for (int c = 0; c < chunks; ++c)
            g += gpart[(int64_t)c * (kP + 1) + i];
        if (grad)
            grad[i] = g;
        if (adam) {
            float m1 = mom[i], m2 = mom[kP + i];
            m1 = 0.9f * m1 + 0.1f * g;
            m2 = 0.999f * m2 + 0.001f * g * g;
            mom[i] = m1;
            mom[kP + i] = m2;
            params[i] -= lr * (m1 / bc1) / (sqrtf(m2 / bc2) + 1e-8f);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        float l = 0.0f;
        for (int c = 0; c < chunks; ++c)
            l += lpart[c];
        loss[0] += l;
    }
}

// parameters -> fp16 in the device inference layout
__global__ void k_to_half(const float *__restrict__ p, uint16_t *__restrict__ h, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const _Float16 v = (_Float16)p[i];
        uint16_t b;
        __builtin_memcpy(&b, &v, 2);
        h[mlp_device_index(i)] = b;
    }
}

__global__ __launch_bounds__(64) void k_mlp_eval(const uint16_t *__restrict__ w, const float *__restrict__ X,
                                                 int64_t n, float *__restrict__ Z)
{
    __shared__ __align__(16) float scratch[64];
    __shared__ __align__(16) float f[8];
    const int j = threadIdx.x;
    const int64_t s = blockIdx.x;
    if (s >= n)
        return;
    if (j < 8)
        f[j] = X[s * 8 + j];
    __syncthreads();
    float z0, z1;
    mlp_infer(w, f, scratch, z0, z1);
    if (j == 0) {
        Z[s * 2] = z0;
        Z[s * 2 + 1] = z1;
    }
}

size_t grad_lds() { return sizeof(float) * ((size_t)kP + 2 + kChunk * 8 + 2 * kChunk * 64 + kChunk * 2 + kChunk); }

int run_grad(const float *params, const float *X, const float *ys, const float *yb, const int32_t *perm,
             int64_t n0, int64_t nb, int64_t n_total, float lam, float *gpart, float *lpart, float *z,
             hipStream_t st)
{
    const int chunks = (int)((nb + kChunk - 1) / kChunk);
    const size_t lds = grad_lds();
    NHQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp_grad_chunk),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_mlp_grad_chunk, dim3(chunks), dim3(256), lds, st, params, X, ys, yb, perm, n0,
                       n0 + nb, 1.0f / (float)n_total, lam, gpart, lpart, z);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // namespace
}  // namespace nhq

using namespace nhq;

extern "C" {

int nhq_trace_samples(const nhq_trace *tr, int64_t nq, const uint32_t *counters, float *X,
                      float *y_stop, float *y_beam, int64_t *n_out, void *stream)
{
    if (!tr || !X || !y_stop || !y_beam || !n_out || nq < 0)
        return fail(NHQ_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> cnt((size_t)nq);
    if (nq > 0) {
        NHQ_HIP(hipMemcpyAsync(cnt.data(), tr->count, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost, st));
        NHQ_HIP(hipStreamSynchronize(st));
    }
    std::vector<int64_t> off((size_t)nq + 1, 0);
    for (int64_t q = 0; q < nq; ++q)
        off[q + 1] = off[q] + std::min(std::max(cnt[q], 0), tr->cap);
    *n_out = off[nq];
    if (nq == 0)
        return NHQ_OK;
    int64_t *doff = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&doff, sizeof(int64_t) * (size_t)(nq + 1), st));
    NHQ_HIP(hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * (size_t)(nq + 1), hipMemcpyHostToDevice, st));
    const int grid = (int)std::min<int64_t>(4096, (nq + 255) / 256);
    hipLaunchKernelGGL(k_trace_samples, dim3(grid), dim3(256), 0, st, tr->feat, tr->hop, tr->hash,
                       tr->count, tr->final_hash, counters, doff, nq, tr->cap, X, y_stop, y_beam);
    NHQ_HIP(hipGetLastError());
    NHQ_HIP(hipFreeAsync(doff, st));
    NHQ_HIP(hipStreamSynchronize(st));
    return NHQ_OK;
}

int nhq_mlp_grad(const float *params, const float *X, const float *y_stop, const float *y_beam,
                 int64_t n, float lam, float *grad, float *loss, float *z, void *stream)
{
    if (!params || !X || !y_stop || !y_beam || !grad || !loss || n < 1)
        return fail(NHQ_EINVAL, "need device arrays and n >= 1");
    hipStream_t st = (hipStream_t)stream;
    const int chunks = (int)((n + kChunk - 1) / kChunk);
    float *gpart = nullptr, *lpart = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&gpart, sizeof(float) * (size_t)chunks * (kP + 1), st));
    NHQ_HIP(hipMallocAsync((void **)&lpart, sizeof(float) * (size_t)chunks, st));
    NHQ_HIP(hipMemsetAsync(loss, 0, sizeof(float), st));
    int rc = run_grad(params, X, y_stop, y_beam, nullptr, 0, n, n, lam, gpart, lpart, z, st);
    if (rc == NHQ_OK) {
        hipLaunchKernelGGL(k_mlp_reduce, dim3(20), dim3(256), 0, st, gpart, lpart, chunks, grad, loss,
                           nullptr, nullptr, 0, 0.0f, 1.0f, 1.0f);
        if (hipGetLastError() != hipSuccess)
            rc = fail(NHQ_EHIP, "reduce launch failed");
    }
    (void)hipFreeAsync(gpart, st);
    (void)hipFreeAsync(lpart, st);
    return rc;
}

int nhq_mlp_train(float *params, float *adam_state, int64_t *step, const float *X, const float *y_stop,
                  const float *y_beam, int64_t n, int32_t epochs, int32_t batch, float lr, float lam,
                  uint64_t seed, float *loss_out, void *stream)
{
    if (!params || !adam_state || !step || !X || !y_stop || !y_beam || n < 1 || epochs < 0)
        return fail(NHQ_EINVAL, "bad training arguments");
    if (batch < kChunk || batch % kChunk != 0)
        return fail(NHQ_EINVAL, "batch must be a positive multiple of 128");
    hipStream_t st = (hipStream_t)stream;
    const int chunks_max = batch / kChunk;
    float *gpart = nullptr, *lpart = nullptr;
    int32_t *perm = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&gpart, sizeof(float) * (size_t)chunks_max * (kP + 1), st));
    NHQ_HIP(hipMallocAsync((void **)&lpart, sizeof(float) * (size_t)chunks_max, st));
    NHQ_HIP(hipMallocAsync((void **)&perm, sizeof(int32_t) * (size_t)n, st));
    std::vector<int32_t> hp((size_t)n);
    uint64_t state = seed;
    int rc = NHQ_OK;
    for (int ep = 0; ep < epochs && rc == NHQ_OK; ++ep) {
        // Fisher-Yates shuffle driven by splitmix64
        std::iota(hp.begin(), hp.end(), 0);
        for (int64_t i = n - 1; i > 0; --i) {
            const int64_t j = (int64_t)(splitmix64_next(state) % (uint64_t)(i + 1));
            std::swap(hp[i], hp[j]);
        }
        if (hipMemcpyAsync(perm, hp.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "permutation upload failed");
            break;
        }
        // the host vector is reused next epoch: wait for the copy
        if (hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "synchronisation failed");
            break;
        }
        float *lacc = loss_out ? loss_out + ep : nullptr;
        if (lacc)
            (void)hipMemsetAsync(lacc, 0, sizeof(float), st);
        for (int64_t b0 = 0; b0 < n && rc == NHQ_OK; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - b0);
            rc = run_grad(params, X, y_stop, y_beam, perm, b0, nb, nb, lam, gpart, lpart, nullptr, st);
            if (rc != NHQ_OK)
                break;
            *step += 1;
            const float bc1 = 1.0f - std::pow(0.9f, (float)*step);
            const float bc2 = 1.0f - std::pow(0.999f, (float)*step);
            const int chunks = (int)((nb + kChunk - 1) / kChunk);
            hipLaunchKernelGGL(k_mlp_reduce, dim3(20), dim3(256), 0, st, gpart, lpart, chunks, nullptr, lacc,
                               params, adam_state, 1, lr, bc1, bc2);
            if (hipGetLastError() != hipSuccess)
                rc = fail(NHQ_EHIP, "reduce launch failed");
        }
        // per-epoch mean: the loss accumulator holds the sum of batch means
        if (rc == NHQ_OK && lacc) {
            const float nb_count = (float)((n + batch - 1) / batch);
            float h = 0.0f;
            (void)hipMemcpyAsync(&h, lacc, sizeof(float), hipMemcpyDeviceToHost, st);
            (void)hipStreamSynchronize(st);
            h /= nb_count;
            (void)hipMemcpyAsync(lacc, &h, sizeof(float), hipMemcpyHostToDevice, st);
            (void)hipStreamSynchronize(st);
        }
    }
    (void)hipFreeAsync(gpart, st);
    (void)hipFreeAsync(lpart, st);
    (void)hipFreeAsync(perm, st);
    (void)hipStreamSynchronize(st);
    return rc;
}

int nhq_mlp_load(nhq_index *h, const float *params, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    Index *ix = &h->impl;
    hipStream_t st = (hipStream_t)stream;
    if (!params) {
        NHQ_HIP(hipStreamSynchronize(st));
        if (ix->mlp)
            NHQ_HIP(hipFree(ix->mlp));
        ix->mlp = nullptr;
        return NHQ_OK;
    }
    if (!ix->mlp && hipMalloc(&ix->mlp, sizeof(uint16_t) * kP) != hipSuccess)
        return fail(NHQ_ENOMEM, "network allocation failed");
    hipLaunchKernelGGL(k_to_half, dim3(20), dim3(256), 0, st, params, (uint16_t *)ix->mlp, kP);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

int nhq_mlp_eval(const nhq_index *h, const float *X, int64_t n, float *Z, void *stream)
{
    if (!h || !X || !Z || n < 0)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    if (!ix->mlp)
        return fail(NHQ_EINVAL, "no network loaded");
    if (n == 0)
        return NHQ_OK;
    hipLaunchKernelGGL(k_mlp_eval, dim3((unsigned)n), dim3(64), 0, (hipStream_t)stream,
                       (const uint16_t *)ix->mlp, X, n, Z);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // extern "C"
