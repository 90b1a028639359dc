// Random-row gather probe: the bandwidth ceiling of the search's memory
// access pattern.  Whole stored rows at random positions are read by groups
// of G lanes with the scoring layout of the search (64 / G rows per round,
// the same rounds in flight), decoded and summed, with no dependent work
// between rounds -- what the row gathers of the search could reach if
// nothing else waited on them.
#include "search_core.h"

namespace nhq {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int DP, int ST>
__global__ __launch_bounds__(256) void k_gather_probe(const void *__restrict__ vbase, const float *__restrict__ scale,
                                                      int64_t n, int rounds, uint64_t seed, float *__restrict__ sink)
{
    using S = Shape<DP>;
    using T = typename Chunk<ST>::T;
    const int lane = threadIdx.x & 63;
    const int g = lane % S::G, gi = lane / S::G;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    float acc = 0.0f;
    constexpr int RB = Lay<DP, ST>::RB;
    for (int r0 = 0; r0 < rounds; r0 += RB) {
        T buf[RB][S::NCH];
        float sc[RB];
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            const uint64_t j = (wave * (uint64_t)rounds + (uint64_t)(r0 + rr)) * S::NG + gi;
            const int64_t id = (int64_t)(mix64(seed + 0x9E3779B97F4A7C15ull * (j + 1)) % (uint64_t)n);
            const T *row = reinterpret_cast<const T *>(vbase) + id * (DP / 4);
#pragma unroll
            for (int c = 0; c < S::NCH; ++c)
                buf[rr][c] = row[g + S::G * c];
            sc[rr] = ST == NHQ_STORAGE_FP8 ? scale[id] : 1.0f;
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr)
#pragma unroll
            for (int c = 0; c < S::NCH; ++c) {
                const float4 x = decode<ST>(buf[rr][c], sc[rr]);
                acc += (x.x + x.y) + (x.z + x.w);
            }
    }
    sink[wave * 64 + lane] = acc;
}

template <int DP>
int launch_probe_dp(const Index *ix, int64_t waves, int rounds, uint64_t seed, float *sink, hipStream_t st)
{
    const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    switch (ix->storage) {
    case NHQ_STORAGE_FP32:
        hipLaunchKernelGGL((k_gather_probe<DP, NHQ_STORAGE_FP32>), grid, block, 0, st, ix->vecs, ix->scale, ix->n,
                           rounds, seed, sink);
        break;
    case NHQ_STORAGE_BF16:
        hipLaunchKernelGGL((k_gather_probe<DP, NHQ_STORAGE_BF16>), grid, block, 0, st, ix->vecs, ix->scale, ix->n,
                           rounds, seed, sink);
        break;
    default:
        hipLaunchKernelGGL((k_gather_probe<DP, NHQ_STORAGE_FP8>), grid, block, 0, st, ix->vecs, ix->scale, ix->n,
                           rounds, seed, sink);
        break;
    }
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // namespace
}  // namespace nhq

using namespace nhq;

extern "C" int nhq_gather_probe(const nhq_index *h, int64_t waves, int32_t rounds, uint64_t seed, float *sink,
                                int64_t *rows_read, void *stream)
{
    if (!h || !sink)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    if (waves < 4 || waves % 4 != 0 || rounds < 1 || waves > (int64_t(1) << 30))
        return fail(NHQ_EINVAL, "waves must be a positive multiple of 4 (at most 2^30), rounds >= 1");
    int rb = 0, ng = 0;
    hipStream_t st = (hipStream_t)stream;
    int rc = NHQ_OK;
    switch (ix->dp) {
#define NHQ_P(DPV)                                                       \
    case DPV:                                                            \
        rb = ix->storage == NHQ_STORAGE_FP32 ? Lay<DPV, NHQ_STORAGE_FP32>::RB \
             : ix->storage == NHQ_STORAGE_BF16 ? Lay<DPV, NHQ_STORAGE_BF16>::RB \
                                               : Lay<DPV, NHQ_STORAGE_FP8>::RB; \
        ng = Shape<DPV>::NG;                                             \
        if (rounds % rb != 0)                                            \
            return fail(NHQ_EINVAL, "rounds must be a multiple of the rounds in flight"); \
        rc = launch_probe_dp<DPV>(ix, waves, rounds, seed, sink, st);    \
        break;
        NHQ_P(32)
        NHQ_P(64)
        NHQ_P(96)
        NHQ_P(128)
        NHQ_P(256)
        NHQ_P(512)
        NHQ_P(960)
        NHQ_P(1024)
#undef NHQ_P
    default:
        return fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    if (rows_read)
        *rows_read = waves * (int64_t)rounds * ng;
    return rc;
}
