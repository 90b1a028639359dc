// In-loop inference of the stop network (8 -> 64 -> 64 -> 2, ReLU) by one
// wavefront: fp16 weights, float32 activations and accumulation.  Lane j
// computes hidden unit j.
//
// Device weight layout (fp16, NHQ_MLP_PARAMS values), chosen so that every
// weight load of the wave is contiguous across lanes:
//   W1 [64][8] (lane j reads its 8 weights as one 16-byte load), b1 [64],
//   W2 as [16][64][4]: element (j, i) of W2 [64][64] at ((i/4)*64 + j)*4 + i%4
//   (lane j reads inputs 4c..4c+3 as one 8-byte load, 64 lanes contiguous),
//   b2 [64], W3 [2][64], b3 [2].
// The parameter vector's order (W1, b1, W2 [64][64] row-major, b2, W3, b3)
// maps to it with mlp_device_index.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nhq {

constexpr int kMlpW1 = 0, kMlpB1 = 512, kMlpW2 = 576, kMlpB2 = 4672, kMlpW3 = 4736, kMlpB3 = 4864;

__host__ __device__ inline int mlp_device_index(int p)
{
    if (p < kMlpW2 || p >= kMlpB2)
        return p;
    const int e = p - kMlpW2, j = e / 64, i = e % 64;
    return kMlpW2 + ((i / 4) * 64 + j) * 4 + (i % 4);
}

__device__ __forceinline__ float mlp_h2f(uint32_t bits16)
{
    _Float16 v;
    const uint16_t b = (uint16_t)bits16;
    __builtin_memcpy(&v, &b, 2);
    return (float)v;
}

// z0 (stop logit) and z1 (log2 hop budget) for the 8 features f (in LDS,
// read by every lane); `scratch` holds 64 floats of LDS.  Both 16-byte
// aligned.  The wave synchronises on
// LDS around its use.
__device__ __forceinline__ void mlp_infer(const uint16_t *w, const float *f, float *scratch, float &z0,
                                          float &z1)
{
    const int j = threadIdx.x & 63;
    f = reinterpret_cast<const float *>(__builtin_assume_aligned(f, 16));
    scratch = reinterpret_cast<float *>(__builtin_assume_aligned(scratch, 16));
    const uint4 w1 = reinterpret_cast<const uint4 *>(w + kMlpW1)[j];
    const uint32_t w1v[4] = {w1.x, w1.y, w1.z, w1.w};
    float a1 = mlp_h2f(w[kMlpB1 + j]);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        a1 = fmaf(mlp_h2f(i & 1 ? w1v[i / 2] >> 16 : w1v[i / 2]), f[i], a1);
    scratch[j] = fmaxf(a1, 0.0f);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint2 *W2 = reinterpret_cast<const uint2 *>(w + kMlpW2);
    float a2 = mlp_h2f(w[kMlpB2 + j]);
    // four 8-byte loads in flight per pass (an unrolled loop would hoist all
    // sixteen and hold 32 registers across the layer)
#pragma unroll 1
    for (int c0 = 0; c0 < 16; c0 += 4) {
        uint2 q[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            q[t] = W2[(c0 + t) * 64 + j];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float *h = scratch + 4 * (c0 + t);
            a2 = fmaf(mlp_h2f(q[t].x), h[0], a2);
            a2 = fmaf(mlp_h2f(q[t].x >> 16), h[1], a2);
            a2 = fmaf(mlp_h2f(q[t].y), h[2], a2);
            a2 = fmaf(mlp_h2f(q[t].y >> 16), h[3], a2);
        }
    }
    const float hh = fmaxf(a2, 0.0f);
    float s0 = mlp_h2f(w[kMlpW3 + j]) * hh, s1 = mlp_h2f(w[kMlpW3 + 64 + j]) * hh;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
    }
    z0 = mlp_h2f(w[kMlpB3]) + s0;
    z1 = mlp_h2f(w[kMlpB3 + 1]) + s1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace nhq
