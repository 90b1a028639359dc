// Seed ranking: every query against the index's random entry sample (the
// seed set B of Alg. 2 is drawn from it), in two kernels.
//
// k_entry_keys (matrix cores): the full key matrix [nq][n_entry_pad] with
//   key = delta^2 (m_q + chi)^2 (delta^2 when m_q = 0),
//   delta^2 = |q|^2 + |e|^2 - 2 q.e   (q.e from v_mfma_f32_16x16x4f32),
// chi over the query's constrained codes; padding columns hold +inf.  A
// workgroup of 4 waves takes 64 queries (16 per wave) against 256 entries.
//
// k_entry_select: one wave per query keeps its row of keys in registers
// (n_entry_pad / 64 per lane), finds the n_cand-th smallest key by a bitwise
// radix select on the float bit patterns (keys are non-negative, so their
// bit patterns order like the values), and writes the positions of the
// n_cand best by (key, position) -- unordered; the search re-scores them.
#include "nhq_internal.h"

namespace nhq {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int chi_of(uint32_t a, uint32_t qword, uint32_t qmask)
{
    uint32_t x = (a ^ qword) & qmask;
    uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
    return __popc(y & 0x80808080u);
}

struct KeyArgs {
    const float *qpad;    // [nq][DP]
    const float *qnorm;   // [nq]
    const uint32_t *qword, *qmask;  // [nq]
    const float *ev;      // [ne][DP]
    const float *en;      // [ne]
    const uint32_t *ea;   // [ne]
    float *keys;          // [nq][ne_pad]
    int64_t nq;
    int ne, ne_pad;
};

template <int DP>
__global__ __launch_bounds__(256) void k_entry_keys(const KeyArgs a)
{
    constexpr int NT = DP / 16;
    constexpr bool ROWS_IN_REGS = NT <= 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rl = lane & 15, lq = lane >> 4;
    const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + rl;
    const bool row_ok = row < a.nq;
    const int64_t rowc = row_ok ? row : a.nq - 1;
    const float4 *qrow = reinterpret_cast<const float4 *>(a.qpad + rowc * DP);
    float4 ra[ROWS_IN_REGS ? NT : 1];
    if constexpr (ROWS_IN_REGS) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
            ra[t] = qrow[4 * t + lq];
    }
    const float rn = a.qnorm[rowc];
    const uint32_t qw = a.qword[rowc], qm = a.qmask[rowc];
    const float mq = (float)(__popc(qm) / 8);
    const int cbeg = blockIdx.y * 256;
    for (int c0 = cbeg; c0 < cbeg + 256 && c0 < a.ne_pad; c0 += 64) {
        f32x4 acc[4];
        const float4 *ecol[4];
        float4 nrm[4];
        uint4 atr[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const int col = min(c0 + 16 * s + rl, a.ne - 1);
            ecol[s] = reinterpret_cast<const float4 *>(a.ev + (int64_t)col * DP);
            const int cb0 = c0 + 16 * s + 4 * lq;
            if (cb0 + 3 < a.ne) {
                nrm[s] = *reinterpret_cast<const float4 *>(a.en + cb0);
                atr[s] = *reinterpret_cast<const uint4 *>(a.ea + cb0);
            } else {
                const int c1 = min(cb0 + 1, a.ne - 1), c2 = min(cb0 + 2, a.ne - 1);
                const int c3 = min(cb0 + 3, a.ne - 1), cz = min(cb0, a.ne - 1);
                nrm[s] = make_float4(a.en[cz], a.en[c1], a.en[c2], a.en[c3]);
                atr[s] = make_uint4(a.ea[cz], a.ea[c1], a.ea[c2], a.ea[c3]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float4 cb[4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                cb[s] = ecol[s][4 * t + lq];
            float4 rv;
            if constexpr (ROWS_IN_REGS)
                rv = ra[t];
            else
                rv = qrow[4 * t + lq];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].x, rv.x, acc[s], 0, 0, 0);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].y, rv.y, acc[s], 0, 0, 0);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].z, rv.z, acc[s], 0, 0, 0);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].w, rv.w, acc[s], 0, 0, 0);
        }
        if (!row_ok)
            continue;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int cb0 = c0 + 16 * s + 4 * lq;
            const float nb4[4] = {nrm[s].x, nrm[s].y, nrm[s].z, nrm[s].w};
            const uint32_t at4[4] = {atr[s].x, atr[s].y, atr[s].z, atr[s].w};
            float k4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float d2 = fmaxf(rn + nb4[r] - 2.0f * acc[s][r], 0.0f);
                const int c = chi_of(at4[r], qw, qm);
                const float mult = mq == 0.0f ? 1.0f : (mq + c) * (mq + c);
                k4[r] = cb0 + r < a.ne ? d2 * mult : __int_as_float(0x7F800000);
            }
            *reinterpret_cast<float4 *>(a.keys + row * a.ne_pad + cb0) = make_float4(k4[0], k4[1], k4[2], k4[3]);
        }
    }
}

// sum over the wave
__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

template <int NJ>
__global__ __launch_bounds__(64) void k_entry_select(const float *__restrict__ keys, int64_t nq,
                                                     int ne, int ne_pad, int K, int32_t *__restrict__ cand)
{
    const int lane = threadIdx.x;
    const int64_t qi = blockIdx.x;
    if (qi >= nq)
        return;
    const float *row = keys + qi * ne_pad;
    uint32_t v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        v[j] = 64 * j + lane < ne ? __float_as_uint(row[64 * j + lane]) : 0xFFFFFFFFu;
    // the K-th smallest bit pattern, one bit at a time from the top
    uint32_t p = 0;
    int want = K;
    for (int b = 31; b >= 0; --b) {
        const uint32_t hi = b == 31 ? 0x80000000u : ~((1u << b) - 1u);
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            cnt += (v[j] & hi) == p ? 1 : 0;
        cnt = wave_sum(cnt);
        if (cnt < want) {
            want -= cnt;
            p |= 1u << b;
        }
    }
    // p is the K-th smallest pattern: take every smaller one, then the
    // `want` equal ones with the smallest positions (position = 64 j + lane)
    int base = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const bool lt = v[j] < p;
        const uint64_t b = __ballot(lt);
        if (lt)
            cand[qi * K + base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = 64 * j + lane;
        base += __popcll(b);
    }
    int left = K - base;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const bool eq = v[j] == p && left > 0;
        const uint64_t b = __ballot(eq);
        const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
        if (eq && r < left)  // padding (only when K > n_entry) becomes -1
            cand[qi * K + base + r] = 64 * j + lane < ne ? 64 * j + lane : -1;
        const int took = min(left, __popcll(b));
        base += took;
        left -= took;
    }
}

}  // namespace

// positions of the n_cand best entry-sample members per query (unordered)
int launch_seed_rank(const Index *ix, const float *qpad, const float *qnorm, const uint32_t *qword,
                     const uint32_t *qmask, int64_t nq, int K, int32_t *cand, hipStream_t st)
{
    const int ne = ix->n_entry;
    const int ne_pad = (ne + 63) / 64 * 64;
    const int nj = ne_pad / 64;
    if (nj > 128)
        return fail(NHQ_EINVAL, "entry sample larger than 8192");
    float *keys = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&keys, sizeof(float) * (size_t)nq * ne_pad, st));
    KeyArgs a{qpad, qnorm, qword, qmask, ix->entry_vec, ix->entry_norm, ix->entry_attr, keys, nq, ne, ne_pad};
    const dim3 grid((unsigned)((nq + 63) / 64), (unsigned)((ne_pad + 255) / 256));
    int rc = NHQ_OK;
    switch (ix->dp) {
#define NHQ_K(DPV)                                                                 \
    case DPV:                                                                      \
        hipLaunchKernelGGL(k_entry_keys<DPV>, grid, dim3(256), 0, st, a);          \
        break;
        NHQ_K(32)
        NHQ_K(64)
        NHQ_K(96)
        NHQ_K(128)
        NHQ_K(256)
        NHQ_K(512)
        NHQ_K(960)
        NHQ_K(1024)
#undef NHQ_K
    default:
        rc = fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    if (rc == NHQ_OK && hipGetLastError() != hipSuccess)
        rc = fail(NHQ_EHIP, "entry key launch failed");
    if (rc == NHQ_OK) {
        const dim3 g2((unsigned)nq);
        if (nj <= 16)
            hipLaunchKernelGGL(k_entry_select<16>, g2, dim3(64), 0, st, keys, nq, ne, ne_pad, K, cand);
        else if (nj <= 32)
            hipLaunchKernelGGL(k_entry_select<32>, g2, dim3(64), 0, st, keys, nq, ne, ne_pad, K, cand);
        else if (nj <= 64)
            hipLaunchKernelGGL(k_entry_select<64>, g2, dim3(64), 0, st, keys, nq, ne, ne_pad, K, cand);
        else
            hipLaunchKernelGGL(k_entry_select<128>, g2, dim3(64), 0, st, keys, nq, ne, ne_pad, K, cand);
        if (hipGetLastError() != hipSuccess)
            rc = fail(NHQ_EHIP, "entry select launch failed");
    }
    (void)hipFreeAsync(keys, st);
    return rc;
}

}  // namespace nhq
