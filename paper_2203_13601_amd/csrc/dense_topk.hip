// Dense tiles with a streaming top-K epilogue (matrix cores).
//
// For every row a of A it finds the K best columns b of B by (key, id), where
//   delta^2 = |a|^2 + |b|^2 - 2 a.b           (a.b from v_mfma_f32_16x16x4f32)
//   fusion mode:   key = delta^2 (m_a + chi)^2 (delta^2 when m_a = 0), chi and
//                  m_a over a's constrained codes (all m codes for an object)
//   filter mode:   key = delta^2, only b with chi(a's constraint, b) = 0
// Fusion mode gives the candidate lists of the composite index (Sec. 4.1 step
// (1) under the fusion distance of Sec. 5.1; b != a) and ranks the entry
// sample for each query's seed set; filter mode gives the exact hybrid k-NN
// of Def. 4.  The GEMM form of delta^2 is exact on integer-valued
// vectors; elsewhere the caller keeps a margin of extra candidates and
// re-scores them exactly.
//
// Work split: a workgroup of 4 waves owns 64 rows (16 per wave) and streams
// every column of B in tiles of 64 (4 MFMA sub-tiles of 16).  MFMA operand A
// holds 16 columns and operand B the wave's 16 rows, so in the 16x16 result
// lane l holds row l % 16 against columns 4 (l / 16) + r, r = 0..3.  Each lane
// supplies point (l % 16) at dims 16 t + 4 (l / 16) + j for k-step 4 t + j:
// both operands use the same dimension order, so the contraction covers every
// dimension once.  Survivors of the per-row threshold (the current K-th best)
// are appended to a per-row LDS buffer that is re-ranked when it fills.
#include "nhq_internal.h"

namespace nhq {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct TopkArgs {
    const float *A;       // [na][dp]
    const float *A_norm;  // [na]
    const uint32_t *A_attr;  // [na] packed codes
    const uint32_t *A_mask;  // [na] constraint masks (filter mode), null = all m bytes
    const float *B;       // [nb][dp]
    const float *B_norm;  // [nb]
    const uint32_t *B_attr;  // [nb]
    int64_t na, nb;
    int m, K, cap, mode;  // mode 0 fusion key, 1 exact-match filter
    int self_exclude;     // skip column == row (A and B are the same set)
    int32_t *out_ids;     // [na][K]
    float *out_keys;      // [na][K]
};

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int chi_of(uint32_t a, uint32_t qword, uint32_t qmask)
{
    uint32_t x = (a ^ qword) & qmask;
    uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
    return __popc(y & 0x80808080u);
}

__device__ __forceinline__ bool lt_key(float ka, uint32_t ia, float kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

constexpr int kWaves = 4;
constexpr int kRowsPerWave = 16;

// Re-rank row r's buffer: keep its `keep` best entries, sorted, in place;
// update the row's threshold when the buffer holds at least `keep` entries.
__device__ void compact_row(float *bk, uint32_t *bi, int *cnt, float *thk, uint32_t *thi, int r,
                            int cap, int keep)
{
    const int lane = threadIdx.x & 63;
    const int n = cnt[r];
    float *rk = bk + r * cap;
    uint32_t *ri = bi + r * cap;
    constexpr int MAXT = 4;  // cap <= 256
    float ke[MAXT];
    uint32_t ie[MAXT];
    int rank[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        const int e = lane + 64 * t;
        rank[t] = 0;
        ke[t] = 0.0f;
        ie[t] = 0u;
        if (e < n) {
            ke[t] = rk[e];
            ie[t] = ri[e];
        }
    }
    for (int i = 0; i < n; ++i) {
        const float ki = rk[i];
        const uint32_t ii = ri[i];
#pragma unroll
        for (int t = 0; t < MAXT; ++t)
            rank[t] += lt_key(ki, ii, ke[t], ie[t]) ? 1 : 0;
    }
    wsync();
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        const int e = lane + 64 * t;
        if (e < n && rank[t] < keep) {
            rk[rank[t]] = ke[t];
            ri[rank[t]] = ie[t];
        }
        if (e < n && rank[t] == keep - 1) {
            thk[r] = ke[t];
            thi[r] = ie[t];
        }
    }
    wsync();
    if (lane == 0)
        cnt[r] = min(n, keep);
    wsync();
}

template <int DP>
__global__ __launch_bounds__(256) void k_dense_topk(const TopkArgs a)
{
    constexpr int NT = DP / 16;             // float4 chunks per lane per point
    constexpr bool ROWS_IN_REGS = NT <= 16;  // rows stay in registers up to 256 dims
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int rl = lane & 15, lq = lane >> 4;
    const int cap = a.cap;

    extern __shared__ __align__(16) uint32_t smem[];
    float *bk = reinterpret_cast<float *>(smem) + (size_t)wave * kRowsPerWave * cap;
    uint32_t *bi = smem + (size_t)kWaves * kRowsPerWave * cap + (size_t)wave * kRowsPerWave * cap;
    uint32_t *tail = smem + (size_t)2 * kWaves * kRowsPerWave * cap + wave * 3 * kRowsPerWave;
    int *cnt = reinterpret_cast<int *>(tail);
    float *thk = reinterpret_cast<float *>(tail + kRowsPerWave);
    uint32_t *thi = tail + 2 * kRowsPerWave;

    const int64_t row0 = (int64_t)blockIdx.x * (kWaves * kRowsPerWave) + wave * kRowsPerWave;
    const int64_t row = row0 + rl;
    const bool row_ok = row < a.na;
    const int64_t rowc = row_ok ? row : a.na - 1;

    if (lane < kRowsPerWave) {
        cnt[lane] = 0;
        thk[lane] = __int_as_float(0x7F800000);
        thi[lane] = 0xFFFFFFFFu;
    }
    wsync();

    const float4 *arow = reinterpret_cast<const float4 *>(a.A + rowc * DP);
    float4 ra[ROWS_IN_REGS ? NT : 1];
    if constexpr (ROWS_IN_REGS) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
            ra[t] = arow[4 * t + lq];
    }
    const float rn = a.A_norm[rowc];
    const uint32_t rattr = a.A_attr ? a.A_attr[rowc] : 0u;
    const uint32_t full = a.m >= 4 ? 0xFFFFFFFFu : ((1u << (8 * a.m)) - 1u);
    const uint32_t rmask = a.A_mask ? a.A_mask[rowc] : full;
    const int mq = __popc(rmask) / 8;
    const float mult_base = (float)mq;

    for (int64_t c0 = 0; c0 < a.nb; c0 += 64) {
        f32x4 acc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            int64_t col = c0 + 16 * s + rl;
            if (col >= a.nb)
                col = a.nb - 1;
            const float4 *bcol = reinterpret_cast<const float4 *>(a.B + col * DP);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float4 cb = bcol[4 * t + lq];
                float4 rv;
                if constexpr (ROWS_IN_REGS)
                    rv = ra[t];
                else
                    rv = arow[4 * t + lq];
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb.x, rv.x, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb.y, rv.y, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb.z, rv.z, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb.w, rv.w, acc[s], 0, 0, 0);
            }
        }
        // epilogue: keys of this lane's 16 columns for its row
        const float tk = thk[rl];
        const uint32_t ti = thi[rl];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = c0 + 16 * s + 4 * lq + r;
                if (!row_ok || col >= a.nb)
                    continue;
                if (a.self_exclude && col == row)
                    continue;
                const int c = chi_of(a.B_attr[col], rattr, rmask);
                if (a.mode == 1 && c != 0)
                    continue;
                float d2 = rn + a.B_norm[col] - 2.0f * acc[s][r];
                d2 = fmaxf(d2, 0.0f);
                const float mult = mult_base == 0.0f ? 1.0f : (mult_base + c) * (mult_base + c);
                const float key = a.mode == 0 ? d2 * mult : d2;
                if (lt_key(key, (uint32_t)col, tk, ti)) {
                    const int slot = atomicAdd(&cnt[rl], 1);
                    bk[rl * cap + slot] = key;
                    bi[rl * cap + slot] = (uint32_t)col;
                }
            }
        }
        wsync();
        // re-rank the rows whose buffers could overflow on the next tile
        const bool full_row = lane < kRowsPerWave && cnt[lane] > cap - 64;
        uint64_t fb = __ballot(full_row);
        while (fb) {
            const int r = __ffsll((unsigned long long)fb) - 1;
            fb &= fb - 1;
            compact_row(bk, bi, cnt, thk, thi, r, cap, a.K);
        }
    }
    // final ranking of every row and output
    for (int r = 0; r < kRowsPerWave; ++r)
        compact_row(bk, bi, cnt, thk, thi, r, cap, a.K);
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int64_t orow = row0 + r;
        if (orow >= a.na)
            break;
        const int n = cnt[r];
        for (int e = lane; e < a.K; e += 64) {
            a.out_ids[orow * a.K + e] = e < n ? (int32_t)bi[r * cap + e] : -1;
            if (a.out_keys)
                a.out_keys[orow * a.K + e] = e < n ? bk[r * cap + e] : __int_as_float(0x7F800000);
        }
    }
}

template <int DP>
int launch_dp(const TopkArgs &a, hipStream_t st)
{
    const size_t lds = sizeof(uint32_t) * ((size_t)2 * kWaves * kRowsPerWave * a.cap + 3 * kWaves * kRowsPerWave);
    auto kern = k_dense_topk<DP>;
    if (lds > 64 * 1024)
        NHQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int64_t blocks = (a.na + kWaves * kRowsPerWave - 1) / (kWaves * kRowsPerWave);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kWaves), lds, st, a);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // namespace

int launch_dense_topk(const float *A, const float *A_norm, const uint32_t *A_attr,
                      const uint32_t *A_mask, int64_t na, const float *B, const float *B_norm,
                      const uint32_t *B_attr, int64_t nb, int dp, int m, int mode,
                      int self_exclude, int K, int32_t *out_ids, float *out_keys, hipStream_t st)
{
    if (K < 1 || K > 160)
        return fail(NHQ_EINVAL, "dense top-K supports 1 <= K <= 160");
    TopkArgs a{};
    a.A = A;
    a.A_norm = A_norm;
    a.A_attr = A_attr;
    a.A_mask = A_mask;
    a.B = B;
    a.B_norm = B_norm;
    a.B_attr = B_attr;
    a.na = na;
    a.nb = nb;
    a.m = m;
    a.K = K;
    a.cap = ((K + 64 + 15) / 16) * 16;
    a.mode = mode;
    a.self_exclude = self_exclude;
    a.out_ids = out_ids;
    a.out_keys = out_keys;
    if (na == 0)
        return NHQ_OK;
    switch (dp) {
    case 32:
        return launch_dp<32>(a, st);
    case 64:
        return launch_dp<64>(a, st);
    case 96:
        return launch_dp<96>(a, st);
    case 128:
        return launch_dp<128>(a, st);
    case 256:
        return launch_dp<256>(a, st);
    case 512:
        return launch_dp<512>(a, st);
    case 960:
        return launch_dp<960>(a, st);
    case 1024:
        return launch_dp<1024>(a, st);
    }
    return fail(NHQ_EINVAL, "unsupported padded dimension");
}

}  // namespace nhq
