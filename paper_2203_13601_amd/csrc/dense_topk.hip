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
// Work split: a workgroup of 2 waves owns 32 rows (16 per wave) and streams
// one range of columns of B (the grid's y dimension splits the columns when
// there are too few row blocks to fill the chip; a merge kernel then joins
// the per-range lists) in tiles of 64 (4 MFMA sub-tiles of 16).  MFMA operand A
// holds 16 columns and operand B the wave's 16 rows, so in the 16x16 result
// lane l holds row l % 16 against columns 4 (l / 16) + r, r = 0..3.  Each lane
// supplies point (l % 16) at dims 16 t + 4 (l / 16) + j for k-step 4 t + j:
// both operands use the same dimension order, so the contraction covers every
// dimension once.  Survivors of the per-row threshold (the current K-th best)
// are appended to a per-row LDS buffer of K + 64 entries, which is re-ranked
// after any 16-column sub-tile that could overflow it.  The buffers bound the
// waves per CU: 64 entries of slack measured faster than 16 (more re-ranking)
// and than 128 (fewer waves).
//
// Rows of 512 elements and more take a second form (k_dense_topk_wide): such
// a row no longer fits a wave's registers, and a wave that fetched its own
// column tiles used each column element for 16 rows only (6.4 flop per byte
// fetched, where the float32 matrix cores need about 20).  There a workgroup
// of W waves owns 16 W rows and walks its columns in tiles of 128; each tile
// goes through LDS in 32-element slices that all W waves read, and the next
// slice (the workgroup's column slice and each wave's row slice) is loaded
// while the current one is multiplied.  A column element then serves 16 W
// rows and a row element 128 columns.  Per lane the products, their order and
// the epilogue are the narrow form's, so both forms give the same keys.
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
    int abits;            // bits per attribute field
    uint32_t hmask;       // high bit of every field
    int self_exclude;     // skip column == row (A and B are the same set)
    int64_t col_span;     // columns per split (multiple of 64)
    int splits;           // gridDim.y
    int32_t *out_ids;     // [na][splits][K] (splits == 1: the final lists)
    float *out_keys;      // [na][splits][K]
    Weights w;            // weight setting of the fusion key (mode 0)
};

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}


__device__ __forceinline__ bool lt_key(float ka, uint32_t ia, float kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

constexpr int kWaves = 2;
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
    constexpr int MAXT = 5;  // cap <= 320
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
    // every lane compares its entries with all n entries; the buffer is read
    // 4 entries per LDS access (rows are 16-byte aligned, padding compares
    // as +inf) so the reads pipeline instead of chaining
    for (int i = 0; i < n; i += 4) {
        const float4 k4 = *reinterpret_cast<const float4 *>(rk + i);
        const uint4 i4 = *reinterpret_cast<const uint4 *>(ri + i);
        const float kk[4] = {k4.x, i + 1 < n ? k4.y : __int_as_float(0x7F800000),
                             i + 2 < n ? k4.z : __int_as_float(0x7F800000),
                             i + 3 < n ? k4.w : __int_as_float(0x7F800000)};
        const uint32_t ii[4] = {i4.x, i4.y, i4.z, i4.w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < MAXT; ++t)
                rank[t] += lt_key(kk[u], ii[u], ke[t], ie[t]) ? 1 : 0;
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

// Row block rb (kWaves x kRowsPerWave rows) against the workgroup's column
// range, its K best per row written out.
template <int DP>
__device__ __forceinline__ void topk_row_block(const TopkArgs &a, int64_t rb, uint32_t *smem)
{
    constexpr int NT = DP / 16;             // float4 chunks per lane per point
    constexpr bool ROWS_IN_REGS = NT <= 16;  // rows stay in registers up to 256 dims
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int rl = lane & 15, lq = lane >> 4;
    const int cap = a.cap;

    float *bk = reinterpret_cast<float *>(smem) + (size_t)wave * kRowsPerWave * cap;
    uint32_t *bi = smem + (size_t)kWaves * kRowsPerWave * cap + (size_t)wave * kRowsPerWave * cap;
    uint32_t *tail = smem + (size_t)2 * kWaves * kRowsPerWave * cap + wave * 3 * kRowsPerWave;
    int *cnt = reinterpret_cast<int *>(tail);
    float *thk = reinterpret_cast<float *>(tail + kRowsPerWave);
    uint32_t *thi = tail + 2 * kRowsPerWave;

    const int64_t row0 = rb * (kWaves * kRowsPerWave) + wave * kRowsPerWave;
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
    const uint32_t full = attr_full_mask(a.m, a.abits);
    const uint32_t rmask = a.A_mask ? a.A_mask[rowc] : full;
    const int mq = __popc(rmask) / a.abits;

    const int64_t cbeg = (int64_t)blockIdx.y * a.col_span;
    const int64_t cend = min(a.nb, cbeg + a.col_span);
    for (int64_t c0 = cbeg; c0 < cend; c0 += 64) {
        f32x4 acc[4];
        const float4 *bcol[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            int64_t col = c0 + 16 * s + rl;
            if (col >= cend)
                col = cend - 1;
            bcol[s] = reinterpret_cast<const float4 *>(a.B + col * DP);
        }
        // norms and codes of this lane's 16 columns, fetched ahead of the MFMAs
        float4 nrm[4];
        uint4 atr[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t cb0 = c0 + 16 * s + 4 * lq;
            if (cb0 + 3 < cend) {
                nrm[s] = *reinterpret_cast<const float4 *>(a.B_norm + cb0);
                atr[s] = *reinterpret_cast<const uint4 *>(a.B_attr + cb0);
            } else {
                const int64_t c1 = min(cb0 + 1, cend - 1), c2 = min(cb0 + 2, cend - 1);
                const int64_t c3 = min(cb0 + 3, cend - 1), cz = min(cb0, cend - 1);
                nrm[s] = make_float4(a.B_norm[cz], a.B_norm[c1], a.B_norm[c2], a.B_norm[c3]);
                atr[s] = make_uint4(a.B_attr[cz], a.B_attr[c1], a.B_attr[c2], a.B_attr[c3]);
            }
        }
        // four independent accumulation chains, interleaved per k-step
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float4 cb[4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                cb[s] = bcol[s][4 * t + lq];
            float4 rv;
            if constexpr (ROWS_IN_REGS)
                rv = ra[t];
            else
                rv = arow[4 * t + lq];
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
        // epilogue: keys of this lane's 16 columns for its row, one 16-column
        // sub-tile at a time (at most 16 appends per row each)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float tk = thk[rl];
            const uint32_t ti = thi[rl];
            const int64_t cb0 = c0 + 16 * s + 4 * lq;  // this lane's 4 columns
            const float nb4[4] = {nrm[s].x, nrm[s].y, nrm[s].z, nrm[s].w};
            const uint32_t at4[4] = {atr[s].x, atr[s].y, atr[s].z, atr[s].w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = cb0 + r;
                if (!row_ok || col >= cend)
                    continue;
                if (a.self_exclude && col == row)
                    continue;
                const int c = chi_of(at4[r], rattr, rmask, a.hmask);
                if (a.mode == 1 && c != 0)
                    continue;
                float d2 = rn + nb4[r] - 2.0f * acc[s][r];
                d2 = fmaxf(d2, 0.0f);
                const float key = a.mode == 0 ? w_key32(d2, c, mq, a.w) : d2;
                if (lt_key(key, (uint32_t)col, tk, ti)) {
                    const int slot = atomicAdd(&cnt[rl], 1);
                    bk[rl * cap + slot] = key;
                    bi[rl * cap + slot] = (uint32_t)col;
                }
            }
            wsync();
            // re-rank the rows whose buffers could overflow on the next sub-tile
            const bool full_row = lane < kRowsPerWave && cnt[lane] > cap - 16;
            uint64_t fb = __ballot(full_row);
            while (fb) {
                const int r = __ffsll((unsigned long long)fb) - 1;
                fb &= fb - 1;
                compact_row(bk, bi, cnt, thk, thi, r, cap, a.K);
            }
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
        const int64_t base = (orow * a.splits + blockIdx.y) * a.K;
        for (int e = lane; e < a.K; e += 64) {
            a.out_ids[base + e] = e < n ? (int32_t)bi[r * cap + e] : -1;
            if (a.out_keys)
                a.out_keys[base + e] = e < n ? bk[r * cap + e] : __int_as_float(0x7F800000);
        }
    }
    wsync();  // the buffers are read out before the next row block resets them
}

// The grid holds about as many workgroups as the device keeps resident, and
// each takes row blocks blockIdx.x, + gridDim.x, ... in turn: the workgroups
// in flight then sweep the columns side by side and share the column rows in
// L2 (a workgroup started whenever another ends would sweep from the first
// column while the others are far along, and read every column row again).
template <int DP>
__global__ __launch_bounds__(128) void k_dense_topk(const TopkArgs a)
{
    extern __shared__ __align__(16) uint32_t smem[];
    const int64_t row_blocks = (a.na + kWaves * kRowsPerWave - 1) / (kWaves * kRowsPerWave);
    for (int64_t rb = blockIdx.x; rb < row_blocks; rb += gridDim.x)
        topk_row_block<DP>(a, rb, smem);
}

constexpr int kWideCols = 128;                // columns per tile (8 sub-tiles)
constexpr int kSlice = 32;                    // elements per staged slice
constexpr int kSliceStride = kSlice + 4;      // padded LDS row: the 16 rows a read touches start in distinct banks
constexpr size_t kMaxLds = 160 * 1024;

__host__ __device__ constexpr size_t wide_lds_bytes(int waves, int cap)
{
    return sizeof(uint32_t) * ((size_t)kWideCols * kSliceStride + (size_t)2 * waves * kRowsPerWave * cap +
                               (size_t)3 * waves * kRowsPerWave);
}

// Row block rb (W x kRowsPerWave rows) against the workgroup's column range,
// the column tiles staged through LDS (rows of DP >= 512 elements).
template <int DP, int W>
__device__ __forceinline__ void topk_row_block_wide(const TopkArgs &a, int64_t rb, uint32_t *smem)
{
    static_assert(DP % kSlice == 0, "rows are padded to whole slices");
    constexpr int NS = DP / kSlice;
    constexpr int RB = W * kRowsPerWave;
    constexpr int PT = kWideCols * kSlice / 4 / (64 * W);  // staged float4 per thread per slice
    static_assert(PT * 64 * W * 4 == kWideCols * kSlice && (PT == 2 || PT == 4),
                  "slice split evenly over the threads");
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int rl = lane & 15, lq = lane >> 4;
    const int cap = a.cap;

    float *bs = reinterpret_cast<float *>(smem);  // [kWideCols][kSliceStride]
    uint32_t *surv = smem + kWideCols * kSliceStride;
    float *bk = reinterpret_cast<float *>(surv) + (size_t)wave * kRowsPerWave * cap;
    uint32_t *bi = surv + (size_t)RB * cap + (size_t)wave * kRowsPerWave * cap;
    uint32_t *tail = surv + (size_t)2 * RB * cap + wave * 3 * kRowsPerWave;
    int *cnt = reinterpret_cast<int *>(tail);
    float *thk = reinterpret_cast<float *>(tail + kRowsPerWave);
    uint32_t *thi = tail + 2 * kRowsPerWave;

    const int64_t row0 = rb * RB + wave * kRowsPerWave;
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
    const float rn = a.A_norm[rowc];
    const uint32_t rattr = a.A_attr ? a.A_attr[rowc] : 0u;
    const uint32_t full = attr_full_mask(a.m, a.abits);
    const uint32_t rmask = a.A_mask ? a.A_mask[rowc] : full;
    const int mq = __popc(rmask) / a.abits;

    const int64_t cbeg = (int64_t)blockIdx.y * a.col_span;
    const int64_t cend = min(a.nb, cbeg + a.col_span);
    for (int64_t c0 = cbeg; c0 < cend; c0 += kWideCols) {
        // this thread's share of every staged slice: float4 q of column col
        const float4 *gsrc[PT];
        int soff[PT];
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int f = threadIdx.x + i * 64 * W;
            const int col = f >> 3, q = f & 7;
            const int64_t gc = min(c0 + col, cend - 1);
            gsrc[i] = reinterpret_cast<const float4 *>(a.B + gc * DP) + q;
            soff[i] = col * kSliceStride + 4 * q;
        }
        // staged slice and row slice in flight (named registers: the
        // compiler kept an array of them in scratch)
        float4 pb0 = gsrc[0][0], pb1 = gsrc[1][0], pb2, pb3;
        if constexpr (PT == 4) {
            pb2 = gsrc[2][0];
            pb3 = gsrc[3][0];
        }
        float4 pa0 = arow[lq], pa1 = arow[4 + lq];
        f32x4 acc[8];
#pragma unroll
        for (int s = 0; s < 8; ++s)
            acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
        for (int ks = 0; ks < NS; ++ks) {
            __syncthreads();  // every wave is done with the previous slice
            *reinterpret_cast<float4 *>(bs + soff[0]) = pb0;
            *reinterpret_cast<float4 *>(bs + soff[1]) = pb1;
            if constexpr (PT == 4) {
                *reinterpret_cast<float4 *>(bs + soff[2]) = pb2;
                *reinterpret_cast<float4 *>(bs + soff[3]) = pb3;
            }
            __syncthreads();
            const float4 ra0 = pa0, ra1 = pa1;
            // the next slice's loads (the last slice loads itself again)
            const int kn = ks + 1 < NS ? ks + 1 : ks;
            pb0 = gsrc[0][8 * kn];
            pb1 = gsrc[1][8 * kn];
            if constexpr (PT == 4) {
                pb2 = gsrc[2][8 * kn];
                pb3 = gsrc[3][8 * kn];
            }
            pa0 = arow[8 * kn + lq];
            pa1 = arow[8 * kn + 4 + lq];
            // keep these loads ahead of the products (the scheduler would
            // otherwise sink them below, next to their use)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                float4 cb[8];
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    cb[s] = *reinterpret_cast<const float4 *>(bs + (16 * s + rl) * kSliceStride + 16 * tt + 4 * lq);
                const float4 rv = tt == 0 ? ra0 : ra1;
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].x, rv.x, acc[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].y, rv.y, acc[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].z, rv.z, acc[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[s].w, rv.w, acc[s], 0, 0, 0);
            }
        }
        // epilogue, as in the narrow form: one 16-column sub-tile at a time,
        // with the norms and codes of this lane's 4 columns in it
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t cb0 = c0 + 16 * s + 4 * lq;
            float4 nrm;
            uint4 atr;
            if (cb0 + 3 < cend) {
                nrm = *reinterpret_cast<const float4 *>(a.B_norm + cb0);
                atr = *reinterpret_cast<const uint4 *>(a.B_attr + cb0);
            } else {
                const int64_t c1 = min(cb0 + 1, cend - 1), c2 = min(cb0 + 2, cend - 1);
                const int64_t c3 = min(cb0 + 3, cend - 1), cz = min(cb0, cend - 1);
                nrm = make_float4(a.B_norm[cz], a.B_norm[c1], a.B_norm[c2], a.B_norm[c3]);
                atr = make_uint4(a.B_attr[cz], a.B_attr[c1], a.B_attr[c2], a.B_attr[c3]);
            }
            const float tk = thk[rl];
            const uint32_t ti = thi[rl];
            const float nb4[4] = {nrm.x, nrm.y, nrm.z, nrm.w};
            const uint32_t at4[4] = {atr.x, atr.y, atr.z, atr.w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = cb0 + r;
                if (!row_ok || col >= cend)
                    continue;
                if (a.self_exclude && col == row)
                    continue;
                const int c = chi_of(at4[r], rattr, rmask, a.hmask);
                if (a.mode == 1 && c != 0)
                    continue;
                float d2 = rn + nb4[r] - 2.0f * acc[s][r];
                d2 = fmaxf(d2, 0.0f);
                const float key = a.mode == 0 ? w_key32(d2, c, mq, a.w) : d2;
                if (lt_key(key, (uint32_t)col, tk, ti)) {
                    const int slot = atomicAdd(&cnt[rl], 1);
                    bk[rl * cap + slot] = key;
                    bi[rl * cap + slot] = (uint32_t)col;
                }
            }
            wsync();
            const bool full_row = lane < kRowsPerWave && cnt[lane] > cap - 16;
            uint64_t fb = __ballot(full_row);
            while (fb) {
                const int r = __ffsll((unsigned long long)fb) - 1;
                fb &= fb - 1;
                compact_row(bk, bi, cnt, thk, thi, r, cap, a.K);
            }
        }
    }
    for (int r = 0; r < kRowsPerWave; ++r)
        compact_row(bk, bi, cnt, thk, thi, r, cap, a.K);
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int64_t orow = row0 + r;
        if (orow >= a.na)
            break;
        const int n = cnt[r];
        const int64_t base = (orow * a.splits + blockIdx.y) * a.K;
        for (int e = lane; e < a.K; e += 64) {
            a.out_ids[base + e] = e < n ? (int32_t)bi[r * cap + e] : -1;
            if (a.out_keys)
                a.out_keys[base + e] = e < n ? bk[r * cap + e] : __int_as_float(0x7F800000);
        }
    }
    wsync();  // the buffers are read out before the next row block resets them
}

// The wide form's grid: the resident workgroups, each looping over row blocks
// as in the narrow form.  Every wave of a workgroup runs the same tiles and
// slices (rows past the end included), so the workgroup barriers match.
template <int DP, int W>
__global__ __launch_bounds__(64 * W) void k_dense_topk_wide(const TopkArgs a)
{
    extern __shared__ __align__(16) uint32_t smem[];
    const int64_t row_blocks = (a.na + W * kRowsPerWave - 1) / (W * kRowsPerWave);
    for (int64_t rb = blockIdx.x; rb < row_blocks; rb += gridDim.x)
        topk_row_block_wide<DP, W>(a, rb, smem);
}

// join the per-range sorted lists of one row: K steps of a k-way merge, the
// head of list s held by lane s (splits <= 64)
__global__ __launch_bounds__(64) void k_merge_lists(const int32_t *__restrict__ pid,
                                                    const float *__restrict__ pkey, int64_t na,
                                                    int splits, int K, int32_t *__restrict__ out_ids,
                                                    float *__restrict__ out_keys)
{
    const int lane = threadIdx.x;
    const int64_t r = blockIdx.x;
    if (r >= na)
        return;
    const int64_t base = r * splits * K;
    int head = 0;
    for (int e = 0; e < K; ++e) {
        float hk = __int_as_float(0x7F800000);
        uint32_t hi = 0xFFFFFFFFu;
        if (lane < splits && head < K) {
            const int32_t v = pid[base + lane * K + head];
            if (v >= 0) {
                hk = pkey[base + lane * K + head];
                hi = (uint32_t)v;
            }
        }
        float bk = hk;
        uint32_t bi = hi;
        for (int o = 32; o > 0; o >>= 1) {
            const float ok = __shfl_xor(bk, o, 64);
            const uint32_t oi = (uint32_t)__shfl_xor((int)bi, o, 64);
            if (lt_key(ok, oi, bk, bi)) {
                bk = ok;
                bi = oi;
            }
        }
        if (lane < splits && hi == bi && hi != 0xFFFFFFFFu)
            head += 1;
        if (lane == 0) {
            out_ids[r * K + e] = bi == 0xFFFFFFFFu ? -1 : (int32_t)bi;
            if (out_keys)
                out_keys[r * K + e] = bk;
        }
    }
}

template <int DP, int W>
int launch_wide(const TopkArgs &a, hipStream_t st)
{
    const size_t lds = wide_lds_bytes(W, a.cap);
    if (lds > kMaxLds)
        return fail(NHQ_EINVAL, "dense top-K: survivor buffers exceed the LDS");
    auto kern = k_dense_topk_wide<DP, W>;
    if (lds > 64 * 1024)
        NHQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int64_t row_blocks = (a.na + W * kRowsPerWave - 1) / (W * kRowsPerWave);
    int dev = 0, n_cu = 0, per_cu = 0;
    NHQ_HIP(hipGetDevice(&dev));
    NHQ_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    NHQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern),
                                                         64 * W, lds));
    const int64_t resident = std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * n_cu / a.splits);
    const int64_t blocks = std::min(row_blocks, resident);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks, (unsigned)a.splits), dim3(64 * W), lds, st, a);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

template <int DP>
int launch_dp(const TopkArgs &a, int waves, hipStream_t st)
{
    if constexpr (DP >= 512) {
        if (waves == 8)
            return launch_wide<DP, 8>(a, st);
        if (waves == 4)
            return launch_wide<DP, 4>(a, st);
        return fail(NHQ_EINVAL, "dense top-K: unsupported workgroup size");
    }
    (void)waves;
    const size_t lds = sizeof(uint32_t) * ((size_t)2 * kWaves * kRowsPerWave * a.cap + 3 * kWaves * kRowsPerWave);
    auto kern = k_dense_topk<DP>;
    if (lds > 64 * 1024)
        NHQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    // as many workgroups as stay resident (the kernel loops over row blocks)
    const int64_t row_blocks = (a.na + kWaves * kRowsPerWave - 1) / (kWaves * kRowsPerWave);
    int dev = 0, n_cu = 0, per_cu = 0;
    NHQ_HIP(hipGetDevice(&dev));
    NHQ_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    NHQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern),
                                                         64 * kWaves, lds));
    const int64_t resident = std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * n_cu / a.splits);
    const int64_t blocks = std::min(row_blocks, resident);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks, (unsigned)a.splits), dim3(64 * kWaves), lds, st, a);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // namespace

int launch_dense_topk(const float *A, const float *A_norm, const uint32_t *A_attr,
                      const uint32_t *A_mask, int64_t na, const float *B, const float *B_norm,
                      const uint32_t *B_attr, int64_t nb, int dp, int m, int abits, int mode,
                      int self_exclude, int K, int32_t *out_ids, float *out_keys, hipStream_t st,
                      const Weights *w)
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
    // slack above the kept K: at least one 16-column sub-tile (16 appends
    // per row); a row is re-ranked once fewer than 16 free entries remain.
    // The wide form takes 8 waves with 64, 48 or 32 entries of slack, the
    // first that fits the LDS beside the staged slice, else 4 waves with 64.
    const bool wide = dp >= 512;
    int waves = kWaves;
    a.cap = ((K + 64 + 15) / 16) * 16;
    if (wide) {
        waves = 4;
        for (int slack = 64; slack >= 32; slack -= 16) {
            const int c = ((K + slack + 15) / 16) * 16;
            if (wide_lds_bytes(8, c) <= kMaxLds) {
                waves = 8;
                a.cap = c;
                break;
            }
        }
    }
    const int rows_per_block = waves * kRowsPerWave;
    a.mode = mode;
    a.abits = abits;
    a.hmask = attr_hmask(abits);
    a.w = w ? *w : Weights{NHQ_WEIGHTS_DEFAULT, 0.0f, 0.0};
    a.self_exclude = self_exclude;
    if (na == 0 || nb == 0)
        return NHQ_OK;
    // split the columns until there are row blocks for about 4096 waves,
    // keeping at least 512 columns per split
    const int64_t row_blocks = (na + rows_per_block - 1) / rows_per_block;
    const int64_t want_blocks = 2048 * kWaves / waves;
    int splits = 1;
    while (splits < 64 && row_blocks * splits < want_blocks && nb / (2 * splits) >= 512)
        splits *= 2;
    a.splits = splits;
    a.col_span = ((nb + splits - 1) / splits + 63) / 64 * 64;
    int32_t *pid = out_ids;
    float *pkey = out_keys;
    if (splits > 1) {
        NHQ_HIP(hipMallocAsync((void **)&pid, sizeof(int32_t) * (size_t)na * splits * K, st));
        NHQ_HIP(hipMallocAsync((void **)&pkey, sizeof(float) * (size_t)na * splits * K, st));
    }
    a.out_ids = pid;
    a.out_keys = pkey;
    int rc = NHQ_OK;
    switch (dp) {
    case 32: rc = launch_dp<32>(a, waves, st); break;
    case 64: rc = launch_dp<64>(a, waves, st); break;
    case 96: rc = launch_dp<96>(a, waves, st); break;
    case 128: rc = launch_dp<128>(a, waves, st); break;
    case 256: rc = launch_dp<256>(a, waves, st); break;
    case 512: rc = launch_dp<512>(a, waves, st); break;
    case 960: rc = launch_dp<960>(a, waves, st); break;
    case 1024: rc = launch_dp<1024>(a, waves, st); break;
    default: rc = fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    if (splits > 1) {
        if (rc == NHQ_OK) {
            hipLaunchKernelGGL(k_merge_lists, dim3((unsigned)na), dim3(64), 0, st, pid, pkey, na, splits,
                               K, out_ids, out_keys);
            if (hipGetLastError() != hipSuccess)
                rc = fail(NHQ_EHIP, "merge launch failed");
        }
        (void)hipFreeAsync(pid, st);
        (void)hipFreeAsync(pkey, st);
    }
    return rc;
}

}  // namespace nhq
