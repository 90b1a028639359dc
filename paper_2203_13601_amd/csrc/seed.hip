// Seed ranking: every query against the index's random entry sample (the
// seed set B of Alg. 2 is drawn from it): a key kernel, then a selection.
//
// k_entry_keys_x3 (matrix cores): the full key matrix [nq][n_entry_pad] with
//   key = delta^2 (m_q + chi)^2 (delta^2 when m_q = 0),
//   delta^2 = |q|^2 + |e|^2 - 2 q.e,
// chi over the query's constrained codes; padding columns hold +inf.  q.e
// comes from the bf16 matrix cores (v_mfma_f32_16x16x32_bf16) on split
// rows: every float32 value v as hi = bf16(v) plus lo = bf16(v - hi), and
// q.e as hi.hi' + hi.lo' + lo.hi' accumulated in float32 -- the split-bf16
// product of Henry, Tang and Heinecke (ARITH 2019), about 2^-17 relative
// error per term against 2^-24 for float32.  The ranking only prefilters:
// the search re-scores its candidates exactly in float32 and keeps the
// n_init best, and the candidates carry a margin of 8 beyond n_init, so an
// error of this size changes which entries seed a search only when keys
// tie to within it.  Values exact in bf16 have lo = 0, and integer rows of
// at most 128 elements keep every partial sum exact (k_entry_keys_b16 takes
// those workgroups with one product per chunk).  A workgroup of 4 waves
// takes 64 or 128 queries (one or two sets of 16 per wave) against TL tiles
// of 64 entries, on a grid remapped so that a query group's tiles share one
// XCD's L2; a tile's split entry rows are staged in LDS a pass of 64 (or
// 32, or the whole row up to 128) elements at a time, the next pass's loads
// in flight during the current pass's products, and the weight setting is a
// template argument chosen once per launch.
//
// The key kernels also write, per query, the minimum of every 16-entry group
// of keys.  The K-th smallest group minimum bounds the K-th smallest key
// from above (K groups each hold a key at or below it), and every key at or
// below the bound lies in a group whose minimum is at or below it.
//
// k_entry_select_g (K <= 64): one wave per query ranks the group minima,
// reads only the keys of the groups at or below the bound (on clustered
// data about K groups: 1/8 of the row at n_entry = 4096), keeps the keys at
// or below it in position order and selects the K best among them.  Should
// the bound admit too many keys, it selects over the whole row instead.
//
// k_entry_select (K > 64): one wave per query keeps its row of keys in
// registers (n_entry_pad / 64 per lane), finds the K-th smallest key by a
// bitwise radix select on the float bit patterns (keys are non-negative, so
// their bit patterns order like the values).
//
// Both write the positions of the K best by (key, position) -- unordered;
// the search re-scores them.
#include "nhq_internal.h"
#include "wave_select.h"

namespace nhq {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


// 64-entry tiles per key workgroup, TL: up to 8 where the grid already has
// enough workgroups (the exact bf16 kernel at d = 128 with 4,096 entries: 8
// beats 1, 2, 4 and 16); fewer for small grids (wide rows with a small entry
// sample), where more workgroups in flight hide the staging latency of each
// tile
constexpr int kMaxKeyTiles = 8;
// a wave's group minima of its chunk, 16 rows in LDS (padded row stride)
template <int TL>
struct GmStride {
    static constexpr int v = 4 * TL + 1;
};

struct KeyArgs {
    const float *qpad;    // [nq][DP] (read by the exact bf16 kernel only)
    const uint16_t *qs;   // [nq][2 DP] split query rows (see the top)
    const float *qnorm;   // [nq]
    const uint32_t *qword, *qmask;  // [nq]
    const uint16_t *es;   // [ne][2 DP] split entry rows
    const float *en;      // [ne]
    const uint32_t *ea;   // [ne]
    const uint16_t *eb;   // [ne][DP] exact bf16 copy of ev, or null
    const uint32_t *qx;   // [nq] query rows exact in bf16 (nullable)
    float *keys;          // [nq][ne_pad]
    float *gmin;          // [nq][ne_pad / 16] minimum of each 16-entry group
    int64_t nq;
    int ne, ne_pad;
    Weights w;            // weight setting of Gamma
    int abits;            // attribute field width
    uint32_t hmask;       // high bit of every attribute field
    // stratified sample (seg non-null): workgroup x ranks its 64 query rows
    // against entry block seg[x] (n_blocks: the n_global global members;
    // < 0: no rows), whose members are entries block_off[b] ..
    // block_off[b + 1] - 1
    const int32_t *seg = nullptr;
    const int32_t *block_off = nullptr;
    int n_blocks = 0, n_global = 0;
    // nullable [nq]: rows with live[row] < 0 hold no query (a stratified
    // block's padding slots); their keys and group minima are not written
    const int32_t *live = nullptr;
};

// Bit r: row row0 + r of a wave's 16 rows holds a query (and is below nq).
__device__ __forceinline__ uint32_t live_rows16(const KeyArgs &a, int64_t row0)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = row0 + (lane & 15);
    const bool on = row < a.nq && (!a.live || a.live[row] >= 0);
    return (uint32_t)(__ballot(on && lane < 16) & 0xFFFFull);
}

// the wave's group minima (16 rows, ng groups from group gbeg) to HBM, each
// row's run of groups contiguous
template <int TL>
__device__ __forceinline__ void flush_gmin(const KeyArgs &a, const float *gm, int64_t row0, int gbeg, int ng,
                                           uint32_t live16)
{
    constexpr int kGmStride = GmStride<TL>::v;
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < 16 * ng; i += 64) {
        const int r = i / ng, g = i - r * ng;
        const int64_t row = row0 + r;
        if ((live16 >> r) & 1u)
            a.gmin[row * (a.ne_pad / 16) + gbeg + g] = gm[r * kGmStride + g];
    }
}

// The norm and attribute word of the tile's 64 entries (columns past the
// sample's end repeat its last entry; their keys become +inf): loaded by
// the first wave together with the tile's rows, written to LDS after them.
struct EntryMeta {
    float n;
    uint32_t w;
};
__device__ __forceinline__ EntryMeta load_entry_meta(const KeyArgs &a, int c0)
{
    EntryMeta m{0.0f, 0u};
    if (threadIdx.x < 64) {
        const int col = min(c0 + (int)threadIdx.x, a.ne - 1);
        m.n = a.en[col];
        m.w = a.ea[col];
    }
    return m;
}
__device__ __forceinline__ void put_entry_meta(const EntryMeta &m, float *ten, uint32_t *tea)
{
    if (threadIdx.x < 64) {
        ten[threadIdx.x] = m.n;
        tea[threadIdx.x] = m.w;
    }
}

// Passes over a split row: KC elements per pass (the whole row up to 128
// wide, else 64, or 32 where 64 does not divide DP: wider passes need more
// registers than three waves per SIMD leave), NCK 32-element chunks per
// pass, NP passes (with one pass, a wave loads its query chunks once for
// every tile); an entry row's
// pass sits in LDS at a stride of ROW bf16 halves (hi and lo of its NCK
// chunks, 16 bytes of padding against bank conflicts).  The staged values
// are native vectors (u32x4): held across the pass loop, HIP's uint4 class
// is not kept in registers.
template <int DP>
struct XShape {
    static constexpr int KC = DP <= 128 ? DP : DP % 64 == 0 ? 64 : 32;
    static constexpr int NCK = KC / 32;
    static constexpr int NP = DP / KC;
    static constexpr int ROW = 2 * KC + 8;
    static constexpr int NV = 64 * (KC / 4) / 256;  // 16-byte staging loads per thread per pass
    static_assert(DP % KC == 0 && KC % 32 == 0 && NV * 256 == 64 * (KC / 4), "whole passes and loads");
};

// a lane's value from another lane of its quad (DPP quad_perm)
template <int CTRL>
__device__ __forceinline__ float quad_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// The ordering key of one pair.  DEF (the default weights, chosen once per
// launch): delta^2 (m_q + chi)^2, with m1 = max(m_q, 1) -- a query with no
// constrained attribute has chi = 0, so its factor is 1 and the key is
// delta^2, as the definition asks; the factor is an integer below 2^24, so
// it is exact in float32 and the key is rounded once, as in w_key32.
template <bool DEF>
__device__ __forceinline__ float pair_key(float d2, int c, int mq, float m1, const Weights &w)
{
    if constexpr (DEF) {
        const float f = m1 + (float)c;
        return d2 * (f * f);
    } else {
        return w_key32(d2, c, mq, w);
    }
}

// Keys of one 64-entry tile for a wave's 16 queries: lane (rl, lq) holds
// query rl against entries c0 + 16 s + 4 lq + r in acc[s][r]; the tile's
// entry norms and attribute words are in LDS (ten, tea).  The keys go
// through the wave's LDS area (16 rows of 68 floats) so that every store
// instruction writes four whole 256-byte rows of the key matrix.
template <bool DEF, int TL>
__device__ __forceinline__ void store_keys(const KeyArgs &a, const f32x4 (&acc)[4], int c0, int64_t row0, int rl,
                                           int lq, float rn, uint32_t qw, uint32_t qm, float mq, const float *ten,
                                           const uint32_t *tea, float *stage, float *gm, int g0,
                                           uint32_t live16)
{
    constexpr int kGmStride = GmStride<TL>::v;
    const int lane = threadIdx.x & 63;
    const float m1 = fmaxf(mq, 1.0f);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int cb0 = c0 + 16 * s + 4 * lq;
        const float4 nrm = *reinterpret_cast<const float4 *>(ten + 16 * s + 4 * lq);
        const uint4 atr = *reinterpret_cast<const uint4 *>(tea + 16 * s + 4 * lq);
        const float nb4[4] = {nrm.x, nrm.y, nrm.z, nrm.w};
        const uint32_t at4[4] = {atr.x, atr.y, atr.z, atr.w};
        float k4[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float d2 = fmaxf(rn + nb4[r] - 2.0f * acc[s][r], 0.0f);
            const int c = chi_of(at4[r], qw, qm, a.hmask);
            k4[r] = cb0 + r < a.ne ? pair_key<DEF>(d2, c, (int)mq, m1, a.w) : __int_as_float(0x7F800000);
        }
        *reinterpret_cast<float4 *>(stage + rl * 68 + 16 * s + 4 * lq) = make_float4(k4[0], k4[1], k4[2], k4[3]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int idx = 64 * u + lane, r = idx >> 4, c4 = idx & 15;
        const int64_t row = row0 + r;
        const float4 x = *reinterpret_cast<const float4 *>(stage + r * 68 + 4 * c4);
        // group minimum over the quad of lanes holding columns 16 (c4 / 4) ..
        float mn = fminf(fminf(x.x, x.y), fminf(x.z, x.w));
        mn = fminf(mn, quad_mov<0xB1>(mn));  // quad_perm(1, 0, 3, 2)
        mn = fminf(mn, quad_mov<0x4E>(mn));  // quad_perm(2, 3, 0, 1)
        if ((live16 >> r) & 1u)
            *reinterpret_cast<float4 *>(a.keys + row * a.ne_pad + c0 + 4 * c4) = x;
        if ((lane & 3) == 0)
            gm[r * kGmStride + g0 + (c4 >> 2)] = mn;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Whether the workgroup's 64 queries are all exact in bf16 and the index
// holds the exact bf16 entry copy (the bf16 kernel's share of the work).
template <int DP>
__device__ __forceinline__ bool group_exact(const KeyArgs &a, int64_t rowc)
{
    if (!(DP <= 128 && DP % 32 == 0) || a.eb == nullptr || a.qx == nullptr)
        return false;
    return __syncthreads_and(a.qx[rowc] != 0u) != 0;
}

// Workgroups go to the 8 XCDs (each with its own L2) round-robin in
// dispatch order.  The logical workgroup: XCD x takes the x-th contiguous
// run of (query group, column tile) pairs, column tile fastest, so the
// tiles of one query group (and the stratified block its neighbours share)
// meet in one L2.  A bijection of 0 .. total - 1.
__device__ __forceinline__ int xcd_logical(int flat, int total)
{
    constexpr int kXcd = 8;
    const int x = flat % kXcd, pos = flat / kXcd;
    return x * (total / kXcd) + min(x, total % kXcd) + pos;
}

// One pass's loads: this thread's share of the 64 split entry rows from
// column c0 (columns past the sample's end repeat its last entry), and the
// lane's query chunks of the pass for each of its QS query rows (16-byte
// units of a split row: chunk t's hi halves 8 lq .. 8 lq + 7 at 8 t + lq,
// its lo halves at 8 t + 4 + lq).
template <int DP, int QS, bool LOADQ>
__device__ __forceinline__ void x3_load(const u32x4 *es4, const u32x4 *const (&qrow)[QS], int c0, int kc, int ne,
                                        int lq, u32x4 (&v)[XShape<DP>::NV], u32x4 (&q)[QS][XShape<DP>::NCK][2])
{
    using X = XShape<DP>;
#pragma unroll
    for (int it = 0; it < X::NV; ++it) {
        const int i = (int)threadIdx.x + 256 * it, r = i / (X::KC / 4), c4 = i - r * (X::KC / 4);
        const int col = min(c0 + r, ne - 1);
        v[it] = es4[(int64_t)col * (DP / 4) + kc * (X::KC / 4) + c4];
    }
    if constexpr (LOADQ) {
#pragma unroll
        for (int h = 0; h < QS; ++h)
#pragma unroll
            for (int j = 0; j < X::NCK; ++j) {
                q[h][j][0] = qrow[h][8 * (kc * X::NCK + j) + lq];
                q[h][j][1] = qrow[h][8 * (kc * X::NCK + j) + 4 + lq];
            }
    }
}

// A workgroup of 4 waves: 64 QS queries (QS sets of 16 per wave) against
// TL tiles of 64 entries, split-bf16 products (see the top); every entry
// fragment read from LDS feeds the products of all QS sets.  Each pass
// writes its staged entry rows to LDS, issues the next pass's loads (the
// next tile's first after a tile's last pass), then runs its products.
// QS = 1 where workgroups may be left to k_entry_keys_b16 (all 64 queries
// exact in bf16) or rank against a stratified block (one per 64 rows).
template <int DP, bool DEF, int TL, int QS>
__global__ __launch_bounds__(256) void k_entry_keys_x3(const KeyArgs a0)
{
    using X = XShape<DP>;
    constexpr int kGmStride = GmStride<TL>::v;
    // a one-dimensional grid of query groups x column tiles: XCD-grouped
    // (see xcd_logical) where every group ranks against the whole sample;
    // query group fastest in dispatch order for a stratified sample, whose
    // groups read disjoint column tiles of a block but share each tile with
    // the block's other groups
    const int nct = (a0.ne_pad / 64 + TL - 1) / TL;
    int qgroup, ctile;
    if (a0.seg) {
        const int groups = (int)gridDim.x / nct;
        ctile = (int)blockIdx.x / groups;
        qgroup = (int)blockIdx.x - ctile * groups;
    } else {
        const int logical = xcd_logical((int)blockIdx.x, (int)gridDim.x);
        qgroup = logical / nct;
        ctile = logical - qgroup * nct;
    }
    KeyArgs a = a0;
    if constexpr (QS == 1) {
        if (a0.seg) {  // stratified: this workgroup's entry block (uniform per workgroup)
            const int b = a0.seg[qgroup];
            if (b < 0)
                return;
            int e0 = 0, cnt = a0.n_global;
            if (b < a0.n_blocks) {
                e0 = a0.block_off[b];
                cnt = a0.block_off[b + 1] - e0;
            }
            a.es += (int64_t)e0 * 2 * DP;
            a.en += e0;
            a.ea += e0;
            a.ne = cnt;
        }
    }
    // one pass of the tile's split rows; afterwards the key staging of the
    // four waves (16 rows of 68 floats each, one query set at a time)
    constexpr int kTile = 64 * X::ROW, kStage = 2 * 4 * 16 * 68;
    __shared__ __align__(16) uint16_t tile[kTile > kStage ? kTile : kStage];
    __shared__ float gms[4 * QS * 16 * kGmStride];
    __shared__ __align__(16) float ten[64];
    __shared__ __align__(16) uint32_t tea[64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rl = lane & 15, lq = lane >> 4;
    const int64_t row0 = (int64_t)qgroup * 64 * QS + wave * 16 * QS;  // the wave's first row
    const u32x4 *qrow[QS];  // the lane's query rows, split, in 16-byte units
    float rn[QS], mq[QS];
    uint32_t qw[QS], qm[QS], live16[QS];
#pragma unroll
    for (int h = 0; h < QS; ++h) {
        live16[h] = live_rows16(a, row0 + 16 * h);
        const int64_t row = row0 + 16 * h + rl;
        const int64_t rowc = row < a.nq ? row : a.nq - 1;
        qrow[h] = reinterpret_cast<const u32x4 *>(a.qs + rowc * 2 * DP);
        rn[h] = a.qnorm[rowc];
        qw[h] = a.qword[rowc];
        qm[h] = a.qmask[rowc];
        mq[h] = (float)(__popc(qm[h]) / a.abits);
    }
    if constexpr (QS == 1) {
        const int64_t row = row0 + rl;
        if (group_exact<DP>(a, row < a.nq ? row : a.nq - 1))
            return;  // done by k_entry_keys_b16
    }
    const int cbeg = ctile * (64 * TL);
    const int cend = min(cbeg + 64 * TL, a.ne_pad);
    const int ntiles = (cend - cbeg) / 64;
    const u32x4 *es4 = reinterpret_cast<const u32x4 *>(a.es);

    u32x4 v[X::NV];                // the next pass's entry rows (this thread's share)
    u32x4 qb[2][QS][X::NCK][2];    // query chunks (hi, lo): this pass's and the next's
    EntryMeta em{0.0f, 0u};
    constexpr bool kQOnce = X::NP == 1;  // the same query chunks for every tile
    if (ntiles > 0) {
        x3_load<DP, QS, true>(es4, qrow, cbeg, 0, a.ne, lq, v, qb[0]);
        em = load_entry_meta(a, cbeg);
    }
    for (int t = 0; t < ntiles; ++t) {
        const int c0 = cbeg + 64 * t;
        f32x4 acc[QS][4];
#pragma unroll
        for (int h = 0; h < QS; ++h)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[h][s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < X::NP; ++kc) {
            __syncthreads();  // the previous pass's readers of the LDS are done
#pragma unroll
            for (int it = 0; it < X::NV; ++it) {
                const int i = (int)threadIdx.x + 256 * it, r = i / (X::KC / 4), c4 = i - r * (X::KC / 4);
                *reinterpret_cast<u32x4 *>(tile + r * X::ROW + 8 * c4) = v[it];
            }
            if (kc == 0)
                put_entry_meta(em, ten, tea);
            __syncthreads();
            // the next pass's loads (the next tile's first pass after the
            // last), in flight during this pass's products; one call with a
            // fixed target buffer, so the buffers stay in registers
            if (kc + 1 < X::NP || t + 1 < ntiles) {
                const bool last = kc + 1 == X::NP;
                x3_load<DP, QS, !kQOnce>(es4, qrow, last ? c0 + 64 : c0, last ? 0 : kc + 1, a.ne, lq, v,
                                         qb[(kc + 1) & 1]);
                if (last)
                    em = load_entry_meta(a, c0 + 64);
            }
            const int cur = kc & 1;
#pragma unroll
            for (int j = 0; j < X::NCK; ++j) {
                bf16x8 ah[4], al[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const uint16_t *er = tile + (16 * s + rl) * X::ROW + 64 * j + 8 * lq;
                    ah[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(er));
                    al[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(er + 32));
                }
#pragma unroll
                for (int h = 0; h < QS; ++h) {
                    if (live16[h] == 0u)
                        continue;  // a set of padding slots (wave-uniform)
                    const bf16x8 bh = __builtin_bit_cast(bf16x8, qb[cur][h][j][0]);
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, qb[cur][h][j][1]);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[h][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], bh, acc[h][s], 0, 0, 0);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[h][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], bl, acc[h][s], 0, 0, 0);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[h][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s], bh, acc[h][s], 0, 0, 0);
                }
            }
        }
        // an odd pass count leaves the next tile's first chunks in buffer 1
        if constexpr (X::NP % 2 == 1 && !kQOnce) {
#pragma unroll
            for (int h = 0; h < QS; ++h)
#pragma unroll
                for (int j = 0; j < X::NCK; ++j) {
                    qb[0][h][j][0] = qb[1][h][j][0];
                    qb[0][h][j][1] = qb[1][h][j][1];
                }
        }
        __syncthreads();  // the tile's products are done: its LDS stages the keys
#pragma unroll
        for (int h = 0; h < QS; ++h)
            if (live16[h] != 0u)
                store_keys<DEF, TL>(a, acc[h], c0, row0 + 16 * h, rl, lq, rn[h], qw[h], qm[h], mq[h], ten, tea,
                                    reinterpret_cast<float *>(tile) + wave * 16 * 68,
                                    gms + (wave * QS + h) * 16 * kGmStride, (c0 - cbeg) / 16, live16[h]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int h = 0; h < QS; ++h)
        flush_gmin<TL>(a, gms + (wave * QS + h) * 16 * kGmStride, row0 + 16 * h, cbeg / 16, (cend - cbeg) / 16,
                       live16[h]);
}

// The same product on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16) for
// workgroups whose queries are all integers of magnitude <= 256 against the
// exact bf16 copy of the entry sample: every product is exact in float32 and
// every partial sum is an integer below 2^24 (rows of at most 128
// elements), so the keys are bit-identical to the split kernel's (whose lo
// halves are zero on such data) and to the float32 definition.
template <int DP, bool DEF, int TL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_entry_keys_b16(const KeyArgs a)
{
    constexpr int kKeyTiles = TL, kGmStride = GmStride<TL>::v;
    static_assert(DP <= 128 && DP % 32 == 0, "bf16 path: rows of at most 128 elements");
    __shared__ __align__(16) uint16_t t16[64 * (DP + 8) < 2 * 4 * 16 * 68 ? 2 * 4 * 16 * 68 : 64 * (DP + 8)];
    __shared__ float gms[4 * 16 * kGmStride];
    __shared__ __align__(16) float ten[64];
    __shared__ __align__(16) uint32_t tea[64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rl = lane & 15, lq = lane >> 4;
    const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + rl;
    const bool row_ok = row < a.nq;
    const int64_t rowc = row_ok ? row : a.nq - 1;
    const float rn = a.qnorm[rowc];
    const uint32_t qw = a.qword[rowc], qm = a.qmask[rowc];
    const float mq = (float)(__popc(qm) / a.abits);
    constexpr int NB = DP / 32;   // 32-element chunks
    constexpr int LDSB = DP + 8;  // row stride in LDS (elements)
    if (!group_exact<DP>(a, rowc))
        return;  // left to the split kernel
    const uint32_t live16 = live_rows16(a, (int64_t)blockIdx.x * 64 + wave * 16);
    bf16x8 qb[NB];
    {
        // query elements 32 t + 8 lq + 0..7, exact in bf16 (the top half of the float)
        const float *qf = a.qpad + rowc * DP;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            uint32_t u[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t lo = __float_as_uint(qf[32 * t + 8 * lq + 2 * e]);
                const uint32_t hi = __float_as_uint(qf[32 * t + 8 * lq + 2 * e + 1]);
                u[e] = (lo >> 16) | (hi & 0xFFFF0000u);
            }
            qb[t] = __builtin_bit_cast(bf16x8, make_uint4(u[0], u[1], u[2], u[3]));
        }
    }
    const int cbeg = blockIdx.y * (64 * kKeyTiles);
    for (int c0 = cbeg; c0 < cbeg + 64 * kKeyTiles && c0 < a.ne_pad; c0 += 64) {
        f32x4 acc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        {
            // stage 64 bf16 entry rows (every load issued before the first
            // write), then 4 x NB matrix-core products
            constexpr int kIt = 64 * (DP / 8) / 256;
            static_assert(kIt * 256 == 64 * (DP / 8), "whole staging rounds");
            __syncthreads();
            uint4 v[kIt];
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int i = (int)threadIdx.x + 256 * it, r = i / (DP / 8), c8 = i - r * (DP / 8);
                const int col = min(c0 + r, a.ne - 1);
                v[it] = reinterpret_cast<const uint4 *>(a.eb + (int64_t)col * DP)[c8];
            }
            const EntryMeta em = load_entry_meta(a, c0);
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int i = (int)threadIdx.x + 256 * it, r = i / (DP / 8), c8 = i - r * (DP / 8);
                *reinterpret_cast<uint4 *>(t16 + r * LDSB + 8 * c8) = v[it];
            }
            put_entry_meta(em, ten, tea);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < NB; ++t) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const uint4 ev = *reinterpret_cast<const uint4 *>(t16 + (16 * s + rl) * LDSB + 32 * t + 8 * lq);
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ev), qb[t],
                                                                    acc[s], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // the tile's products are done: its LDS stages the keys
        store_keys<DEF, TL>(a, acc, c0, (int64_t)blockIdx.x * 64 + wave * 16, rl, lq, rn, qw, qm, mq, ten, tea,
                        reinterpret_cast<float *>(t16) + wave * 16 * 68, gms + wave * 16 * kGmStride,
                        (c0 - cbeg) / 16, live16);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    flush_gmin<TL>(a, gms + wave * 16 * kGmStride, (int64_t)blockIdx.x * 64 + wave * 16, cbeg / 16,
               (min(cbeg + 64 * kKeyTiles, a.ne_pad) - cbeg) / 16, live16);
}

// One wave per query, K > 64: the row in registers, a radix select over it.
template <int NJ>
__global__ __launch_bounds__(64) void k_entry_select(const float *__restrict__ keys, int64_t nq,
                                                     int ne, int ne_pad, int K, int32_t *__restrict__ cand,
                                                     const int32_t *__restrict__ live)
{
    const int lane = threadIdx.x;
    const int64_t qi = blockIdx.x;
    if (qi >= nq || (live && live[qi] < 0))
        return;
    const float *row = keys + qi * ne_pad;
    int32_t *out = cand + qi * K;
    uint32_t v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        v[j] = 64 * j + lane < ne ? __float_as_uint(row[64 * j + lane]) : 0xFFFFFFFFu;
    const uint32_t p = kth_pattern<NJ>(v, K);
    emit_best<NJ>(v, [&](int t) { return 64 * t + lane; }, p, K, ne, out);
}

// One wave per query, K <= 64: the group-minimum bound (see the top).  The
// groups at or below the bound are read 4 at a time in increasing order, so
// the kept keys stay in position order, which breaks ties at the K-th key
// by position.  GPL = group minima per lane.
template <int GPL>
__global__ __launch_bounds__(64) void k_entry_select_g(const float *__restrict__ keys,
                                                       const float *__restrict__ gmin, int64_t nq, int ne,
                                                       int ne_pad, int K, int32_t *__restrict__ cand,
                                                       const int32_t *__restrict__ live)
{
    constexpr int kRounds = 16;  // 64 groups of 16 keys
    constexpr int kCap = 128;    // kept keys
    __shared__ int32_t sg[64 * GPL];
    __shared__ uint32_t cv[256];
    __shared__ int32_t cp[256];
    const int lane = threadIdx.x;
    const int64_t qi = blockIdx.x;
    if (qi >= nq || (live && live[qi] < 0))
        return;
    const int ng = ne_pad / 16;
    const uint32_t *row = reinterpret_cast<const uint32_t *>(keys + qi * ne_pad);
    int32_t *out = cand + qi * K;
    uint32_t mn[GPL];
#pragma unroll
    for (int t = 0; t < GPL; ++t) {
        const int g = 64 * t + lane;
        mn[t] = g < ng ? __float_as_uint(gmin[qi * ng + g]) : 0xFFFFFFFFu;
    }
    const uint32_t u = kth_pattern<GPL>(mn, K);
    int nsel = 0;
#pragma unroll
    for (int t = 0; t < GPL; ++t) {
        const bool in = mn[t] <= u && 64 * t + lane < ng;
        const uint64_t b = __ballot(in);
        if (in)
            sg[nsel + rank_below(b)] = 64 * t + lane;
        nsel += __popcll(b);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (nsel <= 4 * kRounds) {
        uint32_t v[kRounds];
        int32_t ps[kRounds];
#pragma unroll
        for (int it = 0; it < kRounds; ++it) {
            const int j = 4 * it + (lane >> 4);
            v[it] = 0xFFFFFFFFu;
            ps[it] = -1;
            if (j < nsel) {
                const int pos = 16 * sg[j] + (lane & 15);
                if (pos < ne) {
                    v[it] = row[pos];
                    ps[it] = pos;
                }
            }
        }
        int c = 0;
#pragma unroll
        for (int it = 0; it < kRounds; ++it)
            c += __popcll(__ballot(ps[it] >= 0 && v[it] <= u));
        if (c <= kCap) {
            int base = 0;
#pragma unroll
            for (int it = 0; it < kRounds; ++it) {
                const bool in = ps[it] >= 0 && v[it] <= u;
                const uint64_t b = __ballot(in);
                if (in) {
                    const int r = base + rank_below(b);
                    cv[r] = v[it];
                    cp[r] = ps[it];
                }
                base += __popcll(b);
            }
            for (int i = base + lane; i < kCap; i += 64) {
                cv[i] = 0xFFFFFFFFu;
                cp[i] = -1;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            uint32_t w[kCap / 64];
#pragma unroll
            for (int t = 0; t < kCap / 64; ++t)
                w[t] = cv[64 * t + lane];
            const uint32_t p = kth_pattern<kCap / 64>(w, K);
            emit_best<kCap / 64>(w, [&](int t) { return cp[64 * t + lane]; }, p, K, ne, out);
            return;
        }
    }
    select_lds(row, ne, K, cv, cp, out);
}

}  // namespace

// positions of the n_cand best entry-sample members per query (unordered)
namespace {

// tiles per workgroup: the most of (8, 2) that still gives min_wg
// workgroups, else 1
int pick_tiles(int64_t groups, int nj, int64_t min_wg)
{
    for (int t : {kMaxKeyTiles, 2})
        if (groups * ((nj + t - 1) / t) >= min_wg)
            return t;
    return 1;
}

template <template <int, bool, int> class L, int DP>
void launch_tiles(int tl, bool def, dim3 grid, const KeyArgs &a, hipStream_t st)
{
    if (tl == kMaxKeyTiles)
        def ? L<DP, true, kMaxKeyTiles>::go(grid, a, st) : L<DP, false, kMaxKeyTiles>::go(grid, a, st);
    else if (tl == 2)
        def ? L<DP, true, 2>::go(grid, a, st) : L<DP, false, 2>::go(grid, a, st);
    else
        def ? L<DP, true, 1>::go(grid, a, st) : L<DP, false, 1>::go(grid, a, st);
}
template <int DP, bool DEF, int TL>
struct LaunchB16 {
    static void go(dim3 g, const KeyArgs &a, hipStream_t st)
    {
        if constexpr (DP <= 128 && DP % 32 == 0)
            hipLaunchKernelGGL((k_entry_keys_b16<DP, DEF, TL>), g, dim3(256), 0, st, a);
    }
};
template <int DP, bool DEF, int TL>
struct LaunchX3Q1 {
    static void go(dim3 g, const KeyArgs &a, hipStream_t st)
    {
        hipLaunchKernelGGL((k_entry_keys_x3<DP, DEF, TL, 1>), g, dim3(256), 0, st, a);
    }
};
template <int DP, bool DEF, int TL>
struct LaunchX3Q2 {
    static void go(dim3 g, const KeyArgs &a, hipStream_t st)
    {
        hipLaunchKernelGGL((k_entry_keys_x3<DP, DEF, TL, 2>), g, dim3(256), 0, st, a);
    }
};

// workgroups the split kernel aims for (about 2.5 per resident slot on 256
// compute units, so the last round of workgroups is a small share)
constexpr int64_t kX3MinWorkgroups = 2048;

// The key kernels over rows 0 .. a.nq - 1 and entry tiles of a.ne_pad
// columns: the exact bf16 kernel for the workgroups it takes (rows <= 128
// wide, exact bf16 copies present: groups of 64 queries), and the split
// kernel, two query sets per wave where neither that nor a stratified
// sample fixes the groups at 64 queries.
template <int DP>
void launch_keys_dp(bool def, const KeyArgs &a, hipStream_t st)
{
    const int nj = a.ne_pad / 64;
    const bool b16 = DP <= 128 && DP % 32 == 0 && a.eb && a.qx;
    if (b16) {
        const int64_t groups = (a.nq + 63) / 64;
        const int tl = pick_tiles(groups, nj, 1024);
        launch_tiles<LaunchB16, DP>(tl, def, dim3((unsigned)groups, (unsigned)((nj + tl - 1) / tl)), a, st);
    }
    const int qs = (b16 || a.seg) ? 1 : 2;
    const int64_t groups = (a.nq + 64 * qs - 1) / (64 * qs);
    const int tl = pick_tiles(groups, nj, kX3MinWorkgroups);
    const dim3 grid((unsigned)(groups * ((nj + tl - 1) / tl)));
    if (qs == 1)
        launch_tiles<LaunchX3Q1, DP>(tl, def, grid, a, st);
    else
        launch_tiles<LaunchX3Q2, DP>(tl, def, grid, a, st);
}

int launch_keys(const Index *ix, const KeyArgs &a, hipStream_t st)
{
    if (!a.qs || !a.es)
        return fail(NHQ_EINVAL, "seed ranking without split rows");
    const bool def = ix->w.mode == NHQ_WEIGHTS_DEFAULT;
    switch (ix->dp) {
    case 32: launch_keys_dp<32>(def, a, st); break;
    case 64: launch_keys_dp<64>(def, a, st); break;
    case 96: launch_keys_dp<96>(def, a, st); break;
    case 128: launch_keys_dp<128>(def, a, st); break;
    case 256: launch_keys_dp<256>(def, a, st); break;
    case 512: launch_keys_dp<512>(def, a, st); break;
    case 960: launch_keys_dp<960>(def, a, st); break;
    case 1024: launch_keys_dp<1024>(def, a, st); break;
    default: return fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    if (hipGetLastError() != hipSuccess)
        return fail(NHQ_EHIP, "entry key launch failed");
    return NHQ_OK;
}

// positions of the K best keys of each row (rows with live[row] < 0 skipped)
int launch_select(const float *keys, const float *gmin, int64_t rows, int ne, int ne_pad, int K, int32_t *cand,
                  const int32_t *live, hipStream_t st)
{
    const int nj = ne_pad / 64;
    const dim3 g2((unsigned)rows);
    const int gpl = (ne_pad / 16 + 63) / 64;
    if (K <= 64) {
        if (gpl <= 1)
            hipLaunchKernelGGL(k_entry_select_g<1>, g2, dim3(64), 0, st, keys, gmin, rows, ne, ne_pad, K, cand, live);
        else if (gpl <= 2)
            hipLaunchKernelGGL(k_entry_select_g<2>, g2, dim3(64), 0, st, keys, gmin, rows, ne, ne_pad, K, cand, live);
        else if (gpl <= 4)
            hipLaunchKernelGGL(k_entry_select_g<4>, g2, dim3(64), 0, st, keys, gmin, rows, ne, ne_pad, K, cand, live);
        else
            hipLaunchKernelGGL(k_entry_select_g<8>, g2, dim3(64), 0, st, keys, gmin, rows, ne, ne_pad, K, cand, live);
    } else if (nj <= 16)
        hipLaunchKernelGGL(k_entry_select<16>, g2, dim3(64), 0, st, keys, rows, ne, ne_pad, K, cand, live);
    else if (nj <= 32)
        hipLaunchKernelGGL(k_entry_select<32>, g2, dim3(64), 0, st, keys, rows, ne, ne_pad, K, cand, live);
    else if (nj <= 64)
        hipLaunchKernelGGL(k_entry_select<64>, g2, dim3(64), 0, st, keys, rows, ne, ne_pad, K, cand, live);
    else
        hipLaunchKernelGGL(k_entry_select<128>, g2, dim3(64), 0, st, keys, rows, ne, ne_pad, K, cand, live);
    if (hipGetLastError() != hipSuccess)
        return fail(NHQ_EHIP, "entry select launch failed");
    return NHQ_OK;
}

// ---- stratified entry sample: queries grouped by their pattern's block

// zero the block counters, mark every slot empty
__global__ void k_strata_clear(int32_t *hist, int nb, int32_t *inv, int64_t slots)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nb)
        hist[t] = 0;
    if (t < slots)
        inv[t] = -1;
}

// each query's block: its pattern's when every attribute is constrained and
// some object holds the pattern (binary search of the sorted block words),
// else the global members (n_blocks); and its position among the block's
// queries (pos).  Counts go through a histogram in LDS, then one global
// atomic per (workgroup, block) reserves the workgroup's run of positions.
constexpr int kStrataMaxBlocks = 4096 + 1;  // patterns plus the global members
__global__ __launch_bounds__(256) void k_strata_assign(const uint32_t *__restrict__ qword,
                                                       const uint32_t *__restrict__ qmask, int64_t nq, int full_bits,
                                                       const uint32_t *__restrict__ block_word, int n_blocks,
                                                       int32_t *__restrict__ qblock, int32_t *__restrict__ pos,
                                                       int32_t *__restrict__ hist)
{
    __shared__ int32_t lh[kStrataMaxBlocks];
    const int nb = n_blocks + 1;
    for (int t = threadIdx.x; t < nb; t += blockDim.x)
        lh[t] = 0;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = q < nq;
    int b = n_blocks, r = 0;
    if (live) {
        if (__popc(qmask[q]) == full_bits) {
            const uint32_t w = qword[q];
            int lo = 0, hi = n_blocks;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (block_word[mid] < w)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo < n_blocks && block_word[lo] == w)
                b = lo;
        }
        r = atomicAdd(&lh[b], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb; t += blockDim.x)
        if (lh[t] > 0)
            lh[t] = atomicAdd(&hist[t], lh[t]);
    __syncthreads();
    if (live) {
        qblock[q] = b;
        pos[q] = lh[b] + r;
    }
}

// slot ranges: block b owns slots off[b] .. off[b] + hist[b] - 1 (ranges
// start at multiples of 64); seg[g] = the block of slots 64 g .. 64 g + 63,
// -1 past the last
__global__ __launch_bounds__(64) void k_strata_scan(const int32_t *__restrict__ hist, int nb,
                                                    int32_t *__restrict__ off, int32_t *__restrict__ seg,
                                                    int64_t nseg)
{
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int b = 0; b < nb; ++b) {
            off[b] = run;
            run += (hist[b] + 63) & ~63;
        }
        off[nb] = run;
    }
    __syncthreads();
    for (int64_t g = threadIdx.x; g < nseg; g += 64) {
        const int32_t s0 = (int32_t)(64 * g);
        int b = -1;
        if (s0 < off[nb]) {
            int lo = 0, hi = nb - 1;  // the last block whose range starts at or before s0
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (off[mid] <= s0)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            b = lo;
        }
        seg[g] = b;
    }
}

// each query's slot: its block's range start plus its position in the block
__global__ void k_strata_slot(const int32_t *__restrict__ qblock, int64_t nq, const int32_t *__restrict__ off,
                              int32_t *__restrict__ perm, int32_t *__restrict__ inv)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq)
        return;
    const int32_t slot = off[qblock[q]] + perm[q];
    perm[q] = slot;
    inv[slot] = (int32_t)q;
}

// the split query rows (dp 32-bit words each: two bf16 halves per word),
// norms and codes in slot order (empty slots: zeros)
__global__ void k_strata_permute(const uint32_t *__restrict__ qsw, const float *__restrict__ qnorm,
                                 const uint32_t *__restrict__ qword, const uint32_t *__restrict__ qmask,
                                 const int32_t *__restrict__ inv, int64_t slots, int dp, uint32_t *__restrict__ ssw,
                                 float *__restrict__ snorm, uint32_t *__restrict__ sword, uint32_t *__restrict__ smask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= slots * dp)
        return;
    const int64_t s = t / dp;
    const int c = (int)(t - s * dp);
    const int32_t q = inv[s];
    ssw[t] = q >= 0 ? qsw[(int64_t)q * dp + c] : 0u;
    if (c == 0) {
        snorm[s] = q >= 0 ? qnorm[q] : 0.0f;
        sword[s] = q >= 0 ? qword[q] : 0u;
        smask[s] = q >= 0 ? qmask[q] : 0u;
    }
}

// block-local positions of each query's slot -> positions in the whole
// entry sample (-1 past the block's members)
__global__ void k_strata_gather(const int32_t *__restrict__ cslot, const int32_t *__restrict__ perm,
                                const int32_t *__restrict__ qblock, const int32_t *__restrict__ block_off,
                                int n_blocks, int n_global, int64_t nq, int K, int32_t *__restrict__ cand)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * K)
        return;
    const int64_t q = t / K;
    const int j = (int)(t - q * K);
    const int b = qblock[q];
    const int32_t e0 = b < n_blocks ? block_off[b] : 0;
    const int32_t cnt = b < n_blocks ? block_off[b + 1] - e0 : n_global;
    const int32_t loc = cslot[(int64_t)perm[q] * K + j];
    cand[t] = (loc >= 0 && loc < cnt) ? e0 + loc : -1;
}

struct StrataLayout {
    int64_t slots, nseg;
    int nb, ne_pad;
    size_t o_ssplit, o_snorm, o_sword, o_smask, o_keys, o_gmin, o_cslot, o_qblock, o_perm, o_inv, o_hist, o_off,
        o_seg, words;
};

StrataLayout strata_layout(const Index *ix, int64_t nq, int K)
{
    StrataLayout L{};
    L.nb = ix->n_blocks + 1;
    L.slots = (nq + 64 * (int64_t)L.nb + 63) / 64 * 64;
    L.nseg = L.slots / 64;
    int emax = ix->n_entry;
    for (int b = 0; b < ix->n_blocks; ++b)
        emax = std::max(emax, ix->block_off_h[b + 1] - ix->block_off_h[b]);
    L.ne_pad = (emax + 63) / 64 * 64;
    size_t o = 0;
    auto take = [&](size_t words) {
        const size_t at = o;
        o += (words + 63) / 64 * 64;  // 256-byte pieces
        return at;
    };
    L.o_ssplit = take((size_t)L.slots * ix->dp);
    L.o_snorm = take((size_t)L.slots);
    L.o_sword = take((size_t)L.slots);
    L.o_smask = take((size_t)L.slots);
    L.o_keys = take((size_t)L.slots * L.ne_pad);
    L.o_gmin = take((size_t)L.slots * (L.ne_pad / 16));
    L.o_cslot = take((size_t)L.slots * K);
    L.o_qblock = take((size_t)nq);
    L.o_perm = take((size_t)nq);
    L.o_inv = take((size_t)L.slots);
    L.o_hist = take((size_t)L.nb + 1);
    L.o_off = take((size_t)L.nb + 1);
    L.o_seg = take((size_t)L.nseg);
    L.words = o;
    return L;
}

}  // namespace

size_t strata_rank_words(const Index *ix, int64_t nq, int K)
{
    return strata_layout(ix, nq, K).words;
}

int launch_strata_rank(const Index *ix, const uint16_t *qsplit, const float *qnorm, const uint32_t *qword,
                       const uint32_t *qmask, int64_t nq, int K, uint32_t *blk, int32_t *cand, hipStream_t st)
{
    const StrataLayout L = strata_layout(ix, nq, K);
    if (L.nb > kStrataMaxBlocks)
        return fail(NHQ_EINVAL, "a stratified entry sample holds at most 4096 attribute patterns");
    uint32_t *ssw = blk + L.o_ssplit;
    float *snorm = reinterpret_cast<float *>(blk + L.o_snorm);
    uint32_t *sword = blk + L.o_sword, *smask = blk + L.o_smask;
    float *keys = reinterpret_cast<float *>(blk + L.o_keys);
    float *gmin = reinterpret_cast<float *>(blk + L.o_gmin);
    int32_t *cslot = reinterpret_cast<int32_t *>(blk + L.o_cslot);
    int32_t *qblock = reinterpret_cast<int32_t *>(blk + L.o_qblock);
    int32_t *perm = reinterpret_cast<int32_t *>(blk + L.o_perm);
    int32_t *inv = reinterpret_cast<int32_t *>(blk + L.o_inv);
    int32_t *hist = reinterpret_cast<int32_t *>(blk + L.o_hist);
    int32_t *off = reinterpret_cast<int32_t *>(blk + L.o_off);
    int32_t *seg = reinterpret_cast<int32_t *>(blk + L.o_seg);
    const int64_t clear = std::max<int64_t>(L.slots, L.nb);
    hipLaunchKernelGGL(k_strata_clear, dim3((unsigned)((clear + 255) / 256)), dim3(256), 0, st, hist, L.nb,
                       inv, L.slots);
    hipLaunchKernelGGL(k_strata_assign, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, qword, qmask, nq,
                       ix->m * ix->abits, ix->block_word, ix->n_blocks, qblock, perm, hist);
    hipLaunchKernelGGL(k_strata_scan, dim3(1), dim3(64), 0, st, hist, L.nb, off, seg, L.nseg);
    hipLaunchKernelGGL(k_strata_slot, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, qblock, nq, off, perm,
                       inv);
    hipLaunchKernelGGL(k_strata_permute, dim3((unsigned)((L.slots * ix->dp + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const uint32_t *>(qsplit), qnorm, qword, qmask, inv, L.slots, ix->dp, ssw,
                       snorm, sword, smask);
    NHQ_HIP(hipGetLastError());
    KeyArgs a{nullptr, reinterpret_cast<const uint16_t *>(ssw), snorm, sword, smask, ix->entry_split,
              ix->entry_norm, ix->entry_attr, nullptr, nullptr, keys, gmin, L.slots, ix->n_entry, L.ne_pad, ix->w,
              ix->abits, ix->hmask};
    a.seg = seg;
    a.block_off = ix->block_off;
    a.n_blocks = ix->n_blocks;
    a.n_global = ix->n_entry;
    a.live = inv;
    int rc = launch_keys(ix, a, st);
    if (rc != NHQ_OK)
        return rc;
    rc = launch_select(keys, gmin, L.slots, L.ne_pad, L.ne_pad, K, cslot, inv, st);
    if (rc != NHQ_OK)
        return rc;
    hipLaunchKernelGGL(k_strata_gather, dim3((unsigned)((nq * K + 255) / 256)), dim3(256), 0, st, cslot, perm,
                       qblock, ix->block_off, ix->n_blocks, ix->n_entry, nq, K, cand);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

int launch_seed_rank(const Index *ix, const float *qpad, const uint16_t *qsplit, const float *qnorm,
                     const uint32_t *qword, const uint32_t *qmask, const uint32_t *qexact, int64_t nq, int K,
                     float *keys, int32_t *cand, hipStream_t st)
{
    const int ne = ix->n_entry;
    const int ne_pad = (ne + 63) / 64 * 64;
    if (ne_pad / 64 > 128)
        return fail(NHQ_EINVAL, "entry sample larger than 8192");
    KeyArgs a{qpad, qsplit, qnorm, qword, qmask, ix->entry_split, ix->entry_norm, ix->entry_attr, ix->entry_bf16,
              qexact, keys, keys + (size_t)nq * ne_pad, nq, ne, ne_pad, ix->w, ix->abits, ix->hmask};
    int rc = launch_keys(ix, a, st);
    if (rc == NHQ_OK)
        rc = launch_select(keys, a.gmin, nq, ne, ne_pad, K, cand, nullptr, st);
    return rc;
}

}  // namespace nhq
