// Device building blocks of the joint-pruning search (Alg. 2 in beam form):
// per-query arguments, candidate scoring, the LDS pool merge, the visited
// set, the stop network and the whole per-query search by one wavefront.
// Included by the batch search and by the serving loop.
#pragma once
#include <algorithm>

#include "mlp_infer.h"
#include "nhq_internal.h"

namespace nhq {
namespace {

struct SearchArgs {
    const void *vecs;
    const float *vec32;
    const float *scale;
    const uint32_t *attr;
    const int32_t *adj;
    const int32_t *seed_cand;  // [nq][n_seed] positions in the entry sample (-1 padded)
    const int32_t *entry;      // entry sample: position -> vertex id
    const float *entry_vec_f;  // [n_entry][DP] float32 rows of the entry sample
    const uint32_t *entry_attr;  // [n_entry] packed codes of the entry sample
    const float *q;
    const uint8_t *qa;
    int32_t *out_ids;
    float *out_dist;
    uint32_t *counters;
    uint32_t *err;
    int64_t n;
    int64_t nq;
    int d, m, R, n_seed, n_entry;
    int k, L, n_init, out_mode, rerank_n, max_hops;
    int scap;       // staging capacity (entries)
    int vis_words;  // visited-set words
    int use_bitset;
    int hash_log2;
    // checkpoints every `ckpt` hops (0 = none): features for the stop network
    int ckpt, learned;
    int expand;           // vertices expanded per step (1 = Alg. 2 as printed)
    int route_h;          // >= 2: two-stage routing, stage S1 evaluates 1 slot in h
    int seeds_shared;     // every query reads the first row of seed_cand
    int abits;            // attribute field width of the packed words
    uint32_t hmask;       // high bit of every attribute field
    Weights w;            // weight setting of Gamma (the index's)
    float stop_logit;     // learned: stop when the stop logit >= this
    float cap_factor;     // learned, > 0: hop budget cap_factor * 2^(beam output)
    const uint16_t *mlp;  // fp16 weights of the stop network
    const float *logp;    // [m][256] ln(count / n) per attribute code
    float *trace_feat;    // [nq][trace_cap][8] (nullable: no trace)
    uint32_t *trace_hop;  // [nq][trace_cap]
    uint32_t *trace_hash; // [nq][trace_cap]
    int32_t *trace_count; // [nq]
    uint32_t *final_hash; // [nq]
    int trace_cap;
    const int32_t *order;  // nullable: wave i searches query order[i]
};

// padded widths from which a search reads the query row from LDS
constexpr int kQueryLdsMinDp = 512;

template <int DP>
struct Shape {
    static constexpr int G = DP <= 512 ? 8 : 16;           // lanes per row
    static constexpr int NG = 64 / G;                      // rows per round
    static constexpr int NCH = DP / (4 * G);               // 4-element chunks per lane
    static constexpr int RB = NCH <= 4 ? 2 : 1;  // rounds in flight
    // the query row is read from the wave's LDS copy rather than held in
    // registers (4 NCH of them per lane) when rows are this wide: the freed
    // registers hold more waves, and so more row gathers in flight
    static constexpr bool QL = DP >= kQueryLdsMinDp;
    static_assert(DP % (4 * G) == 0, "padded width must split into lane chunks");
};

template <int ST>
struct Chunk;
template <>
struct Chunk<NHQ_STORAGE_FP32> {
    using T = float4;
};
template <>
struct Chunk<NHQ_STORAGE_BF16> {
    using T = uint2;
};
template <>
struct Chunk<NHQ_STORAGE_FP8> {
    using T = uint32_t;
};

// A lane's 4-element chunks of a row: fp8 rows take K4 neighbouring chunks
// per load (up to 16 bytes); the other forms load 16 (fp32) or 8 (bf16)
// bytes per chunk already.  Lane g's c-th chunk is chunk
// K4 (g + G (c / K4)) + c % K4 of the row.
template <int DP, int ST>
struct Lay {
    static constexpr int NCH = Shape<DP>::NCH;
    static constexpr int K4 = ST != NHQ_STORAGE_FP8 ? 1
                              : NCH % 4 == 0       ? 4
                              : NCH % 3 == 0       ? 3
                              : NCH % 2 == 0       ? 2
                                                   : 1;
    // rounds of rows in flight per wave: two when a lane's share of a round
    // is at most 120 bytes (wide bf16 / fp8 rows fit the float32 row's
    // register budget with two rounds), else the width's default.  The
    // checkpointed search keeps the width's default: the stop network's
    // registers plus a second round would cost it a wave per SIMD.
    static constexpr int CHB = ST == NHQ_STORAGE_FP32 ? 16 : ST == NHQ_STORAGE_BF16 ? 8 : 4;
    static constexpr int RB = Shape<DP>::RB > 1 ? Shape<DP>::RB : (NCH * CHB <= 120 ? 2 : 1);
};

template <int DP, int K4>
__device__ __forceinline__ int lane_chunk(int g, int c)
{
    return K4 * (g + Shape<DP>::G * (c / K4)) + c % K4;
}

// The query slice a lane scores with, its c-th chunk at a time (lane g of a
// row group, chunks in the order of lane_chunk<DP, K4>): held in registers
// (v[c]) or, when QL, read from a zero-padded copy of the query row in LDS
// (the row groups of a wave read the same addresses, which LDS broadcasts).
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const f32x4v lds_f32x4;

template <int DP, int K4, bool QL>
struct QSrc {
    const float4 *v;        // registers (QL false)
    const lds_f32x4 *row;   // LDS, DP / 4 chunks (QL true)
    __device__ __forceinline__ float4 at(int c, int g) const
    {
        if constexpr (QL) {
            const f32x4v x = row[lane_chunk<DP, K4>(g, c)];
            return make_float4(x.x, x.y, x.z, x.w);
        } else {
            return v[c];
        }
    }
};

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int rdl_i(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ uint32_t rdl_u(uint32_t v, int i)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, i);
}
__device__ __forceinline__ float rdl_f(float v, int i)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}


__device__ __forceinline__ bool lt_key(float ka, uint32_t ia, float kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

template <int ST>
__device__ __forceinline__ float4 decode(typename Chunk<ST>::T c, float s);

template <>
__device__ __forceinline__ float4 decode<NHQ_STORAGE_FP32>(float4 c, float)
{
    return c;
}
template <>
__device__ __forceinline__ float4 decode<NHQ_STORAGE_BF16>(uint2 c, float)
{
    return make_float4(__uint_as_float(c.x << 16), __uint_as_float(c.x & 0xFFFF0000u),
                       __uint_as_float(c.y << 16), __uint_as_float(c.y & 0xFFFF0000u));
}
template <>
__device__ __forceinline__ float4 decode<NHQ_STORAGE_FP8>(uint32_t c, float s)
{
    // OCP e4m3 (gfx950 hardware conversion), then the per-vector scale
    auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)c, false);
    auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)c, true);
    return make_float4(lo[0] * s, lo[1] * s, hi[0] * s, hi[1] * s);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over a group of G (8 or 16) adjacent lanes, every lane receiving the
// total: DPP lane moves (quad swaps of 1 and 2, then the half-row and row
// mirrors), no LDS traffic.
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(G == 8 || G == 16, "row groups of 8 or 16 lanes");
    v += dpp_mov<0xB1>(v);   // quad_perm(1, 0, 3, 2)
    v += dpp_mov<0x4E>(v);   // quad_perm(2, 3, 0, 1)
    v += dpp_mov<0x141>(v);  // row_half_mirror: lane i <-> 7 - i
    if constexpr (G == 16)
        v += dpp_mov<0x140>(v);  // row_mirror: lane i <-> 15 - i
    return v;
}

// Score staged candidates sid[0..nf): for each, delta^2 of the query and the
// row (storage ST), written to out[j] as the ordering key or as delta^2.
// mode 0: key, chi taken from the staged word; mode 1: key, chi computed
// from the attribute word (fetched together with the row) and written into
// the staged word; mode 2: delta^2.  RB rounds of rows are loaded before
// any of them is scored.
template <int DP, int ST, int K4, int RB, class Q>
__device__ __forceinline__ void score_batch(const void *vbase, const float *scale, const Q &qv,
                                            uint32_t *sid, float *out, int nf, int mq,
                                            int mode, const Weights &wt,
                                            const uint32_t *attr = nullptr,
                                            uint32_t qword = 0, uint32_t qmask = 0,
                                            uint32_t hmask = 0x80808080u)
{
    using S = Shape<DP>;
    using T = typename Chunk<ST>::T;
    const int lane = threadIdx.x & 63;
    const int g = lane % S::G, gi = lane / S::G;
    const int rounds = (nf + S::NG - 1) / S::NG;
    for (int r0 = 0; r0 < rounds; r0 += RB) {
        T buf[RB][S::NCH];
        float sc[RB];
        uint32_t w[RB], aw[RB];
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            const int j = (r0 + rr) * S::NG + gi;
            w[rr] = 0;
            aw[rr] = 0;
            sc[rr] = 1.0f;
            if (j < nf) {
                w[rr] = sid[j];
                const int64_t id = w[rr] & kIdMask;
                const T *row = reinterpret_cast<const T *>(vbase) + id * (DP / 4);
#pragma unroll
                for (int c = 0; c < S::NCH; ++c)
                    buf[rr][c] = row[lane_chunk<DP, K4>(g, c)];
                if (ST == NHQ_STORAGE_FP8)
                    sc[rr] = scale[id];
                if (mode == 1 && g == 0)
                    aw[rr] = attr[id];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            const int j = (r0 + rr) * S::NG + gi;
            float a0 = 0.0f, a1 = 0.0f;
            if (j < nf) {
#pragma unroll
                for (int c = 0; c < S::NCH; ++c) {
                    const float4 x = decode<ST>(buf[rr][c], sc[rr]);
                    const float4 qc = qv.at(c, g);
                    const float t0 = qc.x - x.x, t1 = qc.y - x.y;
                    const float t2 = qc.z - x.z, t3 = qc.w - x.w;
                    a0 = fmaf(t0, t0, a0);
                    a1 = fmaf(t1, t1, a1);
                    a0 = fmaf(t2, t2, a0);
                    a1 = fmaf(t3, t3, a1);
                }
            }
            float d2 = group_sum<S::G>(a0 + a1);
            if (j < nf && g == 0) {
                int c = (int)((w[rr] >> kChiShift) & kChiMask);
                if (mode == 1) {
                    c = chi_of(aw[rr], qword, qmask, hmask);
                    sid[j] = w[rr] | ((uint32_t)c << kChiShift);
                }
                // the default key inline; the other weight settings take
                // delta^2 here and finish in weigh_keys
                out[j] = (mode == 2 || wt.mode != NHQ_WEIGHTS_DEFAULT)
                             ? d2
                             : (mq == 0 ? d2 : d2 * (float)((mq + c) * (mq + c)));
            }
        }
    }
}

// Non-default weight settings: turn the staged delta^2 into the key (Gamma),
// chi taken from the staged words.
__device__ __forceinline__ void weigh_keys(float *skey, const uint32_t *sid, int n, int mq,
                                        const Weights &w)
{
    for (int j = threadIdx.x & 63; j < n; j += 64)
        skey[j] = w_key32(skey[j], (int)((sid[j] >> kChiShift) & kChiMask), mq, w);
    wsync();
}

// Merge one batch of candidates (lane j holds candidate j when `valid`) into
// the sorted pool of capacity `cap`: the pool becomes the cap best of
// pool + batch by (key, id).  Candidates already pooled are dropped.  `lo`
// (first position that may hold an unexpanded entry) is lowered to the
// first insertion point.  Returns the new size; `inserted` (nullable) gets
// the number of candidates written into the pool and `mine` (nullable) each
// lane's own outcome.
__device__ int pool_merge(float *pkey, uint32_t *pid, int size, int cap, float ck, uint32_t cw,
                          bool valid, int &lo, int *inserted = nullptr, bool *mine = nullptr)
{
    const int lane = threadIdx.x & 63;
    const uint32_t cm = cw & kIdMask;
    if (valid && size >= cap) {
        const float wk = pkey[cap - 1];
        const uint32_t wm = pid[cap - 1] & kIdMask;
        valid = lt_key(ck, cm, wk, wm);
    }
    int p = 0;
    if (valid) {
        int a0 = 0, a1 = size;
        while (a0 < a1) {
            const int mid = (a0 + a1) >> 1;
            if (lt_key(pkey[mid], pid[mid] & kIdMask, ck, cm))
                a0 = mid + 1;
            else
                a1 = mid;
        }
        p = a0;
        if (p < size && pkey[p] == ck && (pid[p] & kIdMask) == cm)
            valid = false;
    }
    const uint64_t bal = __ballot(valid);
    if (mine)
        *mine = false;
    if (bal == 0) {
        if (inserted)
            *inserted = 0;
        return size;
    }
    int rank = 0, pmin = size;
    for (uint64_t b = bal; b; b &= b - 1) {
        const int i = __ffsll((unsigned long long)b) - 1;
        const float ki = rdl_f(ck, i);
        const uint32_t mi = rdl_u(cm, i);
        const int pi = rdl_i(p, i);
        rank += lt_key(ki, mi, ck, cm) ? 1 : 0;
        pmin = min(pmin, pi);
    }
    const int nv = __popcll(bal);
    const int nsize = min(cap, size + nv);
    if (pmin < size) {
        for (int base = pmin + ((size - 1 - pmin) & ~63); base >= pmin; base -= 64) {
            const int e = base + lane;
            const bool act = e < size;
            float ek = 0.0f;
            uint32_t ew = 0;
            if (act) {
                ek = pkey[e];
                ew = pid[e];
            }
            int sh = 0;
            for (uint64_t b = bal; b; b &= b - 1) {
                const int i = __ffsll((unsigned long long)b) - 1;
                sh += (rdl_i(p, i) <= e) ? 1 : 0;
            }
            wsync();
            if (act && e + sh < cap) {
                pkey[e + sh] = ek;
                pid[e + sh] = ew;
            }
            wsync();
        }
    }
    if (valid && p + rank < cap) {
        pkey[p + rank] = ck;
        pid[p + rank] = cw;
    }
    if (inserted)
        *inserted = __popcll(__ballot(valid && p + rank < cap));
    if (mine)
        *mine = valid && p + rank < cap;
    wsync();
    lo = min(lo, pmin);
    return nsize;
}

// MurmurHash3's 32-bit finaliser; the eligible top-k is fingerprinted by the
// sum (mod 2^32) of fmix32(id + 0x9E3779B9) over its ids (order-free)
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_sum_f32(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// The first k eligible pool entries (attribute matches; every entry in raw
// mode): how many of the first k positions are eligible, their fingerprint,
// and the key of the k-th one (has_kth false when fewer than k exist).
__device__ void eligible_topk(const float *pkey, const uint32_t *pid, int size, int k, int out_mode,
                              int &in_first_k, uint32_t &hash, float &key_kth, bool &has_kth)
{
    const int lane = threadIdx.x & 63;
    int nel = 0, fk = 0;
    uint32_t h = 0;
    has_kth = false;
    key_kth = 0.0f;
    for (int base = 0; base < size && nel < k; base += 64) {
        const int e = base + lane;
        const uint32_t w = e < size ? pid[e] : 0u;
        const bool el = e < size && (out_mode == 1 || ((w >> kChiShift) & kChiMask) == 0);
        const uint64_t bb = __ballot(el);
        const int pos = nel + lanes_below(bb);
        const bool take = el && pos < k;
        h += take ? fmix32((w & kIdMask) + 0x9E3779B9u) : 0u;
        fk += __popcll(__ballot(el && e < k));
        const uint64_t kb = __ballot(el && pos == k - 1);
        if (kb) {
            has_kth = true;
            key_kth = rdl_f(e < size ? pkey[e] : 0.0f, __ffsll((unsigned long long)kb) - 1);
        }
        nel += __popcll(bb);
    }
    hash = wave_sum_u32(h);
    in_first_k = fk;
}

__device__ __forceinline__ float h2f(uint16_t b)
{
    _Float16 v;
    __builtin_memcpy(&v, &b, 2);
    return (float)v;
}

// visited test-and-set; returns true when v was not yet visited.  `unrec`
// reports a fresh vertex the hash could not record (table region full).
__device__ __forceinline__ bool visit(uint32_t *vis, bool bitset, int hash_log2, uint32_t v,
                                      bool &unrec)
{
    unrec = false;
    if (bitset) {
        const uint32_t bit = 1u << (v & 31u);
        const uint32_t old = atomicOr(&vis[v >> 5], bit);
        return (old & bit) == 0;
    }
    const uint32_t slots_mask = (1u << hash_log2) - 1u;
    uint32_t h = (v * 0x9E3779B1u) >> (32 - hash_log2);
#pragma unroll 1
    for (int probe = 0; probe < 16; ++probe) {
        const uint32_t s = (h + (uint32_t)probe) & slots_mask;
        const uint32_t old = atomicCAS(&vis[s], kEmpty, v);
        if (old == kEmpty)
            return true;
        if (old == v)
            return false;
    }
    unrec = true;
    return true;
}

// Per-query state of the checkpoints, kept in LDS (after the visited set, 16-
// byte aligned) rather than in registers across the expansion loop.
struct CkState {
    float h1[64];  // the stop network's hidden layer
    float f[8];    // the features of the current checkpoint
    float logsel, key_kth_first;
    uint32_t prev_hash;
    int last_change, ntrace, have_first, have_prev, first_ckpt;
};
constexpr int kCkWords = 96;  // LDS words reserved for CkState
constexpr int kNbBatch = 4;   // 64-slot adjacency chunks loaded together
static_assert(sizeof(CkState) <= 4 * kCkWords, "checkpoint state size");

// LDS word offset of the checkpoint state: after pool, staging and visited set
__host__ __device__ inline int ck_offset(int L, int scap, int vis_words)
{
    return (2 * L + 2 * scap + vis_words + 3) & ~3;
}

// LDS word offset of the query row copy (widths with Shape<DP>::QL): after
// the checkpoint state when there is one; DP words
__host__ __device__ inline int q_offset(int L, int scap, int vis_words, bool ck)
{
    return ck_offset(L, scap, vis_words) + (ck ? kCkWords : 0);
}

// LDS words a search of padded width dp needs beyond the checkpoint state
__host__ __device__ inline int query_lds_words(int dp)
{
    return dp >= kQueryLdsMinDp ? dp : 0;
}

// One query's inputs and outputs.  The query vector has d floats; `seeds`
// holds n_seed entry-sample positions (-1 padded) in global memory or LDS.
struct QueryIO {
    const float *q;
    // nullable: the query row already in this wave's LDS, zero-padded to the
    // padded width (else it is copied there when the width reads it from LDS)
    const float *qlds;
    uint32_t qword, qmask;
    const int32_t *seeds;
    int n_seed;
    int32_t *oid;     // [k]
    float *od;        // [k]
    uint32_t *cnt;    // [2] NDC, hops (nullable)
    int64_t trace_row;
    const uint16_t *mlp;  // stop network weights (device layout; LDS or global)
};

__device__ __forceinline__ void pack_query_attrs(const uint8_t *qa, int m, int b, uint32_t &qword,
                                                 uint32_t &qmask)
{
    attr_pack_query(qa, m, b, qword, qmask);
}

// The search of one query by one wave (Alg. 2 in beam form), LDS at smem:
// pool keys [L], pool words [L], staged keys [scap], staged words [scap],
// visited set [vis_words], checkpoint state [kCkWords] at ck_offset (CK),
// then for widths of 512 and more the query row [DP] at q_offset unless
// io.qlds already holds it.
template <int DP, int ST, bool CK>
__device__ void search_one(const SearchArgs &a, const QueryIO &io, uint32_t *smem)
{
    using S = Shape<DP>;
    constexpr int RBS = CK ? S::RB : Lay<DP, ST>::RB;
    const int lane = threadIdx.x & 63;
    const int L = a.L;
    float *pkey = reinterpret_cast<float *>(smem);
    uint32_t *pid = smem + L;
    float *skey = reinterpret_cast<float *>(smem + 2 * L);
    uint32_t *sid = smem + 2 * L + a.scap;
    uint32_t *vis = smem + 2 * L + 2 * a.scap;
    CkState *cks = reinterpret_cast<CkState *>(
        __builtin_assume_aligned(smem + ck_offset(L, a.scap, a.vis_words), 16));
    const bool bitset = a.use_bitset != 0;
    const int g = lane % S::G;

    // query slice in registers, or the query row in LDS (wide rows);
    // query attributes packed like the objects'
    constexpr int K4 = Lay<DP, ST>::K4;
    float4 qreg[S::QL ? 1 : S::NCH];
    const lds_f32x4 *qrow = nullptr;
    if constexpr (S::QL) {
        const float *src = io.qlds;
        if (src == nullptr) {
            float *dst = reinterpret_cast<float *>(smem + q_offset(L, a.scap, a.vis_words, CK));
            for (int c = lane; c < DP; c += 64)
                dst[c] = c < a.d ? io.q[c] : 0.0f;
            src = dst;
        }
        qrow = (const lds_f32x4 *)src;
    } else {
        const float *qp = io.q;
#pragma unroll
        for (int c = 0; c < S::NCH; ++c) {
            const int e = 4 * lane_chunk<DP, K4>(g, c);
            qreg[c].x = e + 0 < a.d ? qp[e + 0] : 0.0f;
            qreg[c].y = e + 1 < a.d ? qp[e + 1] : 0.0f;
            qreg[c].z = e + 2 < a.d ? qp[e + 2] : 0.0f;
            qreg[c].w = e + 3 < a.d ? qp[e + 3] : 0.0f;
        }
    }
    const QSrc<DP, K4, S::QL> qv{qreg, qrow};
    const uint32_t qword = io.qword, qmask = io.qmask;
    const int mq = __popc(qmask) / a.abits;
    if (CK && a.ckpt > 0) {
        float logsel = 0.0f;
        const uint32_t fm = (1u << a.abits) - 1u;
        for (int i = 0; i < a.m; ++i)
            if ((qmask >> (a.abits * i)) & fm)
                logsel += a.logp[i * 256 + ((qword >> (a.abits * i)) & fm)];
        if (lane == 0) {
            cks->logsel = logsel;
            cks->key_kth_first = 0.0f;
            cks->prev_hash = 0;
            cks->last_change = 0;
            cks->ntrace = 0;
            cks->have_first = 0;
            cks->have_prev = 0;
            cks->first_ckpt = 1;
        }
    }
    for (int i = lane; i < a.vis_words; i += 64)
        vis[i] = bitset ? 0u : kEmpty;
    wsync();

    // ---- seed set: the n_init best members of the entry sample, re-scored
    // exactly from the candidates the dense ranking kept
    int size = 0, lo = 0;
    const int cap0 = min(a.n_init, L);
    for (int e0 = 0; e0 < io.n_seed; e0 += 64) {
        const int e = e0 + lane;
        const int32_t pos = e < io.n_seed ? io.seeds[e] : -1;
        const int32_t v = (pos >= 0 && pos < a.n_entry) ? a.entry[pos] : -1;
        const bool ok = v >= 0 && v < a.n;
        const uint64_t vb = __ballot(ok);
        const int ne = __popcll(vb);
        if (ok)
            sid[lanes_below(vb)] = (uint32_t)v;
        wsync();
        score_batch<DP, ST, K4, RBS>(a.vecs, a.scale, qv, sid, skey, ne, mq, 1, a.w, a.attr, qword,
                                                 qmask, a.hmask);
        wsync();
        if (a.w.mode != NHQ_WEIGHTS_DEFAULT)
            weigh_keys(skey, sid, ne, mq, a.w);
        const float ck = lane < ne ? skey[lane] : 0.0f;
        const uint32_t cw = lane < ne ? sid[lane] : 0u;
        size = pool_merge(pkey, pid, size, cap0, ck, cw, lane < ne, lo);
    }
    for (int e = lane; e < size; e += 64) {
        bool unrec;
        visit(vis, bitset, a.hash_log2, pid[e] & kIdMask, unrec);
    }
    wsync();
    lo = 0;

    // ---- expansion loop
    uint32_t ndc = 0, hops = 0;
    bool capped = false, badid = false;
    // checkpoint state (the rest is in LDS)
    int ins_window = 0;
    float budget = 3.0e38f;  // learned hop budget
    int Lq = L;              // pool capacity (learned mode 3 lowers it)
    // E = 1: the adjacency row of the runner-up is fetched one hop ahead (it
    // is the next vertex to expand unless this hop inserts a better one)
    const int E = a.expand;
    const int rshift = (a.R & (a.R - 1)) == 0 ? __ffs(a.R) - 1 : -1;  // R a power of two
    // two-stage routing (Sec. 4.2): stage S1 until a step inserts nothing
    const int route_h = a.route_h;
    bool s1 = route_h > 1;
    int64_t pf_id = -1;
    int pf_nb = -1;
    uint32_t next_ckpt = (uint32_t)a.ckpt;
    for (;;) {
        // ---- the E best unexpanded entries (one more, unexpanded, when E = 1)
        const int want_sel = E == 1 ? 2 : E;
        int nsel = 0, mysel = -1;
        for (int base = lo; base < size && nsel < want_sel; base += 64) {
            const int e = base + lane;
            const bool un = e < size && (pid[e] & kExpBit) == 0;
            uint64_t bb = __ballot(un);
            while (bb && nsel < want_sel) {
                const int pos = base + __ffsll((unsigned long long)bb) - 1;
                bb &= bb - 1;
                if (lane == nsel)
                    mysel = pos;
                nsel += 1;
            }
        }
        if (nsel == 0)
            break;
        const int cur = rdl_i(mysel, 0);
        if (CK && a.ckpt > 0 && hops >= next_ckpt) {
            while (next_ckpt <= hops)
                next_ckpt += (uint32_t)a.ckpt;
            // ---- checkpoint: search-state features (see the stop network);
            // lane i computes feature i
            int fk;
            uint32_t h;
            float kth;
            bool has_kth;
            eligible_topk(pkey, pid, size, a.k, a.out_mode, fk, h, kth, has_kth);
            int last_change = cks->last_change;
            if (cks->have_prev && h != cks->prev_hash)
                last_change = (int)hops;
            float kfirst = cks->key_kth_first;
            const bool have_first = cks->have_first || has_kth;
            if (has_kth && !cks->have_first)
                kfirst = kth;
            const float front = pkey[cur];
            float arg = 1.0f;
            if (lane == 0)
                arg = 1.0f + (float)hops;
            else if (lane == 1)
                arg = 1.0f + (float)ndc;
            else if (lane == 4)
                arg = fmaxf(kth, 1e-30f) / fmaxf(kfirst, 1e-30f);
            else if (lane == 5)
                arg = fmaxf(front, 1e-30f) / fmaxf(kth, 1e-30f);
            const float lg = logf(arg);
            float myf;
            switch (lane) {
            case 0:
            case 1:
                myf = lg * 0.125f;
                break;
            case 2:
                myf = cks->logsel * 0.125f;
                break;
            case 3:
                myf = (float)fk / (float)a.k;
                break;
            case 4:
                myf = has_kth ? lg : 1.0f;
                break;
            case 5:
                myf = has_kth ? lg : -1.0f;
                break;
            case 6:
                myf = (float)ins_window / (float)(a.ckpt * a.R);
                break;
            default:
                myf = fminf((float)((int)hops - last_change) / 64.0f, 1.0f);
                break;
            }
            ins_window = 0;
            const int ntrace = cks->ntrace;
            const bool first_ckpt = cks->first_ckpt != 0;
            wsync();
            if (lane < 8)
                cks->f[lane] = myf;
            if (a.trace_feat && ntrace < a.trace_cap) {
                const int64_t t = io.trace_row * a.trace_cap + ntrace;
                if (lane < 8)
                    a.trace_feat[t * 8 + lane] = myf;
                if (lane == 0) {
                    a.trace_hop[t] = hops;
                    a.trace_hash[t] = h;
                }
            }
            if (lane == 0) {
                cks->last_change = last_change;
                cks->prev_hash = h;
                cks->have_prev = 1;
                cks->key_kth_first = kfirst;
                cks->have_first = have_first ? 1 : 0;
                cks->first_ckpt = 0;
                if (a.trace_feat && ntrace < a.trace_cap)
                    cks->ntrace = ntrace + 1;
            }
            wsync();
            if (a.learned == 3) {
                // the beam-width predictor: the first checkpoint's beam
                // output sets the pool size ceil(cap_factor 2^z1), clamped to
                // [k, L], for the rest of the search; the pool keeps its best
                // entries and the step's selection is made again
                float z0, z1;
                mlp_infer(io.mlp, cks->f, cks->h1, z0, z1);
                next_ckpt = 0xFFFFFFFFu;
                if (first_ckpt) {
                    const float want = ceilf(a.cap_factor * exp2f(z1));
                    const int lp = !(want < (float)Lq) ? Lq : (want < (float)a.k ? a.k : (int)want);
                    if (lp < Lq) {
                        Lq = lp;
                        size = min(size, Lq);
                        lo = min(lo, size);
                        continue;
                    }
                }
            } else if (a.learned) {
                float z0, z1;
                mlp_infer(io.mlp, cks->f, cks->h1, z0, z1);
                if (a.cap_factor > 0.0f && first_ckpt)
                    budget = a.cap_factor * exp2f(z1);
                if (z0 >= a.stop_logit)
                    break;
                if (a.learned == 2)  // one checkpoint: its budget bounds the rest
                    next_ckpt = 0xFFFFFFFFu;
            }
        }
        if (CK && a.learned && (float)hops >= budget)
            break;
        if ((int)hops >= a.max_hops) {
            capped = true;
            break;
        }
        const int nexp = min(min(nsel, E), a.max_hops - (int)hops);
        // mark the selected entries expanded; lane e holds the e-th vertex id
        uint32_t myid = 0;
        if (lane < nexp) {
            const uint32_t w = pid[mysel];
            myid = w & kIdMask;
        }
        wsync();
        if (lane < nexp)
            pid[mysel] = pid[mysel] | kExpBit;
        lo = rdl_i(mysel, nexp - 1) + 1;
        hops += (uint32_t)nexp;
        // ---- unvisited neighbours of the expanded vertices, in (vertex, slot)
        // order.  With several vertices per step the adjacency words of up to
        // kNbBatch 64-slot chunks are loaded before any is examined, so the
        // step waits for one round trip, not one per chunk.
        const int total = nexp * a.R;
        int nf = 0;
        const int64_t u0 = (int64_t)rdl_u(myid, 0);
        auto load_slot = [&](int sl) -> int {
            int qv_;
            if (rshift >= 0)
                qv_ = sl >> rshift;
            else
                qv_ = sl / a.R;
            const int e = min(qv_, nexp - 1), r = sl - qv_ * a.R;
            const int64_t u = (int64_t)(uint32_t)__shfl((int)myid, e, 64);
            bool take = sl < total;
            if (s1 && take) {
                // S1: slot r of the e-th vertex of this step, expansion number t
                const uint32_t t = hops - (uint32_t)nexp + (uint32_t)e;
                const uint32_t off = fmix32((uint32_t)u * 0x9E3779B1u + t) % (uint32_t)route_h;
                take = ((uint32_t)r + off) % (uint32_t)route_h == 0;
            }
            if (!take)
                return -1;
            return (E == 1 && pf_id == u0) ? pf_nb : a.adj[u * a.R + r];
        };
        auto take_fresh = [&](int nb, int s0) {
            if (nb >= a.n || nb < -1) {
                badid = true;
                nb = -1;
            }
            bool fresh = false, unrec = false;
            if (nb >= 0)
                fresh = visit(vis, bitset, a.hash_log2, (uint32_t)nb, unrec);
            // a vertex the hash could not record may repeat in this step
            uint64_t ub = __ballot(unrec);
            if (ub) {
                for (uint64_t b = ub; b; b &= b - 1) {
                    const int i = __ffsll((unsigned long long)b) - 1;
                    if (unrec && lane > i && nb == rdl_i(nb, i))
                        fresh = false;
                }
                if (s0 > 0)
                    for (int i = 0; i < nf; ++i)
                        if (unrec && (uint32_t)nb == sid[i])
                            fresh = false;
            }
            const uint64_t fb = __ballot(fresh);
            if (fresh)
                sid[nf + lanes_below(fb)] = (uint32_t)nb;
            nf += __popcll(fb);
        };
        if (total <= 64) {
            take_fresh(load_slot(lane), 0);
        } else {
            for (int sb = 0; sb < total; sb += 64 * kNbBatch) {
                int nbv[kNbBatch];
#pragma unroll
                for (int c = 0; c < kNbBatch; ++c)
                    nbv[c] = sb + 64 * c < total ? load_slot(sb + 64 * c + lane) : -1;
#pragma unroll
                for (int c = 0; c < kNbBatch; ++c)
                    if (sb + 64 * c < total)
                        take_fresh(nbv[c], sb + 64 * c);
            }
        }
        if (E == 1) {
            pf_id = -1;
            if (nsel > 1) {
                pf_id = pid[rdl_i(mysel, 1)] & kIdMask;
                pf_nb = lane < a.R ? a.adj[pf_id * a.R + lane] : -1;
            }
        }
        if (nf == 0) {
            if (s1) {
                // nothing to insert: stage S2 from here on, every pool entry
                // to be expanded again with all of its neighbours
                s1 = false;
                for (int e = lane; e < size; e += 64)
                    pid[e] &= ~kExpBit;
                wsync();
                lo = 0;
            }
            continue;
        }
        wsync();
        ndc += nf;
        score_batch<DP, ST, K4, RBS>(a.vecs, a.scale, qv, sid, skey, nf, mq, 1, a.w, a.attr, qword,
                                                 qmask, a.hmask);
        wsync();
        if (a.w.mode != NHQ_WEIGHTS_DEFAULT)
            weigh_keys(skey, sid, nf, mq, a.w);
        int step_ins = 0;
        for (int c0 = 0; c0 < nf; c0 += 64) {
            const int j = c0 + lane;
            const bool v = j < nf;
            const float ck = v ? skey[j] : 0.0f;
            const uint32_t cw = v ? sid[j] : 0u;
            int ins = 0;
            bool mine = false;
            size = pool_merge(pkey, pid, size, Lq, ck, cw, v, lo, &ins, &mine);
            // several chunks: mark the staged entries that entered the pool
            // (bit 31 of a staged word is free) for the count below
            if (CK && nf > 64 && mine)
                sid[j] = cw | kExpBit;
            step_ins += ins;
        }
        if (CK) {
            // entries that joined in this step: still pooled once all of its
            // neighbours were offered.  With one chunk that is every insertion;
            // with several, an entry admitted by an early chunk may have been
            // pushed out by a later one.  An admitted entry is still pooled iff
            // it is no worse, by (key, id), than the final pool's worst entry
            // (the worst of a full pool only improves).
            int joined = step_ins;
            if (nf > 64) {
                wsync();
                const bool full = size >= Lq;
                const float wk = pkey[size - 1];
                const uint32_t wm = pid[size - 1] & kIdMask;
                int cnt = 0;
                for (int j = lane; j < nf; j += 64) {
                    const uint32_t sw = sid[j];
                    if (sw & kExpBit)
                        cnt += (!full || !lt_key(wk, wm, skey[j], sw & kIdMask)) ? 1 : 0;
                }
                joined = (int)wave_sum_u32((uint32_t)cnt);
            }
            ins_window += joined;
        }
        if (s1 && step_ins == 0) {
            s1 = false;
            for (int e = lane; e < size; e += 64)
                pid[e] &= ~kExpBit;
            wsync();
            lo = 0;
        }
    }
    if (CK && a.trace_feat) {
        int fk;
        uint32_t h;
        float kth;
        bool has_kth;
        eligible_topk(pkey, pid, size, a.k, a.out_mode, fk, h, kth, has_kth);
        if (lane == 0) {
            a.final_hash[io.trace_row] = h;
            a.trace_count[io.trace_row] = cks->ntrace;
        }
    }

    // ---- output: eligible entries in pool order (Def. 4 filter or raw)
    const int want = a.rerank_n > 0 ? a.rerank_n : a.k;
    int got = 0;
    for (int base = 0; base < size && got < want; base += 64) {
        const int e = base + lane;
        const uint32_t w = e < size ? pid[e] : 0u;
        const bool el = e < size && (a.out_mode == 1 || ((w >> kChiShift) & kChiMask) == 0);
        const uint64_t bb = __ballot(el);
        const int pos = got + lanes_below(bb);
        if (el && pos < want)
            sid[pos] = w & ~kExpBit;
        got += __popcll(bb);
    }
    got = min(got, want);
    wsync();
    // delta^2 from the float32 copy (identical to the loop's for fp32 storage)
    score_batch<DP, NHQ_STORAGE_FP32, K4, Lay<DP, NHQ_STORAGE_FP32>::RB>(a.vec32, nullptr, qv, sid, skey, got, mq,
                                                                        2, a.w);
    wsync();
    // final order into LDS (the pool is no longer needed), then one store
    // per output slot
    for (int j0 = 0; j0 < got; j0 += 64) {
        const int j = j0 + lane;
        if (j < got) {
            const uint32_t w = sid[j];
            const int c = (int)((w >> kChiShift) & kChiMask);
            const float d2 = skey[j];
            int slot = j;
            if (a.rerank_n > 0) {
                // rank by exact (key, id) among the re-scored entries
                const float kj = w_key32(d2, c, mq, a.w);
                const uint32_t ij = w & kIdMask;
                slot = 0;
                for (int i = 0; i < got; ++i) {
                    const uint32_t wi = sid[i];
                    const float ki = w_key32(skey[i], (int)((wi >> kChiShift) & kChiMask), mq, a.w);
                    slot += lt_key(ki, wi & kIdMask, kj, ij) ? 1 : 0;
                }
            }
            if (slot < a.k) {
                const float dl = sqrtf(d2);
                pid[slot] = w & kIdMask;
                pkey[slot] = w_gamma32(dl, c, mq, a.w);
            }
        }
    }
    wsync();
    const int nout = min(got, a.k);
    int32_t *oid = io.oid;
    float *od = io.od;
    for (int j0 = 0; j0 < a.k; j0 += 64) {
        const int j = j0 + lane;
        if (j < a.k) {
            oid[j] = j < nout ? (int32_t)pid[j] : -1;
            od[j] = j < nout ? pkey[j] : __int_as_float(0x7F800000);
        }
    }
    if (lane == 0) {
        if (io.cnt) {
            io.cnt[0] = ndc;
            io.cnt[1] = hops;
        }
        if (capped)
            atomicOr(a.err, NHQ_DEVERR_HOPCAP);
    }
    if (badid && a.err)
        atomicOr(a.err, NHQ_DEVERR_BADID);
}

}  // namespace
}  // namespace nhq
