// Exact selection of the K smallest non-negative float keys by one
// wavefront: a bitwise radix select on the keys' bit patterns (which order
// like the values), ties broken by position.  Shared by the batch seed
// ranking and the serving loop's in-wave seed ranking.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nhq {
namespace {

// The K-th smallest bit pattern over T values per lane (one bit at a time
// from the top; counts by ballot).  Returns p with count(v <= p) >= K and
// count(v < p) < K, or -- when some prefix holds exactly K values -- the
// largest pattern under that prefix, so that count(v <= p) == K.
template <int T>
__device__ __forceinline__ uint32_t kth_pattern(const uint32_t (&v)[T], int K)
{
    uint32_t p = 0;
    int want = K;
    for (int b = 31; b >= 0; --b) {
        const uint32_t hi = ~((1u << b) - 1u);
        int cnt = 0;
#pragma unroll
        for (int t = 0; t < T; ++t)
            cnt += __popcll(__ballot((v[t] & hi) == p));
        if (cnt == want) {
            p |= (1u << b) - 1u;
            break;
        }
        if (cnt < want) {
            want -= cnt;
            p |= 1u << b;
        }
    }
    return p;
}

__device__ __forceinline__ int rank_below(uint64_t b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

// Write the K best by (pattern, order): every value below p, then values
// equal to p in order until K are written.  Element t of lane l is the
// (64 t + l)-th in order; its position is pos(t); positions >= ne are
// padding and become -1.
template <int T, typename Pos>
__device__ __forceinline__ void emit_best(const uint32_t (&v)[T], Pos pos, uint32_t p, int K, int ne,
                                          int32_t *__restrict__ out)
{
    int base = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const bool lt = v[t] < p;
        const uint64_t b = __ballot(lt);
        if (lt)
            out[base + rank_below(b)] = pos(t);
        base += __popcll(b);
    }
    int left = K - base;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const bool eq = v[t] == p && left > 0;
        const uint64_t b = __ballot(eq);
        const int r = rank_below(b);
        if (eq && r < left) {
            const int ps = pos(t);
            out[base + r] = ps < ne ? ps : -1;
        }
        const int took = min(left, __popcll(b));
        base += took;
        left -= took;
    }
}

// The K best of ne keys held in LDS as bit patterns kb[0..ne), by (key,
// position), into out[0..K) (positions; padding beyond ne becomes -1).  For
// K <= 64 the lane-minimum bound and a compaction into cv/cp (256 entries
// each, LDS) come first; otherwise, or when more than 256 keys fall under
// the bound, the radix passes run over the whole row in LDS.
__device__ inline void select_lds(const uint32_t *kb, int ne, int K, uint32_t *cv, int32_t *cp,
                                  int32_t *out)
{
    const int lane = threadIdx.x & 63;
    const int ntot = max((ne + 63) & ~63, (K + 63) & ~63);
    if (K <= 64) {
        uint32_t mn[1] = {0xFFFFFFFFu};
        for (int j = lane; j < ne; j += 64)
            mn[0] = min(mn[0], kb[j]);
        const uint32_t u = kth_pattern<1>(mn, K);
        int c = 0;
        for (int j0 = 0; j0 < ntot; j0 += 64) {
            const int j = j0 + lane;
            const uint32_t v = j < ne ? kb[j] : 0xFFFFFFFFu;
            c += __popcll(__ballot(v <= u));
        }
        if (c <= 256) {
            int base = 0;
            for (int j0 = 0; j0 < ntot; j0 += 64) {
                const int j = j0 + lane;
                const uint32_t v = j < ne ? kb[j] : 0xFFFFFFFFu;
                const bool in = v <= u;
                const uint64_t b = __ballot(in);
                if (in) {
                    const int r = base + rank_below(b);
                    cv[r] = v;
                    cp[r] = j;
                }
                base += __popcll(b);
            }
            for (int i = base + lane; i < 256; i += 64) {
                cv[i] = 0xFFFFFFFFu;
                cp[i] = -1;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            uint32_t w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                w[t] = cv[64 * t + lane];
            const uint32_t p = kth_pattern<4>(w, K);
            emit_best<4>(w, [&](int t) { return cp[64 * t + lane]; }, p, K, ne, out);
            return;
        }
    }
    uint32_t p = 0;
    int want = K;
    for (int b = 31; b >= 0; --b) {
        const uint32_t hi = ~((1u << b) - 1u);
        int cnt = 0;
        for (int j0 = 0; j0 < ntot; j0 += 64) {
            const int j = j0 + lane;
            const uint32_t v = j < ne ? kb[j] : 0xFFFFFFFFu;
            cnt += __popcll(__ballot((v & hi) == p));
        }
        if (cnt == want) {
            p |= (1u << b) - 1u;
            break;
        }
        if (cnt < want) {
            want -= cnt;
            p |= 1u << b;
        }
    }
    int base = 0;
    for (int j0 = 0; j0 < ntot; j0 += 64) {
        const int j = j0 + lane;
        const bool lt = (j < ne ? kb[j] : 0xFFFFFFFFu) < p;
        const uint64_t b = __ballot(lt);
        if (lt)
            out[base + rank_below(b)] = j;
        base += __popcll(b);
    }
    int left = K - base;
    for (int j0 = 0; j0 < ntot && left > 0; j0 += 64) {
        const int j = j0 + lane;
        const bool eq = (j < ne ? kb[j] : 0xFFFFFFFFu) == p;
        const uint64_t b = __ballot(eq);
        const int r = rank_below(b);
        if (eq && r < left)
            out[base + r] = j < ne ? j : -1;
        const int took = min(left, __popcll(b));
        base += took;
        left -= took;
    }
}

}  // namespace
}  // namespace nhq
