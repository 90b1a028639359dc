// Candidate lists of NPG_kgraph (Sec. 4.3) by NN-descent on the GPU: random
// lists refined through the neighbours of neighbours, in synchronous rounds
// (round t reads only the lists of round t - 1, so the result does not
// depend on scheduling).  One wavefront per vertex:
//   round 0   C(i) = the first l distinct values v != i of splitmix64 with
//             state seed ^ (i * 0xD1B54A32D192ED03), taken mod n, ordered by
//             (key, id); every entry new;
//   round t   J = the first s new entries of C(i); the candidates are the
//             ids of C(j), j in J, that are neither i nor in C(i), each
//             once (an LDS hash); C(i) becomes the l best of C(i) and the
//             candidates by (key, id); candidates enter new, J turns old.
// Keys are the object-object fusion keys of the index's weight setting over
// all m attributes, in float32 from the float32 rows (the search's scoring).
// Lists live in HBM as float keys [n][l] and words [n][l]: id in the low 28
// bits, bit 31 set once the entry has been explored ("old").
#include <algorithm>
#include <vector>

#include "search_core.h"

namespace nhq {
namespace {

struct NndArgs {
    const float *vec32;
    const uint32_t *attr;
    int64_t n;
    int d, m, l, s;
    const float *prev_key;
    const uint32_t *prev_word;
    float *next_key;
    uint32_t *next_word;
    unsigned long long *updates;  // entries that entered this round (summed)
    uint64_t seed;
    int init;       // 1: round 0 (random start)
    int hash_log2;  // visited hash: 2^hash_log2 slots
    Weights w;
    int abits;        // attribute field width
    uint32_t hmask;   // high bit of every attribute field
};

// LDS words of one wave: pool keys and words [l], the previous list's ids [l],
// the staging keys and words [64], the visited hash
__host__ __device__ inline int nnd_lds_words(int l, int hash_log2)
{
    return 3 * l + 2 * 64 + (1 << hash_log2);
}

template <int DP>
__global__ __launch_bounds__(64) void k_nnd_round(const NndArgs a)
{
    using S = Shape<DP>;
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x;
    if (i >= a.n)
        return;
    const int l = a.l;
    extern __shared__ __align__(16) uint32_t smem[];
    float *pkey = reinterpret_cast<float *>(smem);
    uint32_t *pid = smem + l;
    uint32_t *prev = smem + 2 * l;
    float *skey = reinterpret_cast<float *>(smem + 3 * l);
    uint32_t *sid = smem + 3 * l + 64;
    uint32_t *vis = smem + 3 * l + 128;
    const int g = lane % S::G;

    // the vertex's own row and attributes play the query
    float4 qv[S::NCH];
    const float *qp = a.vec32 + i * DP;
#pragma unroll
    for (int c = 0; c < S::NCH; ++c)
        qv[c] = *reinterpret_cast<const float4 *>(qp + 4 * (g + S::G * c));
    const QSrc<DP, 1, false> qsrc{qv, nullptr};
    const uint32_t qword = a.attr[i];
    const uint32_t qmask = attr_full_mask(a.m, a.abits);
    const int mq = a.m;
    for (int e = lane; e < (1 << a.hash_log2); e += 64)
        vis[e] = kEmpty;
    wsync();
    bool unrec;
    if (lane == 0)
        visit(vis, false, a.hash_log2, (uint32_t)i, unrec);
    wsync();

    int size = 0, lo = 0;
    // score staged ids sid[0..nf) and merge them into the pool
    auto score_merge = [&](int nf) {
        wsync();
        score_batch<DP, NHQ_STORAGE_FP32, 1, Lay<DP, NHQ_STORAGE_FP32>::RB>(a.vec32, nullptr, qsrc, sid, skey, nf, mq,
                                                                            1, a.w, a.attr, qword, qmask, a.hmask);
        wsync();
        if (a.w.mode != NHQ_WEIGHTS_DEFAULT)
            weigh_keys(skey, sid, nf, mq, a.w);
        const bool v = lane < nf;
        const float ck = v ? skey[lane] : 0.0f;
        const uint32_t cw = v ? (sid[lane] & kIdMask) : 0u;
        size = pool_merge(pkey, pid, size, l, ck, cw, v, lo);
    };

    if (a.init) {
        if (lane == 0) {
            uint64_t st = a.seed ^ ((uint64_t)i * 0xD1B54A32D192ED03ull);
            int got = 0;
            while (got < l) {
                const uint32_t v = (uint32_t)(splitmix64_next(st) % (uint64_t)a.n);
                bool dup = (int64_t)v == i;
                for (int t = 0; t < got && !dup; ++t)
                    dup = prev[t] == v;
                if (!dup)
                    prev[got++] = v;
            }
        }
        wsync();
        for (int c0 = 0; c0 < l; c0 += 64) {
            const int nf = min(64, l - c0);
            if (lane < nf)
                sid[lane] = prev[c0 + lane];
            score_merge(nf);
        }
    } else {
        const int64_t base = i * l;
        for (int e = lane; e < l; e += 64) {
            pkey[e] = a.prev_key[base + e];
            const uint32_t w = a.prev_word[base + e];
            pid[e] = w;
            prev[e] = w & kIdMask;
        }
        size = l;
        wsync();
        for (int e = lane; e < l; e += 64)
            visit(vis, false, a.hash_log2, prev[e], unrec);
        wsync();
        // J: the first s new entries, in list order; they turn old
        int nj = 0, myj = -1;
        for (int b0 = 0; b0 < l && nj < a.s; b0 += 64) {
            const int e = b0 + lane;
            uint64_t bb = __ballot(e < l && (pid[e] & kExpBit) == 0);
            while (bb && nj < a.s) {
                const int pos = b0 + __ffsll((unsigned long long)bb) - 1;
                bb &= bb - 1;
                if (lane == nj)
                    myj = pos;
                nj += 1;
            }
        }
        uint32_t jid = 0;
        if (lane < nj)
            jid = pid[myj] & kIdMask;
        wsync();
        if (lane < nj)
            pid[myj] |= kExpBit;
        wsync();
        for (int e = 0; e < nj; ++e) {
            const int64_t j = (int64_t)rdl_u(jid, e);
            for (int c0 = 0; c0 < l; c0 += 64) {
                const int t = c0 + lane;
                uint32_t v = 0;
                bool fresh = false;
                unrec = false;
                if (t < l) {
                    v = a.prev_word[j * l + t] & kIdMask;
                    fresh = (int64_t)v < a.n && visit(vis, false, a.hash_log2, v, unrec);
                }
                // a vertex the hash could not record may repeat in this batch
                const uint64_t ub = __ballot(unrec);
                for (uint64_t b = ub; b; b &= b - 1) {
                    const int k = __ffsll((unsigned long long)b) - 1;
                    if (unrec && lane > k && v == rdl_u(v, k))
                        fresh = false;
                }
                const uint64_t fb = __ballot(fresh);
                if (fresh)
                    sid[lanes_below(fb)] = v;
                const int nf = __popcll(fb);
                if (nf > 0)
                    score_merge(nf);
            }
        }
    }
    // the new list, and how many of its entries were not in the old one
    int fresh_out = 0;
    for (int e = lane; e < l; e += 64) {
        const uint32_t w = pid[e];
        a.next_key[i * l + e] = pkey[e];
        a.next_word[i * l + e] = w;
        bool in_prev = false;
        if (!a.init)
            for (int t = 0; t < l && !in_prev; ++t)
                in_prev = prev[t] == (w & kIdMask);
        fresh_out += in_prev ? 0 : 1;
    }
    for (int o = 32; o > 0; o >>= 1)
        fresh_out += __shfl_xor(fresh_out, o, 64);
    if (lane == 0 && !a.init)
        atomicAdd(a.updates, (unsigned long long)fresh_out);
}

__global__ void k_words_to_ids(const uint32_t *w, int32_t *ids, int64_t total)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < total)
        ids[e] = (int32_t)(w[e] & kIdMask);
}

template <int DP>
int launch_round(const NndArgs &a, hipStream_t st)
{
    const size_t lds = sizeof(uint32_t) * (size_t)nnd_lds_words(a.l, a.hash_log2);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_nnd_round<DP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(NHQ_EHIP, "hipFuncSetAttribute failed");
    }
    hipLaunchKernelGGL(k_nnd_round<DP>, dim3((unsigned)a.n), dim3(64), lds, st, a);
    return hipGetLastError() == hipSuccess ? NHQ_OK : fail(NHQ_EHIP, "NN-descent launch failed");
}

}  // namespace

// NN-descent lists of every vertex: `rounds` rounds after the random start,
// or fewer when a round brings fewer than stop_frac * n * l new entries
// (stop_frac <= 0: always `rounds`).  ids: device [n][l].  updates_host
// (nullable, [rounds]) receives each round's count; *rounds_run the rounds
// done.  Synchronises the stream once per round.
int nnd_lists(const Index *ix, int l, int s, int rounds, double stop_frac, uint64_t seed,
              int32_t *ids, int64_t *updates_host, int *rounds_run, hipStream_t st)
{
    const int64_t n = ix->n;
    if (l < 1 || l > 128 || n <= l)
        return fail(NHQ_EINVAL, "NN-descent needs 1 <= l <= 128 and n > l");
    if (s < 0 || s > 64 || rounds < 0 || rounds > 1000)
        return fail(NHQ_EINVAL, "NN-descent needs 0 <= s <= 64 and 0 <= rounds <= 1000");
    int hb = 8;
    while (hb < 13 && (1 << hb) < 2 * (1 + l + s * l))
        ++hb;
    NndArgs a{};
    a.vec32 = ix->vec32;
    a.attr = ix->attr;
    a.n = n;
    a.d = ix->d;
    a.m = ix->m;
    a.l = l;
    a.s = s;
    a.seed = seed;
    a.hash_log2 = hb;
    a.w = ix->w;
    a.abits = ix->abits;
    a.hmask = ix->hmask;
    const size_t cells = (size_t)n * l;
    char *blk = nullptr;
    const size_t bytes = 4 * cells * sizeof(uint32_t) + 256;
    NHQ_HIP(hipMallocAsync((void **)&blk, bytes, st));
    float *k0 = reinterpret_cast<float *>(blk);
    uint32_t *w0 = reinterpret_cast<uint32_t *>(k0 + cells);
    float *k1 = reinterpret_cast<float *>(w0 + cells);
    uint32_t *w1 = reinterpret_cast<uint32_t *>(k1 + cells);
    unsigned long long *upd = reinterpret_cast<unsigned long long *>(
        (reinterpret_cast<uintptr_t>(w1 + cells) + 15) & ~uintptr_t(15));
    int rc = NHQ_OK;
    auto launch = [&](const NndArgs &aa) {
        switch (ix->dp) {
        case 32: return launch_round<32>(aa, st);
        case 64: return launch_round<64>(aa, st);
        case 96: return launch_round<96>(aa, st);
        case 128: return launch_round<128>(aa, st);
        case 256: return launch_round<256>(aa, st);
        case 512: return launch_round<512>(aa, st);
        case 960: return launch_round<960>(aa, st);
        case 1024: return launch_round<1024>(aa, st);
        default: return fail(NHQ_EINVAL, "unsupported padded dimension");
        }
    };
    a.init = 1;
    a.prev_key = nullptr;
    a.prev_word = nullptr;
    a.next_key = k0;
    a.next_word = w0;
    a.updates = upd;
    rc = launch(a);
    int done = 0;
    for (int r = 1; r <= rounds && rc == NHQ_OK; ++r) {
        if (hipMemsetAsync(upd, 0, sizeof(unsigned long long), st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "hipMemsetAsync failed");
            break;
        }
        a.init = 0;
        a.prev_key = (r & 1) ? k0 : k1;
        a.prev_word = (r & 1) ? w0 : w1;
        a.next_key = (r & 1) ? k1 : k0;
        a.next_word = (r & 1) ? w1 : w0;
        rc = launch(a);
        if (rc != NHQ_OK)
            break;
        unsigned long long u = 0;
        if (hipMemcpyAsync(&u, upd, sizeof(u), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "reading the update count failed");
            break;
        }
        if (updates_host)
            updates_host[r - 1] = (int64_t)u;
        done = r;
        if (stop_frac > 0.0 && (double)u < stop_frac * (double)cells)
            break;
    }
    if (rc == NHQ_OK) {
        const uint32_t *wf = (done & 1) ? w1 : w0;
        const unsigned blocks = (unsigned)((cells + 255) / 256);
        hipLaunchKernelGGL(k_words_to_ids, dim3(blocks), dim3(256), 0, st, wf, ids, (int64_t)cells);
        if (hipGetLastError() != hipSuccess)
            rc = fail(NHQ_EHIP, "list copy failed");
    }
    (void)hipFreeAsync(blk, st);
    if (rounds_run)
        *rounds_run = done;
    return rc;
}

}  // namespace nhq

using namespace nhq;

extern "C" int nhq_nndescent_lists(const nhq_index *h, int32_t l, int32_t s, int32_t rounds,
                                   double stop_frac, uint64_t seed, int32_t *ids,
                                   int64_t *updates, int32_t *rounds_run, void *stream)
{
    if (!h || !ids)
        return fail(NHQ_EINVAL, "null index or output");
    int done = 0;
    const int rc = nnd_lists(&h->impl, l, s, rounds, stop_frac, seed, ids, updates, &done,
                             (hipStream_t)stream);
    if (rounds_run)
        *rounds_run = done;
    return rc;
}
