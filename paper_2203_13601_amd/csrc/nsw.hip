// NPG_nsw (Sec. 4.3) by insertion in batches: vertices enter in id order,
// each batch as a set of queries.  The first batch takes the exact l nearest
// within itself (dense tiles, then the exact re-score of the selection).
// Every later batch [s, s + nb) searches the graph of the s vertices already
// in -- the joint-pruning search itself (Alg. 2, beam L, all of the
// object's attributes constrained, raw pool order), seeded by the 16 best of
// the first min(s, 256) distinct values of splitmix64(seed) mod s -- for its
// l candidates.  Each new row is then selected from its candidates
// (Sec. 4.1), and every vertex a new row names re-selects its own row with
// the new vertex offered, so links go both ways.  A batch sees only earlier
// vertices; batch size 1 is one-at-a-time insertion.
#include <algorithm>
#include <vector>

#include "nhq_internal.h"

namespace nhq {

constexpr int kNswMargin = 16;  // dense-tile candidates kept beyond l

// the codes of objects s .. s + nb - 1 from their packed words
__global__ void k_unpack_attr(const uint32_t *__restrict__ words, int64_t nb, int m, int b,
                              uint8_t *__restrict__ codes)
{
    const uint32_t fm = (1u << b) - 1u;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nb * m;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / m;
        const int j = (int)(t - e * m);
        codes[t] = (uint8_t)((words[e] >> (b * j)) & fm);
    }
}

// Offers of the rows [s, s + nb) to the vertices they name, grouped by
// target on the host, then the targets' re-selection on the device.
static int nsw_reverse(Index *ix, int64_t s, int64_t nb, hipStream_t st)
{
    const int R = ix->degree;
    std::vector<int32_t> rows((size_t)nb * R);
    NHQ_HIP(hipMemcpyAsync(rows.data(), ix->adj + s * R, sizeof(int32_t) * rows.size(),
                           hipMemcpyDeviceToHost, st));
    NHQ_HIP(hipStreamSynchronize(st));
    std::vector<std::pair<int32_t, int32_t>> offers;  // (target, offered vertex)
    offers.reserve(rows.size());
    for (int64_t e = 0; e < nb; ++e)
        for (int t = 0; t < R; ++t) {
            const int32_t j = rows[(size_t)e * R + t];
            if (j >= 0)
                offers.emplace_back(j, (int32_t)(s + e));
        }
    if (offers.empty())
        return NHQ_OK;
    std::sort(offers.begin(), offers.end());
    std::vector<int32_t> targets, inc;
    std::vector<int64_t> off;
    for (size_t k = 0; k < offers.size(); ++k) {
        if (k == 0 || offers[k].first != offers[k - 1].first) {
            targets.push_back(offers[k].first);
            off.push_back((int64_t)inc.size());
        }
        inc.push_back(offers[k].second);
    }
    off.push_back((int64_t)inc.size());
    const int64_t nt = (int64_t)targets.size();
    int32_t *d_t = nullptr, *d_inc = nullptr;
    int64_t *d_off = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&d_t, sizeof(int32_t) * (size_t)nt, st));
    NHQ_HIP(hipMallocAsync((void **)&d_inc, sizeof(int32_t) * inc.size(), st));
    NHQ_HIP(hipMallocAsync((void **)&d_off, sizeof(int64_t) * off.size(), st));
    NHQ_HIP(hipMemcpyAsync(d_t, targets.data(), sizeof(int32_t) * (size_t)nt, hipMemcpyHostToDevice, st));
    NHQ_HIP(hipMemcpyAsync(d_inc, inc.data(), sizeof(int32_t) * inc.size(), hipMemcpyHostToDevice, st));
    NHQ_HIP(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, st));
    const int rc = launch_reselect_targets(ix, ix->adj, d_t, nt, d_off, d_inc, st);
    (void)hipFreeAsync(d_t, st);
    (void)hipFreeAsync(d_inc, st);
    (void)hipFreeAsync(d_off, st);
    NHQ_HIP(hipStreamSynchronize(st));
    return rc;
}

int nsw_build(Index *ix, int l, int64_t B, int L, uint64_t seed, hipStream_t st)
{
    const int64_t n = ix->n;
    const int R = ix->degree;
    const int m = ix->m, dp = ix->dp;
    if (B < 1 || L < l || l < 1 || L > NHQ_MAX_BEAM)
        return fail(NHQ_EINVAL, "NSW build needs batch >= 1 and 1 <= l <= beam <= 1024");
    NHQ_HIP(hipMemsetAsync(ix->adj, 0xFF, sizeof(int32_t) * (size_t)n * R, st));
    // ---- the first batch: exact candidates within it
    const int64_t b0 = std::min(B, n);
    const int l0 = (int)std::min<int64_t>(l, b0 - 1);
    int rc = NHQ_OK;
    if (l0 > 0) {
        const int K = (int)std::min<int64_t>(std::min(l0 + kNswMargin, 160), b0 - 1);
        int32_t *cand = nullptr;
        NHQ_HIP(hipMallocAsync((void **)&cand, sizeof(int32_t) * (size_t)b0 * K, st));
        rc = launch_dense_topk(ix->vec32, ix->norm, ix->attr, nullptr, b0, ix->vec32, ix->norm,
                               ix->attr, b0, dp, m, ix->abits, 0, 1, K, cand, nullptr, st, &ix->w);
        if (rc == NHQ_OK)
            rc = launch_select_rows(ix, cand, K, l0, ix->adj, 0, b0, st);
        (void)hipFreeAsync(cand, st);
        if (rc == NHQ_OK)
            rc = nsw_reverse(ix, 0, b0, st);
    }
    if (rc != NHQ_OK || b0 == n)
        return rc;
    return nsw_insert(ix, b0, n, l, B, L, seed, st);
}

// Vertices s0 .. s1 - 1 (rows already in the index, no edges yet) enter the
// graph of the vertices below s0, in batches of B: each batch searches the
// graph built so far for its candidates, selects its rows, and every vertex a
// new row names re-selects its own row with the new vertex offered.
int nsw_insert(Index *ix, int64_t s0, int64_t s1, int l, int64_t B, int L, uint64_t seed,
               hipStream_t st)
{
    const int d = ix->d, m = ix->m, dp = ix->dp;
    if (s0 < 1 || s1 <= s0)
        return s1 == s0 ? NHQ_OK : fail(NHQ_EINVAL, "insertion needs a non-empty graph");
    if (B < 1 || L < l || l < 1 || L > NHQ_MAX_BEAM)
        return fail(NHQ_EINVAL, "insertion needs batch >= 1 and 1 <= l <= beam <= 1024");
    int rc = NHQ_OK;
    const int64_t bmax = std::min(B, s1 - s0);
    float *q = nullptr, *dist = nullptr;
    uint8_t *qa = nullptr;
    int32_t *cand = nullptr, *ent = nullptr, *pos = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&q, sizeof(float) * (size_t)bmax * d, st));
    NHQ_HIP(hipMallocAsync((void **)&qa, (size_t)bmax * std::max(m, 1), st));
    NHQ_HIP(hipMallocAsync((void **)&cand, sizeof(int32_t) * (size_t)bmax * l, st));
    NHQ_HIP(hipMallocAsync((void **)&dist, sizeof(float) * (size_t)bmax * l, st));
    NHQ_HIP(hipMallocAsync((void **)&ent, sizeof(int32_t) * 256, st));
    NHQ_HIP(hipMallocAsync((void **)&pos, sizeof(int32_t) * 256, st));
    std::vector<int32_t> hpos(256);
    for (int t = 0; t < 256; ++t)
        hpos[(size_t)t] = t;
    NHQ_HIP(hipMemcpyAsync(pos, hpos.data(), sizeof(int32_t) * 256, hipMemcpyHostToDevice, st));
    std::vector<int32_t> seeds;
    for (int64_t s = s0; s < s1 && rc == NHQ_OK; s += B) {
        const int64_t nb = std::min(B, s1 - s);
        // entry sample of the inserted vertices
        const int want = (int)std::min<int64_t>(s, 256);
        seeds.clear();
        uint64_t state = seed;
        while ((int)seeds.size() < want) {
            const int32_t v = (int32_t)(splitmix64_next(state) % (uint64_t)s);
            if (std::find(seeds.begin(), seeds.end(), v) == seeds.end())
                seeds.push_back(v);
        }
        if (hipMemcpyAsync(ent, seeds.data(), sizeof(int32_t) * (size_t)want, hipMemcpyHostToDevice,
                           st) != hipSuccess ||
            hipMemcpy2DAsync(q, sizeof(float) * d, ix->vec32 + s * dp, sizeof(float) * dp,
                             sizeof(float) * d, (size_t)nb, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "NSW batch staging failed");
            break;
        }
        if (m > 0) {
            const unsigned blocks = (unsigned)std::min<int64_t>(65536, (nb * m + 255) / 256);
            hipLaunchKernelGGL(k_unpack_attr, dim3(blocks), dim3(256), 0, st, ix->attr + s, nb, m,
                               ix->abits, qa);
        }
        SearchLaunch sl{};
        sl.ix = ix;
        sl.q = q;
        sl.qa = qa;
        sl.seed_cand = pos;
        sl.n_seed_cand = want;
        sl.seeds_shared = 1;
        sl.entry_override = ent;
        sl.n_entry_override = want;
        sl.nq = nb;
        sl.k = l;
        sl.L = L;
        sl.n_init = std::min(16, want);
        sl.out_mode = 1;
        sl.max_hops = 1 << 30;
        sl.expand = 1;
        sl.ids = cand;
        sl.dists = dist;
        sl.stream = st;
        rc = launch_search(sl);
        if (rc == NHQ_OK)
            rc = launch_select_rows(ix, cand, l, l, ix->adj, s, nb, st);
        if (rc == NHQ_OK)
            rc = nsw_reverse(ix, s, nb, st);
    }
    void *bufs[] = {q, qa, cand, dist, ent, pos};
    for (void *b : bufs)
        (void)hipFreeAsync(b, st);
    NHQ_HIP(hipStreamSynchronize(st));
    return rc;
}

}  // namespace nhq
