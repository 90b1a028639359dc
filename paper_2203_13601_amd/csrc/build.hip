// Composite-index build on the GPU (Alg. 1 in degree-bounded form, Sec. 4.1
// edge selection, fusion distance in the build per Sec. 5.1) and exact hybrid
// k-NN (Def. 4): orchestration of the dense top-K tiles, the exact re-score,
// the landing-zone selection and the reverse pass.
#include <algorithm>

#include "nhq_internal.h"

namespace nhq {

int launch_select(const Index *ix, const int32_t *cand, int K, int l, int32_t *adj, hipStream_t st);
int launch_reverse(const Index *ix, const int32_t *fwd, int32_t *adj, hipStream_t st);
int launch_refine(const Index *ix, const float *qpad, const int32_t *cand, int64_t nq, int K, int k,
                  int32_t *ids, float *dists, hipStream_t st);

// extra candidates the dense tiles keep beyond l (they rank by a GEMM-form
// key; the exact re-score then keeps the l best)
constexpr int kMargin = 16;

}  // namespace nhq

using namespace nhq;

extern "C" {

int nhq_index_build_graph(nhq_index *h, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    Index *ix = &h->impl;
    hipStream_t st = (hipStream_t)stream;
    if (ix->n < 2)
        return fail(NHQ_EINVAL, "a graph needs at least two objects");
    const int l = (int)std::min<int64_t>(ix->cand, ix->n - 1);
    if (ix->builder == NHQ_BUILD_NSW) {
        ix->nnd_rounds_run = 0;
        return nsw_build(ix, l, ix->nsw_batch, std::max(ix->nsw_beam, l), ix->seed, st);
    }
    const bool nnd = ix->builder == NHQ_BUILD_NNDESCENT && ix->n > l && l <= 128;
    // NN-descent lists hold l candidates; the dense tiles keep a margin more
    const int K = nnd ? l : (int)std::min<int64_t>(std::min(l + kMargin, 160), ix->n - 1);
    int32_t *cand = nullptr, *fwd = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&cand, sizeof(int32_t) * (size_t)ix->n * K, st));
    int rc = NHQ_OK;
    if (nnd) {
        int done = 0;
        rc = nnd_lists(ix, l, ix->nnd_sample, ix->nnd_rounds, ix->nnd_stop, ix->seed,
                       cand, nullptr, &done, st);
        ix->nnd_rounds_run = done;
    } else {
        rc = launch_dense_topk(ix->vec32, ix->norm, ix->attr, nullptr, ix->n, ix->vec32, ix->norm,
                               ix->attr, ix->n, ix->dp, ix->m, ix->abits, 0, 1, K, cand, nullptr, st,
                               &ix->w);
    }
    if (rc == NHQ_OK) {
        if (ix->reverse_edges) {
            if (hipMallocAsync((void **)&fwd, sizeof(int32_t) * (size_t)ix->n * ix->degree, st) != hipSuccess)
                rc = fail(NHQ_ENOMEM, "forward graph allocation failed");
            if (rc == NHQ_OK)
                rc = launch_select(ix, cand, K, l, fwd, st);
            if (rc == NHQ_OK)
                rc = launch_reverse(ix, fwd, ix->adj, st);
        } else {
            rc = launch_select(ix, cand, K, l, ix->adj, st);
        }
    }
    (void)hipFreeAsync(cand, st);
    if (fwd)
        (void)hipFreeAsync(fwd, st);
    return rc;
}

int nhq_index_build_report(const nhq_index *h, int32_t *nnd_rounds_run)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    if (nnd_rounds_run)
        *nnd_rounds_run = h->impl.nnd_rounds_run;
    return NHQ_OK;
}

int nhq_build_index(const float *vecs, const uint8_t *attrs, int64_t n, int32_t d, int32_t m,
                    const nhq_build_params *params, void *stream, nhq_index **out)
{
    int rc = nhq_index_create(vecs, attrs, n, d, m, params, stream, out);
    if (rc != NHQ_OK)
        return rc;
    rc = nhq_index_build_graph(*out, stream);
    if (rc != NHQ_OK) {
        nhq_index_free(*out);
        *out = nullptr;
    }
    return rc;
}

int nhq_bruteforce_hybrid_knn(const nhq_index *h, const float *queries, const uint8_t *qattrs,
                              int64_t nq, int32_t k, int32_t *ids, float *dists, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    const Index *ix = &h->impl;
    if (nq < 0 || k < 1 || k > 128)
        return fail(NHQ_EINVAL, "need nq >= 0 and 1 <= k <= 128");
    if (nq == 0)
        return NHQ_OK;
    if (!queries || !ids || !dists || (ix->m > 0 && !qattrs))
        return fail(NHQ_EINVAL, "null array argument");
    hipStream_t st = (hipStream_t)stream;
    const int K = (int)std::min<int64_t>(k + kMargin, std::max<int64_t>(1, ix->n));
    float *qpad = nullptr, *qnorm = nullptr;
    uint32_t *qw = nullptr, *qm = nullptr;
    int32_t *cand = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&qpad, sizeof(float) * (size_t)nq * ix->dp, st));
    NHQ_HIP(hipMallocAsync((void **)&qnorm, sizeof(float) * (size_t)nq, st));
    NHQ_HIP(hipMallocAsync((void **)&qw, sizeof(uint32_t) * (size_t)nq, st));
    NHQ_HIP(hipMallocAsync((void **)&qm, sizeof(uint32_t) * (size_t)nq, st));
    NHQ_HIP(hipMallocAsync((void **)&cand, sizeof(int32_t) * (size_t)nq * K, st));
    int rc = launch_pad_queries(queries, qattrs, nq, ix->d, ix->dp, ix->m, ix->abits, qpad, qnorm, qw, qm,
                                nullptr, nullptr, st);
    if (rc == NHQ_OK)
        rc = launch_dense_topk(qpad, qnorm, qw, qm, nq, ix->vec32, ix->norm, ix->attr, ix->n, ix->dp,
                               ix->m, ix->abits, 1, 0, K, cand, nullptr, st);
    if (rc == NHQ_OK)
        rc = launch_refine(ix, qpad, cand, nq, K, k, ids, dists, st);
    void *bufs[] = {qpad, qnorm, qw, qm, cand};
    for (void *b : bufs)
        (void)hipFreeAsync(b, st);
    return rc;
}

}  // extern "C"
