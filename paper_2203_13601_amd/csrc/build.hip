// Composite-index build on the GPU and exact hybrid k-NN (placeholders until
// the dense kernels land).
#include "nhq_internal.h"

using namespace nhq;

extern "C" {

int nhq_index_build_graph(nhq_index *h, void *stream)
{
    (void)h;
    (void)stream;
    return fail(NHQ_ENOTSUP, "GPU graph build not available in this build");
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
    (void)h; (void)queries; (void)qattrs; (void)nq; (void)k; (void)ids; (void)dists; (void)stream;
    return fail(NHQ_ENOTSUP, "exact k-NN not available in this build");
}

}  // extern "C"
