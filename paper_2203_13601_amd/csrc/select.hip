// Landing-zone edge selection (Sec. 4.1 steps (2)-(3), Def. 7) under the
// fusion distance between objects (Sec. 5.1), one wavefront per vertex.
//
// Input: K approximate candidates per vertex from the dense tiles.  The wave
// re-scores them exactly (float64 direct form of delta^2 from the float32
// rows, chi over all m codes), keeps the l best by (key, id) and then walks
// them in order: candidate p joins N(i) iff it is strictly closer to i than to
// every neighbour j already chosen (p lies in every landing zone L(i, j));
// the ball B(i, Gamma(i, j)) never needs a test because later candidates are
// at least as far from i.  At most R neighbours.
//
// The reverse pass re-selects every vertex j from N(j) united with the
// vertices that chose j (same rule, same order), which adds in-edges to
// vertices that no one selected.
#include <algorithm>
#include <vector>

#include "nhq_internal.h"

namespace nhq {
namespace {

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}


__device__ __forceinline__ bool lt64(double ka, uint32_t ia, double kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

template <int DP>
struct SShape {
    static constexpr int G = DP <= 512 ? 8 : 16;
    static constexpr int NG = 64 / G;
    static constexpr int NCH = DP / (4 * G);
};

// float64 key of `center` (row held in registers as qv) against ids[0..n):
// the fusion key of the weight setting w over m attributes (default:
// delta^2 * (m + chi)^2, and delta^2 when m = 0).
template <int DP>
__device__ void exact_keys(const float *vec32, const uint32_t *attr, uint32_t cattr,
                           uint32_t mask, uint32_t hmask, int m, const Weights &w,
                           const float4 (&qv)[SShape<DP>::NCH], const uint32_t *ids, double *out,
                           int n)
{
    using S = SShape<DP>;
    const int lane = threadIdx.x & 63;
    const int g = lane % S::G, gi = lane / S::G;
    for (int r0 = 0; r0 < n; r0 += S::NG) {
        const int j = r0 + gi;
        double acc0 = 0.0, acc1 = 0.0;
        uint32_t id = 0;
        if (j < n) {
            id = ids[j];
            const float4 *row = reinterpret_cast<const float4 *>(vec32 + (int64_t)id * DP);
#pragma unroll
            for (int c = 0; c < S::NCH; ++c) {
                const float4 x = row[g + S::G * c];
                const double t0 = (double)qv[c].x - (double)x.x;
                const double t1 = (double)qv[c].y - (double)x.y;
                const double t2 = (double)qv[c].z - (double)x.z;
                const double t3 = (double)qv[c].w - (double)x.w;
                acc0 = fma(t0, t0, acc0);
                acc1 = fma(t1, t1, acc1);
                acc0 = fma(t2, t2, acc0);
                acc1 = fma(t3, t3, acc1);
            }
        }
        double d2 = acc0 + acc1;
#pragma unroll
        for (int o = S::G / 2; o > 0; o >>= 1)
            d2 += __shfl_xor(d2, o, 64);
        if (j < n && g == 0) {
            const int c = chi_of(attr[id], cattr, mask, hmask);
            out[j] = w_key64(d2, c, m, w);
        }
    }
}

template <int DP>
__device__ __forceinline__ void load_center(const float *vec32, int64_t id, float4 (&qv)[SShape<DP>::NCH])
{
    using S = SShape<DP>;
    const int g = (threadIdx.x & 63) % S::G;
    const float4 *row = reinterpret_cast<const float4 *>(vec32 + id * DP);
#pragma unroll
    for (int c = 0; c < S::NCH; ++c)
        qv[c] = row[g + S::G * c];
}

// Sort (key, id) pairs in LDS, in place, by rank counting (n <= 64 * MAXT).
template <int MAXT>
__device__ void sort_pairs(double *k, uint32_t *id, int n)
{
    const int lane = threadIdx.x & 63;
    double ke[MAXT];
    uint32_t ie[MAXT];
    int rank[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        const int e = lane + 64 * t;
        rank[t] = 0;
        ke[t] = 0.0;
        ie[t] = 0u;
        if (e < n) {
            ke[t] = k[e];
            ie[t] = id[e];
        }
    }
    for (int i = 0; i < n; ++i) {
        const double ki = k[i];
        const uint32_t ii = id[i];
#pragma unroll
        for (int t = 0; t < MAXT; ++t)
            rank[t] += lt64(ki, ii, ke[t], ie[t]) ? 1 : 0;
    }
    wsync();
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        const int e = lane + 64 * t;
        if (e < n) {
            k[rank[t]] = ke[t];
            id[rank[t]] = ie[t];
        }
    }
    wsync();
}

// Greedy landing-zone walk over sorted candidates ck/ci[0..nc); the chosen
// ids go to sel[0..), returns their count (<= R).
template <int DP>
__device__ int landing_walk(const float *vec32, const uint32_t *attr, uint32_t mask, uint32_t hmask,
                            int m, const Weights &w, const double *ck, const uint32_t *ci, int nc, int R,
                            uint32_t *sel, double *scratch)
{
    const int lane = threadIdx.x & 63;
    int nsel = 0;
    float4 pv[SShape<DP>::NCH];
    for (int t = 0; t < nc && nsel < R; ++t) {
        const uint32_t p = ci[t];
        bool ok = true;
        if (nsel > 0) {
            load_center<DP>(vec32, p, pv);
            exact_keys<DP>(vec32, attr, attr[p], mask, hmask, m, w, pv, sel, scratch, nsel);
            wsync();
            const double kpi = ck[t];
            const bool blocked = lane < nsel && !(kpi < scratch[lane]);
            ok = __ballot(blocked) == 0;
        }
        if (ok) {
            if (lane == 0)
                sel[nsel] = p;
            nsel += 1;
            wsync();
        }
    }
    return nsel;
}

struct SelArgs {
    const float *vec32;
    const uint32_t *attr;
    const int32_t *cand;  // [n][K] approximate candidates (-1 padded)
    int32_t *adj;         // [n][R]
    int64_t n;
    int m, K, l, R;
    Weights w;
    int64_t row0;   // rows row0 .. row0 + nrows - 1 (cand holds their lists)
    int64_t nrows;
    int abits;      // attribute field width
};

template <int DP>
__global__ __launch_bounds__(64) void k_select(const SelArgs a)
{
    const int lane = threadIdx.x;
    if ((int64_t)blockIdx.x >= a.nrows)
        return;
    const int64_t i = a.row0 + blockIdx.x;
    const int32_t *crow = a.cand + (int64_t)blockIdx.x * a.K;
    extern __shared__ __align__(16) uint32_t smem[];
    double *ck = reinterpret_cast<double *>(smem);      // [K]
    double *scratch = ck + a.K;                         // [64]
    uint32_t *ci = reinterpret_cast<uint32_t *>(scratch + 64);  // [K]
    uint32_t *sel = ci + a.K;                           // [64]
    const uint32_t mask = attr_full_mask(a.m, a.abits);
    const uint32_t hmask = attr_hmask(a.abits);

    int nc = 0;
    for (int e0 = 0; e0 < a.K; e0 += 64) {
        const int e = e0 + lane;
        const int32_t v = e < a.K ? crow[e] : -1;
        const bool ok = v >= 0 && v < a.n && v != i;
        const uint64_t b = __ballot(ok);
        if (ok)
            ci[nc + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = (uint32_t)v;
        nc += __popcll(b);
    }
    wsync();
    float4 qv[SShape<DP>::NCH];
    load_center<DP>(a.vec32, i, qv);
    exact_keys<DP>(a.vec32, a.attr, a.attr[i], mask, hmask, a.m, a.w, qv, ci, ck, nc);
    wsync();
    sort_pairs<4>(ck, ci, nc);
    const int nl = min(nc, a.l);
    const int ns = landing_walk<DP>(a.vec32, a.attr, mask, hmask, a.m, a.w, ck, ci, nl, a.R, sel, scratch);
    for (int e = lane; e < a.R; e += 64)
        a.adj[i * a.R + e] = e < ns ? (int32_t)sel[e] : -1;
}

// reverse pass: pool(j) = fwd(j) united with the vertices that chose j
struct RevArgs {
    const float *vec32;
    const uint32_t *attr;
    const int32_t *fwd;      // [n][R]
    const int64_t *off;      // [n+1] offsets into inc
    const int32_t *inc;      // incoming lists
    int32_t *adj;            // [n][R]
    double *wk;              // [total pool] keys workspace
    uint32_t *wi;            // [total pool] ids workspace
    const int64_t *poff;     // [n+1] offsets into wk / wi
    int64_t n;
    int m, R;
    Weights w;
    const int32_t *targets;  // nullable: re-select these rows only (t -> row)
    int64_t nt;              // rows re-selected (grid)
    int abits;               // attribute field width
};

template <int DP>
__global__ __launch_bounds__(64) void k_reverse(const RevArgs a)
{
    const int lane = threadIdx.x;
    const int64_t ti = blockIdx.x;
    if (ti >= a.nt)
        return;
    const int64_t j = a.targets ? (int64_t)a.targets[ti] : ti;
    extern __shared__ __align__(16) uint32_t smem[];
    double *scratch = reinterpret_cast<double *>(smem);          // [64]
    uint32_t *sel = reinterpret_cast<uint32_t *>(scratch + 64);  // [64]
    const uint32_t mask = attr_full_mask(a.m, a.abits);
    const uint32_t hmask = attr_hmask(a.abits);
    double *pk = a.wk + a.poff[ti];
    uint32_t *pi = a.wi + a.poff[ti];
    const int64_t ninc = a.off[ti + 1] - a.off[ti];
    // the pool: the forward row, then incoming ids not already in it
    int np = 0;
    const int64_t total = a.R + ninc;
    for (int64_t e0 = 0; e0 < total; e0 += 64) {
        const int64_t e = e0 + lane;
        int32_t v = -1;
        if (e < total)
            v = e < a.R ? a.fwd[j * a.R + e] : a.inc[a.off[ti] + (e - a.R)];
        bool ok = v >= 0;
        if (ok && e >= a.R) {
            for (int t = 0; t < a.R; ++t)
                if (a.fwd[j * a.R + t] == v)
                    ok = false;
        }
        const uint64_t b = __ballot(ok);
        if (ok)
            pi[np + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = (uint32_t)v;
        np += __popcll(b);
    }
    __threadfence();
    wsync();
    float4 qv[SShape<DP>::NCH];
    load_center<DP>(a.vec32, j, qv);
    exact_keys<DP>(a.vec32, a.attr, a.attr[j], mask, hmask, a.m, a.w, qv, pi, pk, np);
    __threadfence();
    wsync();
    // landing-zone walk in (key, id) order: extract the next smallest entry
    int nsel = 0;
    bool have_last = false;
    double last_k = 0.0;
    uint32_t last_i = 0;
    for (int used = 0; used < np && nsel < a.R; ++used) {
        double bk = __longlong_as_double(0x7FF0000000000000ll);
        uint32_t bi = 0xFFFFFFFFu;
        for (int e = lane; e < np; e += 64) {
            const double k = pk[e];
            const uint32_t id = pi[e];
            const bool after = !have_last || lt64(last_k, last_i, k, id);
            if (after && lt64(k, id, bk, bi)) {
                bk = k;
                bi = id;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ok_ = __shfl_xor(bk, o, 64);
            const uint32_t oi = (uint32_t)__shfl_xor((int)bi, o, 64);
            if (lt64(ok_, oi, bk, bi)) {
                bk = ok_;
                bi = oi;
            }
        }
        have_last = true;
        last_k = bk;
        last_i = bi;
        bool ok = true;
        if (nsel > 0) {
            float4 pv[SShape<DP>::NCH];
            load_center<DP>(a.vec32, bi, pv);
            exact_keys<DP>(a.vec32, a.attr, a.attr[bi], mask, hmask, a.m, a.w, pv, sel, scratch, nsel);
            wsync();
            const bool blocked = lane < nsel && !(bk < scratch[lane]);
            ok = __ballot(blocked) == 0;
        }
        if (ok) {
            if (lane == 0)
                sel[nsel] = bi;
            nsel += 1;
            wsync();
        }
    }
    for (int e = lane; e < a.R; e += 64)
        a.adj[j * a.R + e] = e < nsel ? (int32_t)sel[e] : -1;
}

__global__ void k_count_incoming(const int32_t *fwd, int64_t n, int R, int64_t *cnt)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * R;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = fwd[t];
        if (v >= 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[v + 1]), 1ull);
    }
}

__global__ void k_fill_incoming(const int32_t *fwd, int64_t n, int R, const int64_t *off,
                                int64_t *fill, int32_t *inc)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * R;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = fwd[t];
        if (v >= 0) {
            const unsigned long long s = atomicAdd(reinterpret_cast<unsigned long long *>(&fill[v]), 1ull);
            inc[off[v] + (int64_t)s] = (int32_t)(t / R);
        }
    }
}

template <int DP>
int launch_select_dp(const SelArgs &a, hipStream_t st)
{
    const size_t lds = sizeof(double) * ((size_t)a.K + 64) + sizeof(uint32_t) * ((size_t)a.K + 64);
    hipLaunchKernelGGL(k_select<DP>, dim3((unsigned)a.nrows), dim3(64), lds, st, a);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

template <int DP>
int launch_reverse_dp(const RevArgs &a, hipStream_t st)
{
    const size_t lds = sizeof(double) * 64 + sizeof(uint32_t) * 64;
    hipLaunchKernelGGL(k_reverse<DP>, dim3((unsigned)a.nt), dim3(64), lds, st, a);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // namespace

int launch_select(const Index *ix, const int32_t *cand, int K, int l, int32_t *adj, hipStream_t st)
{
    if (K > 256)
        return fail(NHQ_EINVAL, "candidate list longer than 256");
    SelArgs a{ix->vec32, ix->attr, cand, adj, ix->n, ix->m, K, l, ix->degree, ix->w, 0, ix->n, ix->abits};
    switch (ix->dp) {
    case 32: return launch_select_dp<32>(a, st);
    case 64: return launch_select_dp<64>(a, st);
    case 96: return launch_select_dp<96>(a, st);
    case 128: return launch_select_dp<128>(a, st);
    case 256: return launch_select_dp<256>(a, st);
    case 512: return launch_select_dp<512>(a, st);
    case 960: return launch_select_dp<960>(a, st);
    case 1024: return launch_select_dp<1024>(a, st);
    }
    return fail(NHQ_EINVAL, "unsupported padded dimension");
}

// exact re-score of K approximate neighbours per query (filter mode of the
// dense tiles) and output of the k best by (delta, id)
struct RefArgs {
    const float *vec32;
    const uint32_t *attr;
    const float *qpad;    // [nq][DP]
    const int32_t *cand;  // [nq][K]
    int32_t *ids;         // [nq][k]
    float *dists;         // [nq][k]
    int64_t nq;
    int K, k;
};

template <int DP>
__global__ __launch_bounds__(64) void k_refine(const RefArgs a)
{
    const int lane = threadIdx.x;
    const int64_t qi = blockIdx.x;
    if (qi >= a.nq)
        return;
    extern __shared__ __align__(16) uint32_t smem[];
    double *ck = reinterpret_cast<double *>(smem);              // [K]
    uint32_t *ci = reinterpret_cast<uint32_t *>(ck + a.K);      // [K]
    int nc = 0;
    for (int e0 = 0; e0 < a.K; e0 += 64) {
        const int e = e0 + lane;
        const int32_t v = e < a.K ? a.cand[qi * a.K + e] : -1;
        const bool ok = v >= 0;
        const uint64_t b = __ballot(ok);
        if (ok)
            ci[nc + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = (uint32_t)v;
        nc += __popcll(b);
    }
    wsync();
    float4 qv[SShape<DP>::NCH];
    load_center<DP>(a.qpad, qi, qv);
    // Def. 4 ground truth: exact matches ranked by delta alone
    exact_keys<DP>(a.vec32, a.attr, 0u, 0u, 0x80808080u, 0, Weights{NHQ_WEIGHTS_DEFAULT, 0.0f, 0.0}, qv,
                   ci, ck, nc);
    wsync();
    sort_pairs<4>(ck, ci, nc);
    for (int e = lane; e < a.k; e += 64) {
        a.ids[qi * a.k + e] = e < nc ? (int32_t)ci[e] : -1;
        a.dists[qi * a.k + e] = e < nc ? (float)sqrt(ck[e]) : __int_as_float(0x7F800000);
    }
}

int launch_refine(const Index *ix, const float *qpad, const int32_t *cand, int64_t nq, int K, int k,
                  int32_t *ids, float *dists, hipStream_t st)
{
    if (nq == 0)
        return NHQ_OK;
    RefArgs a{ix->vec32, ix->attr, qpad, cand, ids, dists, nq, K, k};
    const size_t lds = (sizeof(double) + sizeof(uint32_t)) * (size_t)K;
    switch (ix->dp) {
#define NHQ_REF(DPV)                                                                   \
    case DPV:                                                                          \
        hipLaunchKernelGGL(k_refine<DPV>, dim3((unsigned)nq), dim3(64), lds, st, a);    \
        break;
        NHQ_REF(32)
        NHQ_REF(64)
        NHQ_REF(96)
        NHQ_REF(128)
        NHQ_REF(256)
        NHQ_REF(512)
        NHQ_REF(960)
        NHQ_REF(1024)
#undef NHQ_REF
    default:
        return fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

// Edge selection for rows row0 .. row0 + nrows - 1 from cand [nrows][K]
int launch_select_rows(const Index *ix, const int32_t *cand, int K, int l, int32_t *adj,
                       int64_t row0, int64_t nrows, hipStream_t st)
{
    if (K > 256)
        return fail(NHQ_EINVAL, "candidate list longer than 256");
    if (nrows <= 0)
        return NHQ_OK;
    SelArgs a{ix->vec32, ix->attr, cand, adj, ix->n, ix->m, K, l, ix->degree, ix->w, row0, nrows, ix->abits};
    switch (ix->dp) {
    case 32: return launch_select_dp<32>(a, st);
    case 64: return launch_select_dp<64>(a, st);
    case 96: return launch_select_dp<96>(a, st);
    case 128: return launch_select_dp<128>(a, st);
    case 256: return launch_select_dp<256>(a, st);
    case 512: return launch_select_dp<512>(a, st);
    case 960: return launch_select_dp<960>(a, st);
    case 1024: return launch_select_dp<1024>(a, st);
    }
    return fail(NHQ_EINVAL, "unsupported padded dimension");
}

// Re-selection of the rows targets[0..nt) of adj (in place) from the row
// united with the offers inc[off[t] .. off[t+1]) (device arrays)
int launch_reselect_targets(const Index *ix, int32_t *adj, const int32_t *targets, int64_t nt,
                            const int64_t *off, const int32_t *inc, hipStream_t st)
{
    if (nt <= 0)
        return NHQ_OK;
    const int R = ix->degree;
    std::vector<int64_t> hoff((size_t)nt + 1);
    NHQ_HIP(hipMemcpyAsync(hoff.data(), off, sizeof(int64_t) * (size_t)(nt + 1), hipMemcpyDeviceToHost, st));
    NHQ_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> poff((size_t)nt + 1);
    poff[0] = 0;
    for (int64_t t = 0; t < nt; ++t)
        poff[t + 1] = poff[t] + R + (hoff[t + 1] - hoff[t]);
    int64_t *dpoff = nullptr;
    double *wk = nullptr;
    uint32_t *wi = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&dpoff, sizeof(int64_t) * (size_t)(nt + 1), st));
    NHQ_HIP(hipMallocAsync((void **)&wk, sizeof(double) * (size_t)poff[nt], st));
    NHQ_HIP(hipMallocAsync((void **)&wi, sizeof(uint32_t) * (size_t)poff[nt], st));
    NHQ_HIP(hipMemcpyAsync(dpoff, poff.data(), sizeof(int64_t) * (size_t)(nt + 1), hipMemcpyHostToDevice, st));
    RevArgs a{ix->vec32, ix->attr, adj, off, inc, adj, wk, wi, dpoff, ix->n, ix->m, R, ix->w, targets, nt,
              ix->abits};
    int rc = NHQ_OK;
    switch (ix->dp) {
    case 32: rc = launch_reverse_dp<32>(a, st); break;
    case 64: rc = launch_reverse_dp<64>(a, st); break;
    case 96: rc = launch_reverse_dp<96>(a, st); break;
    case 128: rc = launch_reverse_dp<128>(a, st); break;
    case 256: rc = launch_reverse_dp<256>(a, st); break;
    case 512: rc = launch_reverse_dp<512>(a, st); break;
    case 960: rc = launch_reverse_dp<960>(a, st); break;
    case 1024: rc = launch_reverse_dp<1024>(a, st); break;
    default: rc = fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    void *bufs[] = {dpoff, wk, wi};
    for (void *b : bufs)
        (void)hipFreeAsync(b, st);
    NHQ_HIP(hipStreamSynchronize(st));
    return rc;
}

int launch_reverse(const Index *ix, const int32_t *fwd, int32_t *adj, hipStream_t st)
{
    const int64_t n = ix->n;
    const int R = ix->degree;
    // incoming lists: counts, offsets (host scan), fill
    int64_t *cnt = nullptr, *fill = nullptr;
    int32_t *inc = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&cnt, sizeof(int64_t) * (size_t)(n + 1), st));
    NHQ_HIP(hipMallocAsync((void **)&fill, sizeof(int64_t) * (size_t)n, st));
    NHQ_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (size_t)(n + 1), st));
    NHQ_HIP(hipMemsetAsync(fill, 0, sizeof(int64_t) * (size_t)n, st));
    const int grid = (int)std::min<int64_t>(65536, (n * R + 255) / 256);
    hipLaunchKernelGGL(k_count_incoming, dim3(grid), dim3(256), 0, st, fwd, n, R, cnt);
    std::vector<int64_t> h((size_t)n + 1);
    NHQ_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, st));
    NHQ_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> poff((size_t)n + 1);
    poff[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        poff[v + 1] = poff[v] + R + h[v + 1];
        h[v + 1] += h[v];
    }
    int64_t *off = nullptr, *dpoff = nullptr;
    double *wk = nullptr;
    uint32_t *wi = nullptr;
    NHQ_HIP(hipMallocAsync((void **)&off, sizeof(int64_t) * (size_t)(n + 1), st));
    NHQ_HIP(hipMallocAsync((void **)&dpoff, sizeof(int64_t) * (size_t)(n + 1), st));
    NHQ_HIP(hipMallocAsync((void **)&inc, sizeof(int32_t) * (size_t)std::max<int64_t>(1, h[n]), st));
    NHQ_HIP(hipMallocAsync((void **)&wk, sizeof(double) * (size_t)poff[n], st));
    NHQ_HIP(hipMallocAsync((void **)&wi, sizeof(uint32_t) * (size_t)poff[n], st));
    NHQ_HIP(hipMemcpyAsync(off, h.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, st));
    NHQ_HIP(hipMemcpyAsync(dpoff, poff.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill_incoming, dim3(grid), dim3(256), 0, st, fwd, n, R, off, fill, inc);
    RevArgs a{ix->vec32, ix->attr, fwd, off, inc, adj, wk, wi, dpoff, n, ix->m, R, ix->w, nullptr, n,
              ix->abits};
    int rc = NHQ_OK;
    switch (ix->dp) {
    case 32: rc = launch_reverse_dp<32>(a, st); break;
    case 64: rc = launch_reverse_dp<64>(a, st); break;
    case 96: rc = launch_reverse_dp<96>(a, st); break;
    case 128: rc = launch_reverse_dp<128>(a, st); break;
    case 256: rc = launch_reverse_dp<256>(a, st); break;
    case 512: rc = launch_reverse_dp<512>(a, st); break;
    case 960: rc = launch_reverse_dp<960>(a, st); break;
    case 1024: rc = launch_reverse_dp<1024>(a, st); break;
    default: rc = fail(NHQ_EINVAL, "unsupported padded dimension");
    }
    void *bufs[] = {cnt, fill, off, dpoff, inc, wk, wi};
    for (void *b : bufs)
        (void)hipFreeAsync(b, st);
    NHQ_HIP(hipStreamSynchronize(st));
    return rc;
}

}  // namespace nhq
