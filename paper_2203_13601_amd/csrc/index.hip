// Index object, ingest kernels (attribute packing, storage conversion, row
// norms) and the C entry points of libnhq that are not kernels themselves.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <unordered_set>
#include <vector>

#include <cstring>

#include "nhq_internal.h"

namespace nhq {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int padded_dim(int d)
{
    static const int widths[] = {32, 64, 96, 128, 256, 512, 960, 1024};
    for (int w : widths)
        if (d <= w)
            return w;
    return -1;
}

int ensure_workspace(Index *ix, size_t bytes)
{
    if (ix->ws_bytes >= bytes)
        return NHQ_OK;
    if (ix->ws) {
        NHQ_HIP(hipDeviceSynchronize());
        NHQ_HIP(hipFree(ix->ws));
        ix->ws = nullptr;
        ix->ws_bytes = 0;
    }
    if (hipMalloc(&ix->ws, bytes) != hipSuccess)
        return fail(NHQ_ENOMEM, "workspace allocation failed");
    ix->ws_bytes = bytes;
    return NHQ_OK;
}

namespace {

// ---------------------------------------------------------------- kernels
__global__ void k_pad_copy(const float *__restrict__ src, float *__restrict__ dst, int64_t n,
                           int d, int dp)
{
    const int64_t total = n * dp;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / dp;
        const int c = (int)(t - r * dp);
        dst[t] = c < d ? src[r * d + c] : 0.0f;
    }
}

// attribute codes (one byte each) packed into one word, b bits per code,
// attribute j in bits b*j .. (the codes fit: checked from their histogram)
__global__ void k_pack_attr(const uint8_t *__restrict__ a, uint32_t *__restrict__ out, int64_t n,
                            int m, int b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t w = 0;
        for (int j = 0; j < m; ++j)
            w |= (uint32_t)a[i * m + j] << (b * j);
        out[i] = w;
    }
}

// squared norm of each row: one wavefront per row, lane j summing elements
// j, j + 64, ... (coalesced 256-byte loads), then a butterfly over the wave
__global__ void k_row_norm(const float *__restrict__ v, float *__restrict__ norm, int64_t n, int dp)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += waves) {
        const float *r = v + i * dp;
        float s = 0.0f;
        for (int c = lane; c < dp; c += 64)
            s = fmaf(r[c], r[c], s);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            s += __shfl_xor(s, o, 64);
        if (lane == 0)
            norm[i] = s;
    }
}

// float32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_rne(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__global__ void k_to_bf16(const float *__restrict__ v, uint16_t *__restrict__ out, int64_t total)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = (uint16_t)bf16_rne(v[t]);
}

// The split of one value for the bf16 matrix cores: hi = bf16(v), lo =
// bf16(v - hi) (v - hi is exact in float32), so hi + lo equals v to within
// 2^-17 |v|, and hi * hi' + hi * lo' + lo * hi' equals v v' to within about
// 3 * 2^-17 |v v'|; values exact in bf16 have lo = 0.  Element c of a row
// goes to chunk c / 32: hi at 64 (c / 32) + c % 32, lo 32 further on.
__device__ __forceinline__ void split_bf16(float v, uint32_t &hi, uint32_t &lo)
{
    hi = bf16_rne(v);
    lo = bf16_rne(v - __uint_as_float(hi << 16));
}
__device__ __forceinline__ void put_split(uint16_t *row, int c, float v)
{
    uint32_t hi, lo;
    split_bf16(v, hi, lo);
    const int at = 64 * (c >> 5) + (c & 31);
    row[at] = (uint16_t)hi;
    row[at + 32] = (uint16_t)lo;
}

__global__ void k_split_rows(const float *__restrict__ src, int64_t rows, int dp, uint16_t *__restrict__ dst)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < rows * dp;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / dp;
        const int c = (int)(t - r * dp);
        put_split(dst + r * 2 * dp, c, src[t]);
    }
}

// OCP e4m3 ("FN": bias 7, no infinities, largest finite 448) of a double,
// nearest value with ties to the even code, saturating at +-448.
__device__ uint8_t e4m3_from_double(double x)
{
    const uint32_t sign = signbit(x) ? 0x80u : 0u;
    const double a = fabs(x);
    uint32_t code;
    if (a >= 448.0) {
        code = 0x7Eu;
    } else if (a < 0.015625) {  // below 2^-6: multiples of 2^-9
        code = (uint32_t)rint(a * 512.0);  // 8 lands on 2^-6, code 0x08
    } else {
        int ex;
        const double f = frexp(a, &ex);  // a = f 2^ex, f in [0.5, 1)
        const int e = ex - 1;             // a in [2^e, 2^(e+1))
        uint32_t mant = (uint32_t)rint((2.0 * f - 1.0) * 8.0);
        int be = e + 7;
        if (mant == 8u) {
            mant = 0;
            be += 1;
        }
        code = ((uint32_t)be << 3) | mant;
        if (code > 0x7Eu)
            code = 0x7Eu;
    }
    return (uint8_t)(code | sign);
}

// one wave per row: scale s = max|x| / 448 (1 for a zero row), codes e4m3(x/s)
__global__ __launch_bounds__(64) void k_to_fp8(const float *__restrict__ v, uint8_t *__restrict__ out,
                                               float *__restrict__ scale, int64_t n, int dp)
{
    const int lane = threadIdx.x;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        const float *row = v + r * dp;
        float mx = 0.0f;
        for (int c = lane; c < dp; c += 64)
            mx = fmaxf(mx, fabsf(row[c]));
        for (int o = 32; o > 0; o >>= 1)
            mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
        for (int c = lane; c < dp; c += 64)
            out[r * dp + c] = e4m3_from_double((double)row[c] / (double)s);
        if (lane == 0)
            scale[r] = s;
    }
}

// a lane's value from another lane of its 16-lane row (DPP)
template <int CTRL>
__device__ __forceinline__ float row_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// 16 lanes per query (4 queries per wave): (qpad non-null) zero-padded
// float32 row, squared norm, packed codes and constraint mask, whether every
// value is an integer of magnitude <= 256, and (qsplit non-null) the row's
// hi/lo split
__global__ __launch_bounds__(64) void k_pad_queries(const float *__restrict__ q,
                                                    const uint8_t *__restrict__ qa, int64_t nq, int d,
                                                    int dp, int m, int abits, float *__restrict__ qpad,
                                                    float *__restrict__ qnorm,
                                                    uint32_t *__restrict__ qword,
                                                    uint32_t *__restrict__ qmask,
                                                    uint32_t *__restrict__ qexact,
                                                    uint16_t *__restrict__ qsplit)
{
    const int lane = threadIdx.x, sub = lane & 15, grp = lane >> 4;
    const uint32_t fm = (abits >= 32) ? 0xFFFFFFFFu : ((1u << abits) - 1u);
    for (int64_t i0 = 4 * (int64_t)blockIdx.x; i0 < nq; i0 += 4 * (int64_t)gridDim.x) {
        const int64_t i = i0 + grp;
        const bool live = i < nq;
        // code `sub` of the query (m <= 12), loaded with the row
        const uint32_t code = (live && sub < m) ? (uint32_t)qa[i * m + sub] : 0xFFu;
        float s = 0.0f;
        bool exact = true;
        if (live) {
            // 128 elements per round, 8 consecutive ones per lane (dp is a
            // multiple of 32, so a lane's 8 lie all inside the row or all
            // past it): 16-byte loads where the row allows them, 16-byte
            // stores of the padded row and of the split halves; each lane
            // sums its elements in increasing order
            const bool vec = (d & 3) == 0;
            for (int c0 = 8 * sub; c0 < dp; c0 += 128) {
                float v[8];
                if (vec && c0 + 8 <= d) {
                    const float4 *src = reinterpret_cast<const float4 *>(q + i * d + c0);
                    const float4 lo4 = src[0], hi4 = src[1];
                    v[0] = lo4.x, v[1] = lo4.y, v[2] = lo4.z, v[3] = lo4.w;
                    v[4] = hi4.x, v[5] = hi4.y, v[6] = hi4.z, v[7] = hi4.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        v[u] = c0 + u < d ? q[i * d + c0 + u] : 0.0f;
                }
                if (qpad) {
                    float4 *dst = reinterpret_cast<float4 *>(qpad + i * dp + c0);
                    dst[0] = make_float4(v[0], v[1], v[2], v[3]);
                    dst[1] = make_float4(v[4], v[5], v[6], v[7]);
                }
                if (qsplit) {
                    uint32_t hw[4], lw[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        uint32_t h2[2], l2[2];
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            split_bf16(v[2 * u + e], h2[e], l2[e]);
                        }
                        hw[u] = h2[0] | (h2[1] << 16);
                        lw[u] = l2[0] | (l2[1] << 16);
                    }
                    uint16_t *row = qsplit + i * 2 * dp + 64 * (c0 >> 5) + (c0 & 31);
                    *reinterpret_cast<uint4 *>(row) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
                    *reinterpret_cast<uint4 *>(row + 32) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    s = fmaf(v[u], v[u], s);
                    exact = exact && v[u] == rintf(v[u]) && fabsf(v[u]) <= 256.0f;
                }
            }
        }
        // the codes packed like attr_pack_query, gathered from the group's lanes
        uint32_t w = 0, mk = 0;
        for (int j = 0; j < m; ++j) {
            const uint32_t c = (uint32_t)__shfl((int)code, 16 * grp + j);
            if (c != 0xFFu) {
                w |= (c < fm ? c : fm) << (abits * j);
                mk |= fm << (abits * j);
            }
        }
        // sum over the 16 lanes of the row
        s += row_mov<0xB1>(s);   // quad_perm(1, 0, 3, 2)
        s += row_mov<0x4E>(s);   // quad_perm(2, 3, 0, 1)
        s += row_mov<0x141>(s);  // row_half_mirror
        s += row_mov<0x140>(s);  // row_mirror
        const bool all_exact = ((__ballot(!exact) >> (16 * grp)) & 0xFFFFull) == 0;
        if (live && sub == 0) {
            if (qexact)
                qexact[i] = all_exact ? 1u : 0u;
            qnorm[i] = s;
            qword[i] = w;
            qmask[i] = mk;
        }
    }
}

// counts of every (attribute, code) pair
__global__ void k_code_hist(const uint8_t *__restrict__ a, int64_t n, int m, uint32_t *__restrict__ cnt)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * m;
         t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[(t % m) * 256 + a[t]], 1u);
}

// dense copy of the entry sample's rows, norms and codes
__global__ void k_gather_entry(const int32_t *__restrict__ entry, int ne, const float *__restrict__ vec32,
                               const float *__restrict__ norm, const uint32_t *__restrict__ attr,
                               int dp, float *__restrict__ ev, float *__restrict__ en,
                               uint32_t *__restrict__ ea)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)ne * dp;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / dp;
        const int c = (int)(t - r * dp);
        const int64_t id = entry[r];
        ev[t] = vec32[id * dp + c];
        if (c == 0) {
            en[r] = norm[id];
            ea[r] = attr[id];
        }
    }
}

int grid_for(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

// The stratified entry sample: for every packed attribute word the objects
// hold (in increasing order), the min(per, count) objects with the smallest
// (h(i), i), h(i) = the first splitmix64 output from state
// (seed ^ 0x8F14E45FCEEA167A) ^ (i * 0xD1B54A32D192ED03); appended to ent,
// with each block's word and its first position (plus the end) recorded.
int stratify(const std::vector<uint32_t> &aw, uint64_t seed, int per, std::vector<int32_t> &ent,
             std::vector<uint32_t> &words, std::vector<int32_t> &offs)
{
    struct Key {
        uint32_t w;
        int32_t id;
        uint64_t h;
    };
    const size_t n = aw.size();
    std::vector<Key> keys(n);
    const uint64_t base = seed ^ 0x8F14E45FCEEA167Aull;
    for (size_t i = 0; i < n; ++i) {
        uint64_t state = base ^ ((uint64_t)i * 0xD1B54A32D192ED03ull);
        keys[i] = Key{aw[i], (int32_t)i, splitmix64_next(state)};
    }
    std::sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) {
        return a.w != b.w ? a.w < b.w : (a.h != b.h ? a.h < b.h : a.id < b.id);
    });
    words.clear();
    offs.clear();
    for (size_t i = 0; i < n;) {
        size_t j = i;
        while (j < n && keys[j].w == keys[i].w)
            ++j;
        words.push_back(keys[i].w);
        offs.push_back((int32_t)ent.size());
        for (size_t t = i; t < std::min(j, i + (size_t)per); ++t)
            ent.push_back(keys[t].id);
        i = j;
    }
    offs.push_back((int32_t)ent.size());
    if (words.size() > 4096)
        return fail(NHQ_EINVAL, "a stratified entry sample holds at most 4096 attribute patterns");
    return NHQ_OK;
}

void free_index(Index *ix)
{
    if (!ix)
        return;
    if (ix->vecs && ix->vecs != ix->vec32)
        (void)hipFree(ix->vecs);
    void *ptrs[] = {ix->vec32, ix->scale, ix->attr, ix->norm, ix->adj, ix->entry, ix->entry_vec,
                    ix->entry_norm, ix->entry_attr, ix->entry_bf16, ix->entry_split, ix->err, ix->ws, ix->mlp,
                    ix->logp, ix->block_word, ix->block_off};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
}

int launch_pad_queries(const float *q, const uint8_t *qa, int64_t nq, int d, int dp, int m,
                       int abits, float *qpad, float *qnorm, uint32_t *qword, uint32_t *qmask,
                       uint32_t *qexact, uint16_t *qsplit, hipStream_t st)
{
    if (nq == 0)
        return NHQ_OK;
    hipLaunchKernelGGL(k_pad_queries, dim3(grid_for(nq, 4)), dim3(64), 0, st, q, qa, nq, d, dp, m,
                       abits, qpad, qnorm, qword, qmask, qexact, qsplit);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

int launch_split_rows(const float *src, int64_t rows, int dp, uint16_t *dst, hipStream_t st)
{
    if (rows == 0)
        return NHQ_OK;
    hipLaunchKernelGGL(k_split_rows, dim3(grid_for(rows * dp, 256)), dim3(256), 0, st, src, rows, dp, dst);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

}  // namespace nhq

using namespace nhq;

extern "C" {

int nhq_version(void) { return 1; }

const char *nhq_strerror(int code)
{
    switch (code) {
    case NHQ_OK:
        return "ok";
    case NHQ_EINVAL:
        return "invalid argument";
    case NHQ_ENOMEM:
        return "out of memory";
    case NHQ_EHIP:
        return "HIP runtime error";
    case NHQ_EDEVICE:
        return "device error word set";
    case NHQ_ENOTSUP:
        return "not supported";
    case NHQ_EIO:
        return "i/o error";
    case NHQ_EBUSY:
        return "busy";
    }
    return "unknown error";
}

const char *nhq_last_error(void) { return g_last_error.c_str(); }

int nhq_index_create(const float *vecs, const uint8_t *attrs, int64_t n, int32_t d, int32_t m,
                     const nhq_build_params *params, void *stream, nhq_index **out)
{
    if (!out)
        return fail(NHQ_EINVAL, "out is null");
    *out = nullptr;
    if (!vecs || (m > 0 && !attrs))
        return fail(NHQ_EINVAL, "vecs/attrs is null");
    if (n < 1 || n >= kMaxN)
        return fail(NHQ_EINVAL, "n must be in [1, 2^27)");
    if (d < 1 || d > 1024)
        return fail(NHQ_EINVAL, "d must be in [1, 1024]");
    if (m < 0 || m > NHQ_MAX_ATTRS)
        return fail(NHQ_EINVAL, "m must be in [0, 12]");
    nhq_build_params p{};
    if (params)
        p = *params;
    if (p.degree == 0)
        p.degree = 32;
    if (p.cand == 0)
        p.cand = 64;
    if (p.n_entry == 0)
        p.n_entry = 1024;
    if (p.degree < 1 || p.degree > NHQ_MAX_DEGREE)
        return fail(NHQ_EINVAL, "degree must be in [1, 64]");
    if (p.cand < p.degree || p.cand > 256)
        return fail(NHQ_EINVAL, "cand must be in [degree, 256]");
    if (p.storage < 0 || p.storage > 2)
        return fail(NHQ_EINVAL, "storage must be 0, 1 or 2");
    if (p.n_entry < 1 || p.n_entry > 65536)
        return fail(NHQ_EINVAL, "n_entry must be in [1, 65536]");
    if (p.weights < NHQ_WEIGHTS_DEFAULT || p.weights > NHQ_WEIGHTS_FIXED)
        return fail(NHQ_EINVAL, "weights must be an NHQ_WEIGHTS_* value");
    if ((p.weights == NHQ_WEIGHTS_HARMONIC_C && !(p.weight_param > 1.0)) ||
        (p.weights == NHQ_WEIGHTS_NORMALISED && !(p.weight_param > 0.0)) ||
        (p.weights == NHQ_WEIGHTS_FIXED && !(p.weight_param >= 0.0)) ||
        !(p.weight_param < 3.0e38))
        return fail(NHQ_EINVAL, "weight_param out of range for the weight setting");
    if (p.nnd_rounds == 0)
        p.nnd_rounds = 12;
    if (p.nnd_sample == 0)
        p.nnd_sample = 24;
    if (p.nnd_stop == 0.0f)
        p.nnd_stop = 0.001f;
    if (p.nsw_batch == 0)
        p.nsw_batch = 10000;
    if (p.nsw_beam == 0)
        p.nsw_beam = p.cand;
    if (p.capacity == 0)
        p.capacity = n;
    if (p.capacity < n || p.capacity >= kMaxN)
        return fail(NHQ_EINVAL, "capacity must be in [n, 2^27)");
    if (p.builder < NHQ_BUILD_EXACT || p.builder > NHQ_BUILD_NSW)
        return fail(NHQ_EINVAL, "builder must be an NHQ_BUILD_* value");
    if (p.nsw_batch < 1 || p.nsw_beam < p.cand || p.nsw_beam > NHQ_MAX_BEAM)
        return fail(NHQ_EINVAL, "NSW needs nsw_batch >= 1 and cand <= nsw_beam <= 1024");
    if (p.nnd_rounds < 0 || p.nnd_rounds > 1000 || p.nnd_sample < 1 || p.nnd_sample > 64 ||
        !(p.nnd_stop >= 0.0f))
        return fail(NHQ_EINVAL, "NN-descent needs rounds in [0, 1000], sample in [1, 64], stop >= 0");
    if (p.entry_per_pattern < 0 || p.entry_per_pattern > 8192 ||
        (p.entry_per_pattern > 0 && (m < 1 || p.n_entry > 8192)))
        return fail(NHQ_EINVAL, "a stratified entry sample needs m >= 1, n_entry <= 8192 and "
                                "entry_per_pattern in [1, 8192]");

    hipStream_t st = (hipStream_t)stream;
    nhq_index *h = new (std::nothrow) nhq_index();
    if (!h)
        return fail(NHQ_ENOMEM, "host allocation failed");
    Index *ix = &h->impl;
    int rc = NHQ_OK;
    do {
        if (hipGetDevice(&ix->device) != hipSuccess) {
            rc = fail(NHQ_EHIP, "hipGetDevice failed");
            break;
        }
        ix->n = n;
        ix->d = d;
        ix->dp = padded_dim(d);
        ix->m = m;
        ix->storage = p.storage;
        ix->cand = p.cand;
        ix->reverse_edges = p.reverse_edges ? 1 : 0;
        ix->seed = p.seed;
        ix->w.mode = p.weights;
        ix->w.pd = p.weights == NHQ_WEIGHTS_DEFAULT || p.weights == NHQ_WEIGHTS_HARMONIC
                       ? 0.0 : p.weight_param;
        ix->w.p = (float)ix->w.pd;
        ix->builder = p.builder;
        ix->nnd_rounds = p.nnd_rounds;
        ix->nnd_sample = p.nnd_sample;
        ix->nnd_stop = p.nnd_stop;
        ix->nsw_batch = p.nsw_batch;
        ix->nsw_beam = p.nsw_beam;
        ix->degree = 0;
        ix->cap = p.capacity;
        const int want_degree = p.degree;
        const size_t rows = (size_t)n * ix->dp;
        const size_t cap_rows = (size_t)ix->cap * ix->dp;
        if (hipMalloc(&ix->vec32, cap_rows * sizeof(float)) != hipSuccess ||
            hipMalloc(&ix->attr, (size_t)ix->cap * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&ix->norm, (size_t)ix->cap * sizeof(float)) != hipSuccess ||
            hipMalloc(&ix->err, 2 * sizeof(uint32_t)) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "index allocation failed");
            break;
        }
        ix->degree = want_degree;  // graph allocated now, filled by build/set
        if (hipMalloc(&ix->adj, (size_t)ix->cap * want_degree * sizeof(int32_t)) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "graph allocation failed");
            break;
        }
        if (hipMemsetAsync(ix->adj, 0xFF, (size_t)ix->cap * want_degree * sizeof(int32_t), st) != hipSuccess ||
            hipMemsetAsync(ix->err, 0, 2 * sizeof(uint32_t), st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "memset failed");
            break;
        }
        hipLaunchKernelGGL(k_pad_copy, dim3(grid_for((int64_t)rows, 256)), dim3(256), 0, st, vecs,
                           ix->vec32, n, d, ix->dp);
        // per-attribute code counts: the widest code sets the packing; the
        // counts also give ln(count / n), the selectivity estimate the stop
        // network reads (ln(0.5 / n) for absent codes)
        std::vector<uint32_t> hh((size_t)NHQ_MAX_ATTRS * 256, 0u);
        {
            uint32_t *hist = nullptr;
            if (hipMalloc(&hist, sizeof(uint32_t) * hh.size()) != hipSuccess) {
                rc = fail(NHQ_ENOMEM, "histogram allocation failed");
                break;
            }
            (void)hipMemsetAsync(hist, 0, sizeof(uint32_t) * hh.size(), st);
            if (m > 0)
                hipLaunchKernelGGL(k_code_hist, dim3(grid_for(n * m, 256)), dim3(256), 0, st, attrs, n,
                                   m, hist);
            const bool ok = hipMemcpyAsync(hh.data(), hist, sizeof(uint32_t) * hh.size(),
                                           hipMemcpyDeviceToHost, st) == hipSuccess &&
                            hipStreamSynchronize(st) == hipSuccess;
            (void)hipFree(hist);
            if (!ok) {
                rc = fail(NHQ_EHIP, "ingest synchronisation failed");
                break;
            }
        }
        int max_code = 0;
        for (int j = 0; j < m; ++j)
            for (int c = 0; c < 256; ++c)
                if (hh[(size_t)j * 256 + c])
                    max_code = std::max(max_code, c);
        if (m > 0 && hh.size() && max_code == 255) {
            rc = fail(NHQ_EINVAL, "object attribute code 255 is reserved for query wildcards");
            break;
        }
        ix->abits = m > 0 ? attr_bits(m, max_code) : 8;
        if (ix->abits == 0) {
            rc = fail(NHQ_EINVAL, "attribute codes too wide for m attributes in 32 bits (codes <= 14 "
                                  "for m <= 8, <= 2 for m <= 12)");
            break;
        }
        ix->hmask = attr_hmask(ix->abits);
        if (m > 0) {
            hipLaunchKernelGGL(k_pack_attr, dim3(grid_for(n, 256)), dim3(256), 0, st, attrs,
                               ix->attr, n, m, ix->abits);
        } else {
            (void)hipMemsetAsync(ix->attr, 0, (size_t)n * sizeof(uint32_t), st);
        }
        hipLaunchKernelGGL(k_row_norm, dim3(grid_for(n, 4)), dim3(256), 0, st, ix->vec32, ix->norm,
                           n, ix->dp);
        if (ix->storage == NHQ_STORAGE_FP32) {
            ix->vecs = ix->vec32;
        } else if (ix->storage == NHQ_STORAGE_BF16) {
            if (hipMalloc(&ix->vecs, cap_rows * sizeof(uint16_t)) != hipSuccess) {
                rc = fail(NHQ_ENOMEM, "bf16 storage allocation failed");
                break;
            }
            hipLaunchKernelGGL(k_to_bf16, dim3(grid_for((int64_t)rows, 256)), dim3(256), 0, st,
                               ix->vec32, (uint16_t *)ix->vecs, (int64_t)rows);
        } else {
            if (hipMalloc(&ix->vecs, cap_rows) != hipSuccess ||
                hipMalloc(&ix->scale, (size_t)ix->cap * sizeof(float)) != hipSuccess) {
                rc = fail(NHQ_ENOMEM, "fp8 storage allocation failed");
                break;
            }
            hipLaunchKernelGGL(k_to_fp8, dim3(grid_for(n, 1)), dim3(64), 0, st, ix->vec32,
                               (uint8_t *)ix->vecs, ix->scale, n, ix->dp);
        }
        if (hipGetLastError() != hipSuccess) {
            rc = fail(NHQ_EHIP, "ingest kernel launch failed");
            break;
        }
        // entry sample: first n_entry distinct splitmix64 values mod n
        const int64_t ne = std::min<int64_t>(p.n_entry, n);
        std::vector<int32_t> ent;
        ent.reserve((size_t)ne);
        std::unordered_set<int64_t> seen;
        uint64_t state = p.seed;
        while ((int64_t)ent.size() < ne) {
            const int64_t v = (int64_t)(splitmix64_next(state) % (uint64_t)n);
            if (seen.insert(v).second)
                ent.push_back((int32_t)v);
        }
        ix->n_entry = (int)ne;
        // stratified: per attribute pattern (packed word), the members with
        // the smallest (h(i), i) after the global ones
        if (p.entry_per_pattern > 0) {
            std::vector<uint32_t> aw((size_t)n);
            if (hipMemcpyAsync(aw.data(), ix->attr, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(NHQ_EHIP, "attribute read-back failed");
                break;
            }
            rc = stratify(aw, p.seed, p.entry_per_pattern, ent, ix->block_word_h, ix->block_off_h);
            if (rc != NHQ_OK)
                break;
            ix->n_blocks = (int)ix->block_word_h.size();
            ix->per_pattern = p.entry_per_pattern;
            if (hipMalloc(&ix->block_word, sizeof(uint32_t) * std::max<size_t>(1, ix->block_word_h.size())) !=
                    hipSuccess ||
                hipMalloc(&ix->block_off, sizeof(int32_t) * ix->block_off_h.size()) != hipSuccess ||
                hipMemcpy(ix->block_word, ix->block_word_h.data(), sizeof(uint32_t) * ix->block_word_h.size(),
                          hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(ix->block_off, ix->block_off_h.data(), sizeof(int32_t) * ix->block_off_h.size(),
                          hipMemcpyHostToDevice) != hipSuccess) {
                rc = fail(NHQ_ENOMEM, "entry block table allocation failed");
                break;
            }
        }
        const int64_t ne_all = (int64_t)ent.size();
        ix->n_entry_total = (int)ne_all;
        if (hipMalloc(&ix->entry, (size_t)ne_all * sizeof(int32_t)) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "entry allocation failed");
            break;
        }
        if (hipMemcpyAsync(ix->entry, ent.data(), (size_t)ne_all * sizeof(int32_t), hipMemcpyHostToDevice,
                           st) != hipSuccess) {
            rc = fail(NHQ_EHIP, "entry upload failed");
            break;
        }
        if (hipMalloc(&ix->entry_vec, (size_t)ne_all * ix->dp * sizeof(float)) != hipSuccess ||
            hipMalloc(&ix->entry_norm, (size_t)ne_all * sizeof(float)) != hipSuccess ||
            hipMalloc(&ix->entry_attr, (size_t)ne_all * sizeof(uint32_t)) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "entry sample allocation failed");
            break;
        }
        hipLaunchKernelGGL(k_gather_entry, dim3(grid_for(ne_all * ix->dp, 256)), dim3(256), 0, st, ix->entry,
                           (int)ne_all, ix->vec32, ix->norm, ix->attr, ix->dp, ix->entry_vec,
                           ix->entry_norm, ix->entry_attr);
        if (hipMalloc(&ix->entry_split, (size_t)ne_all * ix->dp * 2 * sizeof(uint16_t)) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "entry sample allocation failed");
            break;
        }
        if ((rc = launch_split_rows(ix->entry_vec, ne_all, ix->dp, ix->entry_split, st)) != NHQ_OK)
            break;
        if (hipMalloc(&ix->logp, sizeof(float) * hh.size()) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "histogram allocation failed");
            break;
        }
        std::vector<float> lp(hh.size());
        for (size_t t = 0; t < lp.size(); ++t)
            lp[t] = (float)std::log((hh[t] > 0 ? (double)hh[t] : 0.5) / (double)n);
        if (hipMemcpy(ix->logp, lp.data(), sizeof(float) * lp.size(), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(NHQ_EHIP, "log-frequency upload failed");
            break;
        }
        // exact bf16 copy of the entry sample (integer values of magnitude <= 256)
        if (ix->dp <= 128) {
            std::vector<float> ev((size_t)ne * ix->dp);
            if (hipMemcpy(ev.data(), ix->entry_vec, sizeof(float) * ev.size(), hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(NHQ_EHIP, "entry sample read-back failed");
                break;
            }
            bool exact = true;
            std::vector<uint16_t> eb(ev.size());
            for (size_t t = 0; t < ev.size() && exact; ++t) {
                const float v = ev[t];
                uint32_t bits;
                std::memcpy(&bits, &v, 4);
                exact = v == std::nearbyint(v) && std::fabs(v) <= 256.0f && (bits & 0xFFFFu) == 0;
                eb[t] = (uint16_t)(bits >> 16);
            }
            if (exact) {
                if (hipMalloc(&ix->entry_bf16, sizeof(uint16_t) * eb.size()) != hipSuccess ||
                    hipMemcpy(ix->entry_bf16, eb.data(), sizeof(uint16_t) * eb.size(), hipMemcpyHostToDevice) !=
                        hipSuccess) {
                    rc = fail(NHQ_ENOMEM, "bf16 entry sample allocation failed");
                    break;
                }
            }
        }
    } while (0);
    if (rc != NHQ_OK) {
        free_index(ix);
        delete h;
        return rc;
    }
    *out = h;
    return NHQ_OK;
}

int nhq_index_set_graph(nhq_index *h, const int32_t *adj, int32_t degree, void *stream)
{
    if (!h || !adj)
        return fail(NHQ_EINVAL, "null argument");
    Index *ix = &h->impl;
    if (degree < 1 || degree > NHQ_MAX_DEGREE)
        return fail(NHQ_EINVAL, "degree must be in [1, 64]");
    hipStream_t st = (hipStream_t)stream;
    if (degree != ix->degree) {
        NHQ_HIP(hipStreamSynchronize(st));
        if (ix->adj)
            NHQ_HIP(hipFree(ix->adj));
        ix->adj = nullptr;
        if (hipMalloc(&ix->adj, (size_t)ix->cap * degree * sizeof(int32_t)) != hipSuccess)
            return fail(NHQ_ENOMEM, "graph allocation failed");
        ix->degree = degree;
        if (ix->cap > ix->n)
            NHQ_HIP(hipMemsetAsync(ix->adj + ix->n * degree, 0xFF,
                                   (size_t)(ix->cap - ix->n) * degree * sizeof(int32_t), st));
    }
    NHQ_HIP(hipMemcpyAsync(ix->adj, adj, (size_t)ix->n * degree * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, st));
    return NHQ_OK;
}

int nhq_index_insert(nhq_index *h, const float *vecs, const uint8_t *attrs, int64_t nb, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    Index *ix = &h->impl;
    if (nb < 0)
        return fail(NHQ_EINVAL, "nb must be >= 0");
    if (nb == 0)
        return NHQ_OK;
    if (!vecs || (ix->m > 0 && !attrs))
        return fail(NHQ_EINVAL, "vecs/attrs is null");
    if (ix->n + nb > ix->cap)
        return fail(NHQ_EINVAL, "insertion beyond the index's capacity");
    if (ix->degree < 1)
        return fail(NHQ_EINVAL, "the index has no graph");
    hipStream_t st = (hipStream_t)stream;
    const int m = ix->m, d = ix->d, dp = ix->dp;
    if (m > 0) {
        std::vector<uint8_t> hc((size_t)nb * m);
        NHQ_HIP(hipMemcpyAsync(hc.data(), attrs, hc.size(), hipMemcpyDeviceToHost, st));
        NHQ_HIP(hipStreamSynchronize(st));
        int mx = 0;
        for (uint8_t c : hc)
            mx = std::max(mx, (int)c);
        if (mx == 255 || mx + 2 > (1 << ix->abits))
            return fail(NHQ_EINVAL, "attribute code too wide for the index's packed fields");
    }
    const int64_t s0 = ix->n;
    const size_t rows = (size_t)nb * dp;
    hipLaunchKernelGGL(k_pad_copy, dim3(grid_for((int64_t)rows, 256)), dim3(256), 0, st, vecs,
                       ix->vec32 + s0 * dp, nb, d, dp);
    if (m > 0)
        hipLaunchKernelGGL(k_pack_attr, dim3(grid_for(nb, 256)), dim3(256), 0, st, attrs, ix->attr + s0,
                           nb, m, ix->abits);
    else
        NHQ_HIP(hipMemsetAsync(ix->attr + s0, 0, (size_t)nb * sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_row_norm, dim3(grid_for(nb, 4)), dim3(256), 0, st, ix->vec32 + s0 * dp,
                       ix->norm + s0, nb, dp);
    if (ix->storage == NHQ_STORAGE_BF16)
        hipLaunchKernelGGL(k_to_bf16, dim3(grid_for((int64_t)rows, 256)), dim3(256), 0, st,
                           ix->vec32 + s0 * dp, (uint16_t *)ix->vecs + s0 * dp, (int64_t)rows);
    else if (ix->storage == NHQ_STORAGE_FP8)
        hipLaunchKernelGGL(k_to_fp8, dim3(grid_for(nb, 1)), dim3(64), 0, st, ix->vec32 + s0 * dp,
                           (uint8_t *)ix->vecs + s0 * dp, ix->scale + s0, nb, dp);
    NHQ_HIP(hipGetLastError());
    ix->n = s0 + nb;
    return nsw_insert(ix, s0, s0 + nb, ix->cand, ix->nsw_batch, std::max(ix->nsw_beam, ix->cand), ix->seed,
                      st);
}

int nhq_index_get_graph(const nhq_index *h, int32_t *adj_out, void *stream)
{
    if (!h || !adj_out)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    NHQ_HIP(hipMemcpyAsync(adj_out, ix->adj, (size_t)ix->n * ix->degree * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return NHQ_OK;
}

int nhq_index_entry_blocks(const nhq_index *h, int32_t *n_blocks, uint8_t *codes, int32_t *offsets,
                           int32_t *ids, void *stream)
{
    if (!h || !n_blocks)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    const int B = ix->n_blocks;
    *n_blocks = B;
    if (codes) {
        const uint32_t fm = (1u << ix->abits) - 1u;
        for (int b = 0; b < B; ++b)
            for (int i = 0; i < ix->m; ++i)
                codes[(size_t)b * ix->m + i] = (uint8_t)((ix->block_word_h[b] >> (ix->abits * i)) & fm);
    }
    if (offsets)
        for (int b = 0; b <= B; ++b)
            offsets[b] = B > 0 ? ix->block_off_h[b] : ix->n_entry;
    if (ids && B > 0) {
        const size_t cnt = (size_t)(ix->block_off_h[B] - ix->n_entry);
        NHQ_HIP(hipMemcpyAsync(ids, ix->entry + ix->n_entry, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
        NHQ_HIP(hipStreamSynchronize((hipStream_t)stream));
    }
    return NHQ_OK;
}

int nhq_index_get_entry(const nhq_index *h, int32_t *entry_out, void *stream)
{
    if (!h || !entry_out)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    NHQ_HIP(hipMemcpyAsync(entry_out, ix->entry, (size_t)ix->n_entry * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return NHQ_OK;
}

int nhq_index_get_storage(const nhq_index *h, void *rows_out, float *scales_out, int32_t *dp_out,
                          void *stream)
{
    if (!h || !rows_out)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    const size_t elem = ix->storage == NHQ_STORAGE_FP32 ? 4 : (ix->storage == NHQ_STORAGE_BF16 ? 2 : 1);
    hipStream_t st = (hipStream_t)stream;
    NHQ_HIP(hipMemcpyAsync(rows_out, ix->vecs, (size_t)ix->n * ix->dp * elem, hipMemcpyDeviceToDevice, st));
    if (scales_out && ix->storage == NHQ_STORAGE_FP8)
        NHQ_HIP(hipMemcpyAsync(scales_out, ix->scale, (size_t)ix->n * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (dp_out)
        *dp_out = ix->dp;
    return NHQ_OK;
}

int nhq_index_info(const nhq_index *h, int64_t *n, int32_t *d, int32_t *m, int32_t *degree,
                   int32_t *storage, int32_t *n_entry)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    const Index *ix = &h->impl;
    if (n)
        *n = ix->n;
    if (d)
        *d = ix->d;
    if (m)
        *m = ix->m;
    if (degree)
        *degree = ix->degree;
    if (storage)
        *storage = ix->storage;
    if (n_entry)
        *n_entry = ix->n_entry;
    return NHQ_OK;
}

int nhq_index_device_error(nhq_index *h, void *stream, uint32_t *bits_out)
{
    if (!h || !bits_out)
        return fail(NHQ_EINVAL, "null argument");
    Index *ix = &h->impl;
    hipStream_t st = (hipStream_t)stream;
    uint32_t bits = 0;
    NHQ_HIP(hipMemcpyAsync(&bits, ix->err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    NHQ_HIP(hipStreamSynchronize(st));
    NHQ_HIP(hipMemsetAsync(ix->err, 0, sizeof(uint32_t), st));
    *bits_out = bits;
    return NHQ_OK;
}

void nhq_index_free(nhq_index *h)
{
    if (!h)
        return;
    (void)hipDeviceSynchronize();
    free_index(&h->impl);
    delete h;
}

}  // extern "C"

namespace {

// ---- launch orders: by selectivity (nhq_query_order) and by seed
// (nhq_seed_order), a counting sort over kOrderBuckets buckets
constexpr int kOrderBuckets = 1024;

// selectivity: buckets of 1/16 of -sum ln(count / n) over the constrained codes
struct SelectivityBucket {
    const uint8_t *qa;
    int m;
    const float *logp;
    __device__ int operator()(int64_t q) const
    {
        float ls = 0.0f;
        for (int i = 0; i < m; ++i) {
            const uint32_t c = qa[q * m + i];
            if (c != 0xFFu)
                ls += logp[i * 256 + c];
        }
        return (int)fminf(fmaxf(-ls * 16.0f, 0.0f), (float)(kOrderBuckets - 1));
    }
};

// seed: the lowest entry-sample position among the query's candidates (a
// member of its seed neighbourhood that many queries of one region share:
// measured, grouping by it keeps more of a batch's row reads in L2 than
// grouping by the best candidate), n_total positions spread over the
// buckets (no candidate: the last position's bucket), the buckets then
// permuted by an odd multiplier mod 1,024.  Neighbouring positions (one
// attribute pattern's block of a stratified sample) land far apart, so each
// XCD's run of the sorted queries mixes many buckets of every kind, and
// their cost evens out across XCDs; the queries of one bucket stay
// together.
struct SeedBucket {
    const int32_t *cand;
    int n_cand;
    int64_t n_total;
    __device__ int operator()(int64_t q) const
    {
        static_assert(kOrderBuckets == 1024, "the permutation is mod 1024");
        int64_t lo = n_total;
        for (int j = 0; j < n_cand; ++j) {
            const int32_t p = cand[q * n_cand + j];
            if (p >= 0 && p < lo)
                lo = p;
        }
        const int b = lo >= n_total ? kOrderBuckets - 1 : (int)(lo * kOrderBuckets / n_total);
        return (b * 757 + 419) & (kOrderBuckets - 1);
    }
};

__global__ void k_order_clear(int32_t *hist)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kOrderBuckets)
        hist[t] = 0;
}

// each query's bucket, and its position among the bucket's queries: counts
// in an LDS histogram, then one global atomic per (workgroup, bucket)
// reserves the workgroup's run of positions
template <class BucketOf>
__global__ __launch_bounds__(256) void k_order_assign(const BucketOf bucket_of, int64_t nq,
                                                      int32_t *__restrict__ bucket, int32_t *__restrict__ pos,
                                                      int32_t *__restrict__ hist)
{
    __shared__ int32_t lh[kOrderBuckets];
    for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x)
        lh[t] = 0;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = q < nq;
    int b = 0, r = 0;
    if (live) {
        b = bucket_of(q);
        r = atomicAdd(&lh[b], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kOrderBuckets; t += blockDim.x)
        if (lh[t] > 0)
            lh[t] = atomicAdd(&hist[t], lh[t]);
    __syncthreads();
    if (live) {
        bucket[q] = b;
        pos[q] = lh[b] + r;
    }
}

// bucket starts (exclusive scan by one wavefront: each lane sums a run of
// kOrderBuckets / 64 buckets, a wave prefix sum of the runs gives their
// starts, and each lane writes its run's starts)
__global__ __launch_bounds__(64) void k_order_scan(int32_t *hist)
{
    constexpr int kRun = kOrderBuckets / 64;
    static_assert(kRun * 64 == kOrderBuckets, "whole runs");
    const int lane = threadIdx.x;
    int32_t c[kRun];
    int32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
        c[u] = hist[lane * kRun + u];
        sum += c[u];
    }
    int32_t incl = sum;  // inclusive prefix over lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t v = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += v;
    }
    int32_t run = incl - sum;
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
        hist[lane * kRun + u] = run;
        run += c[u];
    }
}

// The wavefront that runs sorted position p when a batch of n one-wave
// workgroups keeps each XCD on a contiguous run of the sorted queries:
// workgroups go to the 8 XCDs round-robin (workgroup i to XCD i mod 8), and
// XCD x takes the x-th of 8 contiguous runs (the first n mod 8 runs one
// longer).  A bijection of 0 .. n - 1.
__device__ __forceinline__ int64_t xcd_wave(int64_t p, int64_t n)
{
    constexpr int kXcd = 8;
    const int64_t base = n / kXcd, r = n % kXcd;
    int64_t x, j;
    if (p < r * (base + 1)) {
        x = p / (base + 1);
        j = p - x * (base + 1);
    } else {
        const int64_t pp = p - r * (base + 1);
        x = r + pp / base;
        j = pp - (x - r) * base;
    }
    return x + kXcd * j;
}

// order[wave] = q for each query's sorted position (xcd: the wave that
// runs that position on its XCD's run, else the position itself)
__global__ void k_order_place(const int32_t *__restrict__ bucket, const int32_t *__restrict__ pos,
                              const int32_t *__restrict__ start, int64_t nq, int xcd,
                              int32_t *__restrict__ order)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) {
        const int64_t p = start[bucket[q]] + pos[q];
        order[xcd ? xcd_wave(p, nq) : p] = (int32_t)q;
    }
}

// a launch order by counting sort: scratch of kOrderBuckets + 2 nq words
template <class BucketOf>
int launch_order(const BucketOf &bucket_of, int64_t nq, int xcd, int32_t *scratch, int32_t *order, hipStream_t st)
{
    int32_t *hist = scratch, *bucket = scratch + kOrderBuckets, *pos = bucket + nq;
    const unsigned g = (unsigned)((nq + 255) / 256);
    hipLaunchKernelGGL(k_order_clear, dim3(kOrderBuckets / 256), dim3(256), 0, st, hist);
    hipLaunchKernelGGL(k_order_assign<BucketOf>, dim3(g), dim3(256), 0, st, bucket_of, nq, bucket, pos, hist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, st, hist);
    hipLaunchKernelGGL(k_order_place, dim3(g), dim3(256), 0, st, bucket, pos, hist, nq, xcd, order);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

// batches from this size on are launched grouped by seed candidate when the
// caller gives no order (smaller ones gain less than the order costs)
constexpr int64_t kSeedOrderMinQueries = 2048;

// 32-bit words of a launch order's scratch
size_t order_words(int64_t nq)
{
    return (size_t)kOrderBuckets + 2 * (size_t)nq;
}

// the order grouping queries by the lowest entry position among their seed
// candidates, each group's waves on one XCD (queries that share a seed
// candidate search one part of the graph, so their row gathers share that
// XCD's L2)
int seed_order_at(const Index *ix, const int32_t *cand, int n_cand, int64_t nq, int32_t *order,
                  int32_t *scratch, hipStream_t st)
{
    const int64_t n_total = std::max(ix->n_entry_total, ix->n_entry);
    return launch_order(SeedBucket{cand, n_cand, n_total}, nq, 1, scratch, order, st);
}

// 32-bit words of the seed ranking's scratch: padded rows, norms, codes,
// masks, exactness flags, split rows (each 2 dp bf16 halves, 256-byte
// aligned) and (for the matrix-core ranking) the key matrix and its group
// minima
size_t seed_rank_words(const Index *ix, int64_t nq, int K)
{
    const size_t ne_pad = (size_t)(ix->n_entry + 63) / 64 * 64;
    const bool dense = ix->n_entry <= 8192;
    const size_t pad = 2 * (size_t)nq * ix->dp + 5 * (size_t)nq + 128;
    // the same scratch serves the seed order afterwards (nhq_seed_order)
    if (ix->n_blocks > 0)
        return std::max(order_words(nq), pad + strata_rank_words(ix, nq, K));
    return std::max(order_words(nq), pad + (dense ? (size_t)nq * ne_pad / 16 * 17 : 0));
}

int check_seed_rank_args(const Index *ix, const float *queries, const uint8_t *qattrs, int64_t nq,
                         int32_t n_cand, const int32_t *cand)
{
    if (nq < 0 || n_cand < 1 || n_cand > 144)
        return fail(NHQ_EINVAL, "need nq >= 0 and 1 <= n_cand <= 144");
    if (nq > 0 && (!queries || !cand || (ix->m > 0 && !qattrs)))
        return fail(NHQ_EINVAL, "null array argument");
    return NHQ_OK;
}

// the seed ranking with its scratch (seed_rank_words(ix, nq) words, 256-byte
// aligned) at blk; allocates nothing
int seed_rank_at(const Index *cix, const float *queries, const uint8_t *qattrs, int64_t nq, int32_t n_cand,
                 int32_t *cand, hipStream_t st, uint32_t *blk)
{
    Index *ix = const_cast<Index *>(cix);
    const bool dense = ix->n_entry <= 8192;
    const size_t f_rows = (size_t)nq * ix->dp, f_small = (size_t)nq;
    float *qpad = reinterpret_cast<float *>(blk);
    float *qnorm = qpad + f_rows;
    uint32_t *qw = reinterpret_cast<uint32_t *>(qnorm + f_small);
    uint32_t *qm = qw + f_small;
    uint32_t *qx = qm + f_small;
    uint16_t *qs =
        reinterpret_cast<uint16_t *>((reinterpret_cast<uintptr_t>(qx + f_small) + 255) & ~uintptr_t(255));
    float *keys = reinterpret_cast<float *>(
        (reinterpret_cast<uintptr_t>(qs + 2 * f_rows) + 255) & ~uintptr_t(255));
    // split rows only where the matrix-core ranking reads them; padded
    // float32 rows only for the exact bf16 kernel and the float32 tiles
    const bool need_pad = ix->n_blocks == 0 && (!dense || (ix->entry_bf16 != nullptr && ix->dp <= 128));
    int rc = launch_pad_queries(queries, qattrs, nq, ix->d, ix->dp, ix->m, ix->abits, need_pad ? qpad : nullptr,
                                qnorm, qw, qm, qx, (ix->n_blocks > 0 || dense) ? qs : nullptr, st);
    if (rc == NHQ_OK) {
        if (ix->n_blocks > 0)
            rc = launch_strata_rank(ix, qs, qnorm, qw, qm, nq, n_cand, reinterpret_cast<uint32_t *>(keys),
                                    cand, st);
        else if (dense)
            rc = launch_seed_rank(ix, qpad, qs, qnorm, qw, qm, qx, nq, n_cand, keys, cand, st);
        else
            rc = launch_dense_topk(qpad, qnorm, qw, qm, nq, ix->entry_vec, ix->entry_norm, ix->entry_attr,
                                   ix->n_entry, ix->dp, ix->m, ix->abits, 0, 0, n_cand, cand, nullptr, st,
                                   &ix->w);
    }
    return rc;
}

// nhq_seed_rank with its scratch at byte ws_off of the index's workspace
// (grown when too small; calls on one index are ordered on one stream, so
// the workspace is theirs in turn)
int seed_rank_ws(const nhq_index *h, const float *queries, const uint8_t *qattrs, int64_t nq, int32_t n_cand,
                 int32_t *cand, void *stream, size_t ws_off)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    Index *ix = const_cast<Index *>(&h->impl);
    int rc = check_seed_rank_args(ix, queries, qattrs, nq, n_cand, cand);
    if (rc != NHQ_OK || nq == 0)
        return rc;
    rc = ensure_workspace(ix, ws_off + sizeof(uint32_t) * seed_rank_words(ix, nq, n_cand));
    if (rc != NHQ_OK)
        return rc;
    uint32_t *blk = reinterpret_cast<uint32_t *>(static_cast<char *>(ix->ws) + ws_off);
    return seed_rank_at(ix, queries, qattrs, nq, n_cand, cand, (hipStream_t)stream, blk);
}

// ---- the fixed scratch of nhq_hybrid_search_noalloc: one array in every
// device's memory (each device that runs the library holds its own copy
// until the process ends).  Host code never passes `scratch` itself to a
// kernel (on the host the name is only a stand-in for the symbol); it takes
// each device's address once, with that device current, and uses that.
__device__ __align__(256) uint8_t scratch[NHQ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

int scratch_of_device(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(NHQ_ENOTSUP, "device ordinal beyond the library's scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        NHQ_HIP(hipGetDevice(&cur));
        if (cur != dev)
            NHQ_HIP(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev)
            (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return fail(NHQ_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return NHQ_OK;
}

}  // namespace

extern "C" {

int nhq_seed_rank(const nhq_index *h, const float *queries, const uint8_t *qattrs, int64_t nq,
                  int32_t n_cand, int32_t *cand, void *stream)
{
    return seed_rank_ws(h, queries, qattrs, nq, n_cand, cand, stream, 0);
}

int nhq_seed_rank_workspace_size(const nhq_index *h, int64_t nq, int32_t n_cand, size_t *bytes)
{
    if (!h || !bytes)
        return fail(NHQ_EINVAL, "null argument");
    if (nq < 0 || n_cand < 1 || n_cand > 144)
        return fail(NHQ_EINVAL, "need nq >= 0 and 1 <= n_cand <= 144");
    *bytes = sizeof(uint32_t) * seed_rank_words(&h->impl, nq, n_cand);
    return NHQ_OK;
}

int nhq_seed_rank_ws(const nhq_index *h, const float *queries, const uint8_t *qattrs, int64_t nq,
                     int32_t n_cand, int32_t *cand, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    const Index *ix = &h->impl;
    int rc = check_seed_rank_args(ix, queries, qattrs, nq, n_cand, cand);
    if (rc != NHQ_OK || nq == 0)
        return rc;
    const size_t need = sizeof(uint32_t) * seed_rank_words(ix, nq, n_cand);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0 || workspace_bytes < need)
        return fail(NHQ_EINVAL, "workspace: need 256-byte aligned device memory of " + std::to_string(need) +
                                    " bytes (nhq_seed_rank_workspace_size)");
    return seed_rank_at(ix, queries, qattrs, nq, n_cand, cand, (hipStream_t)stream,
                        static_cast<uint32_t *>(workspace));
}

int nhq_search_seeded(const nhq_index *h, const float *queries, const uint8_t *qattrs, int64_t nq,
                      const int32_t *cand, int32_t n_cand, int32_t k, int32_t beam,
                      const nhq_search_params *sp, int32_t *ids, float *dists, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    const Index *ix = &h->impl;
    if (nq < 0)
        return fail(NHQ_EINVAL, "nq < 0");
    if (nq == 0)
        return NHQ_OK;
    if (!queries || !ids || !dists || !cand || (ix->m > 0 && !qattrs))
        return fail(NHQ_EINVAL, "null array argument");
    if (n_cand < 1 || n_cand > 1024)
        return fail(NHQ_EINVAL, "need 1 <= n_cand <= 1024");
    if (k < 1 || beam < k || beam > NHQ_MAX_BEAM)
        return fail(NHQ_EINVAL, "need 1 <= k <= beam <= 1024");
    nhq_search_params p{};
    if (sp)
        p = *sp;
    if (p.n_init == 0)
        p.n_init = 32;
    if (p.max_hops == 0)
        p.max_hops = 100000;
    if (p.stop_threshold == 0.0f)
        p.stop_threshold = 0.5f;
    if (!(p.stop_threshold > 0.0f && p.stop_threshold < 1.0f))
        return fail(NHQ_EINVAL, "stop_threshold must be in (0, 1)");
    if (p.trace && (p.trace->cap < 1 || !p.trace->feat || !p.trace->hop || !p.trace->hash ||
                    !p.trace->count || !p.trace->final_hash))
        return fail(NHQ_EINVAL, "incomplete trace buffers");
    if (p.check_every == 0)
        p.check_every = 4;
    if (p.expand == 0)
        p.expand = 1;
    if (p.expand < 1 || p.expand > 8)
        return fail(NHQ_EINVAL, "expand must be in [1, 8]");
    if (p.check_every < 1)
        return fail(NHQ_EINVAL, "check_every must be positive");
    if (p.n_init < 1 || p.n_init > 128 || p.max_hops < 1)
        return fail(NHQ_EINVAL, "need 1 <= n_init <= 128 and max_hops >= 1");
    if (p.output_mode != 0 && p.output_mode != 1)
        return fail(NHQ_EINVAL, "output_mode must be 0 or 1");
    if (p.rerank < 0 || p.rerank > 64)
        return fail(NHQ_EINVAL, "rerank must be in [0, 64]");
    if (p.visited_log2 != 0 && (p.visited_log2 < 10 || p.visited_log2 > 13))
        return fail(NHQ_EINVAL, "visited_log2 must be 0 or in [10, 13]");
    if (p.route_h < 0 || p.route_h > NHQ_MAX_DEGREE)
        return fail(NHQ_EINVAL, "route_h must be in [0, 64]");
    if (p.learned < 0 || p.learned > 3)
        return fail(NHQ_EINVAL, "learned must be 0, 1, 2 or 3");
    if (p.learned && !ix->mlp)
        return fail(NHQ_EINVAL, "learned stop requested but no network is loaded");
    if (p.learned == 2 && !(p.cap_factor > 0.0f))
        return fail(NHQ_EINVAL, "learned mode 2 needs cap_factor > 0 (its hop budget)");
    if (p.learned == 3 && !(p.cap_factor > 0.0f))
        return fail(NHQ_EINVAL, "learned mode 3 needs cap_factor > 0 (its pool size factor)");
    SearchLaunch s{};
    s.ix = ix;
    s.seed_cand = cand;
    s.n_seed_cand = n_cand;
    s.q = queries;
    s.qa = qattrs;
    s.nq = nq;
    s.k = k;
    s.L = beam;
    s.n_init = p.n_init;
    s.out_mode = p.output_mode;
    s.rerank_n = (int)std::min<int64_t>((int64_t)p.rerank * k, beam);
    s.max_hops = p.max_hops;
    s.hash_log2 = p.visited_log2;
    s.learned = p.learned;
    s.check_every = p.check_every;
    s.stop_logit = logf(p.stop_threshold / (1.0f - p.stop_threshold));
    s.cap_factor = p.cap_factor;
    s.expand = p.expand;
    s.route_h = p.route_h;
    s.trace = p.trace;
    s.ids = ids;
    s.dists = dists;
    s.counters = p.counters;
    s.order = p.order;
    s.stream = (hipStream_t)stream;
    return launch_search(s);
}

int nhq_query_order(const nhq_index *h, const uint8_t *qattrs, int64_t nq, int32_t *order, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    Index *ix = const_cast<Index *>(&h->impl);
    if (nq < 0 || nq > 0x7FFFFFFF)
        return fail(NHQ_EINVAL, "need 0 <= nq < 2^31");
    if (nq == 0)
        return NHQ_OK;
    if (!order || (ix->m > 0 && !qattrs))
        return fail(NHQ_EINVAL, "null array argument");
    // workspace: bucket counts (then starts) [1024], bucket [nq], position [nq]
    int rc = ensure_workspace(ix, sizeof(int32_t) * order_words(nq));
    if (rc != NHQ_OK)
        return rc;
    return launch_order(SelectivityBucket{qattrs, ix->m, ix->logp}, nq, 0, static_cast<int32_t *>(ix->ws), order,
                        (hipStream_t)stream);
}

int nhq_seed_order(const nhq_index *h, const int32_t *cand, int32_t n_cand, int64_t nq, int32_t *order,
                   void *workspace, size_t workspace_bytes, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    Index *ix = const_cast<Index *>(&h->impl);
    if (nq < 0 || nq > 0x7FFFFFFF || n_cand < 1)
        return fail(NHQ_EINVAL, "need 0 <= nq < 2^31 and n_cand >= 1");
    if (nq == 0)
        return NHQ_OK;
    if (!order || !cand)
        return fail(NHQ_EINVAL, "null array argument");
    int32_t *scratch = static_cast<int32_t *>(workspace);
    if (!scratch) {
        const int rc = ensure_workspace(ix, sizeof(int32_t) * order_words(nq));
        if (rc != NHQ_OK)
            return rc;
        scratch = static_cast<int32_t *>(ix->ws);
    } else if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0 ||
               workspace_bytes < sizeof(int32_t) * order_words(nq)) {
        return fail(NHQ_EINVAL, "workspace: need 256-byte aligned device memory of " +
                                    std::to_string(sizeof(int32_t) * order_words(nq)) + " bytes");
    }
    return seed_order_at(ix, cand, n_cand, nq, order, scratch, (hipStream_t)stream);
}

int nhq_hybrid_search(const nhq_index *h, const float *queries, const uint8_t *qattrs, int64_t nq,
                      int32_t k, int32_t beam, const nhq_search_params *sp, int32_t *ids,
                      float *dists, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    const Index *ix = &h->impl;
    if (nq < 0)
        return fail(NHQ_EINVAL, "nq < 0");
    if (nq == 0)
        return NHQ_OK;
    const int n_init = (sp && sp->n_init > 0) ? sp->n_init : 32;
    if (n_init > 128)
        return fail(NHQ_EINVAL, "need 1 <= n_init <= 128");
    const int ks = std::min(std::max(ix->n_entry, ix->n_blocks > 0 ? ix->per_pattern : 0), n_init + kSeedMargin);
    // the candidates and the launch order at the start of the index's
    // workspace, the ranking's scratch (then the order's) after them
    nhq_search_params p{};
    if (sp)
        p = *sp;
    const bool order = p.order == nullptr && nq >= kSeedOrderMinQueries;
    const size_t cbytes = (sizeof(int32_t) * (size_t)nq * ks + 255) & ~size_t(255);
    const size_t obytes = order ? (sizeof(int32_t) * (size_t)nq + 255) & ~size_t(255) : 0;
    Index *mix = const_cast<Index *>(ix);
    int rc = ensure_workspace(mix, cbytes + obytes + sizeof(uint32_t) * seed_rank_words(ix, nq, ks));
    if (rc != NHQ_OK)
        return rc;
    int32_t *cand = static_cast<int32_t *>(mix->ws);
    rc = seed_rank_ws(h, queries, qattrs, nq, ks, cand, stream, cbytes + obytes);
    if (rc == NHQ_OK && order) {
        int32_t *ord = reinterpret_cast<int32_t *>(static_cast<char *>(mix->ws) + cbytes);
        rc = seed_order_at(ix, cand, ks, nq, ord,
                           reinterpret_cast<int32_t *>(static_cast<char *>(mix->ws) + cbytes + obytes),
                           (hipStream_t)stream);
        p.order = ord;
    }
    if (rc == NHQ_OK)
        rc = nhq_search_seeded(h, queries, qattrs, nq, cand, ks, k, beam, &p, ids, dists, stream);
    return rc;
}

int nhq_hybrid_search_noalloc(const nhq_index *h, const float *queries, const uint8_t *qattrs,
                              int64_t nq, int32_t k, int32_t beam, const nhq_search_params *sp,
                              int32_t *ids, float *dists, void *stream)
{
    if (!h)
        return fail(NHQ_EINVAL, "null index");
    const Index *ix = &h->impl;
    if (nq < 0)
        return fail(NHQ_EINVAL, "nq < 0");
    if (nq == 0)
        return NHQ_OK;
    if (ix->n_entry > 8192)
        return fail(NHQ_ENOTSUP, "the allocation-free search needs an entry sample of at most 8192");
    const int n_init = (sp && sp->n_init > 0) ? sp->n_init : 32;
    if (n_init > 128)
        return fail(NHQ_EINVAL, "need 1 <= n_init <= 128");
    const int ks = std::min(std::max(ix->n_entry, ix->n_blocks > 0 ? ix->per_pattern : 0), n_init + kSeedMargin);
    int rc = check_seed_rank_args(ix, queries, qattrs, nq, ks, ids);
    if (rc != NHQ_OK)
        return rc;
    // the candidates at the start of the scratch, the ranking's scratch after them
    const size_t cbytes = (sizeof(int32_t) * (size_t)nq * ks + 255) & ~size_t(255);
    const size_t need = cbytes + sizeof(uint32_t) * seed_rank_words(ix, nq, ks);
    if (need > (size_t)NHQ_NOALLOC_SCRATCH_BYTES)
        return fail(NHQ_EINVAL, "batch too large for the allocation-free search: it needs " +
                                    std::to_string(need) + " bytes of scratch, the fixed scratch holds " +
                                    std::to_string((size_t)NHQ_NOALLOC_SCRATCH_BYTES) +
                                    "; split the batch");
    void *base = nullptr;
    rc = scratch_of_device(ix->device, &base);
    if (rc != NHQ_OK)
        return rc;
    int32_t *cand = static_cast<int32_t *>(base);
    uint32_t *blk = reinterpret_cast<uint32_t *>(static_cast<char *>(base) + cbytes);
    rc = seed_rank_at(ix, queries, qattrs, nq, ks, cand, (hipStream_t)stream, blk);
    if (rc == NHQ_OK)
        rc = nhq_search_seeded(h, queries, qattrs, nq, cand, ks, k, beam, sp, ids, dists, stream);
    return rc;
}

}  // extern "C"
