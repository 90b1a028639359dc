// Serving loop with continuous batching: hybrid queries (Def. 4) answered by
// joint pruning (Alg. 2) from a stream of requests, each with its own k,
// beam and constrained attributes.
//
// One persistent launch serves every memory class (a class is the largest
// beam its slots hold; a request goes to the smallest class that holds its
// beam, and each class has its own ring).  Workgroup c < ncls is class c's
// doorbell: it reads the class ring's tail (pinned host memory) and marks the
// newly published ring entries ready in device memory.  Every other
// workgroup is one wavefront, one slot of a class: it takes the next request
// index
// (device atomic), waits until that entry is ready, reads the request from
// the host ring, ranks the entry sample for the query itself, runs the same
// per-query search as the batch kernel, writes the results into the host
// output record and releases its completion word at system scope.  A slot
// takes the next request as soon as it finishes one, so requests that
// arrive while others run are admitted at once and share the device with
// them.  A request's result depends only on the request, the index and the
// server parameters: each slot owns its pool and visited set.
//
// Every wait in the kernel is bounded: by the host's stop flag and by a
// wall-clock lifetime after which the kernel ends on its own.
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "search_core.h"
#include "wave_select.h"

namespace nhq {
namespace {

// request record in the host ring: header, then the query's d floats
struct ReqHead {
    int32_t k, L, flags, rerank_n;
    uint32_t qword, qmask;
    int32_t max_hops, reserved;
};
static_assert(sizeof(ReqHead) == 32, "request header layout");

// output record in host memory: header, then ids [max_k] and dists [max_k]
struct OutHead {
    unsigned long long done;  // request index + 1 once the record is complete
    unsigned long long t_begin, t_end;  // device wall clock
    uint32_t ndc, hops;
};
static_assert(sizeof(OutHead) == 32, "output header layout");

constexpr int kReqLearned = 2;  // internal request flag (beam 0 requests); bit 0 is NHQ_SERVE_RAW

struct ServeArgs {
    const uint8_t *ring;             // host: cap request records
    uint8_t *outs;                   // host: cap output records
    const unsigned long long *tail;  // host: requests published so far
    const uint32_t *stop;            // host: nonzero asks the kernel to end
    uint32_t *status;                // host: why the doorbell ended (1 stop, 2 lifetime)
    unsigned long long *next;        // device: next request index to take
    unsigned long long *ready;       // device [cap]: index + 1 once published
    uint32_t *stop_dev;              // device: copy of the stop reason
    int cap, rec_bytes, out_bytes, max_k;
    int n_cand, ne_pad, seed_off, check_every;
    int learned_mode;
    unsigned long long life_ticks;
};

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__device__ void doorbell(const ServeArgs &s, unsigned long long t_end)
{
    const int lane = threadIdx.x & 63;
    unsigned long long last = 0;
    uint32_t why = 0;
    for (;;) {
        // relaxed polls (an acquire would invalidate caches on every poll);
        // one acquire fence once new entries are seen
        unsigned long long t = 0;
        uint32_t stop = 0;
        if (lane == 0) {
            t = __hip_atomic_load(s.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            stop = __hip_atomic_load(s.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        t = bcast64(t);
        stop = (uint32_t)__builtin_amdgcn_readfirstlane((int)stop);
        if (t > last)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        for (unsigned long long idx = last + lane; idx < t; idx += 64)
            __hip_atomic_store(s.ready + (idx % (unsigned)s.cap), idx + 1, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (t > last)
            last = t;
        if (stop) {
            why = 1;
            break;
        }
        if (wall_clock64() > t_end) {
            why = 2;
            break;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    if (lane == 0) {
        __hip_atomic_store(s.stop_dev, why, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(s.status, why, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Keys of the whole entry sample for one query, direct form from the float32
// rows (lane per entry, four entries per pass), as bit patterns into kb.
template <int DP>
__device__ void entry_keys_wave(const float *ev, const uint32_t *ea, int ne, const float *qlds,
                                uint32_t qword, uint32_t qmask, const Weights &w, int abits,
                                uint32_t hmask, uint32_t *kb)
{
    const int lane = threadIdx.x & 63;
    const int mq = __popc(qmask) / abits;
    const float4 *q4 = reinterpret_cast<const float4 *>(qlds);
    for (int e0 = 0; e0 < ne; e0 += 256) {
        const float4 *row[4];
        float acc[4];
        uint32_t at[4];  // attribute words, loaded with the rows
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = min(e0 + 64 * r + lane, ne - 1);
            row[r] = reinterpret_cast<const float4 *>(ev + (int64_t)e * DP);
            at[r] = ea[e];
            acc[r] = 0.0f;
        }
#pragma unroll 4
        for (int c = 0; c < DP / 4; ++c) {
            const float4 qq = q4[c];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float4 x = row[r][c];
                const float t0 = qq.x - x.x, t1 = qq.y - x.y, t2 = qq.z - x.z, t3 = qq.w - x.w;
                acc[r] = fmaf(t0, t0, acc[r]);
                acc[r] = fmaf(t1, t1, acc[r]);
                acc[r] = fmaf(t2, t2, acc[r]);
                acc[r] = fmaf(t3, t3, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = e0 + 64 * r + lane;
            if (e < ne)
                kb[e] = __float_as_uint(w_key32(acc[r], chi_of(at[r], qword, qmask, hmask), mq, w));
        }
    }
}

// The classes of one server in one launch: workgroups 0 .. ncls - 1 are
// their doorbells, then come class 0's slots0 slots and class 1's.  Two
// persistent launches on two streams could share a hardware queue, and then
// the second would wait for the first to end; one launch keeps every class
// running side by side.  The launch's LDS per workgroup is the largest
// class's.
struct ServeLaunch {
    ServeArgs c[2];
    int ncls, slots0;
};

template <int DP, int ST>
__global__ __launch_bounds__(64) void k_serve(const SearchArgs base, const ServeLaunch L)
{
    extern __shared__ __align__(16) uint32_t smem[];
    const int lane = threadIdx.x & 63;
    const int b = (int)blockIdx.x;
    if (b < L.ncls) {
        const ServeArgs &d = b == 0 ? L.c[0] : L.c[1];
        doorbell(d, wall_clock64() + d.life_ticks);
        return;
    }
    const ServeArgs s = b - L.ncls < L.slots0 ? L.c[0] : L.c[1];
    const unsigned long long t_end = wall_clock64() + s.life_ticks;
    float *qlds = reinterpret_cast<float *>(smem + s.seed_off);
    int32_t *seedpos = reinterpret_cast<int32_t *>(smem + s.seed_off + DP);
    uint32_t *kb = smem + s.seed_off + DP + 160;
    uint32_t *cv = kb + s.ne_pad;
    int32_t *cp = reinterpret_cast<int32_t *>(cv + 256);
    for (;;) {
        unsigned long long i = 0;
        if (lane == 0)
            i = atomicAdd(s.next, 1ull);
        i = bcast64(i);
        const int slot = (int)(i % (unsigned)s.cap);
        bool go = false;
        for (int polls = 0;; ++polls) {
            unsigned long long r = 0;
            if (lane == 0)  // relaxed: an acquire per poll would invalidate the CU's L1
                r = __hip_atomic_load(s.ready + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            r = bcast64(r);
            if (r == i + 1) {
                go = true;
                break;
            }
            if ((polls & 31) == 31) {
                uint32_t st = 0;
                if (lane == 0)
                    st = __hip_atomic_load(s.stop_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st = (uint32_t)__builtin_amdgcn_readfirstlane((int)st);
                if (st != 0 || wall_clock64() > t_end)
                    break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        if (!go)
            return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const unsigned long long t_begin = wall_clock64();
        const uint8_t *rec = s.ring + (size_t)slot * s.rec_bytes;
        // header words via lanes 0..7, then broadcast
        const uint32_t hw = lane < 8 ? reinterpret_cast<const uint32_t *>(rec)[lane] : 0u;
        const int k = __builtin_amdgcn_readlane((int)hw, 0);
        const int L = __builtin_amdgcn_readlane((int)hw, 1);
        const int flags = __builtin_amdgcn_readlane((int)hw, 2);
        const int rr = __builtin_amdgcn_readlane((int)hw, 3);
        const uint32_t qword = (uint32_t)__builtin_amdgcn_readlane((int)hw, 4);
        const uint32_t qmask = (uint32_t)__builtin_amdgcn_readlane((int)hw, 5);
        const int max_hops = __builtin_amdgcn_readlane((int)hw, 6);
        const float *qh = reinterpret_cast<const float *>(rec + sizeof(ReqHead));
        for (int c = lane; c < DP; c += 64)
            qlds[c] = c < base.d ? qh[c] : 0.0f;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();

        SearchArgs a = base;
        a.k = k;
        a.L = L;
        a.rerank_n = rr;
        a.out_mode = (flags & NHQ_SERVE_RAW) ? 1 : 0;
        a.max_hops = max_hops;
        const bool learned = (flags & kReqLearned) != 0;
        a.learned = learned ? s.learned_mode : 0;
        a.ckpt = learned ? s.check_every : 0;
        // the visited set the batch search would choose for this beam
        int slots = 1024;
        while (slots < 8 * L && slots < 4096)
            slots <<= 1;
        const int64_t bit_words = (base.n + 31) / 32;
        if (bit_words <= slots) {
            a.use_bitset = 1;
            a.vis_words = (int)bit_words;
            a.hash_log2 = 0;
        } else {
            a.use_bitset = 0;
            a.vis_words = slots;
            a.hash_log2 = 31 - __builtin_clz((unsigned)slots);
        }
        const int want = max(rr > 0 ? rr : k, base.expand * base.R);
        a.scap = want > 64 ? (want + 63) & ~63 : 64;

        // seed set: the n_cand best of the entry sample, then as in the batch search
        entry_keys_wave<DP>(base.entry_vec_f, base.entry_attr, base.n_entry, qlds, qword, qmask,
                            base.w, base.abits, base.hmask, kb);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        select_lds(kb, base.n_entry, s.n_cand, cv, cp, seedpos);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();

        OutHead *o = reinterpret_cast<OutHead *>(s.outs + (size_t)slot * s.out_bytes);
        QueryIO io;
        io.q = qlds;
        io.qlds = qlds;
        io.qword = qword;
        io.qmask = qmask;
        io.seeds = seedpos;
        io.n_seed = s.n_cand;
        io.oid = reinterpret_cast<int32_t *>(o + 1);
        io.od = reinterpret_cast<float *>(io.oid + s.max_k);
        io.cnt = &o->ndc;
        io.trace_row = 0;
        io.mlp = base.mlp;
        if (learned)
            search_one<DP, ST, true>(a, io, smem);
        else
            search_one<DP, ST, false>(a, io, smem);
        if (lane == 0) {
            o->t_begin = t_begin;
            o->t_end = wall_clock64();
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (lane == 0)
            __hip_atomic_store(&o->done, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

template <int DP, int ST>
const void *serve_kernel()
{
    return reinterpret_cast<const void *>(k_serve<DP, ST>);
}

const void *pick_kernel(int dp, int storage)
{
#define NHQ_SK(DPV)                                                      \
    case DPV:                                                            \
        switch (storage) {                                               \
        case NHQ_STORAGE_FP32:                                           \
            return serve_kernel<DPV, NHQ_STORAGE_FP32>();                \
        case NHQ_STORAGE_BF16:                                           \
            return serve_kernel<DPV, NHQ_STORAGE_BF16>();                \
        case NHQ_STORAGE_FP8:                                            \
            return serve_kernel<DPV, NHQ_STORAGE_FP8>();                 \
        }                                                                \
        return nullptr;
    switch (dp) {
        NHQ_SK(32)
        NHQ_SK(64)
        NHQ_SK(96)
        NHQ_SK(128)
        NHQ_SK(256)
        NHQ_SK(512)
        NHQ_SK(960)
        NHQ_SK(1024)
    }
#undef NHQ_SK
    return nullptr;
}

struct ServeClass {
    int lmax = 0, slots = 0, scap = 0, vis = 0;
    size_t lds = 0;
    uint8_t *ring = nullptr, *outs = nullptr;  // host pinned, coherent
    unsigned long long *ctl = nullptr;         // host pinned: [0] tail, [1] stop, [2] status
    unsigned long long *dev = nullptr;         // device: [0] next, [1] stop_dev, [2..] ready
    unsigned long long tail = 0;
    std::vector<uint64_t> owner;  // per ring entry: ticket + 1 while unpolled, else 0
};

// LDS words before the seed region (16-byte aligned for the query rows)
int seed_offset(const ServeClass &c)
{
    return (ck_offset(c.lmax, c.scap, c.vis) + kCkWords + 3) & ~3;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct Server {
    Index *ix = nullptr;
    nhq_server_params p{};
    int n_cand = 0, rec_bytes = 0, out_bytes = 0, ne_pad = 0;
    float stop_logit = 0.0f;
    double tick_hz = 1.0e8;
    double started = 0.0;
    ServeClass cls[2];
    hipStream_t st = nullptr;  // the one launch of every class
    bool running = false;
};

}  // namespace nhq

struct nhq_server {
    nhq::Server impl;
};

using namespace nhq;

namespace {

void release_class(ServeClass &c)
{
    if (c.ring)
        (void)hipHostFree(c.ring);
    if (c.outs)
        (void)hipHostFree(c.outs);
    if (c.ctl)
        (void)hipHostFree(c.ctl);
    if (c.dev)
        (void)hipFree(c.dev);
    c = ServeClass{};
}

// stop the kernel and wait (bounded) for it to end
int stop_server(Server &s)
{
    for (auto &c : s.cls)
        if (c.ctl)
            __atomic_store_n(&c.ctl[1], 1ull, __ATOMIC_RELEASE);
    const double limit = now_s() + 30.0;
    int rc = NHQ_OK;
    if (s.running) {
        for (;;) {
            const hipError_t e = hipStreamQuery(s.st);
            if (e == hipSuccess)
                break;
            if (e != hipErrorNotReady) {
                rc = fail(NHQ_EHIP, std::string("serving kernel: ") + hipGetErrorString(e));
                break;
            }
            if (now_s() > limit) {
                rc = fail(NHQ_EDEVICE, "serving kernel did not end within 30 s of the stop request");
                break;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
        s.running = false;
    }
    return rc;
}

// a class's ring, outputs and control words, and its kernel arguments
int prepare_class(Server &s, ServeClass &c, ServeArgs &a)
{
    const size_t ring_bytes = (size_t)s.p.ring * s.rec_bytes, out_bytes = (size_t)s.p.ring * s.out_bytes;
    NHQ_HIP(hipHostMalloc((void **)&c.ring, ring_bytes, hipHostMallocCoherent | hipHostMallocMapped));
    NHQ_HIP(hipHostMalloc((void **)&c.outs, out_bytes, hipHostMallocCoherent | hipHostMallocMapped));
    NHQ_HIP(hipHostMalloc((void **)&c.ctl, 64, hipHostMallocCoherent | hipHostMallocMapped));
    memset(c.ring, 0, ring_bytes);
    memset(c.outs, 0, out_bytes);
    memset(c.ctl, 0, 64);
    NHQ_HIP(hipMalloc((void **)&c.dev, sizeof(unsigned long long) * (2 + (size_t)s.p.ring)));
    NHQ_HIP(hipMemsetAsync(c.dev, 0, sizeof(unsigned long long) * (2 + (size_t)s.p.ring), s.st));
    c.owner.assign((size_t)s.p.ring, 0);
    uint8_t *ring_d = nullptr, *outs_d = nullptr;
    unsigned long long *ctl_d = nullptr;
    NHQ_HIP(hipHostGetDevicePointer((void **)&ring_d, c.ring, 0));
    NHQ_HIP(hipHostGetDevicePointer((void **)&outs_d, c.outs, 0));
    NHQ_HIP(hipHostGetDevicePointer((void **)&ctl_d, c.ctl, 0));
    a = ServeArgs{};
    a.ring = ring_d;
    a.outs = outs_d;
    a.tail = ctl_d;
    a.stop = reinterpret_cast<const uint32_t *>(ctl_d + 1);
    a.status = reinterpret_cast<uint32_t *>(ctl_d + 2);
    a.next = c.dev;
    a.stop_dev = reinterpret_cast<uint32_t *>(c.dev + 1);
    a.ready = c.dev + 2;
    a.cap = s.p.ring;
    a.rec_bytes = s.rec_bytes;
    a.out_bytes = s.out_bytes;
    a.max_k = s.p.max_k;
    a.n_cand = s.n_cand;
    a.ne_pad = s.ne_pad;
    a.seed_off = seed_offset(c);
    a.check_every = s.p.check_every;
    a.learned_mode = s.p.learned_mode;
    a.life_ticks = (unsigned long long)(s.p.lifetime_s * s.tick_hz);
    return NHQ_OK;
}

// one launch of every class: its doorbells, then class 0's slots, then class 1's
int launch_server(Server &s, int ncls, const void *kern, const SearchArgs &base, size_t lds)
{
    NHQ_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    ServeLaunch L{};
    L.ncls = ncls;
    L.slots0 = s.cls[0].slots;
    for (int ci = 0; ci < ncls; ++ci) {
        const int rc = prepare_class(s, s.cls[ci], L.c[ci]);
        if (rc != NHQ_OK)
            return rc;
    }
    if (lds > 64 * 1024)
        NHQ_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned grid = (unsigned)(ncls + s.cls[0].slots + (ncls > 1 ? s.cls[1].slots : 0));
    void *args[] = {const_cast<SearchArgs *>(&base), &L};
    NHQ_HIP(hipLaunchKernel(kern, dim3(grid), dim3(64), args, lds, s.st));
    s.running = true;
    return NHQ_OK;
}

}  // namespace

extern "C" {

int nhq_server_create(nhq_index *h, const nhq_server_params *pp, nhq_server **out)
{
    if (!h || !out)
        return fail(NHQ_EINVAL, "null argument");
    *out = nullptr;
    Index *ix = &h->impl;
    if (ix->degree <= 0)
        return fail(NHQ_EINVAL, "the index has no graph");
    nhq_server_params p{};
    if (pp)
        p = *pp;
    if (p.beam_small == 0)
        p.beam_small = 128;
    if (p.beam_large == 0)
        p.beam_large = 512;
    if (p.ring == 0)
        p.ring = 4096;
    if (p.max_k == 0)
        p.max_k = 100;
    if (p.n_init == 0)
        p.n_init = 32;
    if (p.expand == 0)
        p.expand = 1;
    if (p.check_every == 0)
        p.check_every = 4;
    if (p.auto_beam == 0)
        p.auto_beam = p.beam_small;
    if (p.max_hops == 0)
        p.max_hops = 100000;
    if (p.stop_threshold == 0.0f)
        p.stop_threshold = 0.5f;
    if (p.lifetime_s == 0.0)
        p.lifetime_s = 600.0;
    if (p.learned_mode == 0)
        p.learned_mode = 1;
    if (p.learned_mode < 1 || p.learned_mode > 3 || (p.learned_mode >= 2 && !(p.cap_factor > 0.0f)))
        return fail(NHQ_EINVAL, "learned_mode must be 1, or 2 or 3 with cap_factor > 0");
    if (p.beam_small < 1 || p.beam_small > NHQ_MAX_BEAM || (p.beam_large > 0 && p.beam_large <= p.beam_small) ||
        p.beam_large > NHQ_MAX_BEAM)
        return fail(NHQ_EINVAL, "need 1 <= beam_small < beam_large <= 1024 (beam_large < 0: no large class)");
    if (p.ring < 1 || p.ring > (1 << 20) || p.max_k < 1 || p.max_k > NHQ_MAX_BEAM)
        return fail(NHQ_EINVAL, "need 1 <= ring <= 2^20 and 1 <= max_k <= 1024");
    if (p.n_init < 1 || p.n_init > 128 || p.expand < 1 || p.expand > 8 || p.check_every < 1 ||
        p.max_hops < 1 || p.rerank < 0 || p.slots_small < 0 || p.slots_large < 0)
        return fail(NHQ_EINVAL, "bad search parameter");
    if (!(p.stop_threshold > 0.0f && p.stop_threshold < 1.0f) || !(p.lifetime_s > 0.0))
        return fail(NHQ_EINVAL, "stop_threshold must be in (0, 1) and lifetime_s positive");
    const int top = p.beam_large > 0 ? p.beam_large : p.beam_small;
    if (p.auto_beam < 1 || p.auto_beam > top)
        return fail(NHQ_EINVAL, "auto_beam must not exceed the largest class beam");
    const void *kern = pick_kernel(ix->dp, ix->storage);
    if (!kern)
        return fail(NHQ_EINVAL, "unsupported padded dimension or storage form");
    NHQ_HIP(hipSetDevice(ix->device));

    auto *hs = new (std::nothrow) nhq_server;
    if (!hs)
        return fail(NHQ_ENOMEM, "host allocation failed");
    Server &s = hs->impl;
    s.ix = ix;
    s.p = p;
    s.n_cand = std::min(ix->n_entry, p.n_init + kSeedMargin);
    s.ne_pad = (ix->n_entry + 63) & ~63;
    s.rec_bytes = (int)((sizeof(ReqHead) + 4 * (size_t)ix->d + 63) & ~(size_t)63);
    s.out_bytes = (int)((sizeof(OutHead) + 8 * (size_t)p.max_k + 63) & ~(size_t)63);
    s.stop_logit = logf(p.stop_threshold / (1.0f - p.stop_threshold));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ix->device) == hipSuccess && khz > 0)
        s.tick_hz = 1000.0 * khz;
    int n_cu = 0;
    NHQ_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ix->device));

    SearchArgs base{};
    base.vecs = ix->vecs;
    base.vec32 = ix->vec32;
    base.scale = ix->scale;
    base.attr = ix->attr;
    base.adj = ix->adj;
    base.entry = ix->entry;
    base.entry_vec_f = ix->entry_vec;
    base.entry_attr = ix->entry_attr;
    base.err = ix->err;
    base.n = ix->n;
    base.d = ix->d;
    base.m = ix->m;
    base.R = ix->degree;
    base.n_entry = ix->n_entry;
    base.n_init = p.n_init;
    base.expand = p.expand;
    base.w = ix->w;
    base.abits = ix->abits;
    base.hmask = ix->hmask;
    base.stop_logit = s.stop_logit;
    base.cap_factor = p.cap_factor;
    base.mlp = reinterpret_cast<const uint16_t *>(ix->mlp);
    base.logp = ix->logp;

    const int ncls = p.beam_large > 0 ? 2 : 1;
    const int64_t bit_words = (ix->n + 31) / 32;
    int rc = NHQ_OK;
    for (int ci = 0; ci < ncls && rc == NHQ_OK; ++ci) {
        ServeClass &c = s.cls[ci];
        c.lmax = ci == 0 ? p.beam_small : p.beam_large;
        const int want = std::max({64, std::min(c.lmax, p.max_k * std::max(1, p.rerank)), p.expand * ix->degree});
        c.scap = (want + 63) & ~63;
        int slots = 1024;
        while (slots < 8 * c.lmax && slots < 4096)
            slots <<= 1;
        c.vis = slots;  // a bitset is used only when it fits in the same words
        (void)bit_words;
        const size_t words = (size_t)seed_offset(c) + ix->dp + 160 + s.ne_pad + 512;
        c.lds = 4 * words;
        if (c.lds > 160 * 1024) {
            rc = fail(NHQ_EINVAL, "a serving slot's LDS exceeds 160 KiB (beam or entry sample too large)");
            break;
        }
    }
    // one launch: every workgroup gets the largest class's LDS, and every
    // class stays resident together, each with its part of the chip
    size_t lds = 0;
    for (int ci = 0; ci < ncls; ++ci)
        lds = std::max(lds, s.cls[ci].lds);
    if (rc == NHQ_OK && lds > 64 * 1024 &&
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        rc = fail(NHQ_EHIP, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (rc == NHQ_OK &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds) != hipSuccess || per_cu < 1))
        rc = fail(NHQ_EHIP, "occupancy query failed for the serving kernel");
    for (int ci = 0; ci < ncls && rc == NHQ_OK; ++ci) {
        ServeClass &c = s.cls[ci];
        const double share = ncls == 1 ? 0.9 : (ci == 0 ? 0.6 : 0.3);
        const int fit = std::max(1, (int)(share * per_cu * n_cu) - ncls);
        const int asked = ci == 0 ? p.slots_small : p.slots_large;
        c.slots = asked > 0 ? std::min(asked, fit) : fit;
    }
    if (rc == NHQ_OK) {
        if (!ix->entry_vec || ix->n_entry < 1)
            rc = fail(NHQ_EINVAL, "the index has no entry sample");
    }
    if (rc == NHQ_OK) {
        // the index's ingest work must be complete before the kernels read it
        if (hipDeviceSynchronize() != hipSuccess)
            rc = fail(NHQ_EHIP, "device synchronisation before serving failed");
    }
    if (rc == NHQ_OK)
        rc = launch_server(s, ncls, kern, base, lds);
    if (rc != NHQ_OK) {
        (void)stop_server(s);
        for (auto &c : s.cls)
            release_class(c);
        if (s.st)
            (void)hipStreamDestroy(s.st);
        delete hs;
        return rc;
    }
    s.started = now_s();
    *out = hs;
    return NHQ_OK;
}

int nhq_server_info(const nhq_server *h, int32_t *slots, int32_t *lds_bytes, int32_t *beam_max,
                    double *tick_hz)
{
    if (!h)
        return fail(NHQ_EINVAL, "null server");
    const Server &s = h->impl;
    for (int ci = 0; ci < 2; ++ci) {
        if (slots)
            slots[ci] = s.cls[ci].slots;
        if (lds_bytes)
            lds_bytes[ci] = (int32_t)s.cls[ci].lds;
        if (beam_max)
            beam_max[ci] = s.cls[ci].lmax;
    }
    if (tick_hz)
        *tick_hz = s.tick_hz;
    return NHQ_OK;
}

int nhq_server_submit(nhq_server *h, const float *q, const uint8_t *qattr, int32_t k, int32_t beam,
                      int32_t flags, uint64_t *ticket)
{
    if (!h || !q || !ticket)
        return fail(NHQ_EINVAL, "null argument");
    Server &s = h->impl;
    const Index *ix = s.ix;
    if (ix->m > 0 && !qattr)
        return fail(NHQ_EINVAL, "null query attributes");
    if (flags & ~NHQ_SERVE_RAW)
        return fail(NHQ_EINVAL, "unknown request flag");
    int learned = 0;
    if (beam == 0) {
        if (!ix->mlp)
            return fail(NHQ_EINVAL, "beam 0 (learned stop) needs a loaded network");
        beam = s.p.auto_beam;
        learned = 1;
    }
    if (k < 1 || k > s.p.max_k || beam < k)
        return fail(NHQ_EINVAL, "need 1 <= k <= max_k and k <= beam");
    int ci = -1;
    for (int c = 0; c < 2; ++c)
        if (ci < 0 && s.cls[c].slots > 0 && beam <= s.cls[c].lmax)
            ci = c;
    if (ci < 0)
        return fail(NHQ_EINVAL, "beam exceeds every memory class of the server");
    ServeClass &c = s.cls[ci];
    const uint32_t st = (uint32_t)__atomic_load_n(&c.ctl[2], __ATOMIC_ACQUIRE);
    if (st != 0 || !s.running)
        return fail(NHQ_EDEVICE, st == 2 ? "serving kernel reached its lifetime" : "serving kernel has ended");
    const size_t slot = (size_t)(c.tail % (unsigned long long)s.p.ring);
    if (c.owner[slot] != 0)
        return NHQ_EBUSY;
    ReqHead r{};
    r.k = k;
    r.L = beam;
    r.flags = (flags & NHQ_SERVE_RAW) | (learned ? kReqLearned : 0);
    r.rerank_n = s.p.rerank > 0 ? std::min(s.p.rerank * k, beam) : 0;
    r.max_hops = s.p.max_hops;
    attr_pack_query(qattr, ix->m, ix->abits, r.qword, r.qmask);
    uint8_t *rec = c.ring + slot * (size_t)s.rec_bytes;
    memcpy(rec, &r, sizeof r);
    memcpy(rec + sizeof r, q, sizeof(float) * (size_t)ix->d);
    const uint64_t t = ((uint64_t)ci << 56) | c.tail;
    c.owner[slot] = t + 1;
    c.tail += 1;
    __atomic_store_n(&c.ctl[0], c.tail, __ATOMIC_RELEASE);
    *ticket = t;
    return NHQ_OK;
}

int nhq_server_poll(nhq_server *h, uint64_t ticket, int32_t *ids, float *dists, uint32_t *counters,
                    uint64_t *ticks)
{
    if (!h || !ids || !dists)
        return fail(NHQ_EINVAL, "null argument");
    Server &s = h->impl;
    const int ci = (int)(ticket >> 56);
    const uint64_t idx = ticket & ((uint64_t(1) << 56) - 1);
    if (ci < 0 || ci > 1 || s.cls[ci].slots == 0)
        return fail(NHQ_EINVAL, "bad ticket");
    ServeClass &c = s.cls[ci];
    const size_t slot = (size_t)(idx % (uint64_t)s.p.ring);
    if (c.owner[slot] != ticket + 1)
        return fail(NHQ_EINVAL, "ticket unknown or already polled");
    const uint8_t *rec = c.outs + slot * (size_t)s.out_bytes;
    const OutHead *o = reinterpret_cast<const OutHead *>(rec);
    const unsigned long long done = __atomic_load_n(&o->done, __ATOMIC_ACQUIRE);
    if (done != idx + 1) {
        const uint32_t st = (uint32_t)__atomic_load_n(&c.ctl[2], __ATOMIC_ACQUIRE);
        if (st != 0)
            return fail(NHQ_EDEVICE, "serving kernel ended before the request finished");
        return NHQ_PENDING;
    }
    const ReqHead *r = reinterpret_cast<const ReqHead *>(c.ring + slot * (size_t)s.rec_bytes);
    const int k = r->k;
    memcpy(ids, rec + sizeof(OutHead), sizeof(int32_t) * (size_t)k);
    memcpy(dists, rec + sizeof(OutHead) + 4 * (size_t)s.p.max_k, sizeof(float) * (size_t)k);
    if (counters) {
        counters[0] = o->ndc;
        counters[1] = o->hops;
    }
    if (ticks) {
        ticks[0] = o->t_begin;
        ticks[1] = o->t_end;
    }
    c.owner[slot] = 0;
    return NHQ_OK;
}

int nhq_server_run(nhq_server *h, const float *q, const uint8_t *qattrs, const int32_t *k,
                   const int32_t *beam, const int32_t *flags, const double *arrival_s, int64_t n,
                   int32_t *ids, float *dists, uint32_t *counters, uint64_t *ticks, double *latency_s,
                   double *elapsed_s, double timeout_s)
{
    if (!h || (!q && n > 0) || !k || !beam || !arrival_s || !ids || !dists || !latency_s)
        return fail(NHQ_EINVAL, "null argument");
    Server &s = h->impl;
    const Index *ix = s.ix;
    if (n < 0 || (ix->m > 0 && !qattrs && n > 0))
        return fail(NHQ_EINVAL, "bad request count or null query attributes");
    for (int64_t i = 1; i < n; ++i)
        if (arrival_s[i] < arrival_s[i - 1])
            return fail(NHQ_EINVAL, "arrival times must be non-decreasing");
    if (timeout_s <= 0.0)
        timeout_s = 60.0;
    const int mk = s.p.max_k;
    std::vector<std::pair<int64_t, uint64_t>> flight;
    flight.reserve(2 * (size_t)s.p.ring);
    const double t0 = now_s();
    int64_t next = 0, done = 0;
    uint32_t cnt[2];
    uint64_t tk[2];
    while (done < n) {
        const double now = now_s() - t0;
        if (now > timeout_s)
            return fail(NHQ_EDEVICE, "request stream did not finish within the timeout");
        while (next < n && arrival_s[next] <= now) {
            uint64_t t = 0;
            const int rc = nhq_server_submit(h, q + next * (int64_t)ix->d,
                                             ix->m > 0 ? qattrs + next * (int64_t)ix->m : nullptr, k[next],
                                             beam[next], flags ? flags[next] : 0, &t);
            if (rc == NHQ_EBUSY)
                break;
            if (rc != NHQ_OK)
                return rc;
            flight.emplace_back(next, t);
            next += 1;
        }
        size_t w = 0;
        for (size_t j = 0; j < flight.size(); ++j) {
            const int64_t i = flight[j].first;
            const int rc = nhq_server_poll(h, flight[j].second, ids + i * mk, dists + i * mk, cnt, tk);
            if (rc == NHQ_OK) {
                latency_s[i] = (now_s() - t0) - arrival_s[i];
                if (counters) {
                    counters[2 * i] = cnt[0];
                    counters[2 * i + 1] = cnt[1];
                }
                if (ticks) {
                    ticks[2 * i] = tk[0];
                    ticks[2 * i + 1] = tk[1];
                }
                for (int j2 = k[i]; j2 < mk; ++j2) {
                    ids[i * mk + j2] = -1;
                    dists[i * mk + j2] = __builtin_inff();
                }
                done += 1;
            } else if (rc == NHQ_PENDING) {
                flight[w++] = flight[j];
            } else {
                return rc;
            }
        }
        flight.resize(w);
    }
    if (elapsed_s)
        *elapsed_s = now_s() - t0;
    return NHQ_OK;
}

int nhq_server_free(nhq_server *h)
{
    if (!h)
        return NHQ_OK;
    Server &s = h->impl;
    const int rc = stop_server(s);
    if (rc != NHQ_OK)
        return rc;  // the kernel may still run: keep its memory
    for (auto &c : s.cls)
        release_class(c);
    if (s.st)
        (void)hipStreamDestroy(s.st);
    delete h;
    return NHQ_OK;
}

}  // extern "C"
