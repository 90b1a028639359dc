// Joint pruning (Alg. 2) in beam form on gfx950: one wavefront per query.
//
// Per wave, in LDS: the pool (the `beam` best vertices by fusion distance,
// sorted by (key, id), each with its chi and an "expanded" flag), a staging
// list for the current batch of candidates, and the visited set (a bitset
// when the object set is small, else an open-addressing hash).  Per lane, in
// registers: this lane's slice of the query vector.
//
// Scoring a candidate row uses G lanes (G = 8 for rows up to 512 elements,
// 16 above): lane g of a group holds 4-element chunks g, g+G, g+2G, ... so a
// group's loads for one row are contiguous 16-, 8- or 4-byte pieces (fp32,
// bf16, fp8 storage) and 64/G rows are scored per round.  Partial sums are
// reduced inside the group with DPP lane moves.  Rows of 512 elements and
// more read the query from the wave's LDS copy instead of registers.
//
// Ordering key: Gamma = delta * (m_q + chi) / m_q is ordered through
// key = delta^2 * (m_q + chi)^2 (delta^2 when m_q = 0), one float multiply of
// the float32 delta^2.  Ties are broken by the smaller id.
#include "search_core.h"

namespace nhq {
namespace {

template <int DP, int ST, bool CK>
__device__ __forceinline__ void search_block(const SearchArgs &a)
{
    extern __shared__ __align__(16) uint32_t smem[];
    const int64_t qi = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
    if (qi < 0 || qi >= a.nq) {
        if (threadIdx.x == 0)
            atomicOr(a.err, NHQ_DEVERR_BADID);
        return;
    }
    QueryIO io;
    io.q = a.q + qi * (int64_t)a.d;
    io.qlds = nullptr;
    pack_query_attrs(a.qa + qi * a.m, a.m, a.abits, io.qword, io.qmask);
    io.seeds = a.seed_cand + (a.seeds_shared ? 0 : qi * a.n_seed);
    io.n_seed = a.n_seed;
    io.oid = a.out_ids + qi * a.k;
    io.od = a.out_dist + qi * a.k;
    io.cnt = a.counters ? a.counters + 2 * qi : nullptr;
    io.trace_row = qi;
    io.mlp = a.mlp;
    search_one<DP, ST, CK>(a, io, smem);
}

// The checkpoint code raises the kernel's register count enough for the
// compiler to settle at 4 waves per SIMD; for rows up to 128 elements asking
// for 6 costs a few spills at the checkpoints but runs the search faster
// (measured).  Wider rows keep the compiler's choice.
#ifndef NHQ_CK_WAVES
#define NHQ_CK_WAVES 6
#endif
#define NHQ_CK_ATTR __attribute__((amdgpu_waves_per_eu(DP <= 128 ? NHQ_CK_WAVES : 1)))

template <int DP, int ST>
__global__ __launch_bounds__(64) void k_search(const SearchArgs a)
{
    search_block<DP, ST, false>(a);
}

// with checkpoints (traces, learned stop)
template <int DP, int ST>
__global__ __launch_bounds__(64) NHQ_CK_ATTR void k_search_ck(const SearchArgs a)
{
    search_block<DP, ST, true>(a);
}

template <int DP, int ST>
int launch_one(const SearchArgs &a, size_t lds, hipStream_t st)
{
    auto kern = a.ckpt > 0 ? k_search_ck<DP, ST> : k_search<DP, ST>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return fail(NHQ_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.nq), dim3(64), lds, st, a);
    NHQ_HIP(hipGetLastError());
    return NHQ_OK;
}

template <int DP>
int launch_dp(const SearchArgs &a, int storage, size_t lds, hipStream_t st)
{
    switch (storage) {
    case NHQ_STORAGE_FP32:
        return launch_one<DP, NHQ_STORAGE_FP32>(a, lds, st);
    case NHQ_STORAGE_BF16:
        return launch_one<DP, NHQ_STORAGE_BF16>(a, lds, st);
    case NHQ_STORAGE_FP8:
        return launch_one<DP, NHQ_STORAGE_FP8>(a, lds, st);
    }
    return fail(NHQ_EINVAL, "unknown storage form");
}

}  // namespace

int launch_search(const SearchLaunch &s)
{
    const Index *ix = s.ix;
    SearchArgs a{};
    a.vecs = ix->vecs;
    a.vec32 = ix->vec32;
    a.scale = ix->scale;
    a.attr = ix->attr;
    a.adj = ix->adj;
    a.seed_cand = s.seed_cand;
    a.entry = s.entry_override ? s.entry_override : ix->entry;
    a.seeds_shared = s.seeds_shared;
    a.q = s.q;
    a.qa = s.qa;
    a.out_ids = s.ids;
    a.out_dist = s.dists;
    a.counters = s.counters;
    a.order = s.order;
    a.err = ix->err;
    a.n = ix->n;
    a.nq = s.nq;
    a.d = ix->d;
    a.m = ix->m;
    a.R = ix->degree;
    a.n_seed = s.n_seed_cand;
    a.n_entry = s.entry_override ? s.n_entry_override : ix->n_entry_total;
    a.k = s.k;
    a.L = s.L;
    a.n_init = s.n_init;
    a.out_mode = s.out_mode;
    a.rerank_n = s.rerank_n;
    a.max_hops = s.max_hops;
    a.ckpt = (s.learned || s.trace) ? s.check_every : 0;
    a.expand = s.expand;
    a.route_h = s.route_h;
    a.w = ix->w;
    a.abits = ix->abits;
    a.hmask = ix->hmask;
    a.learned = s.learned;
    a.stop_logit = s.stop_logit;
    a.cap_factor = s.cap_factor;
    a.mlp = reinterpret_cast<const uint16_t *>(ix->mlp);
    a.logp = ix->logp;
    if (s.trace) {
        a.trace_feat = s.trace->feat;
        a.trace_hop = s.trace->hop;
        a.trace_hash = s.trace->hash;
        a.trace_count = s.trace->count;
        a.final_hash = s.trace->final_hash;
        a.trace_cap = s.trace->cap;
    }
    const int want = std::max(s.rerank_n > 0 ? s.rerank_n : s.k, s.expand * ix->degree);
    a.scap = want > 64 ? ((want + 63) & ~63) : 64;
    // visited set: bitset when it is no larger than the hash would be
    int hb = s.hash_log2;
    if (hb <= 0) {
        int slots = 1024;
        while (slots < 8 * s.L && slots < 4096)
            slots <<= 1;
        hb = 0;
        while ((1 << hb) < slots)
            ++hb;
    }
    const int64_t bit_words = (ix->n + 31) / 32;
    if (bit_words <= (int64_t(1) << hb)) {
        a.use_bitset = 1;
        a.vis_words = (int)bit_words;
        a.hash_log2 = 0;
    } else {
        a.use_bitset = 0;
        a.vis_words = 1 << hb;
        a.hash_log2 = hb;
    }
    // the checkpoint state exists only in the checkpointing kernel; wide
    // rows keep the query row in LDS after it
    const size_t lds = sizeof(uint32_t) *
                       ((size_t)q_offset(a.L, a.scap, a.vis_words, a.ckpt > 0) + query_lds_words(ix->dp));
    if (s.nq > 0x7FFFFFFF)
        return fail(NHQ_EINVAL, "too many queries in one call");
    switch (ix->dp) {
    case 32:
        return launch_dp<32>(a, ix->storage, lds, s.stream);
    case 64:
        return launch_dp<64>(a, ix->storage, lds, s.stream);
    case 96:
        return launch_dp<96>(a, ix->storage, lds, s.stream);
    case 128:
        return launch_dp<128>(a, ix->storage, lds, s.stream);
    case 256:
        return launch_dp<256>(a, ix->storage, lds, s.stream);
    case 512:
        return launch_dp<512>(a, ix->storage, lds, s.stream);
    case 960:
        return launch_dp<960>(a, ix->storage, lds, s.stream);
    case 1024:
        return launch_dp<1024>(a, ix->storage, lds, s.stream);
    }
    return fail(NHQ_EINVAL, "unsupported padded dimension");
}

}  // namespace nhq
