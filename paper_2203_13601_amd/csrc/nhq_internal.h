// Internal declarations shared by the libnhq translation units: the index
// object, error plumbing and the device helpers every kernel uses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "nhq.h"
#include "attr.h"
#include "weights.h"

// ------------------------------------------------------------------ errors
namespace nhq {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define NHQ_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::nhq::fail(NHQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// --------------------------------------------------------------- packing
// Pool / candidate id word: vertex id in the low 27 bits, chi (0..12) in bits
// 27..30, the "expanded" flag in bit 31.  Order comparisons use the id bits.
constexpr uint32_t kIdMask = 0x07FFFFFFu;
constexpr uint32_t kExpBit = 0x80000000u;
constexpr int kChiShift = 27;
constexpr uint32_t kChiMask = 15u;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int64_t kMaxN = int64_t(1) << 27;
// seed candidates kept beyond n_init for the direct-form re-score (guards
// the GEMM form's rounding at near-ties of the dense ranking)
constexpr int kSeedMargin = 8;

// Padded widths the kernels are instantiated for (the stored rows are padded
// with zeros to the next one; zeros change no distance).
int padded_dim(int d);

struct Index {
    int device = 0;
    int64_t n = 0;
    int64_t cap = 0;  // rows allocated (n <= cap; nhq_index_insert appends)
    int d = 0, dp = 0, m = 0;
    int degree = 0;  // 0 until a graph exists
    int storage = NHQ_STORAGE_FP32;
    int cand = 64;
    int reverse_edges = 0;
    int n_entry = 0;
    uint64_t seed = 0;
    Weights w{NHQ_WEIGHTS_DEFAULT, 0.0f, 0.0};  // weight setting of Gamma
    int abits = 8;                 // bits per attribute in the packed words
    uint32_t hmask = 0x80808080u;  // high bit of every attribute field
    // edge candidates: exact all-pairs or NN-descent (rounds, sample, stop)
    int builder = NHQ_BUILD_EXACT;
    int nnd_rounds = 12, nnd_sample = 24;
    float nnd_stop = 0.001f;
    int nnd_rounds_run = 0;  // rounds the last NN-descent build ran
    int nsw_batch = 10000, nsw_beam = 0;  // NSW insertion (beam 0: cand)
    float *vec32 = nullptr;     // [n][dp] float32 copy (rerank / fp32 storage)
    void *vecs = nullptr;       // storage form [n][dp] (== vec32 for fp32)
    float *scale = nullptr;     // fp8: per-row scale [n]
    uint32_t *attr = nullptr;   // [n] packed codes, byte i = attribute i
    float *norm = nullptr;      // [n] squared norms of the float32 rows
    int32_t *adj = nullptr;     // [n][degree]
    int32_t *entry = nullptr;   // [n_entry]
    float *entry_vec = nullptr;     // [n_entry][dp] float32 rows of the entry sample
    float *entry_norm = nullptr;    // [n_entry]
    uint32_t *entry_attr = nullptr; // [n_entry]
    // bf16 copy of entry_vec when every value is an integer of magnitude
    // <= 256 and dp <= 128: then bf16 products summed in float32 are exact,
    // and the ranking uses the bf16 matrix-core instructions (else null)
    uint16_t *entry_bf16 = nullptr;
    // entry_vec split for the bf16 matrix cores: every float32 value v as
    // hi = bf16(v) and lo = bf16(v - hi); row r holds, per 32-element chunk
    // c, the 32 hi halves then the 32 lo halves ([n_entry_total][2 dp])
    uint16_t *entry_split = nullptr;
    // stratified entry sample (entry_per_pattern > 0): after the n_entry
    // global members, one block per attribute pattern the objects hold, in
    // increasing packed-word order; block b holds entry positions
    // block_off[b] .. block_off[b + 1] - 1
    int n_blocks = 0, per_pattern = 0;
    int n_entry_total = 0;           // n_entry + every block
    uint32_t *block_word = nullptr;  // device [n_blocks] packed codes
    int32_t *block_off = nullptr;    // device [n_blocks + 1]
    std::vector<uint32_t> block_word_h;
    std::vector<int32_t> block_off_h;
    uint32_t *err = nullptr;    // device error word
    // per-index workspace (grown on demand)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    std::mutex mu;
    // learned stop network (fp16 weights, device), null when not loaded
    void *mlp = nullptr;
    float *logp = nullptr;  // [m][256] ln(count / n) of every attribute code
};

int ensure_workspace(Index *ix, size_t bytes);
void free_index(Index *ix);  // every device array the index holds

// NPG_nsw by batched insertion (nsw.hip)
int nsw_build(Index *ix, int l, int64_t B, int L, uint64_t seed, hipStream_t st);
int nsw_insert(Index *ix, int64_t s0, int64_t s1, int l, int64_t B, int L, uint64_t seed,
               hipStream_t st);

// NN-descent candidate lists (nndescent.hip)
int nnd_lists(const Index *ix, int l, int s, int rounds, double stop_frac, uint64_t seed,
              int32_t *ids, int64_t *updates_host, int *rounds_run, hipStream_t st);

// splitmix64 (Steele, Lea and Flood, 2014)
__host__ __device__ inline uint64_t splitmix64_next(uint64_t &state)
{
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------ launchers
struct SearchLaunch {
    const Index *ix;
    const float *q;
    const uint8_t *qa;
    const int32_t *seed_cand;  // [nq][n_seed_cand] entry-sample candidates per query
    int n_seed_cand;
    int64_t nq;
    int k, L, n_init, out_mode, rerank_n, max_hops, hash_log2, learned, check_every;
    float stop_logit, cap_factor;
    int expand;
    int route_h;
    const nhq_trace *trace;
    // nullable: the entry sample the seed positions index (else the index's),
    // and whether every query shares the first row of seed_cand
    const int32_t *entry_override;
    int n_entry_override;
    int seeds_shared;
    int32_t *ids;
    float *dists;
    uint32_t *counters;
    const int32_t *order;  // nullable launch order (wave i searches query order[i])
    hipStream_t stream;
};
int launch_search(const SearchLaunch &s);

// edge selection of rows row0 .. row0 + nrows - 1, and re-selection of
// listed rows with offers (select.hip)
int launch_select_rows(const Index *ix, const int32_t *cand, int K, int l, int32_t *adj,
                       int64_t row0, int64_t nrows, hipStream_t st);
int launch_reselect_targets(const Index *ix, int32_t *adj, const int32_t *targets, int64_t nt,
                            const int64_t *off, const int32_t *inc, hipStream_t st);

// dense tiles with a streaming top-K (see dense_topk.hip)
int launch_dense_topk(const float *A, const float *A_norm, const uint32_t *A_attr,
                      const uint32_t *A_mask, int64_t na, const float *B, const float *B_norm,
                      const uint32_t *B_attr, int64_t nb, int dp, int m, int abits, int mode,
                      int self_exclude, int K, int32_t *out_ids, float *out_keys, hipStream_t st,
                      const Weights *w = nullptr);

// seed ranking of a stratified entry sample (see seed.hip): each query
// ranked against its pattern's block, or the global members; scratch of
// strata_rank_words(ix, nq, K) 32-bit words at blk; qsplit: the query rows
// split like Index::entry_split
size_t strata_rank_words(const Index *ix, int64_t nq, int K);
int launch_strata_rank(const Index *ix, const uint16_t *qsplit, const float *qnorm, const uint32_t *qword,
                       const uint32_t *qmask, int64_t nq, int K, uint32_t *blk, int32_t *cand,
                       hipStream_t st);

// seed ranking of the entry sample (see seed.hip): positions of the K best
// keys: scratch of nq * ((n_entry + 63) / 64 * 64) * 17 / 16 floats (the key
// matrix, then its 16-entry group minima); qexact (nullable):
// per query, nonzero when every value is an integer of magnitude <= 256;
// qsplit: the query rows split like Index::entry_split
int launch_seed_rank(const Index *ix, const float *qpad, const uint16_t *qsplit, const float *qnorm,
                     const uint32_t *qword, const uint32_t *qmask, const uint32_t *qexact, int64_t nq, int K,
                     float *keys, int32_t *cand, hipStream_t st);

// queries -> zero-padded float32 rows, squared norms, packed codes and masks,
// (qexact nullable) whether every value is an integer of magnitude <= 256,
// and (qsplit nullable) the rows split like Index::entry_split
int launch_pad_queries(const float *q, const uint8_t *qa, int64_t nq, int d, int dp, int m,
                       int abits, float *qpad, float *qnorm, uint32_t *qword, uint32_t *qmask, uint32_t *qexact,
                       uint16_t *qsplit, hipStream_t st);

// float32 rows [rows][dp] -> their hi/lo bf16 split [rows][2 dp] (the layout
// of Index::entry_split)
int launch_split_rows(const float *src, int64_t rows, int dp, uint16_t *dst, hipStream_t st);

}  // namespace nhq

struct nhq_index {
    nhq::Index impl;
};
