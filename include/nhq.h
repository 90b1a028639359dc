/*
 * libnhq -- native hybrid queries (NHQ, Wang et al., arXiv 2203.13601) on
 * AMD Instinct MI355X (gfx950).
 *
 * A hybrid query (Def. 4) asks for the k objects nearest to a query vector
 * among the objects whose structured attributes equal the query's.  NHQ
 * answers it with one proximity graph, the composite index (Alg. 1, Sec. 5.1),
 * whose edges are chosen under the fusion distance Gamma (Eq. 6) with the
 * landing-zone edge selection (Sec. 4.1, Def. 7), and one best-first search
 * that prunes on vectors and attributes at once (joint pruning, Alg. 2).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    "host".  Vectors are row-major float32 [rows][d]; attribute codes are
 *    row-major uint8 [rows][m], m <= 12.  The index packs an object's codes
 *    into one 32-bit word, 8 bits each for m <= 4, 4 bits for m <= 8 and 2
 *    bits for m <= 12, so object codes must stay below 255, 15 and 3
 *    respectively.  In query codes 255 (0xFF) marks an unconstrained
 *    attribute (wildcard); other query codes no object holds match nothing.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is asynchronous unless stated otherwise: outputs are valid once the
 *    stream has been synchronised.
 *  - Return value: NHQ_OK (0) or a negative NHQ_E* code; nhq_strerror() turns
 *    it into text and nhq_last_error() gives the calling thread's last
 *    detailed message.  No C++ exception crosses this boundary.
 *  - An index owns every device copy it makes; it never aliases caller memory
 *    after a call returns.  Calls that use one index must be ordered on one
 *    stream and made from one host thread at a time (they share the index's
 *    workspace).
 *  - Fusion distance: Gamma(q, e) = delta * (1 + chi / m_q) where delta is the
 *    Euclidean distance (Eq. 1), chi the number of constrained attributes on
 *    which the codes differ (Eq. 4-5) and m_q the number of constrained
 *    attributes (Gamma = delta when m_q = 0).  These are the weights
 *    w_v = 1, w_l = delta / m of Sec. 3.2.  Between two objects m_q = m.
 *  - Results: ids int32 [nq][k] padded with -1, distances float32 [nq][k]
 *    (Gamma) padded with +inf.
 */
#ifndef NHQ_H
#define NHQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NHQ_OK 0
#define NHQ_EINVAL (-1)   /* bad argument: shape, size, mode, null pointer   */
#define NHQ_ENOMEM (-2)   /* device or host allocation failed                 */
#define NHQ_EHIP (-3)     /* a HIP runtime call or kernel launch failed       */
#define NHQ_EDEVICE (-4)  /* a kernel raised its error word (see below)       */
#define NHQ_ENOTSUP (-5)  /* valid request this build does not support        */
#define NHQ_EIO (-6)      /* file error in save / load                        */
#define NHQ_EBUSY (-7)    /* serving: no free slot or ring entry              */

#define NHQ_STORAGE_FP32 0
#define NHQ_STORAGE_BF16 1
#define NHQ_STORAGE_FP8 2 /* OCP e4m3 with one float32 scale per vector */

/* Weight settings of the fusion distance Gamma (Eq. 6), fixed per index:
 * the build and every search of the index use the same one.  delta is the
 * Euclidean distance (Eq. 1), chi the number of mismatched constrained
 * attributes (Eq. 4-5), m_q the number of constrained attributes (m between
 * two objects), p the index's weight_param.  Sec. 6.5 compares them.      */
#define NHQ_WEIGHTS_DEFAULT 0    /* w_v = 1, w_l = delta / m_q:
                                    Gamma = delta (1 + chi / m_q) (Sec. 3.2) */
#define NHQ_WEIGHTS_HARMONIC 1   /* w_v = chi / (delta + chi),
                                    w_l = delta / (delta + chi):
                                    Gamma = 2 delta chi / (delta + chi), 0 when
                                    delta + chi = 0                           */
#define NHQ_WEIGHTS_HARMONIC_C 2 /* the harmonic form with chi replaced by 1
                                    when chi = 0 and by p * chi otherwise
                                    (Eq. 8, p = c > 1)                        */
#define NHQ_WEIGHTS_NORMALISED 3 /* w_v = 1 / p (p = delta_max),
                                    w_l = 1 / m_q (chi term 0 when m_q = 0)   */
#define NHQ_WEIGHTS_FIXED 4      /* w_v = 1, w_l = p (the ratio w_l / w_v)  */

#define NHQ_MAX_DEGREE 64
#define NHQ_MAX_BEAM 1024
#define NHQ_MAX_ATTRS 12

typedef struct nhq_index nhq_index;

/* Build parameters (Alg. 1 / Sec. 4.1 / Sec. 4.3).  Zero fields take the
 * defaults given in brackets. */
typedef struct {
    int32_t degree;        /* R: out-degree bound of the graph            [32] */
    int32_t cand;          /* l: candidate-list size of edge selection    [64] */
    int32_t reverse_edges; /* 1: re-select each row from its forward edges
                              united with the vertices that chose it       [0] */
    int32_t storage;       /* NHQ_STORAGE_*: form the search scores with   [0] */
    int32_t n_entry;       /* size of the random entry sample from which each
                              query's seed set is taken                  [1024] */
    int32_t weights;       /* NHQ_WEIGHTS_*: weight setting of Gamma, for the
                              build and every search of this index          [0] */
    uint64_t seed;         /* splitmix64 seed of the entry sample          [0] */
    double weight_param;   /* p of the weight setting: c > 1 (HARMONIC_C),
                              delta_max > 0 (NORMALISED), w_l / w_v >= 0
                              (FIXED); ignored otherwise                   [0] */
    int32_t builder;       /* where the edge candidates come from:
                              NHQ_BUILD_EXACT: the exact l nearest (all pairs
                              on the matrix cores);
                              NHQ_BUILD_NNDESCENT: NN-descent lists (the
                              NPG_kgraph build, Sec. 4.3) of l = cand entries
                              from nhq_nndescent_lists with this index's seed,
                              re-ordered by the exact FP64 key before the
                              edge selection; needs cand <= 128 < n;
                              NHQ_BUILD_NSW: see below                     [0] */
    int32_t nnd_rounds;    /* NN-descent: most rounds after the start     [12] */
    int32_t nnd_sample;    /* NN-descent: new entries explored per list
                              and round (s)                                [24] */
    float nnd_stop;        /* NN-descent: stop after a round that brings
                              fewer than nnd_stop * n * l new entries  [0.001] */
    int32_t nsw_batch;     /* NSW insertion: vertices inserted per batch
                              (1: one at a time)                       [10000] */
    int32_t nsw_beam;      /* NSW insertion: beam of each insertion search
                              (>= cand)                                 [cand] */
    int64_t capacity;      /* rows the index can hold: nhq_index_insert
                              appends up to capacity - n objects           [n] */
    int32_t entry_per_pattern; /* > 0: stratified entry sample.  Besides the
                              n_entry random members, the index keeps one
                              block per attribute pattern (full code tuple)
                              that objects hold: the min(entry_per_pattern,
                              count) objects of the pattern with the smallest
                              (h(i), i), h(i) the first splitmix64 output
                              from state (seed ^ 0x8F14E45FCEEA167A) ^
                              (i * 0xD1B54A32D192ED03).  A query that
                              constrains every attribute takes its seeds from
                              its pattern's block (ranked by Gamma as the
                              global sample is); other queries, and patterns
                              no object holds, from the global sample.  The
                              seed set B of Alg. 2 is drawn at random
                              (Sec. 3.2); this keeps it random within each
                              pattern.  Needs m >= 1, n_entry and
                              entry_per_pattern <= 8192 and at most 4096
                              patterns.  0: off                        [0] */
} nhq_build_params;

#define NHQ_BUILD_EXACT 0
#define NHQ_BUILD_NNDESCENT 1
#define NHQ_BUILD_NSW 2 /* NPG_nsw (Sec. 4.3): vertices inserted in id order
                           in batches of nsw_batch.  The first batch takes the
                           exact cand nearest within itself; every later batch
                           searches the graph built so far (the search of
                           nhq_hybrid_search with the object's attributes all
                           constrained, beam nsw_beam, first cand pool entries,
                           seeds: the 16 best of the first min(s, 256)
                           distinct splitmix64(seed) values mod s, s the
                           vertices already in).  New rows are selected from
                           their candidates; every vertex a new row names
                           re-selects its row with the new vertex offered.
                           Reverse links are part of it (reverse_edges is
                           ignored).  Synchronises the stream per batch. */

/* NN-descent candidate lists (the refinement of NPG_kgraph, Sec. 4.3; Eq. 7
 * measures their quality), in synchronous rounds so that the result does
 * not depend on scheduling:
 *   round 0: C(i) = the first l distinct values v != i of splitmix64 with
 *            state seed ^ (i * 0xD1B54A32D192ED03), taken mod n, ordered by
 *            (key, id), all entries new;
 *   round t: J = the first s new entries of C(i); the ids of C(j), j in J,
 *            that are neither i nor in C(i) are scored; C(i) becomes the l
 *            best of C(i) and them by (key, id); they enter new, J turns old.
 * Keys: float32 object-object fusion keys of the index's weight setting
 * over all m attributes.  Runs `rounds` rounds, or stops after the first
 * round that brings fewer than stop_frac * n * l new entries (stop_frac
 * <= 0: never).  ids: DEVICE int32 [n][l] (caller-owned), each row sorted
 * by (key, id).  updates: nullable HOST int64 [rounds], the new entries of
 * each round.  rounds_run: nullable HOST, the rounds done.  Needs
 * 1 <= l <= 128, n > l, 0 <= s <= 64.  Synchronises the stream once per
 * round. */
int nhq_nndescent_lists(const nhq_index *ix, int32_t l, int32_t s, int32_t rounds,
                        double stop_frac, uint64_t seed, int32_t *ids, int64_t *updates,
                        int32_t *rounds_run, void *stream);

/* Incremental insertion (NPG_nsw, Sec. 4.3): appends nb objects (DEVICE
 * float32 [nb][d], DEVICE uint8 codes [nb][m]) as ids n .. n + nb - 1 and
 * links them into the graph exactly as the NSW build's later batches do
 * (batches of nsw_batch, insertion beam nsw_beam, the index's seed).  Needs
 * a graph, n + nb <= capacity, and codes that fit the index's packed fields
 * (NHQ_EINVAL otherwise; nothing changes then).  The entry sample and the
 * per-code statistics keep the values of the objects present at creation.
 * Synchronises the stream per batch. */
int nhq_index_insert(nhq_index *ix, const float *vecs, const uint8_t *attrs, int64_t nb,
                     void *stream);

/* Rounds the last NN-descent build of the index ran (0 for an exact build). */
int nhq_index_build_report(const nhq_index *ix, int32_t *nnd_rounds_run);

/* Per-checkpoint search traces (training data of the stop network).  Every
 * check_every hops the search records 8 state features, the hop count and a
 * fingerprint of its current top-k eligible ids; at the end the fingerprint
 * of the final top-k.  Device arrays: feat float32 [nq][cap][8], hop uint32
 * [nq][cap], hash uint32 [nq][cap], count int32 [nq] (checkpoints written),
 * final_hash uint32 [nq]. */
typedef struct {
    float *feat;
    uint32_t *hop;
    uint32_t *hash;
    int32_t *count;
    uint32_t *final_hash;
    int32_t cap;
} nhq_trace;

/* Search parameters (Alg. 2).  Pass NULL for all defaults. */
typedef struct {
    int32_t n_init;      /* seed set size: the best n_init members of the
                            entry sample start the pool                   [32] */
    int32_t rerank;      /* r in [1, 64]: re-score the first min(r*k, beam)
                            eligible pool entries from the float32 copy and
                            re-sort (precision form); 0: off               [0] */
    int32_t output_mode; /* 0: exact attribute matches only (Def. 4);
                            1: the first k pool entries by Gamma           [0] */
    int32_t max_hops;    /* expansion cap; reaching it sets the error word
                            bit NHQ_DEVERR_HOPCAP                      [100000] */
    int32_t visited_log2;/* log2 slots of the per-query visited hash (10..13);
                            0 = automatic                                  [0] */
    int32_t learned;     /* 1: in-loop stop/beam network (needs nhq_mlp_load),
                            evaluated every check_every hops; 2: evaluated
                            once, at hop check_every, where it may stop the
                            search and otherwise sets the hop budget
                            cap_factor * 2^(beam output) (cap_factor > 0);
                            3: the beam-width predictor, evaluated once, at
                            hop check_every: the pool size becomes
                            ceil(cap_factor * 2^(beam output)), clamped to
                            [k, beam], for the rest of the search (the pool
                            keeps its best entries; the stop logit is not
                            read; cap_factor > 0)                          [0] */
    float stop_threshold;/* stop when sigmoid(stop logit) exceeds it    [0.5] */
    int32_t check_every; /* network evaluated every this many hops        [4] */
    uint32_t *counters;  /* nullable DEVICE uint32 [nq][2]: NDC (neighbour
                            distance evaluations) and H (expansions)          */
    float cap_factor;    /* learned 1 or 2, > 0: stop at cap_factor * 2^(beam
                            output at the first checkpoint) hops, checked
                            before every step; learned 3: the pool size
                            factor                                         [0] */
    const nhq_trace *trace; /* nullable: record checkpoint traces           */
    int32_t expand;      /* vertices expanded per step: the `expand` best
                            unexpanded pool entries are expanded together and
                            their neighbours merged as one batch (1..8)    [1] */
    int32_t route_h;     /* h >= 2: two-stage routing (Sec. 4.2).  In stage
                            S1 an expanded vertex u evaluates only its slots r
                            with (r + fmix32(u * 0x9E3779B1 + t)) mod h = 0,
                            t its expansion number (hops before it), i.e.
                            about ceil(R / h) neighbours; at the first step
                            that inserts nothing into the pool every pool
                            entry becomes unexpanded again and stage S2 (all
                            neighbours, Alg. 2) runs to the end.  0 or 1: off
                                                                          [0] */
    const int32_t *order;/* nullable DEVICE int32 [nq]: launch order, the
                            i-th wavefront searching query order[i] (results
                            stay in query order and do not depend on it);
                            nhq_query_order writes one that launches the
                            least selective queries first.  An entry outside
                            [0, nq) is skipped and sets NHQ_DEVERR_BADID;
                            it must be a permutation for every query to be
                            searched                                       [0] */
} nhq_search_params;

/* Device error word bits (accumulated per index; nhq_index_device_error). */
#define NHQ_DEVERR_HOPCAP 0x1u
#define NHQ_DEVERR_BADID 0x2u

/* ------------------------------------------------------------------ index */

/* Ingest an object set (Def. 1): copies the vectors (padded to the kernel
 * width), packs the attribute codes, derives the storage form, the row norms
 * and the entry sample.  The graph is empty until nhq_index_build_graph or
 * nhq_index_set_graph.  vecs: device float32 [n][d]; attrs: device uint8
 * [n][m]; n in [1, 2^28); d in [1, 1024]; m in [0, 4].  Synchronises the
 * stream before returning (ingest statistics are read back). */
int nhq_index_create(const float *vecs, const uint8_t *attrs, int64_t n, int32_t d, int32_t m,
                     const nhq_build_params *params, void *stream, nhq_index **out);

/* Composite-index build on the GPU (Alg. 1 in degree-bounded form with the
 * fusion distance of Sec. 5.1): exact l nearest candidates under Gamma from
 * dense tiles, the landing-zone selection of Sec. 4.1 steps (1)-(3), and the
 * optional reverse-edge pass. */
int nhq_index_build_graph(nhq_index *ix, void *stream);

/* nhq_index_create followed by nhq_index_build_graph. */
int nhq_build_index(const float *vecs, const uint8_t *attrs, int64_t n, int32_t d, int32_t m,
                    const nhq_build_params *params, void *stream, nhq_index **out);

/* Install a graph built elsewhere: adj device int32 [n][degree], -1 padded,
 * ids in [0, n).  degree in [1, 64].  The index keeps its own copy. */
int nhq_index_set_graph(nhq_index *ix, const int32_t *adj, int32_t degree, void *stream);

/* Copy the graph (device int32 [n][degree]) / the entry sample (device int32
 * [n_entry], the global members only) out of the index. */
int nhq_index_get_graph(const nhq_index *ix, int32_t *adj_out, void *stream);
int nhq_index_get_entry(const nhq_index *ix, int32_t *entry_out, void *stream);

/* The blocks of a stratified entry sample (entry_per_pattern > 0): *n_blocks
 * (host) = number of patterns the objects hold (0 when off); codes (host,
 * nullable) uint8 [n_blocks][m]: each block's attribute codes, blocks in
 * increasing order of their packed codes; offsets (host, nullable) int32
 * [n_blocks + 1]: block b holds entry positions offsets[b] ..
 * offsets[b + 1] - 1 (offsets[0] = n_entry: the positions after the global
 * members, as nhq_seed_rank returns them); ids (device, nullable) int32
 * [offsets[n_blocks] - n_entry]: the block members' vertex ids, block after
 * block, each block in increasing (h(i), i).  Synchronises the stream when
 * ids is given. */
int nhq_index_entry_blocks(const nhq_index *ix, int32_t *n_blocks, uint8_t *codes, int32_t *offsets,
                           int32_t *ids, void *stream);

/* Copy the storage form the search scores with: rows padded to the kernel
 * width dp (returned in *dp_out): float32 [n][dp], bf16 bit patterns uint16
 * [n][dp] or OCP e4m3 codes uint8 [n][dp]; scales (fp8 only, else untouched)
 * float32 [n].  Device outputs; scales may be NULL. */
int nhq_index_get_storage(const nhq_index *ix, void *rows_out, float *scales_out, int32_t *dp_out,
                          void *stream);

/* Shape queries (host outputs, any may be NULL). */
int nhq_index_info(const nhq_index *ix, int64_t *n, int32_t *d, int32_t *m, int32_t *degree,
                   int32_t *storage, int32_t *n_entry);

/* Read and clear the index's device error word (synchronises the stream). */
int nhq_index_device_error(nhq_index *ix, void *stream, uint32_t *bits_out);

void nhq_index_free(nhq_index *ix);

/* Index files (the "save / load" of a built index; Alg. 1's output with
 * everything the search reads).  nhq_index_save synchronises `stream`, then
 * writes the index's parameters and its first n rows of every array --
 * float32 rows, storage form (and fp8 scales), packed codes, norms, graph,
 * entry sample (and its exact bf16 copy), code log-frequencies and the stop
 * network when loaded -- to `path` (host path; written as `path`.partial and
 * renamed over `path` once complete, so a failed save leaves `path` as it
 * was).
 * nhq_index_load reads such a file onto the current device and returns a new
 * index with the saved capacity (rows past n free for nhq_index_insert) that
 * answers every call as the saved one did.  NHQ_EIO: the file cannot be
 * opened, written or read, is not an index file of this version, is
 * truncated or has trailing bytes, or its header is inconsistent; the index
 * is then not created. */
int nhq_index_save(const nhq_index *ix, const char *path, void *stream);
int nhq_index_load(const char *path, void *stream, nhq_index **out);

/* ----------------------------------------------------------------- search */

/* Hybrid query (Def. 4) answered by joint pruning (Alg. 2) in beam form: one
 * wavefront per query keeps the `beam` best vertices by Gamma in LDS, expands
 * the best unexpanded one (gathers its adjacency row, the attribute words and
 * vectors of its unvisited neighbours), offers each neighbour to the pool,
 * and stops when every pool entry is expanded.  Output per output_mode.
 * queries: device float32 [nq][d]; qattrs: device uint8 [nq][m];
 * 1 <= k <= beam <= 1024; ids: device int32 [nq][k]; dists: device float32
 * [nq][k].  nq = 0 is a no-op.  Batches of 2,048 queries and more whose
 * parameters name no launch order are launched in nhq_seed_order's order
 * (results do not depend on it). */
int nhq_hybrid_search(const nhq_index *ix, const float *queries, const uint8_t *qattrs,
                      int64_t nq, int32_t k, int32_t beam, const nhq_search_params *sp,
                      int32_t *ids, float *dists, void *stream);

/* The two stages of nhq_hybrid_search, for callers that time or overlap them.
 *
 * nhq_seed_rank: the seed set B of Alg. 2 is taken from the index's random
 * entry sample (Sec. 3.2: seeds are usually drawn at random); this ranks the
 * whole sample for every query by Gamma on the matrix cores and writes the
 * positions (in the entry sample) of the n_cand best, -1 padded, to cand:
 * device int32 [nq][n_cand], 1 <= n_cand <= 144.  Its scratch (about
 * nq * (8 d + 4.25 n_entry) bytes) lives in the index's workspace, which a
 * call that needs more than any call before it grows (that call synchronises
 * the device); nhq_hybrid_search keeps the candidates there too.
 *
 * nhq_search_seeded: the joint-pruning search given those candidates: it
 * re-scores them exactly, starts the pool with the best n_init of them and
 * runs the expansion loop.  nhq_hybrid_search passes n_cand = min(n_entry,
 * n_init + 8); the result then equals a search started from the best n_init
 * members of the whole entry sample unless the dense ranking (the GEMM form
 * of delta^2 on split-bf16 products, about 2^-17 relative error per term)
 * misplaces one past the 8-entry margin (never when the queries and the
 * entry sample hold values exact in bf16 whose partial sums stay exact in
 * float32, such as integers of magnitude <= 256 in rows of at most 128
 * elements: then the ranking is exact). */
int nhq_seed_rank(const nhq_index *ix, const float *queries, const uint8_t *qattrs, int64_t nq,
                  int32_t n_cand, int32_t *cand, void *stream);

/* nhq_seed_rank with the caller's scratch in place of the index's
 * workspace (same ranking, bit-identical candidates): workspace is device
 * memory on the index's device, 256-byte aligned, of at least the
 * workspace_size bytes for the same nq and n_cand (host size_t *bytes; the
 * size depends on the index's padded width and entry sample), owned by the
 * caller.  The call only reads the index, so calls with different
 * workspaces may run at the same time on different streams: that keeps
 * several batches in flight, and each batch's seed ranking and search fill
 * the device while another batch's last queries finish.  NHQ_EINVAL for a
 * null, misaligned or short workspace, else as nhq_seed_rank. */
int nhq_seed_rank_workspace_size(const nhq_index *ix, int64_t nq, int32_t n_cand, size_t *bytes);
int nhq_seed_rank_ws(const nhq_index *ix, const float *queries, const uint8_t *qattrs, int64_t nq,
                     int32_t n_cand, int32_t *cand, void *workspace, size_t workspace_bytes, void *stream);
int nhq_search_seeded(const nhq_index *ix, const float *queries, const uint8_t *qattrs, int64_t nq,
                      const int32_t *cand, int32_t n_cand, int32_t k, int32_t beam,
                      const nhq_search_params *sp, int32_t *ids, float *dists, void *stream);

/* A launch order for nhq_search_params.order: the queries by decreasing
 * selectivity fraction, least selective first, estimated from the object
 * set's code frequencies as sum over the constrained attributes of
 * ln(count(code) / n) (count 0 read as 0.5), in buckets of 1/16.  Queries
 * that match more objects need more hops (fewer constrained attributes,
 * frequent codes), so launching them first shortens the batch's tail, and
 * queries of one attribute pattern run side by side.  The order is a
 * scheduling choice only: results do not depend on it.  qattrs: device
 * uint8 [nq][m]; order: device int32 [nq], a permutation of 0 .. nq - 1 on
 * return.  Uses the index's workspace (see nhq_seed_rank). */
int nhq_query_order(const nhq_index *ix, const uint8_t *qattrs, int64_t nq, int32_t *order, void *stream);

/* A launch order for nhq_search_params.order from the batch's seed
 * candidates (nhq_seed_rank's cand, [nq][n_cand]): the queries grouped by
 * the lowest entry-sample position among their candidates, each group's
 * wavefronts kept on one XCD.  Queries that share a member of the entry
 * sample among their seed candidates search one part of the graph and read
 * many of the same rows; workgroups go to the device's 8 XCDs
 * round-robin, so XCD x is given the x-th of 8 contiguous runs of the
 * grouped queries, and their rows meet in that XCD's L2.  The groups are
 * taken in a scrambled order of their entry positions, so each XCD's run
 * mixes many groups and the runs cost about the same (the blocks of a
 * stratified sample sit at neighbouring positions).  A scheduling
 * choice only: results do not depend on it.  order: device int32 [nq], a
 * permutation of 0 .. nq - 1 (wave i searches query order[i]).  workspace:
 * null for the index's workspace (calls on one index then go on one
 * stream), else 256-byte aligned device memory of at least 4 (1024 + 2 nq)
 * bytes -- the workspace of nhq_seed_rank_ws for the same batch is large
 * enough.  nhq_hybrid_search applies this order itself to batches of 2,048
 * queries and more when its parameters name no order. */
int nhq_seed_order(const nhq_index *ix, const int32_t *cand, int32_t n_cand, int64_t nq, int32_t *order,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Allocation-free nhq_hybrid_search, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and results as
 * nhq_hybrid_search (bit-identical outputs), but the seed ranking's scratch
 * (the candidates and the ranking's padded queries, key matrix and group
 * minima) lives in a fixed array of NHQ_NOALLOC_SCRATCH_BYTES in each
 * device's memory, which the library holds until the process ends; the call
 * itself allocates and frees nothing (its first call on a device looks the
 * array's address up once).  The batch must fit: with ks = min(n_entry,
 * n_init + 8), dp the padded width and E = n_entry rounded up to 64, it
 * needs roundup256(4 nq ks) + 4 (2 nq dp + 5 nq + nq E 17 / 16 + 128) bytes;
 * larger batches fail with NHQ_EINVAL (split them), and an entry sample of
 * more than 8192 with NHQ_ENOTSUP.  Every call on a device shares that
 * device's array and leaves its contents behind (nothing in it needs to start
 * at zero): calls that overlap on one device -- on different streams or from
 * different host threads -- race and must not be made; calls ordered on one
 * stream are safe. */
#define NHQ_NOALLOC_SCRATCH_BYTES (64u << 20)
int nhq_hybrid_search_noalloc(const nhq_index *ix, const float *queries, const uint8_t *qattrs,
                              int64_t nq, int32_t k, int32_t beam, const nhq_search_params *sp,
                              int32_t *ids, float *dists, void *stream);

/* Exact hybrid k-NN (Def. 4 with Def. 2): exact attribute filter, then the k
 * nearest matches by (delta, id).  Same argument layout as the search; k in
 * [1, 128].  dists are delta (= Gamma for matches), rounded to float32 from a
 * float64 direct-form re-score of the dense tiles' k + 16 best.  Uses
 * stream-ordered temporary allocations. */
int nhq_bruteforce_hybrid_knn(const nhq_index *ix, const float *queries, const uint8_t *qattrs,
                              int64_t nq, int32_t k, int32_t *ids, float *dists, void *stream);

/* ------------------------------------------------------ learned stop network
 *
 * A small network (8 -> 64 -> 64 -> 2, ReLU) reads the search-state features
 * at every checkpoint and outputs a stop logit and log2 of a hop budget.
 * The paper names learned routing only as prior art (Sec. 4.2); the network,
 * its features and labels are this library's design (stated in nhq_trace
 * and below).  Parameters are float32 vectors of NHQ_MLP_PARAMS values in the
 * order W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]. */
#define NHQ_MLP_PARAMS 4866

/* Training samples from traces: sample (q, c) for every checkpoint c <
 * count[q]: X = feat, y_stop = 1 when the checkpoint's top-k fingerprint
 * equals the final one (continuing would not change the answer), y_beam =
 * log2 of the hop of the first checkpoint from which every later one holds
 * the final top-k (the final hop count H, from counters [nq][2], when the
 * last one does not).  Outputs are device float32:
 * X [nq*cap][8], y_stop [nq*cap], y_beam [nq*cap]; *n_out (host) = samples
 * written, in (q, c) order.  Synchronises the stream. */
int nhq_trace_samples(const nhq_trace *tr, int64_t nq, const uint32_t *counters, float *X,
                      float *y_stop, float *y_beam, int64_t *n_out, void *stream);

/* Loss and gradient of the mean loss over n samples (binary cross-entropy
 * of the stop logit plus lam * Huber(1) of the beam output) at `params`
 * (device float32 [NHQ_MLP_PARAMS]); grad device [NHQ_MLP_PARAMS], loss
 * device [1], z (nullable) device [n][2] network outputs. */
int nhq_mlp_grad(const float *params, const float *X, const float *y_stop, const float *y_beam,
                 int64_t n, float lam, float *grad, float *loss, float *z, void *stream);

/* Adam training (Kingma and Ba) of `params` in place for `epochs` passes
 * over the samples in mini-batches of `batch` (a multiple of 128), shuffled
 * per epoch from `seed`.  adam_state: device float32 [2 * NHQ_MLP_PARAMS]
 * (first and second moments; zero it to start), step: host in/out count of
 * Adam steps taken.  loss_out (nullable): device float32 [epochs], mean
 * loss per epoch. */
int nhq_mlp_train(float *params, float *adam_state, int64_t *step, const float *X,
                  const float *y_stop, const float *y_beam, int64_t n, int32_t epochs,
                  int32_t batch, float lr, float lam, uint64_t seed, float *loss_out, void *stream);

/* Install the network in the index (rounded to fp16) for learned searches;
 * params NULL removes it. */
int nhq_mlp_load(nhq_index *ix, const float *params, void *stream);

/* The in-loop inference on given features (fp16 weights, float32
 * accumulation): X device [n][8], Z device [n][2]. */
int nhq_mlp_eval(const nhq_index *ix, const float *X, int64_t n, float *Z, void *stream);

/* ---------------------------------------------------------------- serving
 *
 * Continuous batching of hybrid queries (Def. 4, answered as by
 * nhq_hybrid_search): a server keeps one persistent kernel resident on the
 * device, whose slots belong to one or two memory classes.  A class is the
 * largest beam its slots hold and fixes the LDS its requests use (pool,
 * staging, visited set, entry-sample keys); every slot of the launch holds
 * the largest class's LDS.  A slot is one wavefront serving one request at a
 * time.  (One launch keeps the classes running side by side: persistent
 * launches on separate streams may share a hardware queue and then run one
 * after the other.)  Requests go to the
 * smallest class whose beam covers theirs ("admission by memory") and are
 * taken by the next free slot of that class as soon as they are published,
 * while the other slots keep working: requests that arrive while others run
 * share the device with them.  Requests and results travel through pinned
 * host memory (a ring per class); the caller never synchronises a stream.
 *
 * Each request's result depends only on the request, the index and the
 * server parameters (every slot has its own pool and visited set; the seed
 * set is the n_cand best of the entry sample, ranked in-wave in float32
 * direct form, then the search of nhq_search_seeded): the same request gives
 * bit-identical ids, distances and counters alone or in any mix.
 *
 * The server reads the index (which must outlive it and stay unchanged) and
 * the kernel holds its slots until nhq_server_free.  While a server runs,
 * do not synchronise the whole device (hipDeviceSynchronize waits for the
 * persistent kernel); synchronise streams instead.  Every kernel wait is
 * bounded by the stop flag and by lifetime_s, after which the kernel ends
 * by itself and later submits fail with NHQ_EDEVICE.  The server calls
 * are not thread-safe: one host thread drives a server. */
typedef struct nhq_server nhq_server;

typedef struct {
    int32_t beam_small;  /* largest beam of the small memory class        [128] */
    int32_t beam_large;  /* largest beam of the large class; < 0: none     [512] */
    int32_t slots_small; /* slots (concurrent requests) of the small class;
                            0 = as many as 60% of the chip holds (30% for the
                            large class)                                     [0] */
    int32_t slots_large;
    int32_t ring;        /* requests submitted and not yet polled, per class
                            (host ring entries)                           [4096] */
    int32_t max_k;       /* largest k of a request                          [100] */
    int32_t n_init;      /* seed set size (as nhq_search_params)             [32] */
    int32_t expand;      /* vertices expanded per step                        [1] */
    int32_t rerank;      /* r > 0: rerank the first min(r*k, beam) eligible
                            entries from the float32 copy                    [0] */
    int32_t check_every; /* learned stop: checkpoint spacing in hops          [4] */
    int32_t auto_beam;   /* beam of requests submitted with beam 0, which use
                            the learned stop (needs nhq_mlp_load)   [beam_small] */
    int32_t max_hops;    /* expansion cap                               [100000] */
    float stop_threshold;/* learned stop threshold                          [0.5] */
    float cap_factor;    /* learned hop budget factor (0 = none), or the
                            pool size factor of learned mode 3               [0] */
    int32_t learned_mode;/* learned requests: 1, 2 or 3 (as
                            nhq_search_params.learned)                       [1] */
    int32_t reserved1;
    double lifetime_s;   /* the kernel ends by itself after this long      [600] */
} nhq_server_params;

#define NHQ_SERVE_RAW 1 /* request flag: output_mode 1 (first k by Gamma) */
#define NHQ_PENDING 1   /* nhq_server_poll: the request has not finished */

/* Start a server on the index's device (launches the kernel; synchronises
 * the device once before launching). */
int nhq_server_create(nhq_index *ix, const nhq_server_params *params, nhq_server **out);

/* Per class (host arrays of 2; class 1 reads 0 slots when absent): slots,
 * LDS bytes a request of the class uses, largest beam; tick_hz: rate of the
 * device wall clock that nhq_server_poll's ticks count. */
int nhq_server_info(const nhq_server *s, int32_t *slots, int32_t *lds_bytes, int32_t *beam_max,
                    double *tick_hz);

/* Submit one request: q host float32 [d], qattr host uint8 [m] (0xFF =
 * wildcard), 1 <= k <= min(max_k, beam), beam 0 = learned stop with
 * auto_beam.  flags: 0 or NHQ_SERVE_RAW.  Returns NHQ_EBUSY (nothing
 * submitted) when the class's next ring entry still holds an unpolled
 * request.  *ticket identifies the request for nhq_server_poll. */
int nhq_server_submit(nhq_server *s, const float *q, const uint8_t *qattr, int32_t k, int32_t beam,
                      int32_t flags, uint64_t *ticket);

/* Non-blocking: NHQ_PENDING while the request runs; NHQ_OK once it has
 * finished, with ids host int32 [k] (-1 padded), dists host float32 [k]
 * (Gamma, +inf padded), counters host uint32 [2] (NDC, hops; nullable) and
 * ticks host uint64 [2] (device wall clock at the slot's start and end of
 * the request; nullable).  A ticket can be polled to completion once. */
int nhq_server_poll(nhq_server *s, uint64_t ticket, int32_t *ids, float *dists, uint32_t *counters,
                    uint64_t *ticks);

/* Open-loop driver in native code: submits request i at arrival_s[i] seconds
 * after the call starts (non-decreasing; a request that finds its ring full
 * waits and keeps its arrival time), polls completions and records
 * latency_s[i] = time its result was seen - arrival_s[i].  All arrays are
 * host memory: q [n][d], qattrs [n][m], k [n], beam [n], flags [n]
 * (nullable), ids [n][max_k], dists [n][max_k] (padded past k), counters
 * [n][2] and ticks [n][2] (nullable), latency_s [n]; *elapsed_s (nullable)
 * = wall time until the last result.  Fails with NHQ_EDEVICE after
 * timeout_s seconds (<= 0: 60). */
int nhq_server_run(nhq_server *s, const float *q, const uint8_t *qattrs, const int32_t *k,
                   const int32_t *beam, const int32_t *flags, const double *arrival_s, int64_t n,
                   int32_t *ids, float *dists, uint32_t *counters, uint64_t *ticks, double *latency_s,
                   double *elapsed_s, double timeout_s);

/* Stop the kernels (waits up to 30 s for them to end) and release the
 * server.  Returns NHQ_EDEVICE and keeps the server's memory if the kernels
 * did not end. */
int nhq_server_free(nhq_server *s);

/* ------------------------------------------------------------ measurement */

/* Random-row gather probe: `waves` wavefronts (a multiple of 4) each read
 * rounds * (64 / G) whole stored rows of the index at pseudo-random
 * positions (a counter-based hash of seed, wave and row), with the search's
 * lane layout and rounds in flight, and write per-lane sums to sink (device
 * float32 [waves][64]) so that nothing is optimised away.  *rows_read (host,
 * nullable) = rows read.  Timing it gives the bandwidth ceiling of the
 * search's row gathers.  rounds must be a multiple of the rounds the search
 * keeps in flight: 2 when the padded width is at most 128, else 1. */
int nhq_gather_probe(const nhq_index *ix, int64_t waves, int32_t rounds, uint64_t seed, float *sink,
                     int64_t *rows_read, void *stream);

/* ------------------------------------------------------------------ misc */
const char *nhq_strerror(int code);
const char *nhq_last_error(void);
int nhq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NHQ_H */
