// Index files: nhq_index_save writes everything a search, a build step, an
// insertion or the learned stop reads from an index -- its parameters, the
// float32 rows and their storage form, codes, norms, graph, entry sample,
// selectivity table and stop network -- and nhq_index_load rebuilds the
// index on the current device from it, so a loaded index answers every call
// exactly as the saved one.
//
// Layout (little-endian): a fixed header (magic, version, sizes and
// parameters), then the arrays in a fixed order, each as raw bytes of its
// first n rows.  Arrays that an index may lack (storage copy, fp8 scales,
// graph, exact bf16 entry sample, stop network) are present iff the header
// says so.
#include <cstdio>
#include <cstring>
#include <vector>

#include "nhq_internal.h"

namespace nhq {
namespace {

constexpr char kMagic[8] = {'N', 'H', 'Q', 'I', 'D', 'X', 0, 1};
constexpr uint32_t kVersion = 1;
constexpr size_t kChunk = size_t(64) << 20;  // bytes per host staging copy

struct FileHeader {
    char magic[8];
    uint32_t version, header_bytes;
    int64_t n, cap;
    int32_t d, dp, m, degree, storage, cand, reverse_edges, n_entry;
    uint64_t seed;
    int32_t w_mode;
    float w_p;
    double w_pd;
    int32_t abits;
    uint32_t hmask;
    int32_t builder, nnd_rounds, nnd_sample;
    float nnd_stop;
    int32_t nnd_rounds_run, nsw_batch, nsw_beam;
    int32_t has_entry_bf16, has_mlp;
    // stratified entry sample: block count, members per pattern, and all
    // entry positions (the global members and every block); 0 when off
    int32_t n_blocks, per_pattern, n_entry_total;
    int32_t reserved[6];
};

size_t storage_elem(int storage)
{
    return storage == NHQ_STORAGE_BF16 ? 2 : storage == NHQ_STORAGE_FP8 ? 1 : 4;
}

// device -> file in chunks through one host buffer
int write_dev(FILE *f, const void *dev, size_t bytes, std::vector<char> &buf)
{
    for (size_t off = 0; off < bytes; off += kChunk) {
        const size_t b = std::min(kChunk, bytes - off);
        NHQ_HIP(hipMemcpy(buf.data(), static_cast<const char *>(dev) + off, b, hipMemcpyDeviceToHost));
        if (std::fwrite(buf.data(), 1, b, f) != b)
            return fail(NHQ_EIO, "index file write failed");
    }
    return NHQ_OK;
}

// file -> newly allocated device array of `alloc` bytes, the first `bytes`
// read from the file
int read_dev(FILE *f, void **dev, size_t bytes, size_t alloc, std::vector<char> &buf)
{
    if (hipMalloc(dev, std::max<size_t>(alloc, 4)) != hipSuccess) {
        *dev = nullptr;
        return fail(NHQ_ENOMEM, "index allocation failed");
    }
    for (size_t off = 0; off < bytes; off += kChunk) {
        const size_t b = std::min(kChunk, bytes - off);
        if (std::fread(buf.data(), 1, b, f) != b)
            return fail(NHQ_EIO, "index file is truncated");
        NHQ_HIP(hipMemcpy(static_cast<char *>(*dev) + off, buf.data(), b, hipMemcpyHostToDevice));
    }
    return NHQ_OK;
}

// bytes after the header that a file with header `hd` holds
uint64_t payload_bytes(const FileHeader &hd)
{
    const uint64_t n = (uint64_t)hd.n, dp = (uint64_t)hd.dp;
    const uint64_t ne = (uint64_t)(hd.n_blocks > 0 ? hd.n_entry_total : hd.n_entry);
    uint64_t b = 4 * n * dp;                                        // float32 rows
    if (hd.storage != NHQ_STORAGE_FP32)
        b += storage_elem(hd.storage) * n * dp;                     // storage form
    if (hd.storage == NHQ_STORAGE_FP8)
        b += 4 * n;                                                 // scales
    b += 4 * n + 4 * n;                                             // codes, norms
    b += 4 * n * (uint64_t)hd.degree;                               // graph
    b += 4 * ne + 4 * ne * dp + 4 * ne + 4 * ne;                    // entry sample
    if (hd.has_entry_bf16)
        b += 2 * (uint64_t)hd.n_entry * dp;                         // (global members)
    if (hd.n_blocks > 0)
        b += 4 * (uint64_t)hd.n_blocks + 4 * ((uint64_t)hd.n_blocks + 1);  // block words, offsets
    b += 4 * (uint64_t)NHQ_MAX_ATTRS * 256;                         // code log-frequencies
    if (hd.has_mlp)
        b += 2 * (uint64_t)NHQ_MLP_PARAMS;                          // stop network
    return b;
}

struct FileCloser {
    FILE *f;
    ~FileCloser()
    {
        if (f)
            std::fclose(f);
    }
};

}  // namespace
}  // namespace nhq

using namespace nhq;

extern "C" {

int nhq_index_save(const nhq_index *h, const char *path, void *stream)
{
    if (!h || !path)
        return fail(NHQ_EINVAL, "null argument");
    const Index *ix = &h->impl;
    NHQ_HIP(hipStreamSynchronize((hipStream_t)stream));
    FileHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, kMagic, sizeof(kMagic));
    hd.version = kVersion;
    hd.header_bytes = (uint32_t)sizeof(FileHeader);
    hd.n = ix->n;
    hd.cap = ix->cap;
    hd.d = ix->d;
    hd.dp = ix->dp;
    hd.m = ix->m;
    hd.degree = ix->degree;
    hd.storage = ix->storage;
    hd.cand = ix->cand;
    hd.reverse_edges = ix->reverse_edges;
    hd.n_entry = ix->n_entry;
    hd.seed = ix->seed;
    hd.w_mode = ix->w.mode;
    hd.w_p = ix->w.p;
    hd.w_pd = ix->w.pd;
    hd.abits = ix->abits;
    hd.hmask = ix->hmask;
    hd.builder = ix->builder;
    hd.nnd_rounds = ix->nnd_rounds;
    hd.nnd_sample = ix->nnd_sample;
    hd.nnd_stop = ix->nnd_stop;
    hd.nnd_rounds_run = ix->nnd_rounds_run;
    hd.nsw_batch = ix->nsw_batch;
    hd.nsw_beam = ix->nsw_beam;
    hd.has_entry_bf16 = ix->entry_bf16 ? 1 : 0;
    hd.has_mlp = ix->mlp ? 1 : 0;
    hd.n_blocks = ix->n_blocks;
    hd.per_pattern = ix->per_pattern;
    hd.n_entry_total = ix->n_blocks > 0 ? ix->n_entry_total : 0;
    // written to a temporary name, renamed into place once complete
    const std::string tmp = std::string(path) + ".partial";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f)
        return fail(NHQ_EIO, std::string("cannot open for writing: ") + tmp);
    FileCloser fc{f};
    if (std::fwrite(&hd, sizeof(hd), 1, f) != 1) {
        std::remove(tmp.c_str());
        return fail(NHQ_EIO, "index file write failed");
    }
    std::vector<char> buf(kChunk);
    const size_t n = (size_t)ix->n, ne = (size_t)ix->n_entry_total, dp = (size_t)ix->dp;
    int rc = write_dev(f, ix->vec32, sizeof(float) * n * dp, buf);
    if (rc == NHQ_OK && ix->storage != NHQ_STORAGE_FP32)
        rc = write_dev(f, ix->vecs, storage_elem(ix->storage) * n * dp, buf);
    if (rc == NHQ_OK && ix->storage == NHQ_STORAGE_FP8)
        rc = write_dev(f, ix->scale, sizeof(float) * n, buf);
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->attr, sizeof(uint32_t) * n, buf);
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->norm, sizeof(float) * n, buf);
    if (rc == NHQ_OK && ix->degree > 0)
        rc = write_dev(f, ix->adj, sizeof(int32_t) * n * (size_t)ix->degree, buf);
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->entry, sizeof(int32_t) * ne, buf);
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->entry_vec, sizeof(float) * ne * dp, buf);
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->entry_norm, sizeof(float) * ne, buf);
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->entry_attr, sizeof(uint32_t) * ne, buf);
    if (rc == NHQ_OK && ix->entry_bf16)
        rc = write_dev(f, ix->entry_bf16, sizeof(uint16_t) * (size_t)ix->n_entry * dp, buf);
    if (rc == NHQ_OK && ix->n_blocks > 0 &&
        (std::fwrite(ix->block_word_h.data(), sizeof(uint32_t), (size_t)ix->n_blocks, f) != (size_t)ix->n_blocks ||
         std::fwrite(ix->block_off_h.data(), sizeof(int32_t), (size_t)ix->n_blocks + 1, f) !=
             (size_t)ix->n_blocks + 1))
        rc = fail(NHQ_EIO, "index file write failed");
    if (rc == NHQ_OK)
        rc = write_dev(f, ix->logp, sizeof(float) * NHQ_MAX_ATTRS * 256, buf);
    if (rc == NHQ_OK && ix->mlp)
        rc = write_dev(f, ix->mlp, sizeof(uint16_t) * NHQ_MLP_PARAMS, buf);
    if (rc == NHQ_OK && std::fflush(f) != 0)
        rc = fail(NHQ_EIO, "index file write failed");
    const bool closed = std::fclose(f) == 0;
    fc.f = nullptr;
    if (rc == NHQ_OK && !closed)
        rc = fail(NHQ_EIO, "index file write failed");
    if (rc == NHQ_OK && std::rename(tmp.c_str(), path) != 0)
        rc = fail(NHQ_EIO, std::string("cannot rename the index file to ") + path);
    if (rc != NHQ_OK)
        std::remove(tmp.c_str());
    return rc;
}

int nhq_index_load(const char *path, void *stream, nhq_index **out)
{
    if (!path || !out)
        return fail(NHQ_EINVAL, "null argument");
    *out = nullptr;
    NHQ_HIP(hipStreamSynchronize((hipStream_t)stream));
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return fail(NHQ_EIO, std::string("cannot open for reading: ") + path);
    FileCloser fc{f};
    FileHeader hd;
    if (std::fread(&hd, sizeof(hd), 1, f) != 1 || std::memcmp(hd.magic, kMagic, sizeof(kMagic)) != 0)
        return fail(NHQ_EIO, "not an index file");
    if (hd.version != kVersion || hd.header_bytes != sizeof(FileHeader))
        return fail(NHQ_EIO, "unsupported index file version");
    if (hd.n < 1 || hd.n >= kMaxN || hd.cap < hd.n || hd.cap >= kMaxN || hd.d < 1 || hd.d > 1024 ||
        padded_dim(hd.d) != hd.dp || hd.m < 0 || hd.m > NHQ_MAX_ATTRS || hd.degree < 0 ||
        hd.degree > NHQ_MAX_DEGREE || hd.storage < 0 || hd.storage > 2 || hd.n_entry < 1 ||
        hd.n_entry > 65536 || hd.n_entry > hd.n || hd.n_blocks < 0 || hd.n_blocks > 4096 ||
        (hd.n_blocks > 0 && (hd.per_pattern < 1 || hd.per_pattern > 8192 || hd.n_entry_total < hd.n_entry ||
                             hd.n_entry_total > hd.n_entry + hd.n_blocks * hd.per_pattern)) ||
        hd.w_mode < NHQ_WEIGHTS_DEFAULT ||
        hd.w_mode > NHQ_WEIGHTS_FIXED || (hd.abits != 1 && hd.abits != 2 && hd.abits != 4 && hd.abits != 8))
        return fail(NHQ_EIO, "index file header is inconsistent");
    // the file must hold exactly what the header announces (checked before
    // any allocation)
    {
        const long here = std::ftell(f);
        if (here < 0 || std::fseek(f, 0, SEEK_END) != 0)
            return fail(NHQ_EIO, "index file is not seekable");
        const long end = std::ftell(f);
        if (end < 0 || std::fseek(f, here, SEEK_SET) != 0)
            return fail(NHQ_EIO, "index file is not seekable");
        const uint64_t have = (uint64_t)(end - here);
        const uint64_t want = payload_bytes(hd);
        if (have < want)
            return fail(NHQ_EIO, "index file is truncated");
        if (have > want)
            return fail(NHQ_EIO, "index file has trailing bytes");
    }
    nhq_index *h = new nhq_index();
    Index *ix = &h->impl;
    int rc = NHQ_OK;
    do {
        if (hipGetDevice(&ix->device) != hipSuccess) {
            rc = fail(NHQ_EHIP, "hipGetDevice failed");
            break;
        }
        ix->n = hd.n;
        ix->cap = hd.cap;
        ix->d = hd.d;
        ix->dp = hd.dp;
        ix->m = hd.m;
        ix->degree = hd.degree;
        ix->storage = hd.storage;
        ix->cand = hd.cand;
        ix->reverse_edges = hd.reverse_edges;
        ix->n_entry = hd.n_entry;
        ix->seed = hd.seed;
        ix->w.mode = hd.w_mode;
        ix->w.p = hd.w_p;
        ix->w.pd = hd.w_pd;
        ix->abits = hd.abits;
        ix->hmask = hd.hmask;
        ix->builder = hd.builder;
        ix->nnd_rounds = hd.nnd_rounds;
        ix->nnd_sample = hd.nnd_sample;
        ix->nnd_stop = hd.nnd_stop;
        ix->nnd_rounds_run = hd.nnd_rounds_run;
        ix->nsw_batch = hd.nsw_batch;
        ix->nsw_beam = hd.nsw_beam;
        std::vector<char> buf(kChunk);
        ix->n_blocks = hd.n_blocks;
        ix->per_pattern = hd.per_pattern;
        ix->n_entry_total = hd.n_blocks > 0 ? hd.n_entry_total : hd.n_entry;
        const size_t n = (size_t)hd.n, cap = (size_t)hd.cap, ne = (size_t)ix->n_entry_total, dp = (size_t)hd.dp;
        // every array goes straight into its field, so free_index releases
        // whatever a failed load had allocated
        if ((rc = read_dev(f, (void **)&ix->vec32, sizeof(float) * n * dp, sizeof(float) * cap * dp, buf)) !=
            NHQ_OK)
            break;
        if (hd.storage != NHQ_STORAGE_FP32) {
            const size_t el = storage_elem(hd.storage);
            if ((rc = read_dev(f, &ix->vecs, el * n * dp, el * cap * dp, buf)) != NHQ_OK)
                break;
        } else {
            ix->vecs = ix->vec32;
        }
        if (hd.storage == NHQ_STORAGE_FP8 &&
            (rc = read_dev(f, (void **)&ix->scale, sizeof(float) * n, sizeof(float) * cap, buf)) != NHQ_OK)
            break;
        if ((rc = read_dev(f, (void **)&ix->attr, sizeof(uint32_t) * n, sizeof(uint32_t) * cap, buf)) != NHQ_OK)
            break;
        if ((rc = read_dev(f, (void **)&ix->norm, sizeof(float) * n, sizeof(float) * cap, buf)) != NHQ_OK)
            break;
        if (hd.degree > 0) {
            const size_t deg = (size_t)hd.degree;
            if ((rc = read_dev(f, (void **)&ix->adj, sizeof(int32_t) * n * deg, sizeof(int32_t) * cap * deg,
                               buf)) != NHQ_OK)
                break;
            if (cap > n &&
                hipMemset(ix->adj + n * deg, 0xFF, sizeof(int32_t) * (cap - n) * deg) != hipSuccess) {
                rc = fail(NHQ_EHIP, "graph fill failed");
                break;
            }
        }
        if ((rc = read_dev(f, (void **)&ix->entry, sizeof(int32_t) * ne, sizeof(int32_t) * ne, buf)) != NHQ_OK)
            break;
        if ((rc = read_dev(f, (void **)&ix->entry_vec, sizeof(float) * ne * dp, sizeof(float) * ne * dp, buf)) !=
            NHQ_OK)
            break;
        // the matrix-core split of the entry rows is derived, not stored
        if (hipMalloc(&ix->entry_split, sizeof(uint16_t) * 2 * ne * dp) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "entry sample allocation failed");
            break;
        }
        if ((rc = launch_split_rows(ix->entry_vec, (int64_t)ne, (int)dp, ix->entry_split, (hipStream_t)stream)) !=
            NHQ_OK)
            break;
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
            rc = fail(NHQ_EHIP, "entry split failed");
            break;
        }
        if ((rc = read_dev(f, (void **)&ix->entry_norm, sizeof(float) * ne, sizeof(float) * ne, buf)) != NHQ_OK)
            break;
        if ((rc = read_dev(f, (void **)&ix->entry_attr, sizeof(uint32_t) * ne, sizeof(uint32_t) * ne, buf)) !=
            NHQ_OK)
            break;
        const size_t neg = (size_t)hd.n_entry;
        if (hd.has_entry_bf16 && (rc = read_dev(f, (void **)&ix->entry_bf16, sizeof(uint16_t) * neg * dp,
                                                sizeof(uint16_t) * neg * dp, buf)) != NHQ_OK)
            break;
        if (hd.n_blocks > 0) {
            const size_t B = (size_t)hd.n_blocks;
            ix->block_word_h.resize(B);
            ix->block_off_h.resize(B + 1);
            if (std::fread(ix->block_word_h.data(), sizeof(uint32_t), B, f) != B ||
                std::fread(ix->block_off_h.data(), sizeof(int32_t), B + 1, f) != B + 1) {
                rc = fail(NHQ_EIO, "index file is truncated");
                break;
            }
            bool ok = ix->block_off_h[0] == hd.n_entry && ix->block_off_h[B] == hd.n_entry_total;
            for (size_t b = 0; b < B && ok; ++b)
                ok = ix->block_off_h[b] < ix->block_off_h[b + 1] &&
                     ix->block_off_h[b + 1] - ix->block_off_h[b] <= hd.per_pattern &&
                     (b == 0 || ix->block_word_h[b - 1] < ix->block_word_h[b]);
            if (!ok) {
                rc = fail(NHQ_EIO, "index file block table is inconsistent");
                break;
            }
            if (hipMalloc(&ix->block_word, sizeof(uint32_t) * B) != hipSuccess ||
                hipMalloc(&ix->block_off, sizeof(int32_t) * (B + 1)) != hipSuccess ||
                hipMemcpy(ix->block_word, ix->block_word_h.data(), sizeof(uint32_t) * B, hipMemcpyHostToDevice) !=
                    hipSuccess ||
                hipMemcpy(ix->block_off, ix->block_off_h.data(), sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice) !=
                    hipSuccess) {
                rc = fail(NHQ_ENOMEM, "index allocation failed");
                break;
            }
        }
        const size_t lp = sizeof(float) * NHQ_MAX_ATTRS * 256;
        if ((rc = read_dev(f, (void **)&ix->logp, lp, lp, buf)) != NHQ_OK)
            break;
        const size_t mb = sizeof(uint16_t) * NHQ_MLP_PARAMS;
        if (hd.has_mlp && (rc = read_dev(f, &ix->mlp, mb, mb, buf)) != NHQ_OK)
            break;
        if (hipMalloc(&ix->err, 2 * sizeof(uint32_t)) != hipSuccess) {
            rc = fail(NHQ_ENOMEM, "index allocation failed");
            break;
        }
        if (hipMemset(ix->err, 0, 2 * sizeof(uint32_t)) != hipSuccess) {
            rc = fail(NHQ_EHIP, "memset failed");
            break;
        }
        char extra;
        if (std::fread(&extra, 1, 1, f) != 0) {
            rc = fail(NHQ_EIO, "index file has trailing bytes");
            break;
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

}  // extern "C"
