/*
 * CPU oracle for native hybrid queries (NHQ) -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C in FP64.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product path never does.  It shares no code, header or table with the GPU
 * path.
 *
 * What it computes (paper sections cited per function):
 *   chi     attribute distance, Eq. (4)-(5), restricted to the constrained
 *           attributes of a query (wildcards contribute nothing);
 *   delta2  squared Euclidean distance, Eq. (1), FP64 direct form;
 *   gamma   fusion distance, Eq. (6), with the default weights of Sec. 3.2
 *           (w_v = 1, w_l = delta / m) or one of the other settings that
 *           Sec. 6.5 compares (Eq. 8 among them);
 *   bruteforce   exact hybrid top-k (Def. 4 with Def. 2): exact attribute
 *           filter, then exact vector top-k ordered by (delta, id);
 *   build   composite index (Alg. 1 in degree-bounded form): exact l nearest
 *           candidates under Gamma, then the landing-zone edge selection of
 *           Sec. 4.1 steps (1)-(3) (Def. 7), optional reverse-edge pass;
 *   search  joint pruning (Alg. 2) in beam form: a pool of the L best
 *           vertices by Gamma, each expanded once, until no unexpanded entry
 *           remains; output filtered to exact attribute matches (Def. 4).
 *
 * Ordering keys.  Gamma = delta * (m_q + chi) / m_q is ordered through the
 * monotone key (m_q * Gamma)^2 = delta^2 * (m_q + chi)^2 (key = delta^2 when
 * m_q = 0).  KEY64 evaluates it in FP64 (exact on integer-valued vectors).
 * KEY32 rounds delta^2 to float and takes one float multiply, which is the
 * precision a float32 kernel takes the same ordering decision in; on
 * integer-valued vectors (delta^2 < 2^24) it is reproducible bit for bit.
 * Ties are broken by the smaller id everywhere.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_WILDCARD 0xFF
#define OR_MAXM 16 /* attributes the learned-stop features read */
#define OR_KEY64 0
#define OR_KEY32 1

/* ---------------------------------------------------------------- Eq. 1 */
double or_delta2(const float *x, const float *y, int d)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        double t = (double)x[i] - (double)y[i];
        s += t * t;
    }
    return s;
}

/* ------------------------------------------------------------ Eq. 4, 5 */
/* phi = 1 where codes differ; summed over the attributes the query
 * constrains (code != wildcard).  For two objects every attribute counts. */
int or_chi(const uint8_t *qa, const uint8_t *ea, int m)
{
    int c = 0;
    for (int i = 0; i < m; ++i)
        if (qa[i] != OR_WILDCARD && qa[i] != ea[i])
            c += 1;
    return c;
}

int or_arity(const uint8_t *qa, int m)
{
    int c = 0;
    for (int i = 0; i < m; ++i)
        if (qa[i] != OR_WILDCARD)
            c += 1;
    return c;
}

/* ---------------------------------------------------------------- Eq. 6 */
/* The weight settings of Sec. 6.5 (Fig. 10 (i), curves i-v).  Set once per
 * call through or_set_weights; every Gamma and ordering key below follows it.
 *   OR_W_DEFAULT     w_v = 1, w_l = delta / m_q             (curve iv)
 *   OR_W_HARMONIC    w_v = chi / (delta + chi), w_l = delta / (delta + chi):
 *                    Gamma = 2 delta chi / (delta + chi), 0 when both are 0
 *                                                            (curve i)
 *   OR_W_HARMONIC_C  curve i with chi replaced by 1 when chi = 0 and by
 *                    c * chi otherwise (Eq. 8), c = the weight parameter
 *                                                            (curve ii)
 *   OR_W_NORMALISED  w_v = 1 / delta_max, w_l = 1 / chi_max, chi_max = m_q
 *                    (chi / chi_max read as 0 when m_q = 0), delta_max = the
 *                    weight parameter                        (curve iii)
 *   OR_W_FIXED       w_v = 1, w_l = the weight parameter (the ratio
 *                    w_l / w_v)                              (curve v) */
#define OR_W_DEFAULT 0
#define OR_W_HARMONIC 1
#define OR_W_HARMONIC_C 2
#define OR_W_NORMALISED 3
#define OR_W_FIXED 4
static int g_wmode = OR_W_DEFAULT;
static double g_wparam = 0.0;

void or_set_weights(int mode, double param)
{
    g_wmode = mode;
    g_wparam = param;
}

double or_gamma(double delta, int chi, int mq)
{
    double c = (double)chi;
    switch (g_wmode) {
    case OR_W_HARMONIC:
        return (delta + c == 0.0) ? 0.0 : (2.0 * delta * c) / (delta + c);
    case OR_W_HARMONIC_C:
        c = (chi == 0) ? 1.0 : g_wparam * c;
        return (2.0 * delta * c) / (delta + c);
    case OR_W_NORMALISED:
        return delta / g_wparam + (mq == 0 ? 0.0 : c / (double)mq);
    case OR_W_FIXED:
        return delta + g_wparam * c;
    default:
        if (mq == 0)
            return delta;
        return 1.0 * delta + (delta / (double)mq) * c;
    }
}

/* The same Gamma with every operation rounded to float32 (sqrt included),
 * in the order written above: the precision a float32 kernel decides in. */
static float gamma32(double d2, int chi, int mq)
{
    volatile float delta = sqrtf((float)d2);
    volatile float c = (float)chi, p = (float)g_wparam, t, u;
    switch (g_wmode) {
    case OR_W_HARMONIC:
        u = delta + c;
        if (u == 0.0f)
            return 0.0f;
        t = 2.0f * delta;
        t = t * c;
        return t / u;
    case OR_W_HARMONIC_C:
        if (chi == 0)
            c = 1.0f;
        else
            c = p * c;
        t = 2.0f * delta;
        t = t * c;
        u = delta + c;
        return t / u;
    case OR_W_NORMALISED:
        t = delta / p;
        u = mq == 0 ? 0.0f : c / (float)mq;
        return t + u;
    default: /* OR_W_FIXED */
        t = p * c;
        return delta + t;
    }
}

/* Ordering key.  Default weights: (m_q Gamma)^2 = delta^2 (m_q + chi)^2,
 * free of square roots; the other settings order by Gamma itself. */
double or_order_key(double d2, int chi, int mq, int mode)
{
    if (g_wmode != OR_W_DEFAULT) {
        if (mode == OR_KEY32)
            return (double)gamma32(d2, chi, mq);
        return or_gamma(sqrt(d2), chi, mq);
    }
    double mult = (mq == 0) ? 1.0 : (double)((mq + chi) * (mq + chi));
    if (mode == OR_KEY32) {
        volatile float f = (float)d2;
        volatile float g = (float)mult;
        volatile float kk = f * g;
        return (double)kk;
    }
    return d2 * mult;
}

/* (key, id) lexicographic comparison */
static int lt(double ka, int64_t ia, double kb, int64_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

/* ------------------------------------------------ Def. 4 exact top-k */
/* For each query: P = objects whose attributes equal the query's on every
 * constrained attribute; the answer is the k members of P with the smallest
 * (delta, id).  ids padded with -1, dist with +inf.  by_gamma != 0 instead
 * ranks every object by (Gamma, id) (an unfiltered ranking). */
void or_bruteforce(const float *x, const uint8_t *attrs, int64_t n, int d, int m,
                   const float *q, const uint8_t *qa, int64_t nq, int k, int by_gamma,
                   int32_t *out_ids, double *out_dist, int64_t *out_nmatch, int nthreads)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t iq = 0; iq < nq; ++iq) {
        const float *qv = q + iq * (int64_t)d;
        const uint8_t *qav = qa + iq * (int64_t)m;
        int mq = or_arity(qav, m);
        double *bk = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
        int64_t *bi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
        int cnt = 0;
        int64_t nmatch = 0;
        for (int64_t e = 0; e < n; ++e) {
            int c = or_chi(qav, attrs + e * (int64_t)m, m);
            if (c == 0)
                nmatch += 1;
            if (!by_gamma && c != 0)
                continue;
            double d2 = or_delta2(qv, x + e * (int64_t)d, d);
            double key = by_gamma ? or_order_key(d2, c, mq, OR_KEY64) : d2;
            if (k == 0)
                continue;
            if (cnt == k && !lt(key, e, bk[k - 1], bi[k - 1]))
                continue;
            /* insertion into the sorted top-k list */
            int pos = (cnt < k) ? cnt : k - 1;
            while (pos > 0 && lt(key, e, bk[pos - 1], bi[pos - 1])) {
                bk[pos] = bk[pos - 1];
                bi[pos] = bi[pos - 1];
                pos -= 1;
            }
            bk[pos] = key;
            bi[pos] = e;
            if (cnt < k)
                cnt += 1;
        }
        for (int j = 0; j < k; ++j) {
            if (j < cnt) {
                int64_t e = bi[j];
                out_ids[iq * k + j] = (int32_t)e;
                double d2 = or_delta2(qv, x + e * (int64_t)d, d);
                int c = or_chi(qav, attrs + e * (int64_t)m, m);
                out_dist[iq * k + j] = by_gamma ? or_gamma(sqrt(d2), c, mq) : sqrt(d2);
            } else {
                out_ids[iq * k + j] = -1;
                out_dist[iq * k + j] = INFINITY;
            }
        }
        if (out_nmatch)
            out_nmatch[iq] = nmatch;
        free(bk);
        free(bi);
    }
}

/* ---------------------------------------------- candidate lists (Sec. 4.1 (1)) */
/* Object-object fusion key: every one of the m attributes counts. */
static double obj_key(const float *x, const uint8_t *attrs, int d, int m, int64_t a, int64_t b)
{
    double d2 = or_delta2(x + a * (int64_t)d, x + b * (int64_t)d, d);
    int c = or_chi(attrs + a * (int64_t)m, attrs + b * (int64_t)m, m);
    return or_order_key(d2, c, m, OR_KEY64);
}

/* exact l nearest of vertex i among V \ {i}, by (key, id); returns count */
static int nearest_l(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int use_attrs,
                     int64_t i, int l, double *ck, int64_t *ci)
{
    int cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i)
            continue;
        double key = use_attrs ? obj_key(x, attrs, d, m, i, j)
                               : or_delta2(x + i * (int64_t)d, x + j * (int64_t)d, d);
        if (cnt == l && !lt(key, j, ck[l - 1], ci[l - 1]))
            continue;
        int pos = (cnt < l) ? cnt : l - 1;
        while (pos > 0 && lt(key, j, ck[pos - 1], ci[pos - 1])) {
            ck[pos] = ck[pos - 1];
            ci[pos] = ci[pos - 1];
            pos -= 1;
        }
        ck[pos] = key;
        ci[pos] = j;
        if (cnt < l)
            cnt += 1;
    }
    return cnt;
}

/* ------------------------------------- landing-zone selection (Sec. 4.1 (2)-(3)) */
/* Candidates arrive sorted by (key to i, id).  A candidate p joins N(i) iff
 * it lies in the intersection of the landing zones L(i, j) of every j
 * already in N(i): p must be strictly closer to i than to j (half-space
 * H(i, j), Def. 7); the ball B(i, Gamma(i, j)) is excluded because every
 * later candidate is at least as far from i as j is.  At most R neighbours. */
static int landing_zone_select(const float *x, const uint8_t *attrs, int d, int m, int64_t i,
                               const double *ck, const int64_t *ci, int nc, int R, int32_t *out)
{
    int nsel = 0;
    for (int t = 0; t < nc && nsel < R; ++t) {
        int64_t p = ci[t];
        double k_pi = ck[t];
        int ok = 1;
        for (int s = 0; s < nsel; ++s) {
            double k_pj = obj_key(x, attrs, d, m, p, out[s]);
            if (!(k_pi < k_pj)) {
                ok = 0;
                break;
            }
        }
        if (ok)
            out[nsel++] = (int32_t)p;
    }
    (void)i;
    return nsel;
}

/* Build adjacency rows.  rows == NULL: every vertex (then the optional
 * reverse pass runs); otherwise only the listed vertices, forward pass only.
 * adj_out: [nrows][R], -1 padded.  cand_out (nullable): [nrows][l]. */
void or_build(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int l, int R,
              int reverse, const int64_t *rows, int64_t nrows, int32_t *adj_out,
              int32_t *cand_out, int nthreads)
{
    int64_t nr = rows ? nrows : n;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
    for (int64_t r = 0; r < nr; ++r) {
        int64_t i = rows ? rows[r] : r;
        double *ck = (double *)malloc(sizeof(double) * (size_t)l);
        int64_t *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
        int nc = nearest_l(x, attrs, n, d, m, 1, i, l, ck, ci);
        if (cand_out)
            for (int t = 0; t < l; ++t)
                cand_out[r * l + t] = (t < nc) ? (int32_t)ci[t] : -1;
        int32_t *row = adj_out + r * (int64_t)R;
        int ns = landing_zone_select(x, attrs, d, m, i, ck, ci, nc, R, row);
        for (int t = ns; t < R; ++t)
            row[t] = -1;
        free(ck);
        free(ci);
    }
    if (rows || !reverse)
        return;

    /* Reverse pass: every j re-selects from N(j) united with the vertices that
     * chose j, ordered by (key to j, id), under the same landing-zone rule. */
    int64_t *offer_cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < R; ++t) {
            int32_t j = adj_out[i * R + t];
            if (j >= 0)
                offer_cnt[j + 1] += 1;
        }
    for (int64_t j = 0; j < n; ++j)
        offer_cnt[j + 1] += offer_cnt[j];
    int32_t *offers = (int32_t *)malloc(sizeof(int32_t) * (size_t)(offer_cnt[n] + 1));
    int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < R; ++t) {
            int32_t j = adj_out[i * R + t];
            if (j >= 0)
                offers[offer_cnt[j] + fill[j]++] = (int32_t)i;
        }
    int32_t *fwd = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * R);
    memcpy(fwd, adj_out, sizeof(int32_t) * (size_t)n * R);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t j = 0; j < n; ++j) {
        int64_t no = offer_cnt[j + 1] - offer_cnt[j];
        int cap = R + (int)no;
        double *ck = (double *)malloc(sizeof(double) * (size_t)cap);
        int64_t *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        int cnt = 0;
        for (int t = 0; t < cap; ++t) {
            int64_t v = (t < R) ? fwd[j * R + t] : offers[offer_cnt[j] + (t - R)];
            if (v < 0)
                continue;
            int dup = 0;
            for (int s = 0; s < cnt; ++s)
                if (ci[s] == v) {
                    dup = 1;
                    break;
                }
            if (dup)
                continue;
            double key = obj_key(x, attrs, d, m, j, v);
            int pos = cnt;
            while (pos > 0 && lt(key, v, ck[pos - 1], ci[pos - 1])) {
                ck[pos] = ck[pos - 1];
                ci[pos] = ci[pos - 1];
                pos -= 1;
            }
            ck[pos] = key;
            ci[pos] = v;
            cnt += 1;
        }
        int32_t *row = adj_out + j * (int64_t)R;
        int ns = landing_zone_select(x, attrs, d, m, j, ck, ci, cnt, R, row);
        for (int t = ns; t < R; ++t)
            row[t] = -1;
        free(ck);
        free(ci);
    }
    free(fwd);
    free(offers);
    free(fill);
    free(offer_cnt);
}

/* ------------------------------------------- NN-descent (Sec. 4.3, NPG_kgraph) */
/* splitmix64 (Steele, Lea and Flood, 2014): one step of the generator */
static uint64_t sm64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    double key;
    int64_t id;
    int isnew;
} nnd_entry;

static int nnd_cmp(const void *pa, const void *pb)
{
    const nnd_entry *a = (const nnd_entry *)pa, *b = (const nnd_entry *)pb;
    if (lt(a->key, a->id, b->key, b->id))
        return -1;
    if (lt(b->key, b->id, a->key, a->id))
        return 1;
    return 0;
}

/* Candidate lists C(i) of l entries refined through neighbours of
 * neighbours, in synchronous rounds (round t reads only the lists of round
 * t - 1):
 *   round 0: C(i) = the first l distinct values v != i of (splitmix64 with
 *            state seed ^ (i * 0xD1B54A32D192ED03)) mod n, ordered by
 *            (key, id); every entry is new;
 *   round t: J = the first s new entries of C(i) in list order.  The
 *            candidates are the ids of C(j), j in J, that are neither i nor
 *            in C(i), each taken once.  C(i) becomes the l best of C(i) and
 *            the candidates by (key, id); candidates enter as new, the
 *            entries of J become old, the other entries keep their state.
 * Keys are the object-object fusion keys (all m attributes) in key_mode.
 * Needs n > l.  out_ids [n][l] holds the lists after `rounds` rounds;
 * updates[t - 1] = sum over i of |C_t(i) \ C_(t-1)(i)|. */
void or_nndescent(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int l, int s,
                  int rounds, uint64_t seed, int key_mode, int32_t *out_ids, int64_t *updates,
                  int nthreads)
{
    nnd_entry *cur = (nnd_entry *)malloc(sizeof(nnd_entry) * (size_t)n * l);
    nnd_entry *nxt = (nnd_entry *)malloc(sizeof(nnd_entry) * (size_t)n * l);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        nnd_entry *row = cur + i * l;
        uint64_t st = seed ^ ((uint64_t)i * 0xD1B54A32D192ED03ull);
        int got = 0;
        while (got < l) {
            int64_t v = (int64_t)(sm64_next(&st) % (uint64_t)n);
            int dup = v == i;
            for (int t = 0; t < got && !dup; ++t)
                dup = row[t].id == v;
            if (dup)
                continue;
            double d2 = or_delta2(x + i * (int64_t)d, x + v * (int64_t)d, d);
            int c = or_chi(attrs + i * (int64_t)m, attrs + v * (int64_t)m, m);
            row[got].key = or_order_key(d2, c, m, key_mode);
            row[got].id = v;
            row[got].isnew = 1;
            got += 1;
        }
        qsort(row, (size_t)l, sizeof(nnd_entry), nnd_cmp);
    }
    for (int r = 1; r <= rounds; ++r) {
        int64_t upd = 0;
#ifdef _OPENMP
#pragma omp parallel reduction(+ : upd) num_threads(nthreads)
#endif
        {
            int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
            for (int64_t v = 0; v < n; ++v)
                stamp[v] = -1;
            nnd_entry *pool = (nnd_entry *)malloc(sizeof(nnd_entry) * (size_t)(l + (int64_t)s * l));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
            for (int64_t i = 0; i < n; ++i) {
                const nnd_entry *row = cur + i * l;
                int np = 0;
                int64_t J[64];
                int nj = 0;
                stamp[i] = i;
                for (int t = 0; t < l; ++t) {
                    pool[np] = row[t];
                    stamp[row[t].id] = i;
                    if (row[t].isnew && nj < s) {
                        J[nj++] = row[t].id;
                        pool[np].isnew = 0;
                    }
                    np += 1;
                }
                for (int e = 0; e < nj; ++e) {
                    const nnd_entry *rj = cur + J[e] * l;
                    for (int t = 0; t < l; ++t) {
                        int64_t v = rj[t].id;
                        if (stamp[v] == i)
                            continue;
                        stamp[v] = i;
                        double d2 = or_delta2(x + i * (int64_t)d, x + v * (int64_t)d, d);
                        int c = or_chi(attrs + i * (int64_t)m, attrs + v * (int64_t)m, m);
                        pool[np].key = or_order_key(d2, c, m, key_mode);
                        pool[np].id = v;
                        pool[np].isnew = 2; /* a candidate of this round */
                        np += 1;
                    }
                }
                qsort(pool, (size_t)np, sizeof(nnd_entry), nnd_cmp);
                nnd_entry *out = nxt + i * l;
                for (int t = 0; t < l; ++t) {
                    out[t] = pool[t];
                    if (pool[t].isnew == 2) {
                        out[t].isnew = 1;
                        upd += 1;
                    }
                }
            }
            free(pool);
            free(stamp);
        }
        if (updates)
            updates[r - 1] = upd;
        nnd_entry *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    for (int64_t i = 0; i < n * l; ++i)
        out_ids[i] = (int32_t)cur[i].id;
    free(cur);
    free(nxt);
}

/* Edge selection (Sec. 4.1 (2)-(3)) over given candidate lists [n][l]
 * (-1 padded), re-ordered by the exact FP64 key; forward pass only. */
void or_select_lists(const float *x, const uint8_t *attrs, int64_t n, int d, int m,
                     const int32_t *lists, int l, int R, int32_t *adj_out, int nthreads)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        nnd_entry *e = (nnd_entry *)malloc(sizeof(nnd_entry) * (size_t)l);
        double *ck = (double *)malloc(sizeof(double) * (size_t)l);
        int64_t *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
        int nc = 0;
        for (int t = 0; t < l; ++t) {
            int64_t v = lists[i * l + t];
            if (v < 0 || v == i)
                continue;
            e[nc].key = obj_key(x, attrs, d, m, i, v);
            e[nc].id = v;
            e[nc].isnew = 0;
            nc += 1;
        }
        qsort(e, (size_t)nc, sizeof(nnd_entry), nnd_cmp);
        for (int t = 0; t < nc; ++t) {
            ck[t] = e[t].key;
            ci[t] = e[t].id;
        }
        int32_t *row = adj_out + i * (int64_t)R;
        int ns = landing_zone_select(x, attrs, d, m, i, ck, ci, nc, R, row);
        for (int t = ns; t < R; ++t)
            row[t] = -1;
        free(e);
        free(ck);
        free(ci);
    }
}

/* -------------------------------------- NPG_nsw, batched insertion (Sec. 4.3) */
void or_search(const int32_t *adj, int R, const float *xs, const float *xr,
               const uint8_t *attrs, int64_t n, int d, int m, const float *q,
               const uint8_t *qa, int64_t nq, int k, int L, const int32_t *seeds,
               int nseeds, int ninit, int key_mode, int out_mode, int rerank_n, int64_t max_hops,
               int32_t *out_ids, double *out_gamma, int64_t *out_ndc, int64_t *out_hops,
               int32_t *out_flag, int check_every, double *tr_feat, uint32_t *tr_hop,
               uint32_t *tr_hash, int32_t *tr_count, uint32_t *tr_final, int tr_cap,
               const double *mlp, double stop_logit, double cap_factor, int learned_mode, int expand,
               int route_h, int nthreads);

/* One vertex j re-selects N(j) from N(j) united with the offered ids (each
 * once), ordered by (exact key to j, id) (Sec. 4.1 (2)-(3)). */
static void reselect_row(const float *x, const uint8_t *attrs, int d, int m, int64_t j, int R,
                         const int64_t *offers, int noff, int32_t *adj)
{
    int cap = R + noff;
    nnd_entry *e = (nnd_entry *)malloc(sizeof(nnd_entry) * (size_t)cap);
    double *ck = (double *)malloc(sizeof(double) * (size_t)cap);
    int64_t *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int nc = 0;
    for (int t = 0; t < cap; ++t) {
        int64_t v = t < R ? adj[j * R + t] : offers[t - R];
        if (v < 0 || v == j)
            continue;
        int dup = 0;
        for (int u = 0; u < nc && !dup; ++u)
            dup = e[u].id == v;
        if (dup)
            continue;
        e[nc].key = obj_key(x, attrs, d, m, j, v);
        e[nc].id = v;
        e[nc].isnew = 0;
        nc += 1;
    }
    qsort(e, (size_t)nc, sizeof(nnd_entry), nnd_cmp);
    for (int t = 0; t < nc; ++t) {
        ck[t] = e[t].key;
        ci[t] = e[t].id;
    }
    int32_t *row = adj + j * (int64_t)R;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int ns = landing_zone_select(x, attrs, d, m, j, ck, ci, nc, R, tmp);
    for (int t = 0; t < R; ++t)
        row[t] = t < ns ? tmp[t] : -1;
    free(tmp);
    free(e);
    free(ck);
    free(ci);
}

/* Every vertex j named in a row of [s, s + nb) is offered that row's vertex
 * and re-selects N(j) (the reverse links of insertion). */
static void nsw_reverse(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int R,
                        int64_t s, int64_t nb, int32_t *adj)
{
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = s; e < s + nb; ++e)
        for (int t = 0; t < R; ++t)
            if (adj[e * R + t] >= 0)
                cnt[adj[e * R + t] + 1] += 1;
    for (int64_t v = 0; v < n; ++v)
        cnt[v + 1] += cnt[v];
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(off, cnt, sizeof(int64_t) * (size_t)(n + 1));
    int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt[n] + 1));
    for (int64_t e = s; e < s + nb; ++e)
        for (int t = 0; t < R; ++t) {
            int32_t j = adj[e * R + t];
            if (j >= 0)
                inc[cnt[j]++] = e;
        }
    for (int64_t j = 0; j < n; ++j)
        if (off[j + 1] > off[j])
            reselect_row(x, attrs, d, m, j, R, inc + off[j], (int)(off[j + 1] - off[j]), adj);
    free(cnt);
    free(off);
    free(inc);
}

/* NPG_nsw in batches of B: vertices enter in id order.  The first batch
 * takes the exact l nearest within itself as candidates; every later batch
 * [s, s + nb) searches the graph of the s vertices already in (Alg. 2 in
 * beam form, beam L, the object's attributes all constrained, float32 keys,
 * raw pool order, the first min(s, 256) distinct values of splitmix64(seed)
 * mod s as the entry sample and its 16 best as seeds) for its l candidates.
 * Each new row is selected from its candidates (Sec. 4.1), then every vertex
 * it names re-selects its own row with the new vertex offered.  B = 1 is
 * one-at-a-time insertion. */
void or_nsw_insert(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int l, int R,
                   int64_t s0, int64_t B, int L, uint64_t seed, int32_t *adj, int nthreads);

void or_build_nsw(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int l, int R,
                  int64_t B, int L, uint64_t seed, int32_t *adj, int nthreads)
{
    for (int64_t t = 0; t < n * R; ++t)
        adj[t] = -1;
    int64_t b0 = B < n ? B : n;
    int l0 = (int)(l < b0 - 1 ? l : b0 - 1);
    if (l0 > 0) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
        for (int64_t i = 0; i < b0; ++i) {
            double *ck = (double *)malloc(sizeof(double) * (size_t)l0);
            int64_t *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)l0);
            int nc = nearest_l(x, attrs, b0, d, m, 1, i, l0, ck, ci);
            int32_t *row = adj + i * (int64_t)R;
            int ns = landing_zone_select(x, attrs, d, m, i, ck, ci, nc, R, row);
            for (int t = ns; t < R; ++t)
                row[t] = -1;
            free(ck);
            free(ci);
        }
        nsw_reverse(x, attrs, n, d, m, R, 0, b0, adj);
    }
    or_nsw_insert(x, attrs, n, d, m, l, R, b0, B, L, seed, adj, nthreads);
}

/* Vertices s0 .. n - 1 (their rows -1) enter the graph of the vertices
 * below s0 in batches of B, as the later batches of or_build_nsw do. */
void or_nsw_insert(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int l, int R,
                   int64_t s0, int64_t B, int L, uint64_t seed, int32_t *adj, int nthreads)
{
    if (s0 < 1)
        return;
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(B * l + 1));
    double *gam = (double *)malloc(sizeof(double) * (size_t)(B * l + 1));
    int64_t *ndc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(B + 1));
    int64_t *hops = (int64_t *)malloc(sizeof(int64_t) * (size_t)(B + 1));
    int32_t *flag = (int32_t *)malloc(sizeof(int32_t) * (size_t)(B + 1));
    int32_t seeds[256];
    for (int64_t s = s0; s < n; s += B) {
        int64_t nb = (n - s) < B ? (n - s) : B;
        int ns = 0;
        uint64_t st = seed;
        int want = s < 256 ? (int)s : 256;
        while (ns < want) {
            int32_t v = (int32_t)(sm64_next(&st) % (uint64_t)s);
            int dup = 0;
            for (int t = 0; t < ns && !dup; ++t)
                dup = seeds[t] == v;
            if (!dup)
                seeds[ns++] = v;
        }
        or_search(adj, R, x, NULL, attrs, n, d, m, x + s * (int64_t)d, attrs + s * (int64_t)m, nb, l,
                  L, seeds, ns, ns < 16 ? ns : 16, OR_KEY32, 1, 0, INT64_MAX, cand, gam, ndc, hops,
                  flag, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL, 0.0, 0.0, 1, 1, 0, nthreads);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
        for (int64_t e = 0; e < nb; ++e) {
            int64_t offers[256];
            int no = 0;
            for (int t = 0; t < l && no < 256; ++t)
                if (cand[e * l + t] >= 0)
                    offers[no++] = cand[e * l + t];
            reselect_row(x, attrs, d, m, s + e, R, offers, no, adj);
        }
        nsw_reverse(x, attrs, n, d, m, R, s, nb, adj);
    }
    free(cand);
    free(gam);
    free(ndc);
    free(hops);
    free(flag);
}

/* exact k nearest of listed rows (graph quality, Eq. 7): use_attrs selects
 * the fusion key (composite index) or plain delta (vector-only graph). */
void or_knn_rows(const float *x, const uint8_t *attrs, int64_t n, int d, int m, int use_attrs,
                 const int64_t *rows, int64_t nrows, int k, int32_t *out, int nthreads)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
    for (int64_t r = 0; r < nrows; ++r) {
        double *ck = (double *)malloc(sizeof(double) * (size_t)k);
        int64_t *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        int nc = nearest_l(x, attrs, n, d, m, use_attrs, rows[r], k, ck, ci);
        for (int t = 0; t < k; ++t)
            out[r * k + t] = (t < nc) ? (int32_t)ci[t] : -1;
        free(ck);
        free(ci);
    }
}

/* ------------------------------------------------ Alg. 2, beam form */
typedef struct {
    double key;
    double d2;
    int64_t id;
    int chi;
    int expanded;
    int64_t born; /* expansion step during which the entry entered the pool */
} pentry;

/* ---------------------------------------------------------- stop network */
/* Checkpoint state features and the stop network.  The paper cites learned
 * routing only as prior art (Sec. 4.2); these definitions are the library's
 * and are restated here from its interface documentation:
 *   every S expansions (before the next one) the state is summarised by
 *   f1 = ln(1 + H) / 8, f2 = ln(1 + NDC) / 8,
 *   f3 = (sum over constrained attributes of ln(count(code) / n)) / 8
 *        (count 0 read as 0.5),
 *   f4 = eligible entries among the first k pool positions / k,
 *   f5 = ln(key of k-th eligible / that key at its first checkpoint), 1 if
 *        fewer than k eligible,
 *   f6 = ln(key of the next entry to expand / key of k-th eligible), -1 if
 *        fewer than k eligible,
 *   f7 = entries that joined the pool since the last checkpoint / (S R),
 *        an entry joining in a step when it is still pooled at the end of
 *        that step (all of the step's neighbours offered),
 *   f8 = min((H - last H at which the eligible top-k changed) / 64, 1);
 *   the top-k fingerprint is the sum mod 2^32 of fmix32(id + 0x9E3779B9)
 *   (MurmurHash3's finaliser) over the first k eligible ids. */
static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* 8 -> 64 -> 64 -> 2 with ReLU; w in the order W1 [64][8], b1, W2 [64][64],
 * b2, W3 [2][64], b3 */
static void mlp_forward(const double *w, const double *f, double *z)
{
    const double *W1 = w, *b1 = w + 512, *W2 = w + 576, *b2 = w + 4672, *W3 = w + 4736, *b3 = w + 4864;
    double h1[64], h2[64];
    for (int j = 0; j < 64; ++j) {
        double a = b1[j];
        for (int i = 0; i < 8; ++i)
            a += W1[j * 8 + i] * f[i];
        h1[j] = a > 0 ? a : 0;
    }
    for (int j = 0; j < 64; ++j) {
        double a = b2[j];
        for (int i = 0; i < 64; ++i)
            a += W2[j * 64 + i] * h1[i];
        h2[j] = a > 0 ? a : 0;
    }
    for (int o = 0; o < 2; ++o) {
        double a = b3[o];
        for (int j = 0; j < 64; ++j)
            a += W3[o * 64 + j] * h2[j];
        z[o] = a;
    }
}

/* One pass of joint pruning per query.
 *   xs       vectors the loop scores with (the stored form: float32, or the
 *            decoded bf16 / fp8 values);
 *   xr       float32 vectors for the final re-score (nullable);
 *   seeds    the entry sample (nseeds ids); the initial pool (the seed set
 *            B of Alg. 2) is its ninit best members by (key, id);
 *   key_mode OR_KEY64 or OR_KEY32 (ordering precision, see the header);
 *   out_mode 0: exact attribute matches only (Def. 4), in pool order;
 *            1: the first k pool entries, unfiltered;
 *   rerank_n >0 with xr: re-score the first rerank_n output candidates from
 *            xr in FP64, re-sort by (key, id), then cut to k;
 *   max_hops expansion cap (flag set when reached);
 *   mlp      (nullable) the stop network: at every checkpoint (each
 *            check_every hops) it stops the search when its stop logit
 *            reaches stop_logit; with cap_factor > 0 the beam output of the
 *            first checkpoint sets a hop budget cap_factor * 2^z1, checked
 *            before every step; learned_mode 2 takes the first checkpoint
 *            only (its budget then bounds the search); learned_mode 3 is the
 *            beam-width predictor: the first checkpoint's beam output sets
 *            the pool size ceil(cap_factor * 2^z1), clamped to [k, L], for
 *            the rest of the search (no stop logit, no budget);
 *   route_h  >= 2: two-stage routing (Sec. 4.2): stage S1 expands with a
 *            random 1-in-route_h subset of each vertex's slots until a step
 *            adds nothing to the pool, then S2 re-expands the whole pool with
 *            all slots (Alg. 2); 0 or 1 is Alg. 2 throughout.
 * Outputs ids (-1 padded), Gamma (+inf padded), NDC (neighbour distance
 * evaluations; the entry sample is not counted) and H (expansions). */
void or_search(const int32_t *adj, int R, const float *xs, const float *xr,
               const uint8_t *attrs, int64_t n, int d, int m, const float *q,
               const uint8_t *qa, int64_t nq, int k, int L, const int32_t *seeds,
               int nseeds, int ninit, int key_mode, int out_mode, int rerank_n, int64_t max_hops,
               int32_t *out_ids, double *out_gamma, int64_t *out_ndc, int64_t *out_hops,
               int32_t *out_flag, int check_every, double *tr_feat, uint32_t *tr_hop,
               uint32_t *tr_hash, int32_t *tr_count, uint32_t *tr_final, int tr_cap,
               const double *mlp, double stop_logit, double cap_factor, int learned_mode, int expand,
               int route_h, int nthreads)
{
    if (expand < 1)
        expand = 1;
    if (expand > 64)
        expand = 64;
    /* ln(count / n) of every attribute code (count 0 read as 0.5) */
    double logp[OR_MAXM][256];
    for (int i = 0; i < OR_MAXM; ++i)
        for (int c = 0; c < 256; ++c)
            logp[i][c] = 0.0;
    if (check_every > 0) {
        int64_t cnt[OR_MAXM][256];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t e = 0; e < n; ++e)
            for (int i = 0; i < m && i < OR_MAXM; ++i)
                cnt[i][attrs[e * (int64_t)m + i]] += 1;
        for (int i = 0; i < OR_MAXM; ++i)
            for (int c = 0; c < 256; ++c)
                logp[i][c] = log((cnt[i][c] > 0 ? (double)cnt[i][c] : 0.5) / (double)n);
    }
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
    {
        int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v)
            stamp[v] = -1;
        pentry *pool = (pentry *)malloc(sizeof(pentry) * (size_t)(L + 1));
        int ocap = (rerank_n > k ? rerank_n : k) + 1;
        pentry *outl = (pentry *)malloc(sizeof(pentry) * (size_t)ocap);
        pentry *best = (pentry *)malloc(sizeof(pentry) * (size_t)(ninit > 0 ? ninit : 1));
        int64_t *fresh = (int64_t *)malloc(sizeof(int64_t) * (size_t)expand * (size_t)R + 1);
        int *selpos = (int *)malloc(sizeof(int) * (size_t)expand);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t iq = 0; iq < nq; ++iq) {
            const float *qv = q + iq * (int64_t)d;
            const uint8_t *qav = qa + iq * (int64_t)m;
            int mq = or_arity(qav, m);
            int size = 0;
            int Lq = L; /* pool capacity; learned mode 3 lowers it */
            int64_t ndc = 0, hops = 0, step_stamp = 0;
            int flag = 0;

            /* score v and offer it to the pool (insertion keeps (key, id) order) */
#define OFFER(vv)                                                                        \
    do {                                                                                 \
        int64_t v_ = (vv);                                                               \
        double d2_ = or_delta2(qv, xs + v_ * (int64_t)d, d);                            \
        int c_ = or_chi(qav, attrs + v_ * (int64_t)m, m);                               \
        double k_ = or_order_key(d2_, c_, mq, key_mode);                                \
        ndc += 1;                                                                        \
        if (size == Lq && !lt(k_, v_, pool[Lq - 1].key, pool[Lq - 1].id))               \
            break;                                                                       \
        int pos_ = (size < Lq) ? size : Lq - 1;                                          \
        while (pos_ > 0 && lt(k_, v_, pool[pos_ - 1].key, pool[pos_ - 1].id)) {         \
            pool[pos_] = pool[pos_ - 1];                                                 \
            pos_ -= 1;                                                                   \
        }                                                                                \
        pool[pos_].key = k_;                                                             \
        pool[pos_].d2 = d2_;                                                             \
        pool[pos_].id = v_;                                                              \
        pool[pos_].chi = c_;                                                             \
        pool[pos_].expanded = 0;                                                         \
        pool[pos_].born = step_stamp;                                                    \
        if (size < Lq)                                                                   \
            size += 1;                                                                   \
    } while (0)

            /* Alg. 2 initialisation: C <- B, R <- B.  B is the n_init best
             * (by key, id) of the entry sample; they enter the pool and the
             * visited set.  Their scoring is not counted in NDC. */
            {
                int nb = 0;
                for (int s = 0; s < nseeds; ++s) {
                    int64_t v = seeds[s];
                    if (v < 0 || v >= n)
                        continue;
                    double d2 = or_delta2(qv, xs + v * (int64_t)d, d);
                    int c = or_chi(qav, attrs + v * (int64_t)m, m);
                    double key = or_order_key(d2, c, mq, key_mode);
                    int dup = 0;
                    for (int t = 0; t < nb; ++t)
                        if (best[t].id == v)
                            dup = 1;
                    if (dup)
                        continue;
                    if (nb == ninit && !lt(key, v, best[ninit - 1].key, best[ninit - 1].id))
                        continue;
                    int pos = (nb < ninit) ? nb : ninit - 1;
                    while (pos > 0 && lt(key, v, best[pos - 1].key, best[pos - 1].id)) {
                        best[pos] = best[pos - 1];
                        pos -= 1;
                    }
                    best[pos].key = key;
                    best[pos].d2 = d2;
                    best[pos].id = v;
                    best[pos].chi = c;
                    best[pos].expanded = 0;
                    best[pos].born = 0;
                    if (nb < ninit)
                        nb += 1;
                }
                for (int t = 0; t < nb && t < L; ++t) {
                    pool[t] = best[t];
                    stamp[best[t].id] = iq;
                }
                size = nb < L ? nb : L;
            }
            /* expansion loop: take the best unexpanded vertex, score its
             * unvisited neighbours, keep the L best (joint pruning) */
            int have_first = 0, have_prev = 0, ntrace = 0;
            double kth_first = 0.0, budget = 1e300;
            uint32_t prev_hash = 0;
            int64_t last_change = 0, ins_window = 0;
            double logsel = 0.0;
            for (int i = 0; i < m && i < OR_MAXM; ++i)
                if (qav[i] != OR_WILDCARD)
                    logsel += logp[i][qav[i]];
            int64_t next_ckpt = check_every;
            int first_ckpt = 1;
            int stage1 = route_h > 1; /* two-stage routing, Sec. 4.2 */
            for (;;) {
                /* the E best unexpanded entries (E = expand), in pool order */
                int nsel = 0;
                for (int t = 0; t < size && nsel < expand; ++t)
                    if (!pool[t].expanded)
                        selpos[nsel++] = t;
                if (nsel == 0)
                    break;
                int cur = selpos[0];
                if (check_every > 0 && hops >= next_ckpt) {
                    while (next_ckpt <= hops)
                        next_ckpt += check_every;
                    int nel = 0, fk = 0, has_kth = 0;
                    double kth = 0.0;
                    uint32_t h = 0;
                    for (int t = 0; t < size && nel < k; ++t) {
                        int el = out_mode == 1 || pool[t].chi == 0;
                        if (!el)
                            continue;
                        if (t < k)
                            fk += 1;
                        h += fmix32((uint32_t)pool[t].id + 0x9E3779B9u);
                        nel += 1;
                        if (nel == k) {
                            has_kth = 1;
                            kth = pool[t].key;
                        }
                    }
                    if (have_prev && h != prev_hash)
                        last_change = hops;
                    prev_hash = h;
                    have_prev = 1;
                    if (has_kth && !have_first) {
                        kth_first = kth;
                        have_first = 1;
                    }
                    int64_t joined = ins_window;
                    ins_window = 0;
                    double f[8], lo_ = 1e-30;
                    f[0] = log(1.0 + (double)hops) / 8.0;
                    f[1] = log(1.0 + (double)ndc) / 8.0;
                    f[2] = logsel / 8.0;
                    f[3] = (double)fk / (double)k;
                    f[4] = has_kth ? log((kth > lo_ ? kth : lo_) / (kth_first > lo_ ? kth_first : lo_)) : 1.0;
                    f[5] = has_kth ? log((pool[cur].key > lo_ ? pool[cur].key : lo_) / (kth > lo_ ? kth : lo_)) : -1.0;
                    f[6] = (double)joined / (double)(check_every * R);
                    f[7] = (double)(hops - last_change) / 64.0;
                    if (f[7] > 1.0)
                        f[7] = 1.0;
                    if (tr_feat && ntrace < tr_cap) {
                        int64_t tt = iq * (int64_t)tr_cap + ntrace;
                        for (int i = 0; i < 8; ++i)
                            tr_feat[tt * 8 + i] = f[i];
                        tr_hop[tt] = (uint32_t)hops;
                        tr_hash[tt] = h;
                        ntrace += 1;
                    }
                    if (mlp && learned_mode == 3) {
                        /* the beam-width predictor: the first checkpoint's
                         * beam output sets the pool size for the rest of the
                         * search, ceil(cap_factor * 2^z1) clamped to [k, L];
                         * the pool keeps its best entries and the step's
                         * selection is made again from what is left */
                        double z[2];
                        mlp_forward(mlp, f, z);
                        next_ckpt = INT64_MAX;
                        if (first_ckpt) {
                            first_ckpt = 0;
                            double want = ceil(cap_factor * pow(2.0, z[1]));
                            int lp = !(want < (double)Lq) ? Lq : (want < (double)k ? k : (int)want);
                            if (lp < Lq) {
                                Lq = lp;
                                if (size > Lq)
                                    size = Lq;
                                continue;
                            }
                        }
                    } else if (mlp) {
                        double z[2];
                        mlp_forward(mlp, f, z);
                        if (cap_factor > 0 && first_ckpt)
                            budget = cap_factor * pow(2.0, z[1]);
                        first_ckpt = 0;
                        if (z[0] >= stop_logit)
                            break;
                        if (learned_mode == 2) /* one checkpoint: its budget bounds the rest */
                            next_ckpt = INT64_MAX;
                    }
                    first_ckpt = 0;
                }
                if (mlp && (double)hops >= budget)
                    break;
                if (hops >= max_hops) {
                    flag = 1;
                    break;
                }
                if (nsel > max_hops - hops)
                    nsel = (int)(max_hops - hops);
                int64_t us[64];
                for (int e = 0; e < nsel; ++e) {
                    pool[selpos[e]].expanded = 1;
                    us[e] = pool[selpos[e]].id;
                }
                const int64_t hops_before = hops;
                hops += nsel;
                /* unvisited neighbours of the selected vertices, in (vertex,
                 * slot) order; each is scored once.  Stage S1 of two-stage
                 * routing looks at one slot in route_h only: slot t of the
                 * vertex u expanded as the x-th expansion of the search
                 * (x counted from 0) is looked at iff
                 * t + fmix32(u * 0x9E3779B1 + x mod 2^32) is a multiple of
                 * route_h, a random subset of about R / route_h slots. */
                int nf = 0;
                for (int e = 0; e < nsel; ++e)
                    for (int t = 0; t < R; ++t) {
                        if (stage1) {
                            uint32_t x = (uint32_t)(hops_before + e);
                            uint32_t f = fmix32((uint32_t)us[e] * 0x9E3779B1u + x);
                            if (((uint64_t)t + (uint64_t)f) % (uint64_t)route_h != 0)
                                continue;
                        }
                        int64_t v = adj[us[e] * (int64_t)R + t];
                        if (v < 0 || v >= n)
                            continue;
                        if (stamp[v] == iq)
                            continue;
                        stamp[v] = iq;
                        fresh[nf++] = v;
                    }
                /* every fresh neighbour is offered to the pool; the step's
                 * joined count is the number of them still pooled once all
                 * have been offered (an entry admitted and then pushed out
                 * by a better one of the same step does not count) */
                step_stamp += 1;
                for (int c = 0; c < nf; ++c)
                    OFFER(fresh[c]);
                int64_t joined_step = 0;
                for (int t = 0; t < size; ++t)
                    if (pool[t].born == step_stamp)
                        joined_step += 1;
                ins_window += joined_step;
                /* S1 ends at the first step that adds nothing to the pool;
                 * S2 then expands every pool entry again, with all of its
                 * neighbours (greedy routing of Alg. 2 from the S1 pool) */
                if (stage1 && joined_step == 0) {
                    stage1 = 0;
                    for (int t = 0; t < size; ++t)
                        pool[t].expanded = 0;
                }
            }
#undef OFFER
            if (tr_feat) {
                int nel = 0;
                uint32_t h = 0;
                for (int t = 0; t < size && nel < k; ++t)
                    if (out_mode == 1 || pool[t].chi == 0) {
                        h += fmix32((uint32_t)pool[t].id + 0x9E3779B9u);
                        nel += 1;
                    }
                tr_final[iq] = h;
                tr_count[iq] = ntrace;
            }
            /* output: Def. 4 filter (mode 0) or raw pool order (mode 1) */
            int want = (rerank_n > 0 && xr) ? rerank_n : k;
            int no = 0;
            for (int t = 0; t < size && no < want; ++t)
                if (out_mode == 1 || pool[t].chi == 0)
                    outl[no++] = pool[t];
            if (rerank_n > 0 && xr) {
                for (int t = 0; t < no; ++t) {
                    outl[t].d2 = or_delta2(qv, xr + outl[t].id * (int64_t)d, d);
                    outl[t].key = or_order_key(outl[t].d2, outl[t].chi, mq, OR_KEY64);
                }
                for (int t = 1; t < no; ++t) { /* insertion sort by (key, id) */
                    pentry e = outl[t];
                    int p = t;
                    while (p > 0 && lt(e.key, e.id, outl[p - 1].key, outl[p - 1].id)) {
                        outl[p] = outl[p - 1];
                        p -= 1;
                    }
                    outl[p] = e;
                }
            }
            for (int j = 0; j < k; ++j) {
                if (j < no) {
                    out_ids[iq * k + j] = (int32_t)outl[j].id;
                    out_gamma[iq * k + j] = or_gamma(sqrt(outl[j].d2), outl[j].chi, mq);
                } else {
                    out_ids[iq * k + j] = -1;
                    out_gamma[iq * k + j] = INFINITY;
                }
            }
            if (out_ndc)
                out_ndc[iq] = ndc;
            if (out_hops)
                out_hops[iq] = hops;
            if (out_flag)
                out_flag[iq] = flag;
        }
        free(stamp);
        free(pool);
        free(outl);
        free(best);
        free(fresh);
        free(selpos);
    }
}
