/*
 * caps_oracle.c -- plain CPU oracle for CAPS filtered partitioned search.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library
 * shares no source, header, table or helper with it.
 *
 * Written from the paper (Gupta et al., "CAPS: A Practical Partition Index
 * for Filtered Similarity Search", arXiv 2308.15014):
 *   - Definition 1 (query filter) and Definition 2 (filtered NN search),
 *   - Algorithm 1 (index construction: first-level partition f, then the
 *     truncated Attribute Frequency Tree per partition),
 *   - Algorithm 2 (query: top-m partitions, sub-partition choice,
 *     Attribute Match, top-k Vector Match),
 *   - Appendix "Groundtruth" (exact search over the valid points).
 * Where the paper is silent the readings are stated at each function.
 *
 * Arithmetic contract (shared by specification, not by code, with the GPU
 * library): every FP32 dot product and squared distance is a sequential
 * fmaf() chain over dimensions in ascending order; k-means centroid sums are
 * FP64 sequential sums in ascending point id.  Build with
 * -O2 -ffp-contract=off and no fast-math so the compiler keeps that order.
 * OpenMP only splits independent points or queries across threads; it never
 * changes any per-item arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the parallel loops below (over independent points or
 * queries); returns the count in effect.  n <= 0 leaves it unchanged. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Init sampler: splitmix64 (Steele, Lea & Flood, OOPSLA 2014, as in    */
/* Vigna's public-domain splitmix64.c) driving a partial Fisher-Yates.  */
/* ------------------------------------------------------------------ */
static uint64_t orc_splitmix64(uint64_t *state)
{
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ULL;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64_first(uint64_t seed, int32_t count, uint64_t *out)
{
    uint64_t s = seed;
    for (int32_t i = 0; i < count; i++) out[i] = orc_splitmix64(&s);
    return s;
}

/* B distinct ids from 0..n-1: for i = 0..b-1, j = i + (next() mod (n-i)),
 * swap ids[i], ids[j].  The modulo bias is part of the specification. */
int orc_init_ids(uint64_t seed, int64_t n, int32_t b, int32_t *out)
{
    if (b < 0 || (int64_t)b > n) return -1;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!ids) return -2;
    for (int64_t i = 0; i < n; i++) ids[i] = (int32_t)i;
    uint64_t s = seed;
    for (int32_t i = 0; i < b; i++) {
        uint64_t r = orc_splitmix64(&s);
        int64_t j = (int64_t)i + (int64_t)(r % (uint64_t)(n - i));
        int32_t t = ids[i];
        ids[i] = ids[j];
        ids[j] = t;
        out[i] = ids[i];
    }
    free(ids);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Scores.                                                             */
/* ------------------------------------------------------------------ */
static float orc_dot(const float *a, const float *b, int32_t d)
{
    float acc = 0.0f;
    for (int32_t j = 0; j < d; j++) acc = fmaf(a[j], b[j], acc);
    return acc;
}

/* Centroid score used for k-means assignment and for query routing
 * (Algorithm 2 routes on the vector alone).  L2: |c|^2 - 2 q.c, which ranks
 * centroids exactly as |q - c|^2 does up to rounding; IP: -q.c. */
static float orc_cscore(int32_t metric, const float *v, const float *c, float cnorm, int32_t d)
{
    float dt = orc_dot(v, c, d);
    if (metric == 0) return cnorm - 2.0f * dt;
    return -dt;
}

static float orc_canon(float v) { return v == 0.0f ? 0.0f : v; }

void orc_centroid_norms(const float *cent, int32_t b, int32_t d, float *out)
{
    for (int32_t c = 0; c < b; c++) out[c] = orc_dot(cent + (size_t)c * d, cent + (size_t)c * d, d);
}

/* One assignment pass: a_i = argmin_c score(x_i, c), ties to the smaller c. */
void orc_assign(const float *x, int64_t n, int32_t d, const float *cent, int32_t b,
                int32_t metric, int32_t *assign)
{
    float *cn = (float *)malloc(sizeof(float) * (size_t)b);
    orc_centroid_norms(cent, b, d, cn);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const float *xi = x + (size_t)i * d;
        int32_t best = 0;
        float bs = orc_cscore(metric, xi, cent, cn[0], d);
        for (int32_t c = 1; c < b; c++) {
            float s = orc_cscore(metric, xi, cent + (size_t)c * d, cn[c], d);
            if (s < bs) { bs = s; best = c; }
        }
        assign[i] = best;
    }
    free(cn);
}

/* Lloyd update: c = round_f32(sum_{i in c, ascending i} (double)x_i / count).
 * An empty cluster keeps its previous centroid.  metric 1 (inner product)
 * uses the spherical variant: each updated centroid is divided by its FP64
 * norm (sequential sum of squares) and rounded to FP32. */
void orc_update(const float *x, int64_t n, int32_t d, const int32_t *assign, int32_t b,
                int32_t metric, float *cent)
{
    double *sum = (double *)calloc((size_t)b * d, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)b, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        int32_t c = assign[i];
        cnt[c]++;
        for (int32_t j = 0; j < d; j++) sum[(size_t)c * d + j] += (double)x[(size_t)i * d + j];
    }
    for (int32_t c = 0; c < b; c++) {
        if (cnt[c] == 0) continue;
        float *cc = cent + (size_t)c * d;
        for (int32_t j = 0; j < d; j++) cc[j] = (float)(sum[(size_t)c * d + j] / (double)cnt[c]);
        if (metric == 1) {
            double s2 = 0.0;
            for (int32_t j = 0; j < d; j++) s2 += (double)cc[j] * (double)cc[j];
            double nrm = sqrt(s2);
            if (nrm > 0.0)
                for (int32_t j = 0; j < d; j++) cc[j] = (float)((double)cc[j] / nrm);
        }
    }
    free(sum);
    free(cnt);
}

/* Seeded Lloyd k-means: centroids start at the init points, then `iters`
 * rounds of (assign, update), then one final assignment that defines the
 * first-level partition f(x_i). */
int orc_kmeans(const float *x, int64_t n, int32_t d, int32_t b, int32_t iters, int32_t metric,
               const int32_t *init_ids, float *cent, int32_t *assign)
{
    for (int32_t c = 0; c < b; c++)
        memcpy(cent + (size_t)c * d, x + (size_t)init_ids[c] * d, sizeof(float) * (size_t)d);
    for (int32_t it = 0; it < iters; it++) {
        orc_assign(x, n, d, cent, b, metric, assign);
        orc_update(x, n, d, assign, b, metric, cent);
    }
    orc_assign(x, n, d, cent, b, metric, assign);
    return 0;
}

/* Sum over points of the assigned centroid's squared distance (FP64), the
 * Lloyd objective. */
double orc_objective(const float *x, int64_t n, int32_t d, const float *cent, const int32_t *assign)
{
    double tot = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const float *xi = x + (size_t)i * d;
        const float *c = cent + (size_t)assign[i] * d;
        for (int32_t j = 0; j < d; j++) {
            double t = (double)xi[j] - (double)c[j];
            tot += t * t;
        }
    }
    return tot;
}

/* ------------------------------------------------------------------ */
/* Attribute Frequency Tree (Algorithm 1, truncated at height h).       */
/* tok(i) = toks[tok_off[i] .. tok_off[i+1]) (no duplicates).           */
/* Per partition, with R = its points: for j = 0..h-1, t_j = the token  */
/* held by the most points of R (ties to the smaller token), p_j = the   */
/* points of R holding t_j, R <- R \ p_j.  If R holds no token at all,   */
/* t_j = -1 and p_j is empty.  Finally p_h = R (the paper's p_{h+1}).   */
/* Output: tags[p*h + j] = t_j; level[i] = the j of the sub-partition    */
/* holding point i (h for the remainder).                               */
/* ------------------------------------------------------------------ */
int orc_aft(int64_t n, const int32_t *assign, int32_t b, int32_t h,
            const int64_t *tok_off, const int32_t *toks, int32_t n_tok,
            int32_t *tags, int8_t *level)
{
    int64_t *start = (int64_t *)calloc((size_t)b + 1, sizeof(int64_t));
    int64_t *members = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = (int64_t *)calloc((size_t)b, sizeof(int64_t));
    int64_t *count = (int64_t *)calloc((size_t)(n_tok > 0 ? n_tok : 1), sizeof(int64_t));
    if (!start || !members || !fill || !count) return -2;
    for (int64_t i = 0; i < n; i++) start[assign[i] + 1]++;
    for (int32_t p = 0; p < b; p++) start[p + 1] += start[p];
    for (int64_t i = 0; i < n; i++) members[start[assign[i]] + fill[assign[i]]++] = i;

    for (int64_t i = 0; i < n; i++) level[i] = -1;
    for (int32_t p = 0; p < b; p++) {
        for (int32_t j = 0; j < h; j++) {
            memset(count, 0, sizeof(int64_t) * (size_t)(n_tok > 0 ? n_tok : 1));
            for (int64_t u = start[p]; u < start[p + 1]; u++) {
                int64_t i = members[u];
                if (level[i] >= 0) continue;
                for (int64_t e = tok_off[i]; e < tok_off[i + 1]; e++) count[toks[e]]++;
            }
            int32_t best = -1;
            int64_t bc = 0;
            for (int32_t t = 0; t < n_tok; t++)
                if (count[t] > bc) { bc = count[t]; best = t; }
            tags[(size_t)p * h + j] = best;
            if (best < 0) continue;
            for (int64_t u = start[p]; u < start[p + 1]; u++) {
                int64_t i = members[u];
                if (level[i] >= 0) continue;
                for (int64_t e = tok_off[i]; e < tok_off[i + 1]; e++)
                    if (toks[e] == best) { level[i] = (int8_t)j; break; }
            }
        }
        for (int64_t u = start[p]; u < start[p + 1]; u++)
            if (level[members[u]] < 0) level[members[u]] = (int8_t)h;
    }
    free(start);
    free(members);
    free(fill);
    free(count);
    return 0;
}

/* Learned partitions (Section 5.2, CAPS-BLISS): the re-partitioning step of
 * BLISS as published -- every item, in turn (here ascending id), goes to the
 * least loaded of its model's top-K buckets, loads counting the items placed
 * so far; ties go to the better-ranked bucket.  cand: n x k_cand, best
 * first, entries in [0, b).  Returns -1 on a candidate out of range. */
int orc_bliss_assign(const int32_t *cand, int64_t n, int32_t k_cand, int32_t b, int32_t *out)
{
    int64_t *load = (int64_t *)calloc((size_t)b, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        int32_t pick = -1;
        for (int32_t r = 0; r < k_cand; r++) {
            int32_t c = cand[i * k_cand + r];
            if (c < 0 || c >= b) {
                free(load);
                return -1;
            }
            if (pick < 0 || load[c] < load[pick]) pick = c;
        }
        out[i] = pick;
        load[pick]++;
    }
    free(load);
    return 0;
}

/* Dynamic insertion (Table 1 "Dynamic Insertions"; Section 1 and
 * Section 7): the partition model and the tree's tags stay frozen.  A new
 * point joins the partition the k-means assignment picks (orc_assign
 * against the final centroids) and, inside it, the first tagged level whose
 * tag it holds -- the order in which Algorithm 1 split the partition -- or
 * the remainder (level h) when it holds none.  tok(i) as in orc_aft, for the
 * new points only. */
void orc_insert_levels(int64_t n_new, const int32_t *assign, const int32_t *tags, int32_t h,
                       const int64_t *tok_off, const int32_t *toks, int8_t *level)
{
    for (int64_t i = 0; i < n_new; i++) {
        const int32_t *t = tags + (size_t)assign[i] * h;
        int32_t l = h;
        for (int32_t j = 0; j < h && l == h; j++) {
            if (t[j] < 0) continue;
            for (int64_t e = tok_off[i]; e < tok_off[i + 1]; e++)
                if (toks[e] == t[j]) { l = j; break; }
        }
        level[i] = (int8_t)l;
    }
}

/* CSR over sub-partitions (Appendix "Index size"): points grouped by
 * (partition, level); offs[p*(h+1)+j] is the first CSR position of
 * sub-partition j of partition p, offs[B*(h+1)] = n; perm[pos] = point id.
 * The paper leaves the order inside a sub-partition open.  Here it is the
 * order in which `order` lists the points (a permutation of the ids; NULL:
 * ascending id): the caller passes the points sorted by their dense
 * attribute values (attribute 0 first), ties by id, so that points with equal
 * values sit next to each other. */
void orc_csr(int64_t n, const int32_t *assign, const int8_t *level, int32_t b, int32_t h,
             const int32_t *order, int32_t *perm, int32_t *offs)
{
    int64_t nk = (int64_t)b * (h + 1);
    int64_t *pos = (int64_t *)calloc((size_t)nk + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) pos[(int64_t)assign[i] * (h + 1) + level[i] + 1]++;
    for (int64_t s = 0; s < nk; s++) pos[s + 1] += pos[s];
    for (int64_t s = 0; s <= nk; s++) offs[s] = (int32_t)pos[s];
    for (int64_t u = 0; u < n; u++) {
        int64_t i = order ? order[u] : u;
        int64_t key = (int64_t)assign[i] * (h + 1) + level[i];
        perm[pos[key]++] = (int32_t)i;
    }
    free(pos);
}

/* ------------------------------------------------------------------ */
/* Query side.                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    float key;   /* ranking key: L2 distance, or the negated IP score */
    float val;   /* reported value: L2 distance or IP score */
    int32_t id;
} orc_hit;

static int orc_hit_cmp(const void *a, const void *b)
{
    const orc_hit *x = (const orc_hit *)a, *y = (const orc_hit *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    float key;
    int32_t id;
} orc_rank;

static int orc_rank_cmp(const void *a, const void *b)
{
    const orc_rank *x = (const orc_rank *)a, *y = (const orc_rank *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Definition 1 with unconstrained attributes as wildcards: point i is valid
 * iff every query token is among tok(i). */
static int orc_valid(const int32_t *qt, int64_t nqt, const int32_t *pt, int64_t npt)
{
    for (int64_t a = 0; a < nqt; a++) {
        int found = 0;
        for (int64_t e = 0; e < npt; e++)
            if (pt[e] == qt[a]) { found = 1; break; }
        if (!found) return 0;
    }
    return 1;
}

/* Squared L2, or the IP score, as a sequential fmaf chain over j. */
static float orc_dist(int32_t metric, const float *x, const float *q, int32_t d)
{
    float acc = 0.0f;
    if (metric == 0) {
        for (int32_t j = 0; j < d; j++) {
            float t = x[j] - q[j];
            acc = fmaf(t, t, acc);
        }
    } else {
        for (int32_t j = 0; j < d; j++) acc = fmaf(x[j], q[j], acc);
    }
    return orc_canon(acc);
}

static void orc_emit(int32_t metric, orc_hit *hits, int64_t nh, int32_t k, int32_t *ids, float *dist)
{
    qsort(hits, (size_t)nh, sizeof(orc_hit), orc_hit_cmp);
    for (int32_t r = 0; r < k; r++) {
        if (r < nh) {
            ids[r] = hits[r].id;
            dist[r] = hits[r].val;
        } else {
            ids[r] = -1;
            dist[r] = metric == 0 ? INFINITY : -INFINITY;
        }
    }
}

/* Normalised query token set: sorted, duplicates removed.  Returns 0 when
 * the constraints are contradictory (two different values of one dense
 * attribute; tok_attr[t] >= 0 names the dense attribute of token t, -1 marks
 * a label, which may co-occur). */
static int64_t orc_qtokens(const int32_t *in, int64_t nin, const int32_t *tok_attr, int32_t *out, int *ok)
{
    int64_t m = 0;
    for (int64_t a = 0; a < nin; a++) {
        int dup = 0;
        for (int64_t e = 0; e < m; e++)
            if (out[e] == in[a]) { dup = 1; break; }
        if (!dup) out[m++] = in[a];
    }
    *ok = 1;
    for (int64_t a = 0; a < m; a++)
        for (int64_t e = a + 1; e < m; e++)
            if (tok_attr[out[a]] >= 0 && tok_attr[out[a]] == tok_attr[out[e]]) *ok = 0;
    return m;
}

/* A query's constraint list is a disjunction of AND-terms (Section 5.3
 * "Query Algorithm" joins several sub-partitions per partition when the
 * query constrains attributes with OR): token -1 separates terms and a term
 * holding token -2 (a pair outside the vocabularies) is unsatisfiable; a
 * list without separators is one term.  A term's tokens are normalised by
 * orc_qtokens, which also marks contradictory terms.  More than
 * ORC_MAX_TERMS terms: the query is unsatisfiable (returns 0 terms). */
#define ORC_MAX_TERMS 4
typedef struct {
    const int32_t *tok;
    int64_t n;
    int ok;
} orc_term;

static int orc_split_terms(const int32_t *in, int64_t nin, const int32_t *tok_attr, int32_t *buf,
                           orc_term *terms)
{
    int nt = 0;
    int64_t lo = 0, used = 0;
    for (int64_t e = 0; e <= nin; e++) {
        if (e < nin && in[e] != -1) continue;
        if (nt == ORC_MAX_TERMS) return 0;
        int bad = 0;
        for (int64_t f = lo; f < e; f++) bad |= in[f] == -2;
        int ok = 1;
        int64_t m = bad ? 0 : orc_qtokens(in + lo, e - lo, tok_attr, buf + used, &ok);
        terms[nt].tok = buf + used;
        terms[nt].n = m;
        terms[nt].ok = ok && !bad;
        nt++;
        used += m;
        lo = e + 1;
    }
    return nt;
}

/* Valid for a disjunction: some satisfiable term's tokens are all held. */
static int orc_valid_any(const orc_term *terms, int nt, const int32_t *pt, int64_t npt)
{
    for (int t = 0; t < nt; t++)
        if (terms[t].ok && orc_valid(terms[t].tok, terms[t].n, pt, npt)) return 1;
    return 0;
}

static int orc_conflicts(int32_t tag, const int32_t *qt, int64_t nqt, const int32_t *tok_attr)
{
    if (tag < 0 || tok_attr[tag] < 0) return 0;
    for (int64_t a = 0; a < nqt; a++)
        if (tok_attr[qt[a]] == tok_attr[tag] && qt[a] != tag) return 1;
    return 0;
}

static int orc_has(const int32_t *qt, int64_t nqt, int32_t t)
{
    for (int64_t a = 0; a < nqt; a++)
        if (qt[a] == t) return 1;
    return 0;
}

/* Sub-partition choice for one probed partition; returns a bit mask over
 * levels 0..h.
 * rule 0 (exact): with J* = the first tagged level whose tag the query
 *   holds (h if none), scan level j < h iff j <= J*, t_j != -1 and t_j does
 *   not contradict the query; scan level h iff J* = h.  A point of p_j lacks
 *   t_0..t_{j-1}, so every skipped sub-partition holds no valid point.
 * rule 1 (Algorithm 2 read literally): scan only p_{J*} (p_h when J* = h). */
static uint32_t orc_select(int32_t rule, const int32_t *tags, int32_t h, const int32_t *qt, int64_t nqt,
                           const int32_t *tok_attr)
{
    int32_t js = h;
    for (int32_t j = 0; j < h; j++)
        if (tags[j] >= 0 && orc_has(qt, nqt, tags[j])) { js = j; break; }
    if (rule == 1) return 1u << js;
    uint32_t mask = 0;
    for (int32_t j = 0; j < h && j <= js; j++)
        if (tags[j] >= 0 && !orc_conflicts(tags[j], qt, nqt, tok_attr)) mask |= 1u << j;
    if (js == h) mask |= 1u << h;
    return mask;
}

/*
 * CAPS query (Algorithm 2) for a batch.
 *   x, tok_off/toks:    vectors and token sets in original id order
 *   cent (b x d):       first-level centroids; tags (b x h), perm, offs: CSR
 *   qtok_off/qtoks:     constraint tokens per query; q_bad[i] != 0 marks a
 *                       query with an out-of-range attribute or value
 *   m:                  partitions probed; k: results
 * Outputs ids/dist (nq x k), per-query candidate count (points in the chosen
 * sub-partitions) and survivor count (candidates passing the filter), and
 * optionally the probe list (nq x m) and the chosen-level masks (nq x m).
 * A query with contradictory or out-of-range constraints chooses nothing.
 */
int orc_search(const float *x, int64_t n, int32_t d,
               const int64_t *tok_off, const int32_t *toks, const int32_t *tok_attr,
               const float *cent, int32_t b, int32_t metric,
               const int32_t *tags, int32_t h, const int32_t *perm, const int32_t *offs,
               const float *q, int32_t nq, const int64_t *qtok_off, const int32_t *qtoks,
               const uint8_t *q_bad, int32_t k, int32_t m, int32_t rule,
               int32_t *out_ids, float *out_dist, int64_t *n_cand, int64_t *n_surv,
               int32_t *out_probes, uint32_t *out_masks)
{
    (void)n;
    if (m < 1 || m > b || k < 1) return -1;
    float *cn = (float *)malloc(sizeof(float) * (size_t)b);
    orc_centroid_norms(cent, b, d, cn);
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t qi = 0; qi < nq; qi++) {
        const float *qv = q + (size_t)qi * d;
        int64_t nin = qtok_off[qi + 1] - qtok_off[qi];
        int32_t *qt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nin + 1));
        orc_term terms[ORC_MAX_TERMS];
        int nt = orc_split_terms(qtoks + qtok_off[qi], nin, tok_attr, qt, terms);
        if (q_bad && q_bad[qi]) nt = 0;

        orc_rank *rk = (orc_rank *)malloc(sizeof(orc_rank) * (size_t)b);
        for (int32_t c = 0; c < b; c++) {
            rk[c].key = orc_canon(orc_cscore(metric, qv, cent + (size_t)c * d, cn[c], d));
            rk[c].id = c;
        }
        qsort(rk, (size_t)b, sizeof(orc_rank), orc_rank_cmp);

        int64_t cap = 64, nh = 0, cand = 0;
        orc_hit *hits = (orc_hit *)malloc(sizeof(orc_hit) * (size_t)cap);
        for (int32_t r = 0; r < m; r++) {
            int32_t p = rk[r].id;
            if (out_probes) out_probes[(size_t)qi * m + r] = p;
            uint32_t mask = 0u;   /* the union over the satisfiable terms */
            for (int t = 0; t < nt; t++)
                if (terms[t].ok) mask |= orc_select(rule, tags + (size_t)p * h, h, terms[t].tok, terms[t].n, tok_attr);
            if (out_masks) out_masks[(size_t)qi * m + r] = mask;
            for (int32_t j = 0; j <= h; j++) {
                if (!(mask & (1u << j))) continue;
                int32_t lo = offs[(size_t)p * (h + 1) + j], hi = offs[(size_t)p * (h + 1) + j + 1];
                for (int32_t pos = lo; pos < hi; pos++) {
                    int32_t id = perm[pos];
                    cand++;
                    if (!orc_valid_any(terms, nt, toks + tok_off[id], tok_off[id + 1] - tok_off[id])) continue;
                    if (nh == cap) {
                        cap *= 2;
                        hits = (orc_hit *)realloc(hits, sizeof(orc_hit) * (size_t)cap);
                    }
                    float v = orc_dist(metric, x + (size_t)id * d, qv, d);
                    hits[nh].val = v;
                    hits[nh].key = metric == 0 ? v : orc_canon(-v);
                    hits[nh].id = id;
                    nh++;
                }
            }
        }
        orc_emit(metric, hits, nh, k, out_ids + (size_t)qi * k, out_dist + (size_t)qi * k);
        if (n_cand) n_cand[qi] = cand;
        if (n_surv) n_surv[qi] = nh;
        free(hits);
        free(rk);
        free(qt);
    }
    free(cn);
    return rc;
}

/* Ground truth (Appendix "Groundtruth"): exact filtered kNN over all points
 * in FP32 with the same distance arithmetic; n_valid = |D_C|. */
int orc_bruteforce(const float *x, int64_t n, int32_t d,
                   const int64_t *tok_off, const int32_t *toks, const int32_t *tok_attr,
                   int32_t metric, const float *q, int32_t nq,
                   const int64_t *qtok_off, const int32_t *qtoks, const uint8_t *q_bad,
                   int32_t k, int32_t *out_ids, float *out_dist, int64_t *n_valid)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t qi = 0; qi < nq; qi++) {
        const float *qv = q + (size_t)qi * d;
        int64_t nin = qtok_off[qi + 1] - qtok_off[qi];
        int32_t *qt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nin + 1));
        orc_term terms[ORC_MAX_TERMS];
        int nt = orc_split_terms(qtoks + qtok_off[qi], nin, tok_attr, qt, terms);
        if (q_bad && q_bad[qi]) nt = 0;
        int64_t cap = 64, nh = 0;
        orc_hit *hits = (orc_hit *)malloc(sizeof(orc_hit) * (size_t)cap);
        for (int64_t i = 0; nt > 0 && i < n; i++) {
            if (!orc_valid_any(terms, nt, toks + tok_off[i], tok_off[i + 1] - tok_off[i])) continue;
            if (nh == cap) {
                cap *= 2;
                hits = (orc_hit *)realloc(hits, sizeof(orc_hit) * (size_t)cap);
            }
            float v = orc_dist(metric, x + (size_t)i * d, qv, d);
            hits[nh].val = v;
            hits[nh].key = metric == 0 ? v : orc_canon(-v);
            hits[nh].id = (int32_t)i;
            nh++;
        }
        orc_emit(metric, hits, nh, k, out_ids + (size_t)qi * k, out_dist + (size_t)qi * k);
        if (n_valid) n_valid[qi] = nh;
        free(hits);
        free(qt);
    }
    return 0;
}
