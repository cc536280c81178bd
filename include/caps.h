/*
 * caps.h -- C ABI of libcaps, an MI355X (gfx950) implementation of CAPS
 * filtered partitioned search (Gupta et al., "CAPS: A Practical Partition
 * Index for Filtered Similarity Search", arXiv 2308.15014).
 *
 * Problem (Definitions 1 and 2): given points (x_i, a_i) with x_i in R^d and
 * categorical attributes a_i, and a query (q, b), return the k nearest
 * points among D_C = { i : a_i satisfies every constraint of b }.
 * Attributes come in two kinds (Section 2 "Attribute Model", Table 1):
 *   dense:  L_dense attributes with one value each, value < vocab[attr];
 *   labels: a set of up to 128 distinct labels per point, label < label_vocab
 *           (a query constrains at most 8 distinct labels).
 * A query constraint is a pair (attr, val): attr in [0, L_dense) names a
 * dense attribute, attr == L_dense names a label.  Constraints are ANDed;
 * unconstrained attributes match anything.
 *
 * Index (Algorithm 1): first-level partitions f from seeded Lloyd k-means
 * (Section 5.2 "Index creation"), then in every partition a truncated
 * Attribute Frequency Tree of height h giving h+1 disjoint sub-partitions,
 * stored as a CSR (Appendix "Index size").
 * Query (Algorithm 2): score the B centroids, probe the best nprobe
 * partitions, choose the sub-partitions that can hold valid points, filter
 * exactly, scan distances, keep the top k.
 *
 * Conventions
 *   - Status codes only; nothing is thrown across the ABI.  On a non-OK
 *     status outputs are left unspecified and caps_last_error() returns a
 *     thread-local message.
 *   - Buffers are owned by the caller; the index owns its device copies.
 *   - Ranking is a total order: squared L2 ascending, or inner product
 *     descending, then point id ascending.  Fewer than k valid points pad
 *     with id -1 and +inf (L2) / -inf (IP).
 *   - FP32 mode arithmetic: each distance is a sequential fused
 *     multiply-add chain over dimensions in ascending order (L2:
 *     t = x_j - q_j, acc = fma(t, t, acc); IP: acc = fma(x_j, q_j, acc)),
 *     -0 reported as +0.  Results are therefore deterministic and identical
 *     for a query alone or inside any batch.
 */
#ifndef CAPS_H
#define CAPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct caps_index caps_index;

typedef enum {
    CAPS_OK = 0,
    CAPS_EINVAL = -1,        /* an argument is out of range or malformed */
    CAPS_ENOMEM = -2,        /* device or host allocation failed */
    CAPS_EDEVICE = -3,       /* a HIP runtime call failed */
    CAPS_EUNSUPPORTED = -4,  /* valid input outside what this build supports */
    CAPS_EBUSY = -5,         /* server queue full */
    CAPS_EIO = -6            /* file could not be read or written */
} caps_status;

enum { CAPS_METRIC_L2 = 0, CAPS_METRIC_IP = 1 };

/* Low-precision copy of the vectors kept beside the FP32 ones for the
 * MFMA scan of search mode 1.  BF16 and FP16: round-to-nearest-even of each
 * FP32 coordinate.  FP8: OCP E4M3 (finite, max 448) with one FP32 scale per
 * vector, s = max_j |x_j| / 448 (1 for the zero vector), code_j =
 * round-to-nearest-even of x_j / s saturated to +-448; the value is s*code. */
enum { CAPS_PREC_NONE = 0, CAPS_PREC_BF16 = 1, CAPS_PREC_FP8 = 2, CAPS_PREC_FP16 = 3 };

typedef struct {
    int32_t metric;          /* CAPS_METRIC_L2 (squared) or CAPS_METRIC_IP */
    int32_t n_partitions;    /* B, 1 <= B <= min(n, 8192) */
    int32_t kmeans_iters;    /* Lloyd iterations before the final assignment */
    int32_t aft_height;      /* h, 0 <= h <= 15: h tagged levels + remainder */
    uint64_t seed;           /* drives the init sampler (splitmix64 +
                                partial Fisher-Yates over 0..n-1) */
    const int32_t *init_ids; /* optional host array of B initial point ids;
                                overrides seed when not NULL */
    int32_t precision;       /* CAPS_PREC_*: also store a low-precision copy
                                (needed by search mode 1) */
    int32_t reserved;
    const int32_t *assign;   /* optional host array of n first-level partition
                                ids in [0, B) (learned partitions, Section 5.2
                                CAPS-BLISS): used instead of the Lloyd
                                iterations (kmeans_iters ignored); each
                                non-empty partition's centroid is the FP64 mean
                                of its points in ascending id, rounded to FP32
                                (IP: then normalised), an empty one keeps its
                                initial point; NULL: k-means */
} caps_build_params;

/*
 * caps_build -- Algorithm 1.  All pointers are HOST pointers; data is
 * copied to the current device and the index stays resident there.
 *   x          n x d float32, row-major, finite
 *   dense_vals n x n_dense uint32 row-major, dense_vals[i*n_dense+a] <
 *              dense_vocab[a]; NULL when n_dense == 0
 *   dense_vocab n_dense vocabulary sizes (>= 1); packed widths must total
 *              <= 32 bits (ceil(log2(vocab)) bits per attribute)
 *   label_off  n+1 int64 CSR offsets into labels, or NULL (no labels)
 *   labels     label ids < label_vocab <= 65535, at most 128 distinct per
 *              point (a repeated label is an error); sets of more than 8
 *              labels widen every point's slot row to the next power of two
 *   stream     hipStream_t to run on (NULL = default stream); the call
 *              synchronises it before returning
 * k-means: init centroids at the sampled points; each iteration assigns
 * every point to argmin_c (|c|^2 - 2 x.c) [IP: argmin -x.c] with ties to
 * the smaller c, then sets every non-empty centroid to the FP64 mean of its
 * points summed in ascending id, rounded to FP32 (IP: then divided by its
 * FP64 norm); a final assignment defines the partitions.
 * AFT: per partition, h times: tag = the attribute value (dense value or
 * label) held by most remaining points, ties to the smaller token
 * (token = dense offset + value, labels after all dense values); the points
 * holding it form the next sub-partition.
 * Errors: EINVAL (shapes, vocabularies, non-finite x, B > n), EUNSUPPORTED
 * (limits above), ENOMEM, EDEVICE.
 */
caps_status caps_build(const float *x, int64_t n, int32_t d,
                       const uint32_t *dense_vals, int32_t n_dense, const int32_t *dense_vocab,
                       const int64_t *label_off, const uint32_t *labels, int32_t label_vocab,
                       const caps_build_params *params, void *stream, caps_index **out);

/*
 * caps_bliss_assign -- the re-partitioning step of learned partitions
 * (Section 5.2 "Index creation", CAPS-BLISS: partitions learned from
 * filtered near-neighbour labels).  HOST arrays.  cand: n x K candidate
 * partitions per point, best first (the learned router's top-K for the
 * point's own vector, e.g. from caps_search_probes with routing 1); every
 * entry in [0, b).  Points are taken in ascending id; each goes to the
 * least loaded of its K candidates (load = points assigned so far), ties to
 * the earlier candidate; out_assign (n) receives the partitions, ready for
 * caps_build_params.assign.  A host computation (the rule is sequential).
 * Errors: EINVAL (null arrays, n < 0, K < 1, b < 1, a candidate outside
 * [0, b)).
 */
caps_status caps_bliss_assign(const int32_t *cand, int64_t n, int32_t k_cand, int32_t b, int32_t *out_assign);

/*
 * caps_insert -- dynamic insertions (Table 1 "Dynamic Insertions"; Section 1
 * "Practical Utility"): adds n_new points to a built index without
 * rebuilding it.  HOST arrays laid out as for caps_build (x n_new x d;
 * dense_vals n_new x n_dense, NULL without dense attributes; label_off
 * n_new+1 offsets into labels, given exactly when the index has labels).
 * The partition model stays frozen: new point i gets id n + i (n = the
 * index's point count before the call), joins the partition the k-means
 * assignment picks against the final centroids (argmin of |c|^2 - 2 x.c,
 * IP -x.c, ties to the smaller partition) and, inside it, the first tagged
 * level whose tag it holds (the order Algorithm 1 split the partition in),
 * else the remainder.  Centroids, tags and the router do not change; the
 * points already present keep their CSR order, each new point goes to the
 * end of its sub-partition in id order, and every per-point array, the
 * low-precision copy included, grows.  Synchronises `stream`.  Errors:
 * EINVAL (arguments, vocabularies, non-finite x, label sets given to an
 * index without labels or missing), EUNSUPPORTED (limits of caps_build),
 * ENOMEM, EDEVICE; on error the index is unchanged.
 */
caps_status caps_insert(caps_index *idx, const float *x, int64_t n_new, const uint32_t *dense_vals,
                        const int64_t *label_off, const uint32_t *labels, void *stream);

typedef struct {
    int32_t k;        /* 1 <= k <= 64 */
    int32_t nprobe;   /* m, 1 <= m <= B */
    int32_t rule;     /* 0: exact sub-partition choice (skip only
                         sub-partitions whose tags prove them empty of valid
                         points); 1: Algorithm 2 read literally (one
                         sub-partition per partition; lossy, for ablation) */
    int32_t mode;     /* 0: exact: the top k under the FP32 distance of the
                         plain scan (sequential fma over ascending coordinates).
                         On an index with a low-precision copy the copy is
                         scanned with matrix cores to bound each pair's FP32
                         distance from below (with its stored error norms and
                         a rounding margin); pairs whose bound cannot beat the
                         query's current k-th key are skipped and the others
                         are rescored exactly, so the results equal the plain
                         scan's.  1: approximate: the copy is scanned with
                         matrix cores (FP32 accumulation), each query keeps its
                         best `rerank` candidates under the approximate score
                         (L2: |x|^2 - 2 x~.q~ with the FP32 |x|^2; IP: -x~.q~),
                         and those are rescored with the exact FP32 arithmetic
                         to give the final top k.  2: exact with the plain FP32
                         scan only.  The filter is exact in every mode; the
                         distances returned are the exact FP32 distances of the
                         returned ids. */
    int32_t rerank;   /* mode 1: candidates rescored per query, k <= rerank
                         <= 64; 0 means min(4k, 64) */
    int32_t routing;  /* 0: centroid routing (Algorithm 2).  1: the index's
                         learned router (caps_router_train): probes = the m
                         largest logits, ties to the smaller partition, with a
                         per-query fallback to centroid routing when the
                         router's softmax top-1 probability is below its
                         fallback level or its probes hold fewer than k
                         candidates.  EINVAL without a router. */
    int32_t flags;    /* CAPS_SEARCH_* bits below */
    int32_t rescue_grid;  /* workgroups of the exact matrix-core search's
                         rescue pass (the rescan of queries whose candidate
                         pairs overflowed their lists); 0: 8192.  Results do
                         not depend on it. */
    int64_t workspace_bytes;  /* device budget of one call's workspace; the
                         queries are searched in sub-batches that fit it
                         (at least one query each).  0: 4 GiB.  Results do
                         not depend on it. */
} caps_search_params;

/* caps_search_params.flags */
enum {
    /* Synchronise the stream after the search and return CAPS_EINVAL when
     * a query row holds NaN or Inf.  Without it the call stays
     * asynchronous and such a row is answered as a query with an empty
     * D_C (ids -1, distances +inf / -inf). */
    CAPS_SEARCH_VALIDATE = 1,
    /* The constraint lists may be disjunctions (Section 5.3 "Query
     * Algorithm": several sub-partitions per partition are joined when
     * the query constrains attributes with OR): a pair with attr ==
     * CAPS_OR separates the AND-terms of one query, and a point is valid
     * when it satisfies every pair of at least one term.  At most
     * CAPS_MAX_TERMS terms per query.  Without this flag a CAPS_OR pair
     * makes its query unsatisfiable, as any negative attribute does. */
    CAPS_SEARCH_DISJUNCTIVE = 2
};
#define CAPS_OR (-1)
#define CAPS_MAX_TERMS 4

/*
 * caps_search -- Algorithm 2 over a batch.  All pointers are DEVICE
 * pointers on the index's device; work is enqueued on `stream` and the call
 * returns without synchronising.
 *   q           n_q x d float32 row-major
 *   con_off     n_q+1 int32 CSR offsets over constraint pairs
 *   con_attr    constraint attribute: [0, n_dense) dense, n_dense = label
 *   con_val     constraint value
 *   n_con       length of con_attr / con_val; a query whose offsets fall
 *               outside [0, n_con] or decrease is treated as unsatisfiable
 *   out_ids     n_q x k int32     out_dist  n_q x k float32
 *   out_ncand   optional n_q int32: points in the chosen sub-partitions
 *   out_nsurv   optional n_q int32: candidates that pass the filter
 * Not errors (the query is valid with an empty D_C, all ids -1): a value
 * outside its vocabulary, an attribute index outside [0, n_dense], two
 * different values for one dense attribute, more than 8 distinct labels.
 * Duplicate constraints are ignored; zero constraints give plain IVF kNN.
 * A query row holding NaN or Inf is answered with an empty result; with
 * CAPS_SEARCH_VALIDATE in sp->flags the call synchronises `stream` and
 * returns EINVAL instead.
 * Errors: EINVAL (k, nprobe, n_q < 0, NULL pointers, mode 1 on an index
 * without a low-precision copy, rerank outside [k, 64], rescue_grid < 0,
 * unknown flags, non-finite query rows under CAPS_SEARCH_VALIDATE),
 * ENOMEM, EDEVICE.  The device workspace is released on every path: it is
 * taken stream-ordered from a memory pool the library keeps per device, which
 * holds freed memory for later calls (up to the largest workspace in use at
 * once) until the process ends.
 */
caps_status caps_search(const caps_index *idx, const caps_search_params *sp,
                        const float *q, int32_t n_q,
                        const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                        int32_t n_con, int32_t *out_ids, float *out_dist,
                        int32_t *out_ncand, int32_t *out_nsurv, void *stream);

/*
 * caps_search_static -- caps_search (same arguments, results and errors)
 * that allocates nothing, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Its workspace is the library's own static device array of
 * CAPS_STATIC_WORKSPACE_BYTES (64 MiB), held by every GPU the library runs
 * on until the process ends; the batch is searched in sub-batches that fit
 * it (sp->workspace_bytes, if set, must not exceed it: EINVAL).  A single
 * query needing more than the array (very large B x nprobe) gives
 * EUNSUPPORTED.  The index's device must be the current device (else
 * EINVAL).  Every call on one GPU shares that GPU's array and overwrites
 * it: calls that overlap on one GPU (two host threads, or two streams
 * without an ordering between them) race and must not be issued; calls in
 * order on one stream are safe.  Every kernel initialises the workspace
 * memory it reads, so no state carries over from the previous call.
 */
#define CAPS_STATIC_WORKSPACE_BYTES (64ll << 20)
caps_status caps_search_static(const caps_index *idx, const caps_search_params *sp,
                               const float *q, int32_t n_q,
                               const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                               int32_t n_con, int32_t *out_ids, float *out_dist,
                               int32_t *out_ncand, int32_t *out_nsurv, void *stream);

/*
 * caps_search_debug -- caps_search (same arguments and arithmetic) that also
 * writes the filter's pass bits and validates the queries: out_surv_mask
 * (DEVICE, n_q x ceil(n / 64) uint64 words, cleared by the call) gets, for
 * query i, bit pos % 64 of word i * ceil(n / 64) + pos / 64 set exactly when
 * CSR position pos (see caps_index_export: perm[pos] is the point id) lies
 * in a sub-partition the query's search chose (Algorithm 2, sub-partition
 * lookup) and the point there satisfies the query's constraints
 * (Definition 1, "Attribute Match").  Always synchronises `stream`; a query
 * row with NaN or Inf gives EINVAL.  For tests and inspection: the mask is
 * computed by a separate pass over the chosen sub-partitions.
 */
caps_status caps_search_debug(const caps_index *idx, const caps_search_params *sp,
                              const float *q, int32_t n_q,
                              const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                              int32_t n_con, int32_t *out_ids, float *out_dist,
                              int32_t *out_ncand, int32_t *out_nsurv, uint64_t *out_surv_mask, void *stream);

/*
 * caps_search_workspace -- *out_bytes = the device workspace one
 * caps_search call of n_q queries with these parameters allocates (its
 * sub-batch under sp->workspace_bytes included).  Host only; no device work.
 * Errors: EINVAL as caps_search.
 */
caps_status caps_search_workspace(const caps_index *idx, const caps_search_params *sp, int32_t n_q,
                                  int64_t *out_bytes);

/*
 * caps_search_probes -- the routing and sub-partition choice of
 * caps_search alone (device pointers): out_probes n_q x nprobe int32 (best
 * first), out_masks n_q x nprobe uint32 (bit j set = sub-partition j
 * chosen, j = h is the remainder).  Same errors as caps_search.
 */
caps_status caps_search_probes(const caps_index *idx, const caps_search_params *sp,
                               const float *q, int32_t n_q, const int32_t *con_off,
                               const int32_t *con_attr, const int32_t *con_val, int32_t n_con,
                               int32_t *out_probes, uint32_t *out_masks, void *stream);

typedef struct {
    int64_t n;
    int32_t d, n_partitions, aft_height, metric;
    int32_t n_dense, label_vocab, n_tokens;
    int32_t max_subpartition;   /* largest sub-partition size */
    int32_t precision;          /* CAPS_PREC_* of the low-precision copy */
    int32_t lowp_dpad;          /* row width of that copy (0 without one) */
    int32_t label_slots;        /* label slots per point (8, or a power of two up to
                                   128 when a point holds more labels; 0 without labels) */
    int32_t reserved;
    int64_t device_bytes;       /* bytes the index holds on the device */
} caps_index_info_t;

caps_status caps_index_info(const caps_index *idx, caps_index_info_t *out);

/*
 * caps_index_export -- copy index arrays to HOST buffers (any may be NULL):
 * centroids B x d, assign n (partition of point i), level n (sub-partition
 * of point i, h = remainder), perm n (CSR position -> point id; inside a
 * sub-partition the points follow their dense attribute values, attribute 0
 * first, then id),
 * offs B*(h+1)+1 (first CSR position of sub-partition j of partition p at
 * offs[p*(h+1)+j]), tags B x h (token of each tagged level, -1 unused).
 */
caps_status caps_index_export(const caps_index *idx, float *centroids, int32_t *assign,
                              int8_t *level, int32_t *perm, int32_t *offs, int32_t *tags);

/*
 * Stage timing for benchmarks.  While enabled, caps_search records a pair of
 * HIP events around each stage on the stream it runs on; caps_profile_read
 * waits for the recorded events and returns the summed milliseconds and the
 * number of timed launches per stage since caps_profile_enable(1).  Process
 * wide; intended for single-threaded benchmark drivers.
 */
enum {
    CAPS_STAGE_PREP = 0,    /* constraint pairs -> packed filters */
    CAPS_STAGE_ROUTE = 1,   /* query x centroid scores */
    CAPS_STAGE_TOPM = 2,    /* best nprobe partitions */
    CAPS_STAGE_SELECT = 3,  /* sub-partition choice and bucketing */
    CAPS_STAGE_SCAN = 4,    /* filtered distance scan (per-partition top-k) */
    CAPS_STAGE_MERGE = 5,   /* per-query top-k merge */
    CAPS_STAGE_SEED = 6,    /* exact search on the matrix cores: approximate scan of the
                               first probes and the exact seed bound */
    CAPS_STAGE_RESCUE = 7,  /* exact search on the matrix cores: rescan of the queries
                               whose candidate pairs overflowed */
    CAPS_N_STAGES = 8
};
typedef struct {
    double ms[CAPS_N_STAGES];
    int64_t launches[CAPS_N_STAGES];
} caps_profile_t;

caps_status caps_profile_enable(int32_t on);        /* on != 0 clears and starts */
caps_status caps_profile_read(caps_profile_t *out); /* synchronises the events */

/*
 * caps_index_export_lowp -- copy the low-precision copy to HOST buffers (any
 * may be NULL): codes n x dpad (2-byte BF16/FP16 bit patterns or 1-byte FP8
 * codes, CSR order, dpad = lowp_dpad of caps_index_info: the smallest of
 * 32, 64, 128, 256 that is >= d, zero padded),
 * scale n (FP8 per-vector scales, CSR order), xnorm n (exact FP32 |x|^2 of
 * each CSR row, sequential fma).  EINVAL if the index has no such copy.
 */
caps_status caps_index_export_lowp(const caps_index *idx, void *codes, float *scale, float *xnorm);

/*
 * Learned router (a two-layer perceptron on the query and its constraints;
 * the filtered-label training of the paper's CAPS-BLISS variant, Section
 * 5.2, with the k-means partitions kept fixed):
 *   x = [q * in_scale + in_shift || e(C) || 0]  (BF16; width dpad = d + 64
 *       rounded up to 32; e(C) = 64-wide multi-hot: each valid constraint
 *       pair's token -- dense attribute i, value v: off_i + v; label l:
 *       off_L + l -- sets position mix64(token) mod 64, mix64 being
 *       splitmix64's output function)
 *   h = relu(W1 x + b1)  (W1: hidden x dpad, rounded to BF16 after the product)
 *   z = W2 h + b2        (W2: B x hidden; FP32 logits, one per partition)
 * Products use BF16 operands with FP32 accumulation; masters are FP32.
 * Training: Adam on the mean over rows of -(1/|S|) sum_{s in S} log softmax(z)_s,
 * S = a row's distinct labels (partition ids; entries < 0 are padding, a
 * row without labels contributes nothing).  The router lives in the index
 * and is released with it.
 */
typedef struct {
    int32_t hidden;        /* hidden width, a multiple of 16 in [16, 8192] */
    int32_t epochs;        /* passes over the training rows */
    int32_t batch;         /* rows per Adam step, 1..65536 */
    int32_t reset;         /* 1: fresh weights from `seed`; 0: continue the index's router */
    float lr, beta1, beta2, eps;   /* Adam (bias-corrected) */
    float in_scale, in_shift;      /* input map of the query vector */
    float fallback_prob;   /* search falls back to centroid routing below this
                              softmax top-1 probability (0: never; > 1: always) */
    int32_t reserved;
    uint64_t seed;         /* weight init (W ~ U(+-1/sqrt(fan_in)), b = 0) and row shuffling */
} caps_router_params;

typedef struct {
    int32_t present;       /* 0 if the index has no router */
    int32_t din, dpad, hidden, n_out;
    float in_scale, in_shift, fallback_prob;
    int64_t steps;         /* Adam steps taken */
} caps_router_info_t;

/* Labels for training: per query the distinct partitions of its k ids (in
 * order of first appearance, ids < 0 skipped), -1 padded.  ids and
 * out_parts are DEVICE n x k int32 on the index's device; enqueued on
 * `stream`. */
caps_status caps_router_labels(const caps_index *idx, const int32_t *ids, int32_t n, int32_t k,
                               int32_t *out_parts, void *stream);

/* Trains the index's router on n DEVICE rows (q n x d float32, constraint
 * CSR as in caps_search, labels n x n_labels int32).  out_loss: optional
 * HOST array of `epochs` floats, the mean loss of each epoch.  Synchronises
 * `stream` before returning.  Errors: EINVAL (arguments), ENOMEM, EDEVICE. */
caps_status caps_router_train(caps_index *idx, const caps_router_params *p, const float *q, int32_t n,
                              const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                              int32_t n_con, const int32_t *labels, int32_t n_labels, float *out_loss,
                              void *stream);

/* Sets the router from HOST FP32 weights (w1 hidden x dpad, b1 hidden, w2
 * B x hidden, b2 B), or, with all four NULL, from fresh weights drawn from
 * p->seed; Adam state is cleared.  Only hidden, in_scale, in_shift,
 * fallback_prob and seed of p are used.  Synchronous. */
caps_status caps_router_set(caps_index *idx, const caps_router_params *p, const float *w1, const float *b1,
                            const float *w2, const float *b2);

/* Copies the FP32 master weights to HOST arrays (any may be NULL).
 * EINVAL without a router.  Synchronous. */
caps_status caps_router_get(const caps_index *idx, float *w1, float *b1, float *w2, float *b2);

caps_status caps_router_info(const caps_index *idx, caps_router_info_t *out);

/* Router logits (DEVICE n x B float32) of n DEVICE query rows, enqueued on
 * `stream` (the two products on hipBLASLt, FP32 accumulation; scratch for the
 * input and hidden rows from the library's pool).  EINVAL without a router. */
caps_status caps_router_logits(const caps_index *idx, const float *q, int32_t n, const int32_t *con_off,
                               const int32_t *con_attr, const int32_t *con_val, int32_t n_con,
                               float *out_logits, void *stream);

/* Mean loss and parameter gradients of one batch of n DEVICE rows (no
 * update); gradients to HOST arrays laid out like the weights (any may be
 * NULL).  Synchronises `stream`. */
caps_status caps_router_grads(caps_index *idx, const float *q, int32_t n, const int32_t *con_off,
                              const int32_t *con_attr, const int32_t *con_val, int32_t n_con,
                              const int32_t *labels, int32_t n_labels, float *out_loss, float *g_w1,
                              float *g_b1, float *g_w2, float *g_b2, void *stream);

/*
 * Serving loop: continuous batching of filtered queries against one index.
 * Requests (one query vector + its constraint pairs, HOST memory, copied at
 * submit) wait in a bounded queue; a scheduler thread owns `streams` batch
 * slots and, whenever a slot is free, launches the oldest waiting requests
 * (up to the batch cap) as one search on that slot's stream; results carry
 * the latency from submit to completion.  All requests share the search
 * parameters below.  A query's ids and distances do not depend on the batch
 * it lands in.  The index must outlive the server.
 */
typedef struct {
    int32_t k, nprobe, mode, routing, rerank;   /* as caps_search_params */
    int32_t max_batch;        /* queries per launch, 1..65536 */
    int32_t streams;          /* batches in flight, 1..8 */
    int32_t queue_slots;      /* waiting requests admitted; submit returns EBUSY beyond */
    int32_t max_constraints;  /* constraint pairs per request, 0..64 */
    int32_t flags;            /* 0 or CAPS_SEARCH_DISJUNCTIVE (requests may hold
                                 CAPS_OR separators) */
    int64_t workspace_bytes;  /* device memory the search workspaces of all
                                 batches in flight share: a batch is sized to
                                 what the others leave free (and waits when
                                 not one query fits); 0: no budget */
    double batch_window_us;   /* wait up to this long for a batch to fill once a
                                 slot is free (0: launch what is waiting) */
} caps_server_params;

typedef struct {
    int64_t submitted;        /* accepted requests */
    int64_t completed;        /* results produced (failed ones included) */
    int64_t rejected;         /* submits refused with EBUSY */
    int64_t failed;           /* results of batches whose search failed (ids -1) */
    int64_t batches;
    double mean_batch;        /* queries per launched batch */
    double p50_ms, p99_ms, max_ms, mean_ms;   /* submit-to-completion latency */
    double qps;               /* completed / (last completion - first submit) */
    int32_t max_batch;        /* batch cap after the workspace budget */
    int32_t reserved;
} caps_server_stats_t;

typedef struct caps_server caps_server;

/* Starts the scheduler thread.  Errors: EINVAL (parameters; mode 1 without a
 * low-precision copy; routing 1 without a router; a workspace budget below
 * one query), ENOMEM, EDEVICE. */
caps_status caps_server_create(const caps_index *idx, const caps_server_params *p, caps_server **out);

/* Queues one request (q: d floats; n_con pairs).  *ticket identifies its
 * result.  EBUSY when queue_slots requests wait; EINVAL for bad arguments,
 * a NaN or Inf coordinate, or more than max_constraints pairs. */
caps_status caps_server_submit(caps_server *srv, const float *q, int32_t n_con, const int32_t *con_attr,
                               const int32_t *con_val, uint64_t *ticket);

/* Submits n requests (q n x d, constraint CSR con_off n+1) at arrival_s[i]
 * seconds after the call (non-decreasing), from the calling thread, and
 * returns after the last one; tickets[i] = 0 marks a request refused with a
 * full queue.  HOST arrays; con_attr and con_val may be null only when no
 * request has constraints (else EINVAL). */
caps_status caps_server_replay(caps_server *srv, const float *q, const int32_t *con_off, const int32_t *con_attr,
                               const int32_t *con_val, int32_t n, const double *arrival_s, uint64_t *tickets);

/* Moves up to `max` finished results to HOST arrays: tickets, ids (max x k),
 * dist (max x k), optional latency_ms and status (CAPS_OK or the batch's
 * error).  *n_done = number written; never blocks. */
caps_status caps_server_poll(caps_server *srv, int32_t max, uint64_t *tickets, int32_t *ids, float *dist,
                             float *latency_ms, int32_t *status, int32_t *n_done);

/* Waits until every accepted request has a result; EBUSY after timeout_s. */
caps_status caps_server_drain(caps_server *srv, double timeout_s);

/* Counters and latency percentiles since creation or the last reset;
 * reset = 1 starts a new measurement window. */
caps_status caps_server_stats(caps_server *srv, caps_server_stats_t *out, int32_t reset);

/* Stops accepting, finishes what was accepted, joins the scheduler and
 * frees the server (NULL is a no-op).  Unpolled results are dropped. */
void caps_server_destroy(caps_server *srv);

/*
 * Index files.  caps_save writes the index (arrays as they live in HBM, its
 * low-precision copy and its router with the Adam state) to `path` as one
 * versioned little-endian file; caps_load reads it into a new index on the
 * current device (synchronous; `stream` is unused).  A loaded index answers
 * every query exactly as the saved one.  Errors: EINVAL (null arguments),
 * EIO (open/read/write failure, wrong magic or version, inconsistent
 * contents), ENOMEM, EDEVICE.
 */
caps_status caps_save(const caps_index *idx, const char *path);
caps_status caps_load(const char *path, void *stream, caps_index **out);

/* Release the index and its device memory (NULL is a no-op). */
void caps_free(caps_index *idx);

/* Thread-local message for the last non-OK status of this thread. */
const char *caps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
