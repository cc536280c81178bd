// Internal declarations of libcaps (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/caps.h"

namespace caps {

constexpr int kMaxDense = 8;        // dense attributes per point
constexpr int kMaxLabels = 8;       // distinct labels per query; label slots of a narrow point
constexpr int kMaxPointLabels = 128; // labels per point (wide slot rows above kMaxLabels)
constexpr int kMaxHeight = 15;      // AFT height
constexpr int kMaxPartitions = 8192;
constexpr int kMaxTokensLds = 16384;  // token vocabulary the AFT histogram holds in LDS
constexpr int kMaxK = 64;

void set_error(const char *fmt, ...);

#define CAPS_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            ::caps::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                              __FILE__, __LINE__);                                          \
            return e_ == hipErrorOutOfMemory ? CAPS_ENOMEM : CAPS_EDEVICE;                  \
        }                                                                                   \
    } while (0)

// Attribute schema shared by build and search kernels (passed by value).
struct Schema {
    int32_t n_dense;
    int32_t dense_vocab[kMaxDense];
    int32_t dense_off[kMaxDense + 1];   // token offsets; label tokens start at dense_off[n_dense]
    int32_t field_shift[kMaxDense];     // bit position of each dense field in the packed word
    int32_t field_bits[kMaxDense];
    int32_t label_vocab;                // 0: no labels
    int32_t n_tok;
};

// Per-query filter description built on the device from constraint pairs.
// A disjunctive query (AND-terms joined by OR) has one descriptor per
// satisfiable term (kMaxTerms per query, in a separate array) and a summary
// descriptor: flag kQOr, the number of terms, and the dense constraints all
// its terms share (a necessary condition the scans test first).
constexpr uint32_t kQUnsat = 1u;     // contradictory / out of range: chooses nothing
constexpr uint32_t kQNonFinite = 2u; // query row holds NaN or Inf: chooses nothing
constexpr uint32_t kQOr = 4u;        // disjunction: evaluate the terms
constexpr int kMaxTerms = CAPS_MAX_TERMS;
struct alignas(16) QDesc {
    uint32_t dmask;       // packed-field mask of constrained dense attributes
    uint32_t dval;        // required packed values under dmask
    uint32_t flags;       // kQ* bits
    int32_t nlab;         // distinct label constraints (<= kMaxLabels)
    uint64_t lsig;        // OR of signature bits of the label constraints
    uint16_t lab[kMaxLabels];
    int32_t nterm;        // kQOr: satisfiable terms (2..kMaxTerms)
    int32_t pad;
};

struct Index {
    int device = 0;
    int64_t n = 0;
    int32_t d = 0, b = 0, h = 0, metric = 0;
    Schema sch{};
    int32_t max_sub = 0;
    int64_t bytes = 0;
    // device arrays
    float *cent = nullptr;      // b x d
    float *cnorm = nullptr;     // b  (ordered-fma |c|^2)
    int32_t *tags = nullptr;    // b x h tokens (-1 unused)
    int32_t *offs = nullptr;    // b*(h+1)+1
    int32_t *perm = nullptr;    // n: CSR position -> id
    int32_t *assign = nullptr;  // n (original order)
    int8_t *level = nullptr;    // n (original order)
    uint32_t *words = nullptr;  // n packed dense words, CSR order (n_dense > 0)
    uint64_t *sigs = nullptr;   // n label signatures, CSR order (labels)
    uint16_t *slots = nullptr;  // n x lslots sorted labels, 0xFFFF padded
    int32_t lslots = kMaxLabels; // label slots per point: 8, or a power of two up to 128 for wider sets
    float *vecs = nullptr;      // n x d, CSR order
    // low-precision copy for the matrix-core scan (search mode 1)
    int32_t prec = 0;           // CAPS_PREC_*
    int32_t dpad = 0;           // 32, 64, 128 or 256: smallest >= d (zero padded)
    void *lvecs = nullptr;      // n x dpad elements (2 bytes BF16/FP16, 1 byte FP8), CSR order
    float *lscale = nullptr;    // n per-vector FP8 scales (FP8 only)
    float *xnorm = nullptr;     // n exact FP32 |x|^2 (sequential fma), CSR order
    float *lerr = nullptr;      // n upper bounds on |x - x~| (x~: the copy's value), CSR order
    float *lnrm = nullptr;      // n upper bounds on |x~|, CSR order
    void *clow = nullptr;       // b x dpad centroid copy in the same format (precision-mode routing)
    float *cscale = nullptr;    // b per-centroid FP8 scales
    std::vector<int32_t> h_offs;
    struct Router *router = nullptr;   // learned router (owned), if trained or set
};

// Learned router state (caps_router.hip): a two-layer perceptron on
// [q * in_scale + in_shift || 64-wide hashed constraint tokens].
struct Router {
    int32_t din = 0, dpad = 0, hid = 0, nout = 0;   // d + 64, padded to 32, hidden width, B
    float in_scale = 1.0f, in_shift = 0.0f, fb_prob = 0.0f;
    int64_t step = 0;                               // Adam steps taken
    int64_t nparam = 0;                             // w1 (hid x dpad), b1, w2 (nout x hid), b2
    int64_t o_b1 = 0, o_w2 = 0, o_b2 = 0;           // offsets into the parameter arrays
    float *param = nullptr, *mom = nullptr, *vel = nullptr;   // FP32 masters and Adam moments
    uint16_t *w1h = nullptr, *w2h = nullptr;                   // BF16 copies for the products
};
void router_free(Router *r);
// frees every device array of an index and resets it (caps_api.hip)
void release_index(Index &ix);

// signature bit (0..63) of a label: Fibonacci hashing of the label id
__host__ __device__ inline uint32_t label_sig_bit(uint32_t l) {
    return (l * 0x9E3779B1u) >> 26;
}

// float -> uint32 whose unsigned order is the float order (no NaN inputs;
// callers turn -0 into +0 first)
__host__ __device__ inline uint32_t f2ord(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ord2f(uint32_t u) {
    u = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    return __builtin_bit_cast(float, u);
}
__host__ __device__ inline float canon0(float v) { return v == 0.0f ? 0.0f : v; }

// ---- build (caps_build.hip)
caps_status build_index(Index *ix, const float *x, int64_t n, int32_t d, const uint32_t *dense,
                        const int64_t *label_off, const uint32_t *labels,
                        const caps_build_params *p, hipStream_t st);

// ---- search (caps_search.hip)
struct SearchExtra {
    uint64_t *surv_mask = nullptr;   // debug: per query, survivor bits over CSR positions (device)
    void *ws = nullptr;              // caller workspace: the search allocates nothing
    size_t ws_bytes = 0;
};
caps_status search(const Index *ix, const caps_search_params *sp, const float *q, int32_t nq,
                   const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                   int32_t n_con, int32_t *out_ids, float *out_dist, int32_t *out_ncand, int32_t *out_nsurv,
                   int32_t *out_probes, uint32_t *out_masks, hipStream_t st, const SearchExtra *extra = nullptr);

// argument checks shared by the search entry points (caps_api.hip)
caps_status caps_search_check(const caps_index *idx, const caps_search_params *sp, const float *q, int32_t n_q,
                              const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                              int32_t n_con);

// device bytes the workspace of one search call of nq queries takes
size_t search_workspace_bytes(const Index *ix, const caps_search_params *sp, int32_t nq);

// ---- per-call runtime settings (caps_util.hip)
// stream-ordered device memory from the library's pool on `device` (freed
// with hipFreeAsync; the pool keeps it for the next call)
caps_status ws_alloc(void **p, size_t bytes, int device, hipStream_t st);
// hipFuncAttributeMaxDynamicSharedMemorySize of `fn`, set only when `bytes`
// exceeds what was set before on `device`
caps_status set_kernel_lds(const void *fn, size_t bytes, int device);

// ---- stage timer (caps_util.hip): no-ops unless enabled
void prof_begin(int stage, hipStream_t st);
void prof_end(int stage, hipStream_t st);

// ---- low-precision path (caps_mfma.hip)
caps_status build_lowp(Index *ix, hipStream_t st);
caps_status build_lowp_centroids(Index *ix, hipStream_t st);
// precision-mode routing: scores of nb rounded queries against the centroid
// copy; with a row list, score row r belongs to query rows[r], r < *nrows
caps_status lowp_route(const Index *ix, const void *qlow, const float *qscale, int32_t nb, float *scores,
                       hipStream_t st, const int32_t *rows = nullptr, const int32_t *nrows = nullptr);
caps_status lowp_qquant(const Index *ix, const float *q, int32_t nb, void *qlow, float *qscale, float *qaux,
                        hipStream_t st);
// low-precision rows (and their FP32 norms and error norms) of n FP32 rows
caps_status quantize_rows(const Index *ix, const float *x, int64_t n, void *lvec, float *scale, float *xnorm,
                          float *lerr, float *lnrm, hipStream_t st);
// dynamic insertion of n_new points (HOST arrays, validated by the caller)
caps_status insert_points(Index *ix, const float *x, int64_t n_new, const uint32_t *dense, const int64_t *label_off,
                          const uint32_t *labels, hipStream_t st);
// one launch of the matrix-core scan over a sub-batch of nb queries
struct LowpScan {
    int32_t nb, m, r;             // r: keys kept per (query, probe)
    int kind;                     // 0 approximate keys, 1 exact main pass, 2 exact rescue pass, 4 seed lists
                                  // (approximate keys of the seed probes on 32 x 32 blocks)
    int stage;                    // profiling stage of the launch (CAPS_STAGE_SCAN or _SEED)
    int64_t max_tiles;
    const int4 *tiles;            // per tile: partition, first entry, entries (0: none)
    const int32_t *entries;
    const uint32_t *esel;         // level mask per entry, in entry order (or null)
    const uint32_t *sel;
    const QDesc *qd;
    const QDesc *qterms;          // disjunctive searches: term descriptors (kMaxTerms per query)
    bool disj;                    // the batch may hold disjunctions (the filter's slow path is compiled in)
    const float *q;               // nb x d FP32 queries of the sub-batch
    void *qlow;
    float *qscale, *qaux;
    uint64_t *partials, *tau;
    int32_t *pcnt, *nsurv;
    uint64_t *dpos;               // exact main pass: deferred pairs per query, (score key << 32) | position
    int32_t *dcnt;                // and their count
    int32_t dcap;                 // capacity of each query's deferred list
    int32_t *oflow;               // exact: per query, set by the main pass for the rescue pass
    const int32_t *rlist, *rcount;   // rescue pass: tiles with a flagged query and their number
    int32_t rescue_grid;          // rescue pass: workgroups walking its tile list (0: default)
    bool rhalves;                 // rescue pass after a main pass of 128-entry tiles: entries 2 tile + half
};
size_t lowp_scan_lds(const Index *ix, int r, int kind, bool disj);
caps_status lowp_scan(const Index *ix, const LowpScan &S, hipStream_t st);
// The relative rounding margin eta of the exact matrix-core scan's element
// test (its row bound; the merge applies the same test at a second bound).
inline float exact_eta(const Index *ix) { return (float)(6.0 * ix->dpad + 64.0) * 0x1p-24f; }
caps_status lowp_merge(const Index *ix, const float *q, int32_t nb, const uint32_t *sel, int32_t m, int32_t k,
                       int32_t r, const uint64_t *partials, const int32_t *pcnt, const int32_t *cand, int32_t *ncand,
                       int32_t *out_ids, float *out_dist, hipStream_t st);

// ---- shared device utilities (caps_util.hip)
// `sums` is caller workspace of exclusive_scan_tiles(n) ints
int64_t exclusive_scan_tiles(int64_t n);
caps_status exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *sums,
                               hipStream_t st);

// ---- learned routing inside a search (caps_router.hip): fills `scores`
// (nb x B, smaller is better) from the router's logits and `conf` with the
// softmax top-1 probability of each query; X and H are workspace of
// nb x dpad and nb x hid BF16 elements, bneg of B floats (the negated bias).
caps_status router_scores(const Index *ix, const float *q, int32_t nb, const int32_t *con_off,
                          const int32_t *con_attr, const int32_t *con_val, int32_t n_con, uint16_t *X,
                          uint16_t *H, float *bneg, float *scores, float *conf, hipStream_t st);
// Lists the queries whose router probes fall back to centroid routing (top-1
// probability below the fallback level, or fewer than k candidates in the
// router's probes): fbq[0 .. *nfb), in no particular order.
caps_status router_fallback_list(const Index *ix, int32_t nb, int32_t m, int32_t k, const float *conf,
                                 const int32_t *cand, int32_t *fbq, int32_t *nfb, hipStream_t st);
// Copies row r of probes_c (the centroid probes of query fbq[r]) over that
// query's probes, for r < *nfb.
caps_status router_fallback_apply(int32_t nb, int32_t m, const int32_t *fbq, const int32_t *nfb,
                                  const int32_t *probes_c, int32_t *probes, hipStream_t st);

}  // namespace caps

struct caps_index {
    caps::Index ix;
};
