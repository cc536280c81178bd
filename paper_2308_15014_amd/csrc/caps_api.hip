// C ABI of libcaps: argument validation, index lifetime, error reporting.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "caps_internal.h"

namespace caps {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static caps_status fail(caps_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

void release_index(Index &ix) {
    void *ptrs[] = {ix.cent, ix.cnorm, ix.tags, ix.offs, ix.perm, ix.assign, ix.level,
                    ix.words, ix.sigs, ix.slots, ix.vecs, ix.lvecs, ix.lscale, ix.xnorm, ix.lerr, ix.lnrm,
                    ix.clow, ix.cscale};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    router_free(ix.router);
    ix = Index{};
}

// Points to add to an index with schema `sch`: finite vectors, dense
// values inside their vocabularies, label sets of at most max_labels
// distinct labels inside the label vocabulary (HOST arrays).
static caps_status check_points(const char *who, const Schema &sch, const float *x, int64_t n, int32_t d,
                                const uint32_t *dense_vals, const int64_t *label_off, const uint32_t *labels,
                                int32_t max_labels = kMaxPointLabels) {
    const int32_t n_dense = sch.n_dense;
    if (label_off) {
        if (label_off[0] != 0) return fail(CAPS_EINVAL, "%s: label_off[0] != 0", who);
        for (int64_t i = 0; i < n; i++) {
            const int64_t lo = label_off[i], hi = label_off[i + 1];
            if (hi < lo) return fail(CAPS_EINVAL, "%s: label_off decreases at %lld", who, (long long)i);
            if (hi - lo > max_labels)
                return fail(CAPS_EUNSUPPORTED, "%s: point %lld has more than %d labels", who, (long long)i, max_labels);
            for (int64_t e = lo; e < hi; e++) {
                if (labels[e] >= (uint32_t)sch.label_vocab)
                    return fail(CAPS_EINVAL, "%s: label %u outside vocabulary", who, labels[e]);
                for (int64_t f = lo; f < e; f++)
                    if (labels[f] == labels[e])
                        return fail(CAPS_EINVAL, "%s: point %lld repeats label %u", who, (long long)i, labels[e]);
            }
        }
    }
    for (int64_t i = 0; i < n * n_dense; i++)
        if (dense_vals[i] >= (uint32_t)sch.dense_vocab[i % n_dense])
            return fail(CAPS_EINVAL, "%s: dense value outside vocabulary at %lld", who, (long long)i);
    for (int64_t i = 0; i < n * (int64_t)d; i++)
        if (!isfinite(x[i])) return fail(CAPS_EINVAL, "%s: non-finite x at %lld", who, (long long)i);
    return CAPS_OK;
}

}  // namespace caps

using namespace caps;

extern "C" const char *caps_last_error(void) { return g_err; }

extern "C" caps_status caps_build(const float *x, int64_t n, int32_t d, const uint32_t *dense_vals,
                                  int32_t n_dense, const int32_t *dense_vocab, const int64_t *label_off,
                                  const uint32_t *labels, int32_t label_vocab, const caps_build_params *p,
                                  void *stream, caps_index **out) {
    if (!out || !p || !x) return fail(CAPS_EINVAL, "caps_build: null argument");
    *out = nullptr;
    if (n <= 0 || d <= 0) return fail(CAPS_EINVAL, "caps_build: n and d must be positive");
    if (n > INT32_MAX - 1) return fail(CAPS_EUNSUPPORTED, "caps_build: n above 2^31-2");
    if (p->metric != CAPS_METRIC_L2 && p->metric != CAPS_METRIC_IP)
        return fail(CAPS_EINVAL, "caps_build: metric must be 0 (L2) or 1 (IP)");
    const int32_t b = p->n_partitions, h = p->aft_height;
    if (b < 1 || (int64_t)b > n) return fail(CAPS_EINVAL, "caps_build: need 1 <= B <= n (B=%d)", b);
    if (b > kMaxPartitions) return fail(CAPS_EUNSUPPORTED, "caps_build: B above %d", kMaxPartitions);
    if (h < 0) return fail(CAPS_EINVAL, "caps_build: aft_height < 0");
    if (h > kMaxHeight) return fail(CAPS_EUNSUPPORTED, "caps_build: aft_height above %d", kMaxHeight);
    if (p->kmeans_iters < 0) return fail(CAPS_EINVAL, "caps_build: kmeans_iters < 0");
    if (p->precision < CAPS_PREC_NONE || p->precision > CAPS_PREC_FP16)
        return fail(CAPS_EINVAL, "caps_build: precision must be one of CAPS_PREC_*");
    if (p->precision != CAPS_PREC_NONE && d > 256)
        return fail(CAPS_EUNSUPPORTED, "caps_build: the low-precision copy needs d <= 256");
    if (n_dense < 0) return fail(CAPS_EINVAL, "caps_build: n_dense < 0");
    if (n_dense > kMaxDense) return fail(CAPS_EUNSUPPORTED, "caps_build: more than %d dense attributes", kMaxDense);
    if (n_dense > 0 && (!dense_vals || !dense_vocab)) return fail(CAPS_EINVAL, "caps_build: dense arrays missing");
    if (label_off && !labels && label_off[n] != 0)
        return fail(CAPS_EINVAL, "caps_build: labels missing");

    Schema sch{};
    sch.n_dense = n_dense;
    int bits = 0;
    for (int a = 0; a < n_dense; a++) {
        const int32_t v = dense_vocab[a];
        if (v < 1) return fail(CAPS_EINVAL, "caps_build: dense_vocab[%d] < 1", a);
        int w = 1;
        while ((1ll << w) < v) w++;
        sch.dense_vocab[a] = v;
        sch.dense_off[a] = (a == 0) ? 0 : sch.dense_off[a - 1] + sch.dense_vocab[a - 1];
        sch.field_shift[a] = bits;
        sch.field_bits[a] = w;
        bits += w;
    }
    sch.dense_off[n_dense] = n_dense ? sch.dense_off[n_dense - 1] + sch.dense_vocab[n_dense - 1] : 0;
    if (bits > 32) return fail(CAPS_EUNSUPPORTED, "caps_build: packed dense fields need %d > 32 bits", bits);
    const bool has_labels = label_off != nullptr;
    if (has_labels) {
        if (label_vocab < 1 || label_vocab > 65535)
            return fail(label_vocab < 1 ? CAPS_EINVAL : CAPS_EUNSUPPORTED, "caps_build: label_vocab %d", label_vocab);
        sch.label_vocab = label_vocab;
    }
    sch.n_tok = sch.dense_off[n_dense] + (has_labels ? label_vocab : 0);
    if (sch.n_tok > kMaxTokensLds)
        return fail(CAPS_EUNSUPPORTED, "caps_build: %d attribute values exceed %d", sch.n_tok, kMaxTokensLds);
    {
        const caps_status cs = check_points("caps_build", sch, x, n, d, dense_vals, label_off, labels);
        if (cs != CAPS_OK) return cs;
    }
    if (p->init_ids) {
        for (int32_t c = 0; c < b; c++) {
            const int32_t id = p->init_ids[c];
            if (id < 0 || id >= n) return fail(CAPS_EINVAL, "caps_build: init id %d out of range", id);
        }
    }
    if (p->assign) {
        for (int64_t i = 0; i < n; i++)
            if (p->assign[i] < 0 || p->assign[i] >= b)
                return fail(CAPS_EINVAL, "caps_build: assign[%lld] = %d outside [0, B)", (long long)i, p->assign[i]);
    }

    // label slots per point: 8, or the next power of two above the largest set
    int32_t lslots = kMaxLabels;
    if (has_labels) {
        int64_t mx = 0;
        for (int64_t i = 0; i < n; i++) mx = std::max(mx, label_off[i + 1] - label_off[i]);
        while (lslots < mx) lslots <<= 1;
    }
    caps_index *h_idx = new (std::nothrow) caps_index;
    if (!h_idx) return fail(CAPS_ENOMEM, "caps_build: host allocation");
    Index &ix = h_idx->ix;
    ix.lslots = lslots;
    CAPS_HIP(hipGetDevice(&ix.device));
    ix.n = n;
    ix.d = d;
    ix.b = b;
    ix.h = h;
    ix.metric = p->metric;
    ix.sch = sch;
    ix.prec = p->precision;
    caps_status s = build_index(&ix, x, n, d, dense_vals, has_labels ? label_off : nullptr,
                                has_labels ? labels : nullptr, p, (hipStream_t)stream);
    if (s == CAPS_OK) s = build_lowp(&ix, (hipStream_t)stream);
    if (s == CAPS_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) s = CAPS_EDEVICE;
    if (s != CAPS_OK) {
        release_index(ix);
        delete h_idx;
        return s;
    }
    *out = h_idx;
    return CAPS_OK;
}

extern "C" caps_status caps_bliss_assign(const int32_t *cand, int64_t n, int32_t k_cand, int32_t b,
                                         int32_t *out_assign) {
    if (n < 0 || k_cand < 1 || b < 1) return fail(CAPS_EINVAL, "caps_bliss_assign: need n >= 0, K >= 1, b >= 1");
    if (n > 0 && (!cand || !out_assign)) return fail(CAPS_EINVAL, "caps_bliss_assign: null array");
    for (int64_t e = 0; e < n * (int64_t)k_cand; e++)
        if (cand[e] < 0 || cand[e] >= b)
            return fail(CAPS_EINVAL, "caps_bliss_assign: candidate %d outside [0, %d)", cand[e], b);
    std::vector<int64_t> load((size_t)b, 0);
    for (int64_t i = 0; i < n; i++) {
        const int32_t *c = cand + i * k_cand;
        int32_t best = c[0];
        for (int32_t r = 1; r < k_cand; r++)
            if (load[(size_t)c[r]] < load[(size_t)best]) best = c[r];
        out_assign[i] = best;
        load[(size_t)best]++;
    }
    return CAPS_OK;
}

caps_status caps::caps_search_check(const caps_index *idx, const caps_search_params *sp, const float *q, int32_t n_q,
                                const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                                int32_t n_con) {
    if (!idx || !sp) return fail(CAPS_EINVAL, "caps_search: null index or params");
    const Index &ix = idx->ix;
    if (n_q < 0) return fail(CAPS_EINVAL, "caps_search: n_q < 0");
    if (sp->k < 1) return fail(CAPS_EINVAL, "caps_search: k < 1");
    if (sp->k > kMaxK) return fail(CAPS_EUNSUPPORTED, "caps_search: k above %d", kMaxK);
    if (sp->nprobe < 1 || sp->nprobe > ix.b) return fail(CAPS_EINVAL, "caps_search: nprobe outside [1, B]");
    if (sp->rule != 0 && sp->rule != 1) return fail(CAPS_EINVAL, "caps_search: rule must be 0 or 1");
    if (sp->mode < 0 || sp->mode > 2) return fail(CAPS_EINVAL, "caps_search: mode must be 0, 1 or 2");
    if (sp->mode == 1) {
        if (ix.prec == CAPS_PREC_NONE)
            return fail(CAPS_EINVAL, "caps_search: mode 1 needs an index built with a precision");
        if (sp->rerank != 0 && (sp->rerank < sp->k || sp->rerank > kMaxK))
            return fail(CAPS_EINVAL, "caps_search: rerank must be in [k, %d]", kMaxK);
    }
    if (sp->routing != 0 && sp->routing != 1) return fail(CAPS_EINVAL, "caps_search: routing must be 0 or 1");
    if (sp->flags & ~(int32_t)(CAPS_SEARCH_VALIDATE | CAPS_SEARCH_DISJUNCTIVE))
        return fail(CAPS_EINVAL, "caps_search: unknown flags 0x%x", (unsigned)sp->flags);
    if (sp->rescue_grid < 0) return fail(CAPS_EINVAL, "caps_search: rescue_grid < 0");
    if (sp->routing == 1 && !ix.router) return fail(CAPS_EINVAL, "caps_search: routing 1 needs a trained router");
    if (n_con < 0) return fail(CAPS_EINVAL, "caps_search: n_con < 0");
    if (n_q > 0 && (!q || !con_off)) return fail(CAPS_EINVAL, "caps_search: null query arrays");
    if (n_con > 0 && (!con_attr || !con_val)) return fail(CAPS_EINVAL, "caps_search: null constraint arrays");
    return CAPS_OK;
}

extern "C" caps_status caps_search(const caps_index *idx, const caps_search_params *sp, const float *q,
                                   int32_t n_q, const int32_t *con_off, const int32_t *con_attr,
                                   const int32_t *con_val, int32_t n_con, int32_t *out_ids, float *out_dist,
                                   int32_t *out_ncand, int32_t *out_nsurv, void *stream) {
    caps_status s = caps_search_check(idx, sp, q, n_q, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n_q > 0 && (!out_ids || !out_dist)) return fail(CAPS_EINVAL, "caps_search: null outputs");
    return search(&idx->ix, sp, q, n_q, con_off, con_attr, con_val, n_con, out_ids, out_dist, out_ncand,
                  out_nsurv, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" caps_status caps_search_debug(const caps_index *idx, const caps_search_params *sp, const float *q,
                                         int32_t n_q, const int32_t *con_off, const int32_t *con_attr,
                                         const int32_t *con_val, int32_t n_con, int32_t *out_ids, float *out_dist,
                                         int32_t *out_ncand, int32_t *out_nsurv, uint64_t *out_surv_mask,
                                         void *stream) {
    caps_status s = caps_search_check(idx, sp, q, n_q, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n_q > 0 && (!out_ids || !out_dist || !out_surv_mask))
        return fail(CAPS_EINVAL, "caps_search_debug: null outputs");
    caps_search_params p = *sp;
    p.flags |= CAPS_SEARCH_VALIDATE;
    SearchExtra ex;
    ex.surv_mask = out_surv_mask;
    s = search(&idx->ix, &p, q, n_q, con_off, con_attr, con_val, n_con, out_ids, out_dist, out_ncand, out_nsurv,
               nullptr, nullptr, (hipStream_t)stream, &ex);
    if (s == CAPS_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(CAPS_EDEVICE, "caps_search_debug: stream synchronisation failed");
    return s;
}

extern "C" caps_status caps_search_workspace(const caps_index *idx, const caps_search_params *sp, int32_t n_q,
                                             int64_t *out_bytes) {
    caps_status s = caps_search_check(idx, sp, nullptr, 0, nullptr, nullptr, nullptr, 0);
    if (s != CAPS_OK) return s;
    if (n_q < 0 || !out_bytes) return fail(CAPS_EINVAL, "caps_search_workspace: bad arguments");
    *out_bytes = n_q == 0 ? 0 : (int64_t)search_workspace_bytes(&idx->ix, sp, n_q);
    return CAPS_OK;
}

extern "C" caps_status caps_search_probes(const caps_index *idx, const caps_search_params *sp, const float *q,
                                          int32_t n_q, const int32_t *con_off, const int32_t *con_attr,
                                          const int32_t *con_val, int32_t n_con, int32_t *out_probes,
                                          uint32_t *out_masks, void *stream) {
    caps_status s = caps_search_check(idx, sp, q, n_q, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n_q > 0 && (!out_probes || !out_masks)) return fail(CAPS_EINVAL, "caps_search_probes: null outputs");
    return search(&idx->ix, sp, q, n_q, con_off, con_attr, con_val, n_con, nullptr, nullptr, nullptr, nullptr,
                  out_probes, out_masks, (hipStream_t)stream);
}

extern "C" caps_status caps_index_info(const caps_index *idx, caps_index_info_t *out) {
    if (!idx || !out) return fail(CAPS_EINVAL, "caps_index_info: null argument");
    const Index &ix = idx->ix;
    out->n = ix.n;
    out->d = ix.d;
    out->n_partitions = ix.b;
    out->aft_height = ix.h;
    out->metric = ix.metric;
    out->n_dense = ix.sch.n_dense;
    out->label_vocab = ix.sch.label_vocab;
    out->n_tokens = ix.sch.n_tok;
    out->max_subpartition = ix.max_sub;
    out->precision = ix.prec;
    out->lowp_dpad = ix.prec == CAPS_PREC_NONE ? 0 : ix.dpad;
    out->label_slots = ix.sch.label_vocab > 0 ? ix.lslots : 0;
    out->reserved = 0;
    out->device_bytes = ix.bytes;
    return CAPS_OK;
}

extern "C" caps_status caps_index_export(const caps_index *idx, float *centroids, int32_t *assign, int8_t *level,
                                         int32_t *perm, int32_t *offs, int32_t *tags) {
    if (!idx) return fail(CAPS_EINVAL, "caps_index_export: null index");
    const Index &ix = idx->ix;
    if (centroids) CAPS_HIP(hipMemcpy(centroids, ix.cent, sizeof(float) * (size_t)ix.b * ix.d, hipMemcpyDeviceToHost));
    if (assign) CAPS_HIP(hipMemcpy(assign, ix.assign, sizeof(int32_t) * (size_t)ix.n, hipMemcpyDeviceToHost));
    if (level) CAPS_HIP(hipMemcpy(level, ix.level, sizeof(int8_t) * (size_t)ix.n, hipMemcpyDeviceToHost));
    if (perm) CAPS_HIP(hipMemcpy(perm, ix.perm, sizeof(int32_t) * (size_t)ix.n, hipMemcpyDeviceToHost));
    if (offs)
        CAPS_HIP(hipMemcpy(offs, ix.offs, sizeof(int32_t) * ((size_t)ix.b * (ix.h + 1) + 1), hipMemcpyDeviceToHost));
    if (tags && ix.h > 0)
        CAPS_HIP(hipMemcpy(tags, ix.tags, sizeof(int32_t) * (size_t)ix.b * ix.h, hipMemcpyDeviceToHost));
    return CAPS_OK;
}

extern "C" caps_status caps_index_export_lowp(const caps_index *idx, void *codes, float *scale, float *xnorm) {
    if (!idx) return fail(CAPS_EINVAL, "caps_index_export_lowp: null index");
    const Index &ix = idx->ix;
    if (ix.prec == CAPS_PREC_NONE) return fail(CAPS_EINVAL, "caps_index_export_lowp: no low-precision copy");
    const size_t es = ix.prec == CAPS_PREC_FP8 ? 1 : 2;
    if (codes) CAPS_HIP(hipMemcpy(codes, ix.lvecs, (size_t)ix.n * ix.dpad * es, hipMemcpyDeviceToHost));
    if (scale && ix.lscale) CAPS_HIP(hipMemcpy(scale, ix.lscale, sizeof(float) * (size_t)ix.n, hipMemcpyDeviceToHost));
    if (xnorm) CAPS_HIP(hipMemcpy(xnorm, ix.xnorm, sizeof(float) * (size_t)ix.n, hipMemcpyDeviceToHost));
    return CAPS_OK;
}

extern "C" void caps_free(caps_index *idx) {
    if (!idx) return;
    release_index(idx->ix);
    delete idx;
}

extern "C" caps_status caps_insert(caps_index *idx, const float *x, int64_t n_new, const uint32_t *dense_vals,
                                   const int64_t *label_off, const uint32_t *labels, void *stream) {
    if (!idx || n_new < 0) return fail(CAPS_EINVAL, "caps_insert: null index or n_new < 0");
    if (n_new == 0) return CAPS_OK;
    Index &ix = idx->ix;
    if (!x) return fail(CAPS_EINVAL, "caps_insert: null x");
    if (ix.n + n_new > INT32_MAX - 1) return fail(CAPS_EUNSUPPORTED, "caps_insert: more than 2^31-2 points");
    if (ix.sch.n_dense > 0 && !dense_vals) return fail(CAPS_EINVAL, "caps_insert: dense values missing");
    if ((ix.sch.label_vocab > 0) != (label_off != nullptr))
        return fail(CAPS_EINVAL, "caps_insert: label sets must be given exactly when the index has labels");
    if (label_off && !labels && label_off[n_new] != 0) return fail(CAPS_EINVAL, "caps_insert: labels missing");
    caps_status s = check_points("caps_insert", ix.sch, x, n_new, ix.d, dense_vals, label_off, labels, ix.lslots);
    if (s != CAPS_OK) return s;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ix.device)
        return fail(CAPS_EINVAL, "caps_insert: the index's device must be current");
    return insert_points(&ix, x, n_new, dense_vals, label_off, labels, (hipStream_t)stream);
}
