// Query path on the GPU (paper Algorithm 2).
//
//   prep    constraint pairs -> per-query packed filter (QDesc)
//   route   Q x B centroid scores (sequential-fma dots), then the best m
//           partitions per query under the order (score, id)
//   select  per (query, probe): the sub-partitions that may hold valid
//           points (exact rule) and the candidate count
//   bucket  (query, probe) pairs grouped by partition, cut into tiles of at
//           most 128 queries
//   scan    one workgroup per tile: the partition's chosen sub-partitions
//           stream through LDS in chunks; every (query, point) pair is
//           filtered exactly, survivors are compacted and their distances
//           computed one pair per lane, each query keeps its top k
//   merge   per query, the per-partition top-k lists -> final top k
//
// Partition-major scanning reads each probed partition once per tile of up
// to 128 queries instead of once per query.
#include <string.h>

#include <algorithm>

#include "caps_device.h"
#include "caps_internal.h"
#include "caps_mfma.h"

namespace caps {


// ------------------------------------------------------------------ prep
__device__ inline void qd_clear(QDesc &r) {
    r.dmask = 0;
    r.dval = 0;
    r.flags = 0;
    r.nlab = 0;
    r.lsig = 0;
    for (int i = 0; i < kMaxLabels; i++) r.lab[i] = 0xFFFF;
    r.nterm = 1;
    r.pad = 0;
}

// Adds constraint pair (a, v) to the AND-term r: a dense value becomes a
// packed field under dmask, a label joins the label list and signature; a
// pair outside the vocabularies, a second value of one dense attribute or a
// ninth label makes the term unsatisfiable.
__device__ inline void qd_add(QDesc &r, const Schema &sch, int32_t a, int32_t v) {
    if (a < 0 || a > sch.n_dense) {
        r.flags |= kQUnsat;
        return;
    }
    if (a < sch.n_dense) {
        if (v < 0 || v >= sch.dense_vocab[a]) {
            r.flags |= kQUnsat;
            return;
        }
        const uint32_t fm = (uint32_t)(((1ull << sch.field_bits[a]) - 1ull) << sch.field_shift[a]);
        const uint32_t fv = (uint32_t)v << sch.field_shift[a];
        if ((r.dmask & fm) && ((r.dval & fm) != fv)) r.flags |= kQUnsat;
        r.dmask |= fm;
        r.dval = (r.dval & ~fm) | fv;
        return;
    }
    if (sch.label_vocab == 0 || v < 0 || v >= sch.label_vocab) {
        r.flags |= kQUnsat;
        return;
    }
    for (int i = 0; i < r.nlab; i++)
        if (r.lab[i] == (uint16_t)v) return;   // duplicate: AND is idempotent
    if (r.nlab == kMaxLabels) {
        r.flags |= kQUnsat;
        return;
    }
    r.lab[r.nlab++] = (uint16_t)v;
    r.lsig |= 1ull << label_sig_bit((uint32_t)v);
}

// One thread per query.  Without `disj` every pair is ANDed (a pair with a
// negative attribute, CAPS_OR included, makes the query unsatisfiable).
// With `disj` the pairs with attr == CAPS_OR separate AND-terms: the
// satisfiable terms go to terms[q * kMaxTerms ..] and the summary holds
// kQOr, their number and the dense fields every term fixes to the same value
// (a query with one satisfiable term is that term; none, or more than
// kMaxTerms terms: unsatisfiable).
__global__ __launch_bounds__(128) void k_qprep(const int32_t *__restrict__ con_off, const int32_t *__restrict__ con_attr,
                        const int32_t *__restrict__ con_val, int32_t n_con, int32_t nq, Schema sch, int32_t disj,
                        QDesc *__restrict__ out, QDesc *__restrict__ terms) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    QDesc r;
    qd_clear(r);
    int32_t lo = con_off[q], hi = con_off[q + 1];
    if (lo < 0 || hi < lo || hi > n_con) {
        r.flags |= kQUnsat;
        out[q] = r;
        return;
    }
    if (!disj) {
        for (int32_t e = lo; e < hi; e++) qd_add(r, sch, con_attr[e], con_val[e]);
        out[q] = r;
        return;
    }
    QDesc *tq = terms + (int64_t)q * kMaxTerms;
    QDesc cur;
    qd_clear(cur);
    int nt = 0, nsat = 0;
    for (int32_t e = lo; e <= hi; e++) {
        if (e < hi && con_attr[e] != CAPS_OR) {
            qd_add(cur, sch, con_attr[e], con_val[e]);
            continue;
        }
        if (++nt > kMaxTerms) break;
        if (!(cur.flags & kQUnsat)) tq[nsat++] = cur;
        qd_clear(cur);
    }
    if (nt > kMaxTerms || nsat == 0) {
        r.flags |= kQUnsat;
    } else if (nsat == 1) {
        r = tq[0];
    } else {
        uint32_t all = ~0u, diff = 0;
        for (int t = 0; t < nsat; t++) {
            all &= tq[t].dmask;
            diff |= tq[t].dval ^ tq[0].dval;
        }
        uint32_t keep = 0;
        for (int a = 0; a < sch.n_dense; a++) {
            const uint32_t fm = (uint32_t)(((1ull << sch.field_bits[a]) - 1ull) << sch.field_shift[a]);
            if ((all & fm) == fm && !(diff & fm)) keep |= fm;
        }
        r.dmask = keep;
        r.dval = tq[0].dval & keep;
        r.flags = kQOr;
        r.nterm = nsat;
    }
    out[q] = r;
}

// ------------------------------------------------------------------ routing
constexpr int kDC = 32;
constexpr int kTile = 64;

// Q x B scores, 64 x 64 tile per workgroup, sequential fma over dims.
// With a row list, score row r belongs to query rows[r] and only the first
// *nrows rows (a count on the device, at most nq) are computed.
__global__ __launch_bounds__(256) void k_route_scores(const float *__restrict__ q, int32_t nq, int32_t d,
                                                      const float *__restrict__ cent,
                                                      const float *__restrict__ cn, int32_t b,
                                                      int32_t metric, float *__restrict__ scores,
                                                      const int32_t *__restrict__ rows = nullptr,
                                                      const int32_t *__restrict__ nrows = nullptr) {
    __shared__ float xs[kDC][kTile + 4];
    __shared__ float cs[kDC][kTile + 4];
    const int t = threadIdx.x;
    const int ty = t >> 4, tx = t & 15;
    const int64_t r0 = (int64_t)blockIdx.x * kTile;
    const int c0 = blockIdx.y * kTile;
    if (nrows) nq = min(nq, *nrows);
    if (r0 >= nq) return;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[i][k] = 0.0f;
    for (int j0 = 0; j0 < d; j0 += kDC) {
        const int dc = min(kDC, d - j0);
        for (int e = t; e < kTile * kDC; e += 256) {
            const int ri = e / kDC, jj = e % kDC;
            float v = 0.0f, w = 0.0f;
            if (jj < dc) {
                if (r0 + ri < nq) v = q[(rows ? (int64_t)rows[r0 + ri] : r0 + ri) * d + j0 + jj];
                if (c0 + ri < b) w = cent[(int64_t)(c0 + ri) * d + j0 + jj];
            }
            xs[jj][ri] = v;
            cs[jj][ri] = w;
        }
        __syncthreads();
        for (int jj = 0; jj < dc; jj++) {
            const float4 a = *reinterpret_cast<const float4 *>(&xs[jj][ty * 4]);
            const float4 c = *reinterpret_cast<const float4 *>(&cs[jj][tx * 4]);
            const float av[4] = {a.x, a.y, a.z, a.w};
            const float cv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int k = 0; k < 4; k++) acc[i][k] = fmaf(av[i], cv[k], acc[i][k]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int64_t r = r0 + ty * 4 + i;
        if (r >= nq) continue;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int c = c0 + tx * 4 + k;
            if (c >= b) continue;
            scores[r * b + c] = canon0(metric == 0 ? cn[c] - 2.0f * acc[i][k] : -acc[i][k]);
        }
    }
}

// Best m of B per query: bitonic sort of (score, id) keys in LDS.
constexpr int kTopmNT = 256;

__global__ __launch_bounds__(kTopmNT) void k_topm(const float *__restrict__ scores, int32_t b, int32_t pb,
                                                  int32_t m, int32_t *__restrict__ probes,
                                                  const int32_t *__restrict__ nrows) {
    extern __shared__ uint64_t keys[];   // pb (power of two >= b)
    const int64_t q = blockIdx.x;
    if (nrows && q >= *nrows) return;
    const float *s = scores + q * b;
    for (int i = threadIdx.x; i < pb; i += kTopmNT)
        keys[i] = i < b ? (((uint64_t)f2ord(s[i]) << 32) | (uint32_t)i) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= pb; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < pb; i += kTopmNT) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = keys[i], c = keys[l];
                    const bool up = (i & k) == 0;
                    if ((a > c) == up) {
                        keys[i] = c;
                        keys[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < m; i += kTopmNT) probes[q * m + i] = (int32_t)(uint32_t)(keys[i] & 0xFFFFFFFFu);
}

// Same result for 256 <= pb <= 8192: thread t holds keys 4t..; the
// compare-exchange stages of the bitonic network run in registers (partner in
// the same thread), through lane shuffles (partner in the same wave) and
// through LDS only when the partner is in another wave (3 stages at
// pb = 1024 instead of 55 barrier stages).
template <int KPT>
__global__ __launch_bounds__(kTopmNT) void k_topm_reg(const float *__restrict__ scores, int32_t b, int32_t m,
                                                      int32_t *__restrict__ probes,
                                                      const int32_t *__restrict__ nrows) {
    constexpr int PB = KPT * kTopmNT;
    __shared__ uint64_t ex[PB];
    const int64_t q = blockIdx.x;
    if (nrows && q >= *nrows) return;
    const float *s = scores + q * b;
    const int t = threadIdx.x;
    uint64_t v[KPT];
#pragma unroll
    for (int r = 0; r < KPT; r++) {
        const int i = t * KPT + r;
        v[r] = i < b ? (((uint64_t)f2ord(s[i]) << 32) | (uint32_t)i) : ~0ull;
    }
    // element i keeps the smaller of (i, i ^ j) when it is the lower index of
    // an ascending pair or the upper index of a descending one
    auto keep = [](uint64_t a, uint64_t o, int i, int j, int k) {
        const bool take_min = ((i & j) == 0) == ((i & k) == 0);
        return take_min ? (o < a ? o : a) : (o > a ? o : a);
    };
    for (int k = 2; k <= PB; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < KPT) {
#pragma unroll
                for (int r = 0; r < KPT; r++) {
                    const int rp = r ^ j;
                    if (rp > r) {
                        const int i = t * KPT + r;
                        const uint64_t a = v[r], o = v[rp];
                        v[r] = keep(a, o, i, j, k);
                        v[rp] = keep(o, a, i ^ j, j, k);
                    }
                }
            } else if (j < 64 * KPT) {
                const int lm = j / KPT;
#pragma unroll
                for (int r = 0; r < KPT; r++) {
                    const uint64_t o = __shfl_xor(v[r], lm, 64);
                    v[r] = keep(v[r], o, t * KPT + r, j, k);
                }
            } else {
                __syncthreads();   // the previous exchange is read
#pragma unroll
                for (int r = 0; r < KPT; r++) ex[t * KPT + r] = v[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < KPT; r++) {
                    const int i = t * KPT + r;
                    v[r] = keep(v[r], ex[i ^ j], i, j, k);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < KPT; r++) {
        const int i = t * KPT + r;
        if (i < m) probes[q * m + i] = (int32_t)(uint32_t)(v[r] & 0xFFFFFFFFu);
    }
}

// The search itself needs the best m partitions of a query as a set, with
// its best s (the seed probes) in the first s slots, in no particular order
// otherwise.  One wave per query finds the m-th and the s-th smallest key
// (ordered score, then id) by bisection over the score bits, then over the
// ids of the tied scores, and writes the ids in two compacted groups.  KPT =
// pb / 64 scores per lane (position r * 64 + lane).
template <int KPT>
__global__ __launch_bounds__(256) void k_topm_sel(const float *__restrict__ scores, int32_t nq, int32_t b, int32_t m,
                                                  int32_t s, int32_t *__restrict__ probes,
                                                  const int32_t *__restrict__ nrows) {
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq || (nrows && q >= *nrows)) return;
    const float *sc = scores + q * b;
    uint32_t u[KPT];
#pragma unroll
    for (int r = 0; r < KPT; r++) {
        const int i = r * 64 + lane;
        u[r] = i < b ? f2ord(sc[i]) : ~0u;
    }
    // wave-wide counts come from one ballot per register (scalar popcounts,
    // no cross-lane data movement)
    // the n-th smallest key (n >= 1): score su and id iu; ties of su are taken
    // by ascending id up to iu.  The bisection keeps the n-th key inside
    // [ans, ans + 2^(bit+1)) with c_lo keys below the range and c_hi below its
    // end; once the range holds a single key, that key (the smallest at or
    // above ans) is the answer.  When every tie of su is needed the ids are
    // not bisected.
    auto kth = [&](int n, uint32_t &su, int &iu) {
        uint32_t ans = 0;
        int c_lo = 0, c_hi = KPT * 64;
        bool one = false;
        for (int bit = 31; bit >= 0; bit--) {
            const uint32_t t = ans | (1u << bit);
            int c = 0;
#pragma unroll
            for (int r = 0; r < KPT; r++) c += __popcll(__ballot(u[r] < t));
            if (c < n) {
                ans = t;
                c_lo = c;
            } else {
                c_hi = c;
            }
            if (c_hi - c_lo == 1) {
                one = true;
                break;
            }
        }
        if (one) {
            uint64_t mn = ~0ull;
#pragma unroll
            for (int r = 0; r < KPT; r++)
                if (u[r] >= ans && u[r] < mn) mn = u[r];
            su = (uint32_t)wave_min_u64(mn);
        } else {
            su = ans;
        }
        int lt = 0, eq = 0;
#pragma unroll
        for (int r = 0; r < KPT; r++) {
            lt += __popcll(__ballot(u[r] < su));
            eq += __popcll(__ballot(u[r] == su));
        }
        const int need = n - lt;   // >= 1 ties of su to take, by id
        if (need >= eq) {          // all of them
            iu = INT32_MAX;
            return;
        }
        int ia = 0;
        for (int bit = 31 - __builtin_clz((unsigned)(KPT * 64)); bit >= 0; bit--) {
            const int t = ia | (1 << bit);
            int c = 0;
#pragma unroll
            for (int r = 0; r < KPT; r++) c += __popcll(__ballot(u[r] == su && r * 64 + lane < t));
            if (c < need) ia = t;
        }
        iu = ia;
    };
    auto below = [&](uint32_t v, int i, uint32_t su, int iu) { return v < su || (v == su && i <= iu); };
    uint32_t sm, ss = 0;
    int im, is = -1;
    kth(m, sm, im);
    if (s < m) kth(s, ss, is);
    int32_t *out = probes + q * m;
    int n0 = 0, n1 = s < m ? s : 0;
#pragma unroll
    for (int r = 0; r < KPT; r++) {
        const int i = r * 64 + lane;
        const bool in_m = below(u[r], i, sm, im);
        const bool in_s = s < m && below(u[r], i, ss, is);
        const uint64_t b0 = __ballot(in_s), b1 = __ballot(in_m && !in_s);
        const uint64_t lt = lanemask_lt();
        // (exactly s and m - s keys qualify; the bounds are a guard)
        const int p0 = n0 + __popcll(b0 & lt), p1 = n1 + __popcll(b1 & lt);
        if (in_s && p0 < s) out[p0] = i;
        else if (!in_s && in_m && p1 < m) out[p1] = i;
        n0 += __popcll(b0);
        n1 += __popcll(b1);
    }
}

// Launches the register bitonic top-m when pb allows, else the LDS one.
// With s >= 0 (a search, not the probes query) the selection kernel instead,
// for B up to 4096: the best m as a set, the best s in the first slots.
// nrows (a device count, or null): only the first *nrows of the nb rows.
static void launch_topm(const float *scores, int32_t nb, int32_t b, int32_t pb, int32_t m, int32_t *probes,
                        hipStream_t st, int32_t s = -1, const int32_t *nrows = nullptr) {
    if (s >= 0 && pb >= 64 && pb <= 4096) {
        const dim3 g((nb + 3) / 4);
        switch (pb) {
        case 64: hipLaunchKernelGGL(k_topm_sel<1>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        case 128: hipLaunchKernelGGL(k_topm_sel<2>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        case 256: hipLaunchKernelGGL(k_topm_sel<4>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        case 512: hipLaunchKernelGGL(k_topm_sel<8>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        case 1024: hipLaunchKernelGGL(k_topm_sel<16>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        case 2048: hipLaunchKernelGGL(k_topm_sel<32>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        default: hipLaunchKernelGGL(k_topm_sel<64>, g, dim3(256), 0, st, scores, nb, b, m, s, probes, nrows); return;
        }
    }
    switch (pb) {
    case 256: hipLaunchKernelGGL(k_topm_reg<1>, dim3(nb), dim3(kTopmNT), 0, st, scores, b, m, probes, nrows); return;
    case 512: hipLaunchKernelGGL(k_topm_reg<2>, dim3(nb), dim3(kTopmNT), 0, st, scores, b, m, probes, nrows); return;
    case 1024: hipLaunchKernelGGL(k_topm_reg<4>, dim3(nb), dim3(kTopmNT), 0, st, scores, b, m, probes, nrows); return;
    case 2048: hipLaunchKernelGGL(k_topm_reg<8>, dim3(nb), dim3(kTopmNT), 0, st, scores, b, m, probes, nrows); return;
    case 4096: hipLaunchKernelGGL(k_topm_reg<16>, dim3(nb), dim3(kTopmNT), 0, st, scores, b, m, probes, nrows); return;
    case 8192: hipLaunchKernelGGL(k_topm_reg<32>, dim3(nb), dim3(kTopmNT), 0, st, scores, b, m, probes, nrows); return;
    default:
        hipLaunchKernelGGL(k_topm, dim3(nb), dim3(kTopmNT), sizeof(uint64_t) * (size_t)pb, st, scores, b, pb, m,
                           probes, nrows);
    }
}

// ------------------------------------------------------------------ selection
__device__ inline void tag_decode(const Schema &s, int32_t tok, int &attr, int32_t &val) {
    if (tok < s.dense_off[s.n_dense]) {
        int a = 0;
        while (a + 1 < s.n_dense && tok >= s.dense_off[a + 1]) a++;
        attr = a;
        val = tok - s.dense_off[a];
    } else {
        attr = s.n_dense;
        val = tok - s.dense_off[s.n_dense];
    }
}

// Exact rule: J* = first tagged level whose tag the query holds (h if none);
// scan level j < h iff j <= J*, tagged, and its tag does not contradict a
// dense constraint; scan the remainder iff J* = h.  rule 1: only level J*.
__device__ inline uint32_t choose_levels(const Schema &s, const QDesc &qd, const int32_t *tags, int h,
                                         int rule) {
    if (qd.flags & (kQUnsat | kQNonFinite)) return 0u;
    int js = h;
    uint32_t ok = 0;
    for (int j = 0; j < h; j++) {
        const int32_t t = tags[j];
        if (t < 0) continue;
        int a;
        int32_t v;
        tag_decode(s, t, a, v);
        bool held, conflict = false;
        if (a < s.n_dense) {
            const uint32_t fm = (uint32_t)(((1ull << s.field_bits[a]) - 1ull) << s.field_shift[a]);
            const bool constrained = (qd.dmask & fm) != 0;
            const bool same = ((qd.dval & fm) >> s.field_shift[a]) == (uint32_t)v;
            held = constrained && same;
            conflict = constrained && !same;
        } else {
            held = false;
            for (int i = 0; i < qd.nlab; i++) held |= qd.lab[i] == (uint16_t)v;
        }
        if (!conflict) ok |= 1u << j;
        if (held) {
            js = j;
            break;
        }
    }
    if (rule == 1) return 1u << js;
    uint32_t mask = ok & ((js >= 31) ? 0xFFFFFFFFu : ((2u << js) - 1u));
    if (js == h) mask |= 1u << h;
    return mask;
}

// A query's levels: the union over its terms for a disjunction (Section 5.3:
// several sub-partitions per partition join the candidate set).
__device__ inline uint32_t choose_query_levels(const Schema &s, const QDesc &qd, const QDesc *terms,
                                               const int32_t *tags, int h, int rule) {
    if (qd.flags & (kQUnsat | kQNonFinite)) return 0u;
    if (!(qd.flags & kQOr)) return choose_levels(s, qd, tags, h, rule);
    uint32_t mask = 0;
    for (int t = 0; t < qd.nterm; t++) mask |= choose_levels(s, terms[t], tags, h, rule);
    return mask;
}

__global__ void k_select(const int32_t *__restrict__ probes, int32_t nq, int32_t m,
                         const QDesc *__restrict__ qd, const QDesc *__restrict__ qterms, Schema sch,
                         const int32_t *__restrict__ tags, int32_t h, const int32_t *__restrict__ offs, int32_t rule,
                         uint32_t *__restrict__ sel, int32_t *__restrict__ cand_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nq * m) return;
    const int32_t q = (int32_t)(e / m);
    const int32_t p = probes[e];
    const uint32_t mask = choose_query_levels(sch, qd[q], qterms + (int64_t)q * kMaxTerms, tags + (int64_t)p * h, h,
                                              rule);
    int32_t cand = 0;
    for (int j = 0; j <= h; j++)
        if (mask & (1u << j)) cand += offs[(int64_t)p * (h + 1) + j + 1] - offs[(int64_t)p * (h + 1) + j];
    sel[e] = mask;
    cand_out[e] = cand;
}

// Bucketing of the chosen (query, probe) pairs by partition without global
// atomics: block g counts its queries' pairs per partition (hist, stored
// partition-major), an exclusive scan turns the counts into positions, and
// the fill pass places each pair.  k_class_sort then groups each partition's
// pairs by their level mask (nc classes, nc = 2^(h+1) for h <= 3, else 1): a
// tile mostly holds queries that scan the same levels, and the scans skip
// the levels none of a tile's queries selected.  (Folding the classes into
// the bucketing bins made the histogram eight times larger and its strided
// stores cost more than the class pass.)
constexpr int kBucketQ = 32;   // queries per bucketing block
constexpr int kClassShift = 27;   // packed class of an entry (entries < 2^27)

inline int32_t bucket_classes(int32_t h) { return h <= 3 ? 1 << (h + 1) : 1; }

constexpr int kBucketT = 1024;   // threads per bucketing block

// The block's (query, probe-slot) span [q0, q1) x [r0, r1), flattened (with
// qord: positions q0..q1 of that query order): thread
// t visits flat slots t, t + T, ... (coalesced, one division per thread), four
// at a time with all their loads issued before any is used.  visit(e, mask,
// partition) runs for each chosen slot e.
template <typename F>
__device__ inline void bucket_slots(const int32_t *__restrict__ probes, const uint32_t *__restrict__ sel,
                                    const int32_t *__restrict__ qord, int32_t q0, int32_t q1, int32_t m, int32_t r0,
                                    int32_t r1, F &&visit) {
    const int32_t w = r1 - r0;
    if (w <= 0 || q1 <= q0) return;
    const int32_t n = (q1 - q0) * w, T = (int32_t)blockDim.x, t = (int32_t)threadIdx.x;
    const int32_t dq = T / w, dr = T - dq * w;
    int32_t qq = q0 + t / w, rr = r0 + t % w;
    for (int32_t f = t; f < n; f += 4 * T) {
        int64_t e[4];
        uint32_t sm[4];
        int32_t pr[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const bool ok = f + u * T < n;
            e[u] = (int64_t)(ok && qord ? qord[qq] : qq) * m + rr;
            sm[u] = ok ? sel[e[u]] : 0u;
            pr[u] = ok ? probes[e[u]] : 0;
            rr += dr;   // advance the flat slot by T
            qq += dq;
            if (rr >= r1) {
                rr -= w;
                qq++;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (sm[u]) visit(e[u], sm[u], pr[u]);
    }
}

// Query order for the bucketing: the queries sorted by their dense
// constraint in the order in which the CSR lays out the rows of a
// sub-partition (dense values, attribute 0 first), so that the queries
// sharing a tile's wave tend to match the same runs of rows and the exact
// main pass skips the row chunks none of them can match.  Any order gives
// the same results.  The key holds one field per dense attribute, attribute 0
// most significant: the value where the query constrains the attribute, else
// one past every value; a counting sort over its top kQordBits bits (one
// workgroup, LDS histogram; the order inside a bucket is arbitrary).
constexpr int kQordT = 1024;
constexpr int kQordBits = 13;

__device__ inline uint32_t qorder_key(const QDesc &d, const Schema &sch, int32_t shift) {
    uint64_t k = 0;
    for (int a = 0; a < sch.n_dense; a++) {
        const uint32_t fb = (uint32_t)sch.field_bits[a];
        const uint32_t fm = (uint32_t)((1ull << fb) - 1ull);
        const uint32_t f = (d.dmask >> sch.field_shift[a]) & fm ? (d.dval >> sch.field_shift[a]) & fm : fm + 1u;
        k = (k << (fb + 1)) | f;   // (at most 40 bits: fields of at most 32 bits, 8 attributes)
    }
    return (uint32_t)(k >> shift);
}

__global__ __launch_bounds__(kQordT) void k_qorder(const QDesc *__restrict__ qd, int32_t nq, Schema sch,
                                                   int32_t shift, int32_t nk, int32_t *__restrict__ qord) {
    extern __shared__ int32_t cnt[];   // nk buckets
    __shared__ int32_t part[kQordT];
    const int t = threadIdx.x;
    for (int32_t i = t; i < nk; i += kQordT) cnt[i] = 0;
    __syncthreads();
    for (int32_t q = t; q < nq; q += kQordT) atomicAdd(&cnt[qorder_key(qd[q], sch, shift)], 1);
    __syncthreads();
    // exclusive prefix over the buckets: thread t sums its run of buckets,
    // a scan over the threads, then each run is written out
    const int32_t per = (nk + kQordT - 1) / kQordT, b0 = t * per, b1 = min(nk, b0 + per);
    int32_t sum = 0;
    for (int32_t i = b0; i < b1; i++) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < kQordT; o <<= 1) {
        const int32_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
    for (int32_t i = b0; i < b1; i++) {
        const int32_t c = cnt[i];
        cnt[i] = run;
        run += c;
    }
    __syncthreads();
    for (int32_t q = t; q < nq; q += kQordT) qord[atomicAdd(&cnt[qorder_key(qd[q], sch, shift)], 1)] = q;
}

__global__ __launch_bounds__(kBucketT) void k_bucket_hist(const int32_t *__restrict__ probes,
                                                          const uint32_t *__restrict__ sel,
                                                          const int32_t *__restrict__ qord, int32_t nq, int32_t m,
                                                          int32_t r0, int32_t r1, int32_t b, int32_t ngrp,
                                                          int32_t *__restrict__ hist) {
    const int g = xcd_tile(blockIdx.x, ngrp);   // query group (consecutive groups on one XCD)
    if (g < 0) return;
    extern __shared__ int32_t cnt[];
    for (int i = threadIdx.x; i < b; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int32_t q0 = g * kBucketQ, q1 = min(nq, q0 + kBucketQ);
    bucket_slots(probes, sel, qord, q0, q1, m, r0, r1,
                 [&](int64_t, uint32_t, int32_t p) { atomicAdd(&cnt[p], 1); });
    __syncthreads();
    for (int i = threadIdx.x; i < b; i += blockDim.x) hist[(int64_t)i * ngrp + g] = cnt[i];
}

__global__ __launch_bounds__(kBucketT) void k_bucket_fill(const int32_t *__restrict__ probes,
                                                          const uint32_t *__restrict__ sel,
                                                          const int32_t *__restrict__ qord, int32_t nq, int32_t m,
                                                          int32_t r0, int32_t r1, int32_t b, int32_t ngrp,
                                                          const int32_t *__restrict__ hscan, int32_t nc_pack,
                                                          int32_t *__restrict__ entries, uint32_t *__restrict__ esel) {
    // query group g: consecutive groups run on one XCD, so that the adjacent
    // runs they write into each partition's range share that XCD's L2 (runs
    // of neighbouring groups written from different L2s left every output
    // line partly written in several of them)
    const int g = xcd_tile(blockIdx.x, ngrp);
    if (g < 0) return;
    extern __shared__ int32_t run[];
    for (int i = threadIdx.x; i < b; i += blockDim.x) run[i] = hscan[(int64_t)i * ngrp + g];
    __syncthreads();
    const int32_t q0 = g * kBucketQ, q1 = min(nq, q0 + kBucketQ);
    // nc_pack > 1: the level-mask class rides in bits 27.. for k_class_sort
    // esel (if given): the entry's level mask at the same position
    bucket_slots(probes, sel, qord, q0, q1, m, r0, r1, [&](int64_t e, uint32_t sm, int32_t p) {
        const int32_t at = atomicAdd(&run[p], 1);
        entries[at] = (int32_t)e | (nc_pack > 1 ? (int32_t)(sm & (uint32_t)(nc_pack - 1)) << kClassShift : 0);
        if (esel) esel[at] = sm;
    });
}

// One workgroup per partition: copies its entries from `in` to `out` grouped
// by level-mask class (in their order within a class).  The class is packed
// above bit kClassShift of each entry (packed != 0) or read from `sel`.
// With esel_out, each entry's class (its whole level mask: nc = 2^(h+1)) is
// written beside it.
// Counts and ranks come from one ballot per class and 64 entries.
constexpr int kClassW = 8;   // waves per class-sort block

__global__ __launch_bounds__(kClassW * 64) void k_class_sort(const int32_t *__restrict__ in,
                                                             const uint32_t *__restrict__ sel,
                                                             const int32_t *__restrict__ pstart,
                                                             const int32_t *__restrict__ pcount, int32_t nc,
                                                             int32_t packed, int32_t *__restrict__ out,
                                                             uint32_t *__restrict__ esel_out) {
    __shared__ int32_t wcnt[kClassW][16];
    const int32_t p = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int32_t ps = pstart[p], pn = pcount[p];
    const int32_t emask = (1 << kClassShift) - 1;
    auto cls_of = [&](int32_t v) {
        return packed ? (v >> kClassShift) & (nc - 1) : (int32_t)(sel[v] & (uint32_t)(nc - 1));
    };
    // pass 1: per wave and class, its entries (wave w takes a contiguous run
    // of 64-entry blocks, so that a class keeps the order of the fill)
    const int32_t nblk = (pn + 63) / 64, bpw = (nblk + kClassW - 1) / kClassW;
    const int32_t e0 = min(pn, w * bpw * 64), e1 = min(pn, (w + 1) * bpw * 64);
    int32_t cnt = 0;   // lane c < nc: this wave's count of class c
    for (int32_t i0 = e0; i0 < e1; i0 += 64) {
        const int32_t i = i0 + lane;
        const int32_t c = i < e1 ? cls_of(in[ps + i]) : -1;
        for (int k = 0; k < nc; k++) {
            const int32_t n = __popcll(__ballot(c == k));
            if (lane == k) cnt += n;
        }
    }
    if (lane < 16) wcnt[w][lane] = lane < nc ? cnt : 0;
    __syncthreads();
    // base of (wave w, class c): entries of smaller classes, then of the
    // same class in waves before w
    int32_t base = 0;
    if (lane < nc) {
        for (int k = 0; k < lane; k++)
            for (int v = 0; v < kClassW; v++) base += wcnt[v][k];
        for (int v = 0; v < w; v++) base += wcnt[v][lane];
    }
    // pass 2: place
    const uint64_t lt = lanemask_lt();
    for (int32_t i0 = e0; i0 < e1; i0 += 64) {
        const int32_t i = i0 + lane;
        const int32_t v = i < e1 ? in[ps + i] : 0;
        const int32_t c = i < e1 ? cls_of(v) : -1;
        for (int k = 0; k < nc; k++) {
            const uint64_t bk = __ballot(c == k);
            const int32_t bk0 = __shfl(base, k, 64);
            if (c == k) {
                const int32_t at = ps + bk0 + __popcll(bk & lt);
                out[at] = packed ? v & emask : v;
                if (esel_out) esel_out[at] = (uint32_t)k;
            }
            if (lane == k) base += __popcll(bk);
        }
    }
}

// Seed bound: the keep-th best key over a query's first s probes (any keep
// valid candidates bound the final keep-th key from above).  One wave per
// query; ~0 when fewer than keep candidates were found.
constexpr int kSeedCap = 256;

__global__ __launch_bounds__(256) void k_seed_tau(const uint64_t *__restrict__ partials,
                                                  const int32_t *__restrict__ pcnt,
                                                  const uint32_t *__restrict__ sel, int32_t nq, int32_t m,
                                                  int32_t s, int32_t slot_len, int32_t keep,
                                                  uint64_t *__restrict__ tau) {
    __shared__ uint64_t pool_all[4][kSeedCap];
    __shared__ int32_t npool_all[4];
    const int wq = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qq = blockIdx.x * 4 + wq;
    if (qq >= nq) return;
    uint64_t *pool = pool_all[wq];
    int32_t *npool = &npool_all[wq];
    (void)gather_best<kSeedCap>(pool, npool, partials, pcnt, sel, nullptr, (int64_t)qq * m, 0, s, slot_len, keep);
    if (lane == 0 && *npool == keep && pool[keep - 1] < tau[qq]) tau[qq] = pool[keep - 1];
}

// Seed bound for exact keys from an approximate scan of a query's first s
// probes: the keep (<= 64) best approximate candidates are rescored exactly;
// being valid candidates, their k-th best exact key bounds the final k-th key
// from above, and the bound is one past it (~0 when fewer than k).  One wave
// per query.
__global__ __launch_bounds__(256) void k_seed_exact(const uint64_t *__restrict__ partials,
                                                    const int32_t *__restrict__ pcnt,
                                                    const uint32_t *__restrict__ sel, int32_t nq, int32_t m,
                                                    int32_t s, int32_t slot_len, int32_t keep, int32_t k,
                                                    const float *__restrict__ vecs, const float *__restrict__ q,
                                                    const int32_t *__restrict__ perm, int32_t d, int32_t metric,
                                                    uint64_t *__restrict__ tau) {
    __shared__ uint64_t pool_all[4][kSeedCap];
    __shared__ int32_t npool_all[4];
    const int wq = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qq = blockIdx.x * 4 + wq;
    if (qq >= nq) return;
    uint64_t *pool = pool_all[wq];
    int32_t *npool = &npool_all[wq];
    (void)gather_best<kSeedCap>(pool, npool, partials, pcnt, sel, nullptr, (int64_t)qq * m, 0, s, slot_len, keep);
    const int n = *npool;
    uint64_t key = ~0ull;
    if (lane < n) {   // approximate keys carry CSR positions
        const uint32_t pos = (uint32_t)pool[lane];
        const float sc = exact_score<8>(vecs + (int64_t)pos * d, q + (int64_t)qq * d, d, metric == 0);
        key = ((uint64_t)f2ord(sc) << 32) | (uint32_t)perm[pos];
    }
    int rank = 0;   // among the wave's exact keys (distinct ids)
    for (int i = 0; i < n; i++) rank += readlane_u64(key, i) < key ? 1 : 0;
    const uint64_t at = __ballot(lane < n && rank == k - 1);
    // (the bound admits keys below it; that k-th key is itself a candidate
    // of the exact pass, which covers the seed probes too: one past it)
    if (lane == 0) tau[qq] = at ? readlane_u64(key, __builtin_ctzll(at)) + 1 : ~0ull;
}

// Bucket starts, sizes and tile starts per partition (single workgroup).
__global__ __launch_bounds__(1024) void k_plan(const int32_t *__restrict__ hscan, const int32_t *__restrict__ total,
                                               int32_t b, int32_t ngrp, int32_t qb, int32_t *__restrict__ pstart,
                                               int32_t *__restrict__ pcount, int32_t *__restrict__ tstart) {
    __shared__ int scratch[1024 / kWave + 1];
    __shared__ int carry_t;
    if (threadIdx.x == 0) carry_t = 0;
    __syncthreads();
    for (int b0 = 0; b0 < b; b0 += 1024) {
        const int p = b0 + threadIdx.x;
        int c = 0;
        if (p < b) {
            const int32_t s0 = hscan[(int64_t)p * ngrp];
            const int32_t s1 = p + 1 < b ? hscan[(int64_t)(p + 1) * ngrp] : *total;
            pstart[p] = s0;
            pcount[p] = s1 - s0;
            c = s1 - s0;
        }
        int tt;
        const int pt = block_excl_scan<1024>((c + qb - 1) / qb, scratch, &tt);
        if (p < b) tstart[p] = carry_t + pt;
        __syncthreads();
        if (threadIdx.x == 0) carry_t += tt;
        __syncthreads();
    }
    if (threadIdx.x == 0) tstart[b] = carry_t;
}

// Tile table for the scans: tile t < tstart[b] holds partition p with
// tstart[p] <= t < tstart[p + 1] and its entries i0.., i0 = (t - tstart[p])
// qb, up to qb of them; tiles past tstart[b] (up to the grid's range) hold
// none.  One thread per tile.
__global__ __launch_bounds__(256) void k_tile_desc(const int32_t *__restrict__ tstart,
                                                   const int32_t *__restrict__ pstart,
                                                   const int32_t *__restrict__ pcount, int32_t b, int32_t qb,
                                                   int32_t ntiles, int4 *__restrict__ tiles) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int4 dsc = make_int4(0, 0, 0, 0);
    if (t < tstart[b]) {
        int lo = 0, hi = b;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tstart[mid] <= t) lo = mid;
            else hi = mid;
        }
        const int i0 = (t - tstart[lo]) * qb;
        dsc = make_int4(lo, pstart[lo] + i0, min(qb, pcount[lo] - i0), 0);
    }
    tiles[t] = dsc;
}

// Clears the rescue list's length (rcount[0]) and records in rcount[1]
// whether any query of the sub-batch is flagged, so that the tile listing
// ends at once when none is.  One workgroup.
__global__ __launch_bounds__(1024) void k_rescue_init(const int32_t *__restrict__ oflow, int32_t nq,
                                                      int32_t *__restrict__ rcount) {
    int any = 0;
    for (int i = threadIdx.x; i < nq; i += blockDim.x) any |= oflow[i];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) {
        rcount[0] = 0;
        rcount[1] = any != 0;
    }
}

// Tiles of the exact main pass that hold a flagged query: listed (in any
// order) for the rescue pass, whose tiles hold up to `qr` entries.  Main-pass
// tiles of 2 qr entries are listed by half (entry 2 t + half).  One thread
// per tile.
__global__ __launch_bounds__(256) void k_rescue_tiles(const int4 *__restrict__ tiles, int32_t ntiles,
                                                      const int32_t *__restrict__ entries, int32_t m,
                                                      const int32_t *__restrict__ oflow, int32_t qr, int32_t halves,
                                                      int32_t *__restrict__ rlist, int32_t *__restrict__ rcount) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles || rcount[1] == 0) return;
    const int4 dsc = tiles[t];
    for (int hf = 0; hf <= halves; hf++) {
        const int i0 = hf * qr, i1 = halves ? min(dsc.z, i0 + qr) : dsc.z;
        bool hit = false;
        for (int i = i0; i < i1 && !hit; i++) hit = oflow[entries[dsc.y + i] / m] != 0;
        if (hit) rlist[atomicAdd(rcount, 1)] = halves ? 2 * t + hf : t;
    }
}

// ------------------------------------------------------------------ scan
struct ScanArgs {
    const int4 *tiles;     // per tile: partition, first entry, entries (0: no tile)
    int32_t ntiles;        // length of `tiles` (the grid's tile range)
    const int32_t *entries;
    const uint32_t *sel;
    const float *q;
    const QDesc *qd;
    const QDesc *qterms;   // disjunctive searches: kMaxTerms term descriptors per query
    const int32_t *offs, *perm;
    const float *vecs;
    const uint32_t *words;
    const uint64_t *sigs;
    const uint16_t *slots;
    int32_t lslots;       // label slots per point (rows wider than kMaxLabels are read from global memory)
    uint64_t *partials;
    uint64_t *tau;        // per query: shared upper bound on its final k-th key
    int32_t *nsurv;
    int32_t d, m, h, b, k;
};

constexpr int kCH = 64;        // points per chunk (one per lane in the filter)
constexpr int kQPW = 16;       // queries owned by each wave
constexpr int kRing = 128;     // per-wave pending-pair ring

// Per-tile LDS layout: QB = NW * 16 queries, one chunk of kCH points, and a
// candidate buffer of 2*KMAX keys per query.
struct ScanLds {
    size_t qs, xs, xid, xw, xsig, xslot, ring, buf, bcnt, tau, qslot, qd, total;
    int stride;
    __host__ __device__ ScanLds(int d, int nw, int kmax) {
        const int qb = nw * kQPW;
        stride = ((d + 3) & ~3) + 4;
        size_t o = 0;
        auto take = [&](size_t bytes) __host__ __device__ {
            o = (o + 15) & ~(size_t)15;
            size_t r = o;
            o += bytes;
            return r;
        };
        bcnt = take(sizeof(int32_t) * qb);
        tau = take(sizeof(uint64_t) * qb);
        qslot = take(sizeof(int32_t) * qb);
        qd = take(sizeof(QDesc) * qb);
        xid = take(sizeof(int32_t) * kCH);
        xw = take(sizeof(uint32_t) * kCH);
        xsig = take(sizeof(uint64_t) * kCH);
        xslot = take(sizeof(uint16_t) * kCH * kMaxLabels);
        ring = take(sizeof(uint16_t) * (size_t)nw * kRing);
        buf = take(sizeof(uint64_t) * (size_t)qb * 2 * kmax);
        xs = take(sizeof(float) * (size_t)kCH * stride);
        qs = take(sizeof(float) * (size_t)qb * stride);
        total = take(16);
    }
};

// Issues the global loads of one chunk (rows c0.. of sub-partition j) into
// registers; they land in LDS after the next workgroup barrier.  Every load
// is issued on every path (rows past the chunk's end load its last row, every
// thread loads its point's id and word, `wsrc` stands in for absent words),
// so the compiler counts the loads in flight exactly and nothing waits for
// them before their consumers at the top of the next chunk.
template <int XU, bool HAS_LABELS, int NT>
__device__ __attribute__((always_inline)) inline void fetch_chunk(
    const ScanArgs &A, const int32_t *po, int j, int32_t c0, int d, int t, const uint32_t *wsrc,
    const int (&prow)[XU ? XU : 1], const int (&pcol)[XU ? XU : 1],
    float __attribute__((ext_vector_type(4 * (XU ? XU : 1)))) & px, int32_t &pid, uint32_t &pw, uint64_t &psig,
    uint4 &pslot) {
    const int cn = min(kCH, po[j + 1] - c0);
    if (XU) {
        const int d4 = d >> 2;
        const float4 *src = reinterpret_cast<const float4 *>(A.vecs + (int64_t)c0 * d);
#pragma unroll
        for (int u = 0; u < XU; u++) {
            const float4 v = src[min(prow[u], cn - 1) * d4 + pcol[u]];
            px[4 * u + 0] = v.x;
            px[4 * u + 1] = v.y;
            px[4 * u + 2] = v.z;
            px[4 * u + 3] = v.w;
        }
    }
    const int32_t r = c0 + min(t & (kCH - 1), cn - 1);
    pid = A.perm[r];
    pw = wsrc[r];
    if (HAS_LABELS) {
        psig = A.sigs[r];
        pslot = *reinterpret_cast<const uint4 *>(A.slots + (int64_t)r * A.lslots);   // (narrow rows only used)
    }
}

// Partition-major filtered scan.  One workgroup = one tile (a partition and
// up to QB of the queries probing it); wave w owns queries 16w..16w+15 and
// does their filtering, survivor compaction, distances and candidate
// selection with no workgroup barrier beyond the two per chunk.  Chunks of
// 64 points of the chosen sub-partitions go through LDS (the next chunk is
// prefetched into registers); survivors go to a per-wave ring of (query,
// point) pairs and are scanned one pair per lane, dimensions in ascending
// order.  A survivor enters its query's buffer only if it beats the query's
// threshold: the smaller of the tile's own k-th key and the shared bound
// published by finished tiles (any k valid points bound the final k-th key
// from above, so no member of the exact top-k is ever dropped).
//
// XU: float4 loads per thread and chunk (XU * NT >= 64 * d / 4), or 0 for
// rows whose length is not a multiple of 4 (scalar staging).
template <int METRIC, bool HAS_LABELS, int XU, int KMAX, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_scan_fp32(ScanArgs A) {
    constexpr bool VEC4 = XU > 0;
    constexpr int QB = NW * kQPW;
    constexpr int NT = NW * 64;
    constexpr int C = 2 * KMAX;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t lvmask_w[NW];
    __shared__ int32_t spo[kMaxHeight + 2];
    const int tile = xcd_tile(blockIdx.x, A.ntiles);
    if (tile < 0) return;
    const int4 dsc = A.tiles[tile];
    if (dsc.z <= 0) return;
    const int p = dsc.x;
    const int nqt = dsc.z;
    const int32_t *ent = A.entries + dsc.y;

    const int d = A.d, k = A.k, h = A.h;
    const ScanLds L(d, NW, KMAX);
    const int stride = L.stride;
    float *Qs = reinterpret_cast<float *>(smem + L.qs);
    float *Xs = reinterpret_cast<float *>(smem + L.xs);
    int32_t *xid = reinterpret_cast<int32_t *>(smem + L.xid);
    uint32_t *xw = reinterpret_cast<uint32_t *>(smem + L.xw);
    uint64_t *xsig = reinterpret_cast<uint64_t *>(smem + L.xsig);
    uint16_t *xslot = reinterpret_cast<uint16_t *>(smem + L.xslot);
    uint16_t *ring_all = reinterpret_cast<uint16_t *>(smem + L.ring);
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem + L.buf);
    int32_t *bcnt = reinterpret_cast<int32_t *>(smem + L.bcnt);
    uint64_t *tau = reinterpret_cast<uint64_t *>(smem + L.tau);
    int32_t *qslot = reinterpret_cast<int32_t *>(smem + L.qslot);
    QDesc *qds = reinterpret_cast<QDesc *>(smem + L.qd);

    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const bool has_dense = A.words != nullptr;
    const int qbase = w * kQPW;
    if (t <= h + 1) spo[t] = A.offs[(int64_t)p * (h + 1) + t];
    // per-query state; lane i < 16 of wave w keeps query qbase+i in registers
    uint32_t my_sel = 0, my_dmask = 0, my_dval = 0;
    int my_surv = 0;
    int32_t my_qq = -1;
    if (lane < kQPW && qbase + lane < nqt) {
        const int qi = qbase + lane;
        const int32_t slot = ent[qi];
        my_qq = slot / A.m;
        my_sel = A.sel[slot];
        const QDesc qd = A.qd[my_qq];
        my_dmask = qd.dmask;
        my_dval = qd.dval;
        qslot[qi] = slot;
        qds[qi] = qd;
        tau[qi] = __hip_atomic_load(A.tau + my_qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bcnt[qi] = 0;
    }
    {
        uint32_t wor = my_sel;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wor |= __shfl_xor(wor, o, 64);
        if (lane == 0) lvmask_w[w] = wor;
    }
    const int d4 = VEC4 ? (d >> 2) : d;
    for (int r = w; r < nqt; r += NW) {
        const int64_t qrow = (int64_t)(ent[r] / A.m) * d;
        for (int c = lane; c < d4; c += 64) {
            if (VEC4)
                *reinterpret_cast<float4 *>(Qs + r * stride + 4 * c) =
                    *reinterpret_cast<const float4 *>(A.q + qrow + 4 * c);
            else
                Qs[r * stride + c] = A.q[qrow + c];
        }
    }
    __syncthreads();
    uint32_t lv = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) lv |= lvmask_w[i];
    uint16_t *ring = ring_all + w * kRing;

    // chunk cursor over the chosen sub-partitions of partition p
    const int32_t *po = spo;
    auto advance = [&](int &j, int32_t &c0) {
        c0 += kCH;
        while (j <= h && (!(lv & (1u << j)) || c0 >= po[j + 1])) {
            j++;
            if (j <= h) c0 = po[j];
        }
    };
    int cj = -1;
    int32_t cc0 = 0;
    {
        cj = 0;
        cc0 = po[0] - kCH;
        advance(cj, cc0);
    }
    // register prefetch of one chunk: float4 number e of a chunk is row
    // e / d4 (rows are contiguous in the CSR vectors)
    float __attribute__((ext_vector_type(4 * (XU ? XU : 1)))) px = {};
    int prow[XU ? XU : 1], pcol[XU ? XU : 1], plds[XU ? XU : 1];
    if (VEC4) {
#pragma unroll
        for (int u = 0; u < XU; u++) {
            const int e = t + u * NT;
            prow[u] = e / d4;
            pcol[u] = e - prow[u] * d4;
            plds[u] = prow[u] * stride + 4 * pcol[u];
        }
    }
    const uint32_t *wsrc = has_dense ? A.words : reinterpret_cast<const uint32_t *>(A.perm);
    int32_t pid = 0;
    uint32_t pw = 0;
    uint64_t psig = 0;
    uint4 pslot = make_uint4(0, 0, 0, 0);
    if (cj <= h) fetch_chunk<XU, HAS_LABELS, NT>(A, po, cj, cc0, d, t, wsrc, prow, pcol, px, pid, pw, psig, pslot);

    uint64_t g_next = ~0ull;
    while (cj <= h) {
        const int j = cj;
        const int32_t c0 = cc0;
        const int cn = min(kCH, po[j + 1] - c0);
        __syncthreads();   // the previous chunk is no longer read
        if (VEC4) {
#pragma unroll
            for (int u = 0; u < XU; u++)
                if (prow[u] < cn)
                    *reinterpret_cast<float4 *>(Xs + plds[u]) =
                        make_float4(px[4 * u], px[4 * u + 1], px[4 * u + 2], px[4 * u + 3]);
        } else {
            for (int e = t; e < cn * d; e += NT) {
                const int r = e / d, c = e - r * d;
                Xs[r * stride + c] = A.vecs[(int64_t)(c0 + r) * d + c];
            }
        }
        if (t < cn) {
            xid[t] = pid;
            xw[t] = has_dense ? pw : 0u;
            if (HAS_LABELS) {
                xsig[t] = psig;
                *reinterpret_cast<uint4 *>(xslot + t * kMaxLabels) = pslot;
            }
        }
        advance(cj, cc0);
        // (the last chunk fetches itself again: the loads are unconditional)
        const bool more = cj <= h;
        fetch_chunk<XU, HAS_LABELS, NT>(A, po, more ? cj : j, more ? cc0 : c0, d, t, wsrc, prow, pcol, px, pid, pw,
                                        psig, pslot);
        // refresh the shared bounds of my queries with the value loaded one
        // chunk ago, and start the next load (its latency overlaps a chunk)
        if (my_qq >= 0 && g_next < tau[qbase + lane]) tau[qbase + lane] = g_next;
        g_next = __hip_atomic_load(A.tau + max(my_qq, 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();

        // ---- wave-local: filter my queries against the chunk
        const bool lane_ok = lane < cn;
        const uint32_t myw = (has_dense && lane_ok) ? xw[lane] : 0u;
        const uint64_t mysig = (HAS_LABELS && lane_ok) ? xsig[lane] : 0ull;
        int pend = 0, head = 0;   // wave-uniform
        auto process = [&](int n) {
            wave_sync();   // ring entries written by this wave are visible
            const bool v = lane < n;
            const uint16_t en = v ? ring[(head + lane) & (kRing - 1)] : (uint16_t)0;
            const int qi = qbase + (en >> 6);
            const int pi = en & 63;
            uint64_t key = ~0ull;
            if (v) {
                const float *xr = Xs + pi * stride;
                const float *qr = Qs + qi * stride;
                float acc = 0.0f;
                if (VEC4) {
#pragma unroll 8
                    for (int jj = 0; jj < d; jj += 4) {
                        const float4 xv = *reinterpret_cast<const float4 *>(xr + jj);
                        const float4 qv = *reinterpret_cast<const float4 *>(qr + jj);
                        if (METRIC == 0) {
                            float t0 = xv.x - qv.x;
                            acc = fmaf(t0, t0, acc);
                            t0 = xv.y - qv.y;
                            acc = fmaf(t0, t0, acc);
                            t0 = xv.z - qv.z;
                            acc = fmaf(t0, t0, acc);
                            t0 = xv.w - qv.w;
                            acc = fmaf(t0, t0, acc);
                        } else {
                            acc = fmaf(xv.x, qv.x, acc);
                            acc = fmaf(xv.y, qv.y, acc);
                            acc = fmaf(xv.z, qv.z, acc);
                            acc = fmaf(xv.w, qv.w, acc);
                        }
                    }
                } else {
                    for (int jj = 0; jj < d; jj++) {
                        if (METRIC == 0) {
                            const float t0 = xr[jj] - qr[jj];
                            acc = fmaf(t0, t0, acc);
                        } else {
                            acc = fmaf(xr[jj], qr[jj], acc);
                        }
                    }
                }
                const float kf = canon0(METRIC == 0 ? acc : -acc);
                key = ((uint64_t)f2ord(kf) << 32) | (uint32_t)xid[pi];
            }
            // append the qualifying keys to their queries' buffers; the wave
            // owns these queries, so slots come from ballots, not atomics.
            // Each step appends at least one key or empties a full buffer
            // down to k entries, so 2 * 64 + 2 steps always suffice.
            bool qual = v && key < tau[qi];
            for (int guard = 0; guard < 2 * 64 + 2; guard++) {
                const uint64_t todo = __ballot(qual);
                if (!todo) break;
                const int q = __builtin_amdgcn_readlane(qi, __builtin_ctzll(todo));
                const uint64_t grp = __ballot(qual && qi == q);
                const int c = bcnt[q];
                const int room = C - c;
                if (room <= 0) {
                    wave_sync();
                    buf_reduce<C>(buf, bcnt, tau, q, k);
                    if (qual && qi == q) qual = key < tau[q];
                    continue;
                }
                uint64_t take = grp;
                while (__popcll(take) > room) take &= ~(1ull << (63 - __builtin_clzll(take)));
                const bool mine = (take >> lane) & 1ull;
                if (mine) {
                    buf[q * C + c + __popcll(take & lanemask_lt())] = key;
                    qual = false;
                }
                wave_sync();
                if (lane == 0) bcnt[q] = c + __popcll(take);
                wave_sync();
            }
            wave_sync();
            head += n;
        };
        for (int i = 0; i < kQPW; i++) {
            const uint32_t sl = __builtin_amdgcn_readlane(my_sel, i);
            if (!(sl & (1u << j))) continue;
            bool pass;
            if (HAS_LABELS || (qds[qbase + i].flags & kQOr)) {
                const QDesc *terms = A.qterms + (int64_t)(qslot[qbase + i] / A.m) * kMaxTerms;
                const bool wide = A.lslots > kMaxLabels;
                const uint16_t *sl = wide ? A.slots + (int64_t)(c0 + min(lane, cn - 1)) * A.lslots
                                          : xslot + lane * kMaxLabels;
                pass = lane_ok && query_passes(qds[qbase + i], terms, has_dense, HAS_LABELS, myw, mysig, sl,
                                               A.lslots);
            } else {
                const uint32_t dm = __builtin_amdgcn_readlane(my_dmask, i);
                const uint32_t dv = __builtin_amdgcn_readlane(my_dval, i);
                pass = lane_ok && ((myw & dm) == dv);
            }
            const uint64_t mask = __ballot(pass);
            if (!mask) continue;
            const int cnt = __popcll(mask);
            if (pass) ring[(head + pend + __popcll(mask & lanemask_lt())) & (kRing - 1)] =
                          (uint16_t)((i << 6) | lane);
            if (lane == i) my_surv += cnt;
            pend += cnt;
            if (pend >= 64) {
                process(64);
                pend -= 64;
            }
        }
        if (pend > 0) process(pend);
    }
    // ---- finalize my queries: best k sorted, partial list, shared bound,
    // survivor count
    for (int i = 0; i < kQPW; i++) {
        const int qi = qbase + i;
        if (qi >= nqt) break;
        buf_reduce<C>(buf, bcnt, tau, qi, k);
        const int c = bcnt[qi];
        uint64_t *out = A.partials + (int64_t)qslot[qi] * k;
        if (lane < k) out[lane] = lane < c ? buf[qi * C + lane] : ~0ull;
        const int32_t qq = qslot[qi] / A.m;
        if (lane == 0 && c == k)
            atomicMin((unsigned long long *)(A.tau + qq), (unsigned long long)buf[qi * C + k - 1]);
    }
    if (my_qq >= 0 && my_surv) atomicAdd(&A.nsurv[my_qq], my_surv);
}

static int scan_waves(int k) { return k <= 16 ? 8 : 4; }

static size_t scan_lds_bytes(int d, int k) {
    return ScanLds(d, scan_waves(k), k <= 16 ? 16 : 64).total + 64;
}

// ------------------------------------------------------------------ merge
// Deferred pairs of the exact matrix-core scan per query: (ordered score of
// the scan's element test << 32) | CSR position, rescored here with the plain
// scan's arithmetic.
struct Deferred {
    const uint64_t *pos;        // null: none
    const int32_t *cnt;
    const int32_t *oflow;       // queries rescanned by the rescue pass: deferred pairs ignored, partial lists read
    int32_t cap, d;
    const float *vecs, *q;      // FP32 CSR rows, the sub-batch's queries
    const int32_t *perm;
    const float *qaux;          // the scan's per-query terms (|q|^2 lower bound at 4 q + 1)
    float eta;                  // the scan's rounding margin
};

// Deferred pairs kept per query by the exact matrix-core scan (a query with
// more goes to the rescue pass).
constexpr int32_t kDeferCap = 512;
// Pairs rescored first (those with the smallest test scores): k and half
// again, at least 16, at most 64 (one per lane).
__device__ inline int merge_first(int k) { return min(64, max(16, k + (k >> 1))); }

template <int KM>
__global__ __launch_bounds__(256) void k_merge(const uint64_t *__restrict__ partials,
                                               const int32_t *__restrict__ pcnt,
                                               const uint32_t *__restrict__ sel, const int32_t *__restrict__ cand,
                                               int32_t nq, int32_t m, int32_t k, int32_t metric,
                                               int32_t *__restrict__ ids, float *__restrict__ dist,
                                               int32_t *__restrict__ ncand, Deferred D) {
    __shared__ uint64_t mbuf[4][64], mkb[4][64];   // per wave: round 1's pairs and keys
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= nq) return;
    uint64_t lst[KM];
#pragma unroll
    for (int i = 0; i < KM; i++) lst[i] = ~0ull;
    auto insert = [&](uint64_t key) {
#pragma unroll
        for (int u = KM - 1; u > 0; u--) {
            const uint64_t a = lst[u - 1];
            lst[u] = key < a ? a : (key < lst[u] ? key : lst[u]);
        }
        lst[0] = key < lst[0] ? key : lst[0];
    };
    if (D.pos && !D.oflow[q]) {
        const int n = min(D.cnt[q], D.cap);
        const float *qr = D.q + (int64_t)q * D.d;
        const uint64_t *src = D.pos + (int64_t)q * D.cap;
        auto score = [&](uint64_t ent) {   // the pair's exact key
            const int32_t pos = (int32_t)(uint32_t)ent;
            const float sc = exact_score<8>(D.vecs + (int64_t)pos * D.d, qr, D.d, metric == 0);
            return ((uint64_t)f2ord(sc) << 32) | (uint32_t)D.perm[pos];
        };
        const int first = merge_first(k);
        if (n <= first) {
            for (int i = lane; i < n; i += 64) insert(score(src[i]));
        } else {
            // Two rounds.  The scan deferred a pair when its test score passed the
            // row bound of the query's seed key; the same test at any bound tau
            // fails only for pairs whose exact key is above tau.  Round 1
            // rescores the `first` pairs with the smallest test scores (more
            // where scores tie, at most 64); the k-th of their exact keys, K, is
            // at or above the final k-th key, so round 2 needs only the pairs
            // that pass the test at bound K.  (first >= k: K is finite.)
            constexpr int EP = kDeferCap / 64;
            uint64_t e[EP];   // pair lane + 64 j (~0: none)
#pragma unroll
            for (int j = 0; j < EP; j++) {
                const int i = j * 64 + lane;
                e[j] = i < n ? src[i] : ~0ull;
            }
            auto skey = [](uint64_t v) { return (uint32_t)(v >> 32); };   // (~0 never a valid score key)
            // T: the first-th smallest test score key (bisection over its
            // bits, stopped once the range holds a single key)
            uint32_t ans = 0;
            int c_lo = 0, c_hi = EP * 64;
            bool one = false;
            for (int bit = 31; bit >= 0; bit--) {
                const uint32_t t = ans | (1u << bit);
                int c = 0;
#pragma unroll
                for (int j = 0; j < EP; j++) c += __popcll(__ballot(skey(e[j]) < t));
                if (c < first) {
                    ans = t;
                    c_lo = c;
                } else {
                    c_hi = c;
                }
                if (c_hi - c_lo == 1) {
                    one = true;
                    break;
                }
            }
            uint32_t T = ans;
            if (one) {
                uint64_t mn = ~0ull;
#pragma unroll
                for (int j = 0; j < EP; j++)
                    if (skey(e[j]) >= ans && skey(e[j]) < mn) mn = skey(e[j]);
                T = (uint32_t)wave_min_u64(mn);
            }
            // round 1: the pairs below T, then those at T, up to 64, compacted
            uint64_t *buf = mbuf[threadIdx.x >> 6];
            const uint64_t lt = lanemask_lt();
            int n1 = 0;
#pragma unroll
            for (int j = 0; j < EP; j++) {
                const bool s = e[j] != ~0ull && skey(e[j]) < T;
                const uint64_t b = __ballot(s);
                if (s) {
                    buf[n1 + __popcll(b & lt)] = e[j];
                    e[j] = ~0ull;
                }
                n1 += __popcll(b);
            }
#pragma unroll
            for (int j = 0; j < EP; j++) {
                const bool s = e[j] != ~0ull && skey(e[j]) == T;
                const uint64_t b = __ballot(s);
                const int at = n1 + __popcll(b & lt);
                if (s && at < 64) {
                    buf[at] = e[j];
                    e[j] = ~0ull;
                }
                n1 = min(64, n1 + __popcll(b));
            }
            wave_sync();
            uint64_t k1 = ~0ull;
            if (lane < n1) {
                k1 = score(buf[lane]);
                insert(k1);
            }
            // K: the k-th smallest of round 1's keys (distinct: the ids differ)
            uint64_t *kb = mkb[threadIdx.x >> 6];
            kb[lane] = k1;
            wave_sync();
            int rank = 0;
            if (lane < n1)
                for (int i = 0; i < n1; i++) rank += kb[i] < k1 ? 1 : 0;
            const uint64_t kl = __ballot(lane < n1 && rank == k - 1);
            const uint64_t K = kl ? readlane_u64(k1, __builtin_ctzll(kl)) : ~0ull;
            // round 2: the row bound at K's score, as the scan computes it
            const float td = bound_score(K);
            const float nq = D.qaux[4 * (int64_t)q + 1];
            const float tf = !(td < __builtin_huge_valf()) ? __builtin_huge_valf()
                             : metric == 0                 ? fmaf(D.eta, nq + td, td - nq) + 1e-37f
                                                           : fmaf(D.eta, nq + fabsf(td), td) + 1e-37f;
#pragma unroll
            for (int j = 0; j < EP; j++)
                if (e[j] != ~0ull && ord2f(skey(e[j])) <= tf) insert(score(e[j]));
        }
    }
    // with deferred pairs the partial lists hold keys only for the queries the
    // rescue pass rescanned (the main pass writes none)
    const bool lists = !D.pos || D.oflow[q];
    int nc = 0;
    for (int r = lane; r < m; r += 64) {
        const int64_t slot = (int64_t)q * m + r;
        if (sel[slot] == 0) continue;
        nc += cand[slot];
        const uint64_t *src = partials + slot * k;
        const int c = !lists ? 0 : pcnt ? min(pcnt[slot], k) : k;   // else lists padded with ~0
        for (int i = 0; i < c; i++) {
            const uint64_t key = src[i];
            if (key >= lst[KM - 1]) break;   // lists are sorted: the rest is worse
            insert(key);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nc += __shfl_xor(nc, o, 64);
    if (lane == 0) ncand[q] = nc;
    for (int r = 0; r < k; r++) {
        const uint64_t best = wave_min_u64(lst[0]);
        if (lane == 0) {
            const int64_t o = (int64_t)q * k + r;
            if (best == ~0ull) {
                ids[o] = -1;
                dist[o] = metric == 0 ? __builtin_huge_valf() : -__builtin_huge_valf();
            } else {
                ids[o] = (int32_t)(uint32_t)(best & 0xFFFFFFFFu);
                const float key = ord2f((uint32_t)(best >> 32));
                dist[o] = metric == 0 ? key : canon0(-key);
            }
        }
        if (best != ~0ull && lst[0] == best) {
#pragma unroll
            for (int u = 0; u < KM - 1; u++) lst[u] = lst[u + 1];
            lst[KM - 1] = ~0ull;
        }
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void k_copy_i32(const int32_t *__restrict__ a, int32_t *__restrict__ b, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) b[e] = a[e];
}

// ------------------------------------------------------------------ host
typedef void (*ScanFn)(ScanArgs);

// Float4 loads per thread for a chunk of 64 rows of d coordinates: half the
// d = 256 count when d <= 128, else the full count; 0 = scalar staging.
static int scan_xu(int d, int k) {
    if (d % 4 != 0 || d > 256) return 0;
    const int full = 64 * 64 / (scan_waves(k) * 64);
    return d <= 128 ? full / 2 : full;
}

template <int METRIC, bool LAB>
static ScanFn pick_xu(int xu, int k) {
    if (k <= 16) {   // 8 waves: 8 float4 per thread at d = 256
        if (xu == 4) return k_scan_fp32<METRIC, LAB, 4, 16, 8>;
        if (xu == 8) return k_scan_fp32<METRIC, LAB, 8, 16, 8>;
        return k_scan_fp32<METRIC, LAB, 0, 16, 8>;
    }
    if (xu == 8) return k_scan_fp32<METRIC, LAB, 8, 64, 4>;   // 4 waves: 16 at d = 256
    if (xu == 16) return k_scan_fp32<METRIC, LAB, 16, 64, 4>;
    return k_scan_fp32<METRIC, LAB, 0, 64, 4>;
}

static ScanFn pick_scan(int metric, bool labels, int d, int k) {
    const int xu = scan_xu(d, k);
    if (metric == 0) return labels ? pick_xu<0, true>(xu, k) : pick_xu<0, false>(xu, k);
    return labels ? pick_xu<1, true>(xu, k) : pick_xu<1, false>(xu, k);
}

static unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Bump allocator over one workspace allocation.  With base == nullptr it
// only measures, so the same sequence of takes sizes the allocation; with a
// base it refuses to hand out bytes beyond `cap`.
struct Arena {
    char *base = nullptr;
    size_t off = 0, cap = 0;
    bool overflow = false;
    template <class T>
    T *take(size_t count) {
        const size_t a = (off + 255) & ~(size_t)255;
        const size_t bytes = sizeof(T) * (count ? count : 1);
        if (base && a + bytes > cap) {
            overflow = true;
            return nullptr;
        }
        off = a + bytes;
        return base ? reinterpret_cast<T *>(base + a) : nullptr;
    }
};

int lowp_qb();
int lowp_qb_main(const Index *ix, bool disj);
bool lowp_seed_x32(const Index *ix, bool disj, int r);

struct SearchWs {
    uint8_t *qlow;
    float *qscale, *qaux;
    int32_t *pcnt;
    int32_t *ncand, *nsurv;
    QDesc *qd;
    float *scores;
    int32_t *probes;
    uint32_t *sel;
    int32_t *cand, *entries, *entries2;   // entries2: class-grouped copy
    uint32_t *esel;             // exact matrix-core scan: level mask per entry of the scanned entry list
    uint64_t *partials, *tau;
    uint64_t *dpos;             // exact matrix-core scan: deferred pairs per query (score key, position)
    int32_t *dcnt;
    int32_t *oflow;             // exact matrix-core scan: queries for the rescue pass
    int32_t *rlist, *rcount;    // exact matrix-core scan: tiles for the rescue pass
    int32_t *hist, *hscan, *scan_sums, *htotal, *pcount, *pstart, *tstart;
    int4 *tiles;
    uint16_t *rx, *rh;          // learned routing: input rows, hidden activations
    float *rbn;                 // learned routing: the output bias, negated
    float *conf;                // learned routing: softmax top-1 probability
    int32_t *probes_c;          // learned routing: centroid probes of the falling-back queries
    int32_t *fbq, *nfb;         // learned routing: the queries that fall back, their count
    int32_t *bad;               // query rows holding NaN or Inf (one counter per call)
    int32_t *qord;              // bucketing order of the queries (grouped by constraint)
    QDesc *qterms;              // disjunctive searches: term descriptors (kMaxTerms per query)
};

// Tiles of one round at most: every (query, probe) entry in tiles of at
// least 64 entries, plus one partial tile per partition, rounded up to the
// XCD multiple of the grid.
static int64_t tile_cap(int64_t sb, int64_t m, int64_t b) { return (sb * m + 63) / 64 + b + kXcds; }


static void carve(Arena &ar, SearchWs &w, int32_t nq, int32_t sb, int32_t b, int32_t m, int32_t k,
                  bool own_ncand, bool own_nsurv, size_t qlow_row_bytes, const Router *router, bool defer,
                  int32_t nc, bool disj) {
    const int32_t ngrp_max = (sb + kBucketQ - 1) / kBucketQ;
    w.bad = ar.take<int32_t>(1);
    w.qterms = disj ? ar.take<QDesc>((size_t)sb * kMaxTerms) : nullptr;
    w.qlow = qlow_row_bytes ? ar.take<uint8_t>((size_t)sb * qlow_row_bytes) : nullptr;
    w.qscale = qlow_row_bytes ? ar.take<float>((size_t)sb) : nullptr;
    w.qaux = qlow_row_bytes ? ar.take<float>((size_t)sb * 4) : nullptr;
    w.pcnt = qlow_row_bytes ? ar.take<int32_t>((size_t)sb * m) : nullptr;
    w.ncand = own_ncand ? ar.take<int32_t>(nq) : nullptr;
    w.nsurv = own_nsurv ? ar.take<int32_t>(nq) : nullptr;
    w.qd = ar.take<QDesc>(sb);
    w.qord = ar.take<int32_t>(sb);
    w.scores = ar.take<float>((size_t)sb * b);
    w.probes = ar.take<int32_t>((size_t)sb * m);
    w.sel = ar.take<uint32_t>((size_t)sb * m);
    w.cand = ar.take<int32_t>((size_t)sb * m);
    w.entries = ar.take<int32_t>((size_t)sb * m);
    w.partials = ar.take<uint64_t>((size_t)sb * m * k);
    w.tau = ar.take<uint64_t>((size_t)sb);
    w.dpos = defer ? ar.take<uint64_t>((size_t)sb * kDeferCap) : nullptr;
    w.dcnt = defer ? ar.take<int32_t>((size_t)sb) : nullptr;
    w.oflow = defer ? ar.take<int32_t>((size_t)sb) : nullptr;
    // (main-pass tiles of 128 entries are listed by half: one more per partition)
    w.rlist = defer ? ar.take<int32_t>(tile_cap(sb, m, b) + b) : nullptr;
    w.rcount = defer ? ar.take<int32_t>(2) : nullptr;
    w.hist = ar.take<int32_t>((size_t)b * ngrp_max + 1);
    w.hscan = ar.take<int32_t>((size_t)b * ngrp_max + 1);
    w.scan_sums = ar.take<int32_t>((size_t)exclusive_scan_tiles((int64_t)b * ngrp_max) + 1);
    w.entries2 = nc > 1 ? ar.take<int32_t>((size_t)sb * m) : nullptr;
    w.esel = defer ? ar.take<uint32_t>((size_t)sb * m) : nullptr;
    w.htotal = ar.take<int32_t>(1);
    w.pcount = ar.take<int32_t>(b + 1);
    w.pstart = ar.take<int32_t>(b + 1);
    w.tstart = ar.take<int32_t>(b + 1);
    w.tiles = ar.take<int4>(tile_cap(sb, m, b));
    w.rx = router ? ar.take<uint16_t>((size_t)sb * router->dpad) : nullptr;
    w.rh = router ? ar.take<uint16_t>((size_t)sb * router->hid) : nullptr;
    w.rbn = router ? ar.take<float>((size_t)router->nout) : nullptr;
    w.conf = router ? ar.take<float>((size_t)sb) : nullptr;
    w.probes_c = router ? ar.take<int32_t>((size_t)sb * m) : nullptr;
    w.fbq = router ? ar.take<int32_t>((size_t)sb) : nullptr;
    w.nfb = router ? ar.take<int32_t>(1) : nullptr;
}

// Shape of one search call: which scan, keys per (query, probe), the
// sub-batch that keeps the workspace within the budget.
struct SearchPlan {
    bool lowp, mfma, defer;
    int32_t r, sb;
    size_t qlow_row;
    const Router *router;
};

static SearchPlan plan_search(const Index *ix, const caps_search_params *sp, int32_t nq, size_t budget) {
    const int32_t b = ix->b, m = sp->nprobe, k = sp->k;
    SearchPlan P;
    // mode 1: approximate keys on the matrix cores, rescored at the merge;
    // mode 0 on an index with a low-precision copy: the matrix-core scan
    // with exact keys (bounds prune, survivors are rescored exactly);
    // otherwise (or mode 2) the plain FP32 scan
    P.lowp = sp->mode == 1;
    P.mfma = P.lowp || (sp->mode == 0 && ix->prec != CAPS_PREC_NONE);
    P.defer = P.mfma && !P.lowp;
    P.r = P.lowp ? (sp->rerank > 0 ? sp->rerank : std::min(4 * k, kMaxK)) : k;
    P.router = sp->routing == 1 ? ix->router : nullptr;
    P.qlow_row = P.mfma ? (size_t)ix->dpad * (ix->prec == CAPS_PREC_FP8 ? 1 : 2) : 0;
    const size_t per_q = sizeof(float) * (size_t)b + sizeof(int32_t) * 5 * (size_t)m +
                         sizeof(uint64_t) * (size_t)m * P.r + sizeof(QDesc) + sizeof(uint64_t) +
                         2 * sizeof(int32_t) * (size_t)b / kBucketQ + P.qlow_row + 5 * sizeof(float) + 64 +
                         sizeof(int32_t) * (size_t)m +
                         (P.defer ? sizeof(int32_t) * (size_t)(kDeferCap + 2 + m / 64) : 0) +
                         sizeof(int4) * (size_t)m / 64 +
                         ((sp->flags & CAPS_SEARCH_DISJUNCTIVE) ? sizeof(QDesc) * kMaxTerms : 0) +
                         (P.router ? sizeof(uint16_t) * (size_t)(P.router->dpad + P.router->hid) + sizeof(float) +
                                         sizeof(int32_t) * (size_t)(m + 1)
                                   : 0);
    P.sb = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)std::max(nq, 1), budget / per_q));
    return P;
}

// default workspace budget of one call (of 288 GB): a 10k-query batch in
// one go in every mode
static size_t default_budget(const caps_search_params *sp) {
    return sp->workspace_bytes > 0 ? (size_t)sp->workspace_bytes : (size_t)4 << 30;
}

static size_t measure_ws(const Index *ix, const caps_search_params *sp, const SearchPlan &P, int32_t nq,
                         int32_t sb, bool own_ncand, bool own_nsurv) {
    SearchWs W;
    Arena measure;
    carve(measure, W, nq, sb, ix->b, sp->nprobe, P.r, own_ncand, own_nsurv, P.qlow_row, P.router, P.defer,
          bucket_classes(ix->h), (sp->flags & CAPS_SEARCH_DISJUNCTIVE) != 0);
    return measure.off;
}

size_t search_workspace_bytes(const Index *ix, const caps_search_params *sp, int32_t nq) {
    const SearchPlan P = plan_search(ix, sp, nq, default_budget(sp));
    return measure_ws(ix, sp, P, nq, P.sb, true, true);
}

// Non-finite query rows: flagged unsatisfiable (they choose no sub-partition,
// so their results are all padding) and counted.  One wave per query.
__global__ __launch_bounds__(256) void k_qcheck(const float *__restrict__ q, int32_t nq, int32_t d,
                                                QDesc *__restrict__ qd, int32_t *__restrict__ bad) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nq) return;
    bool ok = true;
    for (int j = lane; j < d; j += 64) ok &= __builtin_isfinite(q[i * d + j]);
    if (__ballot(!ok) != 0 && lane == 0) {
        qd[i].flags |= 2u;
        atomicAdd(bad, 1);
    }
}

// Survivor bits for the debug entry point: bit pos % 64 of word pos / 64 of
// a query's row is set when CSR position pos lies in a sub-partition its
// search chose and passes its filter.  One wave per (query, probe) slot.
__global__ __launch_bounds__(256) void k_surv_mask(const int32_t *__restrict__ probes, const uint32_t *__restrict__ sel,
                                                   int32_t nq, int32_t m, const QDesc *__restrict__ qd,
                                                   const QDesc *__restrict__ qterms,
                                                   const int32_t *__restrict__ offs, int32_t h,
                                                   const uint32_t *__restrict__ words, const uint64_t *__restrict__ sigs,
                                                   const uint16_t *__restrict__ slots, int32_t lslots,
                                                   uint64_t *__restrict__ mask, int64_t mask_words) {
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= (int64_t)nq * m) return;
    const uint32_t sm = sel[e];
    if (!sm) return;
    const int64_t qi = e / m;
    const int32_t p = probes[e];
    const QDesc Q = qd[qi];
    for (int j = 0; j <= h; j++) {
        if (!((sm >> j) & 1u)) continue;
        const int32_t lo = offs[(int64_t)p * (h + 1) + j], hi = offs[(int64_t)p * (h + 1) + j + 1];
        for (int32_t pos = lo + lane; pos < hi; pos += 64) {
            const bool pass = query_passes(Q, qterms + qi * kMaxTerms, words != nullptr, sigs != nullptr,
                                           words ? words[pos] : 0u, sigs ? sigs[pos] : 0ull,
                                           slots ? slots + (int64_t)pos * lslots : nullptr, lslots);
            if (pass) atomicOr((unsigned long long *)(mask + qi * mask_words + pos / 64), 1ull << (pos % 64));
        }
    }
}

caps_status search(const Index *ix, const caps_search_params *sp, const float *q, int32_t nq,
                   const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                   int32_t n_con, int32_t *out_ids, float *out_dist, int32_t *out_ncand,
                   int32_t *out_nsurv, int32_t *out_probes, uint32_t *out_masks, hipStream_t st,
                   const SearchExtra *extra) {
    const SearchExtra ex = extra ? *extra : SearchExtra{};
    const int32_t b = ix->b, d = ix->d, h = ix->h, m = sp->nprobe, k = sp->k;
    if (nq == 0) return CAPS_OK;
    // a caller workspace (no allocation) bounds the sub-batch: shrink it
    // until its layout fits
    const size_t budget = ex.ws ? ex.ws_bytes : default_budget(sp);
    SearchPlan P = plan_search(ix, sp, nq, budget);
    size_t need = measure_ws(ix, sp, P, nq, P.sb, !out_ncand, !out_nsurv);
    if (ex.ws) {
        while (need > ex.ws_bytes && P.sb > 1) {
            P.sb = std::max<int32_t>(1, (int32_t)((double)P.sb * (double)ex.ws_bytes / (double)need * 0.95));
            need = measure_ws(ix, sp, P, nq, P.sb, !out_ncand, !out_nsurv);
        }
        if (need > ex.ws_bytes) {
            set_error("caps_search: one query needs %zu bytes of workspace, more than the %zu available", need,
                      ex.ws_bytes);
            return CAPS_EUNSUPPORTED;
        }
    }
    const bool lowp = P.lowp, mfma = P.mfma;
    const int32_t r = P.r, sb = P.sb;
    const int32_t nc = bucket_classes(h);
    const size_t qlow_row = P.qlow_row;
    const Router *router = P.router;
    const bool probes_only = out_probes != nullptr;
    const bool disj = (sp->flags & CAPS_SEARCH_DISJUNCTIVE) != 0;
    const int64_t mask_words = (ix->n + 63) / 64;
    int pb = 1;
    while (pb < b) pb <<= 1;

    SearchWs W;
    Arena ar;
    ar.cap = need;
    if (ex.ws) {
        ar.base = reinterpret_cast<char *>(ex.ws);
    } else {
        const caps_status as = ws_alloc((void **)&ar.base, ar.cap, ix->device, st);
        if (as != CAPS_OK) return as;
    }
    carve(ar, W, nq, sb, b, m, r, !out_ncand, !out_nsurv, qlow_row, router, P.defer, nc, disj);

    // the search proper; every exit below goes through the release at the end
    auto run = [&]() -> caps_status {
    if (ar.overflow) {
        set_error("caps_search: internal workspace layout error");
        return CAPS_EDEVICE;
    }
    int32_t *ncand = out_ncand ? out_ncand : W.ncand;
    int32_t *nsurv = out_nsurv ? out_nsurv : W.nsurv;
    QDesc *qd = W.qd;
    float *scores = W.scores;
    int32_t *probes = W.probes;
    uint32_t *sel = W.sel;
    int32_t *cand = W.cand;
    int32_t *entries = W.entries;
    uint64_t *partials = W.partials;
    uint64_t *tau = W.tau;
    int32_t *hist = W.hist, *hscan = W.hscan, *htotal = W.htotal;
    int32_t *pcount = W.pcount, *pstart = W.pstart, *tstart = W.tstart;

    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, W.bad, (int64_t)1, 0);
    if (!probes_only) hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(nq, 256)), dim3(256), 0, st, nsurv, (int64_t)nq, 0);
    if (ex.surv_mask)
        hipLaunchKernelGGL(k_fill_u64, dim3(nblocks((int64_t)nq * mask_words, 256)), dim3(256), 0, st, ex.surv_mask,
                           (int64_t)nq * mask_words, 0ull);

    const bool has_labels = ix->sch.label_vocab > 0;
    const size_t lds = mfma ? lowp_scan_lds(ix, r, lowp ? 0 : 2, disj) : scan_lds_bytes(d, k);
    const int qb = mfma ? lowp_qb() : scan_waves(k) * kQPW;
    const ScanFn scan_fn = pick_scan(ix->metric, has_labels, d, k);
    if (!probes_only && !mfma) {
        int lds_max = 0;
        CAPS_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device));
        if (lds > (size_t)lds_max) {
            set_error("caps_search: d=%d, k=%d need %zu bytes of LDS per workgroup (limit %d)", d, k, lds,
                      lds_max);
            return CAPS_EUNSUPPORTED;
        }
        const caps_status ls = set_kernel_lds((const void *)scan_fn, lds, ix->device);
        if (ls != CAPS_OK) return ls;
    }
        for (int32_t q0 = 0; q0 < nq; q0 += sb) {
            const int32_t nb = std::min(sb, nq - q0);
            const int64_t pairs = (int64_t)nb * m;
            const int32_t ngrp = (nb + kBucketQ - 1) / kBucketQ;
            const int32_t s_seed = m >= 32 ? std::max(8, m / (P.defer ? 24 : 16)) : m;
            // the probes query returns them sorted; a search takes the best m as
            // a set with the s_seed best first
            const int32_t topm_s = probes_only ? -1 : s_seed;
            prof_begin(CAPS_STAGE_PREP, st);
            hipLaunchKernelGGL(k_qprep, dim3(nblocks(nb, 128)), dim3(128), 0, st, con_off + q0, con_attr,
                               con_val, n_con, nb, ix->sch, (int32_t)disj, qd, W.qterms);
            hipLaunchKernelGGL(k_qcheck, dim3(nblocks(nb, 4)), dim3(256), 0, st, q + (int64_t)q0 * d, nb, d, qd, W.bad);
            if (mfma) {   // the rounded queries of the matrix-core kernels (routing in mode 1, the scans)
                const caps_status qs = lowp_qquant(ix, q + (int64_t)q0 * d, nb, W.qlow, W.qscale, W.qaux, st);
                if (qs != CAPS_OK) return qs;
            }
            prof_end(CAPS_STAGE_PREP, st);
            if (router) {
                // learned routing: router probes and their candidate counts,
                // then centroid routing for only the queries that fall back
                // (low confidence, or fewer than k candidates)
                prof_begin(CAPS_STAGE_ROUTE, st);
                const caps_status rs = router_scores(ix, q + (int64_t)q0 * d, nb, con_off + q0, con_attr, con_val, n_con,
                                                     W.rx, W.rh, W.rbn, scores, W.conf, st);
                if (rs != CAPS_OK) return rs;
                prof_end(CAPS_STAGE_ROUTE, st);
                prof_begin(CAPS_STAGE_TOPM, st);
                launch_topm(scores, nb, b, pb, m, probes, st, topm_s);
                prof_end(CAPS_STAGE_TOPM, st);
                prof_begin(CAPS_STAGE_SELECT, st);
                hipLaunchKernelGGL(k_select, dim3(nblocks(pairs, 256)), dim3(256), 0, st, probes, nb, m, qd, W.qterms, ix->sch,
                                   ix->tags, h, ix->offs, sp->rule, sel, cand);
                const caps_status fl = router_fallback_list(ix, nb, m, k, W.conf, cand, W.fbq, W.nfb, st);
                if (fl != CAPS_OK) return fl;
                prof_end(CAPS_STAGE_SELECT, st);
            }
            // centroid scores: every query, or (learned routing) score row r
            // for falling-back query fbq[r], r < nfb
            const int32_t *rows = router ? W.fbq : nullptr, *nrows = router ? W.nfb : nullptr;
            prof_begin(CAPS_STAGE_ROUTE, st);
            if (lowp) {
                // precision mode: centroid scores on the matrix cores from the
                // rounded queries and the centroid copy
                const caps_status rs = lowp_route(ix, W.qlow, W.qscale, nb, scores, st, rows, nrows);
                if (rs != CAPS_OK) return rs;
            } else {
                hipLaunchKernelGGL(k_route_scores, dim3(nblocks(nb, kTile), nblocks(b, kTile)), dim3(256), 0, st,
                                   q + (int64_t)q0 * d, nb, d, ix->cent, ix->cnorm, b, ix->metric, scores, rows, nrows);
            }
            prof_end(CAPS_STAGE_ROUTE, st);
            prof_begin(CAPS_STAGE_TOPM, st);
            launch_topm(scores, nb, b, pb, m, router ? W.probes_c : probes, st, topm_s, nrows);
            prof_end(CAPS_STAGE_TOPM, st);
            if (router) {
                const caps_status fs = router_fallback_apply(nb, m, W.fbq, W.nfb, W.probes_c, probes, st);
                if (fs != CAPS_OK) return fs;
            }
            prof_begin(CAPS_STAGE_SELECT, st);
            hipLaunchKernelGGL(k_select, dim3(nblocks(pairs, 256)), dim3(256), 0, st, probes, nb, m, qd, W.qterms, ix->sch,
                               ix->tags, h, ix->offs, sp->rule, sel, cand);
            CAPS_HIP(hipGetLastError());
            if (probes_only) {
                prof_end(CAPS_STAGE_SELECT, st);
                hipLaunchKernelGGL(k_copy_i32, dim3(nblocks(pairs, 256)), dim3(256), 0, st, probes,
                                   out_probes + (int64_t)q0 * m, pairs);
                hipLaunchKernelGGL(k_copy_i32, dim3(nblocks(pairs, 256)), dim3(256), 0, st, (const int32_t *)sel,
                                   (int32_t *)(out_masks + (int64_t)q0 * m), pairs);
                CAPS_HIP(hipGetLastError());
                continue;
            }
            if (ex.surv_mask)
                hipLaunchKernelGGL(k_surv_mask, dim3(nblocks(pairs, 4)), dim3(256), 0, st, probes, sel, nb, m, qd, W.qterms, ix->offs,
                                   h, ix->words, ix->sigs, ix->slots, ix->lslots, ex.surv_mask + (int64_t)q0 * mask_words,
                               mask_words);
            hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(nb, 256)), dim3(256), 0, st, tau, (int64_t)nb, ~0ull);
            if (P.defer) {
                hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(nb, 256)), dim3(256), 0, st, W.dcnt, (int64_t)nb, 0);
                hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(nb, 256)), dim3(256), 0, st, W.oflow, (int64_t)nb, 0);
            }
            prof_end(CAPS_STAGE_SELECT, st);
            // Two rounds: the first probes of every query (best first) give each
            // query a tight seed bound on its final r-th key; the remaining probes
            // are scanned against it.  Exact keys on the matrix cores: the first
            // round is an approximate scan of the seed probes (every probe when
            // m < 32) whose best candidates are rescored exactly for the bound
            // (k_seed_exact); the second scans every probe and defers its pairs
            // to the merge, and a rescue pass rescans the queries whose pairs
            // did not fit.  (The approximate seed pass is cheap per probe but
            // its bound looser: m/24 seed probes there, enough that on the
            // 1M-point benchmark no query's pairs overflow.)
            const bool seeded_exact = P.defer;
            const int32_t *qord = nullptr;   // bucketing order of the queries (null: as given)
            if (ix->sch.n_dense > 0) {
                int32_t kbits = 0;
                for (int a = 0; a < ix->sch.n_dense; a++) kbits += ix->sch.field_bits[a] + 1;
                const int32_t shift = std::max(0, kbits - kQordBits), nk = 1 << (kbits - shift);
                prof_begin(CAPS_STAGE_SELECT, st);
                hipLaunchKernelGGL(k_qorder, dim3(1), dim3(kQordT), sizeof(int32_t) * (size_t)nk, st, qd, nb,
                                   ix->sch, shift, nk, W.qord);
                prof_end(CAPS_STAGE_SELECT, st);
                qord = W.qord;
            }
            for (int round = 0; round < 2; round++) {
                const int32_t r0 = round == 0 || seeded_exact ? 0 : s_seed;
                const int32_t r1 = round == 0 ? s_seed : m;
                if (r0 >= r1) continue;
                // tile width of this round: the exact main pass and the seed lists may
                // run 128-entry tiles
                const bool seed_x32 = mfma && !lowp && seeded_exact && round == 0 && lowp_seed_x32(ix, disj, r);
                const int qbr = mfma && !lowp && (!(seeded_exact && round == 0) || seed_x32) ? lowp_qb_main(ix, disj)
                                                                                            : qb;
                prof_begin(CAPS_STAGE_SELECT, st);
                const unsigned ggrid = (unsigned)((ngrp + kXcds - 1) / kXcds * kXcds);   // XCD-mapped groups
                hipLaunchKernelGGL(k_bucket_hist, dim3(ggrid), dim3(kBucketT), sizeof(int32_t) * (size_t)b, st, probes, sel,
                                   qord, nb, m, r0, r1, b, ngrp, hist);
                {
                    const caps_status es = exclusive_scan_i32(hist, hscan, (int64_t)b * ngrp, htotal, W.scan_sums, st);
                    if (es != CAPS_OK) return es;
                }
                hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, hscan, htotal, b, ngrp, qbr, pstart, pcount,
                                   tstart);
                const int64_t max_tiles = ((int64_t)nb * (r1 - r0) + qbr - 1) / qbr + b;
                const int64_t grid = (max_tiles + kXcds - 1) / kXcds * kXcds;
                hipLaunchKernelGGL(k_tile_desc, dim3(nblocks(grid, 256)), dim3(256), 0, st, tstart, pstart, pcount, b,
                                   qbr, (int32_t)grid, W.tiles);
                // the fill packs each entry's class when entries stay below 2^27
                const int32_t nc_pack = nc > 1 && (int64_t)nb * m < ((int64_t)1 << kClassShift) ? nc : 1;
                hipLaunchKernelGGL(k_bucket_fill, dim3(ggrid), dim3(kBucketT), sizeof(int32_t) * (size_t)b, st, probes, sel,
                                   qord, nb, m, r0, r1, b, ngrp, hscan, nc_pack, entries, nc > 1 ? nullptr : W.esel);
                const int32_t *ent = entries;
                const uint32_t *esel = W.esel;   // (the class sort writes the level masks itself)
                if (nc > 1) {
                    hipLaunchKernelGGL(k_class_sort, dim3(b), dim3(kClassW * 64), 0, st, entries, sel, pstart, pcount, nc,
                                       (int32_t)(nc_pack > 1), W.entries2, W.esel);
                    ent = W.entries2;
                }
                CAPS_HIP(hipGetLastError());
                prof_end(CAPS_STAGE_SELECT, st);
                if (mfma) {
                    const bool seed_pass = seeded_exact && round == 0;
                    LowpScan S{};
                    S.nb = nb;
                    S.m = m;
                    S.r = r;
                    S.kind = seed_x32 ? 4 : lowp || seed_pass ? 0 : 1;
                    S.stage = seed_pass ? CAPS_STAGE_SEED : CAPS_STAGE_SCAN;
                    S.max_tiles = grid;
                    S.tiles = W.tiles;
                    S.entries = ent;
                    S.esel = esel;
                    S.sel = sel;
                    S.qd = qd;
                    S.qterms = W.qterms;
                    S.disj = disj;
                    S.q = q + (int64_t)q0 * d;
                    S.qlow = W.qlow;
                    S.qscale = W.qscale;
                    S.qaux = W.qaux;
                    S.partials = partials;
                    S.tau = tau;
                    S.pcnt = W.pcnt;
                    S.nsurv = out_nsurv && !seed_pass ? nsurv + q0 : nullptr;   // counted only when asked for
                    S.dpos = W.dpos;
                    S.dcnt = W.dcnt;
                    S.dcap = kDeferCap;
                    S.oflow = W.oflow;
                    S.rescue_grid = sp->rescue_grid;
                    const caps_status ls = lowp_scan(ix, S, st);
                    if (ls != CAPS_OK) return ls;
                    if (S.kind == 1) {   // rescue pass over the tiles that hold a flagged query
                        hipLaunchKernelGGL(k_rescue_init, dim3(1), dim3(1024), 0, st, W.oflow, nb, W.rcount);
                        hipLaunchKernelGGL(k_rescue_tiles, dim3(nblocks(grid, 256)), dim3(256), 0, st, W.tiles,
                                           (int32_t)grid, ent, m, W.oflow, qb, (int32_t)(qbr != qb), W.rlist,
                                           W.rcount);
                        S.kind = 2;
                        S.rhalves = qbr != qb;
                        S.rlist = W.rlist;
                        S.rcount = W.rcount;
                        S.nsurv = nullptr;
                        S.stage = CAPS_STAGE_RESCUE;
                        const caps_status rs = lowp_scan(ix, S, st);
                        if (rs != CAPS_OK) return rs;
                    }
                } else {
                    ScanArgs A;
                    A.tiles = W.tiles;
                    A.ntiles = (int32_t)grid;
                    A.entries = ent;
                    A.sel = sel;
                    A.q = q + (int64_t)q0 * d;
                    A.qd = qd;
                    A.qterms = W.qterms;
                    A.offs = ix->offs;
                    A.perm = ix->perm;
                    A.vecs = ix->vecs;
                    A.words = ix->words;
                    A.sigs = ix->sigs;
                    A.slots = ix->slots;
                    A.lslots = ix->lslots;
                    A.partials = partials;
                    A.tau = tau;
                    A.nsurv = nsurv + q0;
                    A.d = d;
                    A.m = m;
                    A.h = h;
                    A.b = b;
                    A.k = k;
                    prof_begin(CAPS_STAGE_SCAN, st);
                    hipLaunchKernelGGL(scan_fn, dim3((unsigned)grid), dim3(scan_waves(k) * 64), lds, st, A);
                    prof_end(CAPS_STAGE_SCAN, st);
                    CAPS_HIP(hipGetLastError());
                }
                if (round == 0 && seeded_exact) {
                    prof_begin(CAPS_STAGE_SEED, st);
                    hipLaunchKernelGGL(k_seed_exact, dim3(nblocks(nb, 4)), dim3(256), 0, st, partials, W.pcnt, sel, nb,
                                       m, s_seed, r, std::min(2 * k, 64), k, ix->vecs, q + (int64_t)q0 * d, ix->perm, d,
                                       ix->metric, tau);
                    prof_end(CAPS_STAGE_SEED, st);
                    CAPS_HIP(hipGetLastError());
                } else if (round == 0 && s_seed < m) {
                    prof_begin(CAPS_STAGE_SELECT, st);
                    hipLaunchKernelGGL(k_seed_tau, dim3(nblocks(nb, 4)), dim3(256), 0, st, partials,
                                       lowp ? W.pcnt : nullptr, sel, nb, m, s_seed, r, r, tau);
                    prof_end(CAPS_STAGE_SELECT, st);
                    CAPS_HIP(hipGetLastError());
                }
            }
            if (lowp) {
                const caps_status ls = lowp_merge(ix, q + (int64_t)q0 * d, nb, sel, m, k, r, partials, W.pcnt, cand,
                                                  ncand + q0, out_ids + (int64_t)q0 * k, out_dist + (int64_t)q0 * k, st);
                if (ls != CAPS_OK) return ls;
                continue;
            }
            prof_begin(CAPS_STAGE_MERGE, st);
            int32_t *oi = out_ids + (int64_t)q0 * k;
            float *od = out_dist + (int64_t)q0 * k;
            const int32_t *mcnt = mfma ? W.pcnt : nullptr;   // matrix-core lists are counted, plain ones padded
            Deferred D{};
            if (P.defer) {
                D.pos = W.dpos;
                D.cnt = W.dcnt;
                D.oflow = W.oflow;
                D.cap = kDeferCap;
                D.d = d;
                D.vecs = ix->vecs;
                D.q = q + (int64_t)q0 * d;
                D.perm = ix->perm;
                D.qaux = W.qaux;
                D.eta = exact_eta(ix);
            }
            if (k <= 16)
                hipLaunchKernelGGL(k_merge<16>, dim3(nblocks(nb, 4)), dim3(256), 0, st, partials, mcnt, sel, cand, nb, m,
                                   k, ix->metric, oi, od, ncand + q0, D);
            else if (k <= 32)
                hipLaunchKernelGGL(k_merge<32>, dim3(nblocks(nb, 4)), dim3(256), 0, st, partials, mcnt, sel, cand, nb, m,
                                   k, ix->metric, oi, od, ncand + q0, D);
            else
                hipLaunchKernelGGL(k_merge<64>, dim3(nblocks(nb, 4)), dim3(256), 0, st, partials, mcnt, sel, cand, nb, m,
                                   k, ix->metric, oi, od, ncand + q0, D);
            prof_end(CAPS_STAGE_MERGE, st);
            CAPS_HIP(hipGetLastError());
        }
    return CAPS_OK;
    };
    caps_status s = run();
    if (s == CAPS_OK && (sp->flags & CAPS_SEARCH_VALIDATE)) {
        int32_t nbad = 0;
        hipError_t e = hipMemcpyAsync(&nbad, W.bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_error("caps_search: %s", hipGetErrorString(e));
            s = CAPS_EDEVICE;
        } else if (nbad > 0) {
            set_error("caps_search: %d query rows hold NaN or Inf", nbad);
            s = CAPS_EINVAL;
        }
    }
    if (!ex.ws) {
        const hipError_t e = hipFreeAsync(ar.base, st);
        if (s == CAPS_OK && e != hipSuccess) {
            set_error("caps_search: hipFreeAsync failed: %s", hipGetErrorString(e));
            s = CAPS_EDEVICE;
        }
    }
    return s;
}

}  // namespace caps
