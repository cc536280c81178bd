// Matrix-core scan over the index's low-precision copy.
//
// Build: every CSR vector gets a BF16, FP16 or FP8-E4M3 copy (zero padded to
// 32 x {1, 2, 4, 8} coordinates), its FP32 |x|^2 (sequential fma) and two
// error norms computed in FP64 and rounded up: |x - x~| and |x~| (x~ the
// value the copy represents).  Queries are rounded the same way when a
// search starts, with the matching query-side norms.
//
// Each tile (one partition, up to 64 of the queries probing it) computes
// query x point dot products with MFMA (v_mfma_f32_16x16x32_{bf16,f16,fp8},
// FP32 accumulation) and applies the exact attribute filter to every
// (query, point) pair in the epilogue.  Two uses:
//
// * approximate search (mode 1): each query keeps its best R candidates
//   under the approximate score (L2: |x|^2 - 2 x~.q~, IP: -x~.q~); a merge
//   pass rescores a query's candidates over all probes with the exact FP32
//   arithmetic and keeps the final top k;
// * exact search (mode 0 on an index with a copy): the approximate score,
//   widened by the error norms and a rounding margin, is a lower bound on the
//   exact FP32 distance.  A pair whose bound exceeds its query's current k-th
//   exact key cannot enter the top k; every other pair is rescored exactly
//   (the sequential fma of the plain scan) and competes with its exact key.
//   Results are identical to the plain FP32 scan.
#include <math.h>

#include <algorithm>

#include "caps_mfma.h"

namespace caps {

// ------------------------------------------------------------------ rounding
__device__ inline uint16_t f16_rne_sat(float f) {
    f = fminf(fmaxf(f, -65504.0f), 65504.0f);
    return __builtin_bit_cast(uint16_t, (_Float16)f);
}

// OCP E4M3 (bias 7, max 448, 0x7F/0xFF are NaN): round to nearest even,
// saturating to +-448.
__device__ inline uint8_t e4m3_rne_sat(float v) {
    const uint8_t sign = v < 0.0f ? 0x80 : 0x00;
    const float a = fabsf(v);
    if (!(a < 448.0f)) return sign | 0x7E;
    if (a < 0.015625f) {   // below the smallest normal 2^-6: quantum 2^-9
        const int qi = (int)rintf(a * 512.0f);
        return qi == 0 ? (uint8_t)0 : (uint8_t)(sign | qi);   // single zero; 8 is the smallest normal
    }
    int e2;
    (void)frexpf(a, &e2);
    int e = e2 - 1;                       // a in [2^e, 2^(e+1))
    int q = (int)rintf(ldexpf(a, 3 - e)); // in [8, 16]
    if (q == 16) {
        e += 1;
        q = 8;
    }
    return sign | (uint8_t)(((e + 7) << 3) | (q - 8));
}

// Value of an E4M3 code (finite codes only).
__device__ inline double e4m3_value(uint8_t c) {
    const int e = (c >> 3) & 15, m = c & 7;
    const double v = e == 0 ? ldexp((double)m, -9) : ldexp((double)(8 + m), e - 10);
    return (c & 0x80) ? -v : v;
}

// FP64 -> FP32 rounded towards +inf / -inf (inputs >= 0).
__device__ inline float f32_up(double v) {
    const float f = (float)v;
    return (double)f < v ? nextafterf(f, __builtin_huge_valf()) : f;
}
__device__ inline float f32_down(double v) {
    const float f = (float)v;
    return (double)f > v ? nextafterf(f, 0.0f) : f;
}

// Rounds row r (d coordinates) into `out` (dpad elements) and returns the
// FP8 scale (1 otherwise); e2 / a2 receive, in FP64, sum (r_j - r~_j)^2 and
// sum r~_j^2.
__device__ inline float quantize_row(const float *r, int d, int dpad, int prec, void *out, double &e2,
                                     double &a2) {
    float s = 1.0f;
    e2 = 0.0;
    a2 = 0.0;
    if (prec == CAPS_PREC_FP8) {
        float amax = 0.0f;
        for (int j = 0; j < d; j++) amax = fmaxf(amax, fabsf(r[j]));
        s = amax > 0.0f ? amax / 448.0f : 1.0f;
        uint8_t *o = reinterpret_cast<uint8_t *>(out);
        for (int j = 0; j < dpad; j++) {
            const uint8_t c = j < d ? e4m3_rne_sat(r[j] / s) : (uint8_t)0;
            o[j] = c;
            if (j < d) {
                const double v = (double)s * e4m3_value(c);
                e2 += ((double)r[j] - v) * ((double)r[j] - v);
                a2 += v * v;
            }
        }
    } else {
        uint16_t *o = reinterpret_cast<uint16_t *>(out);
        for (int j = 0; j < dpad; j++) {
            const uint16_t c = j < d ? (prec == CAPS_PREC_BF16 ? bf16_rne(r[j]) : f16_rne_sat(r[j])) : (uint16_t)0;
            o[j] = c;
            if (j < d) {
                const double v = prec == CAPS_PREC_BF16 ? (double)__builtin_bit_cast(float, (uint32_t)c << 16)
                                                        : (double)__builtin_bit_cast(_Float16, c);
                e2 += ((double)r[j] - v) * ((double)r[j] - v);
                a2 += v * v;
            }
        }
    }
    return s;
}

// relative slack covering the FP64 sums and square roots above
constexpr double kNormSlack = 1.0 + 0x1p-40;

// ------------------------------------------------------------------ build
// One thread per point: |x|^2 (sequential fma), rounded copy, FP8 scale and
// the error norms |x - x~| and |x~| (rounded up).
__global__ void k_quantize(const float *__restrict__ x, int64_t n, int32_t d, int32_t dpad, int32_t prec,
                           void *__restrict__ out, float *__restrict__ scale, float *__restrict__ xnorm,
                           float *__restrict__ lerr, float *__restrict__ lnrm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *r = x + i * d;
    float acc = 0.0f;
    for (int j = 0; j < d; j++) acc = fmaf(r[j], r[j], acc);
    xnorm[i] = acc;
    const int64_t eb = prec == CAPS_PREC_FP8 ? 1 : 2;
    double e2, a2;
    const float s = quantize_row(r, d, dpad, prec, reinterpret_cast<uint8_t *>(out) + i * dpad * eb, e2, a2);
    if (prec == CAPS_PREC_FP8) scale[i] = s;
    lerr[i] = f32_up(sqrt(e2) * kNormSlack);
    lnrm[i] = f32_up(sqrt(a2) * kNormSlack);
}

static int esize_of(int prec) { return prec == CAPS_PREC_FP8 ? 1 : 2; }

caps_status quantize_rows(const Index *ix, const float *x, int64_t n, void *lvec, float *scale, float *xnorm,
                          float *lerr, float *lnrm, hipStream_t st) {
    if (n <= 0) return CAPS_OK;
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, ix->d, ix->dpad,
                       ix->prec, lvec, scale, xnorm, lerr, lnrm);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

caps_status build_lowp(Index *ix, hipStream_t st) {
    if (ix->prec == CAPS_PREC_NONE) return CAPS_OK;
    // rows padded to 32 x {1, 2, 4, 8} coordinates: the scan kernels are
    // specialised on the number of 32-wide MFMA K-steps
    int ns = 1;
    while (32 * ns < ix->d) ns <<= 1;
    ix->dpad = 32 * ns;
    const size_t eb = (size_t)esize_of(ix->prec);
    const size_t lbytes = (size_t)ix->n * ix->dpad * eb;
    const size_t fbytes = sizeof(float) * (size_t)ix->n;
    CAPS_HIP(hipMalloc(&ix->lvecs, lbytes));
    ix->bytes += (int64_t)lbytes;
    CAPS_HIP(hipMalloc((void **)&ix->xnorm, fbytes));
    CAPS_HIP(hipMalloc((void **)&ix->lerr, fbytes));
    CAPS_HIP(hipMalloc((void **)&ix->lnrm, fbytes));
    ix->bytes += (int64_t)(3 * fbytes);
    if (ix->prec == CAPS_PREC_FP8) {
        CAPS_HIP(hipMalloc((void **)&ix->lscale, fbytes));
        ix->bytes += (int64_t)fbytes;
    }
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((ix->n + 255) / 256)), dim3(256), 0, st, ix->vecs, ix->n, ix->d,
                       ix->dpad, ix->prec, ix->lvecs, ix->lscale, ix->xnorm, ix->lerr, ix->lnrm);
    CAPS_HIP(hipGetLastError());
    return build_lowp_centroids(ix, st);
}

// ------------------------------------------------------------------ queries
// One wave per query: rounded copy (the codes of quantize_row, element by
// element), FP8 scale and qaux = {|q| (up), |q|^2 (down), |q - q~| (up),
// |q~| (up)}; the FP64 sums are reduced across the wave (their order does
// not matter: kNormSlack covers any order).
__global__ __launch_bounds__(256) void k_qquant(const float *__restrict__ q, int32_t nq, int32_t d, int32_t dpad,
                                                int32_t prec, void *__restrict__ out, float *__restrict__ scale,
                                                float *__restrict__ qaux) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nq) return;
    const float *r = q + i * d;
    float s = 1.0f;
    if (prec == CAPS_PREC_FP8) {
        float amax = 0.0f;
        for (int j = lane; j < d; j += 64) amax = fmaxf(amax, fabsf(r[j]));
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        s = amax > 0.0f ? amax / 448.0f : 1.0f;
    }
    double e2 = 0.0, a2 = 0.0, n2 = 0.0;
    for (int j = lane; j < dpad; j += 64) {
        const float x = j < d ? r[j] : 0.0f;
        double v;
        if (prec == CAPS_PREC_FP8) {
            const uint8_t c = j < d ? e4m3_rne_sat(x / s) : (uint8_t)0;
            reinterpret_cast<uint8_t *>(out)[i * dpad + j] = c;
            v = (double)s * e4m3_value(c);
        } else {
            const uint16_t c = j < d ? (prec == CAPS_PREC_BF16 ? bf16_rne(x) : f16_rne_sat(x)) : (uint16_t)0;
            reinterpret_cast<uint16_t *>(out)[i * dpad + j] = c;
            v = prec == CAPS_PREC_BF16 ? (double)__builtin_bit_cast(float, (uint32_t)c << 16)
                                       : (double)__builtin_bit_cast(_Float16, c);
        }
        if (j < d) {
            e2 += ((double)x - v) * ((double)x - v);
            a2 += v * v;
            n2 += (double)x * (double)x;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        e2 += __shfl_xor(e2, o, 64);
        a2 += __shfl_xor(a2, o, 64);
        n2 += __shfl_xor(n2, o, 64);
    }
    if (lane == 0) {
        scale[i] = s;
        qaux[4 * i + 0] = f32_up(sqrt(n2) * kNormSlack);
        qaux[4 * i + 1] = f32_down(n2 / kNormSlack);
        qaux[4 * i + 2] = f32_up(sqrt(e2) * kNormSlack);
        qaux[4 * i + 3] = f32_up(sqrt(a2) * kNormSlack);
    }
}

// ------------------------------------------------------------------ routing
// Precision-mode routing: query x centroid scores from the low-precision
// copies on the matrix cores (FP32 accumulation).  64 queries x 64
// centroids per workgroup, wave w owning queries 16w..16w+15: per K-step
// one A operand (its query rows) and four B operands (four 16-centroid
// blocks), read straight from global memory (the centroid copy is small and
// stays in cache).  Score: L2 |c|^2 - 2 q~.c~ (|c|^2 of the FP32 centroid,
// sequential fma), IP -q~.c~; FP8 products are scaled by both scales.
template <int PREC, int NS>
__global__ __launch_bounds__(256) void k_route_mfma(const uint8_t *__restrict__ qlow, const float *__restrict__ qscale,
                                                    int32_t nq, const uint8_t *__restrict__ clow,
                                                    const float *__restrict__ cscale, const float *__restrict__ cn,
                                                    int32_t b, int32_t metric, float *__restrict__ scores,
                                                    const int32_t *__restrict__ rows,
                                                    const int32_t *__restrict__ nrows) {
    typedef MfmaOp<PREC> Op;
    typedef typename Op::T VT;
    constexpr int ES = Op::ES;
    constexpr int KSTEP_BYTES = 32 * ES, LANE_BYTES = 8 * ES, ROWB = NS * KSTEP_BYTES;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (nrows) nq = min(nq, *nrows);
    if ((int64_t)blockIdx.x * 64 >= nq) return;
    const int64_t q0 = (int64_t)blockIdx.x * 64 + 16 * w;
    const int c0 = blockIdx.y * 64;
    const int64_t arow = q0 + (lane & 15);
    const bool aok = arow < nq;
    const int64_t asrc_row = aok ? (rows ? (int64_t)rows[arow] : arow) : 0;
    const uint8_t *asrc = qlow + asrc_row * ROWB + (lane >> 4) * LANE_BYTES;
    f32x4 acc[4];
#pragma unroll
    for (int bb = 0; bb < 4; bb++) acc[bb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const VT a = aok ? Op::load(asrc + s * KSTEP_BYTES) : VT{};
        VT bf[4];
#pragma unroll
        for (int bb = 0; bb < 4; bb++) {
            const int c = c0 + bb * 16 + (lane & 15);
            bf[bb] = c < b ? Op::load(clow + (int64_t)c * ROWB + s * KSTEP_BYTES + (lane >> 4) * LANE_BYTES) : VT{};
        }
#pragma unroll
        for (int bb = 0; bb < 4; bb++) acc[bb] = Op::mma(a, bf[bb], acc[bb]);
    }
#pragma unroll
    for (int bb = 0; bb < 4; bb++) {
        const int c = c0 + bb * 16 + (lane & 15);
        if (c >= b) continue;
        const float cs = PREC == CAPS_PREC_FP8 ? cscale[c] : 1.0f;
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const int64_t q = q0 + (lane >> 4) * 4 + rr;
            if (q >= nq) continue;
            float dd = acc[bb][rr];
            if (PREC == CAPS_PREC_FP8) dd = dd * qscale[rows ? (int64_t)rows[q] : q] * cs;
            scores[q * b + c] = canon0(metric == 0 ? fmaf(-2.0f, dd, cn[c]) : -dd);
        }
    }
}

template <int PREC>
static void launch_route(int ns, dim3 g, hipStream_t st, const uint8_t *qlow, const float *qscale, int32_t nq,
                         const uint8_t *clow, const float *cscale, const float *cn, int32_t b, int32_t metric,
                         float *scores, const int32_t *rows, const int32_t *nrows) {
    switch (ns) {
    case 1: hipLaunchKernelGGL((k_route_mfma<PREC, 1>), g, dim3(256), 0, st, qlow, qscale, nq, clow, cscale, cn, b, metric, scores, rows, nrows); return;
    case 2: hipLaunchKernelGGL((k_route_mfma<PREC, 2>), g, dim3(256), 0, st, qlow, qscale, nq, clow, cscale, cn, b, metric, scores, rows, nrows); return;
    case 4: hipLaunchKernelGGL((k_route_mfma<PREC, 4>), g, dim3(256), 0, st, qlow, qscale, nq, clow, cscale, cn, b, metric, scores, rows, nrows); return;
    default: hipLaunchKernelGGL((k_route_mfma<PREC, 8>), g, dim3(256), 0, st, qlow, qscale, nq, clow, cscale, cn, b, metric, scores, rows, nrows); return;
    }
}

// Scores of nb rounded queries (k_qquant output) against the centroid copy.
// With a row list, score row r belongs to query rows[r], for r < *nrows.
caps_status lowp_route(const Index *ix, const void *qlow, const float *qscale, int32_t nb, float *scores,
                       hipStream_t st, const int32_t *rows, const int32_t *nrows) {
    const dim3 g((unsigned)((nb + 63) / 64), (unsigned)((ix->b + 63) / 64));
    const uint8_t *q = reinterpret_cast<const uint8_t *>(qlow), *c = reinterpret_cast<const uint8_t *>(ix->clow);
    const int ns = ix->dpad / 32;
    if (ix->prec == CAPS_PREC_BF16)
        launch_route<CAPS_PREC_BF16>(ns, g, st, q, qscale, nb, c, ix->cscale, ix->cnorm, ix->b, ix->metric, scores,
                                     rows, nrows);
    else if (ix->prec == CAPS_PREC_FP16)
        launch_route<CAPS_PREC_FP16>(ns, g, st, q, qscale, nb, c, ix->cscale, ix->cnorm, ix->b, ix->metric, scores,
                                     rows, nrows);
    else
        launch_route<CAPS_PREC_FP8>(ns, g, st, q, qscale, nb, c, ix->cscale, ix->cnorm, ix->b, ix->metric, scores,
                                    rows, nrows);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

// Rounds the queries of a sub-batch into the index's copy format (codes,
// FP8 scale, error norms) for the matrix-core kernels.
caps_status lowp_qquant(const Index *ix, const float *q, int32_t nb, void *qlow, float *qscale, float *qaux,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_qquant, dim3((nb + 3) / 4), dim3(256), 0, st, q, nb, ix->d, ix->dpad, ix->prec, qlow, qscale,
                       qaux);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

// Low-precision copy of the centroids (the same format as the vectors', FP8
// with one scale per centroid) for precision-mode routing.
caps_status build_lowp_centroids(Index *ix, hipStream_t st) {
    if (ix->prec == CAPS_PREC_NONE) return CAPS_OK;
    const size_t eb = (size_t)esize_of(ix->prec), b = (size_t)ix->b;
    if (!ix->clow) {
        CAPS_HIP(hipMalloc(&ix->clow, b * ix->dpad * eb));
        CAPS_HIP(hipMalloc((void **)&ix->cscale, sizeof(float) * b));
        ix->bytes += (int64_t)(b * ix->dpad * eb + sizeof(float) * b);
    }
    float *tmp = nullptr;   // the norms k_quantize also writes (unused here)
    CAPS_HIP(hipMallocAsync((void **)&tmp, sizeof(float) * 3 * b, st));
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((b + 255) / 256)), dim3(256), 0, st, ix->cent, (int64_t)b, ix->d,
                       ix->dpad, ix->prec, ix->clow, ix->cscale, tmp, tmp + b, tmp + 2 * b);
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(tmp, st);
    if (e != hipSuccess) {
        set_error("build_lowp_centroids: %s", hipGetErrorString(e));
        return CAPS_EDEVICE;
    }
    return CAPS_OK;
}

// ------------------------------------------------------------------ merge + rerank
// One wave per query: collect the approximate candidates of all probes
// (keeping the best r), rescore them with the exact FP32 arithmetic, keep k.
constexpr int kMCap = 256;

template <int METRIC>
__global__ __launch_bounds__(256) void k_merge_rerank(const uint64_t *__restrict__ partials,
                                                      const int32_t *__restrict__ pcnt,
                                                      const uint32_t *__restrict__ sel,
                                                      const int32_t *__restrict__ cand, int32_t nq, int32_t m,
                                                      int32_t r, int32_t k, const float *__restrict__ q,
                                                      int32_t d, const float *__restrict__ vecs,
                                                      const int32_t *__restrict__ perm, int32_t *__restrict__ ids,
                                                      float *__restrict__ dist, int32_t *__restrict__ ncand) {
    __shared__ uint64_t pool_all[4][kMCap];
    __shared__ int32_t npool_all[4];
    const int wq = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qq = blockIdx.x * 4 + wq;
    if (qq >= nq) return;
    uint64_t *pool = pool_all[wq];
    int32_t *npool = &npool_all[wq];
    const int nc = gather_best<kMCap>(pool, npool, partials, pcnt, sel, cand, (int64_t)qq * m, 0, m, r, r);
    if (lane == 0) ncand[qq] = nc;
    const int nr = *npool;   // <= r <= 64, sorted by approximate key
    // exact FP32 rescoring, one candidate per lane
    uint64_t key2 = ~0ull;
    if (lane < nr) {
        const int32_t pos = (int32_t)(uint32_t)(pool[lane] & 0xFFFFFFFFu);
        const float kf = exact_score<8>(vecs + (int64_t)pos * d, q + (int64_t)qq * d, d, METRIC == 0);
        key2 = ((uint64_t)f2ord(kf) << 32) | (uint32_t)perm[pos];
    }
    int rank = 0;
    for (int i = 0; i < nr; i++) rank += readlane_u64(key2, i) < key2 ? 1 : 0;
    if (lane < nr && rank < k) {
        const int64_t o = (int64_t)qq * k + rank;
        ids[o] = (int32_t)(uint32_t)(key2 & 0xFFFFFFFFu);
        const float kf = ord2f((uint32_t)(key2 >> 32));
        dist[o] = METRIC == 0 ? kf : canon0(-kf);
    }
    if (lane >= nr && lane < k) {
        const int64_t o = (int64_t)qq * k + lane;
        ids[o] = -1;
        dist[o] = METRIC == 0 ? __builtin_huge_valf() : -__builtin_huge_valf();
    }
}

// ------------------------------------------------------------------ host
template <int EX>
static LowpFn pick_prec(int prec, int ns, bool lab, int r) {
    if (prec == CAPS_PREC_BF16) return pick_ns<CAPS_PREC_BF16, EX>(ns, lab, r);
    if (prec == CAPS_PREC_FP16) return pick_ns<CAPS_PREC_FP16, EX>(ns, lab, r);
    return pick_ns<CAPS_PREC_FP8, EX>(ns, lab, r);
}

// workgroups of the rescue pass (32 per compute unit): enough to spread a
// long list, few enough that an empty one costs little
constexpr int64_t kRescueWgs = 8192;

size_t lowp_scan_lds(const Index *ix, int r, int kind, bool disj) {
    return LowpLds(kind == 1 || kind == 3 ? 32 : lowp_cb(r), kind, ix->sch.label_vocab > 0 || disj).total + 64;
}

caps_status lowp_scan(const Index *ix, const LowpScan &S, hipStream_t st) {
    LowpArgs A;
    A.tiles = S.tiles;
    A.ntiles = (int32_t)S.max_tiles;
    A.entries = S.entries;
    A.esel = S.esel;
    A.sel = S.sel;
    A.qd = S.qd;
    A.qterms = S.qterms;
    A.offs = ix->offs;
    A.lvecs = reinterpret_cast<const uint8_t *>(ix->lvecs);
    A.lscale = ix->lscale;
    A.xnorm = ix->xnorm;
    A.lerr = ix->lerr;
    A.lnrm = ix->lnrm;
    A.words = ix->words;
    A.sigs = ix->sigs;
    A.slots = ix->slots;
    A.lslots = ix->lslots;
    A.qlow = reinterpret_cast<const uint8_t *>(S.qlow);
    A.qscale = S.qscale;
    A.qaux = S.qaux;
    A.vecs = ix->vecs;
    A.q = S.q;
    A.perm = ix->perm;
    A.partials = S.partials;
    A.pcnt = S.pcnt;
    A.tau = S.tau;
    A.nsurv = S.nsurv;
    A.dpos = S.dpos;
    A.dcnt = S.dcnt;
    A.dcap = S.dcap;
    A.oflow = S.oflow;
    A.rlist = S.rlist;
    A.rcount = S.rcount;
    A.rhalves = S.rhalves ? 1 : 0;
    A.m = S.m;
    A.h = ix->h;
    A.b = ix->b;
    A.r = S.r;
    A.metric = ix->metric;
    A.d = ix->d;
    // Rounding budget of the exact bound, relative to |x|^2 + |q|^2 (+ the
    // bound's own magnitude): the stored |x|^2 (d roundings), the exact
    // distance against its real value (d + 2), the FP32 evaluation of the
    // bound (a dozen) -- about 3 dpad + 24 units of 2^-24, doubled.  The
    // MFMA accumulation (at most dpad additions, each within 2^-23 of the
    // sum of magnitudes) is bounded by gam |x~| |q~|, gam = 8 dpad 2^-24
    // (four times that).
    A.eta = exact_eta(ix);
    A.gam = (float)(8.0 * ix->dpad) * 0x1p-24f;
    // the variant with the filter's slow path: label tests, disjunctions
    const bool lab = ix->sch.label_vocab > 0 || S.disj;
    const LowpFn fn = S.kind == 0   ? pick_prec<0>(ix->prec, ix->dpad / 32, lab, S.r)
                      : S.kind == 4 ? pick_prec<4>(ix->prec, ix->dpad / 32, lab, S.r)
                      : S.kind == 1 ? (S.nsurv ? pick_prec<3>(ix->prec, ix->dpad / 32, lab, S.r)
                                               : pick_prec<1>(ix->prec, ix->dpad / 32, lab, S.r))
                                    : pick_prec<2>(ix->prec, ix->dpad / 32, lab, S.r);
    // (the 32 x 32 main pass holds its arrays in static LDS)
    const bool x32 = (S.kind == 1 || S.kind == 4) && lowp_x32_kernel(ix->prec, ix->dpad / 32, lab);
    const size_t lds = x32 ? 0 : lowp_scan_lds(ix, S.r, S.kind, S.disj);
    {
        const caps_status ls = set_kernel_lds((const void *)fn, lds, ix->device);
        if (ls != CAPS_OK) return ls;
    }
    prof_begin(S.stage, st);
    // the rescue pass walks its (device-side) tile list with a bounded grid
    const int64_t full = (S.max_tiles + kXcds - 1) / kXcds * kXcds;
    const int64_t rcap = S.rescue_grid > 0 ? S.rescue_grid : kRescueWgs;
    const int64_t grid = S.kind == 2 ? std::min<int64_t>(full, rcap) : full;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kLNT), lds, st, A);
    prof_end(S.stage, st);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

caps_status lowp_merge(const Index *ix, const float *q, int32_t nb, const uint32_t *sel, int32_t m, int32_t k,
                       int32_t r, const uint64_t *partials, const int32_t *pcnt, const int32_t *cand, int32_t *ncand,
                       int32_t *out_ids, float *out_dist, hipStream_t st) {
    prof_begin(CAPS_STAGE_MERGE, st);
    if (ix->metric == 0)
        hipLaunchKernelGGL(k_merge_rerank<0>, dim3((nb + 3) / 4), dim3(256), 0, st, partials, pcnt, sel, cand, nb, m,
                           r, k, q, ix->d, ix->vecs, ix->perm, out_ids, out_dist, ncand);
    else
        hipLaunchKernelGGL(k_merge_rerank<1>, dim3((nb + 3) / 4), dim3(256), 0, st, partials, pcnt, sel, cand, nb, m,
                           r, k, q, ix->d, ix->vecs, ix->perm, out_ids, out_dist, ncand);
    prof_end(CAPS_STAGE_MERGE, st);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

int lowp_qb() { return kLQB; }

int lowp_qb_main(const Index *ix, bool disj) {
    return lowp_x32_kernel(ix->prec, ix->dpad / 32, ix->sch.label_vocab > 0 || disj) ? kXQB : kLQB;
}

bool lowp_seed_x32(const Index *ix, bool disj, int r) {
    return r >= 2 && lowp_x32_kernel(ix->prec, ix->dpad / 32, ix->sch.label_vocab > 0 || disj);
}

}  // namespace caps
