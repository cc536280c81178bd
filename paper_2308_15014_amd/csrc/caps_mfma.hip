// Low-precision scan on the matrix cores (search mode 1).
//
// Build: every CSR vector gets a BF16, FP16 or FP8-E4M3 copy (zero padded to
// a multiple of 32 coordinates) and its exact FP32 |x|^2.  Search: queries
// are rounded the same way; each tile (one partition, up to 64 of the
// queries probing it) computes query x point dot products with MFMA
// (v_mfma_f32_16x16x32_{bf16,f16,fp8}, FP32 accumulation), applies the exact
// attribute filter to every (query, point) pair in the epilogue and keeps
// each query's best R candidates under the approximate score; a merge pass
// collects a query's candidates over its probes and rescores them with the
// exact FP32 arithmetic of search mode 0, keeping the final top k.
#include <math.h>

#include <algorithm>

#include "caps_device.h"
#include "caps_internal.h"

namespace caps {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ rounding
__device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

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

// ------------------------------------------------------------------ build
// One thread per point: exact |x|^2 (sequential fma), FP8 scale, rounded copy.
__global__ void k_quantize(const float *__restrict__ x, int64_t n, int32_t d, int32_t dpad, int32_t prec,
                           void *__restrict__ out, float *__restrict__ scale, float *__restrict__ xnorm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *r = x + i * d;
    float acc = 0.0f, amax = 0.0f;
    for (int j = 0; j < d; j++) {
        acc = fmaf(r[j], r[j], acc);
        amax = fmaxf(amax, fabsf(r[j]));
    }
    if (xnorm) xnorm[i] = acc;
    if (prec == CAPS_PREC_FP8) {
        const float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        uint8_t *o = reinterpret_cast<uint8_t *>(out) + i * dpad;
        for (int j = 0; j < dpad; j++) o[j] = j < d ? e4m3_rne_sat(r[j] / s) : (uint8_t)0;
        scale[i] = s;
    } else {
        uint16_t *o = reinterpret_cast<uint16_t *>(out) + i * dpad;
        for (int j = 0; j < dpad; j++)
            o[j] = j < d ? (prec == CAPS_PREC_BF16 ? bf16_rne(r[j]) : f16_rne_sat(r[j])) : (uint16_t)0;
    }
}

static int esize_of(int prec) { return prec == CAPS_PREC_FP8 ? 1 : 2; }

caps_status build_lowp(Index *ix, hipStream_t st) {
    if (ix->prec == CAPS_PREC_NONE) return CAPS_OK;
    ix->dpad = (ix->d + 31) & ~31;
    const size_t eb = (size_t)esize_of(ix->prec);
    const size_t lbytes = (size_t)ix->n * ix->dpad * eb;
    CAPS_HIP(hipMalloc(&ix->lvecs, lbytes));
    ix->bytes += (int64_t)lbytes;
    CAPS_HIP(hipMalloc((void **)&ix->xnorm, sizeof(float) * (size_t)ix->n));
    ix->bytes += (int64_t)(sizeof(float) * (size_t)ix->n);
    if (ix->prec == CAPS_PREC_FP8) {
        CAPS_HIP(hipMalloc((void **)&ix->lscale, sizeof(float) * (size_t)ix->n));
        ix->bytes += (int64_t)(sizeof(float) * (size_t)ix->n);
    }
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((ix->n + 255) / 256)), dim3(256), 0, st, ix->vecs, ix->n, ix->d,
                       ix->dpad, ix->prec, ix->lvecs, ix->lscale, ix->xnorm);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

// ------------------------------------------------------------------ queries
__global__ void k_qquant(const float *__restrict__ q, int32_t nq, int32_t d, int32_t dpad, int32_t prec,
                         void *__restrict__ out, float *__restrict__ scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const float *r = q + (int64_t)i * d;
    float amax = 0.0f;
    for (int j = 0; j < d; j++) amax = fmaxf(amax, fabsf(r[j]));
    if (prec == CAPS_PREC_FP8) {
        const float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        uint8_t *o = reinterpret_cast<uint8_t *>(out) + (int64_t)i * dpad;
        for (int j = 0; j < dpad; j++) o[j] = j < d ? e4m3_rne_sat(r[j] / s) : (uint8_t)0;
        scale[i] = s;
    } else {
        uint16_t *o = reinterpret_cast<uint16_t *>(out) + (int64_t)i * dpad;
        for (int j = 0; j < dpad; j++)
            o[j] = j < d ? (prec == CAPS_PREC_BF16 ? bf16_rne(r[j]) : f16_rne_sat(r[j])) : (uint16_t)0;
        scale[i] = 1.0f;
    }
}

// ------------------------------------------------------------------ scan
struct LowpArgs {
    const int32_t *tstart, *pstart, *pcount, *entries;
    const uint32_t *sel;
    const QDesc *qd;
    const int32_t *offs;
    const uint8_t *lvecs;       // CSR rows of dpad elements
    const float *lscale, *xnorm;
    const uint32_t *words;
    const uint64_t *sigs;
    const uint16_t *slots;
    const uint8_t *qlow;        // query rows of dpad elements
    const float *qscale;
    uint64_t *partials;         // per (query, probe): up to r keys (score << 32 | CSR position)
    int32_t *pcnt;              // per (query, probe): number of keys written
    uint64_t *tau;              // per query: shared bound on its r-th approximate key
    int32_t *nsurv;
    int32_t dpad, m, h, b, r;
};

constexpr int kLNW = 4;          // waves per tile
constexpr int kLQPW = 16;        // queries per wave (MFMA rows)
constexpr int kLQB = kLNW * kLQPW;
constexpr int kLCH = 64;         // points per chunk: four 16-column MFMA blocks
constexpr int kLNT = kLNW * 64;

struct LowpLds {
    size_t xl, xw, xn, xsc, xsig, xslot, buf, bcnt, tau, qslot, qd, total;
    int xstride;   // bytes per staged row
    __host__ __device__ LowpLds(int dpad, int esize, int cb) {
        xstride = dpad * esize + 16;
        size_t o = 0;
        auto take = [&](size_t bytes) __host__ __device__ {
            o = (o + 15) & ~(size_t)15;
            size_t r = o;
            o += bytes;
            return r;
        };
        bcnt = take(sizeof(int32_t) * kLQB);
        tau = take(sizeof(uint64_t) * kLQB);
        qslot = take(sizeof(int32_t) * kLQB);
        qd = take(sizeof(QDesc) * kLQB);
        xw = take(sizeof(uint32_t) * kLCH);
        xn = take(sizeof(float) * kLCH);
        xsc = take(sizeof(float) * kLCH);
        xsig = take(sizeof(uint64_t) * kLCH);
        xslot = take(sizeof(uint16_t) * kLCH * kMaxLabels);
        buf = take(sizeof(uint64_t) * (size_t)kLQB * cb);
        xl = take((size_t)kLCH * xstride);
        total = take(16);
    }
};

template <int PREC>
struct MfmaOp;

template <>
struct MfmaOp<CAPS_PREC_BF16> {
    typedef bf16x8 T;
    static constexpr int ES = 2;
    __device__ static T load(const uint8_t *p) { return __builtin_bit_cast(T, *reinterpret_cast<const uint4 *>(p)); }
    __device__ static f32x4 mma(T a, T b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

template <>
struct MfmaOp<CAPS_PREC_FP16> {
    typedef f16x8 T;
    static constexpr int ES = 2;
    __device__ static T load(const uint8_t *p) { return __builtin_bit_cast(T, *reinterpret_cast<const uint4 *>(p)); }
    __device__ static f32x4 mma(T a, T b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

template <>
struct MfmaOp<CAPS_PREC_FP8> {
    typedef long T;
    static constexpr int ES = 1;
    __device__ static T load(const uint8_t *p) { return *reinterpret_cast<const long *>(p); }
    __device__ static f32x4 mma(T a, T b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
};

// Appends the keys of lanes with `qual` set to their queries' buffers (the
// wave owns those queries; slots come from ballots).  Bounded: every step
// appends at least one key or shrinks a full buffer to r entries.
template <int CB>
__device__ inline void append_keys(bool qual, int qi, uint64_t key, uint64_t *buf, int32_t *bcnt, uint64_t *tau,
                                   int r) {
    const int lane = threadIdx.x & 63;
    for (int guard = 0; guard < 2 * 64 + 2; guard++) {
        const uint64_t todo = __ballot(qual);
        if (!todo) break;
        const int q = __builtin_amdgcn_readlane(qi, __builtin_ctzll(todo));
        const uint64_t grp = __ballot(qual && qi == q);
        const int c = bcnt[q];
        const int room = CB - c;
        if (room <= 0) {
            wave_sync();
            buf_reduce<CB>(buf, bcnt, tau, q, r);
            if (qual && qi == q) qual = key < tau[q];
            continue;
        }
        uint64_t take = grp;
        while (__popcll(take) > room) take &= ~(1ull << (63 - __builtin_clzll(take)));
        if ((take >> lane) & 1ull) {
            buf[q * CB + c + __popcll(take & lanemask_lt())] = key;
            qual = false;
        }
        wave_sync();
        if (lane == 0) bcnt[q] = c + __popcll(take);
        wave_sync();
    }
}

template <int PREC, int METRIC, bool HAS_LABELS, int CB>
__global__ __launch_bounds__(kLNT) void k_scan_mfma(LowpArgs A) {
    typedef MfmaOp<PREC> Op;
    typedef typename Op::T VT;
    constexpr int ES = Op::ES;
    constexpr int KSTEP_BYTES = 32 * ES;                 // one MFMA K-step of a row
    constexpr int LANE_BYTES = 8 * ES;                   // one lane's slice of a K-step
    constexpr int MAXS = 8;                              // dpad <= 256
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t spo[kMaxHeight + 2];
    __shared__ uint32_t lvw[kLNW];

    const int tile = blockIdx.x;
    if (tile >= A.tstart[A.b]) return;
    int lo = 0, hi = A.b;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.tstart[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const int p = lo;
    const int i0 = (tile - A.tstart[p]) * kLQB;
    const int nqt = min(kLQB, A.pcount[p] - i0);
    const int32_t *ent = A.entries + A.pstart[p] + i0;
    const int h = A.h, r = A.r, dpad = A.dpad;
    const int nsteps = dpad / 32;
    const LowpLds L(dpad, ES, CB);
    uint8_t *xl = smem + L.xl;
    uint32_t *xw = reinterpret_cast<uint32_t *>(smem + L.xw);
    float *xn = reinterpret_cast<float *>(smem + L.xn);
    float *xsc = reinterpret_cast<float *>(smem + L.xsc);
    uint64_t *xsig = reinterpret_cast<uint64_t *>(smem + L.xsig);
    uint16_t *xslot = reinterpret_cast<uint16_t *>(smem + L.xslot);
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem + L.buf);
    int32_t *bcnt = reinterpret_cast<int32_t *>(smem + L.bcnt);
    uint64_t *tau = reinterpret_cast<uint64_t *>(smem + L.tau);
    int32_t *qslot = reinterpret_cast<int32_t *>(smem + L.qslot);
    QDesc *qds = reinterpret_cast<QDesc *>(smem + L.qd);

    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int qbase = w * kLQPW;
    const bool has_dense = A.words != nullptr;
    if (t <= h + 1) spo[t] = A.offs[(int64_t)p * (h + 1) + t];
    // per-query state (lane i < 16 of wave w: query qbase + i)
    uint32_t my_sel = 0;
    int32_t my_qq = -1;
    if (lane < kLQPW && qbase + lane < nqt) {
        const int qi = qbase + lane;
        const int32_t slot = ent[qi];
        my_qq = slot / A.m;
        my_sel = A.sel[slot];
        qslot[qi] = slot;
        qds[qi] = A.qd[my_qq];
        tau[qi] = __hip_atomic_load(A.tau + my_qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bcnt[qi] = 0;
    }
    {
        uint32_t wor = my_sel;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wor |= __shfl_xor(wor, o, 64);
        if (lane == 0) lvw[w] = wor;
    }
    // MFMA A operands: query row qbase + lane%16, K slice (lane/16)*8 of each step
    VT a[MAXS];
    {
        const int arow = qbase + (lane & 15);
        const bool aok = arow < nqt;
        const int64_t qq = aok ? (int64_t)(ent[arow] / A.m) : 0;
        const uint8_t *src = A.qlow + qq * dpad * ES + (lane >> 4) * LANE_BYTES;
#pragma unroll
        for (int s = 0; s < MAXS; s++) {
            if (s < nsteps && aok) a[s] = Op::load(src + s * KSTEP_BYTES);
            else a[s] = VT{};
        }
    }
    // per-lane epilogue state: rows (lane/16)*4 + rr are my four queries
    const int g = lane >> 4;
    uint32_t e_sel[4], e_mask[4], e_val[4];
    float e_qsc[4];
    int e_surv[4] = {0, 0, 0, 0};
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        const int qi = qbase + g * 4 + rr;
        e_sel[rr] = __builtin_amdgcn_ds_bpermute((g * 4 + rr) << 2, (int)my_sel);
        if (qi < nqt) {
            const int32_t slot = ent[qi];
            const QDesc qd = A.qd[slot / A.m];
            e_mask[rr] = qd.dmask;
            e_val[rr] = qd.dval;
            e_qsc[rr] = A.qscale[slot / A.m];
        } else {
            e_mask[rr] = 0;
            e_val[rr] = 1;   // never matches
            e_qsc[rr] = 0.0f;
        }
    }
    __syncthreads();
    uint32_t lv = 0;
#pragma unroll
    for (int i = 0; i < kLNW; i++) lv |= lvw[i];
    const int32_t *po = spo;
    auto advance = [&](int &j, int32_t &c0) {
        c0 += kLCH;
        while (j <= h && (!(lv & (1u << j)) || c0 >= po[j + 1])) {
            j++;
            if (j <= h) c0 = po[j];
        }
    };
    int cj = 0;
    int32_t cc0 = po[0] - kLCH;
    advance(cj, cc0);
    const int row_bytes = dpad * ES;
    const int xstride = L.xstride;

    while (cj <= h) {
        const int j = cj;
        const int32_t c0 = cc0;
        const int cn = min(kLCH, po[j + 1] - c0);
        __syncthreads();   // previous chunk fully consumed
        {
            const uint8_t *src = A.lvecs + (int64_t)c0 * row_bytes;
            const int n16 = cn * row_bytes / 16;
            const int per_row = row_bytes / 16;
            for (int e = t; e < n16; e += kLNT) {
                const int rrow = e / per_row, c = e - rrow * per_row;
                *reinterpret_cast<uint4 *>(xl + rrow * xstride + 16 * c) = reinterpret_cast<const uint4 *>(src)[e];
            }
            if (t < cn) {
                xw[t] = has_dense ? A.words[c0 + t] : 0u;
                xn[t] = METRIC == 0 ? A.xnorm[c0 + t] : 0.0f;
                xsc[t] = PREC == CAPS_PREC_FP8 ? A.lscale[c0 + t] : 1.0f;
                if (HAS_LABELS) {
                    xsig[t] = A.sigs[c0 + t];
                    *reinterpret_cast<uint4 *>(xslot + t * kMaxLabels) =
                        *reinterpret_cast<const uint4 *>(A.slots + (int64_t)(c0 + t) * kMaxLabels);
                }
            }
        }
        advance(cj, cc0);
        __syncthreads();

        // ---- MFMA: my 16 queries x the chunk's 64 points
        f32x4 acc[4];
#pragma unroll
        for (int bb = 0; bb < 4; bb++) {
            acc[bb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const uint8_t *xrow = xl + (bb * 16 + (lane & 15)) * xstride + (lane >> 4) * LANE_BYTES;
#pragma unroll
            for (int s = 0; s < MAXS; s++)
                if (s < nsteps) acc[bb] = Op::mma(a[s], Op::load(xrow + s * KSTEP_BYTES), acc[bb]);
        }
        // ---- epilogue: exact filter, approximate key, threshold; keys that
        // beat their query's threshold are appended (rare once bounds are tight)
        float esc[16];
        uint32_t qmask = 0;
#pragma unroll
        for (int bb = 0; bb < 4; bb++) {
            const int pi = bb * 16 + (lane & 15);
            const bool pok = pi < cn;
            const uint32_t pw = pok ? xw[pi] : 0u;
            const float pn = pok ? xn[pi] : 0.0f;
            const float ps = pok ? xsc[pi] : 0.0f;
            const uint64_t psig = (HAS_LABELS && pok) ? xsig[pi] : 0ull;
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const int qi = qbase + g * 4 + rr;
                bool pass = pok && ((e_sel[rr] >> j) & 1u);
                if (HAS_LABELS) {
                    if (pass) pass = point_passes(qds[qi], has_dense, true, pw, psig, xslot + pi * kMaxLabels);
                } else {
                    pass = pass && ((pw & e_mask[rr]) == e_val[rr]);
                }
                float dot = acc[bb][rr];
                if (PREC == CAPS_PREC_FP8) dot = dot * ps * e_qsc[rr];
                const float sc = canon0(METRIC == 0 ? pn - 2.0f * dot : -dot);
                esc[bb * 4 + rr] = sc;
                e_surv[rr] += pass ? 1 : 0;
                const uint64_t key = ((uint64_t)f2ord(sc) << 32) | (uint32_t)(c0 + pi);
                if (pass && key < tau[qi]) qmask |= 1u << (bb * 4 + rr);
            }
        }
        uint32_t anyq = qmask;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) anyq |= __shfl_xor(anyq, o, 64);
        if (anyq) {
#pragma unroll
            for (int e = 0; e < 16; e++) {   // wave-uniform test per element
                if (!((anyq >> e) & 1u)) continue;
                const int bb = e >> 2, rr = e & 3;
                const int qi = qbase + g * 4 + rr;
                const uint64_t key = ((uint64_t)f2ord(esc[e]) << 32) | (uint32_t)(c0 + bb * 16 + (lane & 15));
                const bool qual = ((qmask >> e) & 1u) && key < tau[qi];
                append_keys<CB>(qual, qi, key, buf, bcnt, tau, r);
            }
        }
    }
    // ---- survivors per query: sum over the 16 lanes that share a row group
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        int v = e_surv[rr];
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        const int qi = qbase + g * 4 + rr;
        if ((lane & 15) == 0 && qi < nqt && v) atomicAdd(&A.nsurv[qslot[qi] / A.m], v);
    }
    // ---- finalize my queries: best r sorted, partial list, shared bound
    for (int i = 0; i < kLQPW; i++) {
        const int qi = qbase + i;
        if (qi >= nqt) break;
        buf_reduce<CB>(buf, bcnt, tau, qi, r);
        const int c = bcnt[qi];
        const int32_t slot = qslot[qi];
        uint64_t *out = A.partials + (int64_t)slot * r;
        if (lane < c) out[lane] = buf[qi * CB + lane];
        if (lane == 0) {
            A.pcnt[slot] = c;
            if (c == r) atomicMin((unsigned long long *)(A.tau + slot / A.m), (unsigned long long)buf[qi * CB + r - 1]);
        }
    }
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
        const float *xr = vecs + (int64_t)pos * d;
        const float *qr = q + (int64_t)qq * d;
        float acc = 0.0f;
        for (int jj = 0; jj < d; jj++) {
            if (METRIC == 0) {
                const float t0 = xr[jj] - qr[jj];
                acc = fmaf(t0, t0, acc);
            } else {
                acc = fmaf(xr[jj], qr[jj], acc);
            }
        }
        const float kf = canon0(METRIC == 0 ? acc : -acc);
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
typedef void (*LowpFn)(LowpArgs);

template <int PREC, int METRIC, bool LAB>
static LowpFn pick_cb(int r) {
    if (r <= 48) return k_scan_mfma<PREC, METRIC, LAB, 64>;
    return k_scan_mfma<PREC, METRIC, LAB, 128>;
}

template <int PREC>
static LowpFn pick_ml(int metric, bool lab, int r) {
    if (metric == 0) return lab ? pick_cb<PREC, 0, true>(r) : pick_cb<PREC, 0, false>(r);
    return lab ? pick_cb<PREC, 1, true>(r) : pick_cb<PREC, 1, false>(r);
}

static LowpFn pick_lowp(int prec, int metric, bool lab, int r) {
    if (prec == CAPS_PREC_BF16) return pick_ml<CAPS_PREC_BF16>(metric, lab, r);
    if (prec == CAPS_PREC_FP16) return pick_ml<CAPS_PREC_FP16>(metric, lab, r);
    return pick_ml<CAPS_PREC_FP8>(metric, lab, r);
}

size_t lowp_scan_lds(const Index *ix, int r) {
    return LowpLds(ix->dpad, esize_of(ix->prec), r <= 48 ? 64 : 128).total + 64;
}

caps_status lowp_scan(const Index *ix, int32_t nb, const int32_t *tstart, const int32_t *pstart,
                      const int32_t *pcount, const int32_t *entries, const uint32_t *sel, const QDesc *qd,
                      int32_t m, int32_t r, void *qlow, float *qscale, uint64_t *partials, int32_t *pcnt,
                      uint64_t *tau, int32_t *nsurv, int32_t max_tiles, bool first_round, const float *q,
                      hipStream_t st) {
    if (first_round)
        hipLaunchKernelGGL(k_qquant, dim3((nb + 127) / 128), dim3(128), 0, st, q, nb, ix->d, ix->dpad, ix->prec,
                           qlow, qscale);
    LowpArgs A;
    A.tstart = tstart;
    A.pstart = pstart;
    A.pcount = pcount;
    A.entries = entries;
    A.sel = sel;
    A.qd = qd;
    A.offs = ix->offs;
    A.lvecs = reinterpret_cast<const uint8_t *>(ix->lvecs);
    A.lscale = ix->lscale;
    A.xnorm = ix->xnorm;
    A.words = ix->words;
    A.sigs = ix->sigs;
    A.slots = ix->slots;
    A.qlow = reinterpret_cast<const uint8_t *>(qlow);
    A.qscale = qscale;
    A.partials = partials;
    A.pcnt = pcnt;
    A.tau = tau;
    A.nsurv = nsurv;
    A.dpad = ix->dpad;
    A.m = m;
    A.h = ix->h;
    A.b = ix->b;
    A.r = r;
    const LowpFn fn = pick_lowp(ix->prec, ix->metric, ix->sch.label_vocab > 0, r);
    const size_t lds = lowp_scan_lds(ix, r);
    CAPS_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    prof_begin(CAPS_STAGE_SCAN, st);
    hipLaunchKernelGGL(fn, dim3((unsigned)max_tiles), dim3(kLNT), lds, st, A);
    prof_end(CAPS_STAGE_SCAN, st);
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

}  // namespace caps
