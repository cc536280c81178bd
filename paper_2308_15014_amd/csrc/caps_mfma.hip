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
    // rows padded to 32 x {1, 2, 4, 8} coordinates: the scan kernels are
    // specialised on the number of 32-wide MFMA K-steps
    int ns = 1;
    while (32 * ns < ix->d) ns <<= 1;
    ix->dpad = 32 * ns;
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
    int32_t *nsurv;             // per query survivor counts, or null (not counted)
    int32_t m, h, b, r, metric;
};

constexpr int kLNW = 4;          // waves per tile
constexpr int kLQPW = 16;        // queries per wave (MFMA rows)
constexpr int kLQB = kLNW * kLQPW;
constexpr int kLCH = 64;         // points per chunk: four 16-column MFMA blocks
constexpr int kLNT = kLNW * 64;
constexpr int kTauRefresh = 8;   // chunks between reads of the shared per-query bounds

struct LowpLds {
    size_t xl, xw, xn, xsc, buf, bcnt, tau, qslot, qd, total;
    __host__ __device__ constexpr LowpLds(int row_bytes, int cb)
        : xl(0), xw(0), xn(0), xsc(0), buf(0), bcnt(0), tau(0), qslot(0), qd(0), total(0) {
        size_t o = 0;
        const auto take = [&o](size_t bytes) {
            o = (o + 15) & ~(size_t)15;
            const size_t r = o;
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
        buf = take(sizeof(uint64_t) * (size_t)kLQB * cb);
        xl = take((size_t)kLCH * (row_bytes + 16));
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

// Float image of a bound key: every key below the bound has a score <= it.
__device__ inline float bound_score(uint64_t t) {
    return t == ~0ull ? __builtin_huge_valf() : ord2f((uint32_t)(t >> 32));
}

// One tile = one partition x up to 64 of the (query, probe) entries that
// route to it.  Wave w owns queries 16w..16w+15: their A operands sit in
// registers, their candidate buffers and bounds in LDS.  Chunks of 64 CSR
// rows of the levels any of the tile's queries selected are staged in LDS
// (the next chunk's loads are in flight while the current one is scored).
// Per element the epilogue is branch free: one fused score, a compare against
// the row's cached float bound (NaN for a row whose query skips the chunk's
// level or has no query, NaN score for a padding column, so neither ever
// compares true) and the packed dense-attribute test, reduced by ballots.
// Exact keys, label tests and appends run only for elements that pass.
template <int PREC, bool HAS_LABELS, int CB, int NS>
__global__ __launch_bounds__(kLNT) void k_scan_mfma(LowpArgs A) {
    typedef MfmaOp<PREC> Op;
    typedef typename Op::T VT;
    constexpr int ES = Op::ES;
    constexpr int KSTEP_BYTES = 32 * ES;                 // one MFMA K-step of a row
    constexpr int LANE_BYTES = 8 * ES;                   // one lane's slice of a K-step
    constexpr int ROWB = NS * KSTEP_BYTES;               // bytes per CSR row of the copy
    constexpr int XSTRIDE = ROWB + 16;                   // padded LDS row (bank spread)
    constexpr int V16 = ROWB / 16;                       // 16-byte pieces per row
    constexpr int PIECES = kLCH * V16;
    constexpr int UPT = (PIECES + kLNT - 1) / kLNT;      // pieces per thread per chunk
    constexpr LowpLds L(ROWB, CB);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t spo[kMaxHeight + 2];
    __shared__ uint32_t lvw[kLNW];

    const int tile = xcd_tile(blockIdx.x, A.tstart[A.b]);
    if (tile < 0) return;
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
    const int h = A.h, r = A.r;
    uint8_t *xl = smem + L.xl;
    uint32_t *xw = reinterpret_cast<uint32_t *>(smem + L.xw);
    float *xn = reinterpret_cast<float *>(smem + L.xn);
    float *xsc = reinterpret_cast<float *>(smem + L.xsc);
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem + L.buf);
    int32_t *bcnt = reinterpret_cast<int32_t *>(smem + L.bcnt);
    uint64_t *tau = reinterpret_cast<uint64_t *>(smem + L.tau);
    int32_t *qslot = reinterpret_cast<int32_t *>(smem + L.qslot);
    QDesc *qds = reinterpret_cast<QDesc *>(smem + L.qd);

    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int qbase = w * kLQPW;
    const bool has_dense = A.words != nullptr;
    const bool l2 = A.metric == 0;
    const bool count = A.nsurv != nullptr;
    const float qnan = __builtin_nanf("");
    const float cm = l2 ? -2.0f : -1.0f;   // score = cm * dot + |x|^2 (L2) or + 0 (IP)
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
        if (HAS_LABELS) qds[qi] = A.qd[my_qq];
        tau[qi] = __hip_atomic_load(A.tau + my_qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane < kLQPW) bcnt[qbase + lane] = 0;   // rows without a query too
    {
        uint32_t wor = my_sel;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wor |= __shfl_xor(wor, o, 64);
        if (lane == 0) lvw[w] = wor;
    }
    // MFMA A operands: query row qbase + lane%16, K slice (lane/16)*8 of each step
    VT a[NS];
    {
        const int arow = qbase + (lane & 15);
        const bool aok = arow < nqt;
        const int64_t qq = aok ? (int64_t)(ent[arow] / A.m) : 0;
        const uint8_t *src = A.qlow + qq * ROWB + (lane >> 4) * LANE_BYTES;
#pragma unroll
        for (int s = 0; s < NS; s++) a[s] = aok ? Op::load(src + s * KSTEP_BYTES) : VT{};
    }
    // per-lane epilogue rows: (lane/16)*4 + rr of the wave's 16 queries
    const int g = lane >> 4;
    uint32_t rsel[4], rmask[4], rval[4];
    float rqs[4], rtf[4];
    int rsurv[4] = {0, 0, 0, 0};
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        const int qi = qbase + g * 4 + rr;
        rsel[rr] = __builtin_amdgcn_ds_bpermute((g * 4 + rr) << 2, (int)my_sel);
        if (qi < nqt) {
            const int32_t qq = ent[qi] / A.m;
            const QDesc qd = A.qd[qq];
            rmask[rr] = qd.dmask;
            rval[rr] = qd.dval;
            rqs[rr] = PREC == CAPS_PREC_FP8 ? A.qscale[qq] : 1.0f;
        } else {
            rmask[rr] = 0;
            rval[rr] = 1;   // never matches
            rqs[rr] = 0.0f;
        }
    }
    __syncthreads();
    auto refresh_bounds = [&]() {
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const int qi = qbase + g * 4 + rr;
            rtf[rr] = qi < nqt ? bound_score(tau[qi]) : qnan;
        }
    };
    refresh_bounds();
    uint32_t lv = 0;
#pragma unroll
    for (int i = 0; i < kLNW; i++) lv |= lvw[i];
    lv = __builtin_amdgcn_readfirstlane(lv);
    // chunk cursor (wave-uniform, kept in scalar registers): level j, first
    // row c0 of the chunk, end of the level
    auto po = [&](int i) { return __builtin_amdgcn_readfirstlane(spo[i]); };
    auto next_level = [&](int &j, int32_t &c0, int32_t &end) {
        for (j++; j <= h; j++) {
            if (!((lv >> j) & 1u)) continue;
            c0 = po(j);
            end = po(j + 1);
            if (c0 < end) return;
        }
    };
    auto advance = [&](int &j, int32_t &c0, int32_t &end) {
        c0 += kLCH;
        if (c0 >= end) next_level(j, c0, end);
    };

    // register staging of one chunk: UPT 16-byte pieces per thread, plus the
    // per-point word / norm / scale held by the first 64 threads.  Rows past
    // the level's end load the level's last row (in bounds); their columns are
    // masked by a NaN norm.
    typedef uint32_t PreT __attribute__((ext_vector_type(4 * UPT)));   // stays in VGPRs
    PreT pre = {};
    uint32_t pre_w = 0;
    float pre_n = qnan, pre_s = 1.0f;
    auto fetch = [&](int32_t c0, int cn) {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.lvecs + (int64_t)c0 * ROWB);
#pragma unroll
        for (int u = 0; u < UPT; u++) {
            const int e = t + u * kLNT;
            if (PIECES % kLNT == 0 || e < PIECES) {
                const int row = min(e / V16, cn - 1);
                const uint4 v = src[row * V16 + e % V16];
                pre[4 * u + 0] = v.x;
                pre[4 * u + 1] = v.y;
                pre[4 * u + 2] = v.z;
                pre[4 * u + 3] = v.w;
            }
        }
        if (t < kLCH) {
            const int row = c0 + min(t, cn - 1);
            const float xn2 = l2 ? A.xnorm[row] : 0.0f;
            pre_w = has_dense ? A.words[row] : 0u;
            pre_n = t < cn ? xn2 : qnan;
            if (PREC == CAPS_PREC_FP8) pre_s = A.lscale[row];
        }
    };

    int cj = -1;
    int32_t cc0 = 0, cend = 0;
    next_level(cj, cc0, cend);
    if (cj <= h) fetch(cc0, min(kLCH, cend - cc0));
    int nchunk = 0;

    while (cj <= h) {
        const int j = cj;
        const int32_t c0 = cc0;
        const int cn = min(kLCH, cend - c0);
        __syncthreads();   // previous chunk fully consumed
#pragma unroll
        for (int u = 0; u < UPT; u++) {
            const int e = t + u * kLNT;
            if (PIECES % kLNT == 0 || e < PIECES)
                *reinterpret_cast<uint4 *>(xl + (e / V16) * XSTRIDE + (e % V16) * 16) =
                    make_uint4(pre[4 * u], pre[4 * u + 1], pre[4 * u + 2], pre[4 * u + 3]);
        }
        if (t < kLCH) {
            xw[t] = pre_w;
            xn[t] = pre_n;
            xsc[t] = pre_s;
        }
        const bool refresh = (++nchunk % kTauRefresh) == 0;
        if (refresh && lane < kLQPW && my_qq >= 0) {
            const uint64_t gt = __hip_atomic_load(A.tau + my_qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (gt < tau[qbase + lane]) tau[qbase + lane] = gt;
        }
        advance(cj, cc0, cend);
        if (cj <= h) fetch(cc0, min(kLCH, cend - cc0));
        __syncthreads();
        if (refresh) refresh_bounds();

        // ---- MFMA: my 16 queries x the chunk's 64 points
        f32x4 acc[4];
#pragma unroll
        for (int bb = 0; bb < 4; bb++) acc[bb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const uint8_t *xb = xl + (lane & 15) * XSTRIDE + (lane >> 4) * LANE_BYTES;
#pragma unroll
        for (int s = 0; s < NS; s++)
#pragma unroll
            for (int bb = 0; bb < 4; bb++)
                acc[bb] = Op::mma(a[s], Op::load(xb + bb * 16 * XSTRIDE + s * KSTEP_BYTES), acc[bb]);

        // ---- epilogue, one 16-point block at a time
        float tfj[4];
#pragma unroll
        for (int rr = 0; rr < 4; rr++) tfj[rr] = ((rsel[rr] >> j) & 1u) ? rtf[rr] : qnan;
#pragma unroll
        for (int bb = 0; bb < 4; bb++) {
            const int pi = bb * 16 + (lane & 15);
            const uint32_t pw = xw[pi];
            const float pn = xn[pi];
            const float ps = xsc[pi];
            float esc[4];
            uint64_t hit[4];
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                float dd = acc[bb][rr];
                if (PREC == CAPS_PREC_FP8) dd = dd * ps * rqs[rr];
                esc[rr] = fmaf(cm, dd, pn);
                // two single-compare ballots: each is one v_cmp into an SGPR pair
                hit[rr] = __builtin_amdgcn_ballot_w64(esc[rr] <= tfj[rr]) &
                          __builtin_amdgcn_ballot_w64((pw & rmask[rr]) == rval[rr]);
            }
            if (count) {   // survivors of the exact filter (statistics only)
#pragma unroll
                for (int rr = 0; rr < 4; rr++) {
                    bool ok = pi < cn && ((rsel[rr] >> j) & 1u) && (pw & rmask[rr]) == rval[rr];
                    if (HAS_LABELS && ok) {
                        const int qi = qbase + g * 4 + rr;
                        ok = point_passes(qds[qi], false, true, 0u, A.sigs[c0 + pi],
                                          A.slots + (int64_t)(c0 + pi) * kMaxLabels);
                    }
                    rsurv[rr] += ok ? 1 : 0;
                }
            }
            if (hit[0] | hit[1] | hit[2] | hit[3]) {
                bool reduced = false;
#pragma unroll
                for (int rr = 0; rr < 4; rr++) {   // wave-uniform test per row group
                    if (!hit[rr]) continue;
                    // lanes 16g..16g+15 hold row 4g+rr: one query per 16-lane group
                    const int qi = qbase + g * 4 + rr;
                    bool qual = (hit[rr] >> lane) & 1ull;
                    if (HAS_LABELS && qual)
                        qual = point_passes(qds[qi], false, true, 0u, A.sigs[c0 + pi],
                                            A.slots + (int64_t)(c0 + pi) * kMaxLabels);
                    // the score bound admits ties with the current bound key;
                    // such keys are no better than it and never reach the final r
                    const uint64_t key = ((uint64_t)f2ord(canon0(esc[rr])) << 32) | (uint32_t)(c0 + pi);
                    const uint64_t gm = __builtin_amdgcn_ballot_w64(qual) & (0xFFFFull << (16 * g));
                    const int cnt = __popcll(gm);
                    const int c = bcnt[qi];
                    if (__builtin_amdgcn_ballot_w64(c + cnt > CB) == 0) {
                        // every group's keys fit: direct slots, one count update per group
                        if (qual) buf[qi * CB + c + __popcll(gm & lanemask_lt())] = key;
                        if ((lane & 15) == 0 && cnt) bcnt[qi] = c + cnt;
                        wave_sync();
                    } else {
                        wave_sync();
                        append_keys<CB>(qual, qi, key, buf, bcnt, tau, r);
                        reduced = true;
                    }
                }
                if (reduced) {   // a full buffer was cut back to r keys: bounds moved
                    refresh_bounds();
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) tfj[rr] = ((rsel[rr] >> j) & 1u) ? rtf[rr] : qnan;
                }
            }
        }
    }
    // ---- survivors per query: sum over the 16 lanes that share a row group
    if (count) {
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            int v = rsurv[rr];
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            const int qi = qbase + g * 4 + rr;
            if ((lane & 15) == 0 && qi < nqt && v) atomicAdd(&A.nsurv[qslot[qi] / A.m], v);
        }
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

template <int PREC, bool LAB, int NS>
static LowpFn pick_cb(int r) {
    if (r <= 48) return k_scan_mfma<PREC, LAB, 64, NS>;
    return k_scan_mfma<PREC, LAB, 128, NS>;
}

template <int PREC, int NS>
static LowpFn pick_lab(bool lab, int r) {
    return lab ? pick_cb<PREC, true, NS>(r) : pick_cb<PREC, false, NS>(r);
}

template <int PREC>
static LowpFn pick_ns(int ns, bool lab, int r) {
    switch (ns) {
        case 1: return pick_lab<PREC, 1>(lab, r);
        case 2: return pick_lab<PREC, 2>(lab, r);
        case 4: return pick_lab<PREC, 4>(lab, r);
        default: return pick_lab<PREC, 8>(lab, r);
    }
}

static LowpFn pick_lowp(int prec, int ns, bool lab, int r) {
    if (prec == CAPS_PREC_BF16) return pick_ns<CAPS_PREC_BF16>(ns, lab, r);
    if (prec == CAPS_PREC_FP16) return pick_ns<CAPS_PREC_FP16>(ns, lab, r);
    return pick_ns<CAPS_PREC_FP8>(ns, lab, r);
}

size_t lowp_scan_lds(const Index *ix, int r) {
    return LowpLds(ix->dpad * esize_of(ix->prec), r <= 48 ? 64 : 128).total + 64;
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
    A.m = m;
    A.h = ix->h;
    A.b = ix->b;
    A.r = r;
    A.metric = ix->metric;
    const LowpFn fn = pick_lowp(ix->prec, ix->dpad / 32, ix->sch.label_vocab > 0, r);
    const size_t lds = lowp_scan_lds(ix, r);
    CAPS_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    prof_begin(CAPS_STAGE_SCAN, st);
    const int32_t grid = (max_tiles + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kLNT), lds, st, A);
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
