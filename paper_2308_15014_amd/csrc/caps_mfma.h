// Matrix-core scan kernel (internal): the tile kernel template shared by
// the host dispatch in caps_mfma.hip and the per-precision instantiation
// units (caps_scan_inst.hip, compiled once per precision and key kind).
#pragma once

#include <math.h>

#include "caps_device.h"
#include "caps_internal.h"

namespace caps {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ scan
struct LowpArgs {
    const int4 *tiles;          // per tile: partition, first entry, entries (0: no tile)
    const int32_t *entries;
    const uint32_t *esel;       // level mask per entry, in entry order (null: read sel by slot)
    const uint32_t *sel;
    const QDesc *qd;
    const QDesc *qterms;        // disjunctive searches: kMaxTerms term descriptors per query
    const int32_t *offs;
    const uint8_t *lvecs;       // CSR rows of dpad elements
    const float *lscale, *xnorm, *lerr, *lnrm;
    const uint32_t *words;
    const uint64_t *sigs;
    const uint16_t *slots;
    int32_t lslots;             // label slots per point
    const uint8_t *qlow;        // query rows of dpad elements
    const float *qscale, *qaux;
    const float *vecs, *q;      // FP32 CSR rows and queries (exact rescoring)
    const int32_t *perm;
    uint64_t *partials;         // per (query, probe): up to r keys
    int32_t *pcnt;              // keys written per (query, probe) (sorted, at most r; the exact main pass writes none)
    uint64_t *tau;              // per query: shared bound on its r-th key
    int32_t *nsurv;             // per query survivor counts, or null (not counted)
    uint64_t *dpos;             // exact: per query deferred pairs, (ordered score of the element test << 32) | CSR position
    int32_t *dcnt;              // exact: their count per query
    int32_t *oflow;             // exact: per query flag, set when its pairs did not fit (rescue pass input)
    const int32_t *rlist, *rcount;   // rescue pass: tiles with a flagged query and their number
    int32_t m, h, b, r, metric, d, dcap, ntiles;   // ntiles: length of `tiles` (the grid's tile range)
    int32_t rhalves;            // rescue pass over 128-entry tiles: list entries are 2 tile + half
    float eta, gam;             // exact: relative rounding margin, MFMA accumulation bound
};

constexpr int kLNW = 4;          // waves per tile
constexpr int kLQPW = 16;        // queries per wave (MFMA rows)
constexpr int kLQB = kLNW * kLQPW;
constexpr int kLCH = 64;         // points per chunk: four 16-column MFMA blocks
constexpr int kLNT = kLNW * 64;
constexpr int kTauRefresh = 8;   // chunks between reads of the shared per-query bounds
constexpr int kVRing = 128;      // exact: per-wave ring of pairs awaiting rescoring

struct LowpLds {
    size_t xw, xn, xsc, buf, bcnt, tau, qslot, qd, ring, dhist, qnq, scnt, total;
    // kind: 0 approximate keys, 1 exact main pass (no buffers), 2 exact rescue
    // pass, 3 exact main pass counting the survivors of the filter.
    // The chunk tiles themselves are static arrays of the kernel (two of
    // kLCH rows); the per-point arrays here are double buffered alike.
    __host__ __device__ constexpr LowpLds(int cb, int kind, bool labels)
        : xw(0), xn(0), xsc(0), buf(0), bcnt(0), tau(0), qslot(0), qd(0), ring(0), dhist(0), qnq(0), scnt(0),
          total(0) {
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
        qd = take(labels ? sizeof(QDesc) * kLQB : 0);
        xw = take(sizeof(uint32_t) * 2 * kLCH);
        xn = take(sizeof(float) * 2 * kLCH);
        xsc = take(sizeof(float) * 2 * kLCH);
        ring = take(kind != 0 ? sizeof(uint32_t) * (kind == 1 || kind == 3 ? 3 : 2) * kLNW * kVRing : 0);
        dhist = take(kind == 1 || kind == 3 ? sizeof(int32_t) * kLNW * kLQPW : 0);
        qnq = take(kind != 0 ? sizeof(float) * kLQB : 0);
        scnt = take(sizeof(int32_t) * kLQB);
        buf = take(kind == 1 || kind == 3 ? 0 : sizeof(uint64_t) * (size_t)kLQB * cb);
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

// Exact FP32 score of one pair: the sequential fma over ascending
// coordinates of the plain scan (L2: sum (x_j - q_j)^2; IP: -sum x_j q_j).
// Rows of a multiple of 4 go in batches of XB float4 loads per row, all
// issued before the batch is summed, so one pair costs d / (4 XB) memory
// round trips instead of d / 4; the summation order is unchanged.
template <int XB>
__device__ inline float exact_score(const float *__restrict__ xr, const float *__restrict__ qr, int d, bool l2) {
    float acc = 0.0f;
    auto add4 = [&](const float4 xv, const float4 qv) {
        if (l2) {
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
    };
    if ((d & 3) == 0) {
        const float4 *x4 = reinterpret_cast<const float4 *>(xr);
        const float4 *q4 = reinterpret_cast<const float4 *>(qr);
        const int d4 = d >> 2;
        int j = 0;
        for (; j + XB <= d4; j += XB) {
            float4 xv[XB], qv[XB];
#pragma unroll
            for (int u = 0; u < XB; u++) {
                xv[u] = x4[j + u];
                qv[u] = q4[j + u];
            }
#pragma unroll
            for (int u = 0; u < XB; u++) add4(xv[u], qv[u]);
        }
        for (; j < d4; j++) add4(x4[j], q4[j]);
    } else {
        for (int j = 0; j < d; j++) {
            if (l2) {
                const float t0 = xr[j] - qr[j];
                acc = fmaf(t0, t0, acc);
            } else {
                acc = fmaf(xr[j], qr[j], acc);
            }
        }
    }
    return canon0(l2 ? acc : -acc);
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
// Label tests and buffer updates run only for elements that pass.
//
// EXACT: the per-point term of the score is |x|^2 (IP: 0) lowered by the
// error norms against the tile's largest query norms and a relative margin,
// the per-row bound is the query's k-th exact key raised by the margin, so
// that an element fails only if its exact FP32 key is above the bound.
// Passing elements queue in a per-wave ring.  Taken 64 at a time, they are
// rescored exactly and enter the buffers with their exact keys (distance,
// point id); or, when the launch has deferred lists (later probes, whose
// bounds rarely tighten within a tile), they are appended to their queries'
// lists in global memory and rescored by the merge, which overlaps many
// more of the row reads than one tile can.
// HAS_LABELS selects the variant with the filter's slow path (label tests on
// indexes with labels, the terms of disjunctive searches on any index).
// Register budget per SIMD: four waves (at most 128 VGPRs) for the exact
// main pass up to 128-element rows without label tests (it keeps no key
// buffers), three for the approximate kind, two for the rescue pass (few
// tiles, looped) and with label tests or longer rows (their state does not
// fit).
template <int PREC, bool HAS_LABELS, int CB, int NS, int KIND>
__global__ __launch_bounds__(kLNT) __attribute__((amdgpu_waves_per_eu(NS >= 8 || HAS_LABELS || KIND == 2 ? 2 : KIND == 1 || KIND == 3 ? 4 : 3))) void k_scan_mfma(
    LowpArgs A) {
    constexpr bool EXACT = KIND != 0;    // exact keys (bounds + exact rescoring)
    constexpr bool DEFER = KIND == 1 || KIND == 3;   // main pass: passing pairs go to the deferred lists
    constexpr bool RESCUE = KIND == 2;   // rescue pass: flagged queries only, rescored here
    typedef MfmaOp<PREC> Op;
    typedef typename Op::T VT;
    constexpr int ES = Op::ES;
    constexpr int KSTEP_BYTES = 32 * ES;                 // one MFMA K-step of a row
    constexpr int LANE_BYTES = 8 * ES;                   // one lane's slice of a K-step
    constexpr int ROWB = NS * KSTEP_BYTES;               // bytes per CSR row of the copy
    constexpr int V16 = ROWB / 16;                       // 16-byte pieces per row (a power of two)
    constexpr int NDMA = V16;                            // 1 KB direct loads per chunk (64 lanes x 16 B)
    constexpr int UPW = (NDMA + kLNW - 1) / kLNW;        // of them per wave
    // Tile rows are unpadded; piece p of row r sits at position p ^ swz(r), so
    // that the 16 rows one operand read touches (same K slice) fall in
    // distinct banks: rows of >= 256 bytes XOR their low four row bits,
    // shorter rows (RPL of them share a 256-byte bank line) the bits above.
    constexpr int RPL = ROWB >= 256 ? 1 : 256 / ROWB;
    constexpr int SWZ = ROWB >= 256 ? 15 : V16 - 1;
    constexpr LowpLds L(CB, KIND, HAS_LABELS);
    extern __shared__ __align__(16) unsigned char smem[];
    // the two chunk tiles (ping-pong): distinct arrays, so that the compiler
    // can tell the reads of one from the direct loads into the other
    __shared__ __align__(16) uint8_t xt0[kLCH * ROWB];
    __shared__ __align__(16) uint8_t xt1[kLCH * ROWB];
    __shared__ int32_t spo[kMaxHeight + 2];
    __shared__ uint32_t lvw[kLNW];
    __shared__ float qmx[2][kLNW];

    // one tile per workgroup; the rescue pass (a small grid) walks the list
    // of tiles that hold a flagged query, written by k_rescue_tiles, with a
    // workgroup barrier between consecutive tiles.
    auto run_tile = [&](int4 dsc) {
    if (dsc.z <= 0) return;
    const int p = dsc.x;
    const int nqt = dsc.z;
    const int32_t *ent = A.entries + dsc.y;
    const int h = A.h, r = A.r;
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
    uint32_t *ring_pos = reinterpret_cast<uint32_t *>(smem + L.ring) + w * (DEFER ? 3 : 2) * kVRing;
    uint32_t *ring_row = ring_pos + kVRing;
    uint32_t *ring_key = ring_row + kVRing;   // deferring kinds: the pair's ordered score
    int32_t *dhist = reinterpret_cast<int32_t *>(smem + L.dhist) + w * kLQPW;
    float *qnq = reinterpret_cast<float *>(smem + L.qnq);          // exact: |q|^2 per query
    int32_t *scnt = reinterpret_cast<int32_t *>(smem + L.scnt);    // survivors per query (counted runs)
    const bool has_dense = A.words != nullptr;
    const bool has_lab = A.sigs != nullptr;
    const bool l2 = A.metric == 0;
    // survivor counts: the main pass has a counting kind of its own, so that
    // the uncounted one tests the packed dense fields only where a score passed
    const bool count = KIND == 3 ? true : KIND == 1 ? false : A.nsurv != nullptr;
    const float qnan = __builtin_nanf("");
    const float inf = __builtin_huge_valf();
    const float cm = l2 ? -2.0f : -1.0f;   // score = cm * dot + per-point term
    if (t <= h + 1) spo[t] = A.offs[(int64_t)p * (h + 1) + t];
    // per-query state (lane i < 16 of wave w: query qbase + i)
    uint32_t my_sel = 0;
    int32_t my_qq = -1;
    if (lane < kLQPW && qbase + lane < nqt) {
        const int qi = qbase + lane;
        const int32_t slot = ent[qi];
        const int32_t qq = slot / A.m;
        qslot[qi] = slot;
        if (!RESCUE || A.oflow[qq]) {   // the rescue pass takes flagged queries only
            my_qq = qq;
            my_sel = A.sel[slot];
            if (HAS_LABELS) qds[qi] = A.qd[my_qq];
            tau[qi] = __hip_atomic_load(A.tau + my_qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // rows with a query to scan: bit i for row qbase + i
    const uint32_t active = (uint32_t)__builtin_amdgcn_ballot_w64(lane < kLQPW && my_qq >= 0);
    if (lane < kLQPW) {   // rows without a query too
        bcnt[qbase + lane] = 0;
        scnt[qbase + lane] = 0;
        if (EXACT) qnq[qbase + lane] = my_qq >= 0 ? A.qaux[4 * (int64_t)my_qq + 1] : 0.0f;
    }
    // levels every active row of the wave selects (wave-uniform): a chunk of
    // such a level keeps the row bounds as they are
    uint32_t wall;
    {
        uint32_t wor = my_sel;
        wall = lane < kLQPW && my_qq >= 0 ? my_sel : ~0u;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            wor |= __shfl_xor(wor, o, 64);
            wall &= __shfl_xor(wall, o, 64);
        }
        if (lane == 0) lvw[w] = wor;
        wall = __builtin_amdgcn_readfirstlane(wall);
    }
    if (RESCUE) {   // leave early when no query of the tile is flagged (uniform)
        __syncthreads();
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < kLNW; i++) any |= lvw[i];
        if (any == 0) return;
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
    // MFMA B operands: row lane%16 of each 16-row block, K slice g of each
    // step; per step the lane's byte offset in a tile (same for every block,
    // whose 16 rows span whole swizzle periods)
    uint32_t xoff[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int r16 = lane & 15;
        const int byte = s * KSTEP_BYTES + g * LANE_BYTES;
        xoff[s] = (uint32_t)(r16 * ROWB + 16 * ((byte / 16) ^ ((r16 / RPL) & SWZ)) + byte % 16);
    }
    uint32_t rmask[4], rval[4];
    // level mask of epilogue row rr of this lane (read from the row's lane
    // when needed: rare, so it is not kept in registers)
    auto rsel = [&](int rr) { return (uint32_t)__builtin_amdgcn_ds_bpermute((g * 4 + rr) << 2, (int)my_sel); };
    float rqs[4], rtf[4];
    float qa = 0.0f, qb = 0.0f;   // exact: largest |q| and |q - q~| + gam |q~| of my rows
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        const int qi = qbase + g * 4 + rr;
        if ((active >> (g * 4 + rr)) & 1u) {
            const int32_t qq = ent[qi] / A.m;
            const QDesc qd = A.qd[qq];
            rmask[rr] = qd.dmask;
            rval[rr] = qd.dval;
            rqs[rr] = PREC == CAPS_PREC_FP8 ? A.qscale[qq] : 1.0f;
            if (EXACT) {
                const float4 ax = *reinterpret_cast<const float4 *>(A.qaux + 4 * (int64_t)qq);
                qa = fmaxf(qa, ax.x);
                qb = fmaxf(qb, fmaf(A.gam, ax.w, ax.z));
            }
        } else {
            rmask[rr] = 0;
            rval[rr] = 1;   // never matches
            rqs[rr] = 0.0f;
        }
    }
    if (EXACT) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            qa = fmaxf(qa, __shfl_xor(qa, o, 64));
            qb = fmaxf(qb, __shfl_xor(qb, o, 64));
        }
        if (lane == 0) {
            qmx[0][w] = qa;
            qmx[1][w] = qb;
        }
    }
    __syncthreads();
    if (EXACT) {
#pragma unroll
        for (int i = 0; i < kLNW; i++) {
            qa = fmaxf(qa, qmx[0][i]);
            qb = fmaxf(qb, qmx[1][i]);
        }
    }
    // Row bound for the element test.  EXACT, L2: an element passes when
    // pl - 2 x~.q~ <= tauD - |q|^2 + eta (|q|^2 + tauD); IP: pl - x~.q~ <=
    // tauD + eta (|q|^2 + |tauD|) (pl: the point term of the staging step,
    // tauD: the score of the query's bound key).
    auto row_bound = [&](uint64_t tk, float nq) {
        const float td = bound_score(tk);
        if (!EXACT) return td;
        if (!(td < inf)) return inf;
        return l2 ? fmaf(A.eta, nq + td, td - nq) + 1e-37f : fmaf(A.eta, nq + fabsf(td), td) + 1e-37f;
    };
    auto refresh_bounds = [&]() {
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const int qi = qbase + g * 4 + rr;
            rtf[rr] = ((active >> (qi - qbase)) & 1u) ? row_bound(tau[qi], EXACT ? qnq[qi] : 0.0f) : qnan;
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

    // Staging of one chunk: NDMA direct global->LDS loads of 16 bytes per
    // lane (lane L of load i fills tile bytes 1024 i + 16 L, i.e. row
    // (64 i + L) / V16, position (64 i + L) % V16), issued one chunk ahead
    // into the other tile; rows past the level's end load the level's last
    // row (in bounds) and are masked by a NaN score term.  Wave 0 also loads
    // the per-point word / score-term inputs / scale into registers; they
    // are stored after the chunk's barrier wait.  `wsrc`: the packed words,
    // or any array of n words when there are none (then unused).
    uint32_t voff[UPW];   // per lane and load: byte offset of its piece in the chunk's rows
    int vrow[UPW];        // per lane and load: its tile row
#pragma unroll
    for (int u = 0; u < UPW; u++) {
        const int slot = 64 * (w + kLNW * u) + lane;
        const int row = slot / V16;
        vrow[u] = row;
        voff[u] = (uint32_t)(row * ROWB + 16 * ((slot % V16) ^ ((row / RPL) & SWZ)));
    }
    const uint32_t *wsrc = has_dense ? A.words : reinterpret_cast<const uint32_t *>(A.xnorm);
    uint32_t pre_w = 0;
    float pre_x = 0.0f, pre_e = 0.0f, pre_l = 0.0f, pre_s = 1.0f;
    bool pre_ok = false;
    auto fetch = [&](int32_t c0, int cn, uint8_t *dst) {
        const uint8_t *base = A.lvecs + (int64_t)c0 * ROWB;
#pragma unroll
        for (int u = 0; u < UPW; u++) {
            const int i = w + kLNW * u;   // wave-uniform
            if (NDMA % kLNW == 0 || i < NDMA) {
                uint32_t off = voff[u];
                if (cn < kLCH) off -= (uint32_t)(max(vrow[u] - (cn - 1), 0) * ROWB);
                __builtin_amdgcn_global_load_lds(base + off, (__attribute__((address_space(3))) void *)(dst + 1024 * i),
                                                 16, 0, 0);
            }
        }
        if (w == 0) {
            const int row = c0 + min(lane, cn - 1);
            pre_x = A.xnorm[row];
            if (EXACT) {
                pre_e = A.lerr[row];
                pre_l = A.lnrm[row];
            }
            pre_w = wsrc[row];
            if (PREC == CAPS_PREC_FP8) pre_s = A.lscale[row];
            pre_ok = lane < cn;
        }
    };
    // per-point term of the staged row (NaN for a padding row)
    auto point_term = [&]() {
        float pt;
        if (EXACT) {
            // lower-bound term: |x|^2 less twice the error-norm products and
            // the margin (L2); minus the products and margin (IP)
            const float nx = pre_x;
            // (the product sum rounded in FP32, raised past its rounding)
            const float slack = fmaf(pre_e, qa, pre_l * qb) * (1.0f + 0x1p-20f);
            pt = l2 ? fmaf(-A.eta, nx, fmaf(-2.0f, slack, nx)) : fmaf(-A.eta, nx, -slack);
            if (!(fabsf(pt) < inf)) pt = -inf;   // no usable bound: always rescored
        } else {
            pt = l2 ? pre_x : 0.0f;
        }
        return pre_ok ? pt : qnan;
    };

    // exact: the queued pairs, one per lane.  Main pass: appended to their
    // queries' deferred lists (per-row ranks from an LDS histogram, one
    // returning atomic per row); a query whose list is full is flagged for the
    // rescue pass instead.  Rescue pass: rescored exactly here.
    int vhead = 0, vtail = 0;   // wave-uniform ring cursors
    auto drain = [&](int n) {
        wave_sync();   // ring entries written by this wave are visible
        const bool v = lane < n;
        const int slot = (vtail + lane) & (kVRing - 1);
        const uint32_t pos = v ? ring_pos[slot] : 0u;
        const int qi = v ? (int)ring_row[slot] : qbase;
        const uint32_t pkey = DEFER && v ? ring_key[slot] : 0u;
        vtail += n;
        if (DEFER) {
            const int ri = qi - qbase;   // row of the wave, 0..15
            if (lane < kLQPW) dhist[lane] = 0;
            wave_sync();
            const int rank = v ? atomicAdd(dhist + ri, 1) : 0;
            wave_sync();
            const int cnt = lane < kLQPW ? dhist[lane] : 0;
            int base = 0;
            if (cnt > 0) base = atomicAdd(A.dcnt + my_qq, cnt);
            const int at = __shfl(base, ri, 64) + rank;
            const int32_t qq = qslot[qi] / A.m;
            if (v && at < A.dcap) A.dpos[(int64_t)qq * A.dcap + at] = ((uint64_t)pkey << 32) | pos;
            if (v && at >= A.dcap) A.oflow[qq] = 1;
        }
        if (RESCUE) {
            uint64_t key = ~0ull;
            if (v) {
                const int32_t qq = qslot[qi] / A.m;
                const float sc = exact_score<(HAS_LABELS && NS < 8) ? 2 : 4>(A.vecs + (int64_t)pos * A.d,
                                                                             A.q + (int64_t)qq * A.d, A.d, l2);
                key = ((uint64_t)f2ord(sc) << 32) | (uint32_t)A.perm[pos];
            }
            const bool qual = v && key < tau[qi];
            append_keys<CB>(qual, qi, key, buf, bcnt, tau, r);
        }
    };

    // The filter's slow path (the kernel variant with label tests, also used
    // for disjunctive searches): a pair that passed the packed dense test
    // (the exact test of a conjunction's dense constraints; for a disjunction
    // the fields all its terms share) is checked against the query's labels,
    // or against each term of a disjunction in full.
    auto slow_pass = [&](int qi, uint32_t pw, int64_t pos) -> bool {
        const QDesc &qd = qds[qi];
        if (qd.flags & kQOr)
            return query_passes(qd, A.qterms + (int64_t)(qslot[qi] / A.m) * kMaxTerms, has_dense, has_lab, pw,
                                has_lab ? A.sigs[pos] : 0ull, has_lab ? A.slots + pos * A.lslots : nullptr, A.lslots);
        if (!has_lab) return true;
        return point_passes(qd, false, true, 0u, A.sigs[pos], A.slots + pos * A.lslots, A.lslots);
    };

    int cj = -1;
    int32_t cc0 = 0, cend = 0;
    next_level(cj, cc0, cend);
    if (cj <= h) fetch(cc0, min(kLCH, cend - cc0), xt0);
    int nchunk = 0;

    // One chunk: tile `cur` (loaded by the previous step), point arrays `pb`;
    // loads the next chunk into `nxt`.  Returns whether there is one.
    auto step = [&](const uint8_t *cur, uint8_t *nxt, const int pb) -> bool {
        const int j = cj;
        const int32_t c0 = cc0;
        const int cn = min(kLCH, cend - c0);
        const uint32_t *xwp = xw + pb * kLCH;
        const float *xnp = xn + pb * kLCH;
        const float *xscp = xsc + pb * kLCH;
        if (w == 0) {
            xw[pb * kLCH + lane] = has_dense ? pre_w : 0u;
            xn[pb * kLCH + lane] = point_term();
            xsc[pb * kLCH + lane] = pre_s;
        }
        // this wave's direct loads into `cur` have landed; after the barrier
        // every wave's have, and every wave is done with `nxt` (read by the
        // previous step) and with the point arrays `pb` written two steps ago
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
        // the shared bounds are read before the next chunk's loads are issued
        // and used after them, so that their latency overlaps too.  (Nothing
        // lowers them during the main pass, which keeps no keys: it reads
        // them once per tile.)
        const bool refresh = !DEFER && (++nchunk % kTauRefresh) == 0;
        uint64_t gt = ~0ull;
        if (refresh) gt = __hip_atomic_load(A.tau + max(my_qq, 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        advance(cj, cc0, cend);
        const bool more = cj <= h;
        if (more) fetch(cc0, min(kLCH, cend - cc0), nxt);
        if (refresh) {
            if (lane < kLQPW && my_qq >= 0 && gt < tau[qbase + lane]) tau[qbase + lane] = gt;
            wave_sync();   // the wave's own bound slots, read below
            refresh_bounds();
        }
        if (active == 0) return more;   // a wave without queries only helps stage the chunks

            // ---- MFMA: my 16 queries x the chunk's 64 points
            f32x4 acc[4];
#pragma unroll
            for (int bb = 0; bb < 4; bb++) acc[bb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            // the four B operands of a K-step are read before its products,
            // so that one wait covers them (the order is kept by the
            // scheduling barrier)
#pragma unroll
            for (int s = 0; s < NS; s++) {
                VT bfr[4];
#pragma unroll
                for (int bb = 0; bb < 4; bb++) bfr[bb] = Op::load(cur + bb * 16 * ROWB + xoff[s]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int bb = 0; bb < 4; bb++) acc[bb] = Op::mma(a[s], bfr[bb], acc[bb]);
            }

            // ---- epilogue, one 16-point block at a time
            float tfj[4];
            if ((wall >> j) & 1u) {
#pragma unroll
                for (int rr = 0; rr < 4; rr++) tfj[rr] = rtf[rr];
            } else {
#pragma unroll
                for (int rr = 0; rr < 4; rr++) tfj[rr] = ((rsel(rr) >> j) & 1u) ? rtf[rr] : qnan;
            }
#pragma unroll
            for (int bb = 0; bb < 4; bb++) {
                const int pi = bb * 16 + (lane & 15);
                const uint32_t pw = xwp[pi];
                const float pn = xnp[pi];
                const float ps = xscp[pi];
                float esc[4];
                uint64_t hit[4];
#pragma unroll
                for (int rr = 0; rr < 4; rr++) {
                    float dd = acc[bb][rr];
                    if (PREC == CAPS_PREC_FP8) dd = dd * ps * rqs[rr];
                    esc[rr] = fmaf(cm, dd, pn);
                    // a single-compare ballot: one v_cmp into an SGPR pair
                    hit[rr] = __builtin_amdgcn_ballot_w64(esc[rr] <= tfj[rr]);
                }
                // the packed dense test, only for blocks where a score passed
                // (rare once the bounds are set: most blocks skip it)
                if (hit[0] | hit[1] | hit[2] | hit[3]) {
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) hit[rr] &= __builtin_amdgcn_ballot_w64((pw & rmask[rr]) == rval[rr]);
                }
                if (count) {   // survivors of the exact filter (statistics only)
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) {
                        const uint32_t rs = rsel(rr);   // every lane (a cross-lane read)
                        bool ok = pi < cn && ((rs >> j) & 1u) && (pw & rmask[rr]) == rval[rr];
                        if (HAS_LABELS && ok) ok = slow_pass(qbase + g * 4 + rr, pw, c0 + pi);
                        if (ok) atomicAdd(scnt + qbase + g * 4 + rr, 1);
                    }
                }
                if (hit[0] | hit[1] | hit[2] | hit[3]) {
                    bool moved = false;
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) {   // wave-uniform test per row group
                        if (!hit[rr]) continue;
                        // lanes 16g..16g+15 hold row 4g+rr: one query per 16-lane group
                        const int qi = qbase + g * 4 + rr;
                        bool qual = (hit[rr] >> lane) & 1ull;
                        if (HAS_LABELS && qual) qual = slow_pass(qi, pw, c0 + pi);
                        if (DEFER) {
                            // queue the pair for the deferred lists; when the ring
                            // is full, its query goes to the rescue pass instead
                            const uint64_t qm = __builtin_amdgcn_ballot_w64(qual);
                            if (vhead - vtail + __popcll(qm) > kVRing) {
                                if (qual) A.oflow[qslot[qi] / A.m] = 1;
                                continue;
                            }
                            if (qual) {
                                const int sl = (vhead + __popcll(qm & lanemask_lt())) & (kVRing - 1);
                                ring_pos[sl] = (uint32_t)(c0 + pi);
                                ring_row[sl] = (uint32_t)qi;
                                ring_key[sl] = f2ord(canon0(esc[rr]));
                            }
                            vhead += __popcll(qm);
                            continue;
                        }
                        if (RESCUE) {
                            // queue the pair; rescore once 64 are pending
                            const uint64_t qm = __builtin_amdgcn_ballot_w64(qual);
                            if (qual) {
                                const int sl = (vhead + __popcll(qm & lanemask_lt())) & (kVRing - 1);
                                ring_pos[sl] = (uint32_t)(c0 + pi);
                                ring_row[sl] = (uint32_t)qi;
                            }
                            vhead += __popcll(qm);
                            if (vhead - vtail >= 64) {
                                drain(64);
                                moved = true;
                            }
                            continue;
                        }
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
                            moved = true;
                        }
                    }
                    if (moved) {   // bounds may have tightened
                        refresh_bounds();
#pragma unroll
                        for (int rr = 0; rr < 4; rr++) tfj[rr] = ((rsel(rr) >> j) & 1u) ? rtf[rr] : qnan;
                    }
                }
            }

        return more;
    };
    if (cj <= h)
        while (step(xt0, xt1, 0) && step(xt1, xt0, 1)) {
        }
    if (EXACT)
        while (vhead > vtail) drain(min(64, vhead - vtail));
    // ---- survivors per query
    if (count) {
        wave_sync();
        if (lane < kLQPW && my_qq >= 0 && scnt[qbase + lane]) atomicAdd(&A.nsurv[my_qq], scnt[qbase + lane]);
    }
    // ---- finalize my queries: best r sorted, partial list, shared bound
    // (the main pass keeps no keys and writes no counts: the merge reads the
    // lists of the queries the rescue pass rescanned only)
    if (DEFER) return;
    for (int i = 0; i < kLQPW; i++) {
        const int qi = qbase + i;
        if (qi >= nqt) break;
        if (!((active >> i) & 1u)) continue;
        if (bcnt[qi] > 0) buf_reduce<CB>(buf, bcnt, tau, qi, r);
        const int c = bcnt[qi];
        const int32_t slot = qslot[qi];
        uint64_t *out = A.partials + (int64_t)slot * r;
        if (lane < c) out[lane] = buf[qi * CB + lane];   // the keys written are counted in pcnt
        if (lane == 0) {
            A.pcnt[slot] = c;
            if (c == r) atomicMin((unsigned long long *)(A.tau + slot / A.m), (unsigned long long)buf[qi * CB + r - 1]);
        }
    }
    };
    if (RESCUE) {
        // a workgroup walking several tiles waits for all its waves between
        // them: the cursor and bound arrays (spo, lvw, qmx) are rewritten at
        // the start of a tile and read until its end
        const int nr = *A.rcount;
        for (int i = blockIdx.x; i < nr; i += gridDim.x) {
            const int e = A.rlist[i];
            int4 dsc = A.tiles[A.rhalves ? e >> 1 : e];
            if (A.rhalves) {   // the 64 entries of one half of a 128-entry tile
                dsc.y += kLQB * (e & 1);
                dsc.z = min(kLQB, dsc.z - kLQB * (e & 1));
            }
            run_tile(dsc);
            __syncthreads();
        }
    } else {
        const int tile = xcd_tile(blockIdx.x, A.ntiles);
        if (tile >= 0) run_tile(A.tiles[tile]);
    }
}

// ------------------------------------------------ exact main pass, 32 x 32
// The exact main pass of two-byte copies with rows of at most four 32-element
// steps, without label tests or disjunctions (the other cases run
// k_scan_mfma).  Same bound, point term and element test as k_scan_mfma's
// exact main pass; what differs is the blocking:
//  * a tile holds up to 128 (query, probe) entries of one partition, wave w
//    the 32 queries 32w..32w+31, whose operands stay in registers;
//  * each product is a 32 x 32 block (points x queries, K = 16 per step), so
//    a staged row read from LDS serves 32 queries instead of 16;
//  * chunks are 32 rows, staged by direct loads three chunks ahead into four
//    buffers, with explicit per-wave wait counts and plain barriers;
//  * the packed dense test runs only for the products where a score passed.
// Element r of lane l is point 8(r/4) + 4(l/32) + r%4 of the chunk and query
// l%32 of the wave.  MODE 0 is the exact main pass, MODE 1 the same counting
// the survivors of the filter, MODE 2 the seed pass of the exact search:
// approximate keys (plain point term) of the first probes, of which each
// lane keeps its MH best that pass the filter in registers, written as the
// (query, probe)'s partial list for the exact seed bound.
constexpr int kXW = 4;                 // waves per tile
constexpr int kXQ = 32;                // queries per wave
constexpr int kXQB = kXW * kXQ;        // entries per tile
constexpr int kXCH = 32;               // rows per chunk
constexpr int kXRing = 64;             // per-wave ring of deferred pairs
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int PREC>
struct Mfma32;
template <>
struct Mfma32<CAPS_PREC_BF16> {
    typedef bf16x8 T;
    __device__ static f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma32<CAPS_PREC_FP16> {
    typedef f16x8 T;
    __device__ static f32x16 mma(T a, T b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};

__host__ __device__ constexpr bool lowp_x32_kernel(int prec, int ns, bool lab) {
    return (prec == CAPS_PREC_BF16 || prec == CAPS_PREC_FP16) && (ns == 1 || ns == 2 || ns == 4) && !lab;
}

template <int PREC, int NS, int MODE, int MH>
__global__ __launch_bounds__(kXW * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_scan_x32(LowpArgs A) {
    constexpr bool COUNT = MODE == 1;   // survivor counts of the exact filter
    constexpr bool SEED = MODE == 2;    // approximate keys: per query and probe the best 2 MH
    typedef typename Mfma32<PREC>::T VT;
    constexpr int ROWB = NS * 64;                  // bytes per row of the copy
    constexpr int KS = ROWB / 32;                  // 16-element steps per row
    constexpr int V16 = ROWB / 16;                 // 16-byte pieces per row
    constexpr int NDMA = kXCH * ROWB / 1024;       // 1 KB direct loads per chunk
    constexpr int UPW = (NDMA + kXW - 1) / kXW;
    constexpr int RPL = ROWB >= 256 ? 1 : 256 / ROWB;
    constexpr int SWZ = ROWB >= 256 ? 15 : V16 - 1;
    constexpr int PRE = 4;                         // per-point inputs per chunk (one direct load per wave)
    static_assert(PRE == kXW, "each wave stages one per-point input");
    // the four chunk buffers: distinct arrays, so that the compiler can tell
    // the reads of one from the direct loads into the others
    __shared__ __align__(16) uint8_t xb0[kXCH * ROWB];
    __shared__ __align__(16) uint8_t xb1[kXCH * ROWB];
    __shared__ __align__(16) uint8_t xb2[kXCH * ROWB];
    __shared__ __align__(16) uint8_t xb3[kXCH * ROWB];
    __shared__ __align__(16) float rw0[PRE][kXCH];   // the per-point inputs of each buffer's chunk
    __shared__ __align__(16) float rw1[PRE][kXCH];
    __shared__ __align__(16) float rw2[PRE][kXCH];
    __shared__ __align__(16) float rw3[PRE][kXCH];
    __shared__ __align__(16) uint32_t xw[2][kXCH];
    __shared__ __align__(16) float xn[2][kXCH];
    __shared__ uint32_t xsum[2][2];   // AND and OR of each point slot's packed words (the chunk's rows)
    __shared__ uint32_t ring[kXW][SEED ? 2 : 3][kXRing];
    __shared__ int32_t dhist[kXW][kXQ];   // (before the pipeline starts: also the tile's maxima, below)
    __shared__ int32_t scnt[COUNT ? kXQB : 1];   // (only the counting mode: the modes used per search keep 4 workgroups per CU)
    // the tile prologue's per-wave maxima share the drain histograms' storage:
    // every read of them completes before the pipeline's first barrier, and
    // no drain runs before it
    static_assert(3 * kXW <= kXQ, "the maxima fit in one wave's histogram");
    float(*qmx)[kXW] = reinterpret_cast<float(*)[kXW]>(&dhist[0][0]);
    uint32_t *lvw = reinterpret_cast<uint32_t *>(&dhist[0][2 * kXW]);

    const int tile = xcd_tile(blockIdx.x, A.ntiles);
    if (tile < 0) return;
    const int4 dsc = A.tiles[tile];
    if (dsc.z <= 0) return;
    const int p = dsc.x;
    const int nqt = dsc.z;
    const int32_t *ent = A.entries + dsc.y;
    const int h = A.h;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // (wave-uniform: kept in a scalar register)
    const int g = lane >> 5, c32 = lane & 31;
    const bool has_dense = A.words != nullptr;
    const bool l2 = A.metric == 0;
    const float qnan = __builtin_nanf("");
    const float inf = __builtin_huge_valf();
    const float cm = l2 ? -2.0f : -1.0f;   // score = cm * dot + per-point term

    // ---- the lane's query: tile entry 32w + c32 (lanes l and l + 32 share it)
    const int qi = kXQ * w + c32;
    const bool own = qi < nqt;
    int32_t my_slot = 0, my_qq = 0;
    uint32_t my_sel = 0, my_mask = 0, my_val = 1;   // a lane without a query never matches
    float my_tf = qnan, qa = 0.0f, qb = 0.0f;
    uint64_t my_tk = ~0ull;   // seed: the shared bound key at the tile's start
    if (own) {
        my_slot = ent[qi];
        my_qq = my_slot / A.m;
        my_sel = A.esel ? A.esel[dsc.y + qi] : A.sel[my_slot];   // (in entry order: one coalesced read)
        my_mask = A.qd[my_qq].dmask;
        my_val = A.qd[my_qq].dval;
        const float4 ax = *reinterpret_cast<const float4 *>(A.qaux + 4 * (int64_t)my_qq);
        qa = ax.x;
        qb = fmaf(A.gam, ax.w, ax.z);
        // the bound, read once per tile (the main pass keeps no keys; the
        // seed pass shares it between the tiles of a query by atomic min)
        const uint64_t tk = __hip_atomic_load(A.tau + my_qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const float td = bound_score(tk);
        const float nq = ax.y;
        my_tf = SEED          ? td
                : !(td < inf) ? inf
                : l2          ? fmaf(A.eta, nq + td, td - nq) + 1e-37f
                              : fmaf(A.eta, nq + fabsf(td), td) + 1e-37f;
        if (SEED) my_tk = tk;
    }
    // tile maxima of |q| and |q - q~| + gam |q~| (the point term's error
    // products) and the levels any query of the tile selects
    uint32_t lv = my_sel;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        qa = fmaxf(qa, __shfl_xor(qa, o, 64));
        qb = fmaxf(qb, __shfl_xor(qb, o, 64));
        lv |= __shfl_xor(lv, o, 64);
    }
    if (lane == 0) {
        qmx[0][w] = qa;
        qmx[1][w] = qb;
        lvw[w] = lv;
    }
    if constexpr (COUNT) {
        if (w == 0) {
            scnt[lane] = 0;
            scnt[lane + 64] = 0;
        }
    }
    // level bounds, one per lane: lane j holds the start of level j, lane
    // h + 1 the end of the partition (read out by lane index, no memory wait)
    const int32_t spv = A.offs[(int64_t)p * (h + 1) + min(lane, h + 1)];
    const int32_t spn = __shfl_down(spv, 1, 64);   // every lane takes part
    const uint32_t lne = (uint32_t)__builtin_amdgcn_ballot_w64(lane <= h && spv < spn);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kXW; i++) {
        qa = fmaxf(qa, qmx[0][i]);
        qb = fmaxf(qb, qmx[1][i]);
        lv |= lvw[i];
    }
    // the levels to scan: selected by a query of the tile and not empty
    lv = __builtin_amdgcn_readfirstlane(lv & lne);
    // MFMA B operands: the lane's query, K slice 8g of each step
    VT bq[KS];
    {
        const uint8_t *src = A.qlow + (int64_t)my_qq * ROWB + 16 * g;
#pragma unroll
        for (int s = 0; s < KS; s++)
            bq[s] = own ? __builtin_bit_cast(VT, *reinterpret_cast<const uint4 *>(src + 32 * s)) : VT{};
    }
    // MFMA A operands: row c32 of a staged chunk, K slice 8g of step s at
    // c32 ROWB + 16 ((2s + g) ^ swizzle) = xo ^ 32s (the row's bytes are a
    // power of two and 2s + g = 2s | g)
    const uint32_t xo = (uint32_t)(c32 * ROWB + 16 * (g ^ ((c32 / RPL) & SWZ)));

    // chunk cursors (wave-uniform): level j, first row c0, end of the level;
    // past the last level j = h + 1
    auto next_level = [&](int &j, int32_t &c0, int32_t &end) {
        const uint32_t rest = lv >> (j + 1);   // j + 1 <= h + 1 <= 16
        if (!rest) {
            j = h + 1;
            return;
        }
        j += 1 + __builtin_ctz(rest);
        c0 = __builtin_amdgcn_readlane(spv, j);
        end = __builtin_amdgcn_readlane(spv, j + 1);
    };
    auto advance = [&](int &j, int32_t &c0, int32_t &end) {
        c0 += kXCH;
        if (c0 >= end) next_level(j, c0, end);
    };

    // Staging.  Every wave issues the same loads per chunk (UPW row loads
    // and one per-point load), always, so that one wait count holds for all
    // waves and every path (a missing chunk loads row 0 into the unused
    // buffer instead).  Row load i, lane L fills tile bytes 1024 i + 16 L:
    // row (64 i + L) / V16, piece (64 i + L) % V16, which holds global piece
    // piece ^ swizzle of the row; rows past the level's end load its last row
    // and are masked by a NaN point term; loads past NDMA (short rows) repeat
    // load i - NDMA.  Per-point load of wave w, lane L: input w (squared
    // norm, error norms, packed dense word) of row c0 + min(L, cn - 1), L < 32.
    uint32_t voff[UPW];
    int vrow[UPW];
#pragma unroll
    for (int u = 0; u < UPW; u++) {
        const int i = (w + kXW * u) % NDMA;
        const int slot = 64 * i + lane;
        const int row = slot / V16;
        vrow[u] = row;
        voff[u] = (uint32_t)(row * ROWB + 16 * ((slot % V16) ^ ((row / RPL) & SWZ)));
    }
    constexpr int OPC = UPW + 1;   // loads per wave per chunk
    const uint32_t *wsrc = has_dense ? A.words : reinterpret_cast<const uint32_t *>(A.xnorm);
    const float *psrc = w == 0   ? A.xnorm
                        : w == 1 ? A.lerr
                        : w == 2 ? A.lnrm
                                 : reinterpret_cast<const float *>(wsrc);
    auto fetch_rows = [&](bool real, int32_t c0, int cn, uint8_t *dst) {
        const uint8_t *base = real ? A.lvecs + (int64_t)c0 * ROWB : A.lvecs;
#pragma unroll
        for (int u = 0; u < UPW; u++) {
            const int i = (w + kXW * u) % NDMA;
            uint32_t off = real ? voff[u] : 0u;
            if (real && cn < kXCH) off -= (uint32_t)(max(vrow[u] - (cn - 1), 0) * ROWB);
            __builtin_amdgcn_global_load_lds(base + off, (__attribute__((address_space(3))) void *)(dst + 1024 * i), 16,
                                             0, 0);
        }
    };
    auto fetch_points = [&](bool real, int32_t c0, int cn, float (*raw)[kXCH]) {
        // lanes 0..31 (lane L fills raw[w][L]; every wave has them active, so
        // the load is issued on every path)
        if (lane < kXCH) {
            const int64_t row = real ? c0 + min(lane, cn - 1) : 0;
            __builtin_amdgcn_global_load_lds(psrc + row, (__attribute__((address_space(3))) void *)raw[w], 4, 0, 0);
        }
    };
    // the point terms of a chunk whose per-point inputs have landed (one
    // wave per chunk, in turn)
    auto point_terms = [&](float (*raw)[kXCH], int cn, int pb) {
        const float nx = raw[0][c32];
        const float slack = fmaf(raw[1][c32], qa, raw[2][c32] * qb) * (1.0f + 0x1p-20f);
        float pt = l2 ? fmaf(-A.eta, nx, fmaf(-2.0f, slack, nx)) : fmaf(-A.eta, nx, -slack);
        if (!(fabsf(pt) < inf)) pt = -inf;
        if (SEED) pt = l2 ? nx : 0.0f;   // approximate keys: the plain point term
        xn[pb][c32] = c32 < cn ? pt : qnan;   // (lanes l and l + 32 write alike)
        const uint32_t wd = has_dense ? __float_as_uint(raw[3][c32]) : 0u;
        xw[pb][c32] = wd;
        // the chunk's summary for the skip test: AND and OR of its rows'
        // words, reduced inside each 16-lane row by rotations (DPP row_ror
        // 1, 2, 4, 8), then rows 0 and 1 (lanes 0..31 hold the chunk's rows)
        int wa = c32 < cn ? (int)wd : -1, wo = c32 < cn ? (int)wd : 0;
        wa &= __builtin_amdgcn_mov_dpp(wa, 0x121, 0xF, 0xF, false);
        wo |= __builtin_amdgcn_mov_dpp(wo, 0x121, 0xF, 0xF, false);
        wa &= __builtin_amdgcn_mov_dpp(wa, 0x122, 0xF, 0xF, false);
        wo |= __builtin_amdgcn_mov_dpp(wo, 0x122, 0xF, 0xF, false);
        wa &= __builtin_amdgcn_mov_dpp(wa, 0x124, 0xF, 0xF, false);
        wo |= __builtin_amdgcn_mov_dpp(wo, 0x124, 0xF, 0xF, false);
        wa &= __builtin_amdgcn_mov_dpp(wa, 0x128, 0xF, 0xF, false);
        wo |= __builtin_amdgcn_mov_dpp(wo, 0x128, 0xF, 0xF, false);
        // (the lane reads stay outside the single-lane branch below: they
        // read lanes that branch leaves inactive)
        const uint32_t sa = (uint32_t)(__builtin_amdgcn_readlane(wa, 0) & __builtin_amdgcn_readlane(wa, 16));
        const uint32_t so = (uint32_t)(__builtin_amdgcn_readlane(wo, 0) | __builtin_amdgcn_readlane(wo, 16));
        if (lane == 0) {
            xsum[pb][0] = sa;
            xsum[pb][1] = so;
        }
    };

    // deferred pairs of this wave: (CSR position, wave query) in a ring of
    // 64, appended to their queries' lists when a ballot's pairs would not
    // fit (per-query ranks from an LDS histogram, one returning atomic per
    // query); a query whose list is full is flagged for the rescue pass
    uint32_t *ring_pos = ring[w][0];
    uint32_t *ring_row = ring[w][1];
    uint32_t *ring_key = ring[w][SEED ? 1 : 2];   // the pair's ordered score (not in the seed mode)
    int32_t *hist = dhist[w];
    int vhead = 0, vtail = 0;
    auto drain = [&](int n) {
        wave_sync();
        const bool v = lane < n;
        const int slot = (vtail + lane) & (kXRing - 1);
        const uint32_t pos = v ? ring_pos[slot] : 0u;
        const int qj = v ? (int)ring_row[slot] : 0;
        const uint32_t pkey = v ? ring_key[slot] : 0u;
        vtail += n;
        if (lane < kXQ) hist[lane] = 0;
        wave_sync();
        const int rank = v ? atomicAdd(hist + qj, 1) : 0;
        wave_sync();
        const int cnt = lane < kXQ ? hist[lane] : 0;
        int base = 0;
        if (cnt > 0) base = atomicAdd(A.dcnt + my_qq, cnt);
        const int at = __shfl(base, qj, 64) + rank;
        const int32_t qq = __shfl(my_qq, qj, 64);
        if (v && at < A.dcap) A.dpos[(int64_t)qq * A.dcap + at] = ((uint64_t)pkey << 32) | pos;
        if (v && at >= A.dcap) A.oflow[qq] = 1;
    };

    // ---- pipeline.  Fetch F_c = rows of chunk c into buffer c % 4 and the
    // per-point inputs of chunk c + 1 into slot (c + 1) % 4.  Step k waits
    // for F_k (two later fetches may stay in flight), passes the barrier,
    // issues F_{k+3}, lets wave k % 4 turn the inputs of chunk k + 1 into its
    // point terms, and scores chunk k.
    int cj = -1;
    int32_t cc0 = 0, cend = 0;
    next_level(cj, cc0, cend);
    if (cj > h) {   // nothing to scan
        if (SEED && g == 0 && own) A.pcnt[my_slot] = 0;
        return;
    }
    // fetch cursor (chunk of the rows of the next fetch) and the chunk after it
    int fj = cj, rj = cj;
    int32_t fc0 = cc0, fend = cend, rc0 = cc0, rend = cend;
    advance(rj, rc0, rend);
    auto fetch_next = [&](uint8_t *dst, float (*raw)[kXCH]) {
        const bool fr = fj <= h, rr = rj <= h;
        fetch_rows(fr, fc0, fr ? min(kXCH, fend - fc0) : 1, dst);
        fetch_points(rr, rc0, rr ? min(kXCH, rend - rc0) : 1, raw);
        if (fr) advance(fj, fc0, fend);
        if (rr) advance(rj, rc0, rend);
    };
    fetch_points(true, cc0, min(kXCH, cend - cc0), rw0);   // the inputs of chunk 0
    fetch_next(xb0, rw1);
    fetch_next(xb1, rw2);
    fetch_next(xb2, rw3);
    // the first three chunks have landed on every wave (waiting for all of
    // them lets the compiler's own wait tracking enter the loop with nothing
    // in flight)
    __builtin_amdgcn_s_waitcnt(0xC07F & 0x0F70);   // vmcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    if (w == 0) point_terms(rw0, min(kXCH, cend - cc0), 0);
    int lj = -1;
    float tfj = qnan;
    uint64_t lst[SEED ? MH : 1];   // seed: the lane's best keys, ascending (~0: empty)
#pragma unroll
    for (int i = 0; i < (SEED ? MH : 1); i++) lst[i] = ~0ull;

    // Chunk k from buffer `cur` (point arrays `pb`); `nraw` holds the inputs
    // of chunk k + 1, whose point terms wave `ptw` (k % 4) computes; F_{k+3}
    // goes to `nxt` and `fraw`.  Returns whether another chunk follows.
    auto step = [&](const uint8_t *cur, uint8_t *nxt, const int pb, float (*nraw)[kXCH], float (*fraw)[kXCH],
                    const int ptw) -> bool {
        const int j = cj;
        const int32_t c0 = cc0;
        const int cn = min(kXCH, cend - c0);
        // F_k has landed once at most the two later fetches are outstanding
        // (stores and atomics issued since only make the wait stricter); the
        // point terms wave 0 wrote are complete
        __builtin_amdgcn_s_waitcnt(0xC07F & (0x0F70 | ((2 * OPC) & 15) | (((2 * OPC) >> 4) << 14)));
        __builtin_amdgcn_s_barrier();
        advance(cj, cc0, cend);
        const bool more = cj <= h;
        fetch_next(nxt, fraw);
        if (w == ptw && more) point_terms(nraw, min(kXCH, cend - cc0), pb ^ 1);
        if (kXQ * w >= nqt) return more;   // a wave without queries (small batches) only stages
        {
            // A row passes (w & M) == V only if every bit of V is set in the
            // OR of the chunk's words and every other bit of M is clear in
            // their AND: where no query of the wave can pass a row of the
            // chunk, its products and tests are skipped (the queries of a
            // wave share constraints and a sub-partition's rows are grouped
            // by their values, so this is common)
            const uint32_t wa = xsum[pb][0], wo = xsum[pb][1];
            const uint32_t miss = (my_val & ~wo) | (~my_val & my_mask & wa) | (((my_sel >> j) & 1u) ^ 1u);
            if (!__builtin_amdgcn_ballot_w64(miss == 0u)) return more;
        }

        f32x16 acc = {};
#pragma unroll
        for (int s0 = 0; s0 < KS; s0 += 2) {   // operands of two steps, then their products
            VT a[2];
#pragma unroll
            for (int s = s0; s < s0 + 2; s++)
                a[s - s0] = __builtin_bit_cast(VT, *reinterpret_cast<const uint4 *>(cur + (xo ^ (32u * s))));
#pragma unroll
            for (int s = s0; s < s0 + 2; s++) acc = Mfma32<PREC>::mma(a[s - s0], bq[s], acc);
        }

        if constexpr (SEED) {
            // approximate keys below the lane's bound (the shared bound at the
            // tile's start, then the worst of its MH best) that pass the
            // packed dense test enter its sorted list; lanes l and l + 32 keep
            // one list each for query l % 32 (its half of the chunk's points)
            if (j != lj) {
                lj = j;
                tfj = ((my_sel >> j) & 1u) ? bound_score(lst[MH - 1] < my_tk ? lst[MH - 1] : my_tk) : qnan;
            }
#pragma unroll
            for (int q4 = 0; q4 < 4; q4++) {
                const int rb = 8 * q4 + 4 * g;
                const float4 pn = *reinterpret_cast<const float4 *>(&xn[pb][rb]);
                const float pv[4] = {pn.x, pn.y, pn.z, pn.w};
                float esc[4];
                uint64_t hit[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    esc[e] = fmaf(cm, acc[4 * q4 + e], pv[e]);
                    hit[e] = __builtin_amdgcn_ballot_w64(esc[e] <= tfj);
                }
                if (!(hit[0] | hit[1] | hit[2] | hit[3])) continue;
                const uint4 pw = *reinterpret_cast<const uint4 *>(&xw[pb][rb]);
                const uint32_t wv[4] = {pw.x, pw.y, pw.z, pw.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (!((hit[e] >> lane) & 1ull) || (wv[e] & my_mask) != my_val) continue;
                    const uint64_t key = ((uint64_t)f2ord(canon0(esc[e])) << 32) | (uint32_t)(c0 + rb + e);
                    if (!(key < lst[MH - 1])) continue;
                    uint64_t kk = key;   // one compare-exchange pass keeps the list sorted
#pragma unroll
                    for (int i = 0; i < MH; i++) {
                        const bool lt = kk < lst[i];
                        const uint64_t lo = lt ? kk : lst[i];
                        kk = lt ? lst[i] : kk;
                        lst[i] = lo;
                    }
                    tfj = bound_score(lst[MH - 1] < my_tk ? lst[MH - 1] : my_tk);
                }
            }
        } else {
            if (j != lj) {   // level changed: the query's bound if it selects the level, NaN if not
                lj = j;
                tfj = ((my_sel >> j) & 1u) ? my_tf : qnan;
            }
            const bool sj = (my_sel >> j) & 1u;
            // point terms of the next group read while this one is scored
            float4 pnx = *reinterpret_cast<const float4 *>(&xn[pb][4 * g]);
#pragma unroll
            for (int q4 = 0; q4 < 4; q4++) {   // points 8 q4 + 4 g + e of the chunk, e < 4
                const int rb = 8 * q4 + 4 * g;
                const float4 pn = pnx;
                if (q4 < 3) pnx = *reinterpret_cast<const float4 *>(&xn[pb][rb + 8]);
                const float pv[4] = {pn.x, pn.y, pn.z, pn.w};
                uint64_t hit[4];
                float sc[4];   // the element test's scores (deferred with their pairs)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    sc[e] = fmaf(cm, acc[4 * q4 + e], pv[e]);
                    hit[e] = __builtin_amdgcn_ballot_w64(sc[e] <= tfj);
                }
                if constexpr (COUNT) {   // survivors of the exact filter (statistics only)
                    const uint4 pw = *reinterpret_cast<const uint4 *>(&xw[pb][rb]);
                    const uint32_t wv[4] = {pw.x, pw.y, pw.z, pw.w};
                    int c = 0;
#pragma unroll
                    for (int e = 0; e < 4; e++) c += (sj && rb + e < cn && (wv[e] & my_mask) == my_val) ? 1 : 0;
                    if (c) atomicAdd(&scnt[qi], c);
                }
                if (!(hit[0] | hit[1] | hit[2] | hit[3])) continue;
                {   // the packed dense test where a score passed
                    const uint4 pw = *reinterpret_cast<const uint4 *>(&xw[pb][rb]);
                    const uint32_t wv[4] = {pw.x, pw.y, pw.z, pw.w};
#pragma unroll
                    for (int e = 0; e < 4; e++) hit[e] &= __builtin_amdgcn_ballot_w64((wv[e] & my_mask) == my_val);
                }
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint64_t hm = hit[e];
                    if (!hm) continue;
                    const int n = __popcll(hm);   // at most 64
                    if (vhead - vtail + n > kXRing) drain(vhead - vtail);
                    if ((hm >> lane) & 1ull) {
                        const int sl = (vhead + __popcll(hm & lanemask_lt())) & (kXRing - 1);
                        ring_pos[sl] = (uint32_t)(c0 + rb + e);
                        ring_row[sl] = (uint32_t)c32;
                        ring_key[sl] = f2ord(canon0(sc[e]));
                    }
                    vhead += n;
                }
            }
        }
        return more;
    };
    while (step(xb0, xb3, 0, rw1, rw0, 0) && step(xb1, xb0, 1, rw2, rw1, 1) && step(xb2, xb1, 0, rw3, rw2, 2) &&
           step(xb3, xb2, 1, rw0, rw3, 3)) {
    }
    if constexpr (SEED) {
        // the slot's list: the keys of half 0, then those of half 1 (2 MH <= r
        // entries); a full list of r keys bounds the query's r-th key
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < MH; i++) cnt += lst[i] != ~0ull ? 1 : 0;
        const int c_lo = __shfl(cnt, c32, 64);
        const int c_hi = __shfl(cnt, c32 + 32, 64);
        const uint64_t w_hi = ((uint64_t)(uint32_t)__shfl((int)(lst[MH - 1] >> 32), c32 + 32, 64) << 32) |
                              (uint32_t)__shfl((int)(uint32_t)lst[MH - 1], c32 + 32, 64);
        if (own) {
            uint64_t *out = A.partials + (int64_t)my_slot * A.r + (g ? c_lo : 0);
#pragma unroll
            for (int i = 0; i < MH; i++)
                if (i < cnt) out[i] = lst[i];
            if (g == 0) {
                A.pcnt[my_slot] = c_lo + c_hi;
                if (c_lo + c_hi == A.r) {
                    const uint64_t worst = lst[MH - 1] > w_hi ? lst[MH - 1] : w_hi;
                    atomicMin((unsigned long long *)(A.tau + my_qq), (unsigned long long)worst);
                }
            }
        }
        return;
    } else {
        if (vhead > vtail) drain(vhead - vtail);
        if constexpr (COUNT) {
            __syncthreads();
            if (g == 0 && own && scnt[qi]) atomicAdd(&A.nsurv[my_qq], scnt[qi]);
        }
    }
}

typedef void (*LowpFn)(LowpArgs);

// Buffer capacity per query: r plus room to append before a reduction.  The
// smaller buffers of small r let three workgroups share a compute unit's LDS.
inline int lowp_cb(int r) { return r <= 16 ? 32 : r <= 48 ? 64 : 128; }

template <int PREC, bool LAB, int NS, int KIND>
LowpFn pick_cb(int r) {
    if constexpr ((KIND == 1 || KIND == 3) && lowp_x32_kernel(PREC, NS, LAB)) {
        return k_scan_x32<PREC, NS, KIND == 3 ? 1 : 0, 1>;
    } else if constexpr (KIND == 4 && lowp_x32_kernel(PREC, NS, LAB)) {
        // seed lists: per (query, probe) the best key of each half of the
        // partition's rows (longer lists cost more insertions than their
        // tighter bound saved: MH = 2 and 5 ran 0.34 and 0.44 ms per c2 step
        // against 0.28 ms, with the same main pass)
        (void)r;
        return k_scan_x32<PREC, NS, 2, 1>;
    } else if constexpr (KIND == 4) {
        return k_scan_mfma<PREC, LAB, 32, NS, 0>;   // (not used: the seed kind needs the 32 x 32 pass)
    } else if constexpr (KIND == 1 || KIND == 3) {
        return k_scan_mfma<PREC, LAB, 32, NS, KIND>;   // (keeps no keys)
    } else {
        const int cb = lowp_cb(r);
        if (cb == 32) return k_scan_mfma<PREC, LAB, 32, NS, KIND>;
        if (cb == 64) return k_scan_mfma<PREC, LAB, 64, NS, KIND>;
        return k_scan_mfma<PREC, LAB, 128, NS, KIND>;
    }
}

template <int PREC, int NS, int KIND>
LowpFn pick_lab(bool lab, int r) {
    return lab ? pick_cb<PREC, true, NS, KIND>(r) : pick_cb<PREC, false, NS, KIND>(r);
}

// the kernel for one precision and kind (defined by caps_scan_inst.hip)
template <int PREC, int KIND>
LowpFn pick_ns(int ns, bool lab, int r);
template <> LowpFn pick_ns<CAPS_PREC_BF16, 0>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_BF16, 1>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_BF16, 2>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_BF16, 3>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_BF16, 4>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP16, 0>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP16, 1>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP16, 2>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP16, 3>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP16, 4>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP8, 0>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP8, 1>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP8, 2>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP8, 3>(int, bool, int);
template <> LowpFn pick_ns<CAPS_PREC_FP8, 4>(int, bool, int);

}  // namespace caps
