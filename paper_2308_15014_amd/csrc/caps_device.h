// Device-side helpers shared by the libcaps kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "caps_internal.h"

namespace caps {

constexpr int kWave = 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Workgroups of a launch are dealt to the 8 XCDs of the chip round-robin
// (workgroup i runs on XCD i % 8), each XCD with its own L2.  Maps a launch
// index to a tile so that every XCD receives one contiguous range of the
// `ntiles` live tiles, in order: consecutive tiles (the same partition) then
// share one L2.  Needs a grid of at least 8 * ceil(ntiles / 8) workgroups;
// returns -1 for a workgroup without a tile.
constexpr int kXcds = 8;
__device__ inline int xcd_tile(int bid, int ntiles) {
    const int per = (ntiles + kXcds - 1) / kXcds;
    const int x = bid % kXcds, s = bid / kXcds;
    const int vt = x * per + s;
    return (s < per && vt < ntiles) ? vt : -1;
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

// Inclusive scan of v over the 64 lanes of a wave.
__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan over a block of NT threads (NT a multiple of 64, <= 1024).
// `scratch` holds NT/64 + 1 ints of LDS.  Returns the thread's exclusive
// prefix; *total receives the block sum.  Contains __syncthreads().
template <int NT>
__device__ inline int block_excl_scan(int v, int *scratch, int *total) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) scratch[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < NW; i++) {
            int t = scratch[i];
            scratch[i] = s;
            s += t;
        }
        scratch[NW] = s;
    }
    __syncthreads();
    int r = scratch[w] + inc - v;
    *total = scratch[NW];
    __syncthreads();
    return r;
}

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t u = __shfl_xor(v, o, kWave);
        v = u < v ? u : v;
    }
    return v;
}

__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t u = __shfl_xor(v, o, kWave);
        v = u > v ? u : v;
    }
    return v;
}

// Lanes of the wave whose `key` equals this lane's key (key < 2^nbits).
__device__ inline uint64_t wave_match(uint32_t key, int nbits) {
    uint64_t peers = __ballot(1);
    for (int b = 0; b < nbits; b++) {
        uint64_t bal = __ballot((key >> b) & 1u);
        peers &= ((key >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

// Whether a point's sorted label slots (ns of them, 0xFFFF padded) hold v:
// a comparison with each of 8 slots, a binary search over wider rows.
__device__ inline bool slots_hold(const uint16_t *sl, int ns, uint16_t v) {
    if (ns <= kMaxLabels) {
        bool f = false;
#pragma unroll
        for (int s = 0; s < kMaxLabels; s++) f |= sl[s] == v;
        return f;
    }
    int lo = 0, hi = ns;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sl[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo < ns && sl[lo] == v;
}

// Exact filter of one point against one query (Definition 1 with wildcards).
__device__ inline bool point_passes(const QDesc &qd, bool has_dense, bool has_labels, uint32_t w,
                                    uint64_t sig, const uint16_t *sl, int ns = kMaxLabels) {
    if (has_dense && ((w & qd.dmask) != qd.dval)) return false;
    if (has_labels && qd.nlab > 0) {
        if (qd.lsig & ~sig) return false;
        for (int i = 0; i < qd.nlab; i++)
            if (!slots_hold(sl, ns, qd.lab[i])) return false;
    }
    return true;
}

// Filter of one point against a query (summary descriptor qd; `terms`: the
// query's term descriptors, read only for a disjunction): some term passes.
__device__ inline bool query_passes(const QDesc &qd, const QDesc *terms, bool has_dense, bool has_labels, uint32_t w,
                                    uint64_t sig, const uint16_t *sl, int ns = kMaxLabels) {
    if (qd.flags & kQOr) {
        for (int t = 0; t < qd.nterm; t++)
            if (point_passes(terms[t], has_dense, has_labels, w, sig, sl, ns)) return true;
        return false;
    }
    return point_passes(qd, has_dense, has_labels, w, sig, sl, ns);
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Keeps the best k (k <= 64) of query q's candidate buffer of capacity C,
// sorted ascending at the front, and tightens its threshold.  Whole wave;
// each lane ranks C/64 entries against all of them; ranks are unique because
// keys carry a point id or position.
template <int C>
__device__ inline void buf_reduce(uint64_t *buf, int32_t *bcnt, uint64_t *tau, int q, int k) {
    constexpr int EPL = (C + 63) / 64;
    uint64_t *b = buf + q * C;
    const int c = min(bcnt[q], C);
    const int lane = threadIdx.x & 63;
    uint64_t v[EPL];
    int rk[EPL];
#pragma unroll
    for (int e = 0; e < EPL; e++) {
        v[e] = lane + 64 * e < c ? b[lane + 64 * e] : ~0ull;
        rk[e] = 0;
    }
#pragma unroll 4
    for (int j = 0; j < c; j++) {
        const uint64_t u = b[j];
#pragma unroll
        for (int e = 0; e < EPL; e++) rk[e] += u < v[e] ? 1 : 0;
    }
    wave_sync();
#pragma unroll
    for (int e = 0; e < EPL; e++)
        if (v[e] != ~0ull && rk[e] < k) b[rk[e]] = v[e];
    wave_sync();
    const int nk = min(c, k);
    if (lane == 0) {
        bcnt[q] = nk;
        if (nk == k && b[k - 1] < tau[q]) tau[q] = b[k - 1];
    }
    wave_sync();
}

// One wave: collects the keys of query slots slot0 + [r0, r1) of a partial
// list array (slot_len keys per slot; `pcnt` gives the count per slot, or
// lists are padded with ~0) into an LDS pool of capacity CAP, keeping the
// best `keep` (<= 64) sorted at the front; returns the sum of cand[] over the
// live slots (0 when cand is null).  Slots with sel == 0 hold nothing.
template <int CAP>
__device__ inline int gather_best(uint64_t *pool, int32_t *npool, const uint64_t *partials, const int32_t *pcnt,
                                  const uint32_t *sel, const int32_t *cand, int64_t slot0, int r0, int r1,
                                  int slot_len, int keep) {
    const int lane = threadIdx.x & 63;
    uint64_t unused_bound = ~0ull;
    if (lane == 0) *npool = 0;
    wave_sync();
    int nc = 0;
    for (int rb = r0; rb < r1; rb += 64) {
        const int rr = rb + lane;
        const int64_t slot = slot0 + rr;
        const bool live = rr < r1 && sel[slot] != 0;
        const int c = live ? (pcnt ? pcnt[slot] : slot_len) : 0;
        if (live && cand) nc += cand[slot];
        int cmax = c;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) cmax = max(cmax, __shfl_xor(cmax, o, 64));
        for (int i = 0; i < cmax; i++) {
            const uint64_t key = i < c ? partials[slot * slot_len + i] : ~0ull;
            const bool has = key != ~0ull;
            const uint64_t bal = __ballot(has);
            if (*npool + 64 > CAP) buf_reduce<CAP>(pool, npool, &unused_bound, 0, keep);
            const int n2 = *npool;
            if (has) pool[n2 + __popcll(bal & lanemask_lt())] = key;
            wave_sync();
            if (lane == 0) *npool = n2 + __popcll(bal);
            wave_sync();
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nc += __shfl_xor(nc, o, 64);
    buf_reduce<CAP>(pool, npool, &unused_bound, 0, keep);
    return nc;
}

}  // namespace caps
