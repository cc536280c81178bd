// Index construction on the GPU (paper Algorithm 1; Section 5.2).
//
//   1. k-means (first-level partition f): init centroids at sampled points;
//      `iters` rounds of assign + update, then a final assign.
//        assign: score(x, c) = |c|^2 - 2 x.c (L2) or -x.c (IP), each dot a
//                sequential fma chain over dims; argmin, ties to smaller c.
//        update: FP64 sum of member coordinates in ascending point id,
//                divided by the count, rounded to FP32; empty clusters keep
//                their centroid; IP divides by the FP64 norm (spherical).
//   2. Attribute Frequency Tree per partition, truncated at height h.
//   3. CSR grouped by (partition, level), inside a sub-partition by dense
//      attribute values (attribute 0 first), then id, with vectors and
//      packed attributes permuted alongside (Appendix "Index size").
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "caps_device.h"
#include "caps_internal.h"

namespace caps {

// ------------------------------------------------------------------ sampler
// splitmix64 (Steele, Lea & Flood 2014) and a partial Fisher-Yates shuffle:
// for i < B, j = i + next() mod (n - i), swap.  Sequential and tiny; runs on
// the host inside the library.
static uint64_t sm64(uint64_t &s) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static std::vector<int32_t> sample_init(uint64_t seed, int64_t n, int32_t b) {
    std::vector<int32_t> ids((size_t)n);
    for (int64_t i = 0; i < n; i++) ids[(size_t)i] = (int32_t)i;
    std::vector<int32_t> out((size_t)b);
    uint64_t s = seed;
    for (int32_t i = 0; i < b; i++) {
        uint64_t r = sm64(s);
        int64_t j = (int64_t)i + (int64_t)(r % (uint64_t)(n - i));
        std::swap(ids[(size_t)i], ids[(size_t)j]);
        out[(size_t)i] = ids[(size_t)i];
    }
    return out;
}

// ------------------------------------------------------------------ kernels
__global__ void k_gather_rows(const float *__restrict__ x, const int32_t *__restrict__ ids, int32_t b,
                              int32_t d, float *__restrict__ out) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)b * d) return;
    int32_t c = (int32_t)(e / d), j = (int32_t)(e % d);
    out[e] = x[(int64_t)ids[c] * d + j];
}

// |c|^2 as a sequential fma chain.
__global__ void k_cnorm(const float *__restrict__ cent, int32_t b, int32_t d, float *__restrict__ out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= b) return;
    const float *r = cent + (int64_t)c * d;
    float acc = 0.0f;
    for (int j = 0; j < d; j++) acc = fmaf(r[j], r[j], acc);
    out[c] = acc;
}

// Score tile: 64 rows (points or queries) x 64 centroids per pass, 256
// threads, each owning 4 rows x 4 centroids.  Dimensions stream through LDS
// in chunks of kDC, transposed so that a thread reads 4 consecutive rows or
// centroids with one 16-byte load.  Every (row, centroid) accumulator sees
// dimensions in ascending order.
constexpr int kDC = 32;
constexpr int kTile = 64;

template <bool ARGMIN>
__global__ __launch_bounds__(256) void k_scores(const float *__restrict__ x, int64_t n, int32_t d,
                                                const float *__restrict__ cent,
                                                const float *__restrict__ cn, int32_t b,
                                                int32_t metric, int32_t *__restrict__ out_assign,
                                                float *__restrict__ out_scores) {
    __shared__ float xs[kDC][kTile + 4];
    __shared__ float cs[kDC][kTile + 4];
    const int t = threadIdx.x;
    const int ty = t >> 4, tx = t & 15;
    const int64_t r0 = (int64_t)blockIdx.x * kTile;
    uint64_t best[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    const int c_begin = ARGMIN ? 0 : blockIdx.y * kTile;
    const int c_end = ARGMIN ? b : min(b, c_begin + kTile);
    for (int c0 = c_begin; c0 < c_end; c0 += kTile) {
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
                    if (r0 + ri < n) v = x[(r0 + ri) * d + j0 + jj];
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
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int c = c0 + tx * 4 + k;
                if (c >= b) continue;
                const float s = canon0(metric == 0 ? cn[c] - 2.0f * acc[i][k] : -acc[i][k]);
                if (ARGMIN) {
                    const uint64_t key = ((uint64_t)f2ord(s) << 32) | (uint32_t)c;
                    best[i] = key < best[i] ? key : best[i];
                } else if (r < n) {
                    out_scores[r * b + c] = s;
                }
            }
        }
    }
    if (ARGMIN) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            uint64_t v = best[i];
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {
                uint64_t u = __shfl_xor(v, o, 64);
                v = u < v ? u : v;
            }
            const int64_t r = r0 + ty * 4 + i;
            if (tx == 0 && r < n) out_assign[r] = (int32_t)(uint32_t)(v & 0xFFFFFFFFu);
        }
    }
}

// ---- stable counting sort of item ids by key (ascending id within a key)
constexpr int kSortBlock = 4096;

__global__ __launch_bounds__(256) void k_sort_hist(const int32_t *__restrict__ keys, int64_t n,
                                                   int32_t nkeys, int32_t nblk,
                                                   int32_t *__restrict__ hist) {
    extern __shared__ int32_t cnt[];
    for (int i = threadIdx.x; i < nkeys; i += 256) cnt[i] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kSortBlock;
    const int64_t hi = min(n, lo + kSortBlock);
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) atomicAdd(&cnt[keys[i]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nkeys; i += 256) hist[(int64_t)i * nblk + blockIdx.x] = cnt[i];
}

// One wave per block walks its items in id order; lanes sharing a key get
// consecutive slots in lane order, so the result is stable.
__global__ __launch_bounds__(64) void k_sort_scatter(const int32_t *__restrict__ keys, int64_t n,
                                                     int32_t nkeys, int32_t nblk, int32_t nbits,
                                                     const int32_t *__restrict__ hscan,
                                                     int32_t *__restrict__ out) {
    extern __shared__ int32_t run[];
    for (int i = threadIdx.x; i < nkeys; i += 64) run[i] = hscan[(int64_t)i * nblk + blockIdx.x];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kSortBlock;
    const int64_t hi = min(n, lo + kSortBlock);
    for (int64_t g = lo; g < hi; g += 64) {
        const int64_t i = g + threadIdx.x;
        const bool valid = i < hi;
        const uint32_t key = valid ? (uint32_t)keys[i] : (uint32_t)nkeys;
        const uint64_t peers = wave_match(key, nbits);
        const int rank = __popcll(peers & lanemask_lt());
        const int base = valid ? run[key] : 0;
        if (valid) out[base + rank] = (int32_t)i;
        const bool leader = (peers >> threadIdx.x) == 1ull;   // highest lane of its group
        __syncthreads();
        if (valid && leader) run[key] = base + __popcll(peers);
        __syncthreads();
    }
}

// centroid update: one thread per (cluster, dim); FP64 sum in ascending id.
__global__ void k_update(const float *__restrict__ x, int32_t d, const int32_t *__restrict__ sorted,
                         const int32_t *__restrict__ hscan, int32_t nblk, int32_t b, int64_t n,
                         float *__restrict__ cent) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)b * d) return;
    const int c = (int)(e / d), j = (int)(e % d);
    const int32_t lo = hscan[(int64_t)c * nblk];
    const int32_t hi = (c + 1 < b) ? hscan[(int64_t)(c + 1) * nblk] : (int32_t)n;
    if (hi == lo) return;
    double s = 0.0;
    for (int32_t u = lo; u < hi; u++) s += (double)x[(int64_t)sorted[u] * d + j];
    cent[e] = (float)(s / (double)(hi - lo));
}

__global__ void k_normalize(float *__restrict__ cent, int32_t b, int32_t d,
                            const int32_t *__restrict__ hscan, int32_t nblk, int64_t n) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= b) return;
    const int32_t lo = hscan[(int64_t)c * nblk];
    const int32_t hi = (c + 1 < b) ? hscan[(int64_t)(c + 1) * nblk] : (int32_t)n;
    if (hi == lo) return;
    float *r = cent + (int64_t)c * d;
    double s2 = 0.0;
    for (int j = 0; j < d; j++) s2 += (double)r[j] * (double)r[j];
    const double nrm = sqrt(s2);
    if (nrm > 0.0)
        for (int j = 0; j < d; j++) r[j] = (float)((double)r[j] / nrm);
}

// ---- AFT + CSR, one workgroup per partition
struct AttrSrc {
    const uint32_t *dense;      // n x n_dense (original order)
    const int64_t *label_off;   // n+1 or null
    const uint32_t *labels;
};

__device__ inline bool holds_token(const AttrSrc &a, const Schema &s, int32_t id, int32_t tok) {
    if (tok < s.dense_off[s.n_dense]) {
        int at = 0;
        while (at + 1 < s.n_dense && tok >= s.dense_off[at + 1]) at++;
        return (int32_t)a.dense[(int64_t)id * s.n_dense + at] == tok - s.dense_off[at];
    }
    if (!a.label_off) return false;
    const uint32_t l = (uint32_t)(tok - s.dense_off[s.n_dense]);
    for (int64_t e = a.label_off[id]; e < a.label_off[id + 1]; e++)
        if (a.labels[e] == l) return true;
    return false;
}

constexpr int kAftNT = 256;

__global__ __launch_bounds__(kAftNT) void k_aft(const int32_t *__restrict__ sorted,
                                                const int32_t *__restrict__ hscan, int32_t nblk,
                                                int64_t n, int32_t b, int32_t h, Schema sch,
                                                AttrSrc src, int32_t *__restrict__ lev_tmp,
                                                int8_t *__restrict__ level, int32_t *__restrict__ tags,
                                                int32_t *__restrict__ perm,
                                                int32_t *__restrict__ offs) {
    extern __shared__ int32_t hist[];   // sch.n_tok
    __shared__ uint64_t red[kAftNT / kWave];
    __shared__ int32_t lcount[kMaxHeight + 1], lbase[kMaxHeight + 1], lrun[kMaxHeight + 1];
    __shared__ int scan_scratch[kAftNT / kWave + 1];
    __shared__ int32_t tag_s;
    const int p = blockIdx.x;
    const int t = threadIdx.x;
    const int32_t lo = hscan[(int64_t)p * nblk];
    const int32_t hi = (p + 1 < b) ? hscan[(int64_t)(p + 1) * nblk] : (int32_t)n;
    for (int32_t u = lo + t; u < hi; u += kAftNT) lev_tmp[u] = -1;
    __syncthreads();
    for (int j = 0; j < h; j++) {
        for (int i = t; i < sch.n_tok; i += kAftNT) hist[i] = 0;
        __syncthreads();
        for (int32_t u = lo + t; u < hi; u += kAftNT) {
            if (lev_tmp[u] >= 0) continue;
            const int32_t id = sorted[u];
            for (int a = 0; a < sch.n_dense; a++)
                atomicAdd(&hist[sch.dense_off[a] + (int32_t)src.dense[(int64_t)id * sch.n_dense + a]], 1);
            if (src.label_off)
                for (int64_t e = src.label_off[id]; e < src.label_off[id + 1]; e++)
                    atomicAdd(&hist[sch.dense_off[sch.n_dense] + (int32_t)src.labels[e]], 1);
        }
        __syncthreads();
        // most frequent token, ties to the smaller token
        uint64_t bestk = 0;
        for (int i = t; i < sch.n_tok; i += kAftNT) {
            const uint64_t key = ((uint64_t)(uint32_t)hist[i] << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
            bestk = key > bestk ? key : bestk;
        }
        bestk = wave_max_u64(bestk);
        if ((t & 63) == 0) red[t >> 6] = bestk;
        __syncthreads();
        if (t == 0) {
            uint64_t m = red[0];
            for (int w = 1; w < kAftNT / kWave; w++) m = red[w] > m ? red[w] : m;
            const uint32_t cnt = (uint32_t)(m >> 32);
            tag_s = cnt == 0 ? -1 : (int32_t)(0xFFFFFFFFu - (uint32_t)(m & 0xFFFFFFFFu));
            tags[(int64_t)p * h + j] = tag_s;
        }
        __syncthreads();
        const int32_t tag = tag_s;
        if (tag >= 0) {
            for (int32_t u = lo + t; u < hi; u += kAftNT) {
                if (lev_tmp[u] >= 0) continue;
                if (holds_token(src, sch, sorted[u], tag)) lev_tmp[u] = j;
            }
        }
        __syncthreads();
    }
    // remainder level, per-level counts
    if (t <= h) lcount[t] = 0;
    __syncthreads();
    for (int32_t u = lo + t; u < hi; u += kAftNT) {
        int32_t l = lev_tmp[u];
        if (l < 0) {
            l = h;
            lev_tmp[u] = h;
        }
        level[sorted[u]] = (int8_t)l;
        atomicAdd(&lcount[l], 1);
    }
    __syncthreads();
    if (t == 0) {
        int32_t s = 0;
        for (int l = 0; l <= h; l++) {
            lbase[l] = s;
            lrun[l] = 0;
            offs[(int64_t)p * (h + 1) + l] = lo + s;
            s += lcount[l];
        }
        if (p == b - 1) offs[(int64_t)b * (h + 1)] = (int32_t)n;
    }
    __syncthreads();
    // stable placement: level-major, in the order of `sorted` inside a level
    for (int32_t g = lo; g < hi; g += kAftNT) {
        const int32_t u = g + t;
        const int32_t l = u < hi ? lev_tmp[u] : -1;
        for (int lv = 0; lv <= h; lv++) {
            int tot;
            const int r = block_excl_scan<kAftNT>(l == lv ? 1 : 0, scan_scratch, &tot);
            if (l == lv) perm[lo + lbase[lv] + lrun[lv] + r] = sorted[u];
            __syncthreads();
            if (t == 0) lrun[lv] += tot;
            __syncthreads();
        }
    }
}

__global__ void k_permute_vecs(const float *__restrict__ x, const int32_t *__restrict__ perm, int64_t n,
                               int32_t d, float *__restrict__ vecs) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t pos = e / d;
    const int32_t j = (int32_t)(e % d);
    vecs[e] = x[(int64_t)perm[pos] * d + j];
}

__global__ void k_permute_attrs(const int32_t *__restrict__ perm, int64_t n, Schema sch, AttrSrc src,
                                uint32_t *__restrict__ words, uint64_t *__restrict__ sigs,
                                uint16_t *__restrict__ slots, int32_t lslots) {
    int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const int32_t id = perm[pos];
    if (words) {
        uint32_t w = 0;
        for (int a = 0; a < sch.n_dense; a++)
            w |= src.dense[(int64_t)id * sch.n_dense + a] << sch.field_shift[a];
        words[pos] = w;
    }
    if (sigs) {
        // the point's labels sorted ascending (insertion into its own slot
        // row), 0xFFFF padding after them
        uint16_t *s = slots + pos * lslots;
        int c = 0;
        uint64_t sig = 0;
        for (int64_t e = src.label_off[id]; e < src.label_off[id + 1] && c < lslots; e++) {
            const uint16_t l = (uint16_t)src.labels[e];
            sig |= 1ull << label_sig_bit(l);
            int i = c++;
            while (i > 0 && s[i - 1] > l) {
                s[i] = s[i - 1];
                i--;
            }
            s[i] = l;
        }
        for (int i = c; i < lslots; i++) s[i] = 0xFFFF;
        sigs[pos] = sig;
    }
}

// ------------------------------------------------------------------ host side
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

static caps_status dalloc(void **p, size_t bytes, int64_t *acct) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? CAPS_ENOMEM : CAPS_EDEVICE;
    }
    if (acct) *acct += (int64_t)bytes;
    return CAPS_OK;
}

#define CAPS_TRY(expr)                     \
    do {                                   \
        caps_status s_ = (expr);           \
        if (s_ != CAPS_OK) return s_;      \
    } while (0)

static int nbits_for(int32_t v) {
    int b = 1;
    while ((1 << b) <= v) b++;
    return b;
}

// Stable sort of ids 0..n-1 by keys[0..n) (keys < nkeys).  hscan (nkeys x
// nblk, key-major) ends up with the exclusive prefix: hscan[k*nblk] is the
// first sorted position of key k.
static caps_status stable_sort(const int32_t *keys, int64_t n, int32_t nkeys, int32_t *hist,
                               int32_t *hscan, int32_t *sums, int32_t *sorted, hipStream_t st) {
    const int32_t nblk = (int32_t)((n + kSortBlock - 1) / kSortBlock);
    const size_t lds = sizeof(int32_t) * (size_t)nkeys;
    hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(256), lds, st, keys, n, nkeys, nblk, hist);
    CAPS_TRY(exclusive_scan_i32(hist, hscan, (int64_t)nkeys * nblk, nullptr, sums, st));
    hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(64), lds, st, keys, n, nkeys, nblk,
                       nbits_for(nkeys), hscan, sorted);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

// ------------------------------------------------------------------ insertion
// Level of each new point in its (frozen) partition: the first tagged level
// whose tag the point holds, else the remainder h.
__global__ void k_insert_level(const int32_t *__restrict__ assign, int64_t n_new, int32_t h,
                               const int32_t *__restrict__ tags, Schema sch, AttrSrc src,
                               int8_t *__restrict__ level) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_new) return;
    const int32_t *t = tags + (int64_t)assign[i] * h;
    int8_t l = (int8_t)h;
    for (int j = 0; j < h; j++)
        if (t[j] >= 0 && holds_token(src, sch, (int32_t)i, t[j])) {
            l = (int8_t)j;
            break;
        }
    level[i] = l;
}

// New CSR position of every old one: shifted by the new points that land in
// earlier segments (add[s] = their count before segment s).
__global__ void k_insert_oldpos(const int32_t *__restrict__ offs, int32_t nseg, const int32_t *__restrict__ add,
                                int64_t n_old, int32_t *__restrict__ newpos) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n_old) return;
    int lo = 0, hi = nseg;   // the segment s with offs[s] <= pos < offs[s + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offs[mid] <= pos) lo = mid;
        else hi = mid;
    }
    newpos[pos] = (int32_t)pos + add[lo];
}

// dst row newpos[r] = src row r, rows of `w` 32-bit words.
__global__ void k_scatter_rows(const uint32_t *__restrict__ src, int64_t nrows, int32_t w,
                               const int32_t *__restrict__ newpos, uint32_t *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrows * w) return;
    const int64_t r = e / w;
    dst[(int64_t)newpos[r] * w + (e - r * w)] = src[e];
}

__global__ void k_iota(int32_t *__restrict__ p, int64_t n, int32_t base) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = base + (int32_t)i;
}

// ---- order inside a partition: by dense attribute values, then id
// Each point's dense values as one key, attribute 0 in the most significant
// field (the packed word holds attribute 0 in its least significant field).
__global__ void k_attr_key(const uint32_t *__restrict__ dense, int64_t n, Schema sch, int32_t tot_bits,
                           uint32_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t k = 0;
    for (int a = 0; a < sch.n_dense; a++)
        k |= dense[i * sch.n_dense + a] << (tot_bits - sch.field_shift[a] - sch.field_bits[a]);
    key[i] = k;
}

// out[i] = (key[seq[i]] >> shift) & mask
__global__ void k_seq_digit(const uint32_t *__restrict__ key, const int32_t *__restrict__ seq, int64_t n,
                            int32_t shift, uint32_t mask, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)((key[seq[i]] >> shift) & mask);
}

// out[i] = a[idx[i]]
__global__ void k_gather_i32(const int32_t *__restrict__ a, const int32_t *__restrict__ idx, int64_t n,
                             int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[idx[i]];
}

// The ids grouped by partition (hscan as stable_sort leaves it), inside a
// partition sorted by their dense attribute values (attribute 0 first), ties
// by ascending id: LSD passes of the stable counting sort over the key's
// digits, then the stable partition pass.  Points with equal values end up
// next to each other in every sub-partition, so a run of rows shares its
// values (the scans skip runs no query of a group can match).
static caps_status attribute_grouped(const uint32_t *ddense, const int32_t *assign, int64_t n, int32_t b,
                                     const Schema &sch, int32_t *hist, int32_t *hscan, int32_t *sums,
                                     int32_t *sorted, hipStream_t st) {
    constexpr int kDigit = 8;
    int32_t tot_bits = 0;
    for (int a = 0; a < sch.n_dense; a++) tot_bits += sch.field_bits[a];
    const unsigned grid = (unsigned)((n + 255) / 256);
    const int32_t nblk = (int32_t)((n + kSortBlock - 1) / kSortBlock);
    DevBuf dkey, dseq, dseq2, ddig, dord, dh, dhs, dsm;
    CAPS_HIP(hipMalloc(&dkey.p, sizeof(uint32_t) * (size_t)n));
    CAPS_HIP(hipMalloc(&dseq.p, sizeof(int32_t) * (size_t)n));
    CAPS_HIP(hipMalloc(&dseq2.p, sizeof(int32_t) * (size_t)n));
    CAPS_HIP(hipMalloc(&ddig.p, sizeof(int32_t) * (size_t)n));
    CAPS_HIP(hipMalloc(&dord.p, sizeof(int32_t) * (size_t)n));
    CAPS_HIP(hipMalloc(&dh.p, sizeof(int32_t) * ((size_t)1 << kDigit) * nblk));
    CAPS_HIP(hipMalloc(&dhs.p, sizeof(int32_t) * ((size_t)1 << kDigit) * nblk));
    CAPS_HIP(hipMalloc(&dsm.p, sizeof(int32_t) * (size_t)exclusive_scan_tiles(((int64_t)1 << kDigit) * nblk)));
    uint32_t *key = (uint32_t *)dkey.p;
    int32_t *seq = (int32_t *)dseq.p, *seq2 = (int32_t *)dseq2.p, *dig = (int32_t *)ddig.p, *ord = (int32_t *)dord.p;
    hipLaunchKernelGGL(k_attr_key, dim3(grid), dim3(256), 0, st, ddense, n, sch, tot_bits, key);
    hipLaunchKernelGGL(k_iota, dim3(grid), dim3(256), 0, st, seq, n, 0);
    for (int sh = 0; sh < tot_bits; sh += kDigit) {
        const int bits = std::min(kDigit, tot_bits - sh);
        hipLaunchKernelGGL(k_seq_digit, dim3(grid), dim3(256), 0, st, (const uint32_t *)key, (const int32_t *)seq,
                           n, sh, (uint32_t)((1u << bits) - 1u), dig);
        CAPS_TRY(stable_sort(dig, n, 1 << bits, (int32_t *)dh.p, (int32_t *)dhs.p, (int32_t *)dsm.p, ord, st));
        hipLaunchKernelGGL(k_gather_i32, dim3(grid), dim3(256), 0, st, (const int32_t *)seq, (const int32_t *)ord,
                           n, seq2);
        std::swap(seq, seq2);
    }
    hipLaunchKernelGGL(k_gather_i32, dim3(grid), dim3(256), 0, st, assign, (const int32_t *)seq, n, dig);
    CAPS_TRY(stable_sort(dig, n, b, hist, hscan, sums, ord, st));
    hipLaunchKernelGGL(k_gather_i32, dim3(grid), dim3(256), 0, st, (const int32_t *)seq, (const int32_t *)ord, n,
                       sorted);
    CAPS_HIP(hipGetLastError());
    // the buffers are freed at return: the stream must be done with them
    CAPS_HIP(hipStreamSynchronize(st));
    return CAPS_OK;
}

caps_status build_index(Index *ix, const float *x, int64_t n, int32_t d, const uint32_t *dense,
                        const int64_t *label_off, const uint32_t *labels,
                        const caps_build_params *p, hipStream_t st) {
    const int32_t b = ix->b, h = ix->h;
    const Schema &sch = ix->sch;
    const bool has_labels = label_off != nullptr;
    const int64_t nnz = has_labels ? label_off[n] : 0;

    // inputs on the device (freed at return)
    DevBuf dx, ddense, dloff, dlab, dinit, dassign, dhist, dhscan, dsums, dsorted, dlev;
    CAPS_HIP(hipMalloc(&dx.p, sizeof(float) * (size_t)n * d));
    CAPS_HIP(hipMemcpyAsync(dx.p, x, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice, st));
    if (sch.n_dense) {
        CAPS_HIP(hipMalloc(&ddense.p, sizeof(uint32_t) * (size_t)n * sch.n_dense));
        CAPS_HIP(hipMemcpyAsync(ddense.p, dense, sizeof(uint32_t) * (size_t)n * sch.n_dense,
                                hipMemcpyHostToDevice, st));
    }
    if (has_labels) {
        CAPS_HIP(hipMalloc(&dloff.p, sizeof(int64_t) * (size_t)(n + 1)));
        CAPS_HIP(hipMemcpyAsync(dloff.p, label_off, sizeof(int64_t) * (size_t)(n + 1),
                                hipMemcpyHostToDevice, st));
        CAPS_HIP(hipMalloc(&dlab.p, sizeof(uint32_t) * (size_t)(nnz > 0 ? nnz : 1)));
        if (nnz)
            CAPS_HIP(hipMemcpyAsync(dlab.p, labels, sizeof(uint32_t) * (size_t)nnz,
                                    hipMemcpyHostToDevice, st));
    }
    std::vector<int32_t> init;
    if (p->init_ids) {
        init.assign(p->init_ids, p->init_ids + b);
    } else {
        init = sample_init(p->seed, n, b);
    }
    CAPS_HIP(hipMalloc(&dinit.p, sizeof(int32_t) * (size_t)b));
    CAPS_HIP(hipMemcpyAsync(dinit.p, init.data(), sizeof(int32_t) * (size_t)b, hipMemcpyHostToDevice, st));

    // resident index arrays
    CAPS_TRY(dalloc((void **)&ix->cent, sizeof(float) * (size_t)b * d, &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->cnorm, sizeof(float) * (size_t)b, &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->tags, sizeof(int32_t) * (size_t)b * (h > 0 ? h : 1), &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->offs, sizeof(int32_t) * ((size_t)b * (h + 1) + 1), &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->perm, sizeof(int32_t) * (size_t)n, &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->assign, sizeof(int32_t) * (size_t)n, &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->level, sizeof(int8_t) * (size_t)n, &ix->bytes));
    CAPS_TRY(dalloc((void **)&ix->vecs, sizeof(float) * (size_t)n * d, &ix->bytes));
    if (sch.n_dense) CAPS_TRY(dalloc((void **)&ix->words, sizeof(uint32_t) * (size_t)n, &ix->bytes));
    if (has_labels) {
        CAPS_TRY(dalloc((void **)&ix->sigs, sizeof(uint64_t) * (size_t)n, &ix->bytes));
        CAPS_TRY(dalloc((void **)&ix->slots, sizeof(uint16_t) * (size_t)n * ix->lslots, &ix->bytes));
    }

    const int32_t nblk = (int32_t)((n + kSortBlock - 1) / kSortBlock);
    CAPS_HIP(hipMalloc(&dhist.p, sizeof(int32_t) * (size_t)b * nblk));
    CAPS_HIP(hipMalloc(&dhscan.p, sizeof(int32_t) * (size_t)b * nblk));
    CAPS_HIP(hipMalloc(&dsums.p, sizeof(int32_t) * (size_t)exclusive_scan_tiles((int64_t)b * nblk)));
    CAPS_HIP(hipMalloc(&dsorted.p, sizeof(int32_t) * (size_t)n));
    CAPS_HIP(hipMalloc(&dlev.p, sizeof(int32_t) * (size_t)n));
    float *X = (float *)dx.p;
    int32_t *A = ix->assign;
    int32_t *hist = (int32_t *)dhist.p, *hscan = (int32_t *)dhscan.p, *sorted = (int32_t *)dsorted.p;

    {
        const int64_t tot = (int64_t)b * d;
        hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X,
                           (const int32_t *)dinit.p, b, d, ix->cent);
    }
    const dim3 sgrid((unsigned)((n + kTile - 1) / kTile));
    if (p->assign) {
        // given partitions (learned, validated by the caller): one update of
        // the initial centroids gives each non-empty partition its mean
        CAPS_HIP(hipMemcpyAsync(A, p->assign, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
        CAPS_TRY(stable_sort(A, n, b, hist, hscan, (int32_t *)dsums.p, sorted, st));
        const int64_t tot = (int64_t)b * d;
        hipLaunchKernelGGL(k_update, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, d, sorted, hscan,
                           nblk, b, n, ix->cent);
        if (ix->metric == CAPS_METRIC_IP)
            hipLaunchKernelGGL(k_normalize, dim3((b + 255) / 256), dim3(256), 0, st, ix->cent, b, d, hscan, nblk,
                               n);
        CAPS_HIP(hipGetLastError());
    }
    for (int it = 0; !p->assign && it <= p->kmeans_iters; it++) {
        hipLaunchKernelGGL(k_cnorm, dim3((b + 255) / 256), dim3(256), 0, st, ix->cent, b, d, ix->cnorm);
        hipLaunchKernelGGL(k_scores<true>, sgrid, dim3(256), 0, st, X, n, d, ix->cent, ix->cnorm, b,
                           ix->metric, A, nullptr);
        CAPS_HIP(hipGetLastError());
        CAPS_TRY(stable_sort(A, n, b, hist, hscan, (int32_t *)dsums.p, sorted, st));
        if (it == p->kmeans_iters) break;
        const int64_t tot = (int64_t)b * d;
        hipLaunchKernelGGL(k_update, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, d, sorted,
                           hscan, nblk, b, n, ix->cent);
        if (ix->metric == CAPS_METRIC_IP)
            hipLaunchKernelGGL(k_normalize, dim3((b + 255) / 256), dim3(256), 0, st, ix->cent, b, d, hscan,
                               nblk, n);
        CAPS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_cnorm, dim3((b + 255) / 256), dim3(256), 0, st, ix->cent, b, d, ix->cnorm);

    AttrSrc src{(const uint32_t *)ddense.p, (const int64_t *)dloff.p, (const uint32_t *)dlab.p};
    if (sch.n_dense)
        CAPS_TRY(attribute_grouped((const uint32_t *)ddense.p, A, n, b, sch, hist, hscan, (int32_t *)dsums.p,
                                   sorted, st));
    hipLaunchKernelGGL(k_aft, dim3(b), dim3(kAftNT), sizeof(int32_t) * (size_t)sch.n_tok, st, sorted,
                       hscan, nblk, n, b, h, sch, src, (int32_t *)dlev.p, ix->level, ix->tags, ix->perm,
                       ix->offs);
    CAPS_HIP(hipGetLastError());
    {
        const int64_t tot = n * d;
        hipLaunchKernelGGL(k_permute_vecs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X,
                           ix->perm, n, d, ix->vecs);
        hipLaunchKernelGGL(k_permute_attrs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ix->perm,
                           n, sch, src, ix->words, ix->sigs, ix->slots, ix->lslots);
        CAPS_HIP(hipGetLastError());
    }
    ix->h_offs.resize((size_t)b * (h + 1) + 1);
    CAPS_HIP(hipMemcpyAsync(ix->h_offs.data(), ix->offs, sizeof(int32_t) * ix->h_offs.size(),
                            hipMemcpyDeviceToHost, st));
    CAPS_HIP(hipStreamSynchronize(st));
    int32_t mx = 0;
    for (size_t s = 0; s + 1 < ix->h_offs.size(); s++) mx = std::max(mx, ix->h_offs[s + 1] - ix->h_offs[s]);
    ix->max_sub = mx;
    return CAPS_OK;
}

}  // namespace caps

namespace caps {

// Dynamic insertion (Table 1 "Dynamic Insertions"): the partition model
// stays frozen.  New point i gets id n + i, the partition the k-means
// assignment picks and the first tagged level whose tag it holds; the old
// rows keep their CSR order, each moved by the number of new rows in earlier
// segments, and the new rows go to the end of their segments in id order.  Every per-row array (vectors, packed
// attributes, low-precision copy and its norms, permutation) is laid out
// again in one pass; centroids, tags and the router are unchanged.
caps_status insert_points(Index *ix, const float *x, int64_t n_new, const uint32_t *dense, const int64_t *label_off,
                          const uint32_t *labels, hipStream_t st) {
    const Schema &sch = ix->sch;
    const int64_t n_old = ix->n, n_tot = n_old + n_new;
    const int32_t d = ix->d, b = ix->b, h = ix->h, nseg = b * (h + 1);
    const int64_t nnz = label_off ? label_off[n_new] : 0;
    DevBuf dx, ddense, dloff, dlab, dassign, dlevel, dnewpos_new, dnewpos_old, dadd, diota;
    CAPS_HIP(hipMalloc(&dx.p, sizeof(float) * (size_t)n_new * d));
    CAPS_HIP(hipMemcpyAsync(dx.p, x, sizeof(float) * (size_t)n_new * d, hipMemcpyHostToDevice, st));
    if (sch.n_dense) {
        CAPS_HIP(hipMalloc(&ddense.p, sizeof(uint32_t) * (size_t)n_new * sch.n_dense));
        CAPS_HIP(hipMemcpyAsync(ddense.p, dense, sizeof(uint32_t) * (size_t)n_new * sch.n_dense,
                                hipMemcpyHostToDevice, st));
    }
    if (label_off) {
        CAPS_HIP(hipMalloc(&dloff.p, sizeof(int64_t) * (size_t)(n_new + 1)));
        CAPS_HIP(hipMemcpyAsync(dloff.p, label_off, sizeof(int64_t) * (size_t)(n_new + 1), hipMemcpyHostToDevice, st));
        CAPS_HIP(hipMalloc(&dlab.p, sizeof(uint32_t) * (size_t)(nnz > 0 ? nnz : 1)));
        if (nnz) CAPS_HIP(hipMemcpyAsync(dlab.p, labels, sizeof(uint32_t) * (size_t)nnz, hipMemcpyHostToDevice, st));
    }
    AttrSrc src{(const uint32_t *)ddense.p, (const int64_t *)dloff.p, (const uint32_t *)dlab.p};
    // partition and level of the new points
    CAPS_HIP(hipMalloc(&dassign.p, sizeof(int32_t) * (size_t)n_new));
    CAPS_HIP(hipMalloc(&dlevel.p, sizeof(int8_t) * (size_t)n_new));
    hipLaunchKernelGGL(k_scores<true>, dim3((unsigned)((n_new + kTile - 1) / kTile)), dim3(256), 0, st,
                       (const float *)dx.p, n_new, d, ix->cent, ix->cnorm, b, ix->metric, (int32_t *)dassign.p,
                       nullptr);
    hipLaunchKernelGGL(k_insert_level, dim3((unsigned)((n_new + 255) / 256)), dim3(256), 0, st,
                       (const int32_t *)dassign.p, n_new, h, ix->tags, sch, src, (int8_t *)dlevel.p);
    CAPS_HIP(hipGetLastError());
    std::vector<int32_t> a_new((size_t)n_new);
    std::vector<int8_t> l_new((size_t)n_new);
    CAPS_HIP(hipMemcpyAsync(a_new.data(), dassign.p, sizeof(int32_t) * (size_t)n_new, hipMemcpyDeviceToHost, st));
    CAPS_HIP(hipMemcpyAsync(l_new.data(), dlevel.p, sizeof(int8_t) * (size_t)n_new, hipMemcpyDeviceToHost, st));
    CAPS_HIP(hipStreamSynchronize(st));
    // new layout on the host: counts per segment, offsets, positions
    std::vector<int32_t> cnt((size_t)nseg, 0), add((size_t)nseg + 1, 0), run((size_t)nseg, 0);
    for (int64_t i = 0; i < n_new; i++) cnt[(size_t)a_new[(size_t)i] * (h + 1) + l_new[(size_t)i]]++;
    for (int32_t sgi = 0; sgi < nseg; sgi++) add[(size_t)sgi + 1] = add[(size_t)sgi] + cnt[(size_t)sgi];
    std::vector<int32_t> offs_new((size_t)nseg + 1), pos_new((size_t)n_new);
    for (int32_t sgi = 0; sgi <= nseg; sgi++) offs_new[(size_t)sgi] = ix->h_offs[(size_t)sgi] + add[(size_t)sgi];
    for (int64_t i = 0; i < n_new; i++) {
        const int32_t sg = a_new[(size_t)i] * (h + 1) + l_new[(size_t)i];
        pos_new[(size_t)i] = ix->h_offs[(size_t)sg + 1] + add[(size_t)sg] + run[(size_t)sg]++;
    }
    CAPS_HIP(hipMalloc(&dnewpos_new.p, sizeof(int32_t) * (size_t)n_new));
    CAPS_HIP(hipMemcpyAsync(dnewpos_new.p, pos_new.data(), sizeof(int32_t) * (size_t)n_new, hipMemcpyHostToDevice, st));
    CAPS_HIP(hipMalloc(&dadd.p, sizeof(int32_t) * (size_t)(nseg + 1)));
    CAPS_HIP(hipMemcpyAsync(dadd.p, add.data(), sizeof(int32_t) * (size_t)(nseg + 1), hipMemcpyHostToDevice, st));
    CAPS_HIP(hipMalloc(&dnewpos_old.p, sizeof(int32_t) * (size_t)(n_old > 0 ? n_old : 1)));
    hipLaunchKernelGGL(k_insert_oldpos, dim3((unsigned)((n_old + 255) / 256)), dim3(256), 0, st, ix->offs, nseg,
                       (const int32_t *)dadd.p, n_old, (int32_t *)dnewpos_old.p);
    CAPS_HIP(hipGetLastError());
    const int32_t *np_old = (const int32_t *)dnewpos_old.p, *np_new = (const int32_t *)dnewpos_new.p;

    // every array is first built anew beside the old one; only when all of
    // them are ready are they swapped in (an error leaves the index as it was)
    struct Swap {
        void **slot;
        void *fresh;
        size_t grow;
    };
    std::vector<Swap> swaps;
    struct Pending {
        std::vector<Swap> *v;
        ~Pending() {
            for (auto &sw : *v)
                if (sw.fresh) (void)hipFree(sw.fresh);
        }
    } pending{&swaps};
    // a per-row array in CSR order: old rows moved, new rows (`fresh`, input
    // order) placed
    auto relayout = [&](void **arr, size_t row_bytes, const void *fresh) -> caps_status {
        if (!*arr) return CAPS_OK;
        void *out = nullptr;
        CAPS_TRY(dalloc(&out, row_bytes * (size_t)n_tot, nullptr));
        swaps.push_back({arr, out, row_bytes * (size_t)n_new});
        const int32_t w = (int32_t)(row_bytes / 4);
        hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((n_old * w + 255) / 256)), dim3(256), 0, st,
                           (const uint32_t *)*arr, n_old, w, np_old, (uint32_t *)out);
        hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((n_new * w + 255) / 256)), dim3(256), 0, st,
                           (const uint32_t *)fresh, n_new, w, np_new, (uint32_t *)out);
        CAPS_HIP(hipGetLastError());
        return CAPS_OK;
    };
    // a per-point array in id order: the new points appended
    auto append = [&](void **arr, size_t elem, const void *fresh) -> caps_status {
        void *out = nullptr;
        CAPS_TRY(dalloc(&out, elem * (size_t)n_tot, nullptr));
        swaps.push_back({arr, out, elem * (size_t)n_new});
        CAPS_HIP(hipMemcpyAsync(out, *arr, elem * (size_t)n_old, hipMemcpyDeviceToDevice, st));
        CAPS_HIP(hipMemcpyAsync((char *)out + elem * (size_t)n_old, fresh, elem * (size_t)n_new,
                                hipMemcpyDeviceToDevice, st));
        return CAPS_OK;
    };
    // the new rows of every array, in input order
    DevBuf fperm, fwords, fsigs, fslots, flvec, fscale, fxn, ferr, fnrm;
    CAPS_HIP(hipMalloc(&fperm.p, sizeof(int32_t) * (size_t)n_new));
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n_new + 255) / 256)), dim3(256), 0, st, (int32_t *)fperm.p, n_new,
                       (int32_t)n_old);
    CAPS_HIP(hipMalloc(&diota.p, sizeof(int32_t) * (size_t)n_new));
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n_new + 255) / 256)), dim3(256), 0, st, (int32_t *)diota.p, n_new, 0);
    if (ix->words) CAPS_HIP(hipMalloc(&fwords.p, sizeof(uint32_t) * (size_t)n_new));
    if (ix->sigs) {
        CAPS_HIP(hipMalloc(&fsigs.p, sizeof(uint64_t) * (size_t)n_new));
        CAPS_HIP(hipMalloc(&fslots.p, sizeof(uint16_t) * (size_t)n_new * ix->lslots));
    }
    hipLaunchKernelGGL(k_permute_attrs, dim3((unsigned)((n_new + 255) / 256)), dim3(256), 0, st,
                       (const int32_t *)diota.p, n_new, sch, src, (uint32_t *)fwords.p, (uint64_t *)fsigs.p,
                       (uint16_t *)fslots.p, ix->lslots);
    CAPS_HIP(hipGetLastError());
    const size_t eb = ix->prec == CAPS_PREC_FP8 ? 1 : 2;
    if (ix->prec != CAPS_PREC_NONE) {
        CAPS_HIP(hipMalloc(&flvec.p, (size_t)n_new * ix->dpad * eb));
        CAPS_HIP(hipMalloc(&fxn.p, sizeof(float) * (size_t)n_new));
        CAPS_HIP(hipMalloc(&ferr.p, sizeof(float) * (size_t)n_new));
        CAPS_HIP(hipMalloc(&fnrm.p, sizeof(float) * (size_t)n_new));
        if (ix->prec == CAPS_PREC_FP8) CAPS_HIP(hipMalloc(&fscale.p, sizeof(float) * (size_t)n_new));
        CAPS_TRY(quantize_rows(ix, (const float *)dx.p, n_new, flvec.p, (float *)fscale.p, (float *)fxn.p,
                               (float *)ferr.p, (float *)fnrm.p, st));
    }
    CAPS_TRY(relayout((void **)&ix->perm, sizeof(int32_t), fperm.p));
    CAPS_TRY(relayout((void **)&ix->vecs, sizeof(float) * (size_t)d, dx.p));
    CAPS_TRY(relayout((void **)&ix->words, sizeof(uint32_t), fwords.p));
    CAPS_TRY(relayout((void **)&ix->sigs, sizeof(uint64_t), fsigs.p));
    CAPS_TRY(relayout((void **)&ix->slots, sizeof(uint16_t) * ix->lslots, fslots.p));
    CAPS_TRY(relayout(&ix->lvecs, (size_t)ix->dpad * eb, flvec.p));
    CAPS_TRY(relayout((void **)&ix->lscale, sizeof(float), fscale.p));
    CAPS_TRY(relayout((void **)&ix->xnorm, sizeof(float), fxn.p));
    CAPS_TRY(relayout((void **)&ix->lerr, sizeof(float), ferr.p));
    CAPS_TRY(relayout((void **)&ix->lnrm, sizeof(float), fnrm.p));
    CAPS_TRY(append((void **)&ix->assign, sizeof(int32_t), dassign.p));
    CAPS_TRY(append((void **)&ix->level, sizeof(int8_t), dlevel.p));
    {
        void *o = nullptr;
        CAPS_TRY(dalloc(&o, sizeof(int32_t) * (size_t)(nseg + 1), nullptr));
        swaps.push_back({(void **)&ix->offs, o, 0});
        CAPS_HIP(hipMemcpyAsync(o, offs_new.data(), sizeof(int32_t) * (size_t)(nseg + 1), hipMemcpyHostToDevice, st));
    }
    CAPS_HIP(hipStreamSynchronize(st));
    // commit: swap the new arrays in, release the old ones
    for (auto &sw : swaps) {
        (void)hipFree(*sw.slot);
        *sw.slot = sw.fresh;
        sw.fresh = nullptr;
        ix->bytes += (int64_t)sw.grow;
    }
    ix->h_offs = offs_new;
    int32_t mx = 0;
    for (int32_t sgi = 0; sgi < nseg; sgi++) mx = std::max(mx, offs_new[(size_t)sgi + 1] - offs_new[(size_t)sgi]);
    ix->max_sub = mx;
    ix->n = n_tot;
    return CAPS_OK;
}

}  // namespace caps
