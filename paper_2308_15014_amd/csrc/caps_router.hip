// Learned router: a two-layer perceptron that maps a query vector and its
// constraints to one logit per partition, trained on the GPU on the
// partitions that hold each query's exact filtered top-k (the filtered-label
// idea of the paper's CAPS-BLISS variant, Section 5.2, with the k-means
// partitions kept fixed).
//
//   x = [q * in_scale + in_shift || e(C) || 0]   (BF16, dpad = (d + 64) rounded up to 32)
//   h = relu(W1 x + b1)                           (BF16 after the product)
//   z = W2 h + b2                                 (FP32 logits, one per partition)
//
// e(C) is 64-wide multi-hot: every valid constraint pair's token (dense
// attribute i, value v: off_i + v; label l: off_L + l) sets position
// mix64(token) mod 64, mix64 being splitmix64's output function.
//
// Training products run on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) in this file's GEMM kernels; the two inference products (a
// plain GEMM with a bias or bias + ReLU epilogue) go to hipBLASLt, with these
// kernels for any shape it has no algorithm for.  The softmax cross-entropy,
// bias gradients and Adam (FP32 masters, BF16 copies) are plain kernels.
#include <hipblaslt/hipblaslt.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "caps_device.h"
#include "caps_internal.h"

namespace caps {

constexpr int kEmbed = 64;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------------ input rows (K14)
// One workgroup per query: the affine map of the vector (product, then sum,
// in FP32), BF16-rounded, then the hashed constraint tokens.
__global__ __launch_bounds__(64) void k_router_input(const float *__restrict__ q, int32_t nq, int32_t d,
                                                     const int32_t *__restrict__ con_off,
                                                     const int32_t *__restrict__ con_attr,
                                                     const int32_t *__restrict__ con_val, int32_t n_con, Schema sch,
                                                     float scale, float shift, int32_t dpad,
                                                     uint16_t *__restrict__ X) {
    const int64_t i = blockIdx.x;
    if (i >= nq) return;
    uint16_t *row = X + i * dpad;
    for (int j = threadIdx.x; j < dpad; j += 64) {
        uint16_t v = 0;
        if (j < d) {
            const float a = q[i * d + j] * scale;
            v = bf16_rne(a + shift);
        }
        row[j] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t lo = con_off[i], hi = con_off[i + 1];
        if (lo >= 0 && hi >= lo && hi <= n_con) {
            for (int32_t e = lo; e < hi; e++) {
                const int32_t a = con_attr[e], v = con_val[e];
                int64_t tok = -1;
                if (a >= 0 && a < sch.n_dense && v >= 0 && v < sch.dense_vocab[a])
                    tok = sch.dense_off[a] + v;
                else if (a == sch.n_dense && sch.label_vocab > 0 && v >= 0 && v < sch.label_vocab)
                    tok = sch.dense_off[sch.n_dense] + v;
                if (tok >= 0) row[d + (int)(mix64((uint64_t)tok) % kEmbed)] = 0x3F80;   // BF16 1.0
            }
        }
    }
}

// ------------------------------------------------------------------ GEMM (K11, K12)
// C[m][n] = sum_k A(m, k) B(n, k), A(m, k) = A[m*sam + k*sak], B(n, k) =
// B[n*sbn + k*sbk] (BF16), FP32 accumulation.  128 x 128 tile per
// workgroup, four waves of 64 x 64 (4 x 4 blocks of
// v_mfma_f32_16x16x32_bf16), K in steps of 64 through LDS.
// Tiles are numbered in groups of kGroupM row tiles (every column tile of a
// group before the next group), and when the tile count divides evenly each
// XCD (workgroups are dealt to the 8 dies in turn) takes one contiguous range
// of that order, so a die's working set of rows and columns stays in its L2.
// Epilogue: + bias[n], ReLU, zero where mask(m, n) <= 0 (a BF16 array with
// leading dimension ldm), negation (scores, smaller is better); written as
// FP32 and/or BF16 with leading dimension ldc.
//
// Two kernels: k_gemm_nt for operands whose rows are K-contiguous (every
// forward product and inference), with branch-free loads issued two K steps
// ahead into registers and two LDS buffers (one barrier per step); and
// k_gemm_bf16 for any strides (the transposed operands of the weight
// gradients), which can also split K over blockIdx.y into FP32 partial
// products summed afterwards in a fixed order.
enum { kGemmRelu = 1, kGemmMask = 2, kGemmNeg = 4 };
// operand layouts of the strided kernel: K-contiguous 16-byte runs,
// row-contiguous 16-byte runs, else element gathers
enum { kGemmVecA = 8, kGemmVecB = 16, kGemmRowA = 32, kGemmRowB = 64 };
constexpr int kGT = 128, kGK = 64, kGKP = kGK + 8, kGroupM = 8;
constexpr int kGLoads = kGT * kGK / (8 * 256);   // 16-byte groups per thread per operand and step

__device__ inline void gemm_tile_origin(int32_t M, int32_t N, int64_t &m0, int64_t &n0) {
    const int64_t gm = (M + kGT - 1) / kGT, gn = (N + kGT - 1) / kGT, T = gm * gn;
    int64_t L = blockIdx.x;
    if (T % kXcds == 0) L = (L % kXcds) * (T / kXcds) + L / kXcds;
    const int64_t gsz = (int64_t)kGroupM * gn, g0 = (L / gsz) * kGroupM, rr = L % gsz;
    const int64_t gh = gm - g0 < kGroupM ? gm - g0 : kGroupM;
    m0 = (g0 + rr % gh) * kGT;
    n0 = (rr / gh) * kGT;
}

// The products of one wave's 64 x 64 block: 4 x 4 16 x 16 blocks; D row
// (lane/16)*4 + r, column lane%16 of each.
__device__ inline void gemm_epilogue(const f32x4 (&acc)[4][4], int64_t m0, int64_t n0, int32_t M, int32_t N,
                                     const float *__restrict__ bias, int32_t flags, const uint16_t *__restrict__ mask,
                                     int64_t ldm, float *__restrict__ C32, uint16_t *__restrict__ C16, int64_t ldc) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t mm = m0 + i * 16 + (lane >> 4) * 4 + r;
                const int64_t nn = n0 + j * 16 + (lane & 15);
                if (mm >= M || nn >= N) continue;
                float v = acc[i][j][r];
                if (bias) v = v + bias[nn];
                if (flags & kGemmRelu) v = fmaxf(v, 0.0f);
                if ((flags & kGemmMask) && !(__builtin_bit_cast(float, (uint32_t)mask[mm * ldm + nn] << 16) > 0.0f))
                    v = 0.0f;
                if (flags & kGemmNeg) v = canon0(-v);
                if (C32) C32[mm * ldc + nn] = v;
                if (C16) C16[mm * ldc + nn] = bf16_rne(v);
            }
}

__device__ inline void gemm_mfma_step(const uint16_t (*As)[kGKP], const uint16_t (*Bs)[kGKP], int wm, int wn,
                                      f32x4 (&acc)[4][4]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 32) {
        bf16x8 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            a[i] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&As[wm + i * 16 + (lane & 15)][ks + (lane >> 4) * 8]));
            b[i] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&Bs[wn + i * 16 + (lane & 15)][ks + (lane >> 4) * 8]));
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// K-contiguous operands: A row m at A + m*lda, B row n at B + n*ldb, K a
// multiple of 8, rows 16-byte aligned, every element offset below 2^31.
// Thread t loads rows t/8 + 32u (u < 4) of each operand, columns
// (t%8)*8 .. +7 of the step; rows past M or N and the K tail are loaded
// clamped to an element in range and zeroed by a select.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_nt(
    const uint16_t *__restrict__ A, int32_t lda, const uint16_t *__restrict__ B, int32_t ldb, int32_t M, int32_t N,
    int32_t K, const float *__restrict__ bias, int32_t flags, const uint16_t *__restrict__ mask, int64_t ldm,
    float *__restrict__ C32, uint16_t *__restrict__ C16, int64_t ldc) {
    __shared__ __align__(16) uint16_t As[2][kGT][kGKP];
    __shared__ __align__(16) uint16_t Bs[2][kGT][kGKP];
    const int t = threadIdx.x, w = t >> 6;
    int64_t m0, n0;
    gemm_tile_origin(M, N, m0, n0);
    const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
    const int kk0 = (t & 7) * 8;
    int32_t oa[4], ob[4];
    uint32_t ok = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int r = (t >> 3) + 32 * u;
        const int64_t ra = m0 + r, rb = n0 + r;
        ok |= (ra < M ? 1u : 0u) << u;
        ok |= (rb < N ? 1u : 0u) << (4 + u);
        oa[u] = (int32_t)((ra < M ? ra : M - 1) * (int64_t)lda) + kk0;
        ob[u] = (int32_t)((rb < N ? rb : N - 1) * (int64_t)ldb) + kk0;
    }
    auto fetch = [&](uint4 (&ga)[4], uint4 (&gb)[4], int32_t k0) {
        const bool okk = k0 + kk0 < K;
        const int32_t kc = okk ? k0 : K - 8 - kk0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint4 va = *reinterpret_cast<const uint4 *>(A + oa[u] + kc);
            const uint4 vb = *reinterpret_cast<const uint4 *>(B + ob[u] + kc);
            const bool ka = okk && ((ok >> u) & 1u), kb = okk && ((ok >> (4 + u)) & 1u);
            ga[u] = make_uint4(ka ? va.x : 0u, ka ? va.y : 0u, ka ? va.z : 0u, ka ? va.w : 0u);
            gb[u] = make_uint4(kb ? vb.x : 0u, kb ? vb.y : 0u, kb ? vb.z : 0u, kb ? vb.w : 0u);
        }
    };
    auto stage = [&](int buf, const uint4 (&ga)[4], const uint4 (&gb)[4]) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int r = (t >> 3) + 32 * u;
            *reinterpret_cast<uint4 *>(&As[buf][r][kk0]) = ga[u];
            *reinterpret_cast<uint4 *>(&Bs[buf][r][kk0]) = gb[u];
        }
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // a0/b0 and a1/b1 alternate: while step s is multiplied from LDS buffer
    // s%2, step s+1 is staged into the other buffer and step s+2 (or s+3)
    // is in flight into the registers just staged
    const int32_t ns = (K + kGK - 1) / kGK;
    uint4 a0[4], b0[4], a1[4], b1[4];
    fetch(a0, b0, 0);
    if (ns > 1) fetch(a1, b1, kGK);
    stage(0, a0, b0);
    if (ns > 2) fetch(a0, b0, 2 * kGK);
    __syncthreads();
    for (int32_t s = 0; s < ns; s += 2) {
        gemm_mfma_step(As[0], Bs[0], wm, wn, acc);
        if (s + 1 < ns) {
            stage(1, a1, b1);
            if (s + 3 < ns) fetch(a1, b1, (s + 3) * kGK);
        }
        __syncthreads();
        if (s + 1 < ns) {
            gemm_mfma_step(As[1], Bs[1], wm, wn, acc);
            if (s + 2 < ns) {
                stage(0, a0, b0);
                if (s + 4 < ns) fetch(a0, b0, (s + 4) * kGK);
            }
            __syncthreads();
        }
    }
    gemm_epilogue(acc, m0 + wm, n0 + wn, M, N, bias, flags, mask, ldm, C32, C16, ldc);
}

// Loads one operand tile (rows r0.., k0..) into registers as 16-byte groups
// of 8 elements: 8 consecutive k of one row, or (row-contiguous) 8
// consecutive rows of one k.  Out-of-range elements read as zero.
__device__ inline void gemm_fetch(uint4 (&g)[kGLoads], const uint16_t *__restrict__ P, int64_t srow, int64_t sk,
                                  int64_t r0, int32_t R, int64_t k0, int64_t K, int vec, int rowv) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < kGLoads; u++) {
        const int e = t + u * 256;
        if (rowv) {
            const int kk = e / (kGT / 8), rg = (e % (kGT / 8)) * 8;
            const int64_t k = k0 + kk, r = r0 + rg;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (k < K) {
                if (r + 8 <= R) {
                    v = *reinterpret_cast<const uint4 *>(P + k * sk + r);
                } else {
                    uint16_t h[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) h[i] = r + i < R ? P[k * sk + r + i] : (uint16_t)0;
                    v = __builtin_bit_cast(uint4, h);
                }
            }
            g[u] = v;
        } else {
            const int r = e / (kGK / 8), kk = (e % (kGK / 8)) * 8;
            const int64_t row = r0 + r, k = k0 + kk;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (row < R) {
                if (vec) {   // K-range ends are multiples of 8: the group is all in or all out
                    if (k < K) v = *reinterpret_cast<const uint4 *>(P + row * srow + k);
                } else {
                    uint16_t h[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) h[i] = k + i < K ? P[row * srow + (k + i) * sk] : (uint16_t)0;
                    v = __builtin_bit_cast(uint4, h);
                }
            }
            g[u] = v;
        }
    }
}

__device__ inline void gemm_stage(uint16_t (*S)[kGKP], const uint4 (&g)[kGLoads], int rowv) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < kGLoads; u++) {
        const int e = t + u * 256;
        if (rowv) {
            const int kk = e / (kGT / 8), rg = (e % (kGT / 8)) * 8;
            uint16_t h[8];
            *reinterpret_cast<uint4 *>(h) = g[u];
#pragma unroll
            for (int i = 0; i < 8; i++) S[rg + i][kk] = h[i];
        } else {
            const int r = e / (kGK / 8), kk = (e % (kGK / 8)) * 8;
            *reinterpret_cast<uint4 *>(&S[r][kk]) = g[u];
        }
    }
}

// Any strides.  With gridDim.y = S > 1, workgroup (x, y) multiplies K range
// [y*kchunk, min(K, (y+1)*kchunk)) and writes its plain FP32 partial product
// to C32 + y*M*ldc (no epilogue).
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t *__restrict__ A, int64_t sam, int64_t sak,
                                                   const uint16_t *__restrict__ B, int64_t sbn, int64_t sbk,
                                                   int32_t M, int32_t N, int32_t K, int32_t kchunk,
                                                   const float *__restrict__ bias, int32_t flags,
                                                   const uint16_t *__restrict__ mask, int64_t ldm,
                                                   float *__restrict__ C32, uint16_t *__restrict__ C16,
                                                   int64_t ldc) {
    __shared__ __align__(16) uint16_t As[kGT][kGKP];
    __shared__ __align__(16) uint16_t Bs[kGT][kGKP];
    const int t = threadIdx.x, w = t >> 6;
    int64_t m0, n0;
    gemm_tile_origin(M, N, m0, n0);
    const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
    const int va = (flags & kGemmVecA) != 0, vb = (flags & kGemmVecB) != 0;
    const int ra = (flags & kGemmRowA) != 0, rb = (flags & kGemmRowB) != 0;
    const int64_t klo = (int64_t)blockIdx.y * kchunk, khi = klo + kchunk < K ? klo + kchunk : K;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    uint4 pa[kGLoads], pb[kGLoads];
    gemm_fetch(pa, A, sam, sak, m0, M, klo, khi, va, ra);
    gemm_fetch(pb, B, sbn, sbk, n0, N, klo, khi, vb, rb);
    for (int64_t k0 = klo; k0 < khi; k0 += kGK) {
        gemm_stage(As, pa, ra);
        gemm_stage(Bs, pb, rb);
        __syncthreads();
        if (k0 + kGK < khi) {
            gemm_fetch(pa, A, sam, sak, m0, M, k0 + kGK, khi, va, ra);
            gemm_fetch(pb, B, sbn, sbk, n0, N, k0 + kGK, khi, vb, rb);
        }
        gemm_mfma_step(As, Bs, wm, wn, acc);
        __syncthreads();
    }
    if (gridDim.y > 1)
        gemm_epilogue(acc, m0 + wm, n0 + wn, M, N, nullptr, 0, nullptr, 0, C32 + (int64_t)blockIdx.y * M * ldc,
                      nullptr, ldc);
    else
        gemm_epilogue(acc, m0 + wm, n0 + wn, M, N, bias, flags, mask, ldm, C32, C16, ldc);
}

// out[i] = sum over s = 0..S-1 (in order) of P[s*n + i]
__global__ void k_sum_parts(const float *__restrict__ P, int32_t S, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = 0.0f;
    for (int32_t s = 0; s < S; s++) v += P[s * n + i];
    out[i] = v;
}

// Size in floats of the training scratch that holds split-K partial
// products and column-sum parts (32 MiB).
constexpr int64_t kGemmParts = 8ll << 20;

// parts: kGemmParts floats of scratch for split-K (null: no split)
static caps_status gemm(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbn, int64_t sbk,
                        int32_t M, int32_t N, int32_t K, const float *bias, int32_t flags, const uint16_t *mask,
                        int64_t ldm, float *C32, uint16_t *C16, int64_t ldc, hipStream_t st,
                        float *parts = nullptr) {
    if (M <= 0 || N <= 0) return CAPS_OK;
    const auto aligned = [](const uint16_t *P) { return ((uintptr_t)P & 15) == 0; };
    // K-contiguous rows whose 8-element groups are 16-byte aligned
    const auto vec_ok = [&](const uint16_t *P, int64_t srow, int64_t sk) {
        return sk == 1 && K % 8 == 0 && srow % 8 == 0 && aligned(P);
    };
    // row-contiguous columns (unit row stride) with aligned 8-row groups
    const auto row_ok = [&](const uint16_t *P, int64_t srow, int64_t sk) {
        return srow == 1 && sk != 1 && sk % 8 == 0 && aligned(P);
    };
    const int64_t tiles = (int64_t)((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
    if (tiles > INT32_MAX) {
        set_error("router GEMM: too many tiles");
        return CAPS_EINVAL;
    }
    if (vec_ok(A, sam, sak) && vec_ok(B, sbn, sbk) && (int64_t)M * sam < INT32_MAX && (int64_t)N * sbn < INT32_MAX) {
        hipLaunchKernelGGL(k_gemm_nt, dim3((unsigned)tiles), dim3(256), 0, st, A, (int32_t)sam, B, (int32_t)sbn, M,
                           N, K, bias, flags, mask, ldm, C32, C16, ldc);
        CAPS_HIP(hipGetLastError());
        return CAPS_OK;
    }
    if (vec_ok(A, sam, sak)) flags |= kGemmVecA;
    else if (row_ok(A, sam, sak)) flags |= kGemmRowA;
    if (vec_ok(B, sbn, sbk)) flags |= kGemmVecB;
    else if (row_ok(B, sbn, sbk)) flags |= kGemmRowB;
    // split K when the tiles alone cannot fill the chip (plain FP32 output only)
    int32_t splits = 1, kchunk = K;
    if (parts && C32 && !C16 && !bias && flags == (flags & ~(kGemmRelu | kGemmMask | kGemmNeg)) && ldc == N) {
        const int64_t want = (512 + tiles - 1) / tiles;
        const int64_t most = std::max<int64_t>(1, std::min<int64_t>(K / (4 * kGK), kGemmParts / ((int64_t)M * N)));
        splits = (int32_t)std::min<int64_t>(want, most);
        kchunk = (int32_t)(((K + splits - 1) / splits + kGK - 1) / kGK * kGK);
        splits = (K + kchunk - 1) / kchunk;
    }
    if (splits > 1) {
        hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)tiles, (unsigned)splits), dim3(256), 0, st, A, sam, sak, B,
                           sbn, sbk, M, N, K, kchunk, nullptr, flags, nullptr, 0, parts, nullptr, ldc);
        const int64_t n = (int64_t)M * N;
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, parts, splits, n, C32);
    } else {
        hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)tiles), dim3(256), 0, st, A, sam, sak, B, sbn, sbk, M, N, K,
                           K, bias, flags, mask, ldm, C32, C16, ldc);
    }
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

// ------------------------------------------------------------------ library GEMM (inference)
// D (M x N, row-major, leading dimension ldc) = epi(alpha * A B^T + bias) with
// A (M x K) and B (N x K) row-major BF16 (K-contiguous), FP32 accumulation,
// bias FP32 per column n of D, epi = ReLU or identity, D FP32 or BF16.  In
// hipBLASLt's column-major terms: D^T (N x M) = op_T(B) op_N(A), the bias per
// row of D^T.  One plan (descriptors and the heuristic's first algorithm, no
// workspace) per device and shape, kept for the process; the descriptor's bias
// pointer is set under the lock just before the (asynchronous) enqueue.
namespace {
constexpr int kLtDevices = 64;
struct LtPlan {
    int dev;
    int32_t M, N, K, lda, ldb;
    int64_t ldc;
    bool relu, out16;
    hipblasLtMatmulDesc_t desc = nullptr;
    hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, ld = nullptr;
    hipblasLtMatmulAlgo_t algo;
    bool ok = false;
};
std::mutex g_lt_mu;
hipblasLtHandle_t g_lt[kLtDevices] = {};
bool g_lt_failed[kLtDevices] = {};
std::vector<LtPlan *> g_lt_plans;

LtPlan *lt_plan(int dev, int32_t M, int32_t N, int32_t K, int32_t lda, int32_t ldb, int64_t ldc, bool relu,
                bool out16) {
    for (LtPlan *p : g_lt_plans)
        if (p->dev == dev && p->M == M && p->N == N && p->K == K && p->lda == lda && p->ldb == ldb &&
            p->ldc == ldc && p->relu == relu && p->out16 == out16)
            return p;
    LtPlan *p = new LtPlan{dev, M, N, K, lda, ldb, ldc, relu, out16};
    g_lt_plans.push_back(p);
    if (!g_lt[dev] && !g_lt_failed[dev] && hipblasLtCreate(&g_lt[dev]) != HIPBLAS_STATUS_SUCCESS) {
        g_lt[dev] = nullptr;
        g_lt_failed[dev] = true;
    }
    if (!g_lt[dev]) return p;
    const hipblasOperation_t opT = HIPBLAS_OP_T, opN = HIPBLAS_OP_N;
    const hipblasLtEpilogue_t epi = relu ? HIPBLASLT_EPILOGUE_RELU_BIAS : HIPBLASLT_EPILOGUE_BIAS;
    const int32_t bias_type = HIP_R_32F;
    const uint64_t no_ws = 0;
    hipblasLtMatmulPreference_t pref = nullptr;
    hipblasLtMatmulHeuristicResult_t res[1];
    int nres = 0;
    bool ok = hipblasLtMatmulDescCreate(&p->desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_TRANSA, &opT, sizeof(opT)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_TRANSB, &opN, sizeof(opN)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_EPILOGUE, &epi, sizeof(epi)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_BIAS_DATA_TYPE, &bias_type,
                                              sizeof(bias_type)) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&p->la, HIP_R_16BF, (uint64_t)K, (uint64_t)N, ldb) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&p->lb, HIP_R_16BF, (uint64_t)K, (uint64_t)M, lda) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&p->ld, out16 ? HIP_R_16BF : HIP_R_32F, (uint64_t)N, (uint64_t)M, ldc) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &no_ws,
                                                    sizeof(no_ws)) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulAlgoGetHeuristic(g_lt[dev], p->desc, p->la, p->lb, p->ld, p->ld, pref, 1, res, &nres) ==
                  HIPBLAS_STATUS_SUCCESS &&
              nres > 0 && res[0].state == HIPBLAS_STATUS_SUCCESS && res[0].workspaceSize == 0;
    if (pref) (void)hipblasLtMatmulPreferenceDestroy(pref);
    if (ok) p->algo = res[0].algo;
    p->ok = ok;
    return p;
}
}   // namespace

// Enqueues the product on `st` and returns true, or returns false (nothing
// enqueued) when the library has no algorithm for the shape.
static bool lt_gemm(const uint16_t *A, int32_t lda, const uint16_t *B, int32_t ldb, int32_t M, int32_t N, int32_t K,
                    const float *bias, bool relu, float alpha, float *C32, uint16_t *C16, int64_t ldc,
                    hipStream_t st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kLtDevices || !bias || (C32 == nullptr) == (C16 == nullptr))
        return false;
    std::lock_guard<std::mutex> lk(g_lt_mu);
    LtPlan *p = lt_plan(dev, M, N, K, lda, ldb, ldc, relu, C16 != nullptr);
    if (!p->ok) return false;
    if (hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_BIAS_POINTER, &bias, sizeof(bias)) !=
        HIPBLAS_STATUS_SUCCESS)
        return false;
    const float beta = 0.0f;
    void *D = C16 ? (void *)C16 : (void *)C32;
    return hipblasLtMatmul(g_lt[dev], p->desc, &alpha, B, p->la, A, p->lb, &beta, D, p->ld, D, p->ld, &p->algo,
                           nullptr, 0, st) == HIPBLAS_STATUS_SUCCESS;
}

// y = -x with -0 written as +0 (so that -(acc) + y never yields -0)
__global__ void k_negate(const float *__restrict__ x, int32_t n, float *__restrict__ y) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = canon0(-x[i]);
}

// ------------------------------------------------------------------ loss (K12)
// One workgroup per row: softmax of the logits, loss -(1/|S|) sum_{s in S}
// log p_s over the row's distinct labels S (entries < 0 are padding), and
// the logit gradient (p - y) / M with y uniform on S (both 0 when S is
// empty), as FP32 and BF16.
__global__ __launch_bounds__(256) void k_softmax_ce(const float *__restrict__ Z, int32_t M, int32_t nout,
                                                    const int32_t *__restrict__ labels, int32_t L,
                                                    float *__restrict__ loss_rows, float *__restrict__ dZ32,
                                                    uint16_t *__restrict__ dZ16) {
    __shared__ float red[256];
    __shared__ int32_t lab[64];
    __shared__ int32_t nlab;
    const int64_t i = blockIdx.x;
    const float *z = Z + i * nout;
    const int t = threadIdx.x;
    if (t == 0) {
        int n = 0;
        for (int e = 0; e < L && n < 64; e++) {
            const int32_t v = labels[i * L + e];
            if (v < 0 || v >= nout) continue;
            bool dup = false;
            for (int f = 0; f < n; f++) dup |= lab[f] == v;
            if (!dup) lab[n++] = v;
        }
        nlab = n;
    }
    float mx = -__builtin_huge_valf();
    for (int j = t; j < nout; j += 256) mx = fmaxf(mx, z[j]);
    red[t] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] = fmaxf(red[t], red[t + o]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    float s = 0.0f;
    for (int j = t; j < nout; j += 256) s += expf(z[j] - mx);
    red[t] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    const float sum = red[0];
    const int n = nlab;
    const float inv = n ? 1.0f / (float)n : 0.0f;
    for (int j = t; j < nout; j += 256) {
        float y = 0.0f;
        for (int f = 0; f < n; f++) y += lab[f] == j ? inv : 0.0f;
        const float g = n ? (expf(z[j] - mx) / sum - y) / (float)M : 0.0f;
        dZ32[i * nout + j] = g;
        dZ16[i * nout + j] = bf16_rne(g);
    }
    if (t == 0) {
        float l = 0.0f;
        if (n) {
            const float lse = logf(sum) + mx;
            for (int f = 0; f < n; f++) l += lse - z[lab[f]];
            l *= inv;
        }
        loss_rows[i] = l;
    }
}

// Column sums of an M x N FP32 matrix, rows in ascending order.
// Column sums of an M x N FP32 matrix in two deterministic stages: workgroup
// (x, y) sums rows [rp*y, rp*y + rp) of columns [64x, 64x + 64) (four row
// lanes, each over every fourth row, then the lanes in order) into
// part[y*N + j]; then k_sum_parts adds the parts in order.  rp is 64, or
// more when the parts would not fit kGemmParts floats.
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ X, int32_t M, int32_t N, int32_t rp,
                                                     float *__restrict__ part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, l = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + c, r0 = (int64_t)blockIdx.y * rp;
    float s = 0.0f;
    if (j < N)
        for (int64_t i = r0 + l; i < r0 + rp && i < M; i += 4) s += X[i * N + j];
    red[l][c] = s;
    __syncthreads();
    if (l == 0 && j < N) part[(int64_t)blockIdx.y * N + j] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

static void colsum(const float *X, int32_t M, int32_t N, float *part, float *out, hipStream_t st) {
    int64_t rp = 64;
    while ((M + rp - 1) / rp * (int64_t)N > kGemmParts) rp *= 2;
    const int32_t ry = (int32_t)((M + rp - 1) / rp);
    hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((N + 63) / 64), (unsigned)ry), dim3(256), 0, st, X, M, N,
                       (int32_t)rp, part);
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, part, ry, (int64_t)N, out);
}

// Adds the mean of M values to *acc (single workgroup).
__global__ __launch_bounds__(256) void k_accum_mean(const float *__restrict__ v, int32_t M, float *__restrict__ acc) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < M; i += 256) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *acc += red[0];
}

// ------------------------------------------------------------------ Adam (K13)
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = bf16_rne(x[i]);
}

// Rows perm[0..nb) of X (dpad BF16) and of the labels (L int32).
__global__ void k_gather_batch(const uint16_t *__restrict__ X, const int32_t *__restrict__ labels,
                               const int32_t *__restrict__ perm, int32_t nb, int32_t dpad, int32_t L,
                               uint16_t *__restrict__ Xb, int32_t *__restrict__ Lb) {
    const int64_t i = blockIdx.x;
    if (i >= nb) return;
    const int64_t src = perm[i];
    for (int j = threadIdx.x; j < dpad; j += blockDim.x) Xb[i * dpad + j] = X[src * dpad + j];
    for (int j = threadIdx.x; j < L; j += blockDim.x) Lb[i * L + j] = labels[src * L + j];
}

// ------------------------------------------------------------------ labels
// Distinct partitions of each query's ids (in order of first appearance),
// -1 padded; ids < 0 are skipped.
__global__ void k_router_labels(const int32_t *__restrict__ ids, int32_t n, int32_t k,
                                const int32_t *__restrict__ assign, int64_t npts, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int j = 0; j < k; j++) {
        const int32_t id = ids[i * k + j];
        if (id < 0 || id >= npts) continue;
        const int32_t p = assign[id];
        bool dup = false;
        for (int f = 0; f < c; f++) dup |= out[i * k + f] == p;
        if (!dup) out[i * k + c++] = p;
    }
    for (int j = c; j < k; j++) out[i * k + j] = -1;
}

// ------------------------------------------------------------------ inference
// Softmax top-1 probability per row of negated logits (smaller is better).
__global__ __launch_bounds__(64) void k_router_conf(const float *__restrict__ S, int32_t nb, int32_t nout,
                                                    float *__restrict__ conf) {
    const int64_t i = blockIdx.x;
    if (i >= nb) return;
    const float *s = S + i * nout;
    float mn = __builtin_huge_valf();
    for (int j = threadIdx.x; j < nout; j += 64) mn = fminf(mn, s[j]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mn = fminf(mn, __shfl_xor(mn, o, 64));
    float sum = 0.0f;
    for (int j = threadIdx.x; j < nout; j += 64) sum += expf(mn - s[j]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (threadIdx.x == 0) conf[i] = 1.0f / sum;
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

__global__ void k_router_fb_list(int32_t nb, int32_t m, int32_t k, float fb_prob, const float *__restrict__ conf,
                                 const int32_t *__restrict__ cand, int32_t *__restrict__ fbq,
                                 int32_t *__restrict__ nfb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    int64_t c = 0;
    for (int j = 0; j < m; j++) c += cand[i * m + j];
    if (conf[i] < fb_prob || c < k) fbq[atomicAdd(nfb, 1)] = (int32_t)i;
}

__global__ void k_router_fb_apply(int32_t nb, int32_t m, const int32_t *__restrict__ fbq,
                                  const int32_t *__restrict__ nfb, const int32_t *__restrict__ probes_c,
                                  int32_t *__restrict__ probes) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = e / m;
    if (r >= nb || r >= *nfb) return;
    probes[(int64_t)fbq[r] * m + e % m] = probes_c[e];
}

static int64_t nblk(int64_t n, int t) { return (n + t - 1) / t; }

caps_status router_scores(const Index *ix, const float *q, int32_t nb, const int32_t *con_off,
                          const int32_t *con_attr, const int32_t *con_val, int32_t n_con, uint16_t *X,
                          uint16_t *H, float *bneg, float *scores, float *conf, hipStream_t st) {
    const Router &R = *ix->router;
    hipLaunchKernelGGL(k_router_input, dim3((unsigned)nb), dim3(64), 0, st, q, nb, ix->d, con_off, con_attr,
                       con_val, n_con, ix->sch, R.in_scale, R.in_shift, R.dpad, X);
    hipLaunchKernelGGL(k_negate, dim3((unsigned)nblk(R.nout, 256)), dim3(256), 0, st, R.param + R.o_b2, R.nout,
                       bneg);
    CAPS_HIP(hipGetLastError());
    caps_status s = CAPS_OK;
    if (!lt_gemm(X, R.dpad, R.w1h, R.dpad, nb, R.hid, R.dpad, R.param + R.o_b1, true, 1.0f, nullptr, H, R.hid, st))
        s = gemm(X, R.dpad, 1, R.w1h, R.dpad, 1, nb, R.hid, R.dpad, R.param + R.o_b1, kGemmRelu, nullptr, 0, nullptr,
                 H, R.hid, st);
    if (s != CAPS_OK) return s;
    // scores = -(H W2^T + b2) = (-1) H W2^T + (-b2): negation is exact
    if (!lt_gemm(H, R.hid, R.w2h, R.hid, nb, R.nout, R.hid, bneg, false, -1.0f, scores, nullptr, R.nout, st))
        s = gemm(H, R.hid, 1, R.w2h, R.hid, 1, nb, R.nout, R.hid, R.param + R.o_b2, kGemmNeg, nullptr, 0, scores,
                 nullptr, R.nout, st);
    if (s != CAPS_OK) return s;
    hipLaunchKernelGGL(k_router_conf, dim3((unsigned)nb), dim3(64), 0, st, scores, nb, R.nout, conf);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

caps_status router_fallback_list(const Index *ix, int32_t nb, int32_t m, int32_t k, const float *conf,
                                 const int32_t *cand, int32_t *fbq, int32_t *nfb, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, nfb);
    hipLaunchKernelGGL(k_router_fb_list, dim3((unsigned)nblk(nb, 256)), dim3(256), 0, st, nb, m, k,
                       ix->router->fb_prob, conf, cand, fbq, nfb);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

caps_status router_fallback_apply(int32_t nb, int32_t m, const int32_t *fbq, const int32_t *nfb,
                                  const int32_t *probes_c, int32_t *probes, hipStream_t st) {
    hipLaunchKernelGGL(k_router_fb_apply, dim3((unsigned)nblk((int64_t)nb * m, 256)), dim3(256), 0, st, nb, m, fbq,
                       nfb, probes_c, probes);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

void router_free(Router *r) {
    if (!r) return;
    void *ptrs[] = {r->param, r->mom, r->vel, r->w1h, r->w2h};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete r;
}

// ------------------------------------------------------------------ host helpers
static uint64_t sm64_next(uint64_t &s) {
    s += 0x9E3779B97F4A7C15ull;
    return mix64(s);
}

// Allocates a router for the index with zeroed moments; w1/b1/w2/b2 from
// host arrays, or (when null) W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) drawn
// from splitmix64(seed) and zero biases.
static caps_status router_alloc(Index *ix, int32_t hid, float in_scale, float in_shift, float fb_prob, uint64_t seed,
                                const float *w1, const float *b1, const float *w2, const float *b2) {
    Router *R = new Router;
    R->din = ix->d + kEmbed;
    R->dpad = (R->din + 31) / 32 * 32;
    R->hid = hid;
    R->nout = ix->b;
    R->in_scale = in_scale;
    R->in_shift = in_shift;
    R->fb_prob = fb_prob;
    R->o_b1 = (int64_t)hid * R->dpad;
    R->o_w2 = R->o_b1 + hid;
    R->o_b2 = R->o_w2 + (int64_t)R->nout * hid;
    R->nparam = R->o_b2 + R->nout;
    std::vector<float> h((size_t)R->nparam, 0.0f);
    if (w1) {
        memcpy(h.data(), w1, sizeof(float) * (size_t)R->o_b1);
        memcpy(h.data() + R->o_b1, b1, sizeof(float) * (size_t)hid);
        memcpy(h.data() + R->o_w2, w2, sizeof(float) * (size_t)R->nout * hid);
        memcpy(h.data() + R->o_b2, b2, sizeof(float) * (size_t)R->nout);
    } else {
        uint64_t s = seed;
        const double a1 = 1.0 / sqrt((double)R->din), a2 = 1.0 / sqrt((double)hid);
        for (int64_t r = 0; r < hid; r++)
            for (int64_t c = 0; c < R->dpad; c++) {
                const double u = (double)(sm64_next(s) >> 11) * 0x1p-53;
                h[(size_t)(r * R->dpad + c)] = c < R->din ? (float)((2.0 * u - 1.0) * a1) : 0.0f;
            }
        for (int64_t e = 0; e < (int64_t)R->nout * hid; e++) {
            const double u = (double)(sm64_next(s) >> 11) * 0x1p-53;
            h[(size_t)(R->o_w2 + e)] = (float)((2.0 * u - 1.0) * a2);
        }
    }
    const size_t pb = sizeof(float) * (size_t)R->nparam;
    auto fail_free = [&](hipError_t e) {
        router_free(R);
        set_error("router allocation failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? CAPS_ENOMEM : CAPS_EDEVICE;
    };
    hipError_t e;
    if ((e = hipMalloc((void **)&R->param, pb)) != hipSuccess) return fail_free(e);
    if ((e = hipMalloc((void **)&R->mom, pb)) != hipSuccess) return fail_free(e);
    if ((e = hipMalloc((void **)&R->vel, pb)) != hipSuccess) return fail_free(e);
    if ((e = hipMalloc((void **)&R->w1h, sizeof(uint16_t) * (size_t)R->o_b1)) != hipSuccess) return fail_free(e);
    if ((e = hipMalloc((void **)&R->w2h, sizeof(uint16_t) * (size_t)R->nout * hid)) != hipSuccess)
        return fail_free(e);
    if ((e = hipMemcpy(R->param, h.data(), pb, hipMemcpyHostToDevice)) != hipSuccess) return fail_free(e);
    if ((e = hipMemset(R->mom, 0, pb)) != hipSuccess) return fail_free(e);
    if ((e = hipMemset(R->vel, 0, pb)) != hipSuccess) return fail_free(e);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk(R->o_b1, 256)), dim3(256), 0, 0, R->param, R->o_b1, R->w1h);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk((int64_t)R->nout * hid, 256)), dim3(256), 0, 0,
                       R->param + R->o_w2, (int64_t)R->nout * hid, R->w2h);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_free(e);
    router_free(ix->router);
    ix->router = R;
    return CAPS_OK;
}

// Workspace of one training / gradient batch of up to bs rows.
struct BatchWs {
    uint16_t *Xb, *Hb, *dZ16, *dH16;
    int32_t *Lb;
    float *Z, *dZ32, *dH32, *grad, *loss_rows, *parts;
};

static size_t batch_ws(const Router &R, int32_t bs, int32_t L, uint8_t *base, BatchWs *w) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~(size_t)255;
        uint8_t *p = base ? base + o : nullptr;
        o += bytes;
        return p;
    };
    BatchWs t;
    t.Xb = (uint16_t *)take(sizeof(uint16_t) * (size_t)bs * R.dpad);
    t.Hb = (uint16_t *)take(sizeof(uint16_t) * (size_t)bs * R.hid);
    t.dZ16 = (uint16_t *)take(sizeof(uint16_t) * (size_t)bs * R.nout);
    t.dH16 = (uint16_t *)take(sizeof(uint16_t) * (size_t)bs * R.hid);
    t.Lb = (int32_t *)take(sizeof(int32_t) * (size_t)bs * std::max(L, 1));
    t.Z = (float *)take(sizeof(float) * (size_t)bs * R.nout);
    t.dZ32 = (float *)take(sizeof(float) * (size_t)bs * R.nout);
    t.dH32 = (float *)take(sizeof(float) * (size_t)bs * R.hid);
    t.grad = (float *)take(sizeof(float) * (size_t)R.nparam);
    t.loss_rows = (float *)take(sizeof(float) * (size_t)bs);
    t.parts = (float *)take(sizeof(float) * (size_t)kGemmParts);
    if (w) *w = t;
    return o + 256;
}

// Forward, loss and gradients of one batch already gathered into w.Xb / w.Lb.
static caps_status batch_grads(const Router &R, const BatchWs &w, int32_t nb, int32_t L, hipStream_t st) {
    caps_status s;
    // h = relu(W1 x + b1), z = W2 h + b2
    s = gemm(w.Xb, R.dpad, 1, R.w1h, R.dpad, 1, nb, R.hid, R.dpad, R.param + R.o_b1, kGemmRelu, nullptr, 0,
             nullptr, w.Hb, R.hid, st);
    if (s != CAPS_OK) return s;
    s = gemm(w.Hb, R.hid, 1, R.w2h, R.hid, 1, nb, R.nout, R.hid, R.param + R.o_b2, 0, nullptr, 0, w.Z, nullptr,
             R.nout, st);
    if (s != CAPS_OK) return s;
    hipLaunchKernelGGL(k_softmax_ce, dim3((unsigned)nb), dim3(256), 0, st, w.Z, nb, R.nout, w.Lb, L, w.loss_rows,
                       w.dZ32, w.dZ16);
    CAPS_HIP(hipGetLastError());
    float *gw1 = w.grad, *gb1 = w.grad + R.o_b1, *gw2 = w.grad + R.o_w2, *gb2 = w.grad + R.o_b2;
    // dW2 = dZ^T h;  db2 = column sums of dZ
    s = gemm(w.dZ16, 1, R.nout, w.Hb, 1, R.hid, R.nout, R.hid, nb, nullptr, 0, nullptr, 0, gw2, nullptr, R.hid, st,
             w.parts);
    if (s != CAPS_OK) return s;
    colsum(w.dZ32, nb, R.nout, w.parts, gb2, st);
    // dH = (dZ W2) masked by h > 0;  db1 = column sums of dH
    s = gemm(w.dZ16, R.nout, 1, R.w2h, 1, R.hid, nb, R.hid, R.nout, nullptr, kGemmMask, w.Hb, R.hid, w.dH32, w.dH16,
             R.hid, st);
    if (s != CAPS_OK) return s;
    colsum(w.dH32, nb, R.hid, w.parts, gb1, st);
    // dW1 = dH^T x
    s = gemm(w.dH16, 1, R.hid, w.Xb, 1, R.dpad, R.hid, R.dpad, nb, nullptr, 0, nullptr, 0, gw1, nullptr, R.dpad, st,
             w.parts);
    if (s != CAPS_OK) return s;
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

static caps_status check_queries(const Index &ix, const float *q, int32_t n, const int32_t *con_off,
                                 const int32_t *con_attr, const int32_t *con_val, int32_t n_con) {
    if (n < 0 || n_con < 0) {
        set_error("router: negative count");
        return CAPS_EINVAL;
    }
    if (n > 0 && (!q || !con_off)) {
        set_error("router: null query arrays");
        return CAPS_EINVAL;
    }
    if (n_con > 0 && (!con_attr || !con_val)) {
        set_error("router: null constraint arrays");
        return CAPS_EINVAL;
    }
    (void)ix;
    return CAPS_OK;
}

static caps_status check_params(const caps_router_params *p) {
    if (!p) {
        set_error("router: null params");
        return CAPS_EINVAL;
    }
    if (p->hidden < 16 || p->hidden > 8192 || p->hidden % 16) {
        set_error("router: hidden must be a multiple of 16 in [16, 8192]");
        return CAPS_EINVAL;
    }
    if (!(p->in_scale == p->in_scale) || !(p->in_shift == p->in_shift) || !(p->fallback_prob == p->fallback_prob)) {
        set_error("router: NaN parameter");
        return CAPS_EINVAL;
    }
    return CAPS_OK;
}

}  // namespace caps

using namespace caps;

extern "C" caps_status caps_router_labels(const caps_index *idx, const int32_t *ids, int32_t n, int32_t k,
                                          int32_t *out_parts, void *stream) {
    if (!idx || n < 0 || k < 1 || (n > 0 && (!ids || !out_parts))) {
        set_error("caps_router_labels: bad arguments");
        return CAPS_EINVAL;
    }
    if (n == 0) return CAPS_OK;
    hipLaunchKernelGGL(k_router_labels, dim3((unsigned)nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, ids, n, k,
                       idx->ix.assign, idx->ix.n, out_parts);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

extern "C" caps_status caps_router_set(caps_index *idx, const caps_router_params *p, const float *w1,
                                       const float *b1, const float *w2, const float *b2) {
    if (!idx) {
        set_error("caps_router_set: null index");
        return CAPS_EINVAL;
    }
    caps_status s = check_params(p);
    if (s != CAPS_OK) return s;
    if (!w1 != !b1 || !w1 != !w2 || !w1 != !b2) {
        set_error("caps_router_set: give all four weight arrays or none");
        return CAPS_EINVAL;
    }
    return router_alloc(&idx->ix, p->hidden, p->in_scale, p->in_shift, p->fallback_prob, p->seed, w1, b1, w2, b2);
}

extern "C" caps_status caps_router_info(const caps_index *idx, caps_router_info_t *out) {
    if (!idx || !out) {
        set_error("caps_router_info: null argument");
        return CAPS_EINVAL;
    }
    memset(out, 0, sizeof(*out));
    const Router *R = idx->ix.router;
    if (!R) return CAPS_OK;
    out->present = 1;
    out->din = R->din;
    out->dpad = R->dpad;
    out->hidden = R->hid;
    out->n_out = R->nout;
    out->in_scale = R->in_scale;
    out->in_shift = R->in_shift;
    out->fallback_prob = R->fb_prob;
    out->steps = R->step;
    return CAPS_OK;
}

extern "C" caps_status caps_router_get(const caps_index *idx, float *w1, float *b1, float *w2, float *b2) {
    if (!idx || !idx->ix.router) {
        set_error("caps_router_get: index has no router");
        return CAPS_EINVAL;
    }
    const Router &R = *idx->ix.router;
    CAPS_HIP(hipDeviceSynchronize());
    if (w1) CAPS_HIP(hipMemcpy(w1, R.param, sizeof(float) * (size_t)R.o_b1, hipMemcpyDeviceToHost));
    if (b1) CAPS_HIP(hipMemcpy(b1, R.param + R.o_b1, sizeof(float) * (size_t)R.hid, hipMemcpyDeviceToHost));
    if (w2) CAPS_HIP(hipMemcpy(w2, R.param + R.o_w2, sizeof(float) * (size_t)R.nout * R.hid, hipMemcpyDeviceToHost));
    if (b2) CAPS_HIP(hipMemcpy(b2, R.param + R.o_b2, sizeof(float) * (size_t)R.nout, hipMemcpyDeviceToHost));
    return CAPS_OK;
}

extern "C" caps_status caps_router_logits(const caps_index *idx, const float *q, int32_t n, const int32_t *con_off,
                                          const int32_t *con_attr, const int32_t *con_val, int32_t n_con,
                                          float *out_logits, void *stream) {
    if (!idx || !idx->ix.router) {
        set_error("caps_router_logits: index has no router");
        return CAPS_EINVAL;
    }
    caps_status s = check_queries(idx->ix, q, n, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n == 0) return CAPS_OK;
    if (!out_logits) {
        set_error("caps_router_logits: null output");
        return CAPS_EINVAL;
    }
    const Index &ix = idx->ix;
    const Router &R = *ix.router;
    hipStream_t st = (hipStream_t)stream;
    uint16_t *ws = nullptr;
    const size_t xb = sizeof(uint16_t) * (size_t)n * R.dpad, hb = sizeof(uint16_t) * (size_t)n * R.hid;
    s = ws_alloc((void **)&ws, xb + hb + 256, ix.device, st);   // (the library's pool: the free keeps it)
    if (s != CAPS_OK) return s;
    uint16_t *X = ws, *H = reinterpret_cast<uint16_t *>(reinterpret_cast<uint8_t *>(ws) + ((xb + 255) & ~(size_t)255));
    hipLaunchKernelGGL(k_router_input, dim3((unsigned)n), dim3(64), 0, st, q, n, ix.d, con_off, con_attr, con_val,
                       n_con, ix.sch, R.in_scale, R.in_shift, R.dpad, X);
    if (!lt_gemm(X, R.dpad, R.w1h, R.dpad, n, R.hid, R.dpad, R.param + R.o_b1, true, 1.0f, nullptr, H, R.hid, st))
        s = gemm(X, R.dpad, 1, R.w1h, R.dpad, 1, n, R.hid, R.dpad, R.param + R.o_b1, kGemmRelu, nullptr, 0, nullptr,
                 H, R.hid, st);
    if (s == CAPS_OK &&
        !lt_gemm(H, R.hid, R.w2h, R.hid, n, R.nout, R.hid, R.param + R.o_b2, false, 1.0f, out_logits, nullptr, R.nout,
                 st))
        s = gemm(H, R.hid, 1, R.w2h, R.hid, 1, n, R.nout, R.hid, R.param + R.o_b2, 0, nullptr, 0, out_logits,
                 nullptr, R.nout, st);
    (void)hipFreeAsync(ws, st);
    return s;
}

// Loss and gradients of one batch (all n rows) without updating the router;
// gradients go to host arrays laid out like the weights.
extern "C" caps_status caps_router_grads(caps_index *idx, const float *q, int32_t n, const int32_t *con_off,
                                         const int32_t *con_attr, const int32_t *con_val, int32_t n_con,
                                         const int32_t *labels, int32_t n_labels, float *out_loss, float *g_w1,
                                         float *g_b1, float *g_w2, float *g_b2, void *stream) {
    if (!idx || !idx->ix.router) {
        set_error("caps_router_grads: index has no router");
        return CAPS_EINVAL;
    }
    caps_status s = check_queries(idx->ix, q, n, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n < 1 || n_labels < 1 || !labels) {
        set_error("caps_router_grads: need n >= 1 rows and labels");
        return CAPS_EINVAL;
    }
    const Index &ix = idx->ix;
    const Router &R = *ix.router;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = batch_ws(R, n, n_labels, nullptr, nullptr);
    uint8_t *base = nullptr;
    CAPS_HIP(hipMallocAsync((void **)&base, bytes, st));
    BatchWs w;
    batch_ws(R, n, n_labels, base, &w);
    hipLaunchKernelGGL(k_router_input, dim3((unsigned)n), dim3(64), 0, st, q, n, ix.d, con_off, con_attr, con_val,
                       n_con, ix.sch, R.in_scale, R.in_shift, R.dpad, w.Xb);
    (void)hipMemcpyAsync(w.Lb, labels, sizeof(int32_t) * (size_t)n * n_labels, hipMemcpyDeviceToDevice, st);
    s = batch_grads(R, w, n, n_labels, st);
    float *acc = w.Z;   // the logits are consumed by now: first slot holds the loss sum
    if (s == CAPS_OK) {
        (void)hipMemsetAsync(acc, 0, sizeof(float), st);
        hipLaunchKernelGGL(k_accum_mean, dim3(1), dim3(256), 0, st, w.loss_rows, n, acc);
    }
    std::vector<float> host(s == CAPS_OK ? (size_t)R.nparam : 0);
    float lsum = 0.0f;
    if (s == CAPS_OK) {
        hipError_t e = hipMemcpyAsync(host.data(), w.grad, sizeof(float) * (size_t)R.nparam, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&lsum, acc, sizeof(float), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_error("caps_router_grads: %s", hipGetErrorString(e));
            s = CAPS_EDEVICE;
        }
    }
    (void)hipFreeAsync(base, st);
    if (s != CAPS_OK) return s;
    if (out_loss) *out_loss = lsum / (float)n;
    if (g_w1) memcpy(g_w1, host.data(), sizeof(float) * (size_t)R.o_b1);
    if (g_b1) memcpy(g_b1, host.data() + R.o_b1, sizeof(float) * (size_t)R.hid);
    if (g_w2) memcpy(g_w2, host.data() + R.o_w2, sizeof(float) * (size_t)R.nout * R.hid);
    if (g_b2) memcpy(g_b2, host.data() + R.o_b2, sizeof(float) * (size_t)R.nout);
    return CAPS_OK;
}

extern "C" caps_status caps_router_train(caps_index *idx, const caps_router_params *p, const float *q, int32_t n,
                                         const int32_t *con_off, const int32_t *con_attr, const int32_t *con_val,
                                         int32_t n_con, const int32_t *labels, int32_t n_labels, float *out_loss,
                                         void *stream) {
    if (!idx) {
        set_error("caps_router_train: null index");
        return CAPS_EINVAL;
    }
    caps_status s = check_params(p);
    if (s != CAPS_OK) return s;
    s = check_queries(idx->ix, q, n, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n < 1 || n_labels < 1 || !labels || p->epochs < 0 || p->batch < 1 || p->batch > (1 << 16) ||
        !(p->lr > 0.0f) || !(p->beta1 >= 0.0f && p->beta1 < 1.0f) || !(p->beta2 >= 0.0f && p->beta2 < 1.0f) ||
        !(p->eps > 0.0f)) {
        set_error("caps_router_train: bad rows, labels, epochs, batch or optimiser parameters");
        return CAPS_EINVAL;
    }
    Index &ix = idx->ix;
    if (p->reset || !ix.router || ix.router->hid != p->hidden) {
        s = router_alloc(&ix, p->hidden, p->in_scale, p->in_shift, p->fallback_prob, p->seed, nullptr, nullptr,
                         nullptr, nullptr);
        if (s != CAPS_OK) return s;
    } else {
        ix.router->in_scale = p->in_scale;
        ix.router->in_shift = p->in_shift;
        ix.router->fb_prob = p->fallback_prob;
    }
    Router &R = *ix.router;
    hipStream_t st = (hipStream_t)stream;
    const int32_t bs = std::min(p->batch, n);
    // workspace: every input row once, the shuffle, one batch (256-byte aligned pieces)
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t off_perm = al(sizeof(uint16_t) * (size_t)n * R.dpad);
    const size_t off_batch = al(off_perm + sizeof(int32_t) * (size_t)n);
    const size_t total = off_batch + batch_ws(R, bs, n_labels, nullptr, nullptr);
    uint8_t *base = nullptr;
    CAPS_HIP(hipMallocAsync((void **)&base, total, st));
    uint16_t *X = reinterpret_cast<uint16_t *>(base);
    int32_t *perm = reinterpret_cast<int32_t *>(base + off_perm);
    BatchWs w;
    batch_ws(R, bs, n_labels, base + off_batch, &w);
    hipLaunchKernelGGL(k_router_input, dim3((unsigned)n), dim3(64), 0, st, q, n, ix.d, con_off, con_attr, con_val,
                       n_con, ix.sch, R.in_scale, R.in_shift, R.dpad, X);
    CAPS_HIP(hipGetLastError());
    std::vector<int32_t> order((size_t)n);
    uint64_t rng = p->seed ^ 0xD1B54A32D192ED03ull;
    float *loss_dev = nullptr;
    CAPS_HIP(hipMallocAsync((void **)&loss_dev, sizeof(float), st));
    for (int32_t ep = 0; ep < p->epochs && s == CAPS_OK; ep++) {
        // Fisher-Yates shuffle of the rows from splitmix64
        for (int32_t i = 0; i < n; i++) order[(size_t)i] = i;
        for (int32_t i = n - 1; i > 0; i--) {
            const int32_t j = (int32_t)(sm64_next(rng) % (uint64_t)(i + 1));
            std::swap(order[(size_t)i], order[(size_t)j]);
        }
        hipError_t e = hipMemcpyAsync(perm, order.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // `order` is reused next epoch
        if (e == hipSuccess) e = hipMemsetAsync(loss_dev, 0, sizeof(float), st);
        if (e != hipSuccess) {
            set_error("caps_router_train: %s", hipGetErrorString(e));
            s = CAPS_EDEVICE;
            break;
        }
        for (int32_t b0 = 0; b0 < n && s == CAPS_OK; b0 += bs) {
            const int32_t nb = std::min(bs, n - b0);
            hipLaunchKernelGGL(k_gather_batch, dim3((unsigned)nb), dim3(64), 0, st, X, labels, perm + b0, nb, R.dpad,
                               n_labels, w.Xb, w.Lb);
            s = batch_grads(R, w, nb, n_labels, st);
            if (s != CAPS_OK) break;
            hipLaunchKernelGGL(k_accum_mean, dim3(1), dim3(256), 0, st, w.loss_rows, nb, loss_dev);
            R.step++;
            const double bc1 = 1.0 - pow((double)p->beta1, (double)R.step);
            const double bc2 = 1.0 - pow((double)p->beta2, (double)R.step);
            hipLaunchKernelGGL(k_adam, dim3((unsigned)nblk(R.nparam, 256)), dim3(256), 0, st, R.param, w.grad, R.mom,
                               R.vel, R.nparam, p->lr, p->beta1, p->beta2, p->eps, (float)bc1, (float)bc2);
            hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk(R.o_b1, 256)), dim3(256), 0, st, R.param, R.o_b1,
                               R.w1h);
            hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nblk((int64_t)R.nout * R.hid, 256)), dim3(256), 0, st,
                               R.param + R.o_w2, (int64_t)R.nout * R.hid, R.w2h);
            e = hipGetLastError();
            if (e != hipSuccess) {
                set_error("caps_router_train: %s", hipGetErrorString(e));
                s = CAPS_EDEVICE;
            }
        }
        if (s == CAPS_OK && out_loss) {
            float lsum = 0.0f;
            e = hipMemcpyAsync(&lsum, loss_dev, sizeof(float), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                set_error("caps_router_train: %s", hipGetErrorString(e));
                s = CAPS_EDEVICE;
            }
            out_loss[ep] = lsum / (float)n;   // mean over the epoch's rows
        }
    }
    (void)hipFreeAsync(loss_dev, st);
    (void)hipFreeAsync(base, st);
    if (s == CAPS_OK) CAPS_HIP(hipStreamSynchronize(st));
    return s;
}
