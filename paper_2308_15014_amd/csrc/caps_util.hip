// Device-wide exclusive scan of int32 (three passes: block scans, scan of
// block sums, add-back).
#include <mutex>
#include <vector>

#include "caps_device.h"
#include "caps_internal.h"

namespace caps {

constexpr int kScanNT = 256;
constexpr int kScanIPT = 8;
constexpr int kScanTile = kScanNT * kScanIPT;

__global__ __launch_bounds__(kScanNT) void k_scan_tiles(const int32_t *in, int32_t *out, int64_t n,
                                                        int32_t *sums) {
    __shared__ int scratch[kScanNT / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    int v[kScanIPT];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanIPT; i++) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int total;
    int pre = block_excl_scan<kScanNT>(s, scratch, &total);
#pragma unroll
    for (int i = 0; i < kScanIPT; i++) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the tile sums in place (exclusive) and stores the total.
__global__ __launch_bounds__(1024) void k_scan_sums(int32_t *sums, int64_t nt, int32_t *total) {
    __shared__ int scratch[1024 / kWave + 1];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nt; b0 += 1024) {
        int64_t i = b0 + threadIdx.x;
        int v = i < nt ? sums[i] : 0;
        int tot;
        int pre = block_excl_scan<1024>(v, scratch, &tot);
        if (i < nt) sums[i] = pre + carry;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanNT) void k_scan_add(int32_t *out, int64_t n, const int32_t *sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int add = sums[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kScanNT) {
        int64_t e = base + i;
        if (e < n) out[e] += add;
    }
}

int64_t exclusive_scan_tiles(int64_t n) { return n <= 0 ? 0 : (n + kScanTile - 1) / kScanTile; }

caps_status exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *sums,
                               hipStream_t st) {
    if (n <= 0) return CAPS_OK;
    const int64_t nt = exclusive_scan_tiles(n);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanNT), 0, st, in, out, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, nt, total);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(kScanNT), 0, st, out, n, sums);
    CAPS_HIP(hipGetLastError());
    return CAPS_OK;
}

// ---- host-side caches of the per-call runtime settings
// A library memory pool per device that keeps what is freed into it
// (release threshold: never), so that a search's stream-ordered free does not
// hand its workspace back to the system: with the default pool that free cost
// about 1.7 ms of host time per call, as long as the kernels of a call.
constexpr int kMaxDevices = 64;
static std::mutex g_pool_mu;
static hipMemPool_t g_pool[kMaxDevices];

caps_status ws_alloc(void **p, size_t bytes, int device, hipStream_t st) {
    if (device < 0 || device >= kMaxDevices) {
        CAPS_HIP(hipMallocAsync(p, bytes, st));
        return CAPS_OK;
    }
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> g(g_pool_mu);
        if (!g_pool[device]) {
            hipMemPoolProps props{};
            props.allocType = hipMemAllocationTypePinned;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = device;
            hipMemPool_t np = nullptr;
            CAPS_HIP(hipMemPoolCreate(&np, &props));
            uint64_t keep = ~0ull;
            const hipError_t e = hipMemPoolSetAttribute(np, hipMemPoolAttrReleaseThreshold, &keep);
            if (e != hipSuccess) {
                (void)hipMemPoolDestroy(np);
                set_error("hipMemPoolSetAttribute failed: %s", hipGetErrorString(e));
                return CAPS_EDEVICE;
            }
            g_pool[device] = np;
        }
        pool = g_pool[device];
    }
    CAPS_HIP(hipMallocFromPoolAsync(p, bytes, pool, st));
    return CAPS_OK;
}

// The maximum dynamic LDS of a kernel, set once per (kernel, device) to the
// largest size asked for (each setting cost about 0.2 ms of host time).
static std::mutex g_lds_mu;
static std::vector<std::pair<std::pair<const void *, int>, int>> g_lds;

caps_status set_kernel_lds(const void *fn, size_t bytes, int device) {
    std::lock_guard<std::mutex> g(g_lds_mu);
    for (auto &e : g_lds)
        if (e.first.first == fn && e.first.second == device) {
            if ((int)bytes <= e.second) return CAPS_OK;
            CAPS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
            e.second = (int)bytes;
            return CAPS_OK;
        }
    CAPS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    g_lds.push_back({{fn, device}, (int)bytes});
    return CAPS_OK;
}

// ------------------------------------------------------------------ stage timer
namespace {
struct Rec {
    int stage;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Rec> g_recs;
hipEvent_t g_open[CAPS_N_STAGES];
caps_profile_t g_acc;
}  // namespace

void prof_begin(int stage, hipStream_t st) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    g_open[stage] = e;
}

void prof_end(int stage, hipStream_t st) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on || !g_open[stage]) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    g_recs.push_back({stage, g_open[stage], e});
    g_open[stage] = nullptr;
}

}  // namespace caps

extern "C" caps_status caps_profile_enable(int32_t on) {
    using namespace caps;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &r : g_recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    for (auto &e : g_open) e = nullptr;
    g_acc = caps_profile_t{};
    g_prof_on = on != 0;
    return CAPS_OK;
}

extern "C" caps_status caps_profile_read(caps_profile_t *out) {
    using namespace caps;
    if (!out) return CAPS_EINVAL;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &r : g_recs) {
        float ms = 0.0f;
        CAPS_HIP(hipEventSynchronize(r.b));
        CAPS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        g_acc.ms[r.stage] += ms;
        g_acc.launches[r.stage] += 1;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    *out = g_acc;
    return CAPS_OK;
}
