// Index files: save and load an index (and its router) as one versioned
// little-endian blob.
//
//   "CAPSIDX1"  magic (8 bytes)
//   u32 version (2), u32 header bytes, then the header: n (i64), d, b, h,
//   metric, precision, dpad, max_sub (i32), the attribute schema (i32
//   fields in declaration order), has_router, label slots per point (i32)
//   arrays: u32 tag, u64 bytes, payload -- in the fixed order of `arrays()`,
//   absent ones with 0 bytes
//   router (if present): din, dpad, hid, nout (i32), in_scale, in_shift,
//   fb_prob (f32), step (i64), nparam (i64), then param, mom, vel (FP32)
//
// The BF16 copies of the router weights are rebuilt on load; everything else
// is stored as it lives in HBM, so a loaded index answers every query
// exactly as the saved one.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "caps_device.h"
#include "caps_internal.h"

namespace caps {

static const char kMagic[8] = {'C', 'A', 'P', 'S', 'I', 'D', 'X', '1'};
constexpr uint32_t kVersion = 2;

struct ArrayRef {
    uint32_t tag;
    void **ptr;
    size_t bytes;   // size in the current index (save) / expected size (load; 0 = optional absent)
};

static std::vector<ArrayRef> arrays(Index &ix) {
    const size_t n = (size_t)ix.n, d = (size_t)ix.d, b = (size_t)ix.b, h = (size_t)ix.h;
    const bool lab = ix.sch.label_vocab > 0, dense = ix.sch.n_dense > 0, lowp = ix.prec != CAPS_PREC_NONE;
    const size_t es = ix.prec == CAPS_PREC_FP8 ? 1 : 2;
    return {
        {1, (void **)&ix.cent, 4 * b * d},
        {2, (void **)&ix.cnorm, 4 * b},
        {3, (void **)&ix.tags, 4 * b * (h > 0 ? h : 1)},
        {4, (void **)&ix.offs, 4 * (b * (h + 1) + 1)},
        {5, (void **)&ix.perm, 4 * n},
        {6, (void **)&ix.assign, 4 * n},
        {7, (void **)&ix.level, n},
        {8, (void **)&ix.vecs, 4 * n * d},
        {9, (void **)&ix.words, dense ? 4 * n : 0},
        {10, (void **)&ix.sigs, lab ? 8 * n : 0},
        {11, (void **)&ix.slots, lab ? 2 * n * (size_t)ix.lslots : 0},
        {12, (void **)&ix.lvecs, lowp ? n * (size_t)ix.dpad * es : 0},
        {13, (void **)&ix.lscale, ix.prec == CAPS_PREC_FP8 ? 4 * n : 0},
        {14, (void **)&ix.xnorm, lowp ? 4 * n : 0},
        {15, (void **)&ix.lerr, lowp ? 4 * n : 0},
        {16, (void **)&ix.lnrm, lowp ? 4 * n : 0},
    };
}

struct File {
    FILE *f = nullptr;
    ~File() {
        if (f) fclose(f);
    }
};

static bool put(FILE *f, const void *p, size_t bytes) { return fwrite(p, 1, bytes, f) == bytes; }
static bool get(FILE *f, void *p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

struct Header {
    int64_t n;
    int32_t d, b, h, metric, prec, dpad, max_sub;
    Schema sch;
    int32_t has_router;
    int32_t lslots;
};

static caps_status io_fail(const char *what, const char *path) {
    set_error("%s: %s", what, path);
    return CAPS_EIO;
}

static caps_status save(const Index &cix, const char *path) {
    Index &ix = const_cast<Index &>(cix);   // arrays() hands out pointers; nothing is modified
    CAPS_HIP(hipDeviceSynchronize());
    File F;
    F.f = fopen(path, "wb");
    if (!F.f) return io_fail("caps_save: cannot open", path);
    Header hd{};
    hd.n = ix.n;
    hd.d = ix.d;
    hd.b = ix.b;
    hd.h = ix.h;
    hd.metric = ix.metric;
    hd.prec = ix.prec;
    hd.dpad = ix.dpad;
    hd.max_sub = ix.max_sub;
    hd.sch = ix.sch;
    hd.has_router = ix.router ? 1 : 0;
    hd.lslots = ix.lslots;
    const uint32_t hb = sizeof(Header);
    bool ok = put(F.f, kMagic, 8) && put(F.f, &kVersion, 4) && put(F.f, &hb, 4) && put(F.f, &hd, sizeof hd);
    std::vector<uint8_t> host;
    for (const ArrayRef &a : arrays(ix)) {
        const uint64_t bytes = *a.ptr ? a.bytes : 0;
        ok = ok && put(F.f, &a.tag, 4) && put(F.f, &bytes, 8);
        if (!ok) break;
        if (bytes) {
            host.resize(bytes);
            CAPS_HIP(hipMemcpy(host.data(), *a.ptr, bytes, hipMemcpyDeviceToHost));
            ok = put(F.f, host.data(), bytes);
        }
    }
    if (ok && ix.router) {
        const Router &R = *ix.router;
        ok = put(F.f, &R.din, 4) && put(F.f, &R.dpad, 4) && put(F.f, &R.hid, 4) && put(F.f, &R.nout, 4) &&
             put(F.f, &R.in_scale, 4) && put(F.f, &R.in_shift, 4) && put(F.f, &R.fb_prob, 4) &&
             put(F.f, &R.step, 8) && put(F.f, &R.nparam, 8);
        const size_t pb = sizeof(float) * (size_t)R.nparam;
        host.resize(pb);
        for (float *src : {R.param, R.mom, R.vel}) {
            if (!ok) break;
            CAPS_HIP(hipMemcpy(host.data(), src, pb, hipMemcpyDeviceToHost));
            ok = put(F.f, host.data(), pb);
        }
    }
    if (!ok) return io_fail("caps_save: write failed", path);
    if (fclose(F.f) != 0) {
        F.f = nullptr;
        return io_fail("caps_save: close failed", path);
    }
    F.f = nullptr;
    return CAPS_OK;
}

__global__ void k_io_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = bf16_rne(x[i]);
}

// Checks the header's attribute schema against what caps_build derives
// from the vocabularies (the search kernels index with these fields).
static bool schema_ok(const Schema &s) {
    if (s.n_dense < 0 || s.n_dense > kMaxDense || s.label_vocab < 0 || s.label_vocab > 65535) return false;
    int bits = 0, off = 0;
    for (int a = 0; a < s.n_dense; a++) {
        const int32_t v = s.dense_vocab[a];
        if (v < 1) return false;
        int w = 1;
        while ((1ll << w) < v) w++;
        if (s.dense_off[a] != off || s.field_shift[a] != bits || s.field_bits[a] != w) return false;
        off += v;
        bits += w;
    }
    if (bits > 32 || s.dense_off[s.n_dense] != off) return false;
    return s.n_tok == off + s.label_vocab && s.n_tok <= kMaxTokensLds;
}

// Checks the partition arrays that steer the search's memory accesses: offs
// a monotone cover of [0, n) with one range per (partition, level), perm a
// permutation, assign and level consistent with the range holding each
// point, tags tokens of the schema (or -1 for an empty level), max_sub the
// largest range.  A file failing any of them is refused before any search.
static bool layout_ok(const Index &ix, const std::vector<int32_t> &tags, const std::vector<int32_t> &offs,
                      const std::vector<int32_t> &perm, const std::vector<int32_t> &assign,
                      const std::vector<int8_t> &level) {
    const int64_t n = ix.n, ns = (int64_t)ix.b * (ix.h + 1);
    if ((int64_t)offs.size() != ns + 1 || offs[0] != 0 || offs[(size_t)ns] != n) return false;
    int32_t mx = 0;
    for (int64_t s = 0; s < ns; s++) {
        if (offs[(size_t)s + 1] < offs[(size_t)s]) return false;
        mx = std::max(mx, offs[(size_t)s + 1] - offs[(size_t)s]);
    }
    if (mx != ix.max_sub) return false;
    std::vector<char> seen((size_t)n, 0);
    for (int64_t s = 0; s < ns; s++) {
        const int32_t p = (int32_t)(s / (ix.h + 1)), j = (int32_t)(s % (ix.h + 1));
        for (int32_t pos = offs[(size_t)s]; pos < offs[(size_t)s + 1]; pos++) {
            const int32_t id = perm[(size_t)pos];
            if (id < 0 || id >= n || seen[(size_t)id]) return false;
            seen[(size_t)id] = 1;
            if (assign[(size_t)id] != p || level[(size_t)id] != j) return false;
        }
    }
    for (int64_t t = 0; t < (int64_t)ix.b * ix.h; t++) {
        const int32_t tk = tags[(size_t)t];
        if (tk < -1 || tk >= ix.sch.n_tok) return false;
        const int64_t s = t / ix.h * (ix.h + 1) + t % ix.h;   // the level this tag names
        if (tk < 0 && offs[(size_t)s + 1] != offs[(size_t)s]) return false;
    }
    return true;
}

// Reads the file into a fresh index (device arrays allocated here).
static caps_status load(Index &ix, const char *path) {
    File F;
    F.f = fopen(path, "rb");
    if (!F.f) return io_fail("caps_load: cannot open", path);
    char magic[8];
    uint32_t ver = 0, hb = 0;
    Header hd{};
    if (!get(F.f, magic, 8) || memcmp(magic, kMagic, 8) != 0) return io_fail("caps_load: not an index file", path);
    if (!get(F.f, &ver, 4) || ver != kVersion) return io_fail("caps_load: unsupported file version", path);
    if (!get(F.f, &hb, 4) || hb != sizeof(Header) || !get(F.f, &hd, sizeof hd))
        return io_fail("caps_load: bad header", path);
    if (hd.n < 1 || hd.n > INT32_MAX - 1 || hd.d < 1 || hd.b < 1 || hd.b > kMaxPartitions || hd.b > hd.n ||
        hd.h < 0 || hd.h > kMaxHeight || (hd.metric != 0 && hd.metric != 1) || hd.prec < CAPS_PREC_NONE ||
        hd.prec > CAPS_PREC_FP16 || !schema_ok(hd.sch))
        return io_fail("caps_load: header values out of range", path);
    if (hd.prec != CAPS_PREC_NONE) {   // the copy's row width: the smallest of 32, 64, 128, 256 >= d
        int ns = 1;
        while (32 * ns < hd.d) ns <<= 1;
        if (hd.d > 256 || hd.dpad != 32 * ns) return io_fail("caps_load: low-precision row width does not match d", path);
    }
    CAPS_HIP(hipGetDevice(&ix.device));
    ix.n = hd.n;
    ix.d = hd.d;
    ix.b = hd.b;
    ix.h = hd.h;
    ix.metric = hd.metric;
    ix.prec = hd.prec;
    ix.dpad = hd.dpad;
    ix.max_sub = hd.max_sub;
    ix.sch = hd.sch;
    if (hd.lslots < kMaxLabels || hd.lslots > kMaxPointLabels || (hd.lslots & (hd.lslots - 1)))
        return io_fail("caps_load: label slot width out of range", path);
    ix.lslots = hd.lslots;
    std::vector<uint8_t> host;
    std::vector<int32_t> tags, offs, perm, assign;
    std::vector<int8_t> level;
    auto keep = [&](auto &v) {
        v.resize(host.size() / sizeof(v[0]));
        memcpy(v.data(), host.data(), host.size());
    };
    for (const ArrayRef &a : arrays(ix)) {
        uint32_t tag = 0;
        uint64_t bytes = 0;
        if (!get(F.f, &tag, 4) || !get(F.f, &bytes, 8) || tag != a.tag || bytes != a.bytes)
            return io_fail("caps_load: array table does not match the header", path);
        if (!bytes) continue;
        host.resize(bytes);
        if (!get(F.f, host.data(), bytes)) return io_fail("caps_load: truncated file", path);
        if (a.tag == 3) keep(tags);
        if (a.tag == 4) keep(offs);
        if (a.tag == 5) keep(perm);
        if (a.tag == 6) keep(assign);
        if (a.tag == 7) {   // the last of the layout arrays: check them before any vector is read
            keep(level);
            if (ix.h == 0) tags.clear();
            if (!layout_ok(ix, tags, offs, perm, assign, level))
                return io_fail("caps_load: inconsistent partition layout (offsets, permutation, levels or tags)",
                               path);
        }
        CAPS_HIP(hipMalloc(a.ptr, bytes));
        ix.bytes += (int64_t)bytes;
        CAPS_HIP(hipMemcpy(*a.ptr, host.data(), bytes, hipMemcpyHostToDevice));
    }
    ix.h_offs.resize((size_t)ix.b * (ix.h + 1) + 1);
    CAPS_HIP(hipMemcpy(ix.h_offs.data(), ix.offs, sizeof(int32_t) * ix.h_offs.size(), hipMemcpyDeviceToHost));
    {   // the centroid copy of precision-mode routing is derived, not stored
        const caps_status cs = build_lowp_centroids(&ix, nullptr);
        if (cs != CAPS_OK) return cs;
        CAPS_HIP(hipDeviceSynchronize());
    }
    if (hd.has_router) {
        Router *R = new Router;
        ix.router = R;
        bool ok = get(F.f, &R->din, 4) && get(F.f, &R->dpad, 4) && get(F.f, &R->hid, 4) && get(F.f, &R->nout, 4) &&
                  get(F.f, &R->in_scale, 4) && get(F.f, &R->in_shift, 4) && get(F.f, &R->fb_prob, 4) &&
                  get(F.f, &R->step, 8) && get(F.f, &R->nparam, 8);
        if (!ok || R->din != ix.d + 64 || R->dpad != (R->din + 31) / 32 * 32 || R->hid < 16 || R->hid > 8192 ||
            R->hid % 16 != 0 || R->nout != ix.b || R->step < 0 || !(R->in_scale == R->in_scale) ||
            !(R->in_shift == R->in_shift) || !(R->fb_prob == R->fb_prob) ||
            R->nparam != (int64_t)R->hid * R->dpad + R->hid + (int64_t)R->nout * R->hid + R->nout)
            return io_fail("caps_load: bad router section", path);
        R->o_b1 = (int64_t)R->hid * R->dpad;
        R->o_w2 = R->o_b1 + R->hid;
        R->o_b2 = R->o_w2 + (int64_t)R->nout * R->hid;
        const size_t pb = sizeof(float) * (size_t)R->nparam;
        host.resize(pb);
        for (float **dst : {&R->param, &R->mom, &R->vel}) {
            if (!get(F.f, host.data(), pb)) return io_fail("caps_load: truncated router", path);
            CAPS_HIP(hipMalloc((void **)dst, pb));
            CAPS_HIP(hipMemcpy(*dst, host.data(), pb, hipMemcpyHostToDevice));
        }
        CAPS_HIP(hipMalloc((void **)&R->w1h, sizeof(uint16_t) * (size_t)R->o_b1));
        CAPS_HIP(hipMalloc((void **)&R->w2h, sizeof(uint16_t) * (size_t)R->nout * R->hid));
        hipLaunchKernelGGL(k_io_bf16, dim3((unsigned)((R->o_b1 + 255) / 256)), dim3(256), 0, 0, R->param, R->o_b1,
                           R->w1h);
        hipLaunchKernelGGL(k_io_bf16, dim3((unsigned)(((int64_t)R->nout * R->hid + 255) / 256)), dim3(256), 0, 0,
                           R->param + R->o_w2, (int64_t)R->nout * R->hid, R->w2h);
        CAPS_HIP(hipGetLastError());
        CAPS_HIP(hipDeviceSynchronize());
    }
    return CAPS_OK;
}

}  // namespace caps

using namespace caps;

extern "C" caps_status caps_save(const caps_index *idx, const char *path) {
    if (!idx || !path) {
        set_error("caps_save: null argument");
        return CAPS_EINVAL;
    }
    return save(idx->ix, path);
}

extern "C" caps_status caps_load(const char *path, void *stream, caps_index **out) {
    (void)stream;
    if (!path || !out) {
        set_error("caps_load: null argument");
        return CAPS_EINVAL;
    }
    *out = nullptr;
    caps_index *h = new caps_index;
    const caps_status s = load(h->ix, path);
    if (s != CAPS_OK) {
        release_index(h->ix);
        delete h;
        return s;
    }
    *out = h;
    return CAPS_OK;
}
