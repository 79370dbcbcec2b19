// knnf_api.cpp -- host runtime behind include/knnf.h.
//
// Validation, launch planning, the batch work table and the autotuner.  All
// arithmetic of the method runs in the HIP kernels (knnf_kernels.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/knnf.h"
#include "knnf_device.h"
#include "knnf_internal.h"

namespace {

thread_local std::string g_err;

knnf_status vfail(knnf_status st, const char* fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    g_err = buf;
    return st;
}

knnf_status fail(knnf_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(st, fmt, ap);
    va_end(ap);
    return st;
}

knnf_status hip_fail(hipError_t e, const char* what) {
    return fail(KNNF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// One slot of batch tables: device work table (frame descriptors, task
// prefix, first tiles, claim counter) and a pinned host staging copy.  `done`
// is recorded after the launch that uses the slot, so the slot is reused only
// after that launch has finished.
struct BatchSlot {
    void* dev = nullptr;
    void* host = nullptr;
    void* host_dev = nullptr;  // device address of the pinned staging, if mapped
    size_t cap = 0;           // work items
    hipEvent_t done = nullptr;
    bool recorded = false;
};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
size_t off_task_start(size_t cap) { return round256(cap * sizeof(knnf::FrameDesc)); }
size_t off_tile_base(size_t cap) { return off_task_start(cap) + round256((cap + 1) * sizeof(uint32_t)); }
size_t off_counter(size_t cap) { return off_tile_base(cap) + round256(cap * sizeof(uint32_t)); }
size_t slot_bytes(size_t cap) { return off_counter(cap) + 256; }

constexpr int kSlots = 4;
// Work items every slot holds from context creation on, so that batched
// launches of up to this many items (the serving steps) never allocate.
constexpr size_t kSlotItems = 64;

// Give a slot room for at least n work items.  The slot must be idle (its
// last launch finished).  Allocating synchronises the device, so it is done
// up front for kSlotItems and only grows for larger batches.
hipError_t grow_slot(BatchSlot& s, size_t n) {
    if (s.cap >= n) return hipSuccess;
    size_t cap = std::max<size_t>(kSlotItems, s.cap);
    while (cap < n) cap *= 2;
    if (s.dev) hipFree(s.dev);
    if (s.host) hipHostFree(s.host);
    s.dev = s.host = s.host_dev = nullptr;
    s.cap = 0;
    hipError_t e = hipMalloc(&s.dev, slot_bytes(cap));
    if (e != hipSuccess) return e;
    e = hipHostMalloc(&s.host, slot_bytes(cap), hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(s.dev);
        s.dev = nullptr;
        return e;
    }
    s.host_dev = nullptr;
    if (hipHostGetDevicePointer(&s.host_dev, s.host, 0) != hipSuccess) {
        s.host_dev = nullptr;
        (void)hipGetLastError();  // not mapped: the table is copied instead
    }
    s.cap = cap;
    return hipSuccess;
}

}  // namespace

struct knnf_ctx {
    int device = 0;
    int num_cu = 256;
    knnf_plan plan{};
    std::mutex mu;
    BatchSlot slots[kSlots];
    int next_slot = 0;
    unsigned long long* d_stats = nullptr;  // work counters while enabled
    bool stats_on = false;
    // PC1 workspace: [per-block (min, max) pairs][npix doubles]
    char* pc1_ws = nullptr;
    size_t pc1_ws_bytes = 0;
};

namespace {

knnf_plan default_plan() {
    knnf_plan p{};
    p.search = KNNF_SEARCH_PRUNED;
    p.tile_rows = 1;
    p.tile_cols = 8;
    p.waves = 1;
    p.launch = KNNF_LAUNCH_GRID;
    return p;
}

const int kShapes[][2] = {{1, 8}, {1, 16}, {2, 4}, {2, 8}, {4, 4}};

bool plan_ok_impl(const knnf_plan& p) {
    if (p.search != KNNF_SEARCH_EXHAUSTIVE && p.search != KNNF_SEARCH_PRUNED) return false;
    bool shape = false;
    for (const auto& s : kShapes) shape |= (p.tile_rows == s[0] && p.tile_cols == s[1]);
    if (!shape) return false;
    if (p.waves != 1 && p.waves != 2 && p.waves != 4) return false;
    if (p.launch != KNNF_LAUNCH_PERSISTENT && p.launch != KNNF_LAUNCH_GRID) return false;
    return true;
}

knnf_plan resolve_impl(const knnf_ctx* ctx, const knnf_plan* p) {
    knnf_plan r = ctx->plan;
    if (p) {
        r.search = p->search;
        if (p->tile_rows) r.tile_rows = p->tile_rows;
        if (p->tile_cols) r.tile_cols = p->tile_cols;
        if (p->waves) r.waves = p->waves;
        if (p->launch) r.launch = p->launch;
    }
    return r;
}

knnf::LaunchCfg to_cfg(const knnf_plan& p) {
    knnf::LaunchCfg c;
    c.rows = p.tile_rows;
    c.cols = p.tile_cols;
    c.waves = p.waves;
    c.pruned = p.search == KNNF_SEARCH_PRUNED ? 1 : 0;
    c.persistent = p.launch != KNNF_LAUNCH_GRID;
    return c;
}

knnf::FrameDesc to_desc_impl(const knnf_frame& f) {
    knnf::FrameDesc d;
    d.pc1 = f.pc1;
    d.prob = f.prob;
    d.out_prob = f.out_prob;
    d.out_class = f.out_class;
    d.out_nbr = f.out_nbr;
    d.out_dist = f.out_dist;
    d.H = f.H;
    d.W = f.W;
    d.C = f.C;
    d.K = f.K;
    d.R = f.R;
    d.lambda = f.lambda;
    d.stats = nullptr;
    return d;
}

knnf_status validate_impl(const knnf_frame* f, int index) {
    if (!f) return fail(KNNF_EINVAL, "frame %d: NULL frame", index);
    if (f->H < 1 || f->W < 1)
        return fail(KNNF_EINVAL, "frame %d: H=%d W=%d must be >= 1", index, f->H, f->W);
    if (f->H > KNNF_MAX_SIDE || f->W > KNNF_MAX_SIDE)
        return fail(KNNF_EINVAL, "frame %d: H or W exceeds %d", index, KNNF_MAX_SIDE);
    if ((int64_t)f->H * f->W > 0x7fffffffLL)
        return fail(KNNF_EINVAL, "frame %d: H*W exceeds 2^31-1", index);
    if (f->C < 1 || f->C > KNNF_MAX_C)
        return fail(KNNF_EINVAL, "frame %d: C=%d outside 1..%d", index, f->C, KNNF_MAX_C);
    if (f->R < 0) return fail(KNNF_EINVAL, "frame %d: R=%d < 0", index, f->R);
    if (f->K < 1 || f->K > KNNF_MAX_K)
        return fail(KNNF_EINVAL, "frame %d: K=%d outside 1..%d", index, f->K, KNNF_MAX_K);
    const int64_t minrows = std::min<int64_t>((int64_t)f->R + 1, f->H);
    if ((int64_t)f->K > minrows * f->W)
        return fail(KNNF_EINVAL, "frame %d: K=%d exceeds the smallest window (%lld pixels)",
                    index, f->K, (long long)(minrows * f->W));
    if (!std::isfinite(f->lambda) || f->lambda < 0.0f)
        return fail(KNNF_EINVAL, "frame %d: lambda must be finite and >= 0", index);
    if ((double)f->lambda * (double)std::max(f->H, f->W) > 1e18)
        return fail(KNNF_EINVAL, "frame %d: lambda * max(H, W) exceeds 1e18", index);
    if (!f->pc1 || !f->prob || !f->out_prob || !f->out_class)
        return fail(KNNF_EINVAL, "frame %d: NULL required pointer", index);
    return KNNF_OK;
}

// Relative cost of one tile task of a frame (candidate pairs per tile).
double task_cost(const knnf_frame& f, int Q) {
    const double rows = std::min<double>(2.0 * f.R + 1.0, f.H);
    return (double)Q * rows * (double)f.W;
}

}  // namespace

namespace knnf {

knnf_status set_error(knnf_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(st, fmt, ap);
    va_end(ap);
    return st;
}
knnf_status validate_frame(const knnf_frame* f, int index) { return validate_impl(f, index); }
knnf_plan resolve_plan(const knnf_ctx* ctx, const knnf_plan* p) { return resolve_impl(ctx, p); }
bool plan_valid(const knnf_plan& p) { return plan_ok_impl(p); }
FrameDesc desc_of(const knnf_frame& f) { return to_desc_impl(f); }
uint32_t tiles_of(int H, int W, const knnf_plan& p) {
    return (uint32_t)((H + p.tile_rows - 1) / p.tile_rows) * (uint32_t)((W + p.tile_cols - 1) / p.tile_cols);
}
int ctx_device(const knnf_ctx* ctx) { return ctx->device; }

knnf_status launch_items(knnf_ctx* ctx, const WorkItem* items, int n, const knnf_plan& p,
                         void* stream) {
    uint64_t total = 0;
    for (int k = 0; k < n; ++k) {
        total += items[k].ntiles;
        if (total > 0xfff00000ull) return fail(KNNF_EINVAL, "batched launch: too much work");
    }
    if (total == 0) return KNNF_OK;
    std::lock_guard<std::mutex> lock(ctx->mu);
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};

    BatchSlot& s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % kSlots;
    hipError_t e;
    if (s.recorded) {
        e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return hip_fail(e, "batch slot wait");
        s.recorded = false;
    }
    e = grow_slot(s, (size_t)n);
    if (e != hipSuccess) return fail(KNNF_ENOMEM, "batch table: %s", hipGetErrorString(e));
    hipStream_t hs = (hipStream_t)stream;
    constexpr size_t kDescWords = sizeof(knnf::FrameDesc) / 4;
    static_assert(sizeof(knnf::FrameDesc) % 4 == 0, "descriptor size");
    if ((size_t)n * (kDescWords + 2) + 1 <= (size_t)knnf::kTableWords) {
        // small table (a serving step): written by a kernel that receives it
        // as its argument, so this thread never waits on a copy
        knnf::TableWords t;
        uint32_t* tw = t.w;
        const size_t nd = (size_t)n * kDescWords;
        uint32_t acc = 0;
        for (int k = 0; k < n; ++k) {
            knnf::FrameDesc d = items[k].f;
            d.stats = ctx->stats_on ? ctx->d_stats : nullptr;
            std::memcpy(tw + (size_t)k * kDescWords, &d, sizeof d);
            tw[nd + k] = acc;                // task prefix
            tw[nd + n + 1 + k] = items[k].tile0;  // first tiles
            acc += items[k].ntiles;
        }
        tw[nd + n] = acc;
        t.src[0] = 0;
        t.dst[0] = 0;
        t.len[0] = (uint32_t)nd;
        t.src[1] = (uint32_t)nd;
        t.dst[1] = (uint32_t)(off_task_start(s.cap) / 4);
        t.len[1] = (uint32_t)n + 1;
        t.src[2] = (uint32_t)(nd + n + 1);
        t.dst[2] = (uint32_t)(off_tile_base(s.cap) / 4);
        t.len[2] = (uint32_t)n;
        const int rc = knnf::launch_put_table(t, (uint32_t*)s.dev, stream);
        if (rc != 0) return hip_fail((hipError_t)rc, "batch table write");
    } else {
        knnf::FrameDesc* hf = (knnf::FrameDesc*)s.host;
        uint32_t* hts = (uint32_t*)((char*)s.host + off_task_start(s.cap));
        uint32_t* htb = (uint32_t*)((char*)s.host + off_tile_base(s.cap));
        uint32_t acc = 0;
        for (int k = 0; k < n; ++k) {
            hf[k] = items[k].f;
            hf[k].stats = ctx->stats_on ? ctx->d_stats : nullptr;
            hts[k] = acc;
            htb[k] = items[k].tile0;
            acc += items[k].ntiles;
        }
        hts[n] = acc;
        // the whole table prefix (descriptors, prefix, first tiles) goes to the
        // device in one piece: pulled by a kernel from the mapped staging (a
        // copy call could hold this thread for milliseconds), else copied
        if (s.host_dev) {
            const int rc = knnf::launch_copy_pair((const uint32_t*)s.host_dev, (uint32_t*)s.dev,
                                                  (uint32_t)(off_counter(s.cap) / 4), nullptr,
                                                  nullptr, 0, stream);
            if (rc != 0) return hip_fail((hipError_t)rc, "batch table write");
        } else {
            e = hipMemcpyAsync(s.dev, s.host, off_counter(s.cap), hipMemcpyHostToDevice, hs);
            if (e != hipSuccess) return hip_fail(e, "batch table copy");
        }
    }
    uint32_t* d_ctr = (uint32_t*)((char*)s.dev + off_counter(s.cap));
    const knnf::LaunchCfg cfg = to_cfg(p);
    int rc;
    if (!cfg.persistent) {
        rc = knnf::launch_filter_items((const knnf::FrameDesc*)s.dev,
                                       (const uint32_t*)((char*)s.dev + off_task_start(s.cap)),
                                       (const uint32_t*)((char*)s.dev + off_tile_base(s.cap)),
                                       (uint32_t)n, (uint32_t)total, cfg, stream);
        if (rc != 0) return hip_fail((hipError_t)rc, "batched launch");
        e = hipEventRecord(s.done, hs);
        if (e != hipSuccess) return hip_fail(e, "batch slot record");
        s.recorded = true;
        return KNNF_OK;
    }
    rc = knnf::launch_zero_counter(d_ctr, stream);
    if (rc != 0) return hip_fail((hipError_t)rc, "counter reset");
    const uint64_t need_blocks = (total + p.waves - 1) / p.waves;
    const int per_cu = knnf::persistent_blocks_per_cu(cfg);
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(need_blocks,
                                                  (uint64_t)ctx->num_cu * per_cu));
    rc = knnf::launch_filter_batch((const knnf::FrameDesc*)s.dev,
                                   (const uint32_t*)((char*)s.dev + off_task_start(s.cap)),
                                   (const uint32_t*)((char*)s.dev + off_tile_base(s.cap)),
                                   (uint32_t)n, (uint32_t)total, d_ctr, cfg, (int)grid, stream);
    if (rc != 0) return hip_fail((hipError_t)rc, "batched launch");
    e = hipEventRecord(s.done, hs);
    if (e != hipSuccess) return hip_fail(e, "batch slot record");
    s.recorded = true;
    return KNNF_OK;
}

}  // namespace knnf

extern "C" {

const char* knnf_last_error(void) { return g_err.c_str(); }

const char* knnf_version(void) { return "knnf 0.1.0 gfx950"; }

knnf_status knnf_validate(const knnf_frame* frame) { return validate_impl(frame, 0); }

size_t knnf_frame_bytes(int H, int W, int C, int K, int with_nbr) {
    if (H < 1 || W < 1 || C < 1 || K < 1) return 0;
    auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t px = (size_t)H * (size_t)W;
    size_t t = r(px * 4) + r(px * C * 4) + r(px * C * 4) + r(px * 4);
    if (with_nbr) t += r(px * K * 4) + r(px * K * 4);
    return t;
}

knnf_status knnf_create(knnf_ctx** out, int device) {
    if (!out) return fail(KNNF_EINVAL, "knnf_create: NULL out");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(KNNF_EINVAL, "device %d of %d", device, n);
    knnf_ctx* c = new (std::nothrow) knnf_ctx;
    if (!c) return fail(KNNF_ENOMEM, "knnf_create: out of host memory");
    c->device = device;
    c->plan = default_plan();
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    for (auto& s : c->slots) {
        e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = grow_slot(s, kSlotItems);
        if (e != hipSuccess) {
            hipSetDevice(prev);
            knnf_destroy(c);
            return hip_fail(e, "knnf_create: batch table slots");
        }
    }
    hipSetDevice(prev);
    *out = c;
    return KNNF_OK;
}

knnf_status knnf_destroy(knnf_ctx* ctx) {
    if (!ctx) return KNNF_OK;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    for (auto& s : ctx->slots) {
        if (s.done) {
            if (s.recorded) hipEventSynchronize(s.done);
            hipEventDestroy(s.done);
        }
        if (s.dev) hipFree(s.dev);
        if (s.host) hipHostFree(s.host);
    }
    if (ctx->d_stats) hipFree(ctx->d_stats);
    if (ctx->pc1_ws) {
        hipDeviceSynchronize();
        hipFree(ctx->pc1_ws);
    }
    hipSetDevice(prev);
    delete ctx;
    return KNNF_OK;
}

knnf_status knnf_set_default_plan(knnf_ctx* ctx, const knnf_plan* plan) {
    if (!ctx || !plan) return fail(KNNF_EINVAL, "knnf_set_default_plan: NULL argument");
    knnf_plan p = resolve_impl(ctx, plan);
    if (!plan_ok_impl(p)) return fail(KNNF_EINVAL, "invalid plan");
    ctx->plan = p;
    return KNNF_OK;
}

knnf_status knnf_get_default_plan(const knnf_ctx* ctx, knnf_plan* plan) {
    if (!ctx || !plan) return fail(KNNF_EINVAL, "knnf_get_default_plan: NULL argument");
    *plan = ctx->plan;
    return KNNF_OK;
}

knnf_status knnf_filter(knnf_ctx* ctx, const knnf_frame* frame, const knnf_plan* plan,
                        void* stream) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_filter: NULL context");
    knnf_status st = validate_impl(frame, 0);
    if (st != KNNF_OK) return st;
    const knnf_plan p = resolve_impl(ctx, plan);
    if (!plan_ok_impl(p)) return fail(KNNF_EINVAL, "knnf_filter: invalid plan");
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    knnf::FrameDesc desc = to_desc_impl(*frame);
    desc.stats = ctx->stats_on ? ctx->d_stats : nullptr;
    const int e = knnf::launch_filter_frame(desc, to_cfg(p), stream);
    if (prev != ctx->device) hipSetDevice(prev);
    if (e != 0) return hip_fail((hipError_t)e, "knnf_filter launch");
    return KNNF_OK;
}

knnf_status knnf_filter_batch(knnf_ctx* ctx, const knnf_frame* frames, int n,
                              const knnf_plan* plan, void* stream) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_filter_batch: NULL context");
    if (n < 0 || (n > 0 && !frames)) return fail(KNNF_EINVAL, "knnf_filter_batch: bad frame list");
    if (n == 0) return KNNF_OK;
    for (int i = 0; i < n; ++i) {
        knnf_status st = validate_impl(&frames[i], i);
        if (st != KNNF_OK) return st;
    }
    const knnf_plan p = resolve_impl(ctx, plan);
    if (!plan_ok_impl(p)) return fail(KNNF_EINVAL, "knnf_filter_batch: invalid plan");
    const int Q = p.tile_rows * p.tile_cols;
    // Largest tile cost first: long tasks start early, short ones fill the tail.
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return task_cost(frames[a], Q) > task_cost(frames[b], Q);
    });
    std::vector<knnf::WorkItem> items(n);
    for (int k = 0; k < n; ++k) {
        const knnf_frame& f = frames[order[k]];
        items[k].f = to_desc_impl(f);
        items[k].tile0 = 0;
        items[k].ntiles = knnf::tiles_of(f.H, f.W, p);
    }
    return knnf::launch_items(ctx, items.data(), n, p, stream);
}

knnf_status knnf_pc1(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                     const double* mean, const double* vec, float* out, int32_t normalize,
                     void* stream) {
    if (npix < 1 || npix > KNNF_PC1_MAX_PIXELS)
        return fail(KNNF_EINVAL, "knnf_pc1: npix %lld outside [1, 2^40]", (long long)npix);
    if (bands < 1 || bands > KNNF_PC1_MAX_BANDS)
        return fail(KNNF_EINVAL, "knnf_pc1: bands %d outside [1, %d]", bands, KNNF_PC1_MAX_BANDS);
    if (!cube || !mean || !vec || !out) return fail(KNNF_EINVAL, "knnf_pc1: NULL pointer");
    if (!ctx) return fail(KNNF_EINVAL, "knnf_pc1: NULL context");
    std::lock_guard<std::mutex> lock(ctx->mu);
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};
    const size_t head = ((size_t)2 * knnf::pc1_max_blocks() * sizeof(double) + 255) & ~size_t(255);
    const size_t need = head + (normalize ? (size_t)npix * sizeof(double) : 0);
    if (ctx->pc1_ws_bytes < need) {
        // grow: earlier launches may still use the old buffer
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "knnf_pc1: synchronize");
        const size_t bytes = std::max(need, ctx->pc1_ws_bytes * 2);
        if (ctx->pc1_ws) hipFree(ctx->pc1_ws);
        ctx->pc1_ws = nullptr;
        ctx->pc1_ws_bytes = 0;
        e = hipMalloc((void**)&ctx->pc1_ws, bytes);
        if (e != hipSuccess) return fail(KNNF_ENOMEM, "knnf_pc1 workspace: %s", hipGetErrorString(e));
        ctx->pc1_ws_bytes = bytes;
    }
    double* pairs = (double*)ctx->pc1_ws;
    double* ws = normalize ? (double*)(ctx->pc1_ws + head) : nullptr;
    const int rc = knnf::launch_pc1(cube, npix, bands, mean, vec, out, ws, pairs, ctx->num_cu,
                                    stream);
    if (rc != 0) return hip_fail((hipError_t)rc, "knnf_pc1 launch");
    return KNNF_OK;
}

knnf_status knnf_svm(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                     int32_t classes, const double* w, const double* bias, const double* A,
                     const double* B, float* out, void* stream) {
    if (npix < 1 || npix > KNNF_SVM_MAX_PIXELS)
        return fail(KNNF_EINVAL, "knnf_svm: npix %lld outside [1, 2^31]", (long long)npix);
    if (bands < 1 || bands > KNNF_SVM_MAX_BANDS)
        return fail(KNNF_EINVAL, "knnf_svm: bands %d outside [1, %d]", bands, KNNF_SVM_MAX_BANDS);
    if (classes < 2 || classes > KNNF_SVM_MAX_CLASSES)
        return fail(KNNF_EINVAL, "knnf_svm: classes %d outside [2, %d]", classes,
                    KNNF_SVM_MAX_CLASSES);
    if (!cube || !w || !bias || !A || !B || !out) return fail(KNNF_EINVAL, "knnf_svm: NULL pointer");
    if (!ctx) return fail(KNNF_EINVAL, "knnf_svm: NULL context");
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};
    const int rc = knnf::launch_svm(cube, npix, bands, classes, w, bias, A, B, out, stream);
    if (rc != 0) return hip_fail((hipError_t)rc, "knnf_svm launch");
    return KNNF_OK;
}

knnf_status knnf_stats_enable(knnf_ctx* ctx, int on) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_stats_enable: NULL context");
    if (on && !ctx->d_stats) {
        int prev = 0;
        hipGetDevice(&prev);
        hipSetDevice(ctx->device);
        hipError_t e = hipMalloc((void**)&ctx->d_stats, 2 * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMemset(ctx->d_stats, 0, 2 * sizeof(unsigned long long));
        hipSetDevice(prev);
        if (e != hipSuccess) return fail(KNNF_ENOMEM, "knnf_stats_enable: %s", hipGetErrorString(e));
    }
    ctx->stats_on = on != 0;
    return KNNF_OK;
}

knnf_status knnf_stats_read(knnf_ctx* ctx, uint64_t* pairs, uint64_t* tiles, int reset) {
    if (!ctx || !pairs || !tiles) return fail(KNNF_EINVAL, "knnf_stats_read: NULL argument");
    *pairs = *tiles = 0;
    if (!ctx->d_stats) return KNNF_OK;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h, ctx->d_stats, sizeof h, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) e = hipMemset(ctx->d_stats, 0, sizeof h);
    hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "knnf_stats_read");
    *pairs = h[0];
    *tiles = h[1];
    return KNNF_OK;
}

knnf_status knnf_tune(knnf_ctx* ctx, const knnf_frame* frames, int n, int reps, void* stream,
                      knnf_plan* best) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_tune: NULL context");
    if (n < 1 || !frames || reps < 1) return fail(KNNF_EINVAL, "knnf_tune: bad arguments");
    for (int i = 0; i < n; ++i) {
        knnf_status st = validate_impl(&frames[i], i);
        if (st != KNNF_OK) return st;
    }
    static const int ws[] = {1, 2, 4};
    static const int ss[] = {KNNF_SEARCH_EXHAUSTIVE, KNNF_SEARCH_PRUNED};
    static const int ls[] = {KNNF_LAUNCH_PERSISTENT, KNNF_LAUNCH_GRID};
    hipStream_t hs = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(KNNF_EDEVICE, "knnf_tune: event create");
    float best_ms = 1e30f;
    knnf_plan bp = ctx->plan;
    knnf_status result = KNNF_OK;
    for (int s : ss)
        for (const auto& sh : kShapes)
            for (int w : ws)
                for (int l : ls) {
                if (n == 1 && l == KNNF_LAUNCH_GRID) continue;  // single frames ignore it
                knnf_plan p{};
                p.search = s;
                p.tile_rows = sh[0];
                p.tile_cols = sh[1];
                p.waves = w;
                p.launch = l;
                if (!plan_ok_impl(p)) continue;
                auto run = [&]() -> knnf_status {
                    return n == 1 ? knnf_filter(ctx, frames, &p, stream)
                                  : knnf_filter_batch(ctx, frames, n, &p, stream);
                };
                knnf_status st = run();  // warm-up
                if (st != KNNF_OK) { result = st; goto done; }
                hipEventRecord(e0, hs);
                for (int r = 0; r < reps && st == KNNF_OK; ++r) st = run();
                hipEventRecord(e1, hs);
                if (st != KNNF_OK) { result = st; goto done; }
                if (hipEventSynchronize(e1) != hipSuccess) {
                    result = fail(KNNF_EDEVICE, "knnf_tune: synchronize");
                    goto done;
                }
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_ms) {
                    best_ms = ms;
                    bp = p;
                }
            }
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (result != KNNF_OK) return result;
    if (best) *best = bp;
    return KNNF_OK;
}

}  // extern "C"
