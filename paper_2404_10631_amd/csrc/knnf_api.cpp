// knnf_api.cpp -- host runtime behind include/knnf.h.
//
// Validation, launch planning, the batch work table and the autotuner.  All
// arithmetic of the method runs in the HIP kernels (knnf_kernels.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
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

struct TunedPlan {
    knnf_plan plan{};
    double ms = 0.0;  // time of one call with this plan when it was tuned
};

// Slots of the non-finite input check: a check kernel stores the call's
// generation number into its slot of device-visible pinned host memory.
constexpr int kCheckSlots = 64;

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
    // failure state: once a HIP call failed, every call returns KNNF_EDEVICE
    std::atomic<int> failed{0};
    char failed_msg[256] = {0};
    // non-finite input check flags (host memory, and its device address)
    uint32_t* check_host = nullptr;
    uint32_t* check_dev = nullptr;
    std::atomic<uint32_t> check_gen{0};
    // plans picked by knnf_tune, by frame key; optional JSON file
    std::mutex tune_mu;
    std::map<std::string, TunedPlan> tuned;
    std::string tune_path;
    // knnf_pc1_noalloc's static scratch on this device (device address)
    void* pc1_scratch = nullptr;
};

namespace {

// Mark the context failed after a failed HIP call (first failure kept).
knnf_status ctx_fail(knnf_ctx* ctx, hipError_t e, const char* what) {
    int expect = 0;
    if (ctx->failed.compare_exchange_strong(expect, 1))
        snprintf(ctx->failed_msg, sizeof ctx->failed_msg, "%s: %s", what, hipGetErrorString(e));
    return fail(KNNF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// KNNF_EDEVICE (with the first failure's text) if the context has failed.
knnf_status ctx_check(const knnf_ctx* ctx) {
    if (ctx->failed.load()) return fail(KNNF_EDEVICE, "context failed earlier (%s)", ctx->failed_msg);
    return KNNF_OK;
}

knnf_plan default_plan() {
    knnf_plan p{};
    p.search = KNNF_SEARCH_PRUNED;
    p.tile_rows = 1;
    p.tile_cols = 8;
    p.waves = 1;
    p.launch = KNNF_LAUNCH_GRID;
    p.chunk_rows = 16;
    p.flags = 0;
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
    if (p.chunk_rows != 8 && p.chunk_rows != 16 && p.chunk_rows != 32) return false;
    if (p.flags & ~KNNF_PLAN_NO_INPUT_CHECK) return false;
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
        if (p->chunk_rows) r.chunk_rows = p->chunk_rows;
        r.flags = p->flags;
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
    c.chunk_log2 = p.chunk_rows == 8 ? 3 : (p.chunk_rows == 32 ? 5 : 4);
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

// ---- plans picked by the autotuner -----------------------------------------

// Cache key of a frame list: one frame by its (H, W, K, R, C); a batch by its
// length and a hash (FNV-1a, 64 bits) of those tuples in order.
std::string tune_key(const knnf_frame* f, int n) {
    char buf[96];
    if (n == 1) {
        snprintf(buf, sizeof buf, "frame H=%d W=%d K=%d R=%d C=%d", f->H, f->W, f->K, f->R, f->C);
        return buf;
    }
    uint64_t h = 1469598103934665603ull;
    for (int k = 0; k < n; ++k) {
        const int32_t v[5] = {f[k].H, f[k].W, f[k].K, f[k].R, f[k].C};
        const unsigned char* b = (const unsigned char*)v;
        for (size_t t = 0; t < sizeof v; ++t) h = (h ^ b[t]) * 1099511628211ull;
    }
    snprintf(buf, sizeof buf, "batch n=%d h=%016llx", n, (unsigned long long)h);
    return buf;
}

// The cached plan of a frame list (the context default's flags kept), or
// false when nothing is cached for it.
bool tuned_plan(const knnf_ctx* ctx, const knnf_frame* f, int n, knnf_plan* out) {
    knnf_ctx* c = const_cast<knnf_ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->tune_mu);
    if (c->tuned.empty()) return false;
    auto it = c->tuned.find(tune_key(f, n));
    if (it == c->tuned.end()) return false;
    *out = it->second.plan;
    out->flags = ctx->plan.flags;
    return true;
}

// The tune cache as JSON: {"knnf_tune_cache": 1, "entries": [{"key": ...,
// "search": ..., "tile_rows": ..., "tile_cols": ..., "waves": ..., "launch":
// ..., "chunk_rows": ..., "ms": ...}, ...]}.  Written to a temporary file and
// renamed, so a reader never sees half a file.
bool save_tune_cache(knnf_ctx* ctx) {
    if (ctx->tune_path.empty()) return true;
    const std::string tmp = ctx->tune_path + ".tmp";
    FILE* fp = fopen(tmp.c_str(), "w");
    if (!fp) return false;
    fprintf(fp, "{\"knnf_tune_cache\": 1, \"entries\": [");
    bool first = true;
    for (const auto& kv : ctx->tuned) {
        const knnf_plan& p = kv.second.plan;
        fprintf(fp,
                "%s\n  {\"key\": \"%s\", \"search\": %d, \"tile_rows\": %d, \"tile_cols\": %d, "
                "\"waves\": %d, \"launch\": %d, \"chunk_rows\": %d, \"ms\": %.6f}",
                first ? "" : ",", kv.first.c_str(), p.search, p.tile_rows, p.tile_cols, p.waves,
                p.launch, p.chunk_rows, kv.second.ms);
        first = false;
    }
    fprintf(fp, "\n]}\n");
    const bool ok = fclose(fp) == 0;
    return ok && rename(tmp.c_str(), ctx->tune_path.c_str()) == 0;
}

// Value of "name": <number> inside one JSON object of the cache file.
bool json_number(const std::string& obj, const char* name, double* v) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t at = obj.find(pat);
    if (at == std::string::npos) return false;
    const char* b = obj.c_str() + at + pat.size();
    char* e = nullptr;
    *v = strtod(b, &e);
    return e != b;
}

// Load the entries of a cache file written by save_tune_cache; entries that
// do not parse or hold an invalid plan are skipped.
void load_tune_cache(knnf_ctx* ctx) {
    FILE* fp = fopen(ctx->tune_path.c_str(), "r");
    if (!fp) return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, got);
    fclose(fp);
    size_t pos = 0;
    for (;;) {
        const size_t k = text.find("{\"key\": \"", pos);
        if (k == std::string::npos) break;
        const size_t ks = k + 9, ke = text.find('"', ks), oe = text.find('}', ks);
        if (ke == std::string::npos || oe == std::string::npos || ke > oe) break;
        const std::string key = text.substr(ks, ke - ks);
        const std::string obj = text.substr(ke, oe - ke);
        pos = oe + 1;
        double v[7];
        static const char* names[7] = {"search", "tile_rows", "tile_cols", "waves",
                                       "launch", "chunk_rows", "ms"};
        bool ok = true;
        for (int t = 0; t < 7; ++t) ok = ok && json_number(obj, names[t], &v[t]);
        if (!ok) continue;
        TunedPlan tp;
        tp.plan.search = (int32_t)v[0];
        tp.plan.tile_rows = (int32_t)v[1];
        tp.plan.tile_cols = (int32_t)v[2];
        tp.plan.waves = (int32_t)v[3];
        tp.plan.launch = (int32_t)v[4];
        tp.plan.chunk_rows = (int32_t)v[5];
        tp.plan.flags = 0;
        tp.ms = v[6];
        if (plan_ok_impl(tp.plan)) ctx->tuned[key] = tp;
    }
}

// ---- non-finite input check -------------------------------------------------

// Waits for `stream`, then reports whether the check launched with `gen`
// found a non-finite value.
knnf_status check_result(knnf_ctx* ctx, uint32_t gen, hipStream_t stream) {
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return ctx_fail(ctx, e, "input check");
    if (__atomic_load_n(ctx->check_host + gen % kCheckSlots, __ATOMIC_ACQUIRE) == gen)
        return fail(KNNF_EINVAL, "non-finite value in the pc1 or prob input");
    return KNNF_OK;
}

uint32_t next_check_gen(knnf_ctx* ctx) {
    uint32_t g = ctx->check_gen.fetch_add(1) + 1;
    return g ? g : 1;  // flags start at 0
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
knnf_status ctx_status(const knnf_ctx* ctx) { return ctx_check(ctx); }
void ctx_mark_failed(knnf_ctx* ctx, const char* what) {
    int expect = 0;
    if (ctx->failed.compare_exchange_strong(expect, 1))
        snprintf(ctx->failed_msg, sizeof ctx->failed_msg, "%s", what);
}

knnf_status launch_items(knnf_ctx* ctx, const WorkItem* items, int n, const knnf_plan& p,
                         void* stream) {
    knnf_status cs = ctx_check(ctx);
    if (cs != KNNF_OK) return cs;
    uint64_t total = 0;
    uint64_t max_words = 0;
    for (int k = 0; k < n; ++k) {
        total += items[k].ntiles;
        if (total > 0xfff00000ull) return fail(KNNF_EINVAL, "batched launch: too much work");
        const FrameDesc& f = items[k].f;
        max_words = std::max<uint64_t>(max_words, (uint64_t)f.H * (uint64_t)f.W * (uint64_t)(f.C + 1));
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
        if (e != hipSuccess) return ctx_fail(ctx, e, "batch slot wait");
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
        if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "batch table write");
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
            if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "batch table write");
        } else {
            e = hipMemcpyAsync(s.dev, s.host, off_counter(s.cap), hipMemcpyHostToDevice, hs);
            if (e != hipSuccess) return ctx_fail(ctx, e, "batch table copy");
        }
    }
    if (!(p.flags & KNNF_PLAN_NO_INPUT_CHECK)) {
        // validation of the input values: one pass over every frame through
        // the table just written, then wait; nothing is launched on failure
        const uint32_t gen = next_check_gen(ctx);
        const int rc = knnf::launch_check_items((const knnf::FrameDesc*)s.dev, (uint32_t)n,
                                                (uint32_t)std::min<uint64_t>(max_words, 0xffffffffu),
                                                ctx->check_dev + gen % kCheckSlots, gen, stream);
        if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "input check launch");
        const knnf_status st = check_result(ctx, gen, hs);
        if (st != KNNF_OK) return st;
    }
    uint32_t* d_ctr = (uint32_t*)((char*)s.dev + off_counter(s.cap));
    const knnf::LaunchCfg cfg = to_cfg(p);
    int rc;
    if (!cfg.persistent) {
        rc = knnf::launch_filter_items((const knnf::FrameDesc*)s.dev,
                                       (const uint32_t*)((char*)s.dev + off_task_start(s.cap)),
                                       (const uint32_t*)((char*)s.dev + off_tile_base(s.cap)),
                                       (uint32_t)n, (uint32_t)total, cfg, stream);
        if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "batched launch");
        e = hipEventRecord(s.done, hs);
        if (e != hipSuccess) return ctx_fail(ctx, e, "batch slot record");
        s.recorded = true;
        return KNNF_OK;
    }
    rc = knnf::launch_zero_counter(d_ctr, stream);
    if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "counter reset");
    const uint64_t need_blocks = (total + p.waves - 1) / p.waves;
    const int per_cu = knnf::persistent_blocks_per_cu(cfg);
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(need_blocks,
                                                  (uint64_t)ctx->num_cu * per_cu));
    rc = knnf::launch_filter_batch((const knnf::FrameDesc*)s.dev,
                                   (const uint32_t*)((char*)s.dev + off_task_start(s.cap)),
                                   (const uint32_t*)((char*)s.dev + off_tile_base(s.cap)),
                                   (uint32_t)n, (uint32_t)total, d_ctr, cfg, (int)grid, stream);
    if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "batched launch");
    e = hipEventRecord(s.done, hs);
    if (e != hipSuccess) return ctx_fail(ctx, e, "batch slot record");
    s.recorded = true;
    return KNNF_OK;
}

}  // namespace knnf

extern "C" {

const char* knnf_last_error(void) { return g_err.c_str(); }

const char* knnf_version(void) { return "knnf 0.2.0 gfx950"; }

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
    if (e != hipSuccess) return hip_fail(e, "knnf_create: hipGetDeviceCount");
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
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c->check_host, kCheckSlots * sizeof(uint32_t),
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        std::memset(c->check_host, 0, kCheckSlots * sizeof(uint32_t));
        e = hipHostGetDevicePointer((void**)&c->check_dev, c->check_host, 0);
    }
    if (e == hipSuccess) e = (hipError_t)knnf::pc1_scratch_init(device, &c->pc1_scratch);
    hipSetDevice(prev);
    if (e != hipSuccess) {
        knnf_destroy(c);
        return hip_fail(e, "knnf_create: workspace");
    }
    if (const char* path = getenv("KNNF_TUNE_CACHE")) {
        c->tune_path = path;
        load_tune_cache(c);
    }
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
    if (ctx->pc1_ws || ctx->check_host) hipDeviceSynchronize();
    if (ctx->pc1_ws) hipFree(ctx->pc1_ws);
    if (ctx->check_host) hipHostFree(ctx->check_host);
    hipSetDevice(prev);
    delete ctx;
    return KNNF_OK;
}

knnf_status knnf_ctx_status(const knnf_ctx* ctx) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_ctx_status: NULL context");
    return ctx_check(ctx);
}

knnf_status knnf_inject_fault(knnf_ctx* ctx) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_inject_fault: NULL context");
    knnf::ctx_mark_failed(ctx, "fault injected by knnf_inject_fault");
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
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    st = validate_impl(frame, 0);
    if (st != KNNF_OK) return st;
    knnf_plan p;
    if (plan || !tuned_plan(ctx, frame, 1, &p)) p = resolve_impl(ctx, plan);
    if (!plan_ok_impl(p)) return fail(KNNF_EINVAL, "knnf_filter: invalid plan");
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};
    knnf::FrameDesc desc = to_desc_impl(*frame);
    if (!(p.flags & KNNF_PLAN_NO_INPUT_CHECK)) {
        const uint32_t gen = next_check_gen(ctx);
        const int rc = knnf::launch_check_frame(desc, ctx->check_dev + gen % kCheckSlots, gen, stream);
        if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "input check launch");
        st = check_result(ctx, gen, (hipStream_t)stream);
        if (st != KNNF_OK) return st;
    }
    desc.stats = ctx->stats_on ? ctx->d_stats : nullptr;
    // lambda = 0 under the pruned search: the 1-D selection (work counters not kept)
    const int e = p.search == KNNF_SEARCH_PRUNED && knnf::spectral_fits(desc)
                      ? knnf::launch_spectral_frame(desc, stream)
                      : knnf::launch_filter_frame(desc, to_cfg(p), stream);
    if (e != 0) return ctx_fail(ctx, (hipError_t)e, "knnf_filter launch");
    return KNNF_OK;
}

knnf_status knnf_filter_batch(knnf_ctx* ctx, const knnf_frame* frames, int n,
                              const knnf_plan* plan, void* stream) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_filter_batch: NULL context");
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    if (n < 0 || (n > 0 && !frames)) return fail(KNNF_EINVAL, "knnf_filter_batch: bad frame list");
    if (n == 0) return KNNF_OK;
    for (int i = 0; i < n; ++i) {
        st = validate_impl(&frames[i], i);
        if (st != KNNF_OK) return st;
    }
    knnf_plan p;
    if (plan || !tuned_plan(ctx, frames, n, &p)) p = resolve_impl(ctx, plan);
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
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
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
        if (e != hipSuccess) return ctx_fail(ctx, e, "knnf_pc1: synchronize");
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
    if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "knnf_pc1 launch");
    return KNNF_OK;
}

knnf_status knnf_pc1_noalloc(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                             const double* mean, const double* vec, float* out,
                             int32_t normalize, void* stream) {
    if (npix < 1 || npix > KNNF_PC1_MAX_PIXELS)
        return fail(KNNF_EINVAL, "knnf_pc1_noalloc: npix %lld outside [1, 2^40]", (long long)npix);
    if (normalize && npix > KNNF_PC1_NOALLOC_MAX_PIXELS)
        return fail(KNNF_EINVAL, "knnf_pc1_noalloc: npix %lld exceeds the static scratch (%d pixels)",
                    (long long)npix, KNNF_PC1_NOALLOC_MAX_PIXELS);
    if (bands < 1 || bands > KNNF_PC1_MAX_BANDS)
        return fail(KNNF_EINVAL, "knnf_pc1_noalloc: bands %d outside [1, %d]", bands,
                    KNNF_PC1_MAX_BANDS);
    if (!cube || !mean || !vec || !out) return fail(KNNF_EINVAL, "knnf_pc1_noalloc: NULL pointer");
    if (!ctx) return fail(KNNF_EINVAL, "knnf_pc1_noalloc: NULL context");
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};
    // the scratch's device address from context creation, never the array's name
    char* base = (char*)ctx->pc1_scratch;
    double* pairs = (double*)base;
    double* ws = normalize ? (double*)(base + knnf::pc1_scratch_head()) : nullptr;
    const int rc = knnf::launch_pc1(cube, npix, bands, mean, vec, out, ws, pairs, ctx->num_cu,
                                    stream);
    if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "knnf_pc1_noalloc launch");
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
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};
    const int rc = knnf::launch_svm(cube, npix, bands, classes, w, bias, A, B, out, stream);
    if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "knnf_svm launch");
    return KNNF_OK;
}

knnf_status knnf_svm_pc1(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                         int32_t classes, const double* w, const double* bias, const double* A,
                         const double* B, const double* mean, const double* vec, float* out_prob,
                         float* out_band, int32_t normalize, void* stream) {
    if (npix < 1 || npix > KNNF_SVM_MAX_PIXELS)
        return fail(KNNF_EINVAL, "knnf_svm_pc1: npix %lld outside [1, 2^31]", (long long)npix);
    if (bands < 1 || bands > KNNF_SVM_MAX_BANDS)
        return fail(KNNF_EINVAL, "knnf_svm_pc1: bands %d outside [1, %d]", bands, KNNF_SVM_MAX_BANDS);
    if (classes < 2 || classes > KNNF_SVM_MAX_CLASSES)
        return fail(KNNF_EINVAL, "knnf_svm_pc1: classes %d outside [2, %d]", classes,
                    KNNF_SVM_MAX_CLASSES);
    if (!cube || !w || !bias || !A || !B || !mean || !vec || !out_prob || !out_band)
        return fail(KNNF_EINVAL, "knnf_svm_pc1: NULL pointer");
    if (!ctx) return fail(KNNF_EINVAL, "knnf_svm_pc1: NULL context");
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    std::lock_guard<std::mutex> lock(ctx->mu);
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    struct Restore {
        int prev, dev;
        ~Restore() { if (prev != dev) hipSetDevice(prev); }
    } restore{prev, ctx->device};
    double* pairs = nullptr;
    double* ws = nullptr;
    if (normalize) {
        // workspace: one (min, max) pair per kernel block, then the binary64
        // projection (shared with knnf_pc1; grows like it)
        const int64_t nb = (npix + knnf::svm_pixels_per_block() - 1) / knnf::svm_pixels_per_block();
        const size_t head = ((size_t)nb * 2 * sizeof(double) + 255) & ~size_t(255);
        const size_t need = head + (size_t)npix * sizeof(double);
        if (ctx->pc1_ws_bytes < need) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return ctx_fail(ctx, e, "knnf_svm_pc1: synchronize");
            const size_t bytes = std::max(need, ctx->pc1_ws_bytes * 2);
            if (ctx->pc1_ws) hipFree(ctx->pc1_ws);
            ctx->pc1_ws = nullptr;
            ctx->pc1_ws_bytes = 0;
            e = hipMalloc((void**)&ctx->pc1_ws, bytes);
            if (e != hipSuccess)
                return fail(KNNF_ENOMEM, "knnf_svm_pc1 workspace: %s", hipGetErrorString(e));
            ctx->pc1_ws_bytes = bytes;
        }
        pairs = (double*)ctx->pc1_ws;
        ws = (double*)(ctx->pc1_ws + head);
    }
    int nblocks = 0;
    int rc = knnf::launch_svm_pc1(cube, npix, bands, classes, w, bias, A, B, mean, vec, out_prob,
                                  out_band, ws, pairs, &nblocks, stream);
    if (rc == 0 && normalize)
        rc = knnf::launch_pc1_normalise(ws, npix, pairs, nblocks, out_band, ctx->num_cu, stream);
    if (rc != 0) return ctx_fail(ctx, (hipError_t)rc, "knnf_svm_pc1 launch");
    return KNNF_OK;
}

knnf_status knnf_stats_enable(knnf_ctx* ctx, int on) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_stats_enable: NULL context");
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
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
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    if (!ctx->d_stats) return KNNF_OK;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h, ctx->d_stats, sizeof h, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) e = hipMemset(ctx->d_stats, 0, sizeof h);
    hipSetDevice(prev);
    if (e != hipSuccess) return ctx_fail(ctx, e, "knnf_stats_read");
    *pairs = h[0];
    *tiles = h[1];
    return KNNF_OK;
}

knnf_status knnf_tune(knnf_ctx* ctx, const knnf_frame* frames, int n, int reps, void* stream,
                      knnf_plan* best) {
    if (!ctx) return fail(KNNF_EINVAL, "knnf_tune: NULL context");
    knnf_status st = ctx_check(ctx);
    if (st != KNNF_OK) return st;
    if (n < 1 || !frames || reps < 1) return fail(KNNF_EINVAL, "knnf_tune: bad arguments");
    for (int i = 0; i < n; ++i) {
        st = validate_impl(&frames[i], i);
        if (st != KNNF_OK) return st;
    }
    static const int ws[] = {1, 2, 4};
    static const int ss[] = {KNNF_SEARCH_EXHAUSTIVE, KNNF_SEARCH_PRUNED};
    static const int ls[] = {KNNF_LAUNCH_PERSISTENT, KNNF_LAUNCH_GRID};
    static const int chunks[] = {8, 16, 32};
    hipStream_t hs = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return ctx_fail(ctx, he, "knnf_tune: event create");
    }
    float best_ms = 1e30f;
    knnf_plan bp = ctx->plan;
    knnf_status result = KNNF_OK;
    for (int s : ss)
        for (const auto& sh : kShapes)
            for (int w : ws)
                for (int l : ls)
                    for (int ch : chunks) {
                        if (n == 1 && l == KNNF_LAUNCH_PERSISTENT) continue;  // single frames ignore it
                        if (s == KNNF_SEARCH_EXHAUSTIVE && ch != 16) continue;  // no window chunk there
                        knnf_plan p{};
                        p.search = s;
                        p.tile_rows = sh[0];
                        p.tile_cols = sh[1];
                        p.waves = w;
                        p.launch = l;
                        p.chunk_rows = ch;
                        p.flags = KNNF_PLAN_NO_INPUT_CHECK;  // time the filter alone
                        if (!plan_ok_impl(p)) continue;
                        auto run = [&]() -> knnf_status {
                            return n == 1 ? knnf_filter(ctx, frames, &p, stream)
                                          : knnf_filter_batch(ctx, frames, n, &p, stream);
                        };
                        knnf_status rs = run();  // warm-up
                        if (rs != KNNF_OK) { result = rs; goto done; }
                        hipEventRecord(e0, hs);
                        for (int r = 0; r < reps && rs == KNNF_OK; ++r) rs = run();
                        hipEventRecord(e1, hs);
                        if (rs != KNNF_OK) { result = rs; goto done; }
                        he = hipEventSynchronize(e1);
                        if (he != hipSuccess) {
                            result = ctx_fail(ctx, he, "knnf_tune: synchronize");
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
    bp.flags = 0;
    if (best) *best = bp;
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    TunedPlan tp;
    tp.plan = bp;
    tp.ms = best_ms / reps;
    ctx->tuned[tune_key(frames, n)] = tp;
    if (!save_tune_cache(ctx))
        return fail(KNNF_EINVAL, "knnf_tune: cannot write the tune cache %s", ctx->tune_path.c_str());
    return KNNF_OK;
}

knnf_status knnf_tune_lookup(const knnf_ctx* ctx, const knnf_frame* frames, int n, knnf_plan* plan) {
    if (!ctx || !frames || n < 1 || !plan) return fail(KNNF_EINVAL, "knnf_tune_lookup: bad arguments");
    for (int i = 0; i < n; ++i) {
        const knnf_status st = validate_impl(&frames[i], i);
        if (st != KNNF_OK) return st;
    }
    if (tuned_plan(ctx, frames, n, plan)) return KNNF_OK;
    *plan = ctx->plan;
    return fail(KNNF_ESTATE, "knnf_tune_lookup: no plan cached for these frames");
}

}  // extern "C"
