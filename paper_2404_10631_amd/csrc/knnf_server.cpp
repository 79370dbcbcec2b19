// knnf_server.cpp -- continuous-batching server behind the knnf_server_* C-ABI.
//
// Frames arrive from the host at any time.  A scheduler thread
//   1. admits queued frames in arrival order while the caller's device pool
//      has room (first-fit sub-allocation; the head of the queue is never
//      overtaken, so no frame starves) and hands them to a copier thread,
//      which enqueues the copies of their inputs on a copy stream (a copy
//      call can hold its thread for milliseconds when the copy stream is
//      backed up; the scheduler keeps launching and reaping meanwhile);
//   2. builds GPU steps: one batched launch over tile ranges of all admitted
//      frames in arrival order, up to a tile budget, so a large frame is
//      processed in slices and later arrivals join the next step (a lone
//      frame with nothing waiting runs whole); up to `max_inflight` steps are
//      queued on separate compute streams, each waiting for the input copy of
//      every frame it touches;
//   3. watches step completion events and marks a frame done when the last
//      step holding its tiles has finished.
// In plain mode each step is one whole frame, launched alone (the baseline).
//
// Tracing: every frame carries one roctx range per serving stage, named
// "knnf frame <ticket> <H>x<W> <stage>" with the stages "queued" (submitted,
// waiting for pool memory), "ready" (admitted: inputs copying, waiting for a
// step) and "on gpu" (first tile launched until its last step completes);
// the host calls that enqueue input copies and launch steps are pushed as
// "knnf h2d enqueue" and "knnf step" ranges on the calling thread.
// rocprofv3 --marker-trace records them; without a tool attached they cost
// a call into an empty dispatch table.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/knnf.h"
#include "knnf_device.h"
#include "knnf_internal.h"

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class PoolAllocator {
   public:
    explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }

   private:
    size_t size_;
    std::map<size_t, size_t> free_;
};

enum JobState { QUEUED, COPYING, ADMITTED, DONE, RELEASED };

struct Job {
    uint64_t ticket = 0;
    knnf_host_frame hf{};
    JobState state = QUEUED;
    size_t off = 0, bytes = 0;
    knnf_frame dev{};
    uint32_t ntiles = 0, next_tile = 0;
    int outstanding = 0;          // launched steps holding tiles of this job
    uint32_t waited = 0;          // compute streams (bit per step slot) told to wait for its copy
    hipEvent_t copied = nullptr;  // inputs are in the pool
    const void* map_pc1 = nullptr;   // device views of small pinned inputs (else null)
    const void* map_prob = nullptr;
    double t_arrival = 0, t_admit = 0, t_launch = -1, t_done = 0;
    roctx_range_id_t span = 0;  // roctx range of the current serving stage
    bool span_open = false;
};

// Ends the frame's current stage range and, if `stage` is given, opens the next.
void stage(Job& j, const char* stage) {
    if (j.span_open) roctxRangeStop(j.span);
    j.span_open = false;
    if (!stage) return;
    char name[96];
    std::snprintf(name, sizeof name, "knnf frame %llu %dx%d %s", (unsigned long long)j.ticket,
                  j.hf.H, j.hf.W, stage);
    j.span = roctxRangeStartA(name);
    j.span_open = true;
}

struct Step {
    hipEvent_t done = nullptr;
    hipStream_t stream = nullptr;
    bool active = false;
    std::vector<uint64_t> tickets;  // jobs with tiles in this step
};

}  // namespace

struct knnf_server {
    knnf_ctx* ctx = nullptr;
    int device = 0;
    char* pool = nullptr;
    knnf_server_opts opts{};
    knnf_plan plan{};
    PoolAllocator alloc{0};
    hipStream_t copy_stream = nullptr;
    std::vector<Step> steps;
    std::vector<hipEvent_t> event_pool;

    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<uint64_t, Job> jobs;
    std::deque<uint64_t> queue;   // submitted, not admitted
    std::deque<uint64_t> copyq;   // granted pool memory, copies not yet enqueued
    std::deque<uint64_t> ready;   // admitted, tiles left to launch
    std::condition_variable copy_cv;
    bool copier_busy = false;     // the copier is enqueueing a frame's copies
    uint64_t next_ticket = 1;
    size_t unfinished = 0;
    std::atomic<bool> stop{false};
    std::thread thread;
    std::thread copier;
    knnf_status sticky = KNNF_OK;
    bool check_inputs = true;   // reject non-finite host inputs at submission

    explicit knnf_server(size_t pool_bytes) : alloc(pool_bytes) {}
};

namespace {

// In batched mode, while the copy stream is backed up, inputs that sit in
// pinned, device-mapped host memory are copied by a kernel on the copy
// stream: a host-to-device copy call then sometimes held its thread for
// 7-11 ms, and every frame queued behind it waited as long.  A kernel reads
// mapped host memory as fast as the copy engine (57 GB/s); an idle copy
// stream keeps the copy engine, whose latency is lower.  The plain baseline
// always uses the copy engine.  (Bound: the copy kernel counts words in 32
// bits.)
constexpr size_t kKernelCopyMax = 1u << 30;

// Device address of pinned host memory at p, or null if the runtime does not
// report p as device-mapped host memory.
const void* device_view(const void* p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // not registered: leave no error behind
        return nullptr;
    }
    if (a.type != hipMemoryTypeHost || !a.devicePointer || !a.hostPointer) return nullptr;
    return (const char*)a.devicePointer + ((const char*)p - (const char*)a.hostPointer);
}

hipEvent_t take_event(knnf_server* s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// A HIP call of the server failed: the server and its context stay failed.
void server_fail(knnf_server* s, const char* what) {
    s->sticky = KNNF_EDEVICE;
    knnf::ctx_mark_failed(s->ctx, what);
}

// Any NaN or infinity among n binary32 values (exponent bits all ones).
bool has_nonfinite(const float* v, size_t n) {
    const uint32_t* w = (const uint32_t*)v;
    uint32_t bad = 0;
    for (size_t k = 0; k < n; ++k) bad |= ((w[k] & 0x7f800000u) == 0x7f800000u);
    return bad != 0;
}

// Lay out a frame in the pool: inputs, then outputs, 256-byte aligned.
void place(Job& j, char* base) {
    const size_t px = (size_t)j.hf.H * (size_t)j.hf.W;
    size_t o = j.off;
    auto put = [&](size_t bytes) {
        char* p = base + o;
        o += round256(bytes);
        return p;
    };
    knnf_frame& d = j.dev;
    d.H = j.hf.H;
    d.W = j.hf.W;
    d.C = j.hf.C;
    d.K = j.hf.K;
    d.R = j.hf.R;
    d.lambda = j.hf.lambda;
    d.pc1 = (const float*)put(px * 4);
    d.prob = (const float*)put(px * j.hf.C * 4);
    d.out_prob = (float*)put(px * j.hf.C * 4);
    d.out_class = (int32_t*)put(px * 4);
    d.out_nbr = j.hf.with_nbr ? (int32_t*)put(px * j.hf.K * 4) : nullptr;
    d.out_dist = j.hf.with_nbr ? (float*)put(px * j.hf.K * 4) : nullptr;
}

bool copy_stream_idle(knnf_server* s) {
    const bool idle = hipStreamQuery(s->copy_stream) == hipSuccess;
    (void)hipGetLastError();  // "not ready" is an answer, not an error
    return idle;
}

// Enqueue a frame's input copies and the event marking their end.
hipError_t enqueue_copies(knnf_server* s, void* d1, const void* h1, size_t n1, void* d2,
                          const void* h2, size_t n2, hipEvent_t ev) {
    hipError_t e = ev ? hipSuccess : hipErrorOutOfMemory;
    roctxRangePushA("knnf h2d enqueue");
    if (e == hipSuccess) e = hipMemcpyAsync(d1, h1, n1, hipMemcpyHostToDevice, s->copy_stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d2, h2, n2, hipMemcpyHostToDevice, s->copy_stream);
    if (e == hipSuccess) e = hipEventRecord(ev, s->copy_stream);
    roctxRangePop();
    return e;
}

// Admission: FIFO while the pool has room.  With no copy pending anywhere the
// scheduler enqueues the frame's copies itself (the lowest latency); otherwise
// the frame goes to the copier thread.  Called with the lock held.
void admit(knnf_server* s) {
    while (!s->queue.empty()) {
        Job& j = s->jobs[s->queue.front()];
        size_t off = 0;
        if (!s->alloc.alloc(j.bytes, &off)) return;
        j.off = off;
        place(j, s->pool);
        j.ntiles = knnf::tiles_of(j.hf.H, j.hf.W, s->plan);
        s->queue.pop_front();
        if (s->copyq.empty() && !s->copier_busy && copy_stream_idle(s)) {
            const size_t px = (size_t)j.hf.H * (size_t)j.hf.W;
            j.copied = take_event(s);
            const hipError_t e =
                enqueue_copies(s, (void*)j.dev.pc1, j.hf.pc1, px * 4, (void*)j.dev.prob, j.hf.prob,
                               px * (size_t)j.hf.C * 4, j.copied);
            if (e != hipSuccess) {
                server_fail(s, "server: input copy");
                return;
            }
            j.state = ADMITTED;
            j.t_admit = now_s();
            stage(j, "ready");
            s->ready.push_back(j.ticket);
        } else {
            j.state = COPYING;
            s->copyq.push_back(j.ticket);
            s->copy_cv.notify_one();
        }
    }
}

// Copier thread: enqueues each admitted frame's input copies and the event
// marking their end, without the lock held, then makes the frame ready.
void copier(knnf_server* s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->copy_cv.wait(lk, [s] { return s->stop.load() || !s->copyq.empty(); });
        if (s->stop.load()) return;
        const uint64_t tk = s->copyq.front();
        s->copyq.pop_front();
        s->copier_busy = true;
        hipEvent_t ev = take_event(s);
        const Job& jc = s->jobs[tk];  // not erased before DONE
        const size_t px = (size_t)jc.hf.H * (size_t)jc.hf.W;
        void* d1 = (void*)jc.dev.pc1;
        void* d2 = (void*)jc.dev.prob;
        const void* h1 = jc.hf.pc1;
        const void* h2 = jc.hf.prob;
        const void* m1 = jc.map_pc1;
        const void* m2 = jc.map_prob;
        const size_t n1 = px * 4, n2 = px * (size_t)jc.hf.C * 4;
        lk.unlock();
        hipError_t e;
        if (ev && m1 && m2 && !copy_stream_idle(s)) {
            roctxRangePushA("knnf h2d enqueue");
            e = (hipError_t)knnf::launch_copy_pair((const uint32_t*)m1, (uint32_t*)d1,
                                                   (uint32_t)(n1 / 4), (const uint32_t*)m2,
                                                   (uint32_t*)d2, (uint32_t)(n2 / 4), s->copy_stream);
            if (e == hipSuccess) e = hipEventRecord(ev, s->copy_stream);
            roctxRangePop();
        } else {
            e = enqueue_copies(s, d1, h1, n1, d2, h2, n2, ev);
        }
        lk.lock();
        s->copier_busy = false;
        if (e != hipSuccess) {
            // the frame never becomes ready; polls and drain report the error
            server_fail(s, "server: input copy");
            if (ev) s->event_pool.push_back(ev);
            continue;
        }
        Job& j = s->jobs[tk];
        j.copied = ev;
        j.state = ADMITTED;
        j.t_admit = now_s();
        stage(j, "ready");
        s->ready.push_back(tk);
        s->cv.notify_one();
    }
}

void finish_job(knnf_server* s, Job& j, double t) {
    j.state = DONE;
    j.t_done = t;
    stage(j, nullptr);
    if (j.copied) {
        s->event_pool.push_back(j.copied);
        j.copied = nullptr;
    }
    --s->unfinished;
}

// Completion of queued steps.  Called with the lock held.
bool reap(knnf_server* s) {
    bool any = false;
    for (Step& st : s->steps) {
        if (!st.active) continue;
        const hipError_t q = hipEventQuery(st.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) server_fail(s, "server: step completion");
        const double t = now_s();
        for (uint64_t tk : st.tickets) {
            Job& j = s->jobs[tk];
            if (--j.outstanding == 0 && j.next_tile == j.ntiles) finish_job(s, j, t);
        }
        st.tickets.clear();
        st.active = false;
        any = true;
    }
    return any;
}

// Build and enqueue one step on a free stream.  Called with the lock held.
bool launch_step(knnf_server* s) {
    if (s->ready.empty()) return false;
    Step* st = nullptr;
    for (Step& x : s->steps)
        if (!x.active) {
            st = &x;
            break;
        }
    if (!st) return false;
    const bool plain = s->opts.mode == KNNF_SERVE_PLAIN;
    std::vector<knnf::WorkItem> items;
    uint64_t budget = plain ? ~0ull : (uint64_t)s->opts.step_tiles;
    // an idle server (one frame ready, nothing waiting for admission) runs it
    // whole: slicing only helps frames that arrive behind it, and those still
    // start at once on the other stream
    if (s->ready.size() == 1 && s->queue.empty()) budget = ~0ull;
    while (!s->ready.empty() && budget > 0) {
        Job& j = s->jobs[s->ready.front()];
        const uint32_t left = j.ntiles - j.next_tile;
        const uint32_t take = (uint32_t)std::min<uint64_t>(left, budget);
        // a frame split over several steps may run on several streams: each
        // of them waits for the copy of its inputs before its first tile
        const uint32_t sbit = 1u << (uint32_t)(st - s->steps.data());
        if (!(j.waited & sbit)) {
            if (hipStreamWaitEvent(st->stream, j.copied, 0) != hipSuccess)
                server_fail(s, "server: stream wait");
            j.waited |= sbit;
        }
        knnf::WorkItem w;
        w.f = knnf::desc_of(j.dev);
        w.tile0 = j.next_tile;
        w.ntiles = take;
        items.push_back(w);
        j.next_tile += take;
        ++j.outstanding;
        if (j.t_launch < 0) {
            j.t_launch = now_s();
            stage(j, "on gpu");
        }
        st->tickets.push_back(j.ticket);
        budget -= take;
        if (j.next_tile == j.ntiles) s->ready.pop_front();
        if (plain) break;
    }
    knnf_status rc;
    roctxRangePushA("knnf step");
    if (plain || (items.size() == 1 && items[0].tile0 == 0 &&
                  items[0].ntiles == s->jobs[st->tickets[0]].ntiles)) {
        // one whole frame: the single-frame launch (no work table to copy)
        rc = knnf_filter(s->ctx, &s->jobs[st->tickets[0]].dev, &s->plan, st->stream);
    } else {
        rc = knnf::launch_items(s->ctx, items.data(), (int)items.size(), s->plan, st->stream);
    }
    roctxRangePop();
    if (rc == KNNF_EDEVICE || hipEventRecord(st->done, st->stream) != hipSuccess)
        server_fail(s, "server: step launch");
    else if (rc != KNNF_OK)
        s->sticky = rc;
    st->active = true;
    return true;
}

void scheduler(knnf_server* s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop.load()) {
        bool progress = reap(s);
        admit(s);
        while (launch_step(s)) progress = true;
        if (!progress) {
            // Nothing completed or launched: wait briefly for a submission or
            // for GPU progress (completion is observed by polling events).
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        } else {
            // let the copier and the caller's polls take the lock in between
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

double knnf_server_clock(void) { return now_s(); }

knnf_status knnf_server_create(knnf_server** out, knnf_ctx* ctx, void* pool, size_t pool_bytes,
                               const knnf_server_opts* opts) {
    if (!out || !ctx || !pool || pool_bytes < 4096)
        return knnf::set_error(KNNF_EINVAL, "knnf_server_create: bad arguments");
    const knnf_status cs = knnf::ctx_status(ctx);
    if (cs != KNNF_OK) return cs;
    if ((uintptr_t)pool & 255)
        return knnf::set_error(KNNF_EINVAL, "knnf_server_create: pool not 256-byte aligned");
    *out = nullptr;
    knnf_server_opts o{};
    if (opts) o = *opts;
    if (o.mode != KNNF_SERVE_BATCHED && o.mode != KNNF_SERVE_PLAIN)
        return knnf::set_error(KNNF_EINVAL, "knnf_server_create: bad mode");
    if (o.max_queue <= 0) o.max_queue = 4096;
    if (o.max_inflight <= 0) o.max_inflight = 2;
    if (o.max_inflight > 4) return knnf::set_error(KNNF_EINVAL, "max_inflight above 4");
    if (o.step_tiles <= 0) o.step_tiles = 32768;
    if (o.mode == KNNF_SERVE_PLAIN) o.max_inflight = 1;
    // steps are bounded slices of work: one wavefront per task (the hardware
    // dispatcher balances it) unless the caller asks otherwise
    if (o.plan.launch == KNNF_LAUNCH_DEFAULT) o.plan.launch = KNNF_LAUNCH_GRID;
    const knnf_plan p = knnf::resolve_plan(ctx, &o.plan);
    if (!knnf::plan_valid(p)) return knnf::set_error(KNNF_EINVAL, "knnf_server_create: bad plan");

    knnf_server* s = new (std::nothrow) knnf_server(pool_bytes);
    if (!s) return knnf::set_error(KNNF_ENOMEM, "knnf_server_create: out of host memory");
    s->ctx = ctx;
    s->device = knnf::ctx_device(ctx);
    s->pool = (char*)pool;
    s->opts = o;
    s->plan = p;
    // server frames are checked on the host at submission (the device check
    // would make every step synchronous)
    s->check_inputs = !(p.flags & KNNF_PLAN_NO_INPUT_CHECK);
    s->plan.flags |= KNNF_PLAN_NO_INPUT_CHECK;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(s->device);
    bool ok = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) == hipSuccess;
    s->steps.resize(o.max_inflight);
    for (Step& st : s->steps) {
        ok = ok && hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) == hipSuccess;
    }
    // Warm every stream: HIP sets up a stream's hardware queue and its copy
    // path from pinned host memory on first use, which took about 6 ms each
    // and delayed the first frames a new server admitted.  The warm-up copies
    // one zero word from a pinned buffer to the start of the pool (which
    // holds no frame yet) and launches one tiny kernel per compute stream.
    if (ok) {
        uint32_t* zero = nullptr;
        ok = hipHostMalloc((void**)&zero, 256, hipHostMallocDefault) == hipSuccess;
        if (ok) {
            *zero = 0;
            ok = hipMemcpyAsync(s->pool, zero, sizeof *zero, hipMemcpyHostToDevice,
                                s->copy_stream) == hipSuccess &&
                 hipStreamSynchronize(s->copy_stream) == hipSuccess;
            hipHostFree(zero);
        }
        for (Step& st : s->steps) {
            ok = ok && knnf::launch_zero_counter((uint32_t*)s->pool, st.stream) == 0 &&
                 hipStreamSynchronize(st.stream) == hipSuccess;
        }
    }
    hipSetDevice(prev);
    if (!ok) {
        knnf_server_destroy(s);
        return knnf::set_error(KNNF_EDEVICE, "knnf_server_create: stream setup failed");
    }
    s->thread = std::thread(scheduler, s);
    s->copier = std::thread(copier, s);
    *out = s;
    return KNNF_OK;
}

knnf_status knnf_server_submit(knnf_server* s, const knnf_host_frame* f, uint64_t* ticket) {
    if (!s || !f || !ticket) return knnf::set_error(KNNF_EINVAL, "knnf_server_submit: NULL argument");
    knnf_frame v{};
    v.H = f->H;
    v.W = f->W;
    v.C = f->C;
    v.K = f->K;
    v.R = f->R;
    v.lambda = f->lambda;
    v.pc1 = f->pc1;
    v.prob = f->prob;
    v.out_prob = (float*)1;    // placed in the pool on admission
    v.out_class = (int32_t*)1;
    knnf_status st = knnf::validate_frame(&v, 0);
    if (st != KNNF_OK) return st;
    st = knnf::ctx_status(s->ctx);
    if (st != KNNF_OK) return st;
    if (s->check_inputs) {
        const size_t px = (size_t)f->H * (size_t)f->W;
        if (has_nonfinite(f->pc1, px) || has_nonfinite(f->prob, px * (size_t)f->C))
            return knnf::set_error(KNNF_EINVAL, "non-finite value in the pc1 or prob input");
    }
    const size_t bytes = knnf_frame_bytes(f->H, f->W, f->C, f->K, f->with_nbr ? 1 : 0);
    const void* m1 = nullptr;
    const void* m2 = nullptr;
    if (s->opts.mode == KNNF_SERVE_BATCHED &&
        (size_t)f->H * (size_t)f->W * (size_t)(f->C + 1) * 4 <= kKernelCopyMax) {
        m1 = device_view(f->pc1);
        m2 = device_view(f->prob);
        if (!m1 || !m2) m1 = m2 = nullptr;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != KNNF_OK) return knnf::set_error(s->sticky, "server failed earlier");
    if (bytes > s->alloc.size())
        return knnf::set_error(KNNF_ENOMEM, "frame needs %zu bytes; pool has %zu", bytes,
                               s->alloc.size());
    if ((int)s->queue.size() >= s->opts.max_queue)
        return knnf::set_error(KNNF_EAGAIN, "admission queue full");
    Job j;
    j.ticket = s->next_ticket++;
    j.hf = *f;
    j.bytes = bytes;
    j.t_arrival = f->t_arrival >= 0 ? f->t_arrival : now_s();
    j.map_pc1 = m1;
    j.map_prob = m2;
    Job& stored = s->jobs[j.ticket] = j;
    stage(stored, "queued");
    s->queue.push_back(j.ticket);
    ++s->unfinished;
    *ticket = j.ticket;
    s->cv.notify_one();
    return KNNF_OK;
}

knnf_status knnf_server_poll(knnf_server* s, uint64_t ticket, knnf_ticket_info* info) {
    if (!s || !info) return knnf::set_error(KNNF_EINVAL, "knnf_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return knnf::set_error(KNNF_EINVAL, "unknown ticket");
    const Job& j = it->second;
    info->done = j.state == DONE || j.state == RELEASED;
    info->released = j.state == RELEASED;
    info->t_arrival = j.t_arrival;
    info->t_admit = j.t_admit;
    info->t_launch = j.t_launch;
    info->t_done = j.t_done;
    if (s->sticky != KNNF_OK) return knnf::set_error(s->sticky, "server failed");
    return knnf::ctx_status(s->ctx);
}

knnf_status knnf_server_result(knnf_server* s, uint64_t ticket, knnf_frame* view) {
    if (!s || !view) return knnf::set_error(KNNF_EINVAL, "knnf_server_result: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return knnf::set_error(KNNF_EINVAL, "unknown ticket");
    if (it->second.state != DONE) return knnf::set_error(KNNF_ESTATE, "frame not done or released");
    *view = it->second.dev;
    return KNNF_OK;
}

knnf_status knnf_server_release(knnf_server* s, uint64_t ticket) {
    if (!s) return knnf::set_error(KNNF_EINVAL, "knnf_server_release: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return knnf::set_error(KNNF_EINVAL, "unknown ticket");
    Job& j = it->second;
    if (j.state != DONE) return knnf::set_error(KNNF_ESTATE, "frame not done");
    s->alloc.release(j.off, j.bytes);
    s->jobs.erase(it);
    s->cv.notify_one();
    return KNNF_OK;
}

knnf_status knnf_server_drain(knnf_server* s, double timeout_s) {
    if (!s) return knnf::set_error(KNNF_EINVAL, "knnf_server_drain: NULL server");
    const double t0 = now_s();
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->sticky != KNNF_OK) return knnf::set_error(s->sticky, "server failed");
            const knnf_status cs = knnf::ctx_status(s->ctx);
            if (cs != KNNF_OK) return cs;
            if (s->unfinished == 0) return KNNF_OK;
        }
        if (timeout_s > 0 && now_s() - t0 > timeout_s)
            return knnf::set_error(KNNF_EAGAIN, "knnf_server_drain: timeout");
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

knnf_status knnf_server_destroy(knnf_server* s) {
    if (!s) return KNNF_OK;
    {
        // set under the lock, so a thread between its check and its wait
        // cannot miss the notification
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop.store(true);
    }
    s->cv.notify_all();
    s->copy_cv.notify_all();
    if (s->thread.joinable()) s->thread.join();
    if (s->copier.joinable()) s->copier.join();
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(s->device);
    for (Step& st : s->steps) {
        if (st.stream) {
            hipStreamSynchronize(st.stream);
            hipStreamDestroy(st.stream);
        }
        if (st.done) hipEventDestroy(st.done);
    }
    if (s->copy_stream) {
        hipStreamSynchronize(s->copy_stream);
        hipStreamDestroy(s->copy_stream);
    }
    for (auto& kv : s->jobs) {
        if (kv.second.copied) hipEventDestroy(kv.second.copied);
        stage(kv.second, nullptr);  // frames never finished
    }
    for (hipEvent_t e : s->event_pool) hipEventDestroy(e);
    hipSetDevice(prev);
    delete s;
    return KNNF_OK;
}

}  // extern "C"
