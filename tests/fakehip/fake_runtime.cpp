// CPU stand-in for the HIP runtime calls of the library's host runtime --
// TEST INFRASTRUCTURE ONLY (see hip/hip_runtime.h in this folder).
//
// A stream is a worker thread with a FIFO of operations; an event records the
// point its stream has reached and completes when the worker gets there; a
// stream told to wait for an event blocks its worker until the event
// completes.  "Device" memory is ordinary host memory, and pinned host
// memory is reported as device-mapped (its device address is itself).
#include "hip/hip_runtime.h"
#include "rocprofiler-sdk-roctx/roctx.h"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

struct FakeEvent {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t recorded = 0;   // generation of the last record
    uint64_t completed = 0;  // highest generation reached
    double t_done = 0.0;
};

struct FakeStream {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    uint64_t enq = 0, done = 0;
    bool stop = false;
    std::thread worker;
};

namespace {

thread_local hipError_t g_last = hipSuccess;
std::mutex g_mu;                         // registries below
std::set<FakeStream*> g_streams;
std::map<const char*, size_t> g_pinned;  // pinned host allocations: base -> bytes
std::atomic<int> g_fail_copy{-1};
std::atomic<long> g_ops{0};

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

hipError_t set_last(hipError_t e) {
    if (e != hipSuccess) g_last = e;
    return e;
}

void run_worker(FakeStream* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv.wait(lk, [s] { return s->stop || !s->q.empty(); });
        if (s->q.empty()) return;  // stopping and drained
        std::function<void()> op = std::move(s->q.front());
        s->q.pop_front();
        lk.unlock();
        op();
        g_ops.fetch_add(1);
        lk.lock();
        ++s->done;
        s->cv.notify_all();
    }
}

void* alloc256(size_t n) {
    void* p = nullptr;
    if (posix_memalign(&p, 256, n ? (n + 255) & ~size_t(255) : 256) != 0) return nullptr;
    return p;
}

}  // namespace

namespace fakehip {

hipError_t enqueue(hipStream_t s, std::function<void()> op) {
    if (!s) {
        op();
        g_ops.fetch_add(1);
        return hipSuccess;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->q.push_back(std::move(op));
    ++s->enq;
    s->cv.notify_all();
    return hipSuccess;
}

void fail_copy_after(int n) { g_fail_copy.store(n); }
long ops_run() { return g_ops.load(); }

}  // namespace fakehip

hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return set_last(d == 0 ? hipSuccess : hipErrorInvalidDevice); }
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d) {
    if (d != 0) return set_last(hipErrorInvalidDevice);
    std::memset(p, 0, sizeof *p);
    std::strcpy(p->name, "fake");
    p->multiProcessorCount = 4;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "no error";
        case hipErrorOutOfMemory: return "out of memory";
        case hipErrorNotReady: return "not ready";
        case hipErrorLaunchFailure: return "launch failure (injected)";
        default: return "fake error";
    }
}
hipError_t hipGetLastError(void) {
    const hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
hipError_t hipDeviceSynchronize(void) {
    std::set<FakeStream*> all;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        all = g_streams;
    }
    for (FakeStream* s : all) hipStreamSynchronize(s);
    return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t n) {
    *p = alloc256(n);
    return *p ? hipSuccess : set_last(hipErrorOutOfMemory);
}
hipError_t hipFree(void* p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
    *p = alloc256(n);
    if (!*p) return set_last(hipErrorOutOfMemory);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pinned[(const char*)*p] = n;
    return hipSuccess;
}
hipError_t hipHostFree(void* p) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_pinned.erase((const char*)p);
    }
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned) {
    *dev = host;
    return hipSuccess;
}
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_pinned.upper_bound((const char*)p);
    if (it == g_pinned.begin()) return set_last(hipErrorInvalidValue);
    --it;
    if ((const char*)p >= it->first + it->second) return set_last(hipErrorInvalidValue);
    a->type = hipMemoryTypeHost;
    a->device = 0;
    a->hostPointer = (void*)it->first;
    a->devicePointer = (void*)it->first;
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
    std::memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
    int f = g_fail_copy.load();
    while (f >= 0) {
        if (g_fail_copy.compare_exchange_weak(f, f - 1)) {
            if (f == 0) return set_last(hipErrorLaunchFailure);
            break;
        }
    }
    return fakehip::enqueue(s, [dst, src, n] { std::memcpy(dst, src, n); });
}
hipError_t hipMemset(void* p, int v, size_t n) {
    std::memset(p, v, n);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    FakeStream* x = new FakeStream;
    x->worker = std::thread(run_worker, x);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_streams.insert(x);
    }
    *s = x;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    if (!s) return hipSuccess;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_streams.erase(s);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->worker.join();
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    if (!s) return hipSuccess;
    std::unique_lock<std::mutex> lk(s->mu);
    const uint64_t target = s->enq;
    s->cv.wait(lk, [s, target] { return s->done >= target; });
    return hipSuccess;
}
hipError_t hipStreamQuery(hipStream_t s) {
    if (!s) return hipSuccess;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->done >= s->enq ? hipSuccess : set_last(hipErrorNotReady);
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    uint64_t target;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        target = e->recorded;
    }
    return fakehip::enqueue(s, [e, target] {
        std::unique_lock<std::mutex> lk(e->mu);
        e->cv.wait(lk, [e, target] { return e->completed >= target; });
    });
}

hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new FakeEvent;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        gen = ++e->recorded;
    }
    return fakehip::enqueue(s, [e, gen] {
        std::lock_guard<std::mutex> lk(e->mu);
        if (gen > e->completed) e->completed = gen;
        e->t_done = now_s();
        e->cv.notify_all();
    });
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::unique_lock<std::mutex> lk(e->mu);
    const uint64_t target = e->recorded;
    e->cv.wait(lk, [e, target] { return e->completed >= target; });
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(e->mu);
    return e->completed >= e->recorded ? hipSuccess : set_last(hipErrorNotReady);
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    double ta, tb;
    {
        std::lock_guard<std::mutex> lk(a->mu);
        ta = a->t_done;
    }
    {
        std::lock_guard<std::mutex> lk(b->mu);
        tb = b->t_done;
    }
    *ms = (float)((tb - ta) * 1e3);
    return hipSuccess;
}

// ---- roctx: ranges are counted, and every started name is kept
namespace {
std::mutex g_tx_mu;
std::set<roctx_range_id_t> g_tx_open;
std::vector<std::string> g_tx_names;
roctx_range_id_t g_tx_next = 1;
long g_tx_started = 0, g_tx_bad_stops = 0;
std::atomic<long> g_tx_pushed{0};
thread_local int g_tx_depth = 0;
}  // namespace

extern "C" {
void roctxMarkA(const char*) {}
int roctxRangePushA(const char*) {
    g_tx_pushed.fetch_add(1);
    return g_tx_depth++;
}
int roctxRangePop(void) { return g_tx_depth > 0 ? --g_tx_depth : -1; }
roctx_range_id_t roctxRangeStartA(const char* message) {
    std::lock_guard<std::mutex> lk(g_tx_mu);
    const roctx_range_id_t id = g_tx_next++;
    g_tx_open.insert(id);
    g_tx_names.emplace_back(message);
    ++g_tx_started;
    return id;
}
void roctxRangeStop(roctx_range_id_t id) {
    std::lock_guard<std::mutex> lk(g_tx_mu);
    if (g_tx_open.erase(id) == 0) ++g_tx_bad_stops;
}
}  // extern "C"

namespace fakehip {
long roctx_started() {
    std::lock_guard<std::mutex> lk(g_tx_mu);
    return g_tx_started;
}
long roctx_open() {
    std::lock_guard<std::mutex> lk(g_tx_mu);
    return g_tx_bad_stops ? -g_tx_bad_stops : (long)g_tx_open.size();
}
long roctx_pushed() { return g_tx_pushed.load(); }
int roctx_depth() { return g_tx_depth; }
bool roctx_saw(const char* substring) {
    std::lock_guard<std::mutex> lk(g_tx_mu);
    for (const std::string& n : g_tx_names)
        if (n.find(substring) != std::string::npos) return true;
    return false;
}
}  // namespace fakehip
