// Serving and C-ABI tests of the library's host runtime on the CPU -- TEST
// INFRASTRUCTURE ONLY.  Built from the product's knnf_api.cpp and
// knnf_server.cpp against the fake HIP runtime of this folder, whose
// "device" runs every filtering launch with the CPU oracle; run under
// AddressSanitizer and ThreadSanitizer by tests/test_server_fake.py.
//
// Each test prints "ok <name>" or "FAIL <name>: ..." and the program exits
// non-zero if any failed.  Usage: test_server_fake [name ...]
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "knnf.h"

extern "C" int knn_oracle_filter(int H, int W, int C, int K, int R, float lambda, const float* pc1,
                                 const float* prob, float* out_prob, int32_t* out_class,
                                 int32_t* out_nbr, float* out_dist, int nthreads);
namespace fakedev {
extern std::atomic<double> ns_per_pixel;
extern std::atomic<long> tiles_run;
}  // namespace fakedev

namespace {

int g_failed = 0;
std::string g_why;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            g_why = std::string(#cond) + " (line " + std::to_string(__LINE__) + "): " + \
                    knnf_last_error();                                           \
            return false;                                                        \
        }                                                                        \
    } while (0)

// One frame's inputs (host memory: pinned through hipHostMalloc, or plain)
// and the oracle's outputs for it.
struct Frame {
    int H, W, C, K, R;
    float lam;
    bool pinned, with_nbr;
    float *pc1 = nullptr, *prob = nullptr;
    std::vector<float> ref_prob, ref_dist;
    std::vector<int32_t> ref_class, ref_nbr;

    Frame(int h, int w, int c, int k, int r, float l, uint32_t seed, bool pin, bool nbr)
        : H(h), W(w), C(c), K(k), R(r), lam(l), pinned(pin), with_nbr(nbr) {
        const size_t px = (size_t)H * W;
        if (pinned) {
            hipHostMalloc((void**)&pc1, px * 4, hipHostMallocDefault);
            hipHostMalloc((void**)&prob, px * C * 4, hipHostMallocDefault);
        } else {
            pc1 = (float*)std::malloc(px * 4);
            prob = (float*)std::malloc(px * C * 4);
        }
        uint32_t s = seed * 2654435761u + 12345u;
        auto rnd = [&s]() {
            s = s * 1664525u + 1013904223u;
            return (float)((s >> 8) & 0xffffff) / 16777216.0f;
        };
        for (size_t t = 0; t < px; ++t) pc1[t] = rnd();
        for (size_t t = 0; t < px; ++t) {
            float sum = 0;
            for (int c2 = 0; c2 < C; ++c2) sum += (prob[t * C + c2] = rnd() + 0.01f);
            for (int c2 = 0; c2 < C; ++c2) prob[t * C + c2] /= sum;
        }
        ref_prob.resize(px * C);
        ref_class.resize(px);
        ref_nbr.resize(px * K);
        ref_dist.resize(px * K);
        knn_oracle_filter(H, W, C, K, R, lam, pc1, prob, ref_prob.data(), ref_class.data(),
                          ref_nbr.data(), ref_dist.data(), 1);
    }
    ~Frame() {
        if (pinned) {
            hipHostFree(pc1);
            hipHostFree(prob);
        } else {
            std::free(pc1);
            std::free(prob);
        }
    }
    Frame(const Frame&) = delete;
    Frame& operator=(const Frame&) = delete;

    knnf_host_frame host(double t_arrival = -1.0) const {
        knnf_host_frame f{};
        f.H = H, f.W = W, f.C = C, f.K = K, f.R = R, f.lambda = lam;
        f.pc1 = pc1;
        f.prob = prob;
        f.with_nbr = with_nbr ? 1 : 0;
        f.t_arrival = t_arrival;
        return f;
    }
    uint32_t tiles(int rows, int cols) const {
        return (uint32_t)((H + rows - 1) / rows) * (uint32_t)((W + cols - 1) / cols);
    }
    // the outputs of a device view equal the oracle's, bit for bit
    bool matches(const knnf_frame& v) const {
        const size_t px = (size_t)H * W;
        if (std::memcmp(v.out_prob, ref_prob.data(), px * C * 4) != 0) return false;
        if (std::memcmp(v.out_class, ref_class.data(), px * 4) != 0) return false;
        if (with_nbr) {
            if (!v.out_nbr || !v.out_dist) return false;
            if (std::memcmp(v.out_nbr, ref_nbr.data(), px * K * 4) != 0) return false;
            if (std::memcmp(v.out_dist, ref_dist.data(), px * K * 4) != 0) return false;
        }
        return true;
    }
};

struct Env {
    knnf_ctx* ctx = nullptr;
    void* pool = nullptr;
    size_t pool_bytes = 0;
    Env(size_t bytes) : pool_bytes(bytes) {
        knnf_create(&ctx, 0);
        hipMalloc(&pool, bytes);
        std::memset(pool, 0xff, bytes);  // outputs never written stay NaN / -1
    }
    ~Env() {
        hipFree(pool);
        knnf_destroy(ctx);
    }
};

knnf_server_opts opts(int mode, int step_tiles = 0, int max_queue = 0) {
    knnf_server_opts o{};
    o.mode = mode;
    o.step_tiles = step_tiles;
    o.max_queue = max_queue;
    o.plan.search = KNNF_SEARCH_PRUNED;
    return o;
}

bool wait_done(knnf_server* s, uint64_t t, double timeout_s = 60.0) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        knnf_ticket_info info{};
        if (knnf_server_poll(s, t, &info) != KNNF_OK) return false;
        if (info.done) return true;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::duration<double>(timeout_s)) return false;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

using Frames = std::vector<std::unique_ptr<Frame>>;

Frames mixed_frames(int n, uint32_t seed, bool with_nbr_some) {
    // H, W, C, K, R: small windows keep the CPU oracle quick; several frames
    // span more tiles than one step's budget, so they are sliced
    const int shapes[][5] = {{8, 9, 4, 5, 2}, {20, 33, 4, 16, 3}, {24, 40, 4, 16, 3},
                             {17, 61, 3, 12, 4}, {1, 70, 4, 5, 0}, {30, 36, 4, 40, 5}};
    Frames v;
    for (int k = 0; k < n; ++k) {
        const int* sh = shapes[(k * 7 + seed) % 6];
        v.emplace_back(new Frame(sh[0], sh[1], sh[2], sh[3], sh[4], 0.01f, seed + k, k % 3 != 0,
                                 with_nbr_some && k % 4 == 1));
    }
    return v;
}

// ---- tests ------------------------------------------------------------------

// Frames of mixed sizes arriving together are sliced into small steps (a
// tile budget of 64) and batched with each other: every frame's outputs equal
// the oracle's for that frame alone, and every tile ran exactly once.
bool test_mixed_stream_equals_alone() {
    Env env(16 << 20);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED, 64);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    auto frames = mixed_frames(30, 1, true);
    const long t0 = fakedev::tiles_run.load();
    std::vector<uint64_t> tk;
    for (auto& f : frames) {
        uint64_t t = 0;
        const knnf_host_frame h = f->host();
        CHECK(knnf_server_submit(s, &h, &t) == KNNF_OK);
        tk.push_back(t);
    }
    CHECK(knnf_server_drain(s, 60.0) == KNNF_OK);
    uint64_t tiles = 0;
    for (size_t k = 0; k < frames.size(); ++k) {
        knnf_frame v{};
        CHECK(knnf_server_result(s, tk[k], &v) == KNNF_OK);
        CHECK(frames[k]->matches(v));
        CHECK(knnf_server_release(s, tk[k]) == KNNF_OK);
        tiles += frames[k]->tiles(1, 8);
    }
    CHECK((uint64_t)(fakedev::tiles_run.load() - t0) == tiles);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// Every frame passes through the three stage ranges (queued, ready, on gpu),
// each range opened is closed by the time its frame is done, and the
// thread-local push/pop ranges of the copy and launch calls are balanced.
bool test_trace_ranges() {
    Env env(16 << 20);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED, 64);
    const long open0 = fakehip::roctx_open(), started0 = fakehip::roctx_started();
    const long pushed0 = fakehip::roctx_pushed();
    CHECK(open0 == 0);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    auto frames = mixed_frames(12, 5, false);
    std::vector<uint64_t> tk;
    for (auto& f : frames) {
        uint64_t t = 0;
        const knnf_host_frame h = f->host();
        CHECK(knnf_server_submit(s, &h, &t) == KNNF_OK);
        tk.push_back(t);
    }
    CHECK(knnf_server_drain(s, 60.0) == KNNF_OK);
    CHECK(fakehip::roctx_open() == 0);  // every frame done: no stage left open
    CHECK(fakehip::roctx_started() - started0 == 3 * (long)frames.size());
    CHECK(fakehip::roctx_pushed() - pushed0 >= 2);  // copies and steps
    const std::string last = "knnf frame " + std::to_string(tk.back()) + " ";
    CHECK(fakehip::roctx_saw((last + std::to_string(frames.back()->H) + "x" +
                              std::to_string(frames.back()->W) + " on gpu").c_str()));
    CHECK(fakehip::roctx_saw("queued") && fakehip::roctx_saw("ready"));
    for (uint64_t t : tk) CHECK(knnf_server_release(s, t) == KNNF_OK);
    // a frame still queued when the server is destroyed has its range closed
    uint64_t t = 0;
    const knnf_host_frame h = frames[0]->host();
    CHECK(knnf_server_submit(s, &h, &t) == KNNF_OK);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    CHECK(fakehip::roctx_open() == 0);
    return true;
}

// Admission is first in, first out: with a pool that holds about one large
// frame, small frames behind a large one wait for it (no overtaking), and
// every frame is admitted in submission order.
bool test_fifo_admission() {
    Frame big(40, 48, 4, 40, 5, 0.01f, 7, true, false);
    const size_t big_bytes = knnf_frame_bytes(40, 48, 4, 40, 0);
    // room for the large frame and less than any other frame
    Env env(big_bytes + 1024);
    fakedev::ns_per_pixel = 4000.0;  // about 8 ms for the large frame
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    Frames small;
    for (int k = 0; k < 6; ++k) small.emplace_back(new Frame(8, 9, 4, 5, 2, 0.01f, 40 + k, true, false));
    std::vector<uint64_t> tk(7);
    knnf_host_frame h = big.host();
    CHECK(knnf_server_submit(s, &h, &tk[0]) == KNNF_OK);
    for (int k = 0; k < 6; ++k) {
        h = small[k]->host();
        CHECK(knnf_server_submit(s, &h, &tk[k + 1]) == KNNF_OK);
    }
    // release each frame as soon as it is done, in any order
    std::vector<knnf_ticket_info> info(7);
    std::vector<bool> rel(7, false);
    int left = 7;
    const auto t0 = std::chrono::steady_clock::now();
    while (left > 0) {
        for (int k = 0; k < 7; ++k) {
            if (rel[k]) continue;
            CHECK(knnf_server_poll(s, tk[k], &info[k]) == KNNF_OK);
            if (info[k].done) {
                knnf_frame v{};
                CHECK(knnf_server_result(s, tk[k], &v) == KNNF_OK);
                CHECK(k == 0 ? big.matches(v) : small[k - 1]->matches(v));
                CHECK(knnf_server_release(s, tk[k]) == KNNF_OK);
                rel[k] = true;
                --left;
            }
        }
        CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(60));
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    fakedev::ns_per_pixel = 0.0;
    for (int k = 0; k + 1 < 7; ++k) CHECK(info[k].t_admit <= info[k + 1].t_admit);
    // the small frames could only be admitted after the large one left the pool
    CHECK(info[1].t_admit >= info[0].t_done);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// A full admission queue answers KNNF_EAGAIN; the frames queued are served
// once pool memory is released.
bool test_eagain_when_queue_full() {
    Frame a(20, 33, 4, 16, 7, 0.01f, 1, false, false);
    Env env(knnf_frame_bytes(20, 33, 4, 16, 0) + 256);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED, 0, 2);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    uint64_t t0 = 0, t1 = 0, t2 = 0, t3 = 0;
    const knnf_host_frame h = a.host();
    CHECK(knnf_server_submit(s, &h, &t0) == KNNF_OK);
    CHECK(wait_done(s, t0));  // holds the whole pool until released
    CHECK(knnf_server_submit(s, &h, &t1) == KNNF_OK);
    CHECK(knnf_server_submit(s, &h, &t2) == KNNF_OK);
    CHECK(knnf_server_submit(s, &h, &t3) == KNNF_EAGAIN);
    for (uint64_t t : {t0, t1, t2}) {
        CHECK(wait_done(s, t));
        knnf_frame v{};
        CHECK(knnf_server_result(s, t, &v) == KNNF_OK);
        CHECK(a.matches(v));
        CHECK(knnf_server_release(s, t) == KNNF_OK);
    }
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// A frame larger than the whole pool can never be admitted: KNNF_ENOMEM at
// submission; bad frames are KNNF_EINVAL.
bool test_enomem_and_einval_at_submit() {
    Env env(64 << 10);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    Frame big(40, 48, 4, 40, 5, 0.01f, 3, false, true);
    uint64_t t = 0;
    knnf_host_frame h = big.host();
    CHECK(knnf_server_submit(s, &h, &t) == KNNF_ENOMEM);
    h.K = 0;
    CHECK(knnf_server_submit(s, &h, &t) == KNNF_EINVAL);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// Results and release of an unfinished frame are KNNF_ESTATE; unknown
// tickets are KNNF_EINVAL.
bool test_estate_before_done() {
    Env env(16 << 20);
    fakedev::ns_per_pixel = 20000.0;  // about 20 ms for the frame
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    Frame f(24, 40, 4, 16, 3, 0.01f, 5, true, false);
    uint64_t t = 0;
    const knnf_host_frame h = f.host();
    CHECK(knnf_server_submit(s, &h, &t) == KNNF_OK);
    knnf_frame v{};
    CHECK(knnf_server_result(s, t, &v) == KNNF_ESTATE);
    CHECK(knnf_server_release(s, t) == KNNF_ESTATE);
    knnf_ticket_info info{};
    CHECK(knnf_server_poll(s, t + 1000, &info) == KNNF_EINVAL);
    fakedev::ns_per_pixel = 0.0;
    CHECK(wait_done(s, t));
    CHECK(knnf_server_result(s, t, &v) == KNNF_OK);
    CHECK(f.matches(v));
    CHECK(knnf_server_release(s, t) == KNNF_OK);
    CHECK(knnf_server_release(s, t) == KNNF_EINVAL);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// The plain baseline: one whole frame per launch, in arrival order.
bool test_plain_mode() {
    Env env(16 << 20);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_PLAIN);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    auto frames = mixed_frames(12, 2, true);
    std::vector<uint64_t> tk;
    for (auto& f : frames) {
        uint64_t t = 0;
        const knnf_host_frame h = f->host();
        CHECK(knnf_server_submit(s, &h, &t) == KNNF_OK);
        tk.push_back(t);
    }
    CHECK(knnf_server_drain(s, 60.0) == KNNF_OK);
    double last_done = 0;
    for (size_t k = 0; k < frames.size(); ++k) {
        knnf_ticket_info info{};
        CHECK(knnf_server_poll(s, tk[k], &info) == KNNF_OK);
        CHECK(info.t_done >= last_done);  // one at a time, in order
        last_done = info.t_done;
        knnf_frame v{};
        CHECK(knnf_server_result(s, tk[k], &v) == KNNF_OK);
        CHECK(frames[k]->matches(v));
        CHECK(knnf_server_release(s, tk[k]) == KNNF_OK);
    }
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// A failed input copy fails the server and its context for good.
bool test_copy_failure_is_sticky() {
    Env env(16 << 20);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    Frame f(20, 33, 4, 16, 7, 0.01f, 6, false, false);
    uint64_t t = 0;
    const knnf_host_frame h = f.host();
    fakehip::fail_copy_after(0);
    CHECK(knnf_server_submit(s, &h, &t) == KNNF_OK);
    CHECK(knnf_server_drain(s, 10.0) == KNNF_EDEVICE);
    fakehip::fail_copy_after(-1);
    uint64_t t2 = 0;
    CHECK(knnf_server_submit(s, &h, &t2) == KNNF_EDEVICE);
    CHECK(knnf_ctx_status(env.ctx) == KNNF_EDEVICE);
    knnf_frame fr{};
    fr.H = f.H, fr.W = f.W, fr.C = f.C, fr.K = f.K, fr.R = f.R, fr.lambda = f.lam;
    fr.pc1 = f.pc1, fr.prob = f.prob;
    std::vector<float> op((size_t)f.H * f.W * f.C);
    std::vector<int32_t> oc((size_t)f.H * f.W);
    fr.out_prob = op.data(), fr.out_class = oc.data();
    CHECK(knnf_filter(env.ctx, &fr, nullptr, nullptr) == KNNF_EDEVICE);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// Non-finite host inputs are rejected at submission (the server checks on
// the host unless its plan says the caller vouches for the inputs).
bool test_non_finite_submit() {
    Env env(16 << 20);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    Frame f(20, 33, 4, 16, 7, 0.01f, 8, true, false);
    f.prob[77] = NAN;
    uint64_t t = 0;
    const knnf_host_frame h = f.host();
    CHECK(knnf_server_submit(s, &h, &t) == KNNF_EINVAL);
    CHECK(knnf_ctx_status(env.ctx) == KNNF_OK);
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// Several host threads submit at once while another polls and releases:
// every frame is served, with the oracle's outputs.
bool test_concurrent_submitters() {
    Env env(8 << 20);
    knnf_server* s = nullptr;
    const knnf_server_opts o = opts(KNNF_SERVE_BATCHED, 256);
    CHECK(knnf_server_create(&s, env.ctx, env.pool, env.pool_bytes, &o) == KNNF_OK);
    constexpr int kThreads = 4, kPer = 10;
    std::vector<Frames> frames(kThreads);
    for (int t = 0; t < kThreads; ++t) frames[t] = mixed_frames(kPer, 100 + 17 * t, t % 2 == 0);
    std::vector<std::vector<uint64_t>> tickets(kThreads);
    std::atomic<int> submitted{0}, errors{0};
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t)
        th.emplace_back([&, t] {
            for (auto& f : frames[t]) {
                const knnf_host_frame h = f->host();
                uint64_t tk = 0;
                knnf_status st;
                while ((st = knnf_server_submit(s, &h, &tk)) == KNNF_EAGAIN)
                    std::this_thread::sleep_for(std::chrono::microseconds(100));
                if (st != KNNF_OK) {
                    ++errors;
                    continue;
                }
                tickets[t].push_back(tk);
                ++submitted;
            }
        });
    for (auto& x : th) x.join();
    CHECK(errors == 0 && submitted == kThreads * kPer);
    for (int t = 0; t < kThreads; ++t)
        for (int k = 0; k < kPer; ++k) {
            CHECK(wait_done(s, tickets[t][k]));
            knnf_frame v{};
            CHECK(knnf_server_result(s, tickets[t][k], &v) == KNNF_OK);
            CHECK(frames[t][k]->matches(v));
            CHECK(knnf_server_release(s, tickets[t][k]) == KNNF_OK);
        }
    CHECK(knnf_server_destroy(s) == KNNF_OK);
    return true;
}

// The batched C-ABI call on the fake device: tables of 41 work items (copied
// through the pinned staging) and of 5 (a kernel argument), both launch
// modes, every frame equal to the oracle; a NaN input is rejected before any
// filtering launch.
bool test_filter_batch_tables() {
    Env env(1 << 20);
    for (int n : {5, 41}) {
        auto frames = mixed_frames(n, 9 + n, true);
        std::vector<std::vector<float>> op(n), od(n);
        std::vector<std::vector<int32_t>> oc(n), on(n);
        std::vector<knnf_frame> fr(n);
        for (int k = 0; k < n; ++k) {
            Frame& f = *frames[k];
            const size_t px = (size_t)f.H * f.W;
            op[k].assign(px * f.C, NAN);
            oc[k].assign(px, -1);
            on[k].assign(px * f.K, -1);
            od[k].assign(px * f.K, NAN);
            fr[k] = knnf_frame{f.H, f.W, f.C, f.K, f.R, f.lam, f.pc1, f.prob, op[k].data(),
                               oc[k].data(), f.with_nbr ? on[k].data() : nullptr,
                               f.with_nbr ? od[k].data() : nullptr};
        }
        for (int launch : {KNNF_LAUNCH_PERSISTENT, KNNF_LAUNCH_GRID}) {
            knnf_plan p{};
            p.search = KNNF_SEARCH_PRUNED;
            p.launch = launch;
            const long t0 = fakedev::tiles_run.load();
            CHECK(knnf_filter_batch(env.ctx, fr.data(), n, &p, nullptr) == KNNF_OK);
            CHECK(hipDeviceSynchronize() == hipSuccess);
            uint64_t tiles = 0;
            for (int k = 0; k < n; ++k) {
                CHECK(frames[k]->matches(fr[k]));
                tiles += frames[k]->tiles(1, 8);
            }
            CHECK((uint64_t)(fakedev::tiles_run.load() - t0) == tiles);
        }
        frames[n - 1]->pc1[3] = INFINITY;
        const long t1 = fakedev::tiles_run.load();
        CHECK(knnf_filter_batch(env.ctx, fr.data(), n, nullptr, nullptr) == KNNF_EINVAL);
        CHECK(fakedev::tiles_run.load() == t1);
    }
    return true;
}

struct Test {
    const char* name;
    std::function<bool()> fn;
};

}  // namespace

int main(int argc, char** argv) {
    const std::vector<Test> tests = {
        {"mixed_stream_equals_alone", test_mixed_stream_equals_alone},
        {"fifo_admission", test_fifo_admission},
        {"eagain_when_queue_full", test_eagain_when_queue_full},
        {"enomem_and_einval_at_submit", test_enomem_and_einval_at_submit},
        {"estate_before_done", test_estate_before_done},
        {"plain_mode", test_plain_mode},
        {"non_finite_submit", test_non_finite_submit},
        {"concurrent_submitters", test_concurrent_submitters},
        {"filter_batch_tables", test_filter_batch_tables},
        {"trace_ranges", test_trace_ranges},
        {"copy_failure_is_sticky", test_copy_failure_is_sticky},  // last: fails its context
    };
    for (const Test& t : tests) {
        bool want = argc < 2;
        for (int k = 1; k < argc; ++k) want |= std::strcmp(argv[k], t.name) == 0;
        if (!want) continue;
        g_why.clear();
        const bool ok = t.fn();
        if (ok) {
            std::printf("ok %s\n", t.name);
        } else {
            std::printf("FAIL %s: %s\n", t.name, g_why.c_str());
            ++g_failed;
        }
        std::fflush(stdout);
    }
    return g_failed ? 1 : 0;
}
