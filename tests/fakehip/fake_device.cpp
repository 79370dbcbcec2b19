// The library's device launches, executed on the CPU by the oracle -- TEST
// INFRASTRUCTURE ONLY.  Each launch becomes an operation of its (fake)
// stream that reads the work table from "device" memory when the stream gets
// to it, as a kernel would, and filters exactly the tiles the table assigns
// with the plain CPU oracle, so that a tile the runtime forgets or assigns
// twice, or a table not yet written when the launch runs, shows up in the
// outputs.  A configurable delay per pixel stands in for the kernel's time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "knnf_device.h"

extern "C" int knn_oracle_pixels(int H, int W, int C, int K, int R, float lambda, const float* pc1,
                                 const float* prob, const int32_t* pix, int npix, float* out_prob,
                                 int32_t* out_class, int32_t* out_nbr, float* out_dist,
                                 int nthreads);

namespace fakedev {
std::atomic<double> ns_per_pixel{0.0};
std::atomic<long> tiles_run{0};
}  // namespace fakedev

namespace knnf {
namespace {

void pause_for(size_t pixels) {
    const double ns = fakedev::ns_per_pixel.load() * (double)pixels;
    if (ns > 0) std::this_thread::sleep_for(std::chrono::nanoseconds((long long)ns));
}

// Filter the pixels of tiles [t0, t0 + nt) of frame f (tiles of rows x cols).
void run_tiles(const FrameDesc& f, int rows, int cols, uint32_t t0, uint32_t nt) {
    const uint32_t ntc = (uint32_t)((f.W + cols - 1) / cols);
    std::vector<int32_t> pix;
    for (uint32_t s = t0; s < t0 + nt; ++s) {
        const int band = (int)(s / ntc), tc = (int)(s % ntc);
        for (int a = 0; a < rows; ++a)
            for (int b = 0; b < cols; ++b) {
                const int r = band * rows + a, c = tc * cols + b;
                if (r < f.H && c < f.W) pix.push_back(r * f.W + c);
            }
    }
    fakedev::tiles_run.fetch_add((long)nt);
    if (f.stats) __atomic_fetch_add(&f.stats[1], (unsigned long long)nt, __ATOMIC_RELAXED);
    if (pix.empty()) return;
    const int n = (int)pix.size();
    std::vector<float> op((size_t)n * f.C), od(f.out_dist ? (size_t)n * f.K : 0);
    std::vector<int32_t> oc(n), on(f.out_nbr ? (size_t)n * f.K : 0);
    knn_oracle_pixels(f.H, f.W, f.C, f.K, f.R, f.lambda, f.pc1, f.prob, pix.data(), n, op.data(),
                      oc.data(), f.out_nbr ? on.data() : nullptr, f.out_dist ? od.data() : nullptr, 1);
    for (int t = 0; t < n; ++t) {
        const size_t q = (size_t)pix[t];
        std::memcpy(f.out_prob + q * f.C, op.data() + (size_t)t * f.C, sizeof(float) * f.C);
        f.out_class[q] = oc[t];
        if (f.out_nbr) std::memcpy(f.out_nbr + q * f.K, on.data() + (size_t)t * f.K, 4 * (size_t)f.K);
        if (f.out_dist) std::memcpy(f.out_dist + q * f.K, od.data() + (size_t)t * f.K, 4 * (size_t)f.K);
    }
    pause_for(pix.size());
}

// A batched launch: work item k covers the task ids task_start[k] ..
// task_start[k+1]-1, i.e. tiles tile_base[k] .. of frames[k].
void run_items(const FrameDesc* frames, const uint32_t* ts, const uint32_t* tb, uint32_t n,
               int rows, int cols) {
    for (uint32_t k = 0; k < n; ++k) run_tiles(frames[k], rows, cols, tb[k], ts[k + 1] - ts[k]);
}

bool any_nonfinite(const float* v, size_t n) {
    for (size_t t = 0; t < n; ++t) {
        uint32_t u;
        std::memcpy(&u, v + t, 4);
        if ((u & 0x7f800000u) == 0x7f800000u) return true;
    }
    return false;
}

}  // namespace

int launch_filter_frame(const FrameDesc& f, const LaunchCfg& cfg, void* stream) {
    const FrameDesc d = f;
    const int rows = cfg.rows, cols = cfg.cols;
    const uint32_t nt = (uint32_t)((f.H + rows - 1) / rows) * (uint32_t)((f.W + cols - 1) / cols);
    return fakehip::enqueue((hipStream_t)stream, [d, rows, cols, nt] { run_tiles(d, rows, cols, 0, nt); });
}

// lambda = 0 selection: the same applicability rule as the device's; the
// fake runs it as one 1 x 8 tiling of the frame (the oracle either way)
bool spectral_fits(const FrameDesc& f) {
    const int64_t rows = std::min<int64_t>((int64_t)2 * f.R + 2, f.H);
    return f.lambda == 0.0f && rows * f.W <= 16384;
}

int launch_spectral_frame(const FrameDesc& f, void* stream) {
    const FrameDesc d = f;
    const uint32_t nt = (uint32_t)f.H * (uint32_t)((f.W + 7) / 8);
    return fakehip::enqueue((hipStream_t)stream, [d, nt] { run_tiles(d, 1, 8, 0, nt); });
}

int launch_filter_items(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        const uint32_t* d_tile_base, uint32_t nframes, uint32_t,
                        const LaunchCfg& cfg, void* stream) {
    const int rows = cfg.rows, cols = cfg.cols;
    return fakehip::enqueue((hipStream_t)stream, [=] {
        run_items(d_frames, d_task_start, d_tile_base, nframes, rows, cols);
    });
}

int launch_filter_batch(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        const uint32_t* d_tile_base, uint32_t nframes, uint32_t total_tasks,
                        uint32_t*, const LaunchCfg& cfg, int, void* stream) {
    return launch_filter_items(d_frames, d_task_start, d_tile_base, nframes, total_tasks, cfg, stream);
}

int persistent_blocks_per_cu(const LaunchCfg&) { return 1; }

int launch_zero_counter(uint32_t* d_counter, void* stream) {
    return fakehip::enqueue((hipStream_t)stream, [d_counter] { *d_counter = 0; });
}

int launch_put_table(const TableWords& t, uint32_t* d_base, void* stream) {
    const TableWords c = t;
    return fakehip::enqueue((hipStream_t)stream, [c, d_base] {
        for (int r = 0; r < 3; ++r) std::memcpy(d_base + c.dst[r], c.w + c.src[r], 4 * (size_t)c.len[r]);
    });
}

int launch_copy_pair(const uint32_t* a, uint32_t* da, uint32_t na, const uint32_t* b, uint32_t* db,
                     uint32_t nb, void* stream) {
    return fakehip::enqueue((hipStream_t)stream, [=] {
        if (na) std::memcpy(da, a, 4 * (size_t)na);
        if (nb) std::memcpy(db, b, 4 * (size_t)nb);
    });
}

int launch_check_frame(const FrameDesc& f, uint32_t* flag, uint32_t gen, void* stream) {
    const FrameDesc d = f;
    return fakehip::enqueue((hipStream_t)stream, [d, flag, gen] {
        const size_t px = (size_t)d.H * (size_t)d.W;
        if (any_nonfinite(d.pc1, px) || any_nonfinite(d.prob, px * (size_t)d.C))
            __atomic_store_n(flag, gen, __ATOMIC_RELEASE);
    });
}

int launch_check_items(const FrameDesc* d_frames, uint32_t n, uint32_t, uint32_t* flag, uint32_t gen,
                       void* stream) {
    return fakehip::enqueue((hipStream_t)stream, [=] {
        for (uint32_t k = 0; k < n; ++k) {
            const FrameDesc& d = d_frames[k];
            const size_t px = (size_t)d.H * (size_t)d.W;
            if (any_nonfinite(d.pc1, px) || any_nonfinite(d.prob, px * (size_t)d.C))
                __atomic_store_n(flag, gen, __ATOMIC_RELEASE);
        }
    });
}

// The PC1 and SVM steps are not part of these tests.
int pc1_max_blocks() { return 1024; }
size_t pc1_scratch_head() { return 16384; }
int pc1_scratch_init(int, void** ptr) {
    static char dummy[256];
    *ptr = dummy;
    return hipSuccess;
}
int launch_pc1(const float*, int64_t, int, const double*, const double*, float*, double*, double*,
               int, void*) {
    return hipErrorInvalidValue;
}
int launch_pc1_normalise(const double*, int64_t, const double*, int, float*, int, void*) {
    return hipErrorInvalidValue;
}
int launch_svm(const float*, int64_t, int, int, const double*, const double*, const double*,
               const double*, float*, void*) {
    return hipErrorInvalidValue;
}
int svm_pixels_per_block() { return 256; }
int launch_svm_pc1(const float*, int64_t, int, int, const double*, const double*, const double*,
                   const double*, const double*, const double*, float*, float*, double*, double*,
                   int*, void*) {
    return hipErrorInvalidValue;
}

}  // namespace knnf
