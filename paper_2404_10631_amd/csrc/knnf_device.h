// knnf_device.h -- structures shared by the HIP kernels and the host runtime.
//
// Only plain types: the C-ABI in include/knnf.h never exposes these.
#pragma once

#include <stdint.h>

namespace knnf {

// One frame as the kernels see it (device pointers, sizes, parameters).
struct FrameDesc {
    const float* pc1;     // [H][W]
    const float* prob;    // [H][W][C]
    float* out_prob;      // [H][W][C]
    int32_t* out_class;   // [H][W]
    int32_t* out_nbr;     // [H][W][K] or null
    float* out_dist;      // [H][W][K] or null
    int32_t H, W, C, K, R;
    float lambda;
    unsigned long long* stats;  // [0] pairs evaluated, [1] tiles; null: not counted
};

// Kernel launch configuration chosen by the host (see knnf_plan).
struct LaunchCfg {
    int rows;      // tile rows (query pixels per wavefront = rows * cols)
    int cols;      // tile columns
    int waves;     // wavefronts per workgroup: 1, 2, 4
    int pruned;    // 0 exhaustive, 1 pruned
    int persistent;  // batched launches: 1 persistent claim loop, 0 one wavefront per task
    int chunk_log2;  // pruned search: log2 of the patch rows (3, 4, 5)
};

// Host-side launchers (defined in knnf_kernels.hip).  Return hipError_t as int.
int launch_filter_frame(const FrameDesc& f, const LaunchCfg& cfg, void* stream);
int launch_filter_batch(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        const uint32_t* d_tile_base, uint32_t nframes, uint32_t total_tasks,
                        uint32_t* d_counter, const LaunchCfg& cfg, int grid_blocks, void* stream);
// The filter at lambda = 0 as a 1-D selection in each query row's band sorted
// by value (defined in knnf_spectral.hip): applicable when spectral_fits(f)
// (lambda == 0 and the band of 2R + 2 rows, clipped to H, that serves two
// query rows holds at most 16,384 pixels); same outputs as the scans.
bool spectral_fits(const FrameDesc& f);
int launch_spectral_frame(const FrameDesc& f, void* stream);
// Zero the batched kernel's claim counter.
int launch_zero_counter(uint32_t* d_counter, void* stream);

// Non-finite input check: the kernels store `gen` to *flag (device-visible
// host memory) when any pc1 or prob value of the frames is not finite.
// max_words: the largest H*W*(C+1) of the table's frames (sizes the grid).
int launch_check_frame(const FrameDesc& f, uint32_t* flag, uint32_t gen, void* stream);
int launch_check_items(const FrameDesc* d_frames, uint32_t n, uint32_t max_words, uint32_t* flag,
                       uint32_t gen, void* stream);

// A batch table small enough to travel as a kernel argument: run k copies
// len[k] words from w[src[k]] to d_base[dst[k]].  Writing a small table this
// way needs no host-to-device copy, which could hold up the launching thread
// for milliseconds.
constexpr int kTableWords = 880;
struct TableWords {
    uint32_t w[kTableWords];
    uint32_t src[3], dst[3], len[3];
};
int launch_put_table(const TableWords& t, uint32_t* d_base, void* stream);

// Copy na words a -> da and nb words b -> db with one small kernel (the
// sources may be device-mapped pinned host memory).
int launch_copy_pair(const uint32_t* a, uint32_t* da, uint32_t na, const uint32_t* b,
                     uint32_t* db, uint32_t nb, void* stream);

// A range of tiles of one frame, the unit of a batched launch.
struct WorkItem {
    FrameDesc f;
    uint32_t tile0;    // first tile (row-major over the frame's tile grid)
    uint32_t ntiles;   // number of tiles
};
int persistent_blocks_per_cu(const LaunchCfg& cfg);
// Non-persistent launch over the same work table: one wavefront per task.
int launch_filter_items(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        const uint32_t* d_tile_base, uint32_t nframes, uint32_t total_tasks,
                        const LaunchCfg& cfg, void* stream);

// PC1 projection (defined in knnf_pc1.hip).  ws == nullptr: out = the centred
// projection; otherwise ws (npix doubles) holds it, and out = its min-max
// normalisation; pairs holds 2 * pc1_max_blocks() doubles (scratch).
int pc1_max_blocks();
int launch_pc1(const float* cube, int64_t npix, int bands, const double* mean, const double* vec,
               float* out, double* ws, double* pairs, int num_cu, void* stream);

// Device address of knnf_pc1_noalloc's static scratch on `device` (which must
// be current): looked up once per device; returns hipError_t as int.  The
// pairs occupy the first pc1_scratch_head() bytes, the projection the rest.
int pc1_scratch_init(int device, void** ptr);
size_t pc1_scratch_head();

// Normalisation launch of the PC1 step alone: out[p] = (ws[p] - min) / (max -
// min) with min and max reduced from npairs (min, max) pairs.
int launch_pc1_normalise(const double* ws, int64_t npix, const double* pairs, int npairs,
                         float* out, int num_cu, void* stream);

// SVM probability stage (defined in knnf_svm.hip), 2 <= classes <= 8.
int launch_svm(const float* cube, int64_t npix, int bands, int classes, const double* w,
               const double* bias, const double* A, const double* B, float* out, void* stream);

// SVM maps and the PC1 projection from one read of the cube: `out` as
// launch_svm; the projection goes to band (binary32, ws == nullptr) or to ws
// (binary64) with each block's (min, max) in pairs[2 * block ..], for
// launch_pc1_normalise.  Returns the number of blocks through *nblocks.
int svm_pixels_per_block();
int launch_svm_pc1(const float* cube, int64_t npix, int bands, int classes, const double* w,
                   const double* bias, const double* A, const double* B, const double* mean,
                   const double* vec, float* out, float* band, double* ws, double* pairs,
                   int* nblocks, void* stream);

}  // namespace knnf
