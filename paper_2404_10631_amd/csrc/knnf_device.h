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
};

// Work accounting for the persistent batched launch: frame f owns the task
// ids [task_start[f], task_start[f+1]); a task is one wavefront tile.
struct BatchHeader {
    uint32_t nframes;
    uint32_t total_tasks;
};

// Kernel launch configuration chosen by the host (see knnf_plan).
struct LaunchCfg {
    int rows;      // tile rows (query pixels per wavefront = rows * cols)
    int cols;      // tile columns
    int waves;     // wavefronts per workgroup: 1, 2, 4
    int pruned;    // 0 exhaustive, 1 pruned
};

// Host-side launchers (defined in knnf_kernels.hip).  Return hipError_t as int.
int launch_filter_frame(const FrameDesc& f, const LaunchCfg& cfg, void* stream);
int launch_filter_batch(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        uint32_t nframes, uint32_t total_tasks, uint32_t* d_counter,
                        const LaunchCfg& cfg, int grid_blocks, void* stream);
int persistent_blocks_per_cu(const LaunchCfg& cfg);

}  // namespace knnf
