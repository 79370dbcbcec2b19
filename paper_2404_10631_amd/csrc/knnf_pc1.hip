// knnf_pc1.hip -- the one-band representation I of a hyperspectral cube (the
// PC1 projection step that feeds the KNN filter), for CDNA4 (gfx950).
//
// Method (PCA, Sec. II.C.2): centre every band by its average (step (i)) and
// project the centred image onto the first eigenvector (step (iv)); the GPU
// versions centre the cube and compute one matrix-vector product in double
// precision (Sec. III.A.2.a/d, III.B.2.a/d).  The covariance and eigenvector
// steps are not part of this library: band averages and eigenvector are
// inputs.  The KNN filter reads a normalised I (Sec. II.C.3); the reading
// taken here is min-max normalisation to [0, 1] over the frame.
//
//   I[p]  = sum_b (cube[p][b] - mean[b]) * vec[b]       binary64
//   I'[p] = (I[p] - min I) / (max I - min I)            binary64, 0 if constant
//   out[p] = binary32 rounding of I (or I')
//
// The step is HBM-bound (4 B per pixel and band, read once).  Lane layout of
// the projection kernel: a segment of S lanes covers one pixel, lane j of the
// segment reads bands 4j .. 4j+3 with one 16-byte load, so a wavefront reads
// 64/S whole pixels contiguously per load; the lane keeps its four averages
// and eigenvector entries in registers for the whole launch.  The segment sum
// is a butterfly over the S lanes.  Normalisation needs min and max over the
// frame: each projection block stores its (min, max) pair, and every block of
// the second launch reduces those pairs before rescaling its pixels (no
// atomics on one address, no device-wide fence).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/knnf.h"
#include "knnf_device.h"

namespace knnf {
namespace {

constexpr int PC1_THREADS = 256;
constexpr int PC1_UNROLL = 4;  // pixels per lane per iteration (independent loads in flight)
// Projection grid cap: enough wavefronts to keep HBM busy (each has
// PC1_UNROLL 16-byte loads in flight per lane), few enough partial pairs for
// the normalisation blocks to reduce.
constexpr int PC1_MAX_BLOCKS = 1024;

// Value of the partner lane for one butterfly step (64-bit through two
// 32-bit lane moves): DPP quad_perm xor 1 / xor 2, row_half_mirror (pairs the
// two quads of 8 lanes), row_mirror (the two halves of 16), and the
// permlane16 / permlane32 swaps (rows of 16, halves of 64).
template <int STEP>
__device__ __forceinline__ double partner(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    if constexpr (STEP < 4) {
        constexpr int ctrl = STEP == 0 ? 0xB1 : STEP == 1 ? 0x4E : STEP == 2 ? 0x141 : 0x140;
        lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, ctrl, 0xF, 0xF, false);
        hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, ctrl, 0xF, 0xF, false);
    } else if constexpr (STEP == 4) {
        const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        lo = (lane & 16) ? a[0] : a[1];
        hi = (lane & 16) ? b[0] : b[1];
    } else {
        const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        lo = (lane & 32) ? a[0] : a[1];
        hi = (lane & 32) ? b[0] : b[1];
    }
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over each aligned group of S lanes (S = 16, 32, 64); every lane of the
// group ends with the same value (each step adds two equal-order partial sums,
// and binary64 addition is commutative).
template <int S>
__device__ __forceinline__ double seg_sum(double v) {
    v += partner<0>(v);
    v += partner<1>(v);
    v += partner<2>(v);
    v += partner<3>(v);
    if constexpr (S >= 32) v += partner<4>(v);
    if constexpr (S >= 64) v += partner<5>(v);
    return v;
}

// Block-wide min and max of per-thread values; thread 0 gets the result.
__device__ void block_minmax(double lo, double hi, double* out_lo, double* out_hi) {
    __shared__ double slo[PC1_THREADS / 64], shi[PC1_THREADS / 64];
    for (int m = 1; m < 64; m <<= 1) {
        lo = fmin(lo, __shfl_xor(lo, m));
        hi = fmax(hi, __shfl_xor(hi, m));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slo[w] = lo;
        shi[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < PC1_THREADS / 64; ++k) {
            lo = fmin(lo, slo[k]);
            hi = fmax(hi, shi[k]);
        }
        *out_lo = lo;
        *out_hi = hi;
    }
}

// This block's min and max -> pairs[2 * blockIdx.x .. +1] (plain stores: the
// normalisation reads them in the next launch).
__device__ void publish_minmax(double lo, double hi, double* pairs) {
    __shared__ double blo, bhi;
    block_minmax(lo, hi, &blo, &bhi);
    if (threadIdx.x == 0) {
        pairs[2 * blockIdx.x] = blo;
        pairs[2 * blockIdx.x + 1] = bhi;
    }
}

// Projection, bands % 4 == 0, bands <= 4 * S, 16-byte aligned cube.
template <int S>
__global__ void __launch_bounds__(PC1_THREADS)
pc1_project_vec4(const float* __restrict__ cube, int64_t npix, int bands,
                 const double* __restrict__ mean, const double* __restrict__ vec,
                 float* __restrict__ out, double* __restrict__ ws, double* __restrict__ pairs) {
    constexpr int PW = 64 / S;  // pixels per wavefront per load
    const int lane = threadIdx.x & 63;
    const int j = lane % S;      // slot in the segment
    const int seg = lane / S;    // pixel of the segment within the wavefront group
    const int b0 = 4 * j;
    const bool act = b0 < bands;
    double mu[4], w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        mu[i] = act ? mean[b0 + i] : 0.0;
        w[i] = act ? vec[b0 + i] : 0.0;
    }
    const int64_t waves = (int64_t)gridDim.x * (PC1_THREADS / 64);
    const int64_t wid = (int64_t)blockIdx.x * (PC1_THREADS / 64) + (threadIdx.x >> 6);
    const int64_t stride = waves * PW * PC1_UNROLL;
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int64_t base = wid * PW * PC1_UNROLL; base < npix; base += stride) {
        // every lane loads (past the last pixel or band: a clamped address
        // whose value is dropped), so all loads are in flight together
        float4 x[PC1_UNROLL];
        const int col = act ? b0 : 0;
        if (base + (int64_t)PW * PC1_UNROLL <= npix) {
            const float* __restrict__ rp = cube + (base + seg) * (int64_t)bands + col;
            const int64_t step = (int64_t)PW * bands;
#pragma unroll
            for (int u = 0; u < PC1_UNROLL; ++u) x[u] = *(const float4*)(rp + u * step);
        } else {
#pragma unroll
            for (int u = 0; u < PC1_UNROLL; ++u) {
                int64_t p = base + (int64_t)u * PW + seg;
                p = p < npix ? p : npix - 1;
                x[u] = *(const float4*)(cube + p * (int64_t)bands + col);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // issue every load before the first use
#pragma unroll
        for (int u = 0; u < PC1_UNROLL; ++u) {
            const int64_t p = base + (int64_t)u * PW + seg;
            double t = 0.0;
            t = fma((double)x[u].x - mu[0], w[0], t);
            t = fma((double)x[u].y - mu[1], w[1], t);
            t = fma((double)x[u].z - mu[2], w[2], t);
            t = fma((double)x[u].w - mu[3], w[3], t);
            t = seg_sum<S>(act ? t : 0.0);
            if (p < npix) {
                lo = fmin(lo, t);
                hi = fmax(hi, t);
                if (j == 0) {
                    if (ws) ws[p] = t;
                    else out[p] = (float)t;
                }
            }
        }
    }
    if (ws) publish_minmax(lo, hi, pairs);
}

// Projection for any band count and alignment: one thread per pixel.
__global__ void __launch_bounds__(PC1_THREADS)
pc1_project_scalar(const float* __restrict__ cube, int64_t npix, int bands,
                   const double* __restrict__ mean, const double* __restrict__ vec,
                   float* __restrict__ out, double* __restrict__ ws, double* __restrict__ pairs) {
    const int64_t nthreads = (int64_t)gridDim.x * PC1_THREADS;
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int64_t p = (int64_t)blockIdx.x * PC1_THREADS + threadIdx.x; p < npix; p += nthreads) {
        const float* row = cube + p * (int64_t)bands;
        double t = 0.0;
        for (int b = 0; b < bands; ++b) t = fma((double)row[b] - mean[b], vec[b], t);
        lo = fmin(lo, t);
        hi = fmax(hi, t);
        if (ws) ws[p] = t;
        else out[p] = (float)t;
    }
    if (ws) publish_minmax(lo, hi, pairs);
}

__global__ void __launch_bounds__(PC1_THREADS)
pc1_normalise(const double* __restrict__ ws, int64_t npix, const double* __restrict__ pairs,
              int npairs, float* __restrict__ out) {
    // min and max over the frame from the projection blocks' pairs
    double l = __builtin_inf(), h = -__builtin_inf();
    for (int b = threadIdx.x; b < npairs; b += PC1_THREADS) {
        l = fmin(l, pairs[2 * b]);
        h = fmax(h, pairs[2 * b + 1]);
    }
    __shared__ double pair[2];
    block_minmax(l, h, &pair[0], &pair[1]);
    __syncthreads();
    const double lo = pair[0], hi = pair[1];
    const bool flat = !(hi > lo);
    const double range = hi - lo;
    // four pixels per thread and step, their loads issued together (one at a
    // time, each step waited for its load: the large cubes' passes were
    // latency-bound)
    const int64_t nthreads = (int64_t)gridDim.x * PC1_THREADS;
    for (int64_t p = (int64_t)blockIdx.x * PC1_THREADS + threadIdx.x; p < npix; p += 4 * nthreads) {
        double x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t pk = p + k * nthreads;
            x[k] = pk < npix ? ws[pk] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t pk = p + k * nthreads;
            if (pk < npix) out[pk] = flat ? 0.0f : (float)((x[k] - lo) / range);
        }
    }
}

}  // namespace

int pc1_max_blocks() { return PC1_MAX_BLOCKS; }

int launch_pc1_normalise(const double* ws, int64_t npix, const double* pairs, int npairs,
                         float* out, int num_cu, void* stream) {
    const int64_t nb = (npix + PC1_THREADS - 1) / PC1_THREADS;
    const int nblocks = (int)(nb < (int64_t)num_cu ? nb : (int64_t)num_cu);
    hipLaunchKernelGGL(pc1_normalise, dim3(nblocks), dim3(PC1_THREADS), 0, (hipStream_t)stream, ws,
                       npix, pairs, npairs, out);
    return (int)hipGetLastError();
}

// ---- Static scratch of knnf_pc1_noalloc: the projection blocks' (min, max)
// pairs, then the binary64 projection of up to KNNF_PC1_NOALLOC_MAX_PIXELS
// pixels.  Each device holds its own copy for the life of the process; host
// code uses the device address hipGetSymbolAddress reports for it (the
// array's name is a host-side stand-in, not a device address).
constexpr size_t kScratchHead = 16384;
static_assert(2 * PC1_MAX_BLOCKS * sizeof(double) <= kScratchHead, "pairs fit the scratch head");
constexpr size_t kScratchBytes = kScratchHead + sizeof(double) * (size_t)KNNF_PC1_NOALLOC_MAX_PIXELS;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
}  // namespace

int pc1_scratch_init(int device, void** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    // once per device, with that device current (the caller sets it)
    std::call_once(g_scratch_once[device], [device] {
        g_scratch_err[device] = hipGetSymbolAddress(&g_scratch_ptr[device], HIP_SYMBOL(scratch));
        if (g_scratch_err[device] != hipSuccess) g_scratch_ptr[device] = nullptr;
    });
    *ptr = g_scratch_ptr[device];
    return (int)g_scratch_err[device];
}

size_t pc1_scratch_head() { return kScratchHead; }

int launch_pc1(const float* cube, int64_t npix, int bands, const double* mean, const double* vec,
               float* out, double* ws, double* pairs, int num_cu, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const bool aligned = ((uintptr_t)cube & 15u) == 0;
    int64_t want;
    int blocks;
    if (aligned && bands % 4 == 0 && bands <= 256) {
        const int S = bands <= 64 ? 16 : (bands <= 128 ? 32 : 64);
        const int64_t per_block = (int64_t)(PC1_THREADS / 64) * (64 / S) * PC1_UNROLL;
        want = (npix + per_block - 1) / per_block;
        blocks = (int)(want < PC1_MAX_BLOCKS ? want : PC1_MAX_BLOCKS);
        if (S == 16)
            hipLaunchKernelGGL(pc1_project_vec4<16>, dim3(blocks), dim3(PC1_THREADS), 0, st, cube,
                               npix, bands, mean, vec, out, ws, pairs);
        else if (S == 32)
            hipLaunchKernelGGL(pc1_project_vec4<32>, dim3(blocks), dim3(PC1_THREADS), 0, st, cube,
                               npix, bands, mean, vec, out, ws, pairs);
        else
            hipLaunchKernelGGL(pc1_project_vec4<64>, dim3(blocks), dim3(PC1_THREADS), 0, st, cube,
                               npix, bands, mean, vec, out, ws, pairs);
    } else {
        want = (npix + PC1_THREADS - 1) / PC1_THREADS;
        blocks = (int)(want < PC1_MAX_BLOCKS ? want : PC1_MAX_BLOCKS);
        hipLaunchKernelGGL(pc1_project_scalar, dim3(blocks), dim3(PC1_THREADS), 0, st, cube, npix,
                           bands, mean, vec, out, ws, pairs);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ws) return (int)e;
    const int64_t nb = (npix + PC1_THREADS - 1) / PC1_THREADS;
    const int nblocks = (int)(nb < (int64_t)num_cu ? nb : (int64_t)num_cu);
    hipLaunchKernelGGL(pc1_normalise, dim3(nblocks), dim3(PC1_THREADS), 0, st, ws, npix, pairs,
                       blocks, out);
    return (int)hipGetLastError();
}

}  // namespace knnf
