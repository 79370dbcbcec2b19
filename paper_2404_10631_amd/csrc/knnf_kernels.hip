// knnf_kernels.hip -- KNN filtering kernels for CDNA4 (gfx950), wave64.
//
// Method (Lazcano et al., Sec. II.C.3): for each pixel q, find the K nearest
// window pixels under the Eq. 1 distance of the features (I, lambda*row,
// lambda*col) and average their class probabilities (Eq. 2); the class map is
// the argmax of the summed probabilities.  The window is R rows above and below
// q at full width, clipped at the frame edges (Sec. III.A.3).
//
// Arithmetic contract (identical bits to any other conforming implementation):
//   fr(x) = fl32(lambda * (float)x)
//   a = fl32(fr(r) - fr(i)), b = fl32(fr(c) - fr(j)), e = fl32(I_q - I_p)
//   d = fmaf(e, e, fmaf(b, b, fl32(a * a)))
//   order: key = (bits(d) << 32) | (i*W + j), ascending (d >= +0, so the bit
//   pattern orders like the value)
//   S_c = ((+0 + P[n_0][c]) + P[n_1][c]) + ... in key order; O_c = fl32(S_c/K)
//   class = lowest c with maximal S_c
// The file is built with -ffp-contract=off, so every * and - below is one
// binary32 operation and fmaf is the only fused operation.
//
// Work decomposition (not the paper's; designed for 64-wide wavefronts):
//   * One wavefront task = a vertical strip of Q query pixels at one column c,
//     rows r0 .. r0+Q-1.  Sharing the column makes b depend on the candidate
//     column only, so it is computed once per 64-column chunk.
//   * Lanes sweep candidates: at each step lane L holds candidate column
//     j = j0 + L of one window row; the row's I values are one coalesced
//     256-byte load shared by all Q queries of the strip.
//   * Selection per query is cooperative across the wavefront:
//       pass A: the 64 candidates of a compact block around q (8 rows x 8
//       columns where the window allows) are sorted with a 64-lane bitonic
//       network; the K-th key is an upper bound tau on the final K-th key.
//       pass B: every window candidate is tested against tau (one compare per
//       pair); the rare survivors are appended to a per-query LDS buffer with
//       ballot + mbcnt.  A full buffer is sorted and merged into the query's
//       sorted top-K list, which tightens tau.
//   * The tail is fused: gather the K neighbours' probabilities (L2-resident),
//     sum in key order, divide, argmax, and write the outputs.
//   * Pruned search (optional, bit-identical): candidate rows and column chunks
//     whose spatial part of Eq. 1 already exceeds tau are skipped; all terms of
//     Eq. 1 are non-negative and rounding is monotone, so a skipped candidate
//     always has d > tau.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "knnf_device.h"

namespace knnf {
namespace {

constexpr uint64_t KEY_INF = ~0ull;
constexpr int WAVE = 64;
constexpr int A2ROWS = 32;  // window rows per block of the LDS a2 table
constexpr int MAXC = 16;

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniu(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uniu((uint32_t)(v >> 32)) << 32) | (uint64_t)uniu((uint32_t)v);
}
__device__ __forceinline__ float unif(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int mbcnt(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// Orders LDS traffic of one wavefront (lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ uint32_t shfl(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    return ((uint64_t)shfl((uint32_t)(v >> 32), src) << 32) | (uint64_t)shfl((uint32_t)v, src);
}
__device__ __forceinline__ uint64_t make_key(float d, int idx) {
    return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)(uint32_t)idx;
}

// Ascending bitonic sort of one 64-bit key per lane across the wavefront.
__device__ __forceinline__ uint64_t sort64(uint64_t key) {
    const int L = lane_id();
#pragma unroll
    for (int k = 2; k <= WAVE; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t other = shfl64(key, L ^ j);
            const bool up = (k == WAVE) || ((L & k) == 0);
            const bool lower = (L & j) == 0;
            const bool take = (lower == up) ? (other < key) : (key < other);
            key = take ? other : key;
        }
    }
    return key;
}

// a, b ascending across lanes; returns the 64 smallest of both, ascending.
__device__ __forceinline__ uint64_t merge64(uint64_t a, uint64_t b) {
    const int L = lane_id();
    const uint64_t rb = shfl64(b, WAVE - 1 - L);
    uint64_t key = rb < a ? rb : a;  // bitonic: the 64 smallest of a and b
#pragma unroll
    for (int j = WAVE / 2; j > 0; j >>= 1) {
        const uint64_t other = shfl64(key, L ^ j);
        const bool lower = (L & j) == 0;
        const bool take = lower ? (other < key) : (key < other);
        key = take ? other : key;
    }
    return key;
}

template <int Q>
struct alignas(16) WaveState {
    uint64_t list[Q][WAVE];   // sorted top-K per query (lanes >= K hold KEY_INF)
    uint64_t pend[Q][WAVE];   // candidates that passed the tau test, unsorted
    float a2t[A2ROWS][Q];     // fl32(a*a) for a block of window rows
    uint64_t tau[Q];          // current upper bound on the K-th key
    float iq[Q];              // I of each query pixel
    float sums[Q][MAXC];      // class sums for the argmax
    int cnt[Q];               // pending entries
    int listn[Q];             // valid list entries (<= K)
};

// Row coordinate feature fr(x) = fl32(lambda * (float)x).
__device__ __forceinline__ float feat(float lam, int x) { return lam * (float)x; }

// Merge query q's pending buffer into its top-K list and tighten tau.
template <int Q>
__device__ void flush_query(WaveState<Q>& S, int q, int K) {
    const int L = lane_id();
    wave_sync();
    const int cnt = uni(S.cnt[q]);
    const int listn = uni(S.listn[q]);
    uint64_t p = (L < cnt) ? S.pend[q][L] : KEY_INF;
    p = sort64(p);
    uint64_t l = p;
    if (listn > 0) l = merge64(S.list[q][L], p);
    if (L >= K) l = KEY_INF;
    S.list[q][L] = l;
    const int nl = min(K, listn + cnt);
    const uint64_t kth = uni64(shfl64(l, K - 1));
    const uint64_t tau = uni64(S.tau[q]);
    wave_sync();
    if (L == 0) {
        S.listn[q] = nl;
        S.cnt[q] = 0;
        if (nl == K && kth < tau) S.tau[q] = kth;
    }
    wave_sync();
}

// Append the lanes with key <= tau of query q to its pending buffer.
template <int Q>
__device__ void push_survivors(WaveState<Q>& S, int q, int K, bool valid, uint64_t key) {
    const int L = lane_id();
    uint64_t tau = uni64(S.tau[q]);
    bool ok = valid && key <= tau;
    uint64_t m = ballot(ok);
    if (m == 0) return;
    int cnt = uni(S.cnt[q]);
    int n = __builtin_popcountll(m);
    if (cnt + n > WAVE) {
        flush_query(S, q, K);
        tau = uni64(S.tau[q]);
        ok = valid && key <= tau;
        m = ballot(ok);
        n = __builtin_popcountll(m);
        cnt = 0;
    }
    if (ok) S.pend[q][cnt + mbcnt(m)] = key;
    wave_sync();
    if (L == 0) S.cnt[q] = cnt + n;
    wave_sync();
}

// Pass A for query q: tau = K-th key of a compact block of window candidates.
template <int Q>
__device__ void seed_query(WaveState<Q>& S, const FrameDesc& f, int q, int r, int c) {
    const int L = lane_id();
    const int H = f.H, W = f.W, R = f.R, K = f.K;
    const float lam = f.lambda;
    const int i0 = max(0, r - R), i1 = min(H - 1, r + R);
    const int nr = i1 - i0 + 1;
    int lbr = 0;  // log2 of block rows: 8, 4, 2 or 1 rows
    while (lbr < 3 && (2 << lbr) <= nr) ++lbr;
    const int br = 1 << lbr;
    const int lbc = 6 - lbr;
    const int bc = 1 << lbc;
    const int rb = min(max(r - br / 2, i0), i1 - br + 1);
    const int cb = max(0, min(c - bc / 2, W - bc));
    const int i = rb + (L >> lbc);
    const int j = cb + (L & (bc - 1));
    const bool valid = j < W;
    uint64_t key = KEY_INF;
    if (valid) {
        const float a = feat(lam, r) - feat(lam, i);
        const float b = feat(lam, c) - feat(lam, j);
        const float e = S.iq[q] - f.pc1[(size_t)i * W + j];
        const float d = fmaf(e, e, fmaf(b, b, a * a));
        key = make_key(d, i * W + j);
    }
    key = sort64(key);
    const uint64_t kth = uni64(shfl64(key, K - 1));
    wave_sync();
    if (L == 0) {
        S.tau[q] = kth;
        S.cnt[q] = 0;
        S.listn[q] = 0;
    }
    wave_sync();
}

// Process one strip: queries (r0 + q, c) for q < nq.
template <int Q, bool PRUNE>
__device__ void process_strip(WaveState<Q>& S, const FrameDesc& f, int c, int r0) {
    const int L = lane_id();
    const int H = f.H, W = f.W, R = f.R, K = f.K, C = f.C;
    const float lam = f.lambda;
    const int nq = min(Q, H - r0);
    const float* __restrict__ pc1 = f.pc1;

    // ---- query values (uniform, kept in VGPRs to spare scalar registers)
    if (L < Q) S.iq[L] = (L < nq) ? pc1[(size_t)(r0 + L) * W + c] : 0.0f;
    wave_sync();
    float iq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) iq[q] = S.iq[q];

    // ---- pass A: initial bounds
    for (int q = 0; q < nq; ++q) seed_query(S, f, q, r0 + q, c);

    uint32_t tauhi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) tauhi[q] = q < nq ? (uint32_t)(S.tau[q] >> 32) : 0u;

    // ---- pass B: every window candidate, chunks of 64 columns centred on c
    const float fcq = feat(lam, c);
    const int rlo = max(0, r0 - R);
    const int rhi = min(H - 1, r0 + nq - 1 + R);
    const int nright = (W + 31 - c) / WAVE;  // chunks m = 1..nright exist to the right
    const int nleft = (c + 31) / WAVE;       // chunks m = -1..-nleft exist to the left
    const int nsteps = 2 * max(nleft, nright);
    const float qnan = __int_as_float(0x7fc00000);
    const float pinf = __int_as_float(0x7f800000);

    for (int t = 0; t <= nsteps; ++t) {
        const int m = (t & 1) ? (t + 1) / 2 : -(t / 2);
        if (m > nright || -m > nleft) continue;
        const int jbase = c - 32 + WAVE * m;
        const int j = jbase + L;
        const bool valid = (unsigned)j < (unsigned)W;
        const float b = fcq - feat(lam, j);

        for (int blk = rlo; blk <= rhi; blk += A2ROWS) {
            const int nb = min(A2ROWS, rhi - blk + 1);
            // a2 table for rows blk .. blk+A2ROWS-1; +inf marks a row outside
            // query q's window (or a query beyond the frame), which makes the
            // inner loop branch-free: d = +inf never passes a finite bound.
            wave_sync();
            for (int u = L; u < A2ROWS * Q; u += WAVE) {
                const int rr = u / Q, q = u % Q;
                const int r = r0 + q, i = blk + rr;
                const bool act = q < nq && i >= r - R && i <= r + R;
                const float a = feat(lam, r) - feat(lam, i);
                S.a2t[rr][q] = act ? a * a : pinf;
            }
            wave_sync();

            float ip_next = valid ? pc1[(size_t)blk * W + j] : qnan;
            for (int rr = 0; rr < nb; ++rr) {
                const int i = blk + rr;
                const float ip = ip_next;
                if (rr + 1 < nb) ip_next = valid ? pc1[(size_t)(i + 1) * W + j] : qnan;
                float a2[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) a2[q] = S.a2t[rr][q];
                uint64_t anyb = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const float e = iq[q] - ip;
                    const float tt = fmaf(b, b, a2[q]);
                    const float d = fmaf(e, e, tt);
                    anyb |= ballot(__float_as_uint(d) <= tauhi[q]);
                }
                if (anyb) {
                    for (int q = 0; q < nq; ++q) {
                        const float a2q = unif(S.a2t[rr][q]);
                        if (__float_as_uint(a2q) == 0x7f800000u) continue;  // row outside q's window
                        const float e = S.iq[q] - ip;
                        const float d = fmaf(e, e, fmaf(b, b, a2q));
                        push_survivors(S, q, K, valid, make_key(d, i * W + j));
                    }
#pragma unroll
                    for (int q = 0; q < Q; ++q)
                        if (q < nq) tauhi[q] = (uint32_t)(S.tau[q] >> 32);
                }
            }
        }
    }

    // ---- final merge: list = top-K of each query
    for (int q = 0; q < nq; ++q)
        if (uni(S.cnt[q]) > 0) flush_query(S, q, K);
    wave_sync();

    // ---- outputs: neighbour lists
    const int npx = H * W;
    for (int q = 0; q < nq; ++q) {
        const size_t pix = (size_t)(r0 + q) * W + c;
        const uint64_t key = S.list[q][L];
        if (L < K) {
            if (f.out_nbr) f.out_nbr[pix * K + L] = (int32_t)(uint32_t)key;
            if (f.out_dist) f.out_dist[pix * K + L] = __uint_as_float((uint32_t)(key >> 32));
        }
    }

    // ---- Eq. 2: sums in neighbour order, one lane per (query, class)
    const float* __restrict__ prob = f.prob;
    for (int p = L; p < nq * C; p += WAVE) {
        const int q = p / C, cl = p - q * C;
        float s = 0.0f;
        for (int k = 0; k < K; ++k) {
            const uint32_t idx = (uint32_t)S.list[q][k];
            if (idx < (uint32_t)npx) s = s + prob[(size_t)idx * C + cl];
        }
        S.sums[q][cl] = s;
        const size_t pix = (size_t)(r0 + q) * W + c;
        f.out_prob[pix * C + cl] = s / (float)K;
    }
    wave_sync();
    if (L < nq) {
        int best = 0;
        float bs = S.sums[L][0];
        for (int cl = 1; cl < C; ++cl) {
            const float v = S.sums[L][cl];
            if (v > bs) { bs = v; best = cl; }
        }
        f.out_class[(size_t)(r0 + L) * W + c] = best;
    }
    wave_sync();
}

// Bijective remap of block ids so that each XCD (blocks are dealt round-robin
// to the 8 XCDs) works on a contiguous range of strips, which share window
// rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int full = nb & ~7;
    if (b >= full) return b;
    const int per = full >> 3;
    return (b & 7) * per + (b >> 3);
}

template <int Q, int WPB, bool PRUNE>
__global__ void __launch_bounds__(WPB * WAVE) filter_frame_kernel(FrameDesc f) {
    __shared__ WaveState<Q> lds[WPB];
    const int w = uni((int)(threadIdx.x >> 6));
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int strips_per_col = (f.H + Q - 1) / Q;
    const long long s = (long long)b * WPB + w;
    if (s >= (long long)strips_per_col * f.W) return;
    const int band = (int)(s / f.W);
    const int c = (int)(s - (long long)band * f.W);
    process_strip<Q, PRUNE>(lds[w], f, c, band * Q);
}

// Persistent batched kernel: each wavefront claims strip tasks from a global
// counter until all tasks of all frames are taken.  Every wavefront leaves the
// loop after one failed claim, so the grid always drains.
template <int Q, int WPB, bool PRUNE>
__global__ void __launch_bounds__(WPB * WAVE)
filter_batch_kernel(const FrameDesc* __restrict__ frames, const uint32_t* __restrict__ task_start,
                    uint32_t nframes, uint32_t total_tasks, uint32_t* counter) {
    __shared__ WaveState<Q> lds[WPB];
    const int w = uni((int)(threadIdx.x >> 6));
    const int L = lane_id();
    for (;;) {
        uint32_t t = 0;
        if (L == 0) t = atomicAdd(counter, 1u);
        t = uniu(t);  // lane 0's claim
        if (t >= total_tasks) break;
        // frame f with task_start[f] <= t < task_start[f+1]
        uint32_t lo = 0, hi = nframes;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (task_start[mid] <= t) lo = mid; else hi = mid;
        }
        const FrameDesc f = frames[lo];
        const uint32_t s = t - task_start[lo];
        const int band = (int)(s / (uint32_t)f.W);
        const int c = (int)(s - (uint32_t)band * (uint32_t)f.W);
        process_strip<Q, PRUNE>(lds[w], f, c, band * Q);
    }
}

template <int Q, int WPB, bool PRUNE>
int launch_frame_t(const FrameDesc& f, hipStream_t st) {
    const long long strips = (long long)((f.H + Q - 1) / Q) * f.W;
    const long long blocks = (strips + WPB - 1) / WPB;
    hipLaunchKernelGGL((filter_frame_kernel<Q, WPB, PRUNE>), dim3((unsigned)blocks),
                       dim3(WPB * WAVE), 0, st, f);
    return (int)hipGetLastError();
}

template <int Q, int WPB, bool PRUNE>
int launch_batch_t(const FrameDesc* fr, const uint32_t* ts, uint32_t n, uint32_t tot,
                   uint32_t* ctr, int grid, hipStream_t st) {
    hipLaunchKernelGGL((filter_batch_kernel<Q, WPB, PRUNE>), dim3((unsigned)grid),
                       dim3(WPB * WAVE), 0, st, fr, ts, n, tot, ctr);
    return (int)hipGetLastError();
}

template <int Q, int WPB, bool PRUNE>
int occupancy_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, filter_batch_kernel<Q, WPB, PRUNE>,
                                                     WPB * WAVE, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

#define KNNF_DISPATCH(FN, ...)                                                         \
    do {                                                                               \
        const bool pr = cfg.pruned != 0;                                               \
        switch (cfg.queries * 16 + cfg.waves) {                                        \
        case 4 * 16 + 1: return pr ? FN<4, 1, true>(__VA_ARGS__) : FN<4, 1, false>(__VA_ARGS__);   \
        case 4 * 16 + 2: return pr ? FN<4, 2, true>(__VA_ARGS__) : FN<4, 2, false>(__VA_ARGS__);   \
        case 4 * 16 + 4: return pr ? FN<4, 4, true>(__VA_ARGS__) : FN<4, 4, false>(__VA_ARGS__);   \
        case 8 * 16 + 1: return pr ? FN<8, 1, true>(__VA_ARGS__) : FN<8, 1, false>(__VA_ARGS__);   \
        case 8 * 16 + 2: return pr ? FN<8, 2, true>(__VA_ARGS__) : FN<8, 2, false>(__VA_ARGS__);   \
        case 8 * 16 + 4: return pr ? FN<8, 4, true>(__VA_ARGS__) : FN<8, 4, false>(__VA_ARGS__);   \
        case 16 * 16 + 1: return pr ? FN<16, 1, true>(__VA_ARGS__) : FN<16, 1, false>(__VA_ARGS__); \
        case 16 * 16 + 2: return pr ? FN<16, 2, true>(__VA_ARGS__) : FN<16, 2, false>(__VA_ARGS__); \
        default: return (int)hipErrorInvalidValue;                                     \
        }                                                                              \
    } while (0)

}  // namespace

int launch_filter_frame(const FrameDesc& f, const LaunchCfg& cfg, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    KNNF_DISPATCH(launch_frame_t, f, st);
}

int launch_filter_batch(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        uint32_t nframes, uint32_t total_tasks, uint32_t* d_counter,
                        const LaunchCfg& cfg, int grid_blocks, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    KNNF_DISPATCH(launch_batch_t, d_frames, d_task_start, nframes, total_tasks, d_counter,
                  grid_blocks, st);
}

int persistent_blocks_per_cu(const LaunchCfg& cfg) { KNNF_DISPATCH(occupancy_t); }

__global__ void zero_u32_kernel(uint32_t* p) { *p = 0u; }

int launch_zero_counter(uint32_t* d_counter, void* stream) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, d_counter);
    return (int)hipGetLastError();
}

}  // namespace knnf
