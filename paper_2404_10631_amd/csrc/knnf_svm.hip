// knnf_svm.hip -- the SVM probability stage (the pixel-wise classifier whose
// probability maps the KNN filter averages), for CDNA4 (gfx950).
//
// Method (one-vs-one SVM, classification stage, Sec. II.C.1; GPU versions
// Sec. III.A.1 and III.B.1), per pixel x (a spectrum of `bands` values):
//   (i)   f[m] = sum_b w[m][b] x[b] + bias[m]  for every hyperplane m, one per
//         class pair (i, j), i < j, in lexicographic order;
//   (ii)  r[m] = 1 / (1 + exp(A[m] f[m] + B[m])), clamped to [1e-7, 1 - 1e-7]:
//         the probability of class i within the pair, 1 - r[m] that of j;
//   (iii) pairwise coupling (the second method of Wu, Lin and Weng, cited as
//         [30]): with Q[t][t] = sum_{s != t} r_st^2 and Q[t][j] = -r_jt r_tj,
//         sweep p[t] <- (p^T Q p - sum_{j != t} Q[t][j] p[j]) / Q[t][t], each
//         update followed by renormalising p, from the uniform p, until
//         max_t |(Q p)[t] - p^T Q p| < 0.005 / C or 100 sweeps.
// Every step is binary64; the probabilities are rounded once to binary32,
// pixel-major with the class fastest (the layout the filter reads).
//
// Work shape: the cube is read once (4 B per pixel and band) and everything
// else is per-pixel arithmetic, so the kernel is HBM-bound.  A block owns 256
// consecutive pixels.  It stages the cube through LDS in chunks of 32 bands:
// eight lanes cover one pixel's 128-byte piece of the chunk with 16-byte
// loads.  The hyperplane weights of the chunk (M x 32 values) are staged
// beside it.  Then each lane owns one pixel for the dot products (the weights
// read as LDS broadcasts: read straight from memory at wave-uniform addresses
// they became scalar loads whose waits lay on every wave's critical path) and
// for the coupling iteration, whose sweep count differs from pixel to pixel.
// The loads of the next chunk are in flight while the current one is used.
// The fused variant (PC1 = true) also accumulates the PC1 projection from the
// same chunks, so the pipeline's two steps before the filter read the cube
// once.  knnf_svm on cubes whose pixel rows are not whole cache lines stages
// linear runs of whole rows instead (svm_prob_lin_kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "knnf_device.h"

namespace knnf {
namespace {

constexpr int SVM_THREADS = 256;              // pixels per block
constexpr int SVM_CHUNK = 32;                 // bands per LDS stage
constexpr int SVM_STRIDE = SVM_CHUNK + 4;     // LDS row stride (floats): conflict-free 16-byte reads
constexpr int SVM_SWEEPS = 100;
constexpr double SVM_CLAMP = 1e-7;

// Hyperplane of the pair (i, j), i < j, in the order (0,1), (0,2), ..., (C-2,C-1).
template <int C>
__device__ __forceinline__ constexpr int pair_index(int i, int j) {
    return i * C - i * (i + 1) / 2 + (j - i - 1);
}

// Block-wide (min, max) of per-thread values -> pairs[2 * blockIdx.x ..].
template <int NT>
__device__ void svm_publish_minmax(double lo, double hi, double* pairs) {
    __shared__ double slo[NT / 64], shi[NT / 64];
    for (int m = 1; m < 64; m <<= 1) {
        lo = fmin(lo, __shfl_xor(lo, m));
        hi = fmax(hi, __shfl_xor(hi, m));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slo[wv] = lo;
        shi[wv] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < NT / 64; ++k) {
            lo = fmin(lo, slo[k]);
            hi = fmax(hi, shi[k]);
        }
        pairs[2 * blockIdx.x] = lo;
        pairs[2 * blockIdx.x + 1] = hi;
    }
}

// 1 / x in binary64 for the finite, normal x of the sigmoid and the coupling:
// the hardware reciprocal refined by two Newton steps (an error of an ulp or
// so, far below the 1e-6 the probabilities are held to, for a third of the
// instructions of an IEEE division).
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Weights of the chunk of bands c0 .. c0+31 for thread tid of NT: the M
// hyperplanes, then (PC1) the band averages and the eigenvector, as (m, k)
// = (e / 32, e % 32) with e = tid + NT * i; bands past the cube read as 0.
template <int NT, int M, bool PC1>
struct ChunkWeights {
    static constexpr int NWT = (M + (PC1 ? 2 : 0)) * SVM_CHUNK;
    static constexpr int NW = (NWT + NT - 1) / NT;  // per thread
    double wv[NW];
    __device__ __forceinline__ void fetch(int c0, int bands, const double* __restrict__ w,
                                          const double* __restrict__ mean,
                                          const double* __restrict__ vec) {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const int e = (int)threadIdx.x + NT * i;
            const int m = e / SVM_CHUNK;
            const int bb = c0 + (e % SVM_CHUNK);
            double x = 0.0;
            if (e < NWT && bb < bands)
                x = m < M ? w[(int64_t)m * bands + bb] : (m == M ? mean[bb] : vec[bb]);
            wv[i] = x;
        }
    }
    __device__ __forceinline__ void stage(double* wl) const {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const int e = (int)threadIdx.x + NT * i;
            if (e < NWT) wl[e] = wv[i];
        }
    }
};

// (i) for the bands c0 .. c0+nb-1 of one pixel, from its staged row (the
// chunk's first band at row[0]) and the chunk's weights wl: the decision
// values f and (PC1) the projection pj, band by band in ascending order.
template <int M, bool PC1>
__device__ __forceinline__ void svm_dot_chunk(const float* row, int nb, const double* wl,
                                              double (&f)[M], double& pj) {
    if (nb == SVM_CHUNK) {
#pragma unroll
        for (int k = 0; k < SVM_CHUNK / 4; ++k) {
            const float4 x4 = *(const float4*)(row + 4 * k);
            const double x[4] = {(double)x4.x, (double)x4.y, (double)x4.z, (double)x4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
#pragma unroll
                for (int m = 0; m < M; ++m) f[m] = fma(wl[m * SVM_CHUNK + 4 * k + e], x[e], f[m]);
                if constexpr (PC1)
                    pj = fma(x[e] - wl[M * SVM_CHUNK + 4 * k + e], wl[(M + 1) * SVM_CHUNK + 4 * k + e],
                             pj);
            }
        }
    } else {
        for (int k = 0; k < nb; ++k) {
            const double x = (double)row[k];
#pragma unroll
            for (int m = 0; m < M; ++m) f[m] = fma(wl[m * SVM_CHUNK + k], x, f[m]);
            if constexpr (PC1) pj = fma(x - wl[M * SVM_CHUNK + k], wl[(M + 1) * SVM_CHUNK + k], pj);
        }
    }
}

// Steps (ii) and (iii) for one pixel: sigmoids of the decision values f,
// then the coupling sweeps; writes the C probabilities to o.
template <int C>
__device__ __forceinline__ void svm_couple(const double (&f)[C * (C - 1) / 2],
                                           const double* __restrict__ bias,
                                           const double* __restrict__ A,
                                           const double* __restrict__ B, float* o) {
    constexpr int M = C * (C - 1) / 2;
    // (ii) binary probabilities; r[m] is that of the pair's first class (z is
    // capped where the clamp decides anyway, so 1 + exp(z) stays finite)
    double r[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const double z = fmin((f[m] + bias[m]) * A[m] + B[m], 700.0);
        const double s = rcp64(1.0 + exp(z));
        r[m] = fmin(fmax(s, SVM_CLAMP), 1.0 - SVM_CLAMP);
    }
    // (iii) coupling.  Q[t][t] sums r_st^2 over s in ascending order;
    // the off-diagonal Q[t][j] = -r_jt r_tj is the same for (t, j) and (j, t).
    double qtt[C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < C; ++u) {
            if (u == t) continue;
            const double rut = u < t ? r[pair_index<C>(u, t)] : 1.0 - r[pair_index<C>(t, u)];
            s = s + rut * rut;
        }
        qtt[t] = s;
    }
    double qo[M];
#pragma unroll
    for (int m = 0; m < M; ++m) qo[m] = -((1.0 - r[m]) * r[m]);
    auto Q = [&](int t, int j) -> double {
        return t == j ? qtt[t] : t < j ? qo[pair_index<C>(t, j)] : qo[pair_index<C>(j, t)];
    };

    // The sweep keeps Q p and p^T Q p up to date instead of recomputing
    // them: the new p[t] equals p[t] + d with d = (p^T Q p - (Q p)[t]) / Q[t][t];
    // before renormalising, Q p gains d times column t of Q and p^T Q p gains
    // 2 d (Q p)[t] + d^2 Q[t][t]; renormalising divides p and Q p by 1 + d
    // (the sum of p before it) and p^T Q p by its square.  Same fixed-point
    // step as the plain form, O(C) per update instead of O(C^2).
    double p[C], qp[C], rq[C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
        p[t] = 1.0 / C;
        rq[t] = rcp64(qtt[t]);
    }
    double pqp = 0.0;
#pragma unroll
    for (int t = 0; t < C; ++t) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < C; ++j) s = fma(Q(t, j), p[j], s);
        qp[t] = s;
        pqp = fma(p[t], s, pqp);
    }
    const double eps = 0.005 / C;
    for (int sweep = 0; sweep < SVM_SWEEPS; ++sweep) {
        double err = 0.0;
#pragma unroll
        for (int t = 0; t < C; ++t) err = fmax(err, fabs(qp[t] - pqp));
        if (!(err >= eps)) break;
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const double d = (pqp - qp[t]) * rq[t];
            const double inv = rcp64(1.0 + d);
            pqp = fma(d, fma(d, qtt[t], 2.0 * qp[t]), pqp) * inv * inv;
#pragma unroll
            for (int j = 0; j < C; ++j) qp[j] = fma(d, Q(j, t), qp[j]) * inv;
            p[t] += d;
#pragma unroll
            for (int j = 0; j < C; ++j) p[j] *= inv;
        }
    }
#pragma unroll
    for (int t = 0; t < C; ++t) o[t] = (float)p[t];
}

// A pixel's outputs once its decision values f and projection pj are
// complete (every thread of the block calls it).
template <int C, int NT, bool PC1>
__device__ __forceinline__ void svm_finish(int64_t pix, int64_t npix,
                                           const double (&f)[C * (C - 1) / 2], double pj,
                                           const double* __restrict__ bias,
                                           const double* __restrict__ A,
                                           const double* __restrict__ B, float* __restrict__ out,
                                           float* __restrict__ band, double* __restrict__ ws,
                                           double* __restrict__ pairs) {
    const bool in = pix < npix;
    if constexpr (PC1) {
        if (ws) {
            // every thread of the block takes part (pixels past the frame add nothing)
            svm_publish_minmax<NT>(in ? pj : __builtin_inf(), in ? pj : -__builtin_inf(), pairs);
            if (in) ws[pix] = pj;
        } else if (in) {
            band[pix] = (float)pj;
        }
    }
    if (in) svm_couple<C>(f, bias, A, B, out + pix * C);
}

// PC1 = true also accumulates the PC1 projection of each
// pixel (Sec. II.C.2: the cube centred by the band averages, times the first
// eigenvector), band by band in ascending order in binary64, from the same
// staged chunks: the step before the filter reads the cube once for both of
// its outputs.
template <int C, bool VEC, bool PC1>
__global__ void __launch_bounds__(SVM_THREADS)
svm_prob_kernel(const float* __restrict__ cube, int64_t npix, int bands,
                const double* __restrict__ w, const double* __restrict__ bias,
                const double* __restrict__ A, const double* __restrict__ B,
                float* __restrict__ out, const double* __restrict__ mean,
                const double* __restrict__ vec, float* __restrict__ band,
                double* __restrict__ ws, double* __restrict__ pairs) {
    constexpr int M = C * (C - 1) / 2;
    using Weights = ChunkWeights<SVM_THREADS, M, PC1>;
    __shared__ __attribute__((aligned(16))) float tile[SVM_THREADS * SVM_STRIDE];
    __shared__ __attribute__((aligned(16))) double wl[Weights::NWT];
    const int tid = threadIdx.x;
    const int64_t first = (int64_t)blockIdx.x * SVM_THREADS;
    const int64_t last = npix - 1;

    double f[M];
#pragma unroll
    for (int m = 0; m < M; ++m) f[m] = 0.0;
    double pj = 0.0;  // PC1 projection
    const float* row = tile + tid * SVM_STRIDE;
    // Staging of cube[first .. first+255][c0 .. c0+31] (rows past the frame
    // repeat its last pixel, bands past the cube read as 0).  The next chunk
    // is loaded into registers while the current one is used from LDS.
    // 16-byte path: lane (q, r0) loads column 4q of rows r0, r0 + 32, ...
    // Scalar path: lane (q, r0) loads band q of rows r0, r0 + 8, ...
    constexpr int NLOAD = VEC ? 8 : 32;
    using Piece = typename std::conditional<VEC, float4, float>::type;
    Piece v[NLOAD];
    Weights wt;
    const int q = VEC ? (tid & 7) : (tid & 31);
    const int r0 = VEC ? (tid >> 3) : (tid >> 5);
    constexpr int RSTEP = VEC ? 32 : 8;
    auto fetch = [&](int c0) {
        const int b = c0 + (VEC ? 4 * q : q);
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            int64_t p = first + r0 + RSTEP * i;
            p = p < npix ? p : last;
            if constexpr (VEC)
                v[i] = b < bands ? *(const float4*)(cube + p * (int64_t)bands + b)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
            else
                v[i] = b < bands ? cube[p * (int64_t)bands + b] : 0.f;
        }
        wt.fetch(c0, bands, w, mean, vec);
    };
    fetch(0);
    for (int c0 = 0; c0 < bands; c0 += SVM_CHUNK) {
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            if constexpr (VEC)
                *(float4*)(tile + (r0 + RSTEP * i) * SVM_STRIDE + 4 * q) = v[i];
            else
                tile[(r0 + RSTEP * i) * SVM_STRIDE + q] = v[i];
        }
        wt.stage(wl);
        __syncthreads();
        if (c0 + SVM_CHUNK < bands) fetch(c0 + SVM_CHUNK);
        svm_dot_chunk<M, PC1>(row, min(SVM_CHUNK, bands - c0), wl, f, pj);
        __syncthreads();
    }
    svm_finish<C, SVM_THREADS, PC1>(first + tid, npix, f, pj, bias, A, B, out, band, ws, pairs);
}

// knnf_svm on cubes whose pixel rows are not whole 128-byte lines (bands * 4
// not a multiple of 128, e.g. 100 bands): per-pixel band chunks split lines
// between chunks and between neighbouring pixels, and a line evicted between
// its two uses is fetched twice (1.6x the cube's bytes on the 1000 x 1000 x
// 100 cube).  This variant reads the block's 256 pixels as 4 linear runs of
// 64 whole pixel rows (each line once, in full), staged in LDS with a row
// stride of S = 16 (mod 32) floats.  Four lanes share a pixel of a run: lane
// part t takes the float4 pieces t, t+4, ... of the row (a quarter-
// wavefront's 16-byte reads then cover all 64 banks), and a butterfly over
// the four lanes completes the pixel's sums.  Lane part t keeps the sums of
// run t, so thread 4 pl + t owns pixel 64 t + pl of the block for the
// sigmoids and the coupling.  All weights are staged once, piece by piece.
// The sums run in a different order than band by band (four interleaved
// partial sums), which moves the binary64 results by rounding only.  (With
// the PC1 projection added, the band-chunk kernel above measured faster, so
// the fused call keeps it.)
constexpr int LIN_RUN = 64;                     // pixels per linear run
constexpr int LIN_MAX_BANDS = 128;
constexpr int LIN_MAX_WEIGHTS = 2048;           // doubles of weights staged at once
constexpr int LIN_MAX_C = 4;                    // more classes: the coupling's registers spill

__host__ __device__ constexpr int lin_stride(int bands) {
    return ((bands + 15) / 32) * 32 + 16;       // smallest S >= bands with S = 16 (mod 32)
}
// Doubles per piece of staged weights: the smallest >= 4 M that is 8 (mod
// 16), so the four lanes of a quad (pieces k .. k+3) read on disjoint banks.
__host__ __device__ constexpr int lin_piece(int m) { return ((4 * m + 7) / 16) * 16 + 8; }

__device__ __forceinline__ double quad_sum(double v) {
    // sum over the 4 lanes of a quad (xor 1, then xor 2), every lane gets it
    int lo = __double2loint(v), hi = __double2hiint(v);
    v += __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false));
    lo = __double2loint(v);
    hi = __double2hiint(v);
    return v + __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x4E, 0xF, 0xF, false),
                                __builtin_amdgcn_update_dpp(lo, lo, 0x4E, 0xF, 0xF, false));
}

template <int C>
__global__ void __launch_bounds__(SVM_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
svm_prob_lin_kernel(const float* __restrict__ cube, int64_t npix, int bands,
                    const double* __restrict__ w, const double* __restrict__ bias,
                    const double* __restrict__ A, const double* __restrict__ B,
                    float* __restrict__ out) {
    constexpr int M = C * (C - 1) / 2;
    constexpr int PS = lin_piece(M);
    constexpr int NLD = LIN_RUN * LIN_MAX_BANDS / 4 / SVM_THREADS;  // float4 loads per thread, max
    extern __shared__ __attribute__((aligned(16))) double lin_smem[];
    double* wl = lin_smem;                                 // bands / 4 pieces x PS
    const int S = lin_stride(bands);
    float* tile = (float*)(lin_smem + (bands >> 2) * PS);  // LIN_RUN x S
    const int tid = threadIdx.x;
    const int pl = tid >> 2, t = tid & 3;
    const int64_t first = (int64_t)blockIdx.x * SVM_THREADS;
    const int b4 = bands >> 2;                             // float4 pieces per pixel
    const int nq = LIN_RUN * b4;                           // pieces per run
    const float inv_b4 = 1.0f / (float)b4;

    // weights by piece: wl[k * PS + m * 4 + e] is hyperplane m at band
    // 4 k + e, so a piece's M x 4 weights are contiguous (16-byte LDS reads
    // at constant offsets)
    for (int e = tid; e < M * bands; e += SVM_THREADS) {
        const int m = e / bands, bb = e - m * bands;
        wl[(bb >> 2) * PS + m * 4 + (bb & 3)] = w[(int64_t)m * bands + bb];
    }

    // run r: pixels first + 64 r .. +63, read as one linear range of pieces
    // (pixels past the cube read as 0 and are never written)
    float4 v[NLD];
    auto fetch = [&](int r) {
        const int64_t p0 = first + (int64_t)LIN_RUN * r;
        const char* src = (const char*)(cube + p0 * (int64_t)bands);
        // pieces inside the run and the cube
        const int lim = (int)min((int64_t)nq, max((int64_t)0, npix - p0) * b4);
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int q = tid + SVM_THREADS * i;
            v[i] = q < lim ? *(const float4*)(src + (uint32_t)q * 16u) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    double own[M];
#pragma unroll
    for (int m = 0; m < M; ++m) own[m] = 0.0;
    fetch(0);
#pragma unroll 1
    for (int r = 0; r < SVM_THREADS / LIN_RUN; ++r) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int q = tid + SVM_THREADS * i;
            if (q < nq) {
                // piece q is pixel q / b4 of the run, bands 4 (q % b4) ..
                const int px = (int)(((float)q + 0.5f) * inv_b4);
                *(float4*)(tile + px * S + 4 * (q - px * b4)) = v[i];
            }
        }
        __syncthreads();
        if (r + 1 < SVM_THREADS / LIN_RUN) fetch(r + 1);
        double f[M];
#pragma unroll
        for (int m = 0; m < M; ++m) f[m] = 0.0;
        const float* row = tile + pl * S;
#pragma unroll 1
        for (int k = t; k < b4; k += 4) {
            const float4 xa = *(const float4*)(row + 4 * k);
            const double x[4] = {(double)xa.x, (double)xa.y, (double)xa.z, (double)xa.w};
            const double* wk = wl + k * PS;
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int m = 0; m < M; ++m) f[m] = fma(wk[m * 4 + e], x[e], f[m]);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            f[m] = quad_sum(f[m]);
            own[m] = t == r ? f[m] : own[m];
        }
        __syncthreads();
    }
    svm_finish<C, SVM_THREADS, false>(first + LIN_RUN * t + pl, npix, own, 0.0, bias, A, B, out,
                                      nullptr, nullptr, nullptr);
}

struct SvmArgs {
    const float* cube;
    int64_t npix;
    int bands;
    const double *w, *bias, *A, *B, *mean, *vec;
    float *out, *band;
    double *ws, *pairs;
};

template <int C, bool PC1>
int launch_c(const SvmArgs& a, void* stream, int* nblocks) {
    const hipStream_t st = (hipStream_t)stream;
    const int64_t blocks = (a.npix + SVM_THREADS - 1) / SVM_THREADS;
    const bool vec = a.bands % 4 == 0 && ((uintptr_t)a.cube & 15) == 0;
    bool lin = false;
    if constexpr (C <= LIN_MAX_C && !PC1) {
        constexpr int M = C * (C - 1) / 2;
        const int wd = a.bands / 4 * lin_piece(M);       // doubles of staged weights
        lin = vec && (a.bands * 4) % 128 != 0 && a.bands <= LIN_MAX_BANDS && wd <= LIN_MAX_WEIGHTS;
        if (lin) {
            const size_t lds = (size_t)wd * 8 + (size_t)LIN_RUN * lin_stride(a.bands) * 4;
            hipLaunchKernelGGL((svm_prob_lin_kernel<C>), dim3((uint32_t)blocks), dim3(SVM_THREADS),
                               lds, st, a.cube, a.npix, a.bands, a.w, a.bias, a.A, a.B, a.out);
        }
    }
    if (!lin && vec)
        hipLaunchKernelGGL((svm_prob_kernel<C, true, PC1>), dim3((uint32_t)blocks), dim3(SVM_THREADS),
                           0, st, a.cube, a.npix, a.bands, a.w, a.bias, a.A, a.B, a.out, a.mean,
                           a.vec, a.band, a.ws, a.pairs);
    else if (!lin)
        hipLaunchKernelGGL((svm_prob_kernel<C, false, PC1>), dim3((uint32_t)blocks), dim3(SVM_THREADS),
                           0, st, a.cube, a.npix, a.bands, a.w, a.bias, a.A, a.B, a.out, a.mean,
                           a.vec, a.band, a.ws, a.pairs);
    if (nblocks) *nblocks = (int)blocks;
    return (int)hipGetLastError();
}

template <bool PC1>
int launch_classes(int classes, const SvmArgs& a, void* stream, int* nblocks) {
    switch (classes) {
        case 2: return launch_c<2, PC1>(a, stream, nblocks);
        case 3: return launch_c<3, PC1>(a, stream, nblocks);
        case 4: return launch_c<4, PC1>(a, stream, nblocks);
        case 5: return launch_c<5, PC1>(a, stream, nblocks);
        case 6: return launch_c<6, PC1>(a, stream, nblocks);
        case 7: return launch_c<7, PC1>(a, stream, nblocks);
        case 8: return launch_c<8, PC1>(a, stream, nblocks);
        default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace

int launch_svm(const float* cube, int64_t npix, int bands, int classes, const double* w,
               const double* bias, const double* A, const double* B, float* out, void* stream) {
    const SvmArgs a{cube, npix, bands, w, bias, A, B, nullptr, nullptr, out, nullptr, nullptr, nullptr};
    return launch_classes<false>(classes, a, stream, nullptr);
}

int svm_pixels_per_block() { return SVM_THREADS; }

int launch_svm_pc1(const float* cube, int64_t npix, int bands, int classes, const double* w,
                   const double* bias, const double* A, const double* B, const double* mean,
                   const double* vec, float* out, float* band, double* ws, double* pairs,
                   int* nblocks, void* stream) {
    const SvmArgs a{cube, npix, bands, w, bias, A, B, mean, vec, out, band, ws, pairs};
    return launch_classes<true>(classes, a, stream, nblocks);
}

}  // namespace knnf
