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
//   * One wavefront task = a tile of QR x QC query pixels (default 1 x 8).
//     Per-query state lives in VGPRs and a small per-wavefront LDS block.
//   * pass A (bound): the 128 candidates (8-query tiles; 64 for 16-query
//     tiles) of a compact block around each query (8 rows x 16 columns where
//     the window allows) are evaluated and sorted for all Q queries at once
//     by a segmented bitonic network; any distance with at least K block
//     candidates at or below it bounds the query's final K-th key from
//     above.  8-query tiles sort the block as two interleaved groups of 64
//     (16-bit keys rounded up, both groups in one packed network) and take
//     the larger of the groups' ceil(K/2)-th keys; other tiles take the
//     block's K-th distance.  The larger block's tighter bound lets fewer
//     candidates through the scan than an 8 x 8 block's.
//   * pass B (collect): candidates with d <= d_K are appended to a per-query
//     LDS buffer with ballot + mbcnt; a full buffer is merged into a sorted
//     per-query list, which tightens the bound.  Two scans:
//       - pruned (default): 16-row x 4-column patches swept outward from the
//         tile over the rows and column steps whose spatial lower bound is
//         within some query's bound (bit-identical: every term of Eq. 1 is
//         >= 0 and rounding is monotone);
//       - exhaustive: every window row in 64-column chunks, four rows per
//         group, one coalesced 256-byte load per row shared by all queries.
//   * Final selection: one segmented sort of 32-bit packed keys (distance
//     bits | buffer slot) with exact (d, idx) repair of equal distance parts.
//   * The tail is fused: gather the K neighbours' probabilities (L2-resident),
//     sum in key order, divide, argmax, and write the outputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "knnf_device.h"

namespace knnf {
namespace {

constexpr uint64_t KEY_INF = ~0ull;
constexpr int WAVE = 64;
constexpr int A2ROWS = 64;  // window rows per block of the LDS a2 table
constexpr int A2PAD = 4;    // padding rows (+inf) so a 4-row group may start anywhere
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

// ---- cross-lane exchange with the partner lane L ^ J (no LDS traffic
// except J = 4, which uses the LDS crossbar swizzle)
template <int J>
__device__ __forceinline__ uint32_t xlane(uint32_t v) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (J == 4) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (4 << 10));
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x128, 0xF, 0xF, false);
    } else if constexpr (J == 16) {
        // permlane16_swap(v, v) yields rows {0,0,2,2} and {1,1,3,3}
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane_id() & 16) ? r[0] : r[1];
    } else {
        // permlane32_swap(v, v) yields halves {lo,lo} and {hi,hi}
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane_id() & 32) ? r[0] : r[1];
    }
}

// Compare-exchange of 64-bit keys (hi, lo) with partner L ^ J inside bitonic
// stage S (S = 64: the final, all-ascending stage).
template <int S, int J>
__device__ __forceinline__ void cx_key(uint32_t& hi, uint32_t& lo) {
    const int L = lane_id();
    const uint32_t ph = xlane<J>(hi), pl = xlane<J>(lo);
    const uint64_t me = ((uint64_t)hi << 32) | lo, ot = ((uint64_t)ph << 32) | pl;
    const bool flip = ((L & J) != 0) != (S < WAVE && (L & S) != 0);
    const bool take = (ot < me) != flip;  // keys are unique apart from KEY_INF
    hi = take ? ph : hi;
    lo = take ? pl : lo;
}

template <int S, int J>
__device__ __forceinline__ void stage_key(uint32_t& hi, uint32_t& lo) {
    cx_key<S, J>(hi, lo);
    if constexpr (J > 1) stage_key<S, J / 2>(hi, lo);
}

// Ascending bitonic sort of one 64-bit key per lane across the wavefront.
__device__ __forceinline__ uint64_t sort64(uint64_t key) {
    uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
    stage_key<2, 1>(hi, lo);
    stage_key<4, 2>(hi, lo);
    stage_key<8, 4>(hi, lo);
    stage_key<16, 8>(hi, lo);
    stage_key<32, 16>(hi, lo);
    stage_key<64, 32>(hi, lo);
    return ((uint64_t)hi << 32) | lo;
}

// a, b ascending across lanes; returns the 64 smallest of both, ascending.
__device__ __forceinline__ uint64_t merge64(uint64_t a, uint64_t b) {
    const int L = lane_id();
    const uint64_t rb = shfl64(b, WAVE - 1 - L);
    const uint64_t key = rb < a ? rb : a;  // bitonic: the 64 smallest of a and b
    uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
    stage_key<64, 32>(hi, lo);
    return ((uint64_t)hi << 32) | lo;
}

// ---- segmented sorts: the Q queries of a tile sorted together.  Segment q
// (64 elements) lives in lanes q*P .. q*P+P-1, P = 64 / E; lane L holds
// elements e = (L % P) * E + r in x[r], r < E.
//
// The network is the all-ascending form of the bitonic sort: stage KS first
// compares e with its mirror e ^ (KS - 1) inside each block of KS elements
// (both halves ascending -> the smaller KS/2 in the lower half, as two
// bitonic halves), then half-cleaners compare e with e ^ D, D = KS/4 .. 1.
// The lower element of every pair takes the minimum, so pairs inside a lane
// need no direction, and cross-lane partners are lane ^ 1, 2, 3 or 7 for
// E >= 8: all DPP lane permutations within a row.

// Value of lane L ^ X (X in 1, 2, 3, 7, 15 via DPP; others via xlane).
template <int X>
__device__ __forceinline__ uint32_t lanex(uint32_t v) {
    if constexpr (X == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    } else if constexpr (X == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    } else if constexpr (X == 3) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x1B, 0xF, 0xF, false);  // quad_perm 3,2,1,0
    } else if constexpr (X == 7) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    } else if constexpr (X == 15) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    } else {
        static_assert(X == 4 || X == 8 || X == 16 || X == 32, "unsupported lane permutation");
        return xlane<X>(v);
    }
}

// The u32 network sorts bit patterns of non-negative binary32 values (pass-A
// distances, +inf padding): their unsigned order is their numeric order, so
// a cross-lane pair keeps max(x, p) or min(x, p) as the median of x, p and
// +inf or -inf (one v_med3_f32).
__device__ __forceinline__ float side_sel(bool upper) {
    return __int_as_float(upper ? 0x7f800000 : (int)0xff800000u);
}
__device__ __forceinline__ uint32_t keep_side(uint32_t x, uint32_t p, float sel) {
    return __float_as_uint(__builtin_amdgcn_fmed3f(__uint_as_float(x), __uint_as_float(p), sel));
}

template <int E, int KS>
__device__ __forceinline__ void seg_mirror_u32(uint32_t (&x)[E], int lp) {
    if constexpr (KS <= E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (r & (KS / 2)) continue;
            constexpr int M = KS - 1;
            const uint32_t a = x[r], b = x[r ^ M];
            x[r] = min(a, b);
            x[r ^ M] = max(a, b);
        }
    } else {
        const float sel = side_sel((lp & (KS / (2 * E))) != 0);
        uint32_t p[E];
#pragma unroll
        for (int r = 0; r < E; ++r) p[r] = lanex<KS / E - 1>(x[E - 1 - r]);
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = keep_side(x[r], p[r], sel);
    }
}

template <int E, int D>
__device__ __forceinline__ void seg_half_u32(uint32_t (&x)[E], int lp) {
    if constexpr (D < E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (r & D) continue;
            const uint32_t a = x[r], b = x[r | D];
            x[r] = min(a, b);
            x[r | D] = max(a, b);
        }
    } else {
        const float sel = side_sel((lp & (D / E)) != 0);
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = keep_side(x[r], lanex<D / E>(x[r]), sel);
    }
}

template <int E, int KS, int D>
__device__ __forceinline__ void seg_halves_u32(uint32_t (&x)[E], int lp) {
    if constexpr (D >= 1) {
        seg_half_u32<E, D>(x, lp);
        seg_halves_u32<E, KS, D / 2>(x, lp);
    }
}

template <int E, int KS, int SEG = WAVE>
__device__ __forceinline__ void seg_stage_u32(uint32_t (&x)[E], int lp) {
    seg_mirror_u32<E, KS>(x, lp);
    seg_halves_u32<E, KS, KS / 4>(x, lp);
    if constexpr (KS < SEG) seg_stage_u32<E, KS * 2, SEG>(x, lp);
}

template <int E, int SEG = WAVE>
__device__ __forceinline__ void seg_sort_u32(uint32_t (&x)[E], int lp) {
    seg_stage_u32<E, 2, SEG>(x, lp);
}

// ---- the same network on pairs of 16-bit keys: register r of lane L holds
// element (L % P) * E + r of two independent segments, one in each half,
// sorted together with packed unsigned 16-bit min / max (v_pk_min_u16,
// v_pk_max_u16: integer instructions).  Cross-lane pairs keep min or max by
// lane.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_keep(uint32_t x, uint32_t p, bool upper) {
    return upper ? pk_max(x, p) : pk_min(x, p);
}

template <int E, int KS>
__device__ __forceinline__ void seg_mirror_pk(uint32_t (&x)[E], int lp) {
    if constexpr (KS <= E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (r & (KS / 2)) continue;
            constexpr int M = KS - 1;
            const uint32_t a = x[r], b = x[r ^ M];
            x[r] = pk_min(a, b);
            x[r ^ M] = pk_max(a, b);
        }
    } else {
        const bool upper = (lp & (KS / (2 * E))) != 0;
        uint32_t p[E];
#pragma unroll
        for (int r = 0; r < E; ++r) p[r] = lanex<KS / E - 1>(x[E - 1 - r]);
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = pk_keep(x[r], p[r], upper);
    }
}

template <int E, int D>
__device__ __forceinline__ void seg_half_pk(uint32_t (&x)[E], int lp) {
    if constexpr (D < E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (r & D) continue;
            const uint32_t a = x[r], b = x[r | D];
            x[r] = pk_min(a, b);
            x[r | D] = pk_max(a, b);
        }
    } else {
        const bool upper = (lp & (D / E)) != 0;
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = pk_keep(x[r], lanex<D / E>(x[r]), upper);
    }
}

template <int E, int KS, int D>
__device__ __forceinline__ void seg_halves_pk(uint32_t (&x)[E], int lp) {
    if constexpr (D >= 1) {
        seg_half_pk<E, D>(x, lp);
        seg_halves_pk<E, KS, D / 2>(x, lp);
    }
}

template <int E, int KS, int SEG>
__device__ __forceinline__ void seg_stage_pk(uint32_t (&x)[E], int lp) {
    seg_mirror_pk<E, KS>(x, lp);
    seg_halves_pk<E, KS, KS / 4>(x, lp);
    if constexpr (KS < SEG) seg_stage_pk<E, KS * 2, SEG>(x, lp);
}

template <int E, int SEG>
__device__ __forceinline__ void seg_sort_pk(uint32_t (&x)[E], int lp) {
    seg_stage_pk<E, 2, SEG>(x, lp);
}

// Two non-negative binary32 bit patterns (or +inf / NaN bits) as a pair of
// 16-bit keys rounded up: key = ceil(d / 2^16), so d <= key << 16.
__device__ __forceinline__ uint32_t pack_up(uint32_t lo, uint32_t hi) {
    return ((lo + 0xffffu) >> 16) | ((hi + 0xffffu) & 0xffff0000u);
}

// Per-wavefront LDS state of one tile of QR x QC query pixels.
template <int QR, int QC>
struct alignas(16) TileState {
    static constexpr int Q = QR * QC;
    union {
        uint64_t pend[Q][WAVE];  // keys of candidates that passed the bound, unsorted
        float sums[Q][MAXC + 1]; // class sums for the argmax (after the final selection);
                                 // the odd row stride spreads the queries over the banks
    };
    // sorted top-K linear indices (first listn valid); rows padded by 16
    // bytes so that the queries' rows start on different banks (Eq. 2 reads
    // the same entry of every query at once, the final selection stores them)
    uint32_t list[Q][WAVE + 4];
                              // before the scan: pass-A block distances
    uint32_t tauhi[Q];        // distance bits of the current bound on the K-th key
    float iq[Q];              // I of each query pixel (NaN for pixels off the frame)
    int listn[Q];             // valid list entries (<= K)
    int cnt[Q];               // pending entries (mirror of the scan's registers)
};

// The exhaustive scan also keeps a table of row terms; the pruned scan
// computes them per lane.
template <int QR, int QC, bool PRUNE>
struct alignas(16) TileLds : TileState<QR, QC> {
    float a2t[A2ROWS + A2PAD][QR];  // fl32(a*a) for a block of window rows (+inf: inactive)
};
template <int QR, int QC>
struct alignas(16) TileLds<QR, QC, true> : TileState<QR, QC> {};

// Coordinate feature fr(x) = fl32(lambda * (float)x).
__device__ __forceinline__ float feat(float lam, int x) { return lam * (float)x; }

// Eq. 1 between query (r, c, iq) and the candidate with linear index idx,
// evaluated exactly as in the scan loop.
__device__ __forceinline__ float dist_to(const float* __restrict__ pc1, int W, float lam, int r,
                                         int c, float iq, uint32_t idx) {
    const int i = (int)(idx / (uint32_t)W);
    const int j = (int)idx - i * W;
    const float a = feat(lam, r) - feat(lam, i);
    const float a2 = a * a;
    const float b = feat(lam, c) - feat(lam, j);
    const float e = iq - pc1[idx];
    return fmaf(e, e, fmaf(b, b, a2));
}

// Merge query q's pending candidates into its sorted top-K list.  Returns the
// new K-th key (KEY_INF while fewer than K candidates are known).  With
// `final`, also writes the neighbour outputs of the query pixel.
template <int QR, int QC>
__device__ __forceinline__ uint64_t flush_query(TileState<QR, QC>& S, const FrameDesc& f, int r0,
                                             int c0, int q, int cnt, bool final) {
    const int L = lane_id();
    const int W = f.W, K = f.K;
    const float lam = f.lambda;
    const int r = r0 + q / QC, c = c0 + q % QC;
    wave_sync();
    const float iq = S.iq[q];
    const int listn = uni(S.listn[q]);
    uint64_t key = KEY_INF;
    if (cnt > 0) {
        if (L < cnt) key = S.pend[q][L];
        key = sort64(key);
    }
    if (listn > 0) {
        uint64_t lk = KEY_INF;
        if (L < listn) {
            const uint32_t idx = S.list[q][L];
            lk = make_key(dist_to(f.pc1, W, lam, r, c, iq, idx), (int)idx);
        }
        key = (cnt > 0) ? merge64(lk, key) : lk;
    }
    if (L >= K) key = KEY_INF;
    const int nl = min(K, listn + cnt);
    wave_sync();
    // a slot without a candidate (only with non-finite inputs, or inputs that
    // change during the launch) gathers the query pixel's own row, never an
    // address outside the frame
    if (L < K) S.list[q][L] = (final && key == KEY_INF) ? (uint32_t)(r * W + c) : (uint32_t)key;
    if (final && L < K) {
        const size_t pix = (size_t)r * W + c;
        if (f.out_nbr) f.out_nbr[pix * K + L] = (int32_t)(uint32_t)key;
        if (f.out_dist) f.out_dist[pix * K + L] = __uint_as_float((uint32_t)(key >> 32));
    }
    const uint64_t kth = uni64(shfl64(key, K - 1));
    if (L == 0) S.listn[q] = nl;
    wave_sync();
    return nl == K ? kth : KEY_INF;
}

// Pruned scan (bit-identical to the exhaustive one).  Every term of Eq. 1 is
// >= 0 and binary32 rounding is monotone, so fmaf(b, b, a2) with the smallest
// |b| and a2 of a set of candidates bounds all their distances from below;
// a set whose bound exceeds every query's current bound tau cannot hold a
// neighbour.  The scan visits the window in patches of PR rows x SW = 64/PR
// columns (the window chunk, PR = 2^lpr = 8, 16 or 32): lane L holds row
// blk + (L % PR), column jc + L / PR, so a lane's row term stays fixed while a
// row block is swept outward column step by column step.
//   * live rows: rows where some query's row term alone is within its bound
//     (its own column has b = 0);
//   * per block of 16 live rows: the tile's own column steps, then steps to
//     the right and to the left until the first step whose bound exceeds
//     every query's (further steps only have larger column terms).
// Survivors (d <= tau's distance) are appended per query with ballot +
// mbcnt; a full buffer is merged into the query's sorted list, which
// tightens its bound.
template <int QR, int QC>
__device__ __forceinline__ void scan_pruned(TileState<QR, QC>& S, const FrameDesc& f, int r0,
                                            int c0, int nqr, int nqc, int lpr,
                                            const float (&iq)[QR * QC],
                                            uint32_t (&th)[QR * QC], int (&cnt)[QR * QC],
                                            unsigned long long& pairs) {
    constexpr int Q = QR * QC;
    const int L = lane_id();
    const int H = f.H, W = f.W, R = f.R;
    const float lam = f.lambda;
    const float* __restrict__ pc1 = f.pc1;
    const float pinf = __int_as_float(0x7f800000);
    const int rlo = max(0, r0 - R), rhi = min(H - 1, r0 + nqr - 1 + R);

    // ---- live rows
    int lo = 0x7fffffff, hi = -1;
    {
        uint32_t thr[QR];  // loosest bound of each query row
#pragma unroll
        for (int qr = 0; qr < QR; ++qr) {
            thr[qr] = th[qr * QC];
#pragma unroll
            for (int qc = 1; qc < QC; ++qc) thr[qr] = max(thr[qr], th[qr * QC + qc]);
        }
        for (int base = rlo; base <= rhi; base += WAVE) {
            const int i = base + L;
            const float fi = feat(lam, i);
            bool live = false;
#pragma unroll
            for (int qr = 0; qr < QR; ++qr) {
                const int r = r0 + qr;
                const float a = feat(lam, r) - fi;
                live |= qr < nqr && i <= rhi && i >= r - R && i <= r + R &&
                        __float_as_uint(a * a) <= thr[qr];
            }
            const uint64_t m = ballot(live);
            if (m) {
                lo = min(lo, base + (int)__builtin_ctzll(m));
                hi = max(hi, base + 63 - (int)__builtin_clzll(m));
            }
        }
    }

    const int PR = 1 << lpr, lsw = 6 - lpr, SW = 1 << lsw;  // patch rows, step columns
    const int lr = L & (PR - 1), lc = L >> lpr;
    const int ncen = (nqc + SW - 1) >> lsw;  // steps over the tile's own columns
    for (int blk = lo; blk <= hi; blk += PR) {
        const int bhi = min(blk + PR - 1, hi);
        const int i = blk + lr;
        float a2[QR];   // this lane's row term per query row
        bool rok[QR];   // this lane's row is live and in the query row's window
        float a2n[QR];  // smallest row term of the block per query row (uniform)
#pragma unroll
        for (int qr = 0; qr < QR; ++qr) {
            const int r = r0 + qr;
            const float a = feat(lam, r) - feat(lam, i);
            a2[qr] = a * a;
            rok[qr] = qr < nqr && i <= bhi && i >= r - R && i <= r + R;
            const int wl = max(blk, r - R), wh = min(bhi, r + R);
            const float an = feat(lam, r) - feat(lam, min(max(r, wl), wh));
            a2n[qr] = (qr < nqr && wl <= wh) ? an * an : pinf;
        }
        uint64_t rm[QR];  // lanes whose row is live and in the query row's window
#pragma unroll
        for (int qr = 0; qr < QR; ++qr) rm[qr] = ballot(rok[qr]);

        // live column steps on each side: a prefix, found 64 steps at a time
        int nside[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            int n = 0;
            for (;;) {
                const int st = n + L;
                const int jc = side == 0 ? c0 + SW * (ncen + st) : c0 - SW * (st + 1);
                const int jn = side == 0 ? jc : jc + SW - 1;  // the step's column nearest the tile
                const float fj = feat(lam, jn);
                uint64_t m = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const float b = feat(lam, c0 + q % QC) - fj;
                    m |= ballot(__float_as_uint(fmaf(b, b, a2n[q / QC])) <= th[q]);
                }
                m &= ballot(side == 0 ? jc < W : jn >= 0);
                const int k = (~m) ? (int)__builtin_ctzll(~m) : WAVE;
                n += k;
                if (k < WAVE) break;
            }
            nside[side] = n;
        }
        const int nright = nside[0], ns = ncen + nright + nside[1];

        // rows past the frame or the window are loaded clamped and never pass
        const float* __restrict__ rowp = pc1 + (size_t)min(i, rhi) * W;
        auto step_col = [&](int st) {
            return st < ncen + nright ? c0 + SW * st : c0 - SW * (st - ncen - nright + 1);
        };
        float ipn = rowp[min(max(step_col(0) + lc, 0), W - 1)];
        for (int st = 0; st < ns; ++st) {
            const int jc = step_col(st);
            const float ip = ipn;
            if (st + 1 < ns) ipn = rowp[min(max(step_col(st + 1) + lc, 0), W - 1)];
            const int j = jc + lc;
            const bool jok = j >= 0 && j < W;
            const uint32_t idx = (uint32_t)i * (uint32_t)W + (uint32_t)j;
            float b[QC];
#pragma unroll
            for (int qc = 0; qc < QC; ++qc) b[qc] = feat(lam, c0 + qc) - feat(lam, j);
            const uint64_t jm = ballot(jok);
            if (f.stats) {
#pragma unroll
                for (int qr = 0; qr < QR; ++qr)
                    pairs += (unsigned long long)__builtin_popcountll(jm & rm[qr]) * nqc;
            }
            uint32_t ovf = 0;  // queries whose buffer cannot take this step's survivors
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int qr = q / QC, qc = q % QC;
                const float e = iq[q] - ip;
                const float d = fmaf(e, e, fmaf(b[qc], b[qc], a2[qr]));
                const bool pass = jok && rok[qr] && __float_as_uint(d) <= th[q];
                const uint64_t m = ballot(__float_as_uint(d) <= th[q]) & jm & rm[qr];
                if (m) {
                    const int n = __builtin_popcountll(m);
                    if (cnt[q] + n <= WAVE) {
                        if (pass) S.pend[q][cnt[q] + mbcnt(m)] = make_key(d, (int)idx);
                        cnt[q] += n;
                    } else {
                        ovf |= 1u << q;
                    }
                }
            }
            if (ovf) {
                // rare: merge the full buffers into the sorted lists (which
                // tightens the bounds), then append this step's survivors
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    if (L == 0) S.cnt[q] = cnt[q];
                wave_sync();
                while (ovf) {
                    const int q = __builtin_ctz(ovf);
                    ovf &= ovf - 1;
                    const int qr = q / QC, qc = q % QC;
                    const int r = r0 + qr;
                    const float a = feat(lam, r) - feat(lam, i);
                    const float bq = feat(lam, c0 + qc) - feat(lam, j);
                    const float e = S.iq[q] - ip;
                    const float d = fmaf(e, e, fmaf(bq, bq, a * a));
                    const bool rq = i <= bhi && i >= r - R && i <= r + R;
                    const uint64_t kth = flush_query(S, f, r0, c0, q, uni(S.cnt[q]), false);
                    uint32_t thq = uniu(S.tauhi[q]);
                    if (kth != KEY_INF) thq = min(thq, (uint32_t)(kth >> 32));
                    const bool pass = jok && rq && __float_as_uint(d) <= thq;
                    const uint64_t m = ballot(pass);
                    if (pass) S.pend[q][mbcnt(m)] = make_key(d, (int)idx);
                    wave_sync();
                    if (L == 0) {
                        S.cnt[q] = __builtin_popcountll(m);
                        S.tauhi[q] = thq;
                    }
                    wave_sync();
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    cnt[q] = uni(S.cnt[q]);
                    th[q] = S.tauhi[q];
                }
            }
        }
    }
}

// s + v[0] + v[1] + ... + v[N-1], left to right, where v[u] is the float at
// pb + lst[u] * rowb: all N gathers are issued before the first add.  lst is
// 16-byte aligned and N a multiple of 4.
template <int N>
__device__ __forceinline__ float gather_add(float s, const char* __restrict__ pb,
                                            const uint32_t* lst, uint32_t rowb) {
    float v[N];
#pragma unroll
    for (int u = 0; u < N; u += 4) {
        const uint4 id = *(const uint4*)(lst + u);
        v[u + 0] = *(const float*)(pb + (uint64_t)id.x * rowb);
        v[u + 1] = *(const float*)(pb + (uint64_t)id.y * rowb);
        v[u + 2] = *(const float*)(pb + (uint64_t)id.z * rowb);
        v[u + 3] = *(const float*)(pb + (uint64_t)id.w * rowb);
    }
#pragma unroll
    for (int u = 0; u < N; ++u) s = s + v[u];
    return s;
}

// As gather_add, with 32-bit byte offsets from a wave-uniform base: v[u] is
// the float at base + lst[u] * rowb + cb, for frames whose linear indices fit
// 24 bits and whose probability array fits 2^32 bytes (one full-rate 24-bit
// multiply-add per gather instead of a 64-bit one).
template <int N>
__device__ __forceinline__ float gather_add24(float s, const char* __restrict__ base,
                                              const uint32_t* lst, uint32_t rowb, uint32_t cb) {
    float v[N];
#pragma unroll
    for (int u = 0; u < N; u += 4) {
        const uint4 id = *(const uint4*)(lst + u);
        v[u + 0] = *(const float*)(base + (__umul24(id.x, rowb) + cb));
        v[u + 1] = *(const float*)(base + (__umul24(id.y, rowb) + cb));
        v[u + 2] = *(const float*)(base + (__umul24(id.z, rowb) + cb));
        v[u + 3] = *(const float*)(base + (__umul24(id.w, rowb) + cb));
    }
#pragma unroll
    for (int u = 0; u < N; ++u) s = s + v[u];
    return s;
}

// Process one tile: query pixels (r0 + qr, c0 + qc), qr < QR, qc < QC.
// NA: pass-A block candidates per query (128 or 64; 64 for 16-query tiles).
// NG: groups the NA candidates are split into for the bound (1, 2 or 4).
template <int QR, int QC, bool PRUNE, int NA = (QR * QC == 8 ? 128 : WAVE),
          int NG = (NA == 128 ? 2 : 1)>
__device__ __forceinline__ void process_tile(TileLds<QR, QC, PRUNE>& S, const FrameDesc& f, int r0,
                                             int c0, int lpr) {
    constexpr int Q = QR * QC;
    const int L = lane_id();
    const int H = f.H, W = f.W, R = f.R, K = f.K, C = f.C;
    const float lam = f.lambda;
    const int nqr = min(QR, H - r0), nqc = min(QC, W - c0);
    const float* __restrict__ pc1 = f.pc1;
    const float qnan = __int_as_float(0x7fc00000);
    const float pinf = __int_as_float(0x7f800000);

    if (L < Q) S.listn[L] = 0;

    // ---- pass A.  Any set of block candidates of which at least K have a
    // distance <= d bounds the query's final K-th key from above by
    // (d, max index).  The block's NA candidates are split into NG groups of
    // the same spatial spread; with m = ceil(K / NG), the largest of the
    // groups' m-th smallest distances is such a d (NG = 1: the block's K-th
    // smallest).  All Q blocks are evaluated and sorted together: segment q
    // of the wavefront (P lanes) holds query q's NA block candidates, EA per
    // lane; group g is the segment's lanes g*LG .. g*LG + LG - 1.
    constexpr int E = Q, P = WAVE / Q;          // final selection: 64 slots per query
    constexpr int EA = NA / P;                  // pass-A candidates per lane
    constexpr int LNA = NA == 128 ? 7 : 6;
    constexpr int LG = P / NG, GS = NA / NG;    // lanes and candidates per group
    constexpr bool PK = NA == 128 && NG == 2;   // two groups as 16-bit key pairs
    static_assert(NA == WAVE || (NA == 128 && Q == 8), "pass-A block size");
    static_assert((NG == 1 || NG == 2 || NG == 4) && LG >= 1 && (WAVE + NG - 1) / NG <= GS,
                  "pass-A groups");
    const int sq = L / P, lp = L % P;  // this lane's query (segment) and slot in it
    const int sqr = sq / QC, sqc = sq % QC;
    const bool sok = sqr < nqr && sqc < nqc;
    const bool off32 = (uint64_t)H * (uint64_t)W <= (1u << 30);  // band byte offsets fit 32 bits
    {
        const int r = r0 + sqr, c = c0 + sqc;
        const int i0w = max(0, r - R), i1w = min(H - 1, r + R);
        const int nr = i1w - i0w + 1;
        const int lbr = nr >= 8 ? 3 : (nr >= 4 ? 2 : (nr >= 2 ? 1 : 0));
        const int br = 1 << lbr;
        const int lbc = LNA - lbr;
        const int bc = 1 << lbc;
        const int rb = min(max(r - br / 2, i0w), i1w - br + 1);
        const int cb = max(0, min(c - bc / 2, W - bc));
        // I of the segment's query pixel (NaN for pixels off the frame)
        const float iqs = sok ? pc1[(uint32_t)r * (uint32_t)W + (uint32_t)c] : qnan;
        const float frq = feat(lam, r), fcq = feat(lam, c);
        // Element e = u * P + lp of the block is row rb + (e >> lbc), column
        // cb + (e & (bc - 1)): the P lanes of a segment read P consecutive
        // columns of one row per load, so a load touches few cache lines.
        // Every lane loads (columns past the right edge clamped and given
        // +inf; rows rb .. rb+br-1 are inside the frame even for queries off
        // its bottom edge), so all EA loads are in flight together.
        if constexpr (PK) {
            // 128 candidates as 8 registers of 16-bit key pairs: group 0 in
            // the low halves, group 1 in the high halves, each group's 64
            // keys (8 per lane) sorted by one packed network
            uint32_t xp[8];
            if (W >= 16 && off32 && !ballot(lbr != 3)) {
                // every block is 8 x 16: lane lp takes columns cb + 2 lp
                // (group 0) and cb + 2 lp + 1 (group 1) of rows rb .. rb + 7,
                // so both groups hold every row and alternate columns
                const int j = cb + 2 * lp;
                const uint32_t o4 = ((uint32_t)rb * (uint32_t)W + (uint32_t)j) * 4u;
                const char* __restrict__ pcb = (const char*)pc1;
                float p0[8], p1[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const char* row = pcb + (o4 + (uint32_t)u * (uint32_t)W * 4u);
                    p0[u] = *(const float*)row;
                    p1[u] = *(const float*)(row + 4);
                }
                const float b0 = fcq - feat(lam, j), b1 = fcq - feat(lam, j + 1);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float a = frq - feat(lam, rb + u);
                    const float a2 = a * a;
                    const float e0 = iqs - p0[u], e1 = iqs - p1[u];
                    // NaN bits for a query off the frame (segment unused)
                    xp[u] = pack_up(__float_as_uint(fmaf(e0, e0, fmaf(b0, b0, a2))),
                                    __float_as_uint(fmaf(e1, e1, fmaf(b1, b1, a2))));
                }
            } else {
                // element e = u * 8 + lp of the block (u < 16): group 0 the
                // elements u < 8, group 1 the rest
                float pv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = u * P + lp;
                    const int i = rb + (e >> lbc);
                    const int j = min(cb + (e & (bc - 1)), W - 1);
                    pv[u] = pc1[(uint32_t)i * (uint32_t)W + (uint32_t)j];
                }
                uint32_t x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = u * P + lp;
                    const int i = rb + (e >> lbc);
                    const int j = cb + (e & (bc - 1));
                    const float a = frq - feat(lam, i);
                    const float b = fcq - feat(lam, j);
                    const float ee = iqs - pv[u];
                    const uint32_t d = __float_as_uint(fmaf(ee, ee, fmaf(b, b, a * a)));
                    x[u] = (sok && j < W) ? d : 0x7f800000u;  // +inf: no candidate
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) xp[u] = pack_up(x[u], x[u + 8]);
            }
            if (lp == 0) S.iq[sq] = iqs;
            seg_sort_pk<8, WAVE>(xp, lp);
            // each group's element m - 1 (lane (m-1) / 8, register (m-1) % 8);
            // at least K candidates lie at or below the larger key
            const int m = (K + 1) / 2;
            const uint32_t v = xp[uni((m - 1) % 8)];  // uniform register index
            const uint32_t kk = max(v & 0xffffu, v >> 16);
            if (lp == (m - 1) / 8) S.tauhi[sq] = sok ? kk << 16 : 0u;
        } else {
            uint32_t x[EA];
            float pv[EA];
            // full blocks: lane lp takes block column offset jl (a permutation of
            // 0..7), so that the columns of every group spread over the block
            const int jl = NG * (lp % LG) + lp / LG;
            if (EA == 8 && NA == WAVE && W >= 8 && !ballot(lbr != 3)) {
                // every block is 8 x 8 (P = 8): element u * 8 + lp is row rb + u,
                // column cb + jl < W, so a lane's column term is computed once
                const int j = cb + jl;
                const uint32_t o = (uint32_t)rb * (uint32_t)W + (uint32_t)j;
#pragma unroll
                for (int u = 0; u < EA; ++u) pv[u] = pc1[o + (uint32_t)u * (uint32_t)W];
                const float b = fcq - feat(lam, j);
#pragma unroll
                for (int u = 0; u < EA; ++u) {
                    const float a = frq - feat(lam, rb + u);
                    const float ee = iqs - pv[u];
                    const uint32_t d = __float_as_uint(fmaf(ee, ee, fmaf(b, b, a * a)));
                    x[u] = d;  // NaN bits for a query off the frame (segment unused)
                }
            } else if (EA == 16 && NA == 128 && W >= 16 && off32 && !ballot(lbr != 3)) {
                // every block is 8 x 16 (P = 8): element u * 8 + lp is row
                // rb + u / 2, column cb + 8 (u % 2) + jl < W, so a lane has two
                // column terms and each row term serves two elements.  Byte
                // offsets from the band's base fit 32 bits (off32): one add per
                // row, the second column half as the load's immediate offset.
                const int j = cb + jl;
                const uint32_t o4 = ((uint32_t)rb * (uint32_t)W + (uint32_t)j) * 4u;
                const char* __restrict__ pcb = (const char*)pc1;
#pragma unroll
                for (int u = 0; u < EA; ++u)
                    pv[u] = *(const float*)(pcb + (o4 + (uint32_t)(u >> 1) * (uint32_t)W * 4u) +
                                            32u * (u & 1));
                const float b0 = fcq - feat(lam, j), b1 = fcq - feat(lam, j + 8);
#pragma unroll
                for (int u = 0; u < EA; u += 2) {
                    const float a = frq - feat(lam, rb + (u >> 1));
                    const float a2 = a * a;
                    const float e0 = iqs - pv[u], e1 = iqs - pv[u + 1];
                    const uint32_t d0 = __float_as_uint(fmaf(e0, e0, fmaf(b0, b0, a2)));
                    const uint32_t d1 = __float_as_uint(fmaf(e1, e1, fmaf(b1, b1, a2)));
                    x[u] = d0;  // NaN bits for a query off the frame (segment unused)
                    x[u + 1] = d1;
                }
            } else {
#pragma unroll
                for (int u = 0; u < EA; ++u) {
                    const int e = u * P + lp;
                    const int i = rb + (e >> lbc);
                    const int j = min(cb + (e & (bc - 1)), W - 1);
                    pv[u] = pc1[(uint32_t)i * (uint32_t)W + (uint32_t)j];
                }
#pragma unroll
                for (int u = 0; u < EA; ++u) {
                    const int e = u * P + lp;
                    const int i = rb + (e >> lbc);
                    const int j = cb + (e & (bc - 1));
                    const float a = frq - feat(lam, i);
                    const float b = fcq - feat(lam, j);
                    const float ee = iqs - pv[u];
                    const uint32_t d = __float_as_uint(fmaf(ee, ee, fmaf(b, b, a * a)));
                    x[u] = (sok && j < W) ? d : 0x7f800000u;  // +inf: no candidate
                }
            }
            if (lp == 0) S.iq[sq] = iqs;
            seg_sort_u32<EA, GS>(x, lp);
            // each group's element m - 1 (group lane (m-1) / EA, register
            // (m-1) % EA); the largest of the NG goes to the group-0 holder,
            // which writes the bound
            const int m = (K + NG - 1) / NG;
            const int uk = uni((m - 1) % EA);
            uint32_t dk = x[uk];  // uniform register index
            if constexpr (NG > 1) {
                dk = (lp % LG) == (m - 1) / EA ? dk : 0u;
                if constexpr (LG == 2) dk = max(dk, xlane<2>(dk));
                dk = max(dk, xlane<4>(dk));
            }
            if (lp == (m - 1) / EA) S.tauhi[sq] = sok ? dk : 0u;
        }
        wave_sync();
    }

    // Work counter (only reported when f.stats is set): candidate distances
    // evaluated for on-frame queries; pass A counts its NA block slots.
    unsigned long long pairs = (unsigned long long)(nqr * nqc) * NA;

    // Uniform per-query values live in VGPRs (read from LDS) to keep the
    // scalar register file free for loop state.  Queries off the frame have
    // iq = NaN and bound 0, so they never pass the test below.
    float iq[Q];
    uint32_t th[Q];
    int cnt[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        iq[q] = S.iq[q];
        th[q] = S.tauhi[q];
        cnt[q] = 0;
    }

    // ---- pass B
    if constexpr (PRUNE) {
        scan_pruned<QR, QC>(S, f, r0, c0, nqr, nqc, lpr, iq, th, cnt, pairs);
    } else {
        // exhaustive: window rows x 64-column chunks, nearest chunk first
        const int rlo = max(0, r0 - R);
        const int rhi = min(H - 1, r0 + nqr - 1 + R);
        const int nch = (W + WAVE - 1) / WAVE;
        const int cc = (c0 + (nqc - 1) / 2) / WAVE;
        int tab_base = -1;       // first row of the a2 table contents

        for (int t = 0; t < 2 * nch; ++t) {
            const int m = (t & 1) ? cc + (t + 1) / 2 : cc - t / 2;
            if (m < 0 || m >= nch) continue;
            const int J = m * WAVE;
            const int j = J + L;
            const bool valid = j < W;
            const uint64_t vm = ballot(valid);
            const int jl = valid ? j : W - 1;
            // lanes past the right edge get b = +inf, so every distance there is
            // +inf (never below a finite bound; the append step checks `valid`)
            float b[QC];
#pragma unroll
            for (int qc = 0; qc < QC; ++qc) b[qc] = valid ? feat(lam, c0 + qc) - feat(lam, j) : pinf;

            const int lo = rlo, hi = rhi;

            // Table blocks are aligned to rlo: block k holds rows rlo + 64k ...
            // rlo + 64k + 63 (+inf past rhi and in the padding), so windows of up
            // to 64 rows fill it once per tile.
            for (int blk = rlo + ((lo - rlo) / A2ROWS) * A2ROWS; blk <= hi; blk += A2ROWS) {
                if (blk != tab_base) {
                    wave_sync();
                    for (int u = L; u < (A2ROWS + A2PAD) * QR; u += WAVE) {
                        const int rr = u / QR, qr = u % QR;
                        const int r = r0 + qr, i = blk + rr;
                        const bool act = rr < A2ROWS && qr < nqr && i <= rhi && i >= r - R && i <= r + R;
                        const float a = feat(lam, r) - feat(lam, i);
                        S.a2t[rr][qr] = act ? a * a : pinf;
                    }
                    wave_sync();
                    tab_base = blk;
                }
                const int g0 = max(lo, blk) - blk;
                const int g1 = min(hi, blk + A2ROWS - 1) - blk;  // last table row used
                const uint32_t joff = (uint32_t)jl;
                const float* __restrict__ rowp = pc1 + (size_t)(blk + g0) * W;
                float ipn[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    ipn[u] = rowp[(size_t)min(u, g1 - g0) * W + joff];
                for (int g = g0; g <= g1; g += 4) {
                    float ip[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) ip[u] = ipn[u];
                    if (g + 4 <= g1) {
                        const float* __restrict__ np = pc1 + (size_t)(blk + g + 4) * W;
#pragma unroll
                        for (int u = 0; u < 4; ++u) ipn[u] = np[(size_t)min(u, g1 - g - 4) * W + joff];
                    }
                    float a2[4][QR];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int qr = 0; qr < QR; ++qr) a2[u][qr] = S.a2t[g + u][qr];
                    const int i0 = blk + g;
                    if (f.stats) {
                        const int nvl = min(WAVE, W - J);
#pragma unroll
                        for (int qr = 0; qr < QR; ++qr) {
                            const int r = r0 + qr;
                            const int a = max(i0, max(lo, r - R)), z = min(i0 + 3, min(hi, r + R));
                            if (qr < nqr && z >= a) pairs += (unsigned long long)(z - a + 1) * nqc * nvl;
                        }
                    }
                    uint32_t ovf = 0;  // queries whose buffer cannot take this group's survivors
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int qr = q / QC, qc = q % QC;
                        float d[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float e = iq[q] - ip[u];
                            const float tt = fmaf(b[qc], b[qc], a2[u][qr]);
                            d[u] = fmaf(e, e, tt);
                        }
                        const uint32_t mn = min(min(__float_as_uint(d[0]), __float_as_uint(d[1])),
                                                min(__float_as_uint(d[2]), __float_as_uint(d[3])));
                        if (ballot(mn <= th[q])) {
                            // rare: some candidate of the group is within the
                            // bound; append the group's survivors if they fit
                            const int r = r0 + qr;
                            bool rok[4];  // group rows inside the query row's window
                            uint64_t mu[4];
                            int n = 0;
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int i = i0 + u;
                                rok[u] = i <= hi && i >= r - R && i <= r + R;
                                mu[u] = rok[u] ? ballot(__float_as_uint(d[u]) <= th[q]) & vm : 0ull;
                                n += __builtin_popcountll(mu[u]);
                            }
                            if (cnt[q] + n <= WAVE) {
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    if (valid && rok[u] && __float_as_uint(d[u]) <= th[q])
                                        S.pend[q][cnt[q] + mbcnt(mu[u])] = make_key(d[u], (i0 + u) * W + j);
                                    cnt[q] += __builtin_popcountll(mu[u]);
                                }
                            } else {
                                ovf |= 1u << q;
                            }
                        }
                    }
                    if (ovf) {
                        // rare: merge full buffers into the sorted lists (which
                        // tightens the bounds), appending the group row by row
#pragma unroll
                        for (int q = 0; q < Q; ++q)
                            if (L == 0) S.cnt[q] = cnt[q];
                        wave_sync();
                        while (ovf) {
                            const int q = __builtin_ctz(ovf);
                            ovf &= ovf - 1;
                            const int qr = q / QC, qc = q % QC;
                            const int r = r0 + qr;
                            int cq = uni(S.cnt[q]);
                            uint32_t thq = uniu(S.tauhi[q]);
                            const float bq = valid ? feat(lam, c0 + qc) - feat(lam, j) : pinf;
                            const float iqq = S.iq[q];
                            for (int u = 0; u < 4; ++u) {
                                const int i = i0 + u;
                                if (qr >= nqr || i > hi || i < r - R || i > r + R) continue;
                                const float a2q = S.a2t[g + u][qr];
                                const float e = iqq - ip[u];
                                const float du = fmaf(e, e, fmaf(bq, bq, a2q));
                                uint64_t msk = ballot(__float_as_uint(du) <= thq) & vm;
                                if (!msk) continue;
                                if (cq + __builtin_popcountll(msk) > WAVE) {
                                    const uint64_t kth = flush_query(S, f, r0, c0, q, cq, false);
                                    cq = 0;
                                    if (kth != KEY_INF) thq = min(thq, (uint32_t)(kth >> 32));
                                    msk = ballot(__float_as_uint(du) <= thq) & vm;
                                }
                                if (valid && __float_as_uint(du) <= thq)
                                    S.pend[q][cq + mbcnt(msk)] = make_key(du, i * W + j);
                                cq += __builtin_popcountll(msk);
                            }
                            wave_sync();
                            if (L == 0) {
                                S.cnt[q] = cq;
                                S.tauhi[q] = thq;
                            }
                            wave_sync();
                        }
#pragma unroll
                        for (int q = 0; q < Q; ++q) {
                            cnt[q] = uni(S.cnt[q]);
                            th[q] = S.tauhi[q];
                        }
                    }
                }
            }
        }
    }

    // ---- final selection; neighbour outputs
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (L == 0) S.cnt[q] = cnt[q];
    wave_sync();
    // queries whose buffer overflowed during the scan already hold a sorted
    // list: merge their last candidates one query at a time (rare)
    for (int q = 0; q < Q; ++q) {
        const int qr = q / QC, qc = q % QC;
        if (qr < nqr && qc < nqc && uni(S.listn[q]) > 0)
            flush_query(S, f, r0, c0, q, uni(S.cnt[q]), true);
    }
    wave_sync();
    {
        // all other queries: one segmented sort of their candidate buffers.
        // The network sorts 32-bit packed keys: the distance bits (clamped
        // below +inf) with their 6 low bits replaced by the buffer slot.
        // Packed order is exact wherever the distance parts differ; runs of
        // equal distance parts are then put in (d, idx) order on the full
        // keys by odd-even transposition (rarely needed).
        const int cq = S.cnt[sq];
        const bool own = sok && S.listn[sq] == 0;
        uint32_t x[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            // slot blocks permuted by segment (u ^ sq: E is a power of two and
            // sq < E), so the segments' reads of one u spread over the banks
            const int e = (u ^ sq) * P + lp;
            const uint32_t dh = (uint32_t)(S.pend[sq][e] >> 32);
            x[u] = (own && e < cq) ? ((min(dh, 0x7f7fffc0u) & ~63u) | (uint32_t)e) : 0x7f800000u;
        }
        seg_sort_u32<E>(x, lp);
        uint64_t y[E];
#pragma unroll
        for (int u = 0; u < E; ++u) y[u] = x[u] < 0x7f800000u ? S.pend[sq][x[u] & 63u] : KEY_INF;
        // neighbours in sorted order: element lp*E + u, the next one is u + 1
        // or the next lane's element 0 (same segment while lp < P - 1)
        // two neighbours share the distance part iff their keys differ in the
        // slot bits only: 1 <= (a ^ b) <= 63 (keys of candidates are distinct;
        // two empty slots, both 0x7f800000, give 0; a candidate next to an
        // empty slot differs above bit 22)
        bool tie = false;
#pragma unroll
        for (int u = 0; u + 1 < E; ++u) tie |= (uint32_t)((x[u] ^ x[u + 1]) - 1u) < 63u;
        {
            const uint32_t nx = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[0], 0x101, 0xF, 0xF, false);  // row_shl:1
            tie |= lp < P - 1 && (uint32_t)((x[E - 1] ^ nx) - 1u) < 63u;
        }
        if (ballot(tie)) {
            for (;;) {
                bool sw = false;
#pragma unroll
                for (int ph = 0; ph < 2; ++ph) {
#pragma unroll
                    for (int u = ph; u + 1 < E; u += 2) {
                        const uint64_t a = y[u], b = y[u + 1];
                        const bool t = b < a;
                        y[u] = t ? b : a;
                        y[u + 1] = t ? a : b;
                        sw |= t;
                    }
                    if ((ph == 1) == ((E & 1) == 0)) {
                        // pair (lane's last, next lane's first)
                        const uint64_t nx = (uint64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)y[0], 0x101, 0xF, 0xF, false) |
                                            ((uint64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(y[0] >> 32), 0x101, 0xF, 0xF, false) << 32);
                        const uint64_t pv = (uint64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)y[E - 1], 0x111, 0xF, 0xF, false) |
                                            ((uint64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(y[E - 1] >> 32), 0x111, 0xF, 0xF, false) << 32);
                        const bool tn = lp < P - 1 && nx < y[E - 1];  // this lane keeps the smaller
                        const bool tp = lp > 0 && y[0] < pv;          // this lane keeps the larger
                        y[E - 1] = tn ? nx : y[E - 1];
                        y[0] = tp ? pv : y[0];
                        sw |= tn;
                    }
                }
                if (!ballot(sw)) break;
            }
        }
        const size_t pix = (size_t)(r0 + sqr) * W + c0 + sqc;
        if (own && lp * E < K) {
            // the lane's E neighbours go to the list as 16-byte stores (entries
            // from K on are never read); a slot without a candidate gathers
            // the query's own row (see flush_query)
#pragma unroll
            for (int u = 0; u < E; u += 4) {
                uint4 v;
                v.x = y[u] == KEY_INF ? (uint32_t)pix : (uint32_t)y[u];
                v.y = y[u + 1] == KEY_INF ? (uint32_t)pix : (uint32_t)y[u + 1];
                v.z = y[u + 2] == KEY_INF ? (uint32_t)pix : (uint32_t)y[u + 2];
                v.w = y[u + 3] == KEY_INF ? (uint32_t)pix : (uint32_t)y[u + 3];
                *(uint4*)&S.list[sq][lp * E + u] = v;
            }
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int e = lp * E + u;
            if (own && e < K) {
                if (f.out_nbr) f.out_nbr[pix * K + e] = (int32_t)(uint32_t)y[u];
                if (f.out_dist) f.out_dist[pix * K + e] = __uint_as_float((uint32_t)(y[u] >> 32));
            }
        }
    }
    wave_sync();

    // ---- Eq. 2: sums in neighbour order, one lane per (query, class).  The
    // neighbours' rows are L2-resident; up to 16 gathers are in flight.
    const uint32_t rowb = (uint32_t)C * 4u;  // bytes per probability row
    const uint64_t npix = (uint64_t)H * (uint64_t)W;
    const bool off24 = npix <= (1u << 24) && npix * rowb <= 0xFFFFFFFFull;
    // p / C by a reciprocal: (p + 0.5) / C sits at least 1/(2C) >= 1/32 from
    // an integer and p < 2^10, far beyond the reciprocal's rounding
    const float rc = __builtin_amdgcn_rcpf((float)C);
    for (int p = L; p < Q * C; p += WAVE) {
        const int q = (int)(uint32_t)(((float)p + 0.5f) * rc), cl = p - q * C;
        const int qr = (int)((uint32_t)q / QC), qc = (int)((uint32_t)q % QC);
        if (qr >= nqr || qc >= nqc) continue;
        const uint32_t* lst = S.list[q];
        float s = 0.0f;
        int k = 0;
        if (off24) {
            const char* __restrict__ base = (const char*)f.prob;
            const uint32_t cb = (uint32_t)cl * 4u;
            for (; k + 16 <= K; k += 16) s = gather_add24<16>(s, base, lst + k, rowb, cb);
            if (k + 8 <= K) {
                s = gather_add24<8>(s, base, lst + k, rowb, cb);
                k += 8;
            }
            for (; k < K; ++k) s = s + *(const float*)(base + (__umul24(lst[k], rowb) + cb));
        } else {
            const char* __restrict__ pb = (const char*)(f.prob + cl);
            for (; k + 16 <= K; k += 16) s = gather_add<16>(s, pb, lst + k, rowb);
            if (k + 8 <= K) {
                s = gather_add<8>(s, pb, lst + k, rowb);
                k += 8;
            }
            for (; k < K; ++k) s = s + *(const float*)(pb + (uint64_t)lst[k] * rowb);
        }
        S.sums[q][cl] = s;
        if (off24) {
            // the pixel's byte offset in the probability map fits 32 bits
            const uint32_t pix = (uint32_t)(r0 * W + c0) + __umul24((uint32_t)qr, (uint32_t)W) + (uint32_t)qc;
            *(float*)((char*)f.out_prob + (__umul24(pix, rowb) + (uint32_t)cl * 4u)) = s / (float)K;
        } else {
            const size_t pix = (size_t)(r0 + qr) * W + c0 + qc;
            f.out_prob[pix * C + cl] = s / (float)K;
        }
    }
    wave_sync();
    if (L < Q) {
        const int qr = L / QC, qc = L % QC;
        if (qr < nqr && qc < nqc) {
            int best = 0;
            float bs = S.sums[L][0];
            for (int cl = 1; cl < C; ++cl) {
                const float v = S.sums[L][cl];
                if (v > bs) { bs = v; best = cl; }
            }
            if (off24)
                f.out_class[(uint32_t)(r0 * W + c0) + __umul24((uint32_t)qr, (uint32_t)W) + (uint32_t)qc] = best;
            else
                f.out_class[(size_t)(r0 + qr) * W + c0 + qc] = best;
        }
    }
    if (f.stats && L == 0) {
        atomicAdd(&f.stats[0], pairs);
        atomicAdd(&f.stats[1], 1ull);
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

// 8-query tiles are held to 80 VGPRs (six wavefronts per SIMD, the LDS
// limit too): without the hint some instantiations took 81-90 registers and
// ran at five, which cost the batched 1x8 launch 11 %.
#define KNNF_WAVES_PER_EU(QR, QC) __attribute__((amdgpu_waves_per_eu((QR) * (QC) == 8 ? 6 : 1)))

template <int QR, int QC, int WPB, bool PRUNE>
__global__ void __launch_bounds__(WPB * WAVE) KNNF_WAVES_PER_EU(QR, QC)
filter_frame_kernel(FrameDesc f, int lpr) {
    __shared__ TileLds<QR, QC, PRUNE> lds[WPB];
    const int w = uni((int)(threadIdx.x >> 6));
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    // tiles <= H * W < 2^31 (checked on the host): 32-bit index arithmetic
    const uint32_t ntc = (uint32_t)((f.W + QC - 1) / QC);
    const uint32_t ntiles = (uint32_t)((f.H + QR - 1) / QR) * ntc;
    const uint32_t s = (uint32_t)b * WPB + (uint32_t)w;
    if (s >= ntiles) return;
    const uint32_t band = s / ntc;
    const uint32_t tc = s - band * ntc;
    process_tile<QR, QC, PRUNE>(lds[w], f, (int)band * QR, (int)tc * QC, lpr);
}

// Persistent batched kernel: each wavefront claims tile tasks from one global
// counter until all tasks of all work items are taken.  Work item k is a range
// of tiles of frames[k] starting at tile_base[k]; its tasks are the ids
// task_start[k] .. task_start[k+1]-1.  Claims go out in task order, so the
// whole device sweeps neighbouring tiles (which share window rows) at the same
// time.  Every wavefront leaves the loop after one failed claim, so the grid
// always drains.  The claim loop's state would otherwise push the 8-query
// tiles to 110 VGPRs (four wavefronts per SIMD); held at 80 they spill a few
// dwords to scratch, reloaded once per tile.
template <int QR, int QC, int WPB, bool PRUNE>
__global__ void __launch_bounds__(WPB * WAVE) KNNF_WAVES_PER_EU(QR, QC)
filter_batch_kernel(const FrameDesc* __restrict__ frames, const uint32_t* __restrict__ task_start,
                    const uint32_t* __restrict__ tile_base, uint32_t nframes, uint32_t total_tasks,
                    uint32_t claim, uint32_t* counter, int lpr) {
    __shared__ TileLds<QR, QC, PRUNE> lds[WPB];
    const int w = uni((int)(threadIdx.x >> 6));
    const int L = lane_id();
    for (;;) {
        // claim `claim` consecutive tasks: fewer atomics on the counter
        uint32_t t0 = 0;
        if (L == 0) t0 = atomicAdd(counter, claim);
        t0 = uniu(t0);  // lane 0's claim
        if (t0 >= total_tasks) break;
        const uint32_t t1 = min(total_tasks, t0 + claim);
        uint32_t k = 0, next = 0;  // work item of the current task, its end
        for (uint32_t t = t0; t < t1; ++t) {
            if (t >= next || t == t0) {
                // work item k with task_start[k] <= t < task_start[k+1]
                uint32_t lo = 0, hi = nframes;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (task_start[mid] <= t) lo = mid; else hi = mid;
                }
                k = lo;
                next = task_start[k + 1];
            }
            const FrameDesc f = frames[k];
            const uint32_t s = t - task_start[k] + tile_base[k];
            const uint32_t ntc = (uint32_t)((f.W + QC - 1) / QC);
            const int band = (int)(s / ntc);
            const int tc = (int)(s - (uint32_t)band * ntc);
            // the claim loop's registers leave no room for 128-candidate blocks
            process_tile<QR, QC, PRUNE, WAVE, 1>(lds[w], f, band * QR, tc * QC, lpr);
        }
    }
}

// Non-persistent batched kernel over the same work table: one wavefront per
// task, the hardware dispatcher balances the load, XCD-aware block order.
template <int QR, int QC, int WPB, bool PRUNE>
__global__ void __launch_bounds__(WPB * WAVE) KNNF_WAVES_PER_EU(QR, QC)
filter_items_kernel(const FrameDesc* __restrict__ frames, const uint32_t* __restrict__ task_start,
                    const uint32_t* __restrict__ tile_base, uint32_t nframes,
                    uint32_t total_tasks, int lpr) {
    __shared__ TileLds<QR, QC, PRUNE> lds[WPB];
    const int w = uni((int)(threadIdx.x >> 6));
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const uint64_t t64 = (uint64_t)b * WPB + w;
    if (t64 >= total_tasks) return;
    const uint32_t t = (uint32_t)t64;
    uint32_t lo = 0, hi = nframes;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (task_start[mid] <= t) lo = mid; else hi = mid;
    }
    const FrameDesc f = frames[lo];
    const uint32_t s = t - task_start[lo] + tile_base[lo];
    const uint32_t ntc = (uint32_t)((f.W + QC - 1) / QC);
    const int band = (int)(s / ntc);
    const int tc = (int)(s - (uint32_t)band * ntc);
    process_tile<QR, QC, PRUNE>(lds[w], f, band * QR, tc * QC, lpr);
}

template <int QR, int QC, int WPB, bool PRUNE>
int launch_items_t(const FrameDesc* fr, const uint32_t* ts, const uint32_t* tb, uint32_t n,
                   uint32_t tot, int lpr, hipStream_t st) {
    const uint64_t blocks = ((uint64_t)tot + WPB - 1) / WPB;
    hipLaunchKernelGGL((filter_items_kernel<QR, QC, WPB, PRUNE>), dim3((unsigned)blocks),
                       dim3(WPB * WAVE), 0, st, fr, ts, tb, n, tot, lpr);
    return (int)hipGetLastError();
}

template <int QR, int QC, int WPB, bool PRUNE>
int launch_frame_t(const FrameDesc& f, int lpr, hipStream_t st) {
    const long long tiles = (long long)((f.H + QR - 1) / QR) * ((f.W + QC - 1) / QC);
    const long long blocks = (tiles + WPB - 1) / WPB;
    hipLaunchKernelGGL((filter_frame_kernel<QR, QC, WPB, PRUNE>), dim3((unsigned)blocks),
                       dim3(WPB * WAVE), 0, st, f, lpr);
    return (int)hipGetLastError();
}

template <int QR, int QC, int WPB, bool PRUNE>
int launch_batch_t(const FrameDesc* fr, const uint32_t* ts, const uint32_t* tb, uint32_t n,
                   uint32_t tot, uint32_t* ctr, int grid, int lpr, hipStream_t st) {
    // at least four claims per resident wavefront, at most 8 tasks per claim
    const uint64_t waves = (uint64_t)grid * WPB;
    const uint32_t claim = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8, tot / (waves * 4)));
    hipLaunchKernelGGL((filter_batch_kernel<QR, QC, WPB, PRUNE>), dim3((unsigned)grid),
                       dim3(WPB * WAVE), 0, st, fr, ts, tb, n, tot, claim, ctr, lpr);
    return (int)hipGetLastError();
}

template <int QR, int QC, int WPB, bool PRUNE>
int occupancy_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, filter_batch_kernel<QR, QC, WPB, PRUNE>, WPB * WAVE, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// Supported tile shapes (rows x columns) and workgroup sizes.
#define KNNF_SHAPE(FN, QR, QC, ...)                                                        \
    case (QR) * 10000 + (QC) * 100 + 1:                                                    \
        return pr ? FN<QR, QC, 1, true>(__VA_ARGS__) : FN<QR, QC, 1, false>(__VA_ARGS__);  \
    case (QR) * 10000 + (QC) * 100 + 2:                                                    \
        return pr ? FN<QR, QC, 2, true>(__VA_ARGS__) : FN<QR, QC, 2, false>(__VA_ARGS__);  \
    case (QR) * 10000 + (QC) * 100 + 4:                                                    \
        return pr ? FN<QR, QC, 4, true>(__VA_ARGS__) : FN<QR, QC, 4, false>(__VA_ARGS__);

#define KNNF_DISPATCH(FN, ...)                                                  \
    do {                                                                        \
        const bool pr = cfg.pruned != 0;                                        \
        switch (cfg.rows * 10000 + cfg.cols * 100 + cfg.waves) {                \
            KNNF_SHAPE(FN, 1, 8, __VA_ARGS__)                                   \
            KNNF_SHAPE(FN, 1, 16, __VA_ARGS__)                                  \
            KNNF_SHAPE(FN, 2, 4, __VA_ARGS__)                                   \
            KNNF_SHAPE(FN, 2, 8, __VA_ARGS__)                                   \
            KNNF_SHAPE(FN, 4, 4, __VA_ARGS__)                                   \
        default:                                                                \
            return (int)hipErrorInvalidValue;                                   \
        }                                                                       \
    } while (0)

}  // namespace

int launch_filter_frame(const FrameDesc& f, const LaunchCfg& cfg, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    KNNF_DISPATCH(launch_frame_t, f, cfg.chunk_log2, st);
}

int launch_filter_batch(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        const uint32_t* d_tile_base, uint32_t nframes, uint32_t total_tasks,
                        uint32_t* d_counter, const LaunchCfg& cfg, int grid_blocks, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    KNNF_DISPATCH(launch_batch_t, d_frames, d_task_start, d_tile_base, nframes, total_tasks,
                  d_counter, grid_blocks, cfg.chunk_log2, st);
}

int persistent_blocks_per_cu(const LaunchCfg& cfg) { KNNF_DISPATCH(occupancy_t); }

int launch_filter_items(const FrameDesc* d_frames, const uint32_t* d_task_start,
                        const uint32_t* d_tile_base, uint32_t nframes, uint32_t total_tasks,
                        const LaunchCfg& cfg, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    KNNF_DISPATCH(launch_items_t, d_frames, d_task_start, d_tile_base, nframes, total_tasks,
                  cfg.chunk_log2, st);
}

// ---- Input check (validation before a launch): *flag = gen when any pc1 or
// prob value of the frames is NaN or infinite (exponent bits all ones).
__device__ __forceinline__ bool nonfinite(uint32_t u) { return (u & 0x7f800000u) == 0x7f800000u; }

// Any non-finite value among words t0, t0 + stride, ... of n words at p
// (16-byte loads where p is 16-byte aligned).
__device__ __forceinline__ bool scan_nonfinite(const float* p, size_t n, size_t t0, size_t stride) {
    bool bad = false;
    size_t k = t0;
    if (((uintptr_t)p & 15) == 0) {
        const uint4* __restrict__ q = (const uint4*)p;
        const size_t n4 = n >> 2;
        for (; k < n4; k += stride) {
            const uint4 v = q[k];
            bad = bad || nonfinite(v.x) || nonfinite(v.y) || nonfinite(v.z) || nonfinite(v.w);
        }
        k = (n4 << 2) + t0;
    }
    const uint32_t* __restrict__ w = (const uint32_t*)p;
    for (; k < n; k += stride) bad = bad || nonfinite(w[k]);
    return bad;
}

__device__ __forceinline__ void check_frame(const FrameDesc& f, size_t t0, size_t stride,
                                            uint32_t* flag, uint32_t gen) {
    const size_t px = (size_t)f.H * (size_t)f.W;
    const bool bad = scan_nonfinite(f.pc1, px, t0, stride) ||
                     scan_nonfinite(f.prob, px * (size_t)f.C, t0, stride);
    if (ballot(bad) && lane_id() == 0)
        __hip_atomic_store(flag, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(256) check_frame_kernel(FrameDesc f, uint32_t* flag, uint32_t gen) {
    check_frame(f, (size_t)blockIdx.x * blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x,
                flag, gen);
}

// Frames of a batch table: blockIdx.y strides over the frames, blockIdx.x
// over each frame's values.
__global__ void __launch_bounds__(256)
check_items_kernel(const FrameDesc* __restrict__ frames, uint32_t n, uint32_t* flag, uint32_t gen) {
    for (uint32_t k = blockIdx.y; k < n; k += gridDim.y)
        check_frame(frames[k], (size_t)blockIdx.x * blockDim.x + threadIdx.x,
                    (size_t)gridDim.x * blockDim.x, flag, gen);
}

int launch_check_frame(const FrameDesc& f, uint32_t* flag, uint32_t gen, void* stream) {
    const size_t words = (size_t)f.H * (size_t)f.W * (size_t)(f.C + 1);
    // about 16 words per thread, at most 1024 workgroups
    const size_t blocks = std::min<size_t>(1024, std::max<size_t>(1, words / (256 * 16)));
    hipLaunchKernelGGL(check_frame_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, f, flag, gen);
    return (int)hipGetLastError();
}

int launch_check_items(const FrameDesc* d_frames, uint32_t n, uint32_t max_words, uint32_t* flag,
                       uint32_t gen, void* stream) {
    const unsigned bx = (unsigned)std::min<size_t>(64, std::max<size_t>(1, max_words / (256 * 16)));
    const unsigned by = std::min<unsigned>(n, 65535u);
    hipLaunchKernelGGL(check_items_kernel, dim3(bx, by), dim3(256), 0, (hipStream_t)stream,
                       d_frames, n, flag, gen);
    return (int)hipGetLastError();
}

__global__ void zero_counter_kernel(uint32_t* p) { *p = 0u; }

int launch_zero_counter(uint32_t* d_counter, void* stream) {
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, d_counter);
    return (int)hipGetLastError();
}

__global__ void __launch_bounds__(256) put_table_kernel(TableWords t, uint32_t* __restrict__ base) {
    for (int r = 0; r < 3; ++r)
        for (uint32_t k = threadIdx.x; k < t.len[r]; k += blockDim.x) base[t.dst[r] + k] = t.w[t.src[r] + k];
}

int launch_put_table(const TableWords& t, uint32_t* d_base, void* stream) {
    hipLaunchKernelGGL(put_table_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, t, d_base);
    return (int)hipGetLastError();
}

// Four independent loads in flight per thread: reads of mapped host memory
// have long latency.
__device__ __forceinline__ uint32_t pair_word(const uint32_t* __restrict__ a, uint32_t na,
                                              const uint32_t* __restrict__ b, uint32_t k) {
    return k < na ? a[k] : b[k - na];
}
__device__ __forceinline__ void pair_put(uint32_t* __restrict__ da, uint32_t na,
                                         uint32_t* __restrict__ db, uint32_t k, uint32_t v) {
    if (k < na)
        da[k] = v;
    else
        db[k - na] = v;
}

__global__ void __launch_bounds__(256)
copy_pair_kernel(const uint32_t* __restrict__ a, uint32_t* __restrict__ da, uint32_t na,
                 const uint32_t* __restrict__ b, uint32_t* __restrict__ db, uint32_t nb) {
    const uint32_t n = na + nb;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    for (; k + 3 * stride < n; k += 4 * stride) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = pair_word(a, na, b, k + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) pair_put(da, na, db, k + u * stride, v[u]);
    }
    for (; k < n; k += stride) pair_put(da, na, db, k, pair_word(a, na, b, k));
}

int launch_copy_pair(const uint32_t* a, uint32_t* da, uint32_t na, const uint32_t* b,
                     uint32_t* db, uint32_t nb, void* stream) {
    const uint32_t n = na + nb;
    // 64 workgroups already reach the host link's bandwidth (57 GB/s measured)
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(64, (n + 1023) / 1024));
    hipLaunchKernelGGL(copy_pair_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a, da,
                       na, b, db, nb);
    return (int)hipGetLastError();
}

}  // namespace knnf
