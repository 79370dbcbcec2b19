// knnf_spectral.hip -- the KNN filter at lambda = 0 (Sec. II.C.3, Eq. 1 with
// the spatial weight set to zero), for CDNA4 (gfx950).
//
// With lambda = 0 the row and column terms of Eq. 1 vanish (fl32(0 * x) = 0,
// so a = b = 0) and the distance of a candidate p to the query q is
// d = fl32(e * e), e = fl32(I_q - I_p): a function of the PC1 values alone,
// and a monotone one on each side of I_q (binary32 subtraction and squaring
// round monotonically).  The candidates of q are the pixels of rows
// max(0, r - R) .. min(H - 1, r + R), every column: the same set for every
// pixel of query row r.  So the K nearest are found as a 1-D selection in
// a band sorted by value; one workgroup serves two query rows r0, r0 + 1
// and sorts the band of both windows (2R + 2 rows, clipped):
//   1. the workgroup sorts the band's (value, linear index) keys in LDS:
//      each thread sorts the T <= 16 keys it loaded in registers (a bitonic
//      network), then ten merge-path rounds double the sorted runs (each
//      thread finds its output range with one binary search along the merge
//      diagonal, merges T keys into registers, and writes them back after a
//      barrier, so the merge needs no second buffer); keys sit in LDS at
//      XOR-swizzled positions, which spreads a wavefront's stores of 16
//      consecutive keys per lane over the banks;
//   2. each lane takes one query pixel of the two rows: a binary search finds
//      where I_q falls in the sorted band; two cursors walk outward (values
//      below and above I_q), skipping the band row that lies outside the
//      query's own window, taking at each step the whole run of candidates
//      whose distance equals the smaller of the two cursors' distances (a
//      run's extent is found by a binary search, since the distance is
//      monotone on each side), so the candidates come out in ascending
//      distance; within a run, ascending linear index.  A run whose values
//      are all equal on each side is already in index order in the sorted
//      band (keys sort by value, then index), so its keys inside the query's
//      window are found by two binary searches on the index, and two such
//      runs merge in index order; a run spanning several values (rounding of
//      the subtraction can give distinct values the same distance) is
//      emitted by repeated minimum.  That is the strict (d, idx) order of the
//      general kernels, so the neighbour lists are the same;
//   3. Eq. 2: the class sums add the neighbours' probabilities in that order
//      from +0 (binary32), then one correctly rounded division by K; the
//      class map is the argmax of the sums, lowest class on ties.  The
//      probabilities are gathered eight neighbours at a time, so the loads of
//      a group are in flight together (one at a time, each waited for its
//      predecessor's latency).
// Work: O(n log n) per query row for the sort (n = band size) and
// O(log n + K) per query, against O(n) distances per query for the scans.
// Two query rows per workgroup halve the sorting per row and put the
// W480 x H380 frame's 190 workgroups on the chip in one round (one row per
// workgroup: 380 workgroups, two rounds, 0.255 against 0.183 ms).  Used for a
// single frame under the pruned search when lambda == 0 and the band holds at
// most 16,384 pixels (it must fit in LDS).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/knnf.h"
#include "knnf_device.h"

namespace knnf {
namespace {

constexpr int SP_THREADS = 1024;               // threads per workgroup (one query row)
constexpr int SP_T = 16;                       // keys per thread at most
constexpr int SP_MAX = SP_THREADS * SP_T;      // band size at most (16,384 keys, 128 KiB)
constexpr uint64_t SP_PAD = ~0ull;             // sorts after every real key
constexpr int SP_MAX_C = KNNF_MAX_C;           // class sums held per lane
constexpr int SP_RING = 8;                     // neighbours per group of Eq. 2 gathers
static_assert(SP_MAX_C % 4 == 0, "classes are gathered four at a time");

// Order-preserving map of binary32 bit patterns to unsigned integers
// (negative values reversed below the positive ones; -0 just below +0).
__device__ __forceinline__ uint32_t sortable(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unsortable(uint32_t s) {
    return __uint_as_float((s & 0x80000000u) ? (s & 0x7fffffffu) : ~s);
}
// LDS position of band key e: the low four bits of e are XORed with the next
// four, so the 16 keys a thread writes one after another (one store per key,
// 64 lanes at a stride of 16 keys) spread over the banks instead of landing
// in the same two.
__device__ __forceinline__ int sw(int e) { return e ^ ((e >> 4) & 15); }
__device__ __forceinline__ float key_value(uint64_t k) { return unsortable((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_index(uint64_t k) { return (uint32_t)k; }

// Eq. 1 at lambda = 0, as the binary32 bit pattern (non-negative values
// compare as unsigned integers): fmaf(e, e, fmaf(b, b, a * a)) with a = b = 0.
__device__ __forceinline__ uint32_t dist0(float x, float v) {
    const float e = x - v;
    return __float_as_uint(fmaf(e, e, 0.0f));
}

template <int N>
__device__ __forceinline__ void sort_regs(uint64_t (&v)[N]) {
    // bitonic network over N (a power of two) keys held in registers
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t a = v[i], b = v[l];
                    const bool sw = up ? (a > b) : (a < b);
                    v[i] = sw ? b : a;
                    v[l] = sw ? a : b;
                }
            }
        }
    }
}

// Sorts keys[0 .. SP_THREADS * T) (T a power of two <= SP_T) in LDS.
__device__ __forceinline__ void sort_band(uint64_t* keys, int T, uint64_t (&v)[SP_T]) {
    const int t = threadIdx.x;
    sort_regs<SP_T>(v);  // pads sort last, so the first T hold this thread's keys
#pragma unroll
    for (int o = 0; o < SP_T; ++o)
        if (o < T) keys[sw(t * T + o)] = v[o];
    __syncthreads();
    for (int s = T; s < SP_THREADS * T; s <<= 1) {
        // this thread's T outputs of the merge of runs A = [base, base + s)
        // and B = [base + s, base + 2s)
        const int out0 = t * T;
        const int base = out0 & ~(2 * s - 1);
        const int k = out0 - base;
        const int bA = base, bB = base + s;  // runs A and B (key positions)
        int lo = max(0, k - s), hi = min(k, s);
        while (lo < hi) {  // first i with A[i] > B[k - i - 1] (A first on ties)
            const int mid = (lo + hi) >> 1;
            if (keys[sw(bA + mid)] <= keys[sw(bB + k - mid - 1)]) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = k - lo;
        uint64_t a = i < s ? keys[sw(bA + i)] : SP_PAD, b = j < s ? keys[sw(bB + j)] : SP_PAD;
#pragma unroll
        for (int o = 0; o < SP_T; ++o) {
            if (o < T) {
                const bool ta = j >= s || (i < s && a <= b);
                v[o] = ta ? a : b;
                if (ta) {
                    ++i;
                    a = i < s ? keys[sw(bA + i)] : SP_PAD;
                } else {
                    ++j;
                    b = j < s ? keys[sw(bB + j)] : SP_PAD;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < SP_T; ++o)
            if (o < T) keys[sw(out0 + o)] = v[o];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SP_THREADS)
spectral_filter_kernel(FrameDesc f, int T) {
    __shared__ uint64_t keys[SP_MAX];
    // two query rows per workgroup share one band: the rows of both windows
    const int r0 = 2 * (int)blockIdx.x;
    const int t = threadIdx.x;
    const int W = f.W, C = f.C, K = f.K;
    const int lo = max(0, r0 - f.R), hi = min(f.H - 1, r0 + 1 + f.R);
    const int n = (hi - lo + 1) * W;
    const uint32_t first = (uint32_t)lo * (uint32_t)W;

    // ---- 1. the band's keys, sorted
    uint64_t v[SP_T];
#pragma unroll
    for (int u = 0; u < SP_T; ++u) {
        const int e = t + SP_THREADS * u;
        v[u] = SP_PAD;
        if (u < T && e < n)
            v[u] = ((uint64_t)sortable(f.pc1[first + e]) << 32) | (uint64_t)(first + e);
    }
    sort_band(keys, T, v);

    // ---- 2. + 3. one lane per query pixel of rows r0 and r0 + 1
    const float* __restrict__ prob = f.prob;
    const bool vec4 = C % 4 == 0 && ((uintptr_t)prob & 15) == 0;
    for (int qi = t; qi < 2 * W; qi += SP_THREADS) {
        const int qr = qi >= W ? 1 : 0;
        const int r = r0 + qr, c = qi - qr * W;
        if (r >= f.H) break;
        // the query's own window as band offsets [lo_q, hi_q): keys of the
        // band's other rows are skipped
        const int lo_q = (max(0, r - f.R) - lo) * W;
        const int hi_q = (min(f.H - 1, r + f.R) - lo + 1) * W;
        auto valid = [&](int p) __attribute__((always_inline)) {
            const int e = (int)(key_index(keys[sw(p)]) - first);
            return e >= lo_q && e < hi_q;
        };
        const uint32_t q = (uint32_t)r * (uint32_t)W + (uint32_t)c;
        const float x = f.pc1[q];
        // first key whose value is >= x
        const uint64_t probe = (uint64_t)sortable(x) << 32;
        int a0 = 0, a1 = n;
        while (a0 < a1) {
            const int mid = (a0 + a1) >> 1;
            if (keys[sw(mid)] < probe) a0 = mid + 1;
            else a1 = mid;
        }
        int L = a0 - 1, Rc = a0;  // next candidates below and above
        float s[SP_MAX_C];
#pragma unroll
        for (int cl = 0; cl < SP_MAX_C; ++cl) s[cl] = 0.0f;
        int k = 0;  // neighbours emitted
        // Eq. 2 gathers in groups of SP_RING neighbours, so that a group's
        // loads are in flight together; each class still adds its
        // neighbours' probabilities one by one in order
        uint32_t ring[SP_RING];
        int nring = 0;
        auto flush = [&](int cnt) __attribute__((always_inline)) {
#pragma unroll
            for (int c4 = 0; c4 < SP_MAX_C; c4 += 4) {
                if (c4 < C) {
                    float pv[SP_RING][4];
                    if (vec4) {  // C a multiple of 4: one 16-byte load per neighbour
#pragma unroll
                        for (int u = 0; u < SP_RING; ++u) {
                            const float4 x4 = u < cnt ? *(const float4*)(prob + (size_t)ring[u] * C + c4)
                                                     : make_float4(0.f, 0.f, 0.f, 0.f);
                            pv[u][0] = x4.x;
                            pv[u][1] = x4.y;
                            pv[u][2] = x4.z;
                            pv[u][3] = x4.w;
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < SP_RING; ++u)
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                pv[u][j] = (u < cnt && c4 + j < C) ? prob[(size_t)ring[u] * C + c4 + j]
                                                                   : 0.0f;
                    }
#pragma unroll
                    for (int u = 0; u < SP_RING; ++u)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (u < cnt && c4 + j < C) s[c4 + j] = s[c4 + j] + pv[u][j];
                }
            }
        };
        auto emit = [&](uint64_t key, uint32_t d) __attribute__((always_inline)) {
            const uint32_t idx = key_index(key);
            if (f.out_nbr) {
                f.out_nbr[(size_t)q * K + k] = (int32_t)idx;
                f.out_dist[(size_t)q * K + k] = __uint_as_float(d);
            }
#pragma unroll
            for (int u = 0; u < SP_RING; ++u) ring[u] = u == nring ? idx : ring[u];
            if (++nring == SP_RING) {
                flush(SP_RING);
                nring = 0;
            }
            ++k;
        };
        const uint32_t NONE = 0xffffffffu;  // above every distance pattern
        while (k < K) {
            while (L >= 0 && !valid(L)) --L;
            while (Rc < n && !valid(Rc)) ++Rc;
            const uint32_t dL = L >= 0 ? dist0(x, key_value(keys[sw(L)])) : NONE;
            const uint32_t dR = Rc < n ? dist0(x, key_value(keys[sw(Rc)])) : NONE;
            const uint32_t dm = min(dL, dR);
            if (dm == NONE) break;  // the band holds fewer than K pixels (not a valid frame)
            // the run of distance dm on each side: [aL, L] and [Rc, bR]
            int aL = L + 1, bR = Rc - 1;
            if (dL == dm) {
                aL = L;
                if (aL > 0 && dist0(x, key_value(keys[sw(aL - 1)])) == dm) {
                    int b0 = 0, b1 = L;  // first index whose distance is <= dm
                    while (b0 < b1) {
                        const int mid = (b0 + b1) >> 1;
                        if (dist0(x, key_value(keys[sw(mid)])) <= dm) b1 = mid;
                        else b0 = mid + 1;
                    }
                    aL = b0;
                }
            }
            if (dR == dm) {
                bR = Rc;
                if (bR + 1 < n && dist0(x, key_value(keys[sw(bR + 1)])) == dm) {
                    int b0 = Rc, b1 = n - 1;  // last index whose distance is <= dm
                    while (b0 < b1) {
                        const int mid = (b0 + b1 + 1) >> 1;
                        if (dist0(x, key_value(keys[sw(mid)])) <= dm) b0 = mid;
                        else b1 = mid - 1;
                    }
                    bR = b0;
                }
            }
            const bool oneL = aL > L || (keys[sw(aL)] >> 32) == (keys[sw(L)] >> 32);
            const bool oneR = Rc > bR || (keys[sw(Rc)] >> 32) == (keys[sw(bR)] >> 32);
            if (oneL && oneR) {
                // each side one value, so index order is storage order: keep
                // the positions whose index lies in the query's window (two
                // binary searches per side), then merge the two sides
                const uint32_t ilo = first + (uint32_t)lo_q, ihi = first + (uint32_t)hi_q;
                auto restrict_to = [&](int a, int b, int& sa, int& sb) __attribute__((always_inline)) {
                    int p0 = a, p1 = b + 1;
                    while (p0 < p1) {  // first position with index >= ilo
                        const int mid = (p0 + p1) >> 1;
                        if (key_index(keys[sw(mid)]) < ilo) p0 = mid + 1;
                        else p1 = mid;
                    }
                    sa = p0;
                    p1 = b + 1;
                    while (p0 < p1) {  // first position with index >= ihi
                        const int mid = (p0 + p1) >> 1;
                        if (key_index(keys[sw(mid)]) < ihi) p0 = mid + 1;
                        else p1 = mid;
                    }
                    sb = p0 - 1;
                };
                int la = aL, lb = L, ra = Rc, rb = bR;
                if (aL <= L) restrict_to(aL, L, la, lb);
                if (Rc <= bR) restrict_to(Rc, bR, ra, rb);
                const int m = min(max(0, lb - la + 1) + max(0, rb - ra + 1), K - k);
                int i = la, j = ra;
                for (int e = 0; e < m; ++e) {
                    const bool ti = j > rb || (i <= lb && key_index(keys[sw(i)]) < key_index(keys[sw(j)]));
                    emit(ti ? keys[sw(i)] : keys[sw(j)], dm);
                    if (ti) ++i;
                    else ++j;
                }
            } else {
                // several values in the run: ascending index by repeated minimum
                // over the run's keys inside the query's window
                int cntv = 0;
                for (int p = aL; p <= L; ++p) cntv += valid(p) ? 1 : 0;
                for (int p = Rc; p <= bR; ++p) cntv += valid(p) ? 1 : 0;
                const int m = min(cntv, K - k);
                int64_t last = -1;
                for (int e = 0; e < m; ++e) {
                    uint32_t best = 0xffffffffu;
                    uint64_t bk = 0;
                    for (int p = aL; p <= L; ++p) {
                        const uint32_t ix = key_index(keys[sw(p)]);
                        if ((int64_t)ix > last && ix <= best && valid(p)) {
                            best = ix;
                            bk = keys[sw(p)];
                        }
                    }
                    for (int p = Rc; p <= bR; ++p) {
                        const uint32_t ix = key_index(keys[sw(p)]);
                        if ((int64_t)ix > last && ix <= best && valid(p)) {
                            best = ix;
                            bk = keys[sw(p)];
                        }
                    }
                    emit(bk, dm);
                    last = best;
                }
            }
            L = aL - 1;
            Rc = bR + 1;
        }
        flush(nring);
        // Eq. 2 and the class map
        const float kf = (float)K;
        float* op = f.out_prob + (size_t)q * C;
        int best = 0;
        float bs = s[0];
#pragma unroll
        for (int cl = 0; cl < SP_MAX_C; ++cl) {
            if (cl < C) {
                op[cl] = s[cl] / kf;
                if (s[cl] > bs) {
                    bs = s[cl];
                    best = cl;
                }
            }
        }
        f.out_class[q] = best;
    }
}

}  // namespace

// Rows of the band one workgroup sorts: both query rows' windows.
int64_t spectral_band_rows(const FrameDesc& f) { return std::min<int64_t>((int64_t)2 * f.R + 2, f.H); }

bool spectral_fits(const FrameDesc& f) {
    return f.lambda == 0.0f && spectral_band_rows(f) * f.W <= SP_MAX;
}

int launch_spectral_frame(const FrameDesc& f, void* stream) {
    const int64_t n = spectral_band_rows(f) * f.W;
    int T = 1;
    while ((int64_t)T * SP_THREADS < n) T <<= 1;
    hipLaunchKernelGGL(spectral_filter_kernel, dim3((uint32_t)((f.H + 1) / 2)), dim3(SP_THREADS), 0,
                       (hipStream_t)stream, f, T);
    return (int)hipGetLastError();
}

}  // namespace knnf
