/*
 * knn_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for the KNN filtering stage of
 * the spatial-spectral classifier (Lazcano et al., "Parallel Implementations
 * Assessment of a Spatial-Spectral Classifier for Hyperspectral Clinical
 * Applications", Sec. II.C.3, Eq. 1 and Eq. 2; window of Sec. III.A.3).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or helper with the GPU path.
 *
 * What is computed, for every pixel q = (r, c) of an H x W frame:
 *   1. Features (Sec. II.C.3): the one-band value I[q] and the coordinates
 *      scaled by the spatial weight lambda, fr(r) = fl32(lambda * r),
 *      fc(c) = fl32(lambda * c).
 *   2. Window (Sec. III.A.3): candidate rows max(0, r-R) .. min(H-1, r+R),
 *      every column; clipped at the frame edges, the pixel itself included.
 *   3. Distance (Eq. 1, squared Euclidean, no square root), in IEEE binary32
 *      with round-to-nearest-even and no other contraction:
 *         a = fl32(fr(r) - fr(i)),  b = fl32(fc(c) - fc(j)),
 *         e = fl32(I[q] - I[p]),
 *         d = fmaf(e, e, fmaf(b, b, fl32(a * a))).
 *      (Eq. 1 prints (r - j)^2 for the column term; by the definitions under
 *      the equation j is the column, so the term is (c - j)^2.)
 *   4. Selection: all candidates sorted by the strict total order
 *      (d ascending, then linear index i*W + j ascending); the first K are the
 *      neighbours, kept in that order.
 *   5. Averaging (Eq. 2): S_c = sum over the K neighbours, in that order,
 *      starting from +0, each addition rounded to binary32; O_c = fl32(S_c / K)
 *      (a true division).
 *   6. Class map (end of Sec. II.C.3 and Sec. III.A.3.b): the class whose
 *      summed probability is largest; on equal sums the lowest class index.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no -ffast-math), so every float
 * operation is one IEEE binary32 operation and fmaf is the correctly rounded
 * library fused multiply-add.  Rows are split across threads; each pixel is
 * computed independently, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

typedef struct {
    float d;
    int32_t idx;
} cand_t;

/* Strict total order of step 4: distance first, then linear index. */
static int cand_cmp(const void* pa, const void* pb) {
    const cand_t* x = (const cand_t*)pa;
    const cand_t* y = (const cand_t*)pb;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/* Parameter rules shared by every entry point of this file. */
static int check_params(int H, int W, int C, int K, int R, float lambda) {
    if (H < 1 || W < 1) return ORC_EINVAL;
    if (H > (1 << 24) || W > (1 << 24)) return ORC_EINVAL; /* coordinates exact in binary32 */
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX) return ORC_EINVAL;
    if (C < 1 || C > 16) return ORC_EINVAL;
    if (R < 0) return ORC_EINVAL;
    if (K < 1 || K > 64) return ORC_EINVAL;
    /* The smallest window is at the frame edge: min(H, R+1) full rows. */
    {
        int64_t rows = (R + 1 < H) ? (int64_t)(R + 1) : (int64_t)H;
        if ((int64_t)K > rows * (int64_t)W) return ORC_EINVAL;
    }
    if (!isfinite(lambda) || lambda < 0.0f) return ORC_EINVAL;
    if ((double)lambda * (double)(H > W ? H : W) > 1e18) return ORC_EINVAL;
    return ORC_OK;
}

static int check_values(const float* v, int64_t n) {
    for (int64_t t = 0; t < n; ++t)
        if (!isfinite(v[t])) return ORC_EINVAL;
    return ORC_OK;
}

/*
 * One pixel: steps 2-6 above.  cand must hold (2R+1)*W entries.
 */
static void filter_one(int H, int W, int C, int K, int R, float lambda,
                       const float* pc1, const float* prob, int32_t q,
                       cand_t* cand, float* o_prob, int32_t* o_class,
                       int32_t* o_nbr, float* o_dist) {
    const int r = q / W;
    const int c = q % W;
    const int i0 = (r - R < 0) ? 0 : r - R;
    const int i1 = (r + R > H - 1) ? H - 1 : r + R;
    const float fr_q = lambda * (float)r;
    const float fc_q = lambda * (float)c;
    const float iq = pc1[q];
    int n = 0;
    for (int i = i0; i <= i1; ++i) {
        const float a = fr_q - lambda * (float)i;
        const float aa = a * a;
        for (int j = 0; j < W; ++j) {
            const int32_t p = (int32_t)i * W + j;
            const float b = fc_q - lambda * (float)j;
            const float e = iq - pc1[p];
            cand[n].d = fmaf(e, e, fmaf(b, b, aa));
            cand[n].idx = p;
            ++n;
        }
    }
    qsort(cand, (size_t)n, sizeof(cand_t), cand_cmp);

    float s[16];
    for (int cl = 0; cl < C; ++cl) s[cl] = 0.0f;
    for (int k = 0; k < K; ++k) {
        const float* pk = prob + (int64_t)cand[k].idx * C;
        for (int cl = 0; cl < C; ++cl) s[cl] = s[cl] + pk[cl];
    }
    int best = 0;
    for (int cl = 1; cl < C; ++cl)
        if (s[cl] > s[best]) best = cl;
    for (int cl = 0; cl < C; ++cl) o_prob[cl] = s[cl] / (float)K;
    *o_class = best;
    if (o_nbr)
        for (int k = 0; k < K; ++k) o_nbr[k] = cand[k].idx;
    if (o_dist)
        for (int k = 0; k < K; ++k) o_dist[k] = cand[k].d;
}

/*
 * Pixels listed in pix[0..npix-1] (linear indices r*W + c).  Output row t of
 * out_prob (C floats), out_class (1), out_nbr / out_dist (K each, may be NULL)
 * belongs to pix[t].  All pointers are host memory owned by the caller.
 * Returns 0, ORC_EINVAL (bad parameters, non-finite input, index out of
 * range) or ORC_ENOMEM.
 */
int knn_oracle_pixels(int H, int W, int C, int K, int R, float lambda,
                      const float* pc1, const float* prob, const int32_t* pix,
                      int npix, float* out_prob, int32_t* out_class,
                      int32_t* out_nbr, float* out_dist, int nthreads) {
    int st = check_params(H, W, C, K, R, lambda);
    if (st != ORC_OK) return st;
    if (!pc1 || !prob || !out_prob || !out_class || npix < 0) return ORC_EINVAL;
    if (npix > 0 && !pix) return ORC_EINVAL;
    const int64_t npx = (int64_t)H * W;
    if (check_values(pc1, npx) || check_values(prob, npx * C)) return ORC_EINVAL;
    for (int t = 0; t < npix; ++t)
        if (pix[t] < 0 || (int64_t)pix[t] >= npx) return ORC_EINVAL;
    if (nthreads < 1) nthreads = 1;

    const int64_t rows = (2 * (int64_t)R + 1 < H) ? 2 * (int64_t)R + 1 : H;
    const size_t cap = (size_t)(rows * W);
    int fail = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
    {
        cand_t* cand = (cand_t*)malloc(cap * sizeof(cand_t));
        if (!cand) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            fail = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
            for (int t = 0; t < npix; ++t)
                filter_one(H, W, C, K, R, lambda, pc1, prob, pix[t], cand,
                           out_prob + (int64_t)t * C, out_class + t,
                           out_nbr ? out_nbr + (int64_t)t * K : NULL,
                           out_dist ? out_dist + (int64_t)t * K : NULL);
        }
        free(cand);
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

/*
 * Whole frame.  pc1: H*W row-major; prob: H*W*C, class fastest.  Outputs:
 * out_prob H*W*C, out_class H*W, out_nbr / out_dist H*W*K or NULL.
 */
int knn_oracle_filter(int H, int W, int C, int K, int R, float lambda,
                      const float* pc1, const float* prob, float* out_prob,
                      int32_t* out_class, int32_t* out_nbr, float* out_dist,
                      int nthreads) {
    int st = check_params(H, W, C, K, R, lambda);
    if (st != ORC_OK) return st;
    const int64_t npx = (int64_t)H * W;
    int32_t* pix = (int32_t*)malloc((size_t)npx * sizeof(int32_t));
    if (!pix) return ORC_ENOMEM;
    for (int64_t t = 0; t < npx; ++t) pix[t] = (int32_t)t;
    st = knn_oracle_pixels(H, W, C, K, R, lambda, pc1, prob, pix, (int)npx,
                           out_prob, out_class, out_nbr, out_dist, nthreads);
    free(pix);
    return st;
}

/* Number of OpenMP threads a call with nthreads <= 0 would not exceed. */
int knn_oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
