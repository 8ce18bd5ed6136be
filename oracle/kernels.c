/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct loops for the eight workload kernels of the
 * co-execution mix.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this file's library; the product path never calls it.
 * It shares no source with the GPU path.
 *
 * The paper names its workloads only by name and size (its benchmark
 * description table); the precise definition of each workload is the one
 * stated beside each function below.  Floating point truth is computed in
 * double; the polynomial also has a single-precision fused-multiply-add
 * variant in the same evaluation order as the GPU kernel, for bit-exact
 * comparison.  OpenMP only splits the loop over independent outputs.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

/* K_A polynomial: y[t] = sum_{k=0}^{ncoef-1} c[k] * x[t]^k, in double.
 * scale[t] = sum_k |c[k]| |x[t]|^k bounds the rounding error of any
 * evaluation order. */
void orc_poly_f64(const float *x, int64_t n, const float *c, int ncoef,
                  double *y, double *scale) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; ++t) {
        double xt = x[t], p = 1.0, s = 0.0, a = 0.0;
        for (int k = 0; k < ncoef; ++k) {
            s += (double)c[k] * p;
            a += fabs((double)c[k]) * fabs(p);
            p *= xt;
        }
        y[t] = s;
        if (scale) scale[t] = a;
    }
}

/* Same polynomial by Horner's rule in single precision, one fused
 * multiply-add per coefficient from the highest degree down:
 * acc = c[n-1]; acc = fmaf(acc, x, c[k]) for k = n-2 .. 0. */
void orc_poly_f32_horner(const float *x, int64_t n, const float *c, int ncoef,
                         float *y) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; ++t) {
        float acc = c[ncoef - 1];
        for (int k = ncoef - 2; k >= 0; --k) acc = fmaf(acc, x[t], c[k]);
        y[t] = acc;
    }
}

/* K_B random gather: out[t] = table[idx[t]]. */
void orc_gather_i32(const int32_t *idx, int64_t n, const int32_t *table,
                    int32_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; ++t) out[t] = table[idx[t]];
}

/* SGEMM: C = A B, A m x k, B k x n, row-major, accumulated in double. */
void orc_sgemm_f64(const float *A, const float *B, int64_t m, int64_t n,
                   int64_t k, double *C) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double *ci = C + i * n;
        for (int64_t j = 0; j < n; ++j) ci[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double a = A[i * k + p];
            const float *bp = B + p * n;
            for (int64_t j = 0; j < n; ++j) ci[j] += a * (double)bp[j];
        }
    }
}

/* Selected entries of C = A B: out[s] = sum_p A[ri[s], p] B[p, cj[s]]. */
void orc_sgemm_entries(const float *A, const float *B, int64_t n, int64_t k,
                       const int64_t *ri, const int64_t *cj, int64_t ns,
                       double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        double acc = 0.0;
        for (int64_t p = 0; p < k; ++p)
            acc += (double)A[ri[s] * k + p] * (double)B[p * n + cj[s]];
        out[s] = acc;
    }
}

/* CSR sparse matrix times dense vector: y[i] = sum_j val[j] x[col[j]] over
 * row i's entries; scale[i] = sum_j |val[j] x[col[j]]|. */
void orc_spmv_f64(const int32_t *row_ptr, const int32_t *col, const float *val,
                  const float *x, int64_t nrows, double *y, double *scale) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0, a = 0.0;
        for (int32_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
            double v = (double)val[j] * (double)x[col[j]];
            s += v;
            a += fabs(v);
        }
        y[i] = s;
        if (scale) scale[i] = a;
    }
}

/* Five-point stencil, `iters` Jacobi sweeps on an ny x nx row-major grid:
 * interior u'[i][j] = c0 u[i][j] + c1 (u[i-1][j] + u[i+1][j] + u[i][j-1] +
 * u[i][j+1]); boundary cells keep their value.  Result in out (double). */
void orc_stencil_f64(const float *u0, int64_t ny, int64_t nx, int iters,
                     double c0, double c1, double *out) {
    double *a = (double *)malloc(sizeof(double) * ny * nx);
    double *b = out;
    for (int64_t i = 0; i < ny * nx; ++i) a[i] = u0[i];
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < ny; ++i) {
            for (int64_t j = 0; j < nx; ++j) {
                int64_t q = i * nx + j;
                if (i == 0 || j == 0 || i == ny - 1 || j == nx - 1)
                    b[q] = a[q];
                else
                    b[q] = c0 * a[q] +
                           c1 * (a[q - nx] + a[q + nx] + a[q - 1] + a[q + 1]);
            }
        }
        double *t = a; a = b; b = t;
    }
    /* after the loop the newest field is in `a` */
    if (a != out) memcpy(out, a, sizeof(double) * ny * nx);
    free(a == out ? b : a);
}

/* The same stencil's value after `iters` sweeps at selected cells only.
 * A cell's value after t sweeps depends only on cells within Manhattan
 * distance t, so each sample sweeps a (2 iters + 1)^2 window around it (cut
 * at the grid edge); window cells whose neighbours fall outside the window
 * go stale one ring per sweep, which never reaches the centre. */
void orc_stencil_points(const float *u0, int64_t ny, int64_t nx, int iters,
                        double c0, double c1, const int64_t *pi,
                        const int64_t *pj, int64_t ns, double *out) {
#pragma omp parallel for schedule(dynamic)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i0 = pi[s] - iters, i1 = pi[s] + iters;
        int64_t j0 = pj[s] - iters, j1 = pj[s] + iters;
        if (i0 < 0) i0 = 0;
        if (j0 < 0) j0 = 0;
        if (i1 > ny - 1) i1 = ny - 1;
        if (j1 > nx - 1) j1 = nx - 1;
        int64_t h = i1 - i0 + 1, w = j1 - j0 + 1;
        double *a = (double *)malloc(sizeof(double) * h * w);
        double *b = (double *)malloc(sizeof(double) * h * w);
        for (int64_t i = 0; i < h; ++i)
            for (int64_t j = 0; j < w; ++j)
                a[i * w + j] = u0[(i0 + i) * nx + (j0 + j)];
        for (int it = 0; it < iters; ++it) {
            for (int64_t i = 0; i < h; ++i) {
                for (int64_t j = 0; j < w; ++j) {
                    int64_t gi = i0 + i, gj = j0 + j, q = i * w + j;
                    int edge = gi == 0 || gj == 0 || gi == ny - 1 || gj == nx - 1;
                    int inside = i > 0 && j > 0 && i < h - 1 && j < w - 1;
                    if (edge || !inside)
                        b[q] = a[q];
                    else
                        b[q] = c0 * a[q] + c1 * (a[q - w] + a[q + w] +
                                                 a[q - 1] + a[q + 1]);
                }
            }
            double *t = a; a = b; b = t;
        }
        out[s] = a[(pi[s] - i0) * w + (pj[s] - j0)];
        free(a);
        free(b);
    }
}

/* Black-Scholes European call and put (no dividends), in double:
 *   d1 = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt T),  d2 = d1 - sigma sqrt T
 *   N(z) = erfc(-z / sqrt 2) / 2
 *   call = S N(d1) - K e^{-rT} N(d2),  put = K e^{-rT} N(-d2) - S N(-d1). */
void orc_bs_f64(const float *S, const float *K, const float *T, int64_t n,
                double r, double sigma, double *call, double *put) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = S[i], k = K[i], t = T[i];
        double sq = sigma * sqrt(t);
        double d1 = (log(s / k) + (r + 0.5 * sigma * sigma) * t) / sq;
        double d2 = d1 - sq;
        double disc = k * exp(-r * t);
        double nd1 = 0.5 * erfc(-d1 / sqrt(2.0));
        double nd2 = 0.5 * erfc(-d2 / sqrt(2.0));
        double nmd1 = 0.5 * erfc(d1 / sqrt(2.0));
        double nmd2 = 0.5 * erfc(d2 / sqrt(2.0));
        call[i] = s * nd1 - disc * nd2;
        put[i] = disc * nmd2 - s * nmd1;
    }
}

/* 256-bin histogram of bytes: bins[v] = #{t : data[t] == v}. */
void orc_hist_u8(const uint8_t *data, int64_t n, uint64_t *bins) {
    for (int v = 0; v < 256; ++v) bins[v] = 0;
#pragma omp parallel
    {
        uint64_t loc[256];
        for (int v = 0; v < 256; ++v) loc[v] = 0;
#pragma omp for schedule(static)
        for (int64_t t = 0; t < n; ++t) loc[data[t]]++;
#pragma omp critical
        for (int v = 0; v < 256; ++v) bins[v] += loc[v];
    }
}

/* Sorted-array lookup: out[q] = smallest i with keys[i] >= query[q]
 * (nkeys if there is none), by plain binary search over [0, nkeys). */
void orc_lower_bound_u32(const uint32_t *keys, int64_t nkeys,
                         const uint32_t *query, int64_t nq, int32_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nq; ++t) {
        int64_t lo = 0, hi = nkeys;
        uint32_t v = query[t];
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (keys[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        out[t] = (int32_t)lo;
    }
}
