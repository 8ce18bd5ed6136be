/*
 * Seeded synthetic inputs for the workload kernels.
 *
 * This module only draws random numbers and lays them out in the shapes the
 * workloads use.  It holds none of the scheduling method's arithmetic and none
 * of the workload kernels' arithmetic; the CPU oracle and the GPU path both
 * take their inputs from here.
 *
 * Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used counter-style:
 *   key(seed, stream) = seed * 2^32 + stream            (uint64, wrapping)
 *   r(seed, stream, i) = output number i (0-based) of the SplitMix64
 *                        sequence whose state starts at key, i.e.
 *                        mix(key + (i + 1) * GOLDEN_GAMMA)
 * Derived values:
 *   uniform f32 in [a, b): fmaf(b - a, (float)(r >> 40) * 2^-24, a)
 *   uniform integer in [0, n), n <= 2^32: ((r >> 32) * n) >> 32   (Lemire)
 *   byte: r >> 56
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm_key(uint64_t seed, uint64_t stream) {
    return seed * 0x100000000ULL + stream;
}

static inline uint64_t sm_at(uint64_t key, uint64_t i) {
    return sm_mix(key + (i + 1) * GOLDEN_GAMMA);
}

static inline uint32_t sm_below(uint64_t r, uint64_t n) {
    return (uint32_t)(((r >> 32) * n) >> 32);
}

static inline float sm_unif(uint64_t r, float a, float b) {
    float u = (float)(r >> 40) * 0x1p-24f;
    return fmaf(b - a, u, a);
}

void synth_u64(uint64_t seed, uint64_t stream, uint64_t start, int64_t n,
               uint64_t *out) {
    uint64_t key = sm_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = sm_at(key, start + (uint64_t)i);
}

void synth_uniform_f32(uint64_t seed, uint64_t stream, uint64_t start,
                       int64_t n, float a, float b, float *out) {
    uint64_t key = sm_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = sm_unif(sm_at(key, start + (uint64_t)i), a, b);
}

void synth_below_u32(uint64_t seed, uint64_t stream, uint64_t start,
                     int64_t n, uint64_t bound, uint32_t *out) {
    uint64_t key = sm_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = sm_below(sm_at(key, start + (uint64_t)i), bound);
}

void synth_bytes(uint64_t seed, uint64_t stream, uint64_t start, int64_t n,
                 uint8_t *out) {
    uint64_t key = sm_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = (uint8_t)(sm_at(key, start + (uint64_t)i) >> 56);
}

/* CSR structure: row i holds minlen + below(maxlen - minlen + 1) entries;
 * its columns are drawn uniformly over [0, ncols) with replacement and then
 * sorted ascending within the row.  row_ptr has nrows + 1 entries. */
int64_t synth_csr_rowptr(uint64_t seed, uint64_t stream_len, int64_t nrows,
                         uint32_t minlen, uint32_t maxlen, int32_t *row_ptr) {
    uint64_t key = sm_key(seed, stream_len);
    int64_t acc = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        uint32_t len = minlen + sm_below(sm_at(key, (uint64_t)i),
                                         (uint64_t)(maxlen - minlen + 1));
        acc += len;
        row_ptr[i + 1] = (int32_t)acc;
    }
    return acc;
}

void synth_csr_cols(uint64_t seed, uint64_t stream_col, int64_t nrows,
                    uint32_t ncols, const int32_t *row_ptr, int32_t *col) {
    uint64_t key = sm_key(seed, stream_col);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        int32_t b = row_ptr[i], e = row_ptr[i + 1];
        for (int32_t j = b; j < e; ++j) {
            int32_t c = (int32_t)sm_below(sm_at(key, (uint64_t)j), ncols);
            int32_t k = j;
            while (k > b && col[k - 1] > c) {  /* insertion sort */
                col[k] = col[k - 1];
                --k;
            }
            col[k] = c;
        }
    }
}

/* Strictly increasing keys: key[i] = sum_{j<=i} (1 + below(gap_max)). */
void synth_sorted_keys(uint64_t seed, uint64_t stream, int64_t n,
                       uint32_t gap_max, uint32_t *out) {
    uint64_t key = sm_key(seed, stream);
    uint64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) {
        acc += 1 + sm_below(sm_at(key, (uint64_t)i), gap_max);
        out[i] = (uint32_t)acc;
    }
}

/* FNV-1a over a byte buffer, for quick equality checks of large inputs. */
uint64_t synth_fnv1a(const uint8_t *p, int64_t n) {
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int64_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ULL;
    }
    return h;
}
