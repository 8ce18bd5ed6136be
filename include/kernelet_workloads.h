/*
 * kernelet_workloads.h -- argument blocks of the eight built-in workload
 * kernels of libkernelet.so (see kernelet_builtin in kernelet.h).
 *
 * Each kernel is launched by the runtime as fn(Args a, kl_slice s) on
 * 256-thread workgroups; the ORIGINAL grid is what kernelet_builtin_grid
 * returns for the argument block, and kernelet_submit rejects any other.
 * All pointers are device pointers; all arrays are dense and row-major.
 * The paper's evaluation names its workloads only by name and size (its
 * benchmark description table); the eight here take their roles (compute
 * bound, memory bound, irregular, latency bound).
 */
#ifndef KERNELET_WORKLOADS_H
#define KERNELET_WORKLOADS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* poly: y[t] = sum_{k<ncoef} coef[k] x[t]^k by Horner's rule in fp32 with one
 * fused multiply-add per coefficient, highest degree first.  One thread per
 * element; grid = ceil(n / 256).  ncoef in [1, 1024]. */
typedef struct {
    const float* x;
    const float* coef;
    float* y;
    uint32_t n;
    uint32_t ncoef;
} kl_poly_args;

/* gather: out[t] = table[idx[t]], idx[t] in [0, table_n).  One thread per
 * element; grid = ceil(n / 256).  Indices outside the table are not read
 * (out[t] = 0). */
typedef struct {
    const int32_t* idx;
    const int32_t* table;
    int32_t* out;
    uint32_t n;
    uint32_t table_n;
} kl_gather_args;

/* sgemm: C = A B in fp32 on matrix cores, A m x k, B k x n, C m x n.
 * m, n multiples of 128, k a multiple of 16.  grid = (m/128) (n/128). */
typedef struct {
    const float* a;
    const float* b;
    float* c;
    uint32_t m, n, k;
} kl_sgemm_args;

/* spmv: y = A x, A in CSR (row_ptr[nrows+1], col[nnz], val[nnz]),
 * x[ncols], y[nrows] in fp32.  16 lanes per row; grid = ceil(nrows / 16).
 * Entries past nnz and columns outside [0, ncols) are skipped. */
typedef struct {
    const int32_t* row_ptr;
    const int32_t* col;
    const float* val;
    const float* x;
    float* y;
    uint32_t nrows;
    uint32_t ncols;
    uint32_t nnz;
    uint32_t reserved;
} kl_spmv_args;

/* stencil: one Jacobi sweep of the 5-point stencil on an ny x nx grid:
 * interior out = c0 in + c1 ((N + S) + (W + E)), boundary cells copied.
 * nx a multiple of 4, in/out 16-byte aligned.  Tiles of 1024 x 32 cells;
 * grid = (ceil(nx/1024), ceil(ny/32), 1). */
typedef struct {
    const float* in;
    float* out;
    uint32_t ny, nx;
    float c0, c1;
} kl_stencil_args;

/* bs: Black-Scholes European call and put for n options (S, K, T) at rate
 * r and volatility sigma.  Four options per thread; grid = ceil(n / 1024).
 * n a multiple of 4. */
typedef struct {
    const float* s;
    const float* k;
    const float* t;
    float* call;
    float* put;
    uint32_t n;
    float r, sigma;
} kl_bs_args;

/* hist: bins[v] += #{t < n : data[t] == v} for 256 bins (the caller zeroes
 * bins first; not idempotent).  n a multiple of 16; each workgroup counts
 * a chunk of 65536 bytes; grid = ceil(n / 65536). */
typedef struct {
    const uint8_t* data;
    uint32_t* bins;
    uint64_t n;
} kl_hist_args;

/* lookup: out[t] = lower_bound(keys, q[t]) = smallest i with keys[i] >=
 * q[t], or nkeys if none; keys sorted ascending.  The search descends a
 * static 32-ary tree of 128-byte nodes to a compressed leaf: leaf j holds
 * keys 64 j .. 64 j + 63 as 16-bit distances below its largest key
 * keys[min(64 j + 63, n - 1)], two per uint32 word (slot 2w in the low
 * half), 32 words per leaf, slots past the last key 0; a leaf whose keys
 * span more than 65534 has 0xffff in the first slot of each of its eight
 * 16-byte pieces (slots 0, 8, ..., 56) and is searched in `keys`.
 * Level 1 entry j is leaf j's largest key, level k + 1 entry i is level k
 * entry min(32 i + 31, m_k - 1); sizes m_1 = ceil(n / 64), m_{k+1} =
 * ceil(m_k / 32), stopping at the first level with at most 1024 entries
 * (searched in LDS); each level padded to 32 entries with 0xffffffff.
 * `index` holds the levels back to back (level 1 first), then the leaves:
 * kernelet_lookup_index_entries(n) uint32 words in all.  The
 * "lookup_index" kernel writes it (one thread per four words, grid =
 * ceil(words / 1024)) and the "lookup" kernel reads it (four queries per
 * thread, eight threads searching each query together, grid =
 * ceil(nq / 1024)).  nq a multiple of 4, 1 <= nkeys <= 2^31 - 64; keys, q, out, index
 * 16-byte aligned. */
typedef struct {
    const uint32_t* keys;
    const uint32_t* q;
    int32_t* out;
    uint32_t* index;
    uint32_t nkeys;
    uint32_t nq;
} kl_lookup_args;

/* Number of uint32 entries of the lookup tree index for n keys. */
uint64_t kernelet_lookup_index_entries(uint32_t nkeys);

/* probe (not a workload): workgroup w adds 1 to visits[w] and writes
 * info[3w] = (XCC_ID << 32) | HW_ID, info[3w+1] = start, info[3w+2] = end
 * (wall clock ticks), after `spin` dependent fmas per thread.
 * grid = n_wg; spin <= 2^24. */
typedef struct {
    uint32_t* visits;
    uint64_t* info;
    uint32_t n_wg;
    uint32_t spin;
} kl_probe_args;

/* ceil_fma, ceil_mfma (not workloads: probes of the chip's FP32 compute
 * ceilings).  ceil_fma: thread t (t < n_wg * 256) keeps 16 chains a_k,
 * starting at k, of a_k <- fma(a_k, mul, add) for `iters` iterations
 * (unpacked VALU FMAs) and writes sum_k a_k to out[t].  ceil_mfma: every
 * wave keeps four 32 x 32 FP32 accumulators, each updated `iters` times by
 * one v_mfma_f32_32x32x2f32 whose A and B hold `mul` and `add` in every
 * lane (so every accumulator entry grows by 2 * mul * add), and thread t
 * writes the sum of its 64 accumulator registers to out[t].  Work:
 * ceil_fma 32 * iters FLOPs per thread; ceil_mfma 4 * 4096 * iters FLOPs
 * per wave.  grid = n_wg; iters <= 2^20. */
typedef struct {
    float* out;
    float mul, add;
    uint32_t n_wg;
    uint32_t iters;
} kl_ceiling_args;

/* ceil_read (a probe of the chip's HBM read bandwidth, not a workload):
 * workgroup w reads the 256 * per_thread float4 at src + 4 * (w * 256 *
 * per_thread), thread t the ones at t, t + 256, t + 512, ... (coalesced
 * 16-byte loads), and writes the sum of its 4 * per_thread floats to
 * out[w * 256 + t].  src holds n_wg * 256 * per_thread float4 (16-byte
 * aligned); out n_wg * 256 floats.  grid = n_wg; per_thread a positive
 * multiple of 8, at most 2^16. */
typedef struct {
    const float* src;
    float* out;
    uint32_t n_wg;
    uint32_t per_thread;
} kl_read_args;

/* synthk_v<V>_l<L> (synthetic kernels of known character, the training
 * population of the surrogate model): thread t (t < n_threads) runs `iters`
 * iterations of one load of src[addr] followed by a chain of `alu`
 * dependent fmas on it; dst[t] receives the result.  addr is
 *   pattern 0 (coalesced): (t + it * n_threads) & mask,
 *   pattern 1 (strided):   (32 t + 7919 it) & mask (one 128-byte line per lane),
 *   pattern 2 (random):    a per-thread linear congruential sequence & mask.
 * The compile-time classes hold about V in {32, 64, 128, 256} VGPRs per lane
 * live across the loop and L in {0, 16, 32, 64} KiB of static LDS per
 * workgroup.  src holds mask + 1 floats (a power of two); dst n_threads;
 * grid = ceil(n_threads / 256); alu <= 4096, iters <= 2^20. */
typedef struct {
    const float* src;
    float* dst;
    uint32_t mask;
    uint32_t n_threads;
    uint32_t iters;
    uint32_t alu;
    uint32_t pattern;
    uint32_t reserved;
} kl_synthk_args;

#ifdef __cplusplus
}
#endif
#endif /* KERNELET_WORKLOADS_H */
