// The eight sliceable workload kernels of the co-execution mix, for gfx950.
//
// Every kernel is launched on a 1-D grid of slice.count workgroups of 256
// threads and recovers its workgroup's id in the original grid as
// slice.offset + blockIdx.x (index rectification, Kernelet Section 4.1).
// Nothing here reads gridDim.  Argument blocks are declared in
// kernelet_workloads.h; the host-side checks of each block and the original
// grid it needs are at the end of this file.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "kernelet.h"
#include "kernelet_device.h"
#include "kernelet_workloads.h"

#define KL_WG 256

// ------------------------------------------------------------------ poly
// Horner's rule, one fma per coefficient from the highest degree down; the
// coefficient index is uniform across the wave, so coefficients come through
// scalar loads.
__global__ __launch_bounds__(KL_WG) void kl_poly(kl_poly_args a, kl_slice s) {
    uint64_t t = (uint64_t)kl_wg_linear(s) * KL_WG + threadIdx.x;
    if (t >= a.n) return;
    const float x = a.x[t];
    const float* __restrict__ c = a.coef;
    int k = (int)a.ncoef - 1;
    float acc = c[k];
#pragma unroll 16
    for (--k; k >= 0; --k) acc = __builtin_fmaf(acc, x, c[k]);
    a.y[t] = acc;
}

// ---------------------------------------------------------------- gather
__global__ __launch_bounds__(KL_WG) void kl_gather(kl_gather_args a, kl_slice s) {
    uint64_t t = (uint64_t)kl_wg_linear(s) * KL_WG + threadIdx.x;
    if (t >= a.n) return;
    int32_t i = a.idx[t];
    a.out[t] = (uint32_t)i < a.table_n ? a.table[i] : 0;
}

// ----------------------------------------------------------------- sgemm
// 128 x 128 output tile per workgroup, K staged through LDS 16 at a time;
// each of the 4 waves owns a 64 x 64 quadrant computed as 2 x 2 blocks of
// v_mfma_f32_32x32x2f32 (A: lane l holds A[l%32][l/32]; B: lane l holds
// B[l/32][l%32]; D register r of lane l is D[8(r/4) + 4(l/32) + r%4][l%32]).
// The next K-panel is prefetched into registers while the current one is
// multiplied.  Tiles are assigned XCD by XCD: workgroup i runs on XCD i % 8,
// so each XCD gets a compact block of tiles that share A rows and B
// columns in its own L2.
typedef float kl_f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void sgemm_tile(uint32_t lin, uint32_t tm, uint32_t tn,
                                           uint32_t* ti, uint32_t* tj) {
    if (tm % 2 == 0 && tn % 4 == 0) {
        uint32_t xcd = lin % 8, j = lin / 8;
        uint32_t rh = tm / 2, rw = tn / 4;
        *ti = (xcd / 4) * rh + j / rw;
        *tj = (xcd % 4) * rw + j % rw;
    } else {
        *ti = lin / tn;
        *tj = lin % tn;
    }
}

__global__ __launch_bounds__(KL_WG) void kl_sgemm(kl_sgemm_args a, kl_slice s) {
    constexpr int BM = 128, BN = 128, BK = 16, PAD = 4;
    __shared__ float As[BK][BM + PAD];
    __shared__ float Bs[BK][BN + PAD];
    const uint32_t tm = a.m / BM, tn = a.n / BN;
    const uint32_t lin = kl_wg_linear(s);
    if (lin >= tm * tn) return;
    uint32_t ti, tj;
    sgemm_tile(lin, tm, tn, &ti, &tj);

    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int wm = (wave / 2) * 64, wn = (wave % 2) * 64;
    const float* __restrict__ A = a.a + (size_t)ti * BM * a.k;
    const float* __restrict__ B = a.b + (size_t)tj * BN;
    const uint32_t K = a.k, N = a.n;

    kl_f32x16 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // global -> register mapping of one K-panel
    const int ar = tid / 4, ac = (tid % 4) * 4;     // A: rows ar, ar+64
    const int br = tid / 32, bc = (tid % 32) * 4;   // B: rows br, br+8
    const float* pa0 = A + (size_t)ar * K + ac;
    const float* pa1 = A + (size_t)(ar + 64) * K + ac;
    const float* pb0 = B + (size_t)br * N + bc;
    const float* pb1 = B + (size_t)(br + 8) * N + bc;
    float4 ra0 = *(const float4*)pa0, ra1 = *(const float4*)pa1;
    float4 rb0 = *(const float4*)pb0, rb1 = *(const float4*)pb1;
    for (uint32_t k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        As[ac + 0][ar] = ra0.x;
        As[ac + 1][ar] = ra0.y;
        As[ac + 2][ar] = ra0.z;
        As[ac + 3][ar] = ra0.w;
        As[ac + 0][ar + 64] = ra1.x;
        As[ac + 1][ar + 64] = ra1.y;
        As[ac + 2][ar + 64] = ra1.z;
        As[ac + 3][ar + 64] = ra1.w;
        *(float4*)&Bs[br][bc] = rb0;
        *(float4*)&Bs[br + 8][bc] = rb1;
        __syncthreads();
        if (k0 + BK < K) {
            const size_t kn = k0 + BK;
            ra0 = *(const float4*)(pa0 + kn);
            ra1 = *(const float4*)(pa1 + kn);
            rb0 = *(const float4*)(pb0 + kn * N);
            rb1 = *(const float4*)(pb1 + kn * N);
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            const int kr = kk + lane / 32, lc = lane % 32;
            float av0 = As[kr][wm + lc], av1 = As[kr][wm + 32 + lc];
            float bv0 = Bs[kr][wn + lc], bv1 = Bs[kr][wn + 32 + lc];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0, bv0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0, bv1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1, bv0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1, bv1, acc[1][1], 0, 0, 0);
        }
    }
    float* __restrict__ C = a.c + (size_t)ti * BM * N + (size_t)tj * BN;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 16; ++r) {
                const int row = wm + 32 * i + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
                const int col = wn + 32 * j + lane % 32;
                C[(size_t)row * N + col] = acc[i][j][r];
            }
}

// ------------------------------------------------------------------ spmv
// 16 lanes per CSR row: strided partial sums, then a butterfly over the 16
// lanes (fixed order, so every launch gives the same bits).
__global__ __launch_bounds__(KL_WG) void kl_spmv(kl_spmv_args a, kl_slice s) {
    const uint32_t row = kl_wg_linear(s) * 16 + threadIdx.x / 16;
    const int l = threadIdx.x % 16;
    float sum = 0.0f;
    if (row < a.nrows) {
        const uint32_t b = (uint32_t)a.row_ptr[row];
        uint32_t e = (uint32_t)a.row_ptr[row + 1];
        if (e > a.nnz) e = a.nnz;
        for (uint32_t j = b + l; j < e; j += 16) {
            const int c = a.col[j];
            if ((uint32_t)c < a.ncols) sum = __builtin_fmaf(a.val[j], a.x[c], sum);
        }
    }
    for (int off = 8; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 16);
    if (row < a.nrows && l == 0) a.y[row] = sum;
}

// --------------------------------------------------------------- stencil
// 1024 x 32 cells per workgroup.  Each wave covers 256 consecutive cells of
// a row (four per lane, one 16-byte access) and walks the 32 rows, keeping
// the rows above and below in registers; the west / east neighbours of a
// lane's four cells come from the adjacent lanes by shuffles, and from
// memory at the two ends of the wave.  Original grid: (ceil(nx/1024),
// ceil(ny/32), 1).
__device__ __forceinline__ float st_cell(float c0, float c1, float mid, float n, float s,
                                         float w, float e) {
    return __builtin_fmaf(c1, (n + s) + (w + e), c0 * mid);
}

// A workgroup owns 1024 x 32 cells: its four waves sit side by side, each
// 256 columns wide (four per lane), and roll down the 32 rows, so a row's
// west / east halo lines are fetched once per 1024 columns and its north /
// south halo rows once per 32 rows.
__global__ __launch_bounds__(KL_WG) void kl_stencil(kl_stencil_args a, kl_slice s) {
    const uint3 wg = kl_wg_id3(s);
    const uint32_t bx = wg.x, by = wg.y;
    const int lane = threadIdx.x & 63;
    const uint32_t nx = a.nx, ny = a.ny;
    const uint32_t x0 = bx * 1024 + (threadIdx.x >> 6) * 256 + lane * 4;
    const uint32_t y0 = by * 32;
    if (y0 >= ny) return;                   // uniform over the workgroup
    const bool act = x0 < nx;               // nx % 4 == 0: all four cells or none
    const uint32_t xc = act ? x0 : nx - 4;  // in-range column for idle lanes' loads
    const float* __restrict__ in = a.in;
    float* __restrict__ out = a.out;
    const float c0 = a.c0, c1 = a.c1;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 up = zero;
    if (y0 > 0) up = *(const float4*)(in + (size_t)(y0 - 1) * nx + xc);
    float4 mid = *(const float4*)(in + (size_t)y0 * nx + xc);
    for (int r = 0; r < 32; ++r) {
        const uint32_t y = y0 + r;
        if (y >= ny) break;                 // uniform over the wave
        const size_t row = (size_t)y * nx;
        float4 down = zero;
        if (y + 1 < ny) down = *(const float4*)(in + row + nx + xc);
        float w = __shfl_up(mid.w, 1);
        float e = __shfl_down(mid.x, 1);
        if (lane == 0) w = (act && x0 > 0) ? in[row + x0 - 1] : 0.0f;
        if (lane == 63) e = (act && x0 + 4 < nx) ? in[row + x0 + 4] : 0.0f;
        if (act) {
            float4 v = mid;
            if (y != 0 && y != ny - 1) {
                if (x0 != 0) v.x = st_cell(c0, c1, mid.x, up.x, down.x, w, mid.y);
                v.y = st_cell(c0, c1, mid.y, up.y, down.y, mid.x, mid.z);
                v.z = st_cell(c0, c1, mid.z, up.z, down.z, mid.y, mid.w);
                if (x0 + 3 != nx - 1) v.w = st_cell(c0, c1, mid.w, up.w, down.w, mid.z, e);
            }
            *(float4*)(out + row + x0) = v;
        }
        up = mid;
        mid = down;
    }
}

// -------------------------------------------------------- black-scholes
__device__ __forceinline__ void bs_one(float S, float K, float T, float r, float sig,
                                       float* call, float* put) {
    const float rs2 = 0.70710678118654752f;
    const float sq = sig * sqrtf(T);
    const float d1 = (logf(S / K) + (r + 0.5f * sig * sig) * T) / sq;
    const float d2 = d1 - sq;
    const float disc = K * expf(-r * T);
    *call = S * (0.5f * erfcf(-d1 * rs2)) - disc * (0.5f * erfcf(-d2 * rs2));
    *put = disc * (0.5f * erfcf(d2 * rs2)) - S * (0.5f * erfcf(d1 * rs2));
}

__global__ __launch_bounds__(KL_WG) void kl_bs(kl_bs_args a, kl_slice s) {
    const uint64_t i = ((uint64_t)kl_wg_linear(s) * KL_WG + threadIdx.x) * 4;
    if (i >= a.n) return;
    const float4 S = *(const float4*)(a.s + i);
    const float4 K = *(const float4*)(a.k + i);
    const float4 T = *(const float4*)(a.t + i);
    float4 c, p;
    bs_one(S.x, K.x, T.x, a.r, a.sigma, &c.x, &p.x);
    bs_one(S.y, K.y, T.y, a.r, a.sigma, &c.y, &p.y);
    bs_one(S.z, K.z, T.z, a.r, a.sigma, &c.z, &p.z);
    bs_one(S.w, K.w, T.w, a.r, a.sigma, &c.w, &p.w);
    *(float4*)(a.call + i) = c;
    *(float4*)(a.put + i) = p;
}

// ------------------------------------------------------------- histogram
// Each workgroup counts a 64 KiB chunk into one LDS copy of the bins per
// wave, then adds its non-zero totals to the global bins.
__global__ __launch_bounds__(KL_WG) void kl_hist(kl_hist_args a, kl_slice s) {
    __shared__ uint32_t h[4][256];
    const int tid = threadIdx.x, w = tid / 64;
    for (int i = tid; i < 4 * 256; i += KL_WG) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)kl_wg_linear(s) * 65536;
    for (int it = 0; it < 16; ++it) {
        const uint64_t off = base + ((uint64_t)it * KL_WG + tid) * 16;
        if (off + 16 <= a.n) {
            const uint4 v = *(const uint4*)(a.data + off);
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b) atomicAdd(&h[w][(wd[q] >> (8 * b)) & 255u], 1u);
        } else {
            for (uint64_t o = off; o < a.n && o < off + 16; ++o) atomicAdd(&h[w][a.data[o]], 1u);
        }
    }
    __syncthreads();
    const uint32_t c = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
    if (c) atomicAdd(&a.bins[tid], c);
}

// ---------------------------------------------------------------- lookup
// lower_bound through a static 32-ary tree of 128-byte nodes over
// compressed leaves.  A leaf is 64 consecutive keys kept as 16-bit
// distances below the leaf's largest key, one 128-byte line (the L2 line)
// per leaf, so the searched structure takes 2 bytes per key: for 2^26 keys
// 128 MiB of leaves and a 4 MiB level 1, which the 256 MiB last-level cache
// can hold while the 256 MiB key array is not read.  A leaf whose keys span
// more than 65534 is flagged (the first distance of each 16-byte piece is
// 0xffff, so every lane reading a piece sees the flag) and searched in
// the key array instead.  Level 1 holds the largest key of every leaf, level
// k + 1 the largest entry of every 32-entry node of level k, up to a top
// level of at most 1024 entries that each workgroup keeps in LDS.  Levels
// and leaves start on 128-byte boundaries; the tail of each level's last
// node is padded with 0xffffffff, a leaf's slots past the last key hold 0.
//
// Eight lanes search one query together: each reads 16 bytes of the same
// 128-byte node or leaf and the eight partial counts are summed across the
// lanes, so a wave's load touches 8 lines, not 64 (the per-CU address
// path, about one line per clock, bounds a search whose every lane reads
// its own line).
constexpr uint32_t kLkLeaf = 64;       // keys per leaf
constexpr uint32_t kLkLeafWords = 32;  // uint32 words per leaf (two distances each)
constexpr uint32_t kLkFan = 32;        // entries per node
constexpr uint32_t kLkEscape = 0xffffu;
// lanes that search one query together: each reads 128 / kLkGroup bytes of
// every node and leaf line
constexpr int kLkGroup = 8;

struct LkLevels {
    uint32_t nlev;
    uint64_t off[8];  // first entry of each level (level 1 first)
    uint64_t m[8];    // entries of each level
    uint64_t leaf_off;  // first word of the leaves
    uint64_t nleaf;
    uint64_t total;   // words including padding and leaves
};

// Fully unrolled so that every array index is a constant: the level
// tables stay in registers (n < 2^31 needs at most 4 levels).
__host__ __device__ inline void lk_levels(uint32_t n, LkLevels* L) {
    const uint64_t nleaf = ((uint64_t)n + kLkLeaf - 1) / kLkLeaf;
    uint64_t m = nleaf, off = 0;
    bool done = false;
    L->nlev = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        L->m[k] = done ? 0 : m;
        L->off[k] = off;
        if (!done) {
            L->nlev = k + 1;
            off += (m + kLkFan - 1) / kLkFan * kLkFan;
            if (m <= 1024)
                done = true;
            else
                m = (m + kLkFan - 1) / kLkFan;
        }
    }
    L->leaf_off = off;
    L->nleaf = nleaf;
    L->total = off + nleaf * kLkLeafWords;
}

// One thread per four words of the index (16 bytes): four level entries, or
// eight leaf distances.
__global__ __launch_bounds__(KL_WG) void kl_lookup_index(kl_lookup_args a, kl_slice s) {
    LkLevels L;
    lk_levels(a.nkeys, &L);
    const uint64_t e = ((uint64_t)kl_wg_linear(s) * KL_WG + threadIdx.x) * 4;
    if (e >= L.total) return;
    const uint32_t n = a.nkeys;
    uint4 v;
    if (e >= L.leaf_off) {
        const uint64_t w = e - L.leaf_off;
        const uint64_t j = w / kLkLeafWords;
        const uint64_t k0 = j * kLkLeaf + 2 * (w % kLkLeafWords);  // 8 keys from k0
        const uint64_t last = j * kLkLeaf + kLkLeaf - 1 < n ? j * kLkLeaf + kLkLeaf - 1 : n - 1;
        const uint32_t mx = a.keys[last];
        if (mx - a.keys[j * kLkLeaf] > kLkEscape - 1) {
            // searched in the keys: the flag in the first slot of every
            // 16-byte piece, so each lane of a group sees it in its own piece
            v = make_uint4(kLkEscape, 0u, 0u, 0u);
        } else {
            uint32_t d[8];
            if (k0 + 8 <= n) {
                const uint4* kp = (const uint4*)(a.keys + k0);  // 32-byte aligned
                const uint4 x = kp[0], y = kp[1];
                d[0] = mx - x.x; d[1] = mx - x.y; d[2] = mx - x.z; d[3] = mx - x.w;
                d[4] = mx - y.x; d[5] = mx - y.y; d[6] = mx - y.z; d[7] = mx - y.w;
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) d[i] = k0 + i < n ? mx - a.keys[k0 + i] : 0u;
            }
            v = make_uint4(d[0] | (d[1] << 16), d[2] | (d[3] << 16), d[4] | (d[5] << 16),
                           d[6] | (d[7] << 16));
        }
    } else {
        // the level holding entries e .. e + 3 (levels are padded to 32)
        uint32_t k = 0;
        uint64_t base = L.off[0], mk = L.m[0];
#pragma unroll
        for (int jl = 1; jl < 8; ++jl)
            if (jl < (int)L.nlev && e >= L.off[jl]) {
                k = jl;
                base = L.off[jl];
                mk = L.m[jl];
            }
        // entry i of level k + 1 covers keys [64 32^k i, 64 32^k (i + 1))
        const uint64_t span = (uint64_t)kLkLeaf << (5 * k);
        uint32_t x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint64_t i = e + t - base;
            uint64_t last = (i + 1) * span;
            if (last > n) last = n;
            x[t] = i < mk ? a.keys[last - 1] : 0xffffffffu;
        }
        v = make_uint4(x[0], x[1], x[2], x[3]);
    }
    *(uint4*)(a.index + e) = v;
}

// The queries and results stream through once: nontemporal accesses keep
// them from displacing the tree and the leaves in the caches.
typedef uint32_t kl_u32x4 __attribute__((ext_vector_type(4)));

// Sum over the G lanes of a group (lanes G g .. G g + G - 1 of the wave, G
// = 4 or 8) by data-parallel-primitive moves: swap neighbours (quad_perm
// 1,0,3,2), swap pairs (quad_perm 2,3,0,1), and for eight lanes add the
// other quad (row_half_mirror: lane i of a half row reads lane 7 - i).
template <int G>
__device__ __forceinline__ uint32_t lk_sum(uint32_t v) {
    static_assert(G == 4 || G == 8, "groups of four or eight lanes");
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
    if (G == 8) x += __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);
    return (uint32_t)x;
}

// The LDS copy of the top level: its entries (at most 1024, sorted), then
// all-ones up to kLkTopPad, which no query is above.  A search that finds
// all 1024 entries below q goes on reading past them, at most 16 entries.
constexpr uint32_t kLkTopPad = 1024 + 16;

// Entries of the LDS top level that are < q, found by the G lanes of a
// group together: while the range left is longer than 16 entries it is cut
// into G blocks and lane r tests the last entry of block r; then each lane
// tests 16 / G entries of the last 16.  The padding makes every read valid,
// so the rounds need no bounds tests (and no branches).
template <int G>
__device__ __forceinline__ uint32_t lk_top_count(const uint32_t* top, uint32_t q, uint32_t r) {
    uint32_t base = 0;
#pragma unroll
    for (uint32_t R = 1024; R > 16; R /= G) {
        const uint32_t B = R / G;
        base += B * lk_sum<G>(top[base + B * r + B - 1] < q);
    }
    uint32_t c = 0;
#pragma unroll
    for (uint32_t u = 0; u < 16 / G; ++u) c += top[base + (16 / G) * r + u] < q;
    return base + lk_sum<G>(c);
}

// Leaf distances of a uint32 word (two slots) above tc (tc <= 0xffff),
// compared as two 16-bit lanes.
typedef uint16_t kl_u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t lk_above2(uint32_t w, kl_u16x2 tc) {
    const kl_u16x2 d = __builtin_bit_cast(kl_u16x2, w);
    typedef short kl_s16x2 __attribute__((ext_vector_type(2)));
    const kl_s16x2 gt = d > tc;  // lanes -1 where true, 0 where false
    return (uint32_t)(gt.x & 1) + (uint32_t)(gt.y & 1);
}

// Reads of the index by raw buffer loads with 32-bit byte offsets (fewer
// address instructions than 64-bit flat addresses): one buffer resource for
// the levels and one for the leaves, each under 4 GiB (nkeys <= 2^31 - 64:
// fewer than 2^25 leaves of 128 bytes).
struct LkIndex {
    __amdgpu_buffer_rsrc_t lv, lf;
    __device__ LkIndex(const uint32_t* idx, const LkLevels& L) {
        // word 3 of a raw buffer resource on gfx9 (32-bit data format)
        lv = __builtin_amdgcn_make_buffer_rsrc((void*)idx, 0, (int)(L.leaf_off * 4), 0x00020000);
        const uint64_t lb = L.nleaf * kLkLeafWords * 4;
        lf = __builtin_amdgcn_make_buffer_rsrc((void*)(idx + L.leaf_off), 0,
                                               (int)(uint32_t)(lb < 0xffffffffull ? lb : 0xffffffffull),
                                               0x00020000);
    }
    // 16 bytes at word w of the levels, or of the leaves
    __device__ __forceinline__ uint4 level4(uint32_t w) const {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(lv, (int)(4u * w), 0, 0);
        return make_uint4(t[0], t[1], t[2], t[3]);
    }
    __device__ __forceinline__ uint4 leaf4(uint32_t w) const {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(lf, (int)(4u * w), 0, 0);
        return make_uint4(t[0], t[1], t[2], t[3]);
    }
};

template <int G>
__device__ __forceinline__ void lookup_body(const kl_lookup_args& a, const kl_slice& s) {
    constexpr int W4 = 8 / G;  // 16-byte pieces of a 128-byte line per lane
    __shared__ uint32_t top[kLkTopPad];
    LkLevels L;
    lk_levels(a.nkeys, &L);
    const uint32_t T = L.nlev - 1;
    uint32_t mt = 0;
    uint64_t top_off = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j == (int)T) {
            mt = (uint32_t)L.m[j];
            top_off = L.off[j];
        }
    for (uint32_t i = threadIdx.x; i < kLkTopPad; i += KL_WG)
        top[i] = i < mt ? a.index[top_off + i] : 0xffffffffu;
    __syncthreads();
    // every lane loads its own four queries; lanes past the end search dummy
    // queries (the lanes of a group work together) and store nothing
    const uint64_t t0 = ((uint64_t)kl_wg_linear(s) * KL_WG + threadIdx.x) * 4;
    const bool valid = t0 < a.nq;
    kl_u32x4 qv = {0u, 0u, 0u, 0u};
    if (valid) qv = __builtin_nontemporal_load((const kl_u32x4*)(a.q + t0));
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g0 = lane & ~(uint32_t)(G - 1);  // first lane of this lane's group
    const uint32_t r = lane & (uint32_t)(G - 1);    // this lane's part of a line
    const uint32_t n = a.nkeys;
    const LkIndex idx(a.index, L);
    kl_u32x4 o = {n, n, n, n};
    // the group searches the four queries of each of its lanes in turn
    for (uint32_t b = 0; b < (uint32_t)G; ++b) {
        const int src = (int)(g0 + b);
        uint32_t q[4], c[4];
        bool past[4];
        uint32_t mx[4];  // the largest key of each query's leaf
        q[0] = (uint32_t)__shfl((int)qv.x, src);
        q[1] = (uint32_t)__shfl((int)qv.y, src);
        q[2] = (uint32_t)__shfl((int)qv.z, src);
        q[3] = (uint32_t)__shfl((int)qv.w, src);
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = lk_top_count<G>(top, q[i], r);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            past[i] = c[i] >= mt;  // above every key
            if (past[i]) c[i] = 0;  // searched as query 0, answer n
        }
#pragma unroll
        for (int k = 6; k >= 0; --k) {
            if (k >= (int)T) continue;  // uniform: levels below the top only
            uint4 x[4][W4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int v = 0; v < W4; ++v)
                    x[i][v] = idx.level4((uint32_t)L.off[k] + kLkFan * c[i] + 4 * (W4 * r + v));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t cnt = 0;
#pragma unroll
                for (int v = 0; v < W4; ++v)
                    cnt += (x[i][v].x < q[i]) + (x[i][v].y < q[i]) + (x[i][v].z < q[i]) +
                           (x[i][v].w < q[i]);
                const uint32_t e = lk_sum<G>(cnt);
                c[i] = kLkFan * c[i] + e;
                if (k == 0) {
                    // level 1: entry e of the node just read is the leaf's
                    // largest key (e < 32 unless past[i]), held in piece
                    // e / 4 of the line: lane e / (4 W4) of the group
                    const uint32_t j = e & (4 * W4 - 1);
                    uint32_t v = 0;
#pragma unroll
                    for (int u = 0; u < W4; ++u) {
                        v = j == 4u * u ? x[i][u].x : v;
                        v = j == 4u * u + 1 ? x[i][u].y : v;
                        v = j == 4u * u + 2 ? x[i][u].z : v;
                        v = j == 4u * u + 3 ? x[i][u].w : v;
                    }
                    mx[i] = (uint32_t)__shfl((int)v, (int)(g0 + e / (4 * W4)));
                }
            }
        }
        // c[i]: the leaf holding the answer, the first whose largest key
        // is >= q[i]
        uint4 w[4][W4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int v = 0; v < W4; ++v)
                w[i][v] = idx.leaf4(kLkLeafWords * c[i] + 4 * (W4 * r + v));
            if (T == 0) mx[i] = top[c[i]];  // level 1 is the top (c[i] < mt)
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // a leaf searched in the keys is flagged in every lane's piece
            const bool esc = (w[i][0].x & 0xffffu) == kLkEscape;
            uint32_t cnt = 0;
            if (!esc) {
                // key < q exactly when its distance below the leaf's largest
                // key exceeds mx - q (q <= mx here; distances are < 0xffff)
                const uint32_t t = mx[i] - q[i];
                const uint16_t t16 = (uint16_t)(t < 0xffffu ? t : 0xffffu);
                const kl_u16x2 tc = {t16, t16};
#pragma unroll
                for (int v = 0; v < W4; ++v)
                    cnt += lk_above2(w[i][v].x, tc) + lk_above2(w[i][v].y, tc) +
                           lk_above2(w[i][v].z, tc) + lk_above2(w[i][v].w, tc);
            } else {
                const uint64_t k0 = (uint64_t)c[i] * kLkLeaf + (kLkLeaf / G) * r;
#pragma unroll
                for (int u = 0; u < (int)(kLkLeaf / G); ++u)
                    cnt += k0 + u < n && a.keys[k0 + u] < q[i];
            }
            cnt = lk_sum<G>(cnt);  // the whole group takes the same branch
            const uint32_t res = past[i] ? n : c[i] * kLkLeaf + cnt;
            if (lane == (uint32_t)src) o[i] = res;
        }
    }
    if (valid) __builtin_nontemporal_store(o, (kl_u32x4*)(a.out + t0));
}

__global__ __launch_bounds__(KL_WG) void kl_lookup(kl_lookup_args a, kl_slice s) {
    lookup_body<kLkGroup>(a, s);
}


// ------------------------------------------------------ synthetic kernels
// One load and a chain of dependent fmas per iteration; NACC values made
// opaque to the compiler stay live across the loop (register pressure
// class) and LDSB bytes of static LDS are touched (LDS class).
template <int NACC, int LDSB>
__device__ __forceinline__ void synthk_body(const kl_synthk_args& a, const kl_slice& s) {
    constexpr int NL = LDSB > 0 ? LDSB / 4 : 1;
    static_assert(LDSB == 0 || NL >= KL_WG, "an LDS class holds a value per thread");
    __shared__ float lds[NL];
    const uint32_t t = kl_wg_linear(s) * KL_WG + threadIdx.x;
    const bool active = t < a.n_threads;
    float keep[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        keep[k] = (float)(t ^ (uint32_t)(k * 2654435761u)) * 1e-9f;
        asm volatile("" : "+v"(keep[k]));
    }
    float x = (float)(t & 1023u) * 1e-3f;
    uint32_t h = t * 2654435761u + 12345u;
    if (active) {
        for (uint32_t it = 0; it < a.iters; ++it) {
            uint32_t addr;
            if (a.pattern == 0) {
                addr = (t + it * a.n_threads) & a.mask;
            } else if (a.pattern == 1) {
                addr = (32u * t + 7919u * it) & a.mask;
            } else {
                h = h * 1664525u + 1013904223u;
                addr = (h ^ (h >> 13)) & a.mask;
            }
            const float v = a.src[addr];
            for (uint32_t j = 0; j < a.alu; ++j) x = __builtin_fmaf(x, v, 0.5f);
        }
    }
    if (LDSB > 0) {   // every value read here was written by this workgroup
        lds[threadIdx.x] = x;
        __syncthreads();
        x += lds[(threadIdx.x + 1) % KL_WG];
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        asm volatile("" : "+v"(keep[k]));
        x += keep[k];
    }
    if (active) a.dst[t] = x;
}

#define KL_SYNTHK_CLASSES(X) \
    X(32, 0) X(32, 16) X(32, 32) X(32, 64) \
    X(64, 0) X(64, 16) X(64, 32) X(64, 64) \
    X(128, 0) X(128, 16) X(128, 32) X(128, 64) \
    X(256, 0) X(256, 16) X(256, 32) X(256, 64)

// live values per VGPR class: the class less what the loop itself needs
template <int V>
constexpr int synthk_nacc() { return V == 32 ? 16 : V == 64 ? 48 : V == 128 ? 112 : 236; }

// one kernel per class (where LDS already limits occupancy the compiler
// may reserve more VGPRs than the loop keeps live)
#define KL_SYNTHK_DEF(V, L)                                                              \
    __global__ __launch_bounds__(KL_WG) void kl_synthk_v##V##_l##L(kl_synthk_args a,     \
                                                                   kl_slice s) {         \
        synthk_body<synthk_nacc<V>(), (L) * 1024>(a, s);                                 \
    }
KL_SYNTHK_CLASSES(KL_SYNTHK_DEF)
#undef KL_SYNTHK_DEF

// ----------------------------------------------------------------- probe
// Records where and when each workgroup ran and counts its visits; used to
// check that a slicing plan runs every workgroup exactly once and to see
// how the dispatcher places co-running slices on CUs.  `spin` dependent
// fmas per thread stand for work.
__global__ __launch_bounds__(KL_WG) void kl_probe(kl_probe_args a, kl_slice s) {
    const uint32_t lin = kl_wg_linear(s);
    if (lin >= a.n_wg) return;
    const uint64_t t0 = wall_clock64();
    float v = (float)threadIdx.x;
    for (uint32_t i = 0; i < a.spin; ++i) v = __builtin_fmaf(v, 0.999f, 1.0f);
    asm volatile("" ::"v"(v));
    __syncthreads();
    if (threadIdx.x == 0) {
        // HW_ID (hardware register 4): CU_ID 11:8, SH_ID 12, SE_ID 14:13;
        // XCC_ID (hardware register 20) bits 3:0
        const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
        const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
        const uint64_t t1 = wall_clock64();
        atomicAdd(&a.visits[lin], 1u);
        a.info[3 * (uint64_t)lin] = ((uint64_t)xcc << 32) | hw;
        a.info[3 * (uint64_t)lin + 1] = t0;
        a.info[3 * (uint64_t)lin + 2] = t1;
    }
}

// ------------------------------------------------------------- ceilings
// FP32 compute ceilings of the chip, for the roofs kernels are measured
// against: 16 independent FMA chains per thread (unpacked VALU), and four
// independent MFMA accumulators per wave (the SGEMM's instruction).
__global__ __launch_bounds__(KL_WG) void kl_ceil_fma(kl_ceiling_args a, kl_slice s) {
    const uint32_t lin = kl_wg_linear(s);
    if (lin >= a.n_wg) return;
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (float)k;
    for (uint32_t i = 0; i < a.iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = __builtin_fmaf(v[k], a.mul, a.add);
    }
    float sum = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += v[k];
    a.out[(uint64_t)lin * KL_WG + threadIdx.x] = sum;
}

__global__ __launch_bounds__(KL_WG) void kl_ceil_mfma(kl_ceiling_args a, kl_slice s) {
    const uint32_t lin = kl_wg_linear(s);
    if (lin >= a.n_wg) return;
    kl_f32x16 acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = kl_f32x16{};
    const float av = a.mul, bv = a.add;
    for (uint32_t i = 0; i < a.iters; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[k], 0, 0, 0);
    }
    float sum = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < 16; ++e) sum += acc[k][e];
    a.out[(uint64_t)lin * KL_WG + threadIdx.x] = sum;
}

// HBM read ceiling: every thread streams per_thread float4, eight loads in
// flight, into four independent sums.
__global__ __launch_bounds__(KL_WG) void kl_ceil_read(kl_read_args a, kl_slice s) {
    const uint32_t lin = kl_wg_linear(s);
    if (lin >= a.n_wg) return;
    const float4* p = (const float4*)a.src + (uint64_t)lin * KL_WG * a.per_thread + threadIdx.x;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t i = 0; i < a.per_thread; i += 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(uint64_t)(i + u) * KL_WG];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    a.out[(uint64_t)lin * KL_WG + threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
}

// ===================================================== host-side registry
namespace {

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Validates an argument block and returns its original grid; "" on success.
std::string grid_of(const char* name, const void* args, uint32_t bytes, kl_dim3* g) {
    std::string n(name);
    *g = {1, 1, 1};
#define KL_ARGS(T)                                                     \
    if (bytes != sizeof(T)) return "argument block size mismatch";    \
    T a;                                                               \
    std::memcpy(&a, args, sizeof(T));
    if (n == "poly") {
        KL_ARGS(kl_poly_args);
        if (!a.x || !a.coef || !a.y || a.n == 0) return "null pointer or n == 0";
        if (a.ncoef < 1 || a.ncoef > 1024) return "ncoef outside [1, 1024]";
        g->x = cdiv(a.n, KL_WG);
    } else if (n == "gather") {
        KL_ARGS(kl_gather_args);
        if (!a.idx || !a.table || !a.out || a.n == 0 || a.table_n == 0)
            return "null pointer or empty input";
        g->x = cdiv(a.n, KL_WG);
    } else if (n == "sgemm") {
        KL_ARGS(kl_sgemm_args);
        if (!a.a || !a.b || !a.c) return "null pointer";
        if (a.m == 0 || a.n == 0 || a.k == 0 || a.m % 128 || a.n % 128 || a.k % 16)
            return "sgemm needs m, n multiples of 128 and k a multiple of 16";
        if (!aligned16(a.a) || !aligned16(a.b)) return "a, b must be 16-byte aligned";
        uint64_t tiles = (uint64_t)(a.m / 128) * (a.n / 128);
        if (tiles > 0xffffffffull) return "too many tiles";
        g->x = (uint32_t)tiles;
    } else if (n == "spmv") {
        KL_ARGS(kl_spmv_args);
        if (!a.row_ptr || !a.col || !a.val || !a.x || !a.y || a.nrows == 0)
            return "null pointer or nrows == 0";
        if (a.nrows > 0xffffffffu - 16) return "nrows too large";
        g->x = cdiv(a.nrows, 16);
    } else if (n == "stencil") {
        KL_ARGS(kl_stencil_args);
        if (!a.in || !a.out || a.nx == 0 || a.ny == 0) return "null pointer or empty grid";
        if (a.in == a.out) return "stencil in and out must differ";
        if (a.nx % 4) return "stencil nx must be a multiple of 4";
        if (!aligned16(a.in) || !aligned16(a.out)) return "stencil in, out must be 16-byte aligned";
        g->x = cdiv(a.nx, 1024);
        g->y = cdiv(a.ny, 32);
    } else if (n == "bs") {
        KL_ARGS(kl_bs_args);
        if (!a.s || !a.k || !a.t || !a.call || !a.put || a.n == 0 || a.n % 4)
            return "null pointer, or n not a positive multiple of 4";
        if (!aligned16(a.s) || !aligned16(a.k) || !aligned16(a.t) || !aligned16(a.call) ||
            !aligned16(a.put))
            return "bs arrays must be 16-byte aligned";
        g->x = cdiv(a.n, 4 * KL_WG);
    } else if (n == "hist") {
        KL_ARGS(kl_hist_args);
        if (!a.data || !a.bins || a.n == 0 || a.n % 16) return "null pointer or n % 16 != 0";
        if (!aligned16(a.data)) return "hist data must be 16-byte aligned";
        uint64_t wg = (a.n + 65535) / 65536;
        if (wg > 0xffffffffull) return "input too large";
        g->x = (uint32_t)wg;
    } else if (n.rfind("synthk_", 0) == 0) {
        KL_ARGS(kl_synthk_args);
        if (!a.src || !a.dst || a.n_threads == 0) return "null pointer or n_threads == 0";
        if ((a.mask & (a.mask + 1)) != 0) return "mask + 1 must be a power of two";
        if (a.pattern > 2 || a.alu > 4096 || a.iters > (1u << 20))
            return "pattern > 2, alu > 4096 or iters > 2^20";
        g->x = cdiv(a.n_threads, KL_WG);
    } else if (n == "probe") {
        KL_ARGS(kl_probe_args);
        if (!a.visits || !a.info || a.n_wg == 0) return "null pointer or n_wg == 0";
        if (a.spin > (1u << 24)) return "spin above 2^24";
        g->x = a.n_wg;
    } else if (n == "ceil_fma" || n == "ceil_mfma") {
        KL_ARGS(kl_ceiling_args);
        if (!a.out || a.n_wg == 0) return "null out or n_wg == 0";
        if (a.iters > (1u << 20)) return "iters above 2^20";
        g->x = a.n_wg;
    } else if (n == "ceil_read") {
        KL_ARGS(kl_read_args);
        if (!a.src || !a.out || a.n_wg == 0) return "null src or out, or n_wg == 0";
        if (!aligned16(a.src)) return "src must be 16-byte aligned";
        if (a.per_thread == 0 || a.per_thread % 8 || a.per_thread > (1u << 16))
            return "per_thread not a positive multiple of 8 up to 2^16";
        g->x = a.n_wg;
    } else if (n == "lookup" || n == "lookup_index") {
        KL_ARGS(kl_lookup_args);
        if (!a.keys || !a.index || a.nkeys == 0 || a.nkeys > 0x7fffffc0u)
            return "null keys or index, or nkeys outside [1, 2^31 - 64]";
        if (!aligned16(a.keys) || !aligned16(a.index)) return "keys, index must be 16-byte aligned";
        if (n == "lookup_index") {
            LkLevels L;
            lk_levels(a.nkeys, &L);
            g->x = cdiv(L.total / 4, KL_WG);
        } else {
            if (!a.q || !a.out || a.nq == 0 || a.nq % 4)
                return "null q or out, or nq not a positive multiple of 4";
            if (!aligned16(a.q) || !aligned16(a.out)) return "q, out must be 16-byte aligned";
            g->x = cdiv(a.nq, 4 * KL_WG);
        }
    } else {
        return "unknown built-in kernel";
    }
#undef KL_ARGS
    return "";
}

struct BuiltinEntry {
    const char* name;
    const void* fn;
    uint32_t args_bytes;
    uint32_t flags;
};

const BuiltinEntry kBuiltins[] = {
    {"poly", (const void*)kl_poly, sizeof(kl_poly_args), KL_KF_IDEMPOTENT},
    {"gather", (const void*)kl_gather, sizeof(kl_gather_args), KL_KF_IDEMPOTENT},
    {"sgemm", (const void*)kl_sgemm, sizeof(kl_sgemm_args), KL_KF_IDEMPOTENT},
    {"spmv", (const void*)kl_spmv, sizeof(kl_spmv_args), KL_KF_IDEMPOTENT},
    {"stencil", (const void*)kl_stencil, sizeof(kl_stencil_args), KL_KF_IDEMPOTENT},
    {"bs", (const void*)kl_bs, sizeof(kl_bs_args), KL_KF_IDEMPOTENT},
    {"hist", (const void*)kl_hist, sizeof(kl_hist_args), 0u},
    {"lookup", (const void*)kl_lookup, sizeof(kl_lookup_args), KL_KF_IDEMPOTENT},
    {"lookup_index", (const void*)kl_lookup_index, sizeof(kl_lookup_args), KL_KF_IDEMPOTENT},
    {"probe", (const void*)kl_probe, sizeof(kl_probe_args), 0u},
    {"ceil_fma", (const void*)kl_ceil_fma, sizeof(kl_ceiling_args), KL_KF_IDEMPOTENT},
    {"ceil_mfma", (const void*)kl_ceil_mfma, sizeof(kl_ceiling_args), KL_KF_IDEMPOTENT},
    {"ceil_read", (const void*)kl_ceil_read, sizeof(kl_read_args), KL_KF_IDEMPOTENT},
#define KL_SYNTHK_ENTRY(V, L)                                                 \
    {"synthk_v" #V "_l" #L, (const void*)kl_synthk_v##V##_l##L, sizeof(kl_synthk_args), \
     KL_KF_IDEMPOTENT},
    KL_SYNTHK_CLASSES(KL_SYNTHK_ENTRY)
#undef KL_SYNTHK_ENTRY
};

}  // namespace

extern "C" uint64_t kernelet_lookup_index_entries(uint32_t nkeys) {
    if (nkeys == 0) return 0;
    LkLevels L;
    lk_levels(nkeys, &L);
    return L.total;
}

namespace kl {
void set_error(const std::string& msg);

bool builtin_check(const char* name, const void* args, uint32_t bytes, kl_dim3* grid,
                   std::string* err) {
    *err = grid_of(name, args, bytes, grid);
    return err->empty();
}

bool is_builtin_fn(const void* fn, const char** name) {
    for (const auto& b : kBuiltins)
        if (b.fn == fn) {
            *name = b.name;
            return true;
        }
    return false;
}
}  // namespace kl

extern "C" kl_status kernelet_builtin(const char* name, kl_kernel_desc* out) {
    if (!name || !out) {
        kl::set_error("kernelet_builtin: null argument");
        return KL_EINVAL;
    }
    for (const auto& b : kBuiltins) {
        if (std::strcmp(b.name, name) == 0) {
            out->name = b.name;
            out->host_fn = b.fn;
            out->block_threads = KL_WG;
            out->args_bytes = b.args_bytes;
            out->flags = b.flags;
            out->profile = nullptr;
            return KL_OK;
        }
    }
    kl::set_error(std::string("kernelet_builtin: unknown kernel ") + name);
    return KL_ENOTFOUND;
}

extern "C" kl_status kernelet_builtin_grid(const char* name, const void* args,
                                           uint32_t args_bytes, kl_dim3* grid) {
    if (!name || !args || !grid) {
        kl::set_error("kernelet_builtin_grid: null argument");
        return KL_EINVAL;
    }
    std::string err = grid_of(name, args, args_bytes, grid);
    if (!err.empty()) {
        kl::set_error(std::string("kernelet_builtin_grid(") + name + "): " + err);
        return err == "unknown built-in kernel" ? KL_ENOTFOUND : KL_EINVAL;
    }
    return KL_OK;
}
