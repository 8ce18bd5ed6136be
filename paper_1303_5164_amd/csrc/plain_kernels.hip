// Kernels written without any knowledge of slicing: they read blockIdx and
// gridDim as usual and take one argument block.  irslice.py makes them
// sliceable by rewriting their device IR (the analogue of the paper's
// rewriting of compiled kernels, Section 4.1); the library never links
// this file.
#include <hip/hip_runtime.h>
#include <stdint.h>

// The paper's slicing example (Section 4.1): C = A + B on an n x n matrix,
// one 16 x 16 block of elements per workgroup, a 2-D grid of
// ceil(n/16) x ceil(n/16) workgroups.
struct kl_matadd_args {
    const float* a;
    const float* b;
    float* c;
    uint32_t n;
};

extern "C" __global__ void __launch_bounds__(256) kl_plain_matadd(kl_matadd_args p) {
    const uint32_t x = blockIdx.x * 16 + threadIdx.x % 16;
    const uint32_t y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x < p.n && y < p.n) {
        const size_t i = (size_t)y * p.n + x;
        p.c[i] = p.a[i] + p.b[i];
    }
}

// Every workgroup of a 3-D grid counts itself at its row-major index and
// the first one records gridDim: a sliced run must count each index once
// and see the original grid.  An index at or past n (visits holds n
// counters) is counted in dims[3] instead.
struct kl_visit3d_args {
    uint32_t* visits;
    uint32_t* dims;
    uint32_t n;
};

extern "C" __global__ void __launch_bounds__(256) kl_plain_visit3d(kl_visit3d_args p) {
    if (threadIdx.x == 0) {
        const uint32_t id = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        if (id < p.n)
            atomicAdd(&p.visits[id], 1u);
        else
            atomicAdd(&p.dims[3], 1u);
        if (id == 0) {
            p.dims[0] = gridDim.x;
            p.dims[1] = gridDim.y;
            p.dims[2] = gridDim.z;
        }
    }
}
