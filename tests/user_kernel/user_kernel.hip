// A kernel a user of the library writes against the public headers alone
// (include/kernelet.h, include/kernelet_device.h): a tiled matrix
// transpose over a 2-D grid of 16 x 16 tiles, 1-D workgroups of 256
// work-items.  Built into its own shared library; the test passes its
// host stub to kernelet_register.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernelet_device.h"

struct user_transpose_args {
    const float* in;  // rows x cols, row-major
    float* out;       // cols x rows, row-major
    uint32_t rows, cols;
};

__global__ __launch_bounds__(256) void user_transpose(user_transpose_args a, kl_slice s) {
    __shared__ float tile[16][17];
    const uint3 wg = kl_wg_id3(s);  // (column tile, row tile, 0) of the original grid
    const uint32_t tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const uint32_t r = wg.y * 16 + ty, c = wg.x * 16 + tx;
    if (r < a.rows && c < a.cols) tile[ty][tx] = a.in[(size_t)r * a.cols + c];
    __syncthreads();
    const uint32_t orow = wg.x * 16 + ty, ocol = wg.y * 16 + tx;
    if (orow < a.cols && ocol < a.rows) a.out[(size_t)orow * a.rows + ocol] = tile[tx][ty];
}

extern "C" const void* user_transpose_fn(void) { return (const void*)user_transpose; }
extern "C" uint32_t user_transpose_args_bytes(void) { return sizeof(user_transpose_args); }
