/*
 * kernelet_device.h -- the device half of the slicing ABI (header-only HIP,
 * gfx950).  Include it in a kernel's source to make the kernel sliceable.
 *
 * Index rectification (Kernelet, Section 4.1 "Kernel Slicing"): a slice of
 * a kernel is a contiguous range of its workgroup ids (Section 2.2), launched
 * on its own small 1-D grid; every workgroup adds the slice's offset to its
 * built-in index and recovers its position in the ORIGINAL grid, which the
 * slice descriptor carries (kl_slice, include/kernelet.h).  A sliceable
 * kernel
 *   - takes (ArgsT args, kl_slice s) by value, args first, in that order;
 *   - is launched with 1-D workgroups of block_threads work-items (a
 *     multiple of 256; threadIdx.y and .z are 0);
 *   - takes its workgroup's position from kl_wg_linear(s) or kl_wg_id3(s)
 *     and the original grid from s.gx, s.gy, s.gz, never from blockIdx or
 *     gridDim (loops striding over the grid included): a slice's launch grid
 *     is s.count workgroups along x.
 * Linearisation is row-major: id = x + gx (y + gy z), so slice k of size c
 * covers ids [k c, min((k + 1) c, gx gy gz)).
 */
#ifndef KERNELET_DEVICE_H
#define KERNELET_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernelet.h"

/* Workgroup id of this workgroup in the original grid, linearised. */
__device__ __forceinline__ uint32_t kl_wg_linear(const kl_slice& s) {
    return s.offset + blockIdx.x;
}

/* (x, y, z) of this workgroup in the original grid (gx, gy, gz). */
__device__ __forceinline__ uint3 kl_wg_id3(const kl_slice& s) {
    const uint32_t lin = kl_wg_linear(s);
    const uint32_t q = lin / s.gx;
    return make_uint3(lin - q * s.gx, q % s.gy, q / s.gy);
}

/* Workgroups in the original grid. */
__device__ __forceinline__ uint64_t kl_grid_wgs(const kl_slice& s) {
    return (uint64_t)s.gx * s.gy * s.gz;
}

#endif /* KERNELET_DEVICE_H */
