// TEST DOUBLE of the two launch calls of hip_ext.h the runtime uses: a
// launch whose start and stop events (either may be null) complete when the
// stream reaches the launch and when the launch has run.
#pragma once
#include "hip_runtime.h"

hipError_t hipExtLaunchKernel(const void* fn, dim3 grid, dim3 block, void** args,
                              size_t shmem, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                              int flags);
hipError_t hipExtModuleLaunchKernel(hipFunction_t f, uint32_t gwx, uint32_t gwy, uint32_t gwz,
                                    uint32_t lx, uint32_t ly, uint32_t lz, size_t shmem,
                                    hipStream_t s, void** params, void** extra,
                                    hipEvent_t start = nullptr, hipEvent_t stop = nullptr,
                                    uint32_t flags = 0);
