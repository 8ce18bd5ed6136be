// TEST DOUBLE of the small part of the HIP runtime API that the engine's
// runtime uses.  Streams are host threads that run their operations in
// order; "kernels" are host functions registered with fake_register_kernel;
// events complete when their stream reaches them.  Compiling the runtime
// against this header gives a CPU-only library for testing the dispatcher.
#pragma once
#include <cstddef>
#include <cstdint>

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorNotReady = 600,
    hipErrorLaunchFailure = 719
} hipError_t;

struct FakeStream;
struct FakeEvent;
typedef FakeStream* hipStream_t;
typedef FakeEvent* hipEvent_t;

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

struct hipDeviceProp_t {
    int multiProcessorCount;
    char name[256];
};

struct hipFuncAttributes {
    size_t sharedSizeBytes;
    int numRegs;
    int maxThreadsPerBlock;
};

#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipLaunchKernel(const void* fn, dim3 grid, dim3 block, void** args, size_t shmem,
                           hipStream_t s);
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void* fn);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* fn, int block,
                                                        size_t dyn);
const char* hipGetErrorString(hipError_t e);

// code objects: an image is the text "fake-module"; its functions are the
// host functions registered by symbol with fake_register_symbol
struct FakeModule;
struct FakeModuleFn;
typedef FakeModule* hipModule_t;
typedef const FakeModuleFn* hipFunction_t;
typedef enum {
    HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES = 1,
    HIP_FUNC_ATTRIBUTE_NUM_REGS = 4
} hipFunction_attribute;
hipError_t hipModuleLoadData(hipModule_t* m, const void* image);
hipError_t hipModuleUnload(hipModule_t m);
hipError_t hipModuleGetFunction(hipFunction_t* f, hipModule_t m, const char* name);
hipError_t hipModuleLaunchKernel(hipFunction_t f, unsigned gx, unsigned gy, unsigned gz,
                                 unsigned bx, unsigned by, unsigned bz, unsigned shmem,
                                 hipStream_t s, void** params, void** extra);
hipError_t hipFuncGetAttribute(int* v, hipFunction_attribute a, hipFunction_t f);
hipError_t hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(int* n, hipFunction_t f,
                                                              int block, size_t dyn);

// memory: plain host memory; copies are synchronous
typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 } hipMemcpyKind;
hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags = 0);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k,
                          hipStream_t s);
