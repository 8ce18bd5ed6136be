// TEST DOUBLE: host-thread implementation of hip_runtime.h (see there).
#include "hip/hip_runtime.h"
#include "hip/hip_ext.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "kernelet.h"

struct FakeEvent {
    uint64_t recorded = 0, done = 0;
    double t_done_ms = 0;
    bool err = false;  // recorded after a failed kernel on its stream
};

namespace {
std::mutex g_mu;                 // guards every stream, event and the kernel table
std::condition_variable g_cv;
int g_ncu = 256;

typedef int (*fake_kernel_fn)(const void* args, const kl_slice* s);
struct FakeKernel {
    fake_kernel_fn fn;
    uint32_t args_bytes;
};
std::map<const void*, FakeKernel> g_kernels;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Op {
    int kind;  // 0 launch, 1 record, 2 wait
    FakeKernel k;
    std::vector<uint8_t> args;
    kl_slice slice;
    FakeEvent* ev = nullptr;
    uint64_t gen = 0;
};
}  // namespace

struct FakeStream {
    std::deque<Op> q;
    bool busy = false, stop = false, failed = false;
    std::thread th;
};

namespace {
void stream_main(FakeStream* s) {
    std::unique_lock<std::mutex> lk(g_mu);
    for (;;) {
        g_cv.wait(lk, [&] { return s->stop || !s->q.empty(); });
        if (s->q.empty() && s->stop) return;
        Op op = std::move(s->q.front());
        s->q.pop_front();
        s->busy = true;
        if (op.kind == 0) {
            lk.unlock();
            int rc = op.k.fn(op.args.data(), &op.slice);
            lk.lock();
            if (rc) s->failed = true;
        } else if (op.kind == 1) {
            if (op.gen > op.ev->done) {
                op.ev->done = op.gen;
                op.ev->t_done_ms = now_ms();
                op.ev->err = s->failed;
            }
        } else {
            g_cv.wait(lk, [&] { return op.ev->done >= op.gen; });
        }
        s->busy = false;
        g_cv.notify_all();
    }
}
}  // namespace

struct FakeModule {
    int loaded;
};
struct FakeModuleFn {
    int (*fn)(const void* args, const kl_slice* s);
    uint32_t args_bytes;
};
namespace {
std::map<std::string, FakeModuleFn> g_symbols;  // guarded by g_mu
}

extern "C" {
// Register a host function as the kernel `name` of every fake code object.
void fake_register_symbol(const char* name, fake_kernel_fn fn, uint32_t args_bytes) {
    std::lock_guard<std::mutex> g(g_mu);
    g_symbols[name] = FakeModuleFn{fn, args_bytes};
}
// Register a host function that stands for a GPU kernel.
void fake_register_kernel(const void* key, fake_kernel_fn fn, uint32_t args_bytes) {
    std::lock_guard<std::mutex> g(g_mu);
    g_kernels[key] = FakeKernel{fn, args_bytes};
}
void fake_set_cu(int n) { g_ncu = n; }
}

hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    std::memset(p, 0, sizeof(*p));
    p->multiProcessorCount = g_ncu;
    std::strcpy(p->name, "fake");
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    auto* st = new FakeStream();
    st->th = std::thread(stream_main, st);
    *s = st;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    {
        std::lock_guard<std::mutex> g(g_mu);
        s->stop = true;
    }
    g_cv.notify_all();
    s->th.join();
    delete s;
    return hipSuccess;
}
// Test knob: microseconds a stream synchronisation lingers after the stream
// drained, widening the window in which another host thread launches more.
static std::atomic<int> g_sync_linger_us{0};
extern "C" void fake_set_sync_linger_us(int us) { g_sync_linger_us = us; }

hipError_t hipStreamSynchronize(hipStream_t s) {
    bool failed;
    {
        std::unique_lock<std::mutex> lk(g_mu);
        g_cv.wait(lk, [&] { return s->q.empty() && !s->busy; });
        failed = s->failed;
    }
    if (const int us = g_sync_linger_us.load())
        std::this_thread::sleep_for(std::chrono::microseconds(us));
    return failed ? hipErrorLaunchFailure : hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    std::lock_guard<std::mutex> g(g_mu);
    if (e->recorded > e->done) {
        Op op;
        op.kind = 2;
        op.ev = e;
        op.gen = e->recorded;
        s->q.push_back(std::move(op));
        g_cv.notify_all();
    }
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new FakeEvent();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!s) {
        // the null stream holds no queued work here: complete at once
        e->done = ++e->recorded;
        e->t_done_ms = now_ms();
        g_cv.notify_all();
        return hipSuccess;
    }
    Op op;
    op.kind = 1;
    op.ev = e;
    op.gen = ++e->recorded;
    s->q.push_back(std::move(op));
    g_cv.notify_all();
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    std::lock_guard<std::mutex> g(g_mu);
    if (e->done < e->recorded) return hipErrorNotReady;
    return e->err ? hipErrorLaunchFailure : hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> g(g_mu);
    if (a->done < a->recorded || b->done < b->recorded) return hipErrorNotReady;
    *ms = (float)(b->t_done_ms - a->t_done_ms);
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void* fn, dim3 grid, dim3, void** args, size_t,
                           hipStream_t s) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_kernels.find(fn);
    if (it == g_kernels.end()) return hipErrorInvalidValue;
    Op op;
    op.kind = 0;
    op.k = it->second;
    op.args.assign((const uint8_t*)args[0], (const uint8_t*)args[0] + it->second.args_bytes);
    std::memcpy(&op.slice, args[1], sizeof(kl_slice));
    if (op.slice.count != grid.x) return hipErrorInvalidValue;
    s->q.push_back(std::move(op));
    g_cv.notify_all();
    return hipSuccess;
}
hipError_t hipModuleLoadData(hipModule_t* m, const void* image) {
    if (std::strcmp((const char*)image, "fake-module") != 0) return hipErrorInvalidValue;
    *m = new FakeModule{1};
    return hipSuccess;
}
hipError_t hipModuleUnload(hipModule_t m) {
    delete m;
    return hipSuccess;
}
hipError_t hipModuleGetFunction(hipFunction_t* f, hipModule_t, const char* name) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_symbols.find(name);
    if (it == g_symbols.end()) return hipErrorInvalidValue;
    *f = &it->second;
    return hipSuccess;
}
hipError_t hipModuleLaunchKernel(hipFunction_t f, unsigned gx, unsigned, unsigned, unsigned,
                                 unsigned, unsigned, unsigned, hipStream_t s, void** args,
                                 void**) {
    std::lock_guard<std::mutex> g(g_mu);
    Op op;
    op.kind = 0;
    op.k = FakeKernel{f->fn, f->args_bytes};
    op.args.assign((const uint8_t*)args[0], (const uint8_t*)args[0] + f->args_bytes);
    std::memcpy(&op.slice, args[1], sizeof(kl_slice));
    if (op.slice.count != gx) return hipErrorInvalidValue;
    s->q.push_back(std::move(op));
    g_cv.notify_all();
    return hipSuccess;
}
// The start event completes when the stream reaches the launch, the stop
// event when the launch has run (both recorded around it on its stream).
hipError_t hipExtLaunchKernel(const void* fn, dim3 grid, dim3 block, void** args,
                              size_t shmem, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                              int) {
    if (start && hipEventRecord(start, s) != hipSuccess) return hipErrorInvalidValue;
    hipError_t e = hipLaunchKernel(fn, grid, block, args, shmem, s);
    if (e != hipSuccess) return e;
    return stop ? hipEventRecord(stop, s) : hipSuccess;
}
hipError_t hipExtModuleLaunchKernel(hipFunction_t f, uint32_t gwx, uint32_t gwy, uint32_t gwz,
                                    uint32_t lx, uint32_t ly, uint32_t lz, size_t shmem,
                                    hipStream_t s, void** params, void** extra,
                                    hipEvent_t start, hipEvent_t stop, uint32_t) {
    if (lx == 0 || gwx % lx) return hipErrorInvalidValue;
    if (start && hipEventRecord(start, s) != hipSuccess) return hipErrorInvalidValue;
    hipError_t e = hipModuleLaunchKernel(f, gwx / lx, gwy, gwz, lx, ly, lz, (unsigned)shmem, s,
                                         params, extra);
    if (e != hipSuccess) return e;
    return stop ? hipEventRecord(stop, s) : hipSuccess;
}
hipError_t hipFuncGetAttribute(int* v, hipFunction_attribute a, hipFunction_t) {
    *v = a == HIP_FUNC_ATTRIBUTE_NUM_REGS ? 32 : 0;
    return hipSuccess;
}
hipError_t hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(int* n, hipFunction_t, int,
                                                              size_t) {
    *n = 8;
    return hipSuccess;
}
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void*) {
    a->sharedSizeBytes = 0;
    a->numRegs = 32;
    a->maxThreadsPerBlock = 1024;
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
    *n = 8;
    return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
    *p = std::malloc(n ? n : 1);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFree(void* p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
    std::memcpy(dst, src, n);
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "hipSuccess";
        case hipErrorNotReady: return "hipErrorNotReady";
        case hipErrorLaunchFailure: return "hipErrorLaunchFailure";
        default: return "hipErrorInvalidValue";
    }
}

// ---------------------------------------------------------------- builtins
// The fake library has no built-in kernels.
namespace kl {
bool builtin_check(const char*, const void*, uint32_t, kl_dim3*, std::string* err) {
    *err = "no built-in kernels in the fake library";
    return false;
}
bool is_builtin_fn(const void*, const char**) { return false; }
}  // namespace kl

// The surrogate network's forward pass on the host (the double's "device"
// memory is host memory): same parameter layout as the library's kernel.
extern "C" kl_status kernelet_mlp_forward(const float* p, const float* x, uint32_t n, float* y,
                                          void*) {
    const int I = 16, H = 64;
    const float *W1 = p, *b1 = W1 + I * H, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H,
                *b3 = W3 + H;
    for (uint32_t s = 0; s < n; ++s) {
        float h1[64], out = b3[0];
        for (int j = 0; j < H; ++j) {
            float a = b1[j];
            for (int i = 0; i < I; ++i) a += x[s * I + i] * W1[i * H + j];
            h1[j] = a > 0 ? a : 0;
        }
        for (int j = 0; j < H; ++j) {
            float a = b2[j];
            for (int i = 0; i < H; ++i) a += h1[i] * W2[i * H + j];
            out += (a > 0 ? a : 0) * W3[j];
        }
        y[s] = out;
    }
    return KL_OK;
}

extern "C" kl_status kernelet_builtin(const char*, kl_kernel_desc*) { return KL_ENOTFOUND; }
extern "C" kl_status kernelet_builtin_grid(const char*, const void*, uint32_t, kl_dim3*) {
    return KL_ENOTFOUND;
}

// ------------------------------------------------------------ fake kernels
// "visit": every workgroup of the slice adds one to visits[its id] (host
// memory), then the slice sleeps us_per_wg microseconds per workgroup; the
// slice is appended to a log (tag, offset, count, start ms, end ms).
struct FakeVisitArgs {
    uint32_t* visits;
    double* log;        // 5 doubles per entry
    uint32_t* log_len;  // entries written
    uint32_t log_cap;
    uint32_t tag;
    uint32_t us_per_wg;
    uint32_t fail;      // nonzero: report a device error
};

extern "C" int fake_visit(const void* a_, const kl_slice* s) {
    FakeVisitArgs a;
    std::memcpy(&a, a_, sizeof(a));
    double t0 = now_ms();
    // the slice's work takes its time first and its writes land at its end,
    // as a kernel's results are complete only when it finishes
    if (a.us_per_wg)
        std::this_thread::sleep_for(std::chrono::microseconds((uint64_t)a.us_per_wg * s->count));
    for (uint32_t b = 0; b < s->count; ++b) a.visits[s->offset + b]++;
    double t1 = now_ms();
    std::lock_guard<std::mutex> g(g_mu);
    if (a.log && *a.log_len < a.log_cap) {
        double* e = a.log + 5 * (*a.log_len);
        e[0] = a.tag;
        e[1] = s->offset;
        e[2] = s->count;
        e[3] = t0;
        e[4] = t1;
        ++*a.log_len;
    }
    return a.fail ? 1 : 0;
}

extern "C" uint32_t fake_visit_args_bytes() { return sizeof(FakeVisitArgs); }
