// Runtime of the sliced co-execution engine: the C ABI of kernelet.h, the
// kernel registry, the job table, the dispatcher that executes Algorithm 1
// (Kernelet, Section 4.2) over HIP streams, and the FIFO baseline.
//
// Execution model on the GPU.  The runtime owns `lanes` HIP streams (two by
// default, each on its own hardware queue) plus the FIFO stream.  A
// co-schedule <K1, K2, b1, b2> puts K1 on one lane and K2 on the other and
// launches their slices (b_i workgroups per CU, i.e. b_i * n_cu workgroups
// per slice) back to back, keeping at most `inflight` slices queued per
// lane.  Each slice's completion event is attached to its dispatch
// (hipExtLaunchKernel's stop event), not recorded behind it: a recorded
// event is a packet of its own that holds the queue until the slice has
// drained (about 3.5 us of idle GPU per slice on MI355X), while an event
// carried by the dispatch costs the GPU nothing.  Consecutive slices of a
// lane are ordered by the stream; a job that changes lanes, or depends on a
// job last launched on another lane, first makes the new lane wait on that
// job's last event.  When one kernel of the
// pair has launched all its workgroups the co-schedule ends and
// FindCoSchedule runs again on the pending set, which holds the other
// kernel's residual (Section 2.2: residuals and new arrivals are
// re-optimised together).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <set>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <sys/prctl.h>
#include <thread>
#include <vector>

#include "kernelet.h"
#include "model.hpp"

namespace kl {

thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

bool builtin_check(const char* name, const void* args, uint32_t bytes, kl_dim3* grid,
                   std::string* err);
bool is_builtin_fn(const void* fn, const char** name);

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// A short timed wait on the runtime's condition variable.  Thread-sanitizer
// builds wait on the system clock (pthread_cond_timedwait, which their
// runtime intercepts; a steady-clock wait goes through
// pthread_cond_clockwait, which older ones do not see, and they then report
// lock errors that are not there); other builds wait on the steady clock,
// immune to clock steps.
template <class Lock>
static void wait_us(std::condition_variable& cv, Lock& lk, int64_t us) {
#if defined(__SANITIZE_THREAD__)
    cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(us));
#else
    cv.wait_for(lk, std::chrono::microseconds(us));
#endif
}

#define KL_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
            return KL_EHIP;                                                       \
        }                                                                         \
    } while (0)

// ------------------------------------------------------------ event pool
struct EvPool {
    std::vector<hipEvent_t> ev;
    std::vector<int> refs;
    std::vector<int> free_;
    int get() {
        if (free_.empty()) {
            hipEvent_t e;
            // timing enabled: a timed slice measures from its start event
            // to this, its completion event
            if (hipEventCreate(&e) != hipSuccess) return -1;
            ev.push_back(e);
            refs.push_back(0);
            free_.push_back((int)ev.size() - 1);
        }
        int i = free_.back();
        free_.pop_back();
        refs[i] = 1;
        return i;
    }
    void ref(int i) {
        if (i >= 0) ++refs[i];
    }
    void unref(int i) {
        if (i >= 0 && --refs[i] == 0) free_.push_back(i);
    }
    void destroy() {
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
        refs.clear();
        free_.clear();
    }
};

// ------------------------------------------------------------- objects
struct KernelType {
    std::string name;
    const void* fn = nullptr;
    // a kernel loaded from a code object (kernelet_register_image)
    hipModule_t mod = nullptr;
    hipFunction_t mfn = nullptr;
    uint32_t block = 256, args_bytes = 0, flags = 0;
    const char* builtin = nullptr;
    kl_profile prof{};
    bool has_prof = false;
    int static_lds = 0;
    // launch timing (kernelet_time_kernel)
    bool timed = false;
    double time_ms = 0;
    int64_t time_launches = 0, time_wgs = 0;
};

// A slice in flight on a lane: its completion event (pool index), its job,
// and for a timed kernel the event its dispatch started.
struct Inflight {
    int ev;
    kl_job job;
    hipEvent_t start;
    int type;
    uint32_t wgs;
    double pred_us;  // predicted duration (0: unknown)
    int si;          // stream index: lane * 2 + the lane's stream
};

// Streams a job's slices may use: two per lane, at most four lanes.
constexpr int kMaxStreams = 8;

enum JobState { J_WAIT_DEP = 0, J_PENDING, J_LAUNCHED, J_DONE, J_CANCELED };

struct Job {
    kl_job id = -1;
    int type = -1;
    kl_dim3 grid{1, 1, 1};
    uint32_t total = 0, next = 0, fixed_slice = 0;
    int occ = 0;  // FIXED policy: workgroups per CU (0: the kernel's maximum)
    std::vector<uint8_t> args;
    kl_job after = KL_NO_JOB;
    uint32_t client = 0;
    uint64_t footprint = 0;
    int64_t carry = 0;  // footprint of finished predecessors released with this job
    JobState st = J_PENDING;
    bool admitted = false;
    // slices launched and not yet retired; per stream, the event of the
    // job's latest slice on it (pool index, ref held): the slices on one
    // stream finish in order, so these events finishing means all have
    int outstanding = 0;
    int tail[kMaxStreams] = {-1, -1, -1, -1, -1, -1, -1, -1};
    uint32_t waited = 0;  // streams already ordered after the predecessor's slices
    std::vector<kl_job> dependents;
    int64_t t_submit = 0, t_start = 0, t_done = 0;
    bool error = false;
};

struct Lane {
    // one or two streams (cfg.lane_streams); a co-schedule alternates a
    // job's slices between them
    hipStream_t s[2] = {nullptr, nullptr};
    int nsub = 1;
    int next_sub = 0;
    std::deque<Inflight> inflight;
    double queued_us = 0;  // predicted work of the slices in flight
    int unpredicted = 0;   // slices in flight without a prediction
    kl_job job = KL_NO_JOB;
    uint32_t slice = 0;
    uint32_t dyn_lds = 0;
    std::vector<int> barrier;  // wait on these before the next launch (solo runs)
};

}  // namespace kl

struct kl_runtime {
    int device = 0;
    kl_config cfg{};
    std::unique_ptr<kl::Planner> planner;
    std::vector<kl::KernelType> kernels;
    std::map<kl_job, kl::Job> jobs;
    std::set<kl_job> live;  // jobs neither finished nor cancelled, in submission order
    // live jobs with workgroups still to launch (waiting on a predecessor or
    // pending), all and per kernel type, and live jobs not yet admitted by
    // the memory budget: the dispatcher's scans visit these, not every job
    std::set<kl_job> unlaunched;
    std::vector<std::set<kl_job>> unlaunched_by_type;
    std::set<kl_job> unadmitted;
    kl_job next_id = 0;
    std::vector<kl::Lane> lanes;
    kl::EvPool pool;
    std::mutex mu;
    std::condition_variable cv;  // submissions, launches, completions
    std::thread worker;
    std::atomic<bool> stop{false};
    bool worker_running = false;
    kl_policy worker_policy = KL_POLICY_MARKOV;
    uint32_t worker_flags = 0;
    bool scheduling = false;  // a dispatcher loop is active
    int64_t resident = 0;     // admitted footprint bytes
    int64_t resident_peak = 0;
    kl_stats stats{};
    std::vector<kl_decision> declog;
    int64_t t0_dec = 0;
    // co-schedule currently issued
    bool cs_active = false;
    kl_job cs_job[3] = {KL_NO_JOB, KL_NO_JOB, KL_NO_JOB};
    // start events of timed launches
    std::vector<hipEvent_t> tev_free;
    // surrogate network (kernelet_set_surrogate): parameters and batch
    // buffers on the device, staging in pinned host memory, its own stream
    float* sur_params = nullptr;
    float* sur_x = nullptr;
    float* sur_y = nullptr;
    float* sur_hx = nullptr;
    float* sur_hy = nullptr;
    uint32_t sur_cap = 0;
    hipStream_t sur_stream = nullptr;
    // OPT: measured co-runs were loaded; RANDOM: decisions drawn so far
    bool have_measures = false;
    uint64_t random_draws = 0;
};

namespace kl {

static kl_config defaults() {
    kl_config c{};
    c.n_cu = 0;
    c.wmax = 8;
    c.vgpr_file = 512;
    c.lds_cu = 160 * 1024;
    c.alpha_p = 0.4;
    c.alpha_m = 0.1;
    c.use_prune = 1;
    c.ratio_mode = KL_MODE_CP;
    c.cp_min = -1.0;
    c.pair_same_type = 1;
    c.group_max = 2;
    c.mem_latency = 400.0;
    c.beta = 0.0;
    c.lanes = 2;
    c.inflight = 2;
    c.inflight_us = 50;
    c.auto_profile = 1;
    c.lane_streams = 1;
    c.lds_reserve = 2;
    c.max_slices = 0;
    c.hbm_budget = 0;
    c.surrogate_topk = 4;
    return c;
}

static kl_status check_cfg(const kl_config& c) {
    if (c.wmax < 1 || c.wmax > 16 || c.vgpr_file < 1 || c.lds_cu < 0 || c.lanes < 1 ||
        c.lanes > 4 || c.inflight < 1 || c.inflight > 64 || c.n_cu < 0 || c.mem_latency < 1 ||
        c.beta < 0 || !(c.beta_lds >= 0) || !(c.min_pair_slots >= 0) || c.alpha_p < 0 || c.alpha_m < 0 || c.ratio_mode < 0 || c.ratio_mode > 2 ||
        c.lds_reserve < 0 || c.lds_reserve > 2 || c.inflight_us < 0 ||
        c.inflight_us > 100000 || c.auto_profile < 0 || c.auto_profile > 1 ||
        c.lane_streams < 1 || c.lane_streams > 2 ||
 c.surrogate_topk < 0 || c.max_slices < 0 ||
        c.solo_overlap < 0 || c.solo_overlap > 1 || c.pair_same_type < 0 ||
        c.pair_same_type > 1 || c.group_max < 2 || c.group_max > 3 ||
        c.hbm_budget < 0) {
        set_error("invalid kl_config field");
        return KL_EINVAL;
    }
    return KL_OK;
}

static kl_status check_profile(const kl_profile& p) {
    if (!(p.r_mem >= 0 && p.r_comp >= 0 && p.r_mem + p.r_comp <= 1.0) || p.mem_req < 0 ||
        p.lat_mem < 0 || (p.r_comp > 0 && !(p.lat_comp >= 1.0)) || !(p.instr_per_wave > 0) ||
        p.max_wg_per_cu < 1 || p.waves_per_simd < 1 || p.max_wg_per_cu > 64 ||
        p.waves_per_simd > 64 || p.max_wg_per_cu * p.waves_per_simd > 64 || p.vgpr < 0 ||
        p.lds_bytes < 0 ||
        p.access < 0 || p.access > 2 || p.comp_pool < 0 || p.comp_pool > 1) {
        set_error("invalid kl_profile field");
        return KL_EINVAL;
    }
    return KL_OK;
}

// ---------------------------------------------------------- bookkeeping
// All helpers below run with rt->mu held.

static void release_dependents(kl_runtime* rt, Job& j) {
    for (kl_job d : j.dependents) {
        auto it = rt->jobs.find(d);
        if (it != rt->jobs.end() && it->second.st == J_WAIT_DEP) it->second.st = J_PENDING;
    }
}

// The job has no workgroups left to launch (or will never launch them).
static void leave_unlaunched(kl_runtime* rt, const Job& j) {
    rt->unlaunched.erase(j.id);
    if (j.type >= 0 && j.type < (int)rt->unlaunched_by_type.size())
        rt->unlaunched_by_type[j.type].erase(j.id);
}

// The job leaves every scan set (finished or cancelled).
static void forget_job(kl_runtime* rt, const Job& j) {
    rt->live.erase(j.id);
    rt->unadmitted.erase(j.id);
    leave_unlaunched(rt, j);
}

static void mark_done(kl_runtime* rt, Job& j, bool error) {
    if (j.st == J_DONE) return;
    j.st = J_DONE;
    forget_job(rt, j);
    j.error = error;
    j.t_done = now_ns();
    int64_t rel = j.carry + (j.admitted ? (int64_t)j.footprint : 0);
    j.carry = 0;
    j.admitted = false;
    rt->stats.jobs_done++;
    if (rel == 0) return;
    // the memory of a chain of dependent launches stays charged until its
    // last launch: hand the release on to a dependant that is still to run
    for (kl_job d : j.dependents) {
        auto it = rt->jobs.find(d);
        if (it != rt->jobs.end() && it->second.st != J_DONE && it->second.st != J_CANCELED) {
            it->second.carry += rel;
            return;
        }
    }
    rt->resident -= rel;
}

static hipEvent_t timing_event(kl_runtime* rt) {
    if (!rt->tev_free.empty()) {
        hipEvent_t e = rt->tev_free.back();
        rt->tev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Drop the job's references to its latest slice events.
static void release_tails(kl_runtime* rt, Job& j) {
    for (int& e : j.tail) {
        if (e >= 0) rt->pool.unref(e);
        e = -1;
    }
}

// Whether every slice of a fully launched job has finished (its latest
// slice on each stream has); *failed: one of them failed.
static bool tails_done(kl_runtime* rt, const Job& j, bool* failed) {
    *failed = false;
    for (int e : j.tail) {
        if (e < 0) continue;
        const hipError_t q = hipEventQuery(rt->pool.ev[e]);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) *failed = true;
    }
    return true;
}

// The job's events other lanes must wait on to start after all of it.
static void tails_of(const Job& j, std::vector<int>* out) {
    for (int e : j.tail)
        if (e >= 0) out->push_back(e);
}

// Retire finished slices on every lane (in any order: a lane's two streams
// run side by side) and the jobs whose last slice they were; a timed slice
// adds its dispatch's duration (start event to completion event) to its
// kernel's counters.
static void poll_lanes(kl_runtime* rt) {
    for (auto& ln : rt->lanes) {
        for (size_t i = 0; i < ln.inflight.size();) {
            const Inflight f = ln.inflight[i];
            const int e = f.ev;
            hipError_t q = hipEventQuery(rt->pool.ev[e]);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            const kl_job jid = f.job;
            ln.inflight.erase(ln.inflight.begin() + (std::ptrdiff_t)i);
            ln.queued_us = ln.inflight.empty() ? 0.0 : std::max(0.0, ln.queued_us - f.pred_us);
            if (f.pred_us <= 0) --ln.unpredicted;
            if (f.start) {
                float ms = 0.f;
                if (q == hipSuccess &&
                    hipEventElapsedTime(&ms, f.start, rt->pool.ev[e]) == hipSuccess) {
                    KernelType& kt = rt->kernels[f.type];
                    kt.time_ms += ms;
                    kt.time_launches++;
                    kt.time_wgs += f.wgs;
                }
                rt->tev_free.push_back(f.start);
            }
            auto it = rt->jobs.find(jid);
            if (it != rt->jobs.end()) {
                Job& j = it->second;
                if (q != hipSuccess) j.error = true;
                if (j.outstanding > 0) --j.outstanding;
                if (j.tail[f.si] == e) {
                    rt->pool.unref(e);
                    j.tail[f.si] = -1;
                }
                if (j.st == J_LAUNCHED && j.outstanding == 0) {
                    mark_done(rt, j, j.error);
                    release_tails(rt, j);
                }
            }
            rt->pool.unref(e);
        }
        for (size_t i = 0; i < ln.barrier.size();) {
            if (hipEventQuery(rt->pool.ev[ln.barrier[i]]) == hipSuccess) {
                rt->pool.unref(ln.barrier[i]);
                ln.barrier.erase(ln.barrier.begin() + (std::ptrdiff_t)i);
            } else {
                ++i;
            }
        }
    }
}

// Largest LDS one workgroup may allocate, static plus dynamic.
static const int64_t kLdsPerWg = 65536;

// Dynamic LDS for kernel `kt` in a co-schedule where it runs at b_self
// workgroups per CU beside partners at b_others workgroups per CU in all,
// whose workgroups hold others_lds bytes of static LDS per CU in all.
static uint32_t dyn_lds_for(kl_runtime* rt, const KernelType& kt, int b_self, int b_others,
                            int64_t others_lds, bool capped) {
    const int64_t lds = rt->cfg.lds_cu;
    int64_t per = 0;
    if (rt->cfg.lds_reserve == 1) {
        if (b_self + b_others <= 0) return 0;
        per = lds / (b_self + b_others) - kt.static_lds;
    } else if (rt->cfg.lds_reserve == 2) {
        if (!capped || b_self < 1) return 0;
        // (b_self + 1) workgroups must not fit, b_self must leave room for the
        // partners' static LDS
        int64_t total = lds / (b_self + 1) + 256;
        int64_t room = lds - others_lds;
        if ((int64_t)b_self * total > room || total > kLdsPerWg) return 0;  // cannot cap
        per = total - kt.static_lds;
    } else {
        return 0;
    }
    int64_t cap = kLdsPerWg - kt.static_lds;
    if (per > cap) per = cap;
    return per > 0 ? (uint32_t)((per + 255) & ~255ll) : 0u;
}

// Predicted duration of `count` workgroups of kernel kt run alone, in
// microseconds (its profile's solo rate; an issue slot is 4 cycles at
// 2.4 GHz); 0 when the kernel has no profile.
static double predict_us(kl_runtime* rt, const KernelType& kt, int type, uint32_t count) {
    if (!kt.has_prof) return 0.0;
    const double ipc = kt.prof.solo_ipc > 0 ? kt.prof.solo_ipc : rt->planner->solo(type);
    const double rate = wg_rate(kt.prof, ipc, rt->cfg.n_cu);  // workgroups per slot
    return rate > 0 ? (double)count / rate * (4.0 / 2400.0) : 0.0;
}

// Whether lane ln may queue another slice of a co-schedule: fewer than
// `inflight` slices, or less than `inflight_us` of predicted work when every
// slice in flight has a prediction (at most 64 slices).
static bool lane_has_room(kl_runtime* rt, const Lane& ln) {
    // the window is per stream: a lane with two streams queues twice as much
    const size_t n = ln.inflight.size();
    if ((int)n < rt->cfg.inflight * ln.nsub) return true;
    if (rt->cfg.inflight_us <= 0 || n >= 64 || ln.unpredicted > 0) return false;
    return ln.queued_us < (double)rt->cfg.inflight_us * ln.nsub;
}

// Launch the next slice of job `jid` on lane `li`, `count` workgroups: on
// the lane's first stream, or with `alternate` on its two streams in turn.
// Slices of one job need no order among themselves (their workgroups are
// independent); a job starts after its predecessor's every slice, and after
// the lane's barrier.
static kl_status launch_slice(kl_runtime* rt, int li, kl_job jid, uint32_t count,
                              bool alternate) {
    Lane& ln = rt->lanes[li];
    Job& j = rt->jobs.at(jid);
    const KernelType& kt = rt->kernels[j.type];
    if (count > j.total - j.next) count = j.total - j.next;
    if (count == 0) return KL_OK;
    int sub = 0;
    if (alternate && ln.nsub > 1) {
        sub = ln.next_sub;
        ln.next_sub = (ln.next_sub + 1) % ln.nsub;
    }
    hipStream_t st = ln.s[sub];
    const int si = li * 2 + sub;
    // ordering against work on other lanes: every stream of the lane waits
    if (!ln.barrier.empty()) {
        for (int b = 0; b < ln.nsub; ++b)
            for (int e : ln.barrier) KL_HIP(hipStreamWaitEvent(ln.s[b], rt->pool.ev[e], 0));
        for (int e : ln.barrier) rt->pool.unref(e);
        ln.barrier.clear();
    }
    if (j.after != KL_NO_JOB && !(j.waited & (1u << si))) {
        auto it = rt->jobs.find(j.after);
        if (it != rt->jobs.end() && it->second.st != J_DONE)
            for (int y = 0; y < kMaxStreams; ++y)
                if (y != si && it->second.tail[y] >= 0)  // same stream: in order already
                    KL_HIP(hipStreamWaitEvent(st, rt->pool.ev[it->second.tail[y]], 0));
        j.waited |= 1u << si;
    }
    kl_slice s;
    s.offset = j.next;
    s.count = count;
    s.gx = j.grid.x;
    s.gy = j.grid.y;
    s.gz = j.grid.z;
    s.reserved = 0;
    void* params[2] = {j.args.data(), &s};
    hipEvent_t ta = nullptr;
    if (kt.timed) {
        ta = timing_event(rt);
        if (!ta) {
            set_error("hipEventCreate failed");
            return KL_EHIP;
        }
    }
    if (kt.mfn && (uint64_t)count * kt.block > 0xffffffffull) {
        if (ta) rt->tev_free.push_back(ta);
        set_error("launch of " + kt.name + ": more than 2^32 work-items in one slice");
        return KL_EINVAL;
    }
    int ev = rt->pool.get();
    if (ev < 0) {
        if (ta) rt->tev_free.push_back(ta);
        set_error("hipEventCreate failed");
        return KL_EHIP;
    }
    // the completion event (and the start event of a timed kernel) travel
    // with the dispatch itself
    hipError_t e = kt.mfn ? hipExtModuleLaunchKernel(kt.mfn, count * kt.block, 1, 1, kt.block,
                                                     1, 1, ln.dyn_lds, st, params, nullptr,
                                                     ta, rt->pool.ev[ev], 0)
                          : hipExtLaunchKernel(kt.fn, dim3(count), dim3(kt.block), params,
                                               ln.dyn_lds, st, ta, rt->pool.ev[ev], 0);
    if (e != hipSuccess) {
        rt->pool.unref(ev);
        if (ta) rt->tev_free.push_back(ta);
        set_error(std::string("hipExtLaunchKernel(") + kt.name + "): " + hipGetErrorString(e));
        j.error = true;
        return KL_EHIP;
    }
    if (j.next == 0) j.t_start = now_ns();
    j.next += count;
    rt->stats.slices_launched++;
    const double pred = predict_us(rt, kt, j.type, count);
    ln.inflight.push_back(Inflight{ev, jid, ta, j.type, count, pred, si});
    ln.queued_us += pred;
    if (pred <= 0) ++ln.unpredicted;
    ++j.outstanding;
    rt->pool.ref(ev);  // the job's reference
    if (j.tail[si] >= 0) rt->pool.unref(j.tail[si]);
    j.tail[si] = ev;
    if (j.next >= j.total) {
        j.st = J_LAUNCHED;
        leave_unlaunched(rt, j);
        release_dependents(rt, j);
    }
    return KL_OK;
}

// Admission by the memory budget: jobs in submission order while the
// admitted footprint fits.
static void admit(kl_runtime* rt) {
    while (!rt->unadmitted.empty()) {
        Job& j = rt->jobs.at(*rt->unadmitted.begin());
        if (rt->cfg.hbm_budget > 0 &&
            rt->resident + (int64_t)j.footprint > rt->cfg.hbm_budget)
            break;  // keep submission order: nothing later overtakes
        j.admitted = true;
        rt->resident += (int64_t)j.footprint;
        rt->resident_peak = std::max(rt->resident_peak, rt->resident);
        rt->unadmitted.erase(rt->unadmitted.begin());
    }
}

static bool runnable(const Job& j) {
    return j.admitted && j.st == J_PENDING && j.next < j.total;
}

static void log_decision(kl_runtime* rt, const Decision& d, const uint32_t* sl, double us) {
    kl_decision x{};
    x.j1 = d.j1;
    x.j2 = d.j2;
    x.j3 = d.j3;
    x.b1 = d.b1;
    x.b2 = d.b2;
    x.b3 = d.b3;
    x.slice1 = sl[0];
    x.slice2 = sl[1];
    x.slice3 = sl[2];
    x.value = d.value;
    x.cipc1 = d.cipc1;
    x.cipc2 = d.cipc2;
    x.cipc3 = d.cipc3;
    if (rt->declog.empty() && rt->t0_dec == 0) rt->t0_dec = now_ns();
    x.t_us = (now_ns() - rt->t0_dec) / 1e3;
    rt->declog.push_back(x);
    rt->stats.decisions++;
    rt->stats.decision_us_total += us;
}

static uint32_t slice_size(kl_runtime* rt, const Job& j, int b) {
    if (j.fixed_slice) return j.fixed_slice;
    uint64_t s = (uint64_t)b * (uint64_t)rt->cfg.n_cu;
    const KernelType& kt = rt->kernels[j.type];
    if (kt.has_prof && kt.prof.min_slice_wgs > 0 && s < (uint64_t)kt.prof.min_slice_wgs)
        s = (uint64_t)kt.prof.min_slice_wgs;
    if (rt->cfg.max_slices > 0) {
        uint64_t floor_s = (j.total + rt->cfg.max_slices - 1) / rt->cfg.max_slices;
        if (s < floor_s) s = floor_s;
    }
    return s > 0xffffffffull ? 0xffffffffu : (uint32_t)std::max<uint64_t>(s, 1);
}

// One step of the FIFO policy: launch every runnable job whole, in id order,
// stopping at the first job that is not yet runnable.
static kl_status fifo_step(kl_runtime* rt, bool* progressed) {
    Lane& ln = rt->lanes[0];
    ln.dyn_lds = 0;
    for (auto it = rt->unlaunched.begin(); it != rt->unlaunched.end();) {
        Job& j = rt->jobs.at(*it);
        ++it;  // launching the job takes it out of the set
        if (!runnable(j)) break;
        kl_status s = launch_slice(rt, 0, j.id, j.total - j.next, false);
        if (s) return s;
        *progressed = true;
    }
    return KL_OK;
}

// Plain concurrent execution (KL_POLICY_CONCURRENT): every lane, while its
// in-flight window has room, takes the earliest runnable job not yet
// launched and launches it whole; dependencies across lanes are kept by
// launch_slice's event waits.
static kl_status concurrent_step(kl_runtime* rt, bool* progressed) {
    for (int li = 0; li < (int)rt->lanes.size(); ++li) {
        Lane& ln = rt->lanes[li];
        ln.dyn_lds = 0;
        ln.job = KL_NO_JOB;
        while ((int)ln.inflight.size() < rt->cfg.inflight) {
            Job* next = nullptr;
            for (kl_job id : rt->unlaunched) {
                Job& j = rt->jobs.at(id);
                if (runnable(j) && j.next == 0) {
                    next = &j;
                    break;
                }
            }
            if (!next) break;
            kl_status s = launch_slice(rt, li, next->id, next->total, false);
            if (s) return s;
            *progressed = true;
        }
    }
    return KL_OK;
}

// Surrogate scores of candidate pairs: one batched inference over every
// feasible slice ratio of every pair; a pair's score is its best predicted
// weighted speedup.  False (the caller then evaluates every pair with the
// Markov model) on a device error.
static bool surrogate_scores(
    kl_runtime* rt, const std::vector<std::pair<const kl_profile*, const kl_profile*>>& pp,
    std::vector<double>* scores, std::vector<std::pair<int, int>>* ratios) {
    auto t0 = std::chrono::steady_clock::now();
    const kl_config& c = rt->cfg;
    std::vector<int> owner;  // candidate -> pair
    std::vector<std::pair<int, int>> cand;  // candidate -> (b1, b2)
    std::vector<float> feat;
    for (size_t i = 0; i < pp.size(); ++i) {
        const kl_profile& a = *pp[i].first;
        const kl_profile& b = *pp[i].second;
        for (int b1 = 1; b1 <= a.max_wg_per_cu; ++b1)
            for (int b2 = 1; b2 <= b.max_wg_per_cu; ++b2) {
                if (!ratio_feasible(a, b, c, b1, b2)) continue;
                float f[16];
                surrogate_features(a, b1, c.wmax, f);
                surrogate_features(b, b2, c.wmax, f + 8);
                feat.insert(feat.end(), f, f + 16);
                owner.push_back((int)i);
                cand.emplace_back(b1, b2);
            }
    }
    const uint32_t n = (uint32_t)owner.size();
    scores->assign(pp.size(), -1e30);
    ratios->assign(pp.size(), std::make_pair(0, 0));
    if (n == 0) return true;
    if (n > rt->sur_cap) {
        uint32_t cap = 1024;
        while (cap < n) cap *= 2;
        (void)hipFree(rt->sur_x);
        (void)hipFree(rt->sur_y);
        (void)hipHostFree(rt->sur_hx);
        (void)hipHostFree(rt->sur_hy);
        rt->sur_x = rt->sur_y = rt->sur_hx = rt->sur_hy = nullptr;
        rt->sur_cap = 0;
        if (hipMalloc((void**)&rt->sur_x, (size_t)cap * 16 * sizeof(float)) != hipSuccess ||
            hipMalloc((void**)&rt->sur_y, (size_t)cap * sizeof(float)) != hipSuccess ||
            hipHostMalloc((void**)&rt->sur_hx, (size_t)cap * 16 * sizeof(float)) != hipSuccess ||
            hipHostMalloc((void**)&rt->sur_hy, (size_t)cap * sizeof(float)) != hipSuccess)
            return false;
        rt->sur_cap = cap;
    }
    std::memcpy(rt->sur_hx, feat.data(), feat.size() * sizeof(float));
    if (hipMemcpyAsync(rt->sur_x, rt->sur_hx, feat.size() * sizeof(float),
                       hipMemcpyHostToDevice, rt->sur_stream) != hipSuccess)
        return false;
    if (kernelet_mlp_forward(rt->sur_params, rt->sur_x, n, rt->sur_y, rt->sur_stream) != KL_OK)
        return false;
    if (hipMemcpyAsync(rt->sur_hy, rt->sur_y, n * sizeof(float), hipMemcpyDeviceToHost,
                       rt->sur_stream) != hipSuccess ||
        hipStreamSynchronize(rt->sur_stream) != hipSuccess)
        return false;
    for (uint32_t k = 0; k < n; ++k)
        if ((double)rt->sur_hy[k] > (*scores)[owner[k]]) {
            (*scores)[owner[k]] = (double)rt->sur_hy[k];
            (*ratios)[owner[k]] = cand[k];
        }
    rt->stats.surrogate_us_total +=
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    rt->stats.surrogate_candidates += n;
    return true;
}

// Choose the next co-schedule (FindCoSchedule) and bind it to lanes.
// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output i of the stream whose state starts at
// `seed` mixes the state after i + 1 steps of the golden-ratio increment.
static uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Code-object resources of kernel kt: resident workgroups per CU alone,
// VGPRs per lane and static LDS bytes per workgroup.
static kl_status kernel_resources(const KernelType& kt, int* nb, int* regs, int* lds) {
    if (kt.mfn) {
        KL_HIP(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(nb, kt.mfn, (int)kt.block, 0));
        KL_HIP(hipFuncGetAttribute(regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, kt.mfn));
        KL_HIP(hipFuncGetAttribute(lds, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, kt.mfn));
        return KL_OK;
    }
    hipFuncAttributes attr;
    KL_HIP(hipFuncGetAttributes(&attr, kt.fn));
    KL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, kt.fn, (int)kt.block, 0));
    *regs = attr.numRegs;
    *lds = (int)attr.sharedSizeBytes;
    return KL_OK;
}

// The model's IPC of a kernel alone at w waves per SIMD.
static double model_ipc(kl_runtime* rt, const kl_profile& p, int w) {
    KernelModel km = kernel_model(p, rt->cfg);
    double ipc = 0.0;
    chain_ipc(&km, &w, 1, rt->cfg.beta, rt->cfg.beta_lds, &ipc);
    return ipc;
}

// Launch `count` workgroups of job jid alone on lane 0 at dynamic LDS `dyn`
// and wait for them; *ms receives their time from the events the dispatch
// carries.
static kl_status timed_solo_slice(kl_runtime* rt, kl_job jid, uint32_t count, uint32_t dyn,
                                  double* ms) {
    Job& j = rt->jobs.at(jid);
    KernelType& kt = rt->kernels[j.type];
    Lane& ln = rt->lanes[0];
    const bool was_timed = kt.timed;
    const double t0 = kt.time_ms;
    const int64_t n0 = kt.time_launches, w0 = kt.time_wgs;
    kt.timed = true;
    ln.dyn_lds = dyn;
    kl_status s = launch_slice(rt, 0, jid, count, false);
    if (s == KL_OK && hipStreamSynchronize(ln.s[0]) != hipSuccess) {
        set_error("kernelet: a profiling slice failed on the device");
        s = KL_EHIP;
    }
    poll_lanes(rt);
    *ms = kt.time_ms - t0;
    kt.timed = was_timed;
    if (!was_timed) {
        kt.time_ms = t0;
        kt.time_launches = n0;
        kt.time_wgs = w0;
    }
    return s;
}

// Profile a kernel type from its job jid (Section 4.4 takes the model's
// inputs from a few thread blocks run ahead of the rest).  The job's first
// workgroups run alone on lane 0, timed by the events their dispatch
// carries: four rounds at the kernel's full occupancy, then, if it can be
// held there by LDS reservation, four rounds at two workgroups per CU; they
// are the job's own progress, so nothing runs twice.  Without hardware
// counters the memory-instruction ratio is the one whose two-state chain
// (memory latency cfg.mem_latency) reproduces the measured ratio of the
// two rates, the instructions per wave those that give the measured rate at
// full occupancy, PUR the model's solo IPC, and MUR unknown (-1: the pair
// is never pruned).  Occupancy, VGPRs and static LDS come from the code
// object.
static kl_status profile_by_preexecution(kl_runtime* rt, kl_job jid) {
    Job& j = rt->jobs.at(jid);
    KernelType& kt = rt->kernels[j.type];
    const int n_cu = rt->cfg.n_cu;
    int nb = 0, regs = 0, lds = 0;
    if (kl_status s = kernel_resources(kt, &nb, &regs, &lds)) return s;
    const int wps = std::max(1, (int)kt.block / 256);  // waves per SIMD per workgroup
    const int bmax = std::max(1, std::min(nb, rt->cfg.wmax / wps));
    // alone: wait for every lane to drain first
    for (auto& ln : rt->lanes)
        for (int b = 0; b < ln.nsub; ++b) KL_HIP(hipStreamSynchronize(ln.s[b]));
    poll_lanes(rt);
    const uint64_t rounds = 4;
    uint32_t sa = (uint32_t)std::min<uint64_t>(j.total - j.next, rounds * n_cu * bmax);
    double ta = 0.0;
    if (kl_status s = timed_solo_slice(rt, jid, sa, 0, &ta)) return s;
    kl_profile p{};
    p.waves_per_simd = wps;
    p.max_wg_per_cu = bmax;
    p.vgpr = regs;
    p.lds_bytes = lds;
    p.lat_mem = 0.0;  // the configuration's memory latency
    p.mem_req = 1.0;
    p.r_comp = 0.0;
    p.lat_comp = 1.0;
    p.instr_per_wave = 1.0;
    p.mur = -1.0;
    p.access = 0;
    p.comp_pool = 0;
    p.min_slice_wgs = 0;
    double rho = 0.0;  // rate at full occupancy over rate at two per CU
    const uint32_t dyn2 = bmax > 2 ? dyn_lds_for(rt, kt, 2, 0, 0, true) : 0;
    const uint64_t rem = j.total - j.next;
    if (dyn2 > 0 && rem >= (uint64_t)2 * n_cu) {
        const uint32_t sb = (uint32_t)std::min<uint64_t>(rem, rounds * n_cu * 2);
        double tb = 0.0;
        if (kl_status s = timed_solo_slice(rt, jid, sb, dyn2, &tb)) return s;
        if (ta > 0 && tb > 0) rho = ((double)sa / ta) / ((double)sb / tb);
    }
    const int wf = bmax * wps, wl = 2 * wps;
    p.r_mem = 0.01;  // no second point: a nominal ratio
    if (rho > 0) {
        const double hi_ratio = (double)wf / wl;
        const double target = std::min(std::max(rho, 1.0), hi_ratio);
        double lo = 1e-4, hi = 0.5;
        for (int it = 0; it < 40; ++it) {
            const double mid = 0.5 * (lo + hi);
            p.r_mem = mid;
            const double ratio = model_ipc(rt, p, wf) / model_ipc(rt, p, wl);
            if (ratio < target)
                lo = mid;
            else
                hi = mid;
        }
        p.r_mem = 0.5 * (lo + hi);
    }
    const double ipc = model_ipc(rt, p, wf);
    // workgroups per issue slot measured at full occupancy (an issue slot is
    // 4 cycles at 2.4 GHz, 600000 slots per millisecond)
    const double rate = ta > 0 ? (double)sa / ta / 600000.0 : 0.0;
    p.instr_per_wave = rate > 0 ? (double)n_cu * ipc / ((double)wps * rate) : 1.0;
    p.pur = std::min(ipc, 1.0);
    p.solo_ipc = ipc;
    if (kl_status s = check_profile(p)) return s;
    kt.prof = p;
    kt.has_prof = true;
    rt->planner->set_type(j.type, p);
    rt->stats.kernels_profiled++;
    return KL_OK;
}

static bool model_policy(kl_policy p) {
    return p == KL_POLICY_MARKOV || p == KL_POLICY_SURROGATE || p == KL_POLICY_OPT ||
           p == KL_POLICY_RANDOM;
}

static kl_status decide(kl_runtime* rt, kl_policy policy) {
    // kernels without a profile are profiled from their earliest runnable job
    if (model_policy(policy) && rt->cfg.auto_profile) {
        for (int t = 0; t < (int)rt->unlaunched_by_type.size(); ++t) {
            if (rt->kernels[t].has_prof) continue;
            for (kl_job id : rt->unlaunched_by_type[t]) {
                if (!runnable(rt->jobs.at(id))) continue;
                if (kl_status s = profile_by_preexecution(rt, id)) return s;
                break;
            }
        }
    }
    // FindCoSchedule's candidates are the earliest runnable jobs of each
    // kernel type (two per type when two instances of a kernel may pair):
    // collect those, not every pending job
    std::vector<PendingJob> pend;
    for (const auto& ids : rt->unlaunched_by_type) {
        int got = 0;
        for (kl_job id : ids) {
            const Job& j = rt->jobs.at(id);
            if (!runnable(j)) continue;
            pend.push_back({id, j.type, (double)(j.total - j.next)});
            if (++got == 2) break;
        }
    }
    rt->cs_active = false;
    rt->cs_job[0] = rt->cs_job[1] = rt->cs_job[2] = KL_NO_JOB;
    if (pend.empty()) {
        for (auto& ln : rt->lanes) ln.job = KL_NO_JOB;
        return KL_OK;
    }
    auto t0 = std::chrono::steady_clock::now();
    Decision d;
    if (policy == KL_POLICY_FIXED) {
        // the two earliest jobs of different kernel types, their own plans
        std::sort(pend.begin(), pend.end(),
                  [](const PendingJob& a, const PendingJob& b) { return a.id < b.id; });
        auto occ = [&](kl_job id) {
            const Job& j = rt->jobs.at(id);
            if (j.occ > 0) return j.occ;
            const KernelType& kt = rt->kernels[j.type];
            return kt.has_prof ? kt.prof.max_wg_per_cu : 8;
        };
        d.j1 = pend[0].id;
        d.b1 = occ(d.j1);
        for (auto& p : pend)
            if (p.type != pend[0].type) {
                d.j2 = p.id;
                d.b2 = occ(d.j2);
                break;
            }
    } else if (policy == KL_POLICY_SURROGATE) {
        d = rt->planner->find_ranked(
            pend, std::max(0, rt->cfg.surrogate_topk),
            [rt](const std::vector<std::pair<const kl_profile*, const kl_profile*>>& pp,
                 std::vector<double>* sc, std::vector<std::pair<int, int>>* rat) {
                return surrogate_scores(rt, pp, sc, rat);
            });
    } else if (policy == KL_POLICY_OPT) {
        d = rt->planner->find_opt(pend);
    } else if (policy == KL_POLICY_RANDOM) {
        const uint64_t k = rt->random_draws++;
        d = rt->planner->find_random(pend, splitmix64(rt->cfg.random_seed, 2 * k),
                                     splitmix64(rt->cfg.random_seed, 2 * k + 1));
    } else {
        d = rt->planner->find(pend);
    }
    double us = std::chrono::duration<double, std::micro>(
                    std::chrono::steady_clock::now() - t0).count();
    rt->stats.model_us_total = rt->planner->model_us;
    rt->stats.cache_hits = rt->planner->cache_hits;

    // one lane per kernel of the co-schedule; a kernel keeps the lane it
    // already runs on
    const int ng = d.j2 == KL_NO_JOB ? 1 : (d.j3 == KL_NO_JOB ? 2 : 3);
    const kl_job want[3] = {d.j1, ng > 1 ? d.j2 : KL_NO_JOB, ng > 2 ? d.j3 : KL_NO_JOB};
    const int bw[3] = {d.b1, d.b2, d.b3};
    int lane_of[3] = {-1, -1, -1};
    const int nl = std::min<int>((int)rt->lanes.size(), 3);
    auto taken = [&](int li) {
        return li == lane_of[0] || li == lane_of[1] || li == lane_of[2];
    };
    for (int k = 0; k < ng; ++k)
        for (int li = 0; li < nl; ++li)
            if (rt->lanes[li].job == want[k]) lane_of[k] = li;
    for (int k = 0; k < ng; ++k) {
        if (lane_of[k] >= 0) continue;
        int best = -1;
        for (int li = 0; li < nl; ++li) {
            if (taken(li)) continue;
            if (best < 0 || rt->lanes[li].inflight.size() < rt->lanes[best].inflight.size())
                best = li;
        }
        lane_of[k] = best;
    }
    for (int li = 0; li < (int)rt->lanes.size(); ++li)
        if (!taken(li)) rt->lanes[li].job = KL_NO_JOB;

    uint32_t sl[3] = {0, 0, 0};
    const bool solo = ng == 1 || lane_of[1] < 0;
    const KernelType* kts[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < ng; ++k) kts[k] = &rt->kernels[rt->jobs.at(want[k]).type];
    // the kernel capped by LDS reservation (mode 2): the largest register
    // footprint at its target occupancy (the first on ties)
    int capped = -1;
    if (!solo) {
        int64_t top = -1;
        for (int k = 0; k < ng; ++k) {
            const int64_t f = (int64_t)bw[k] * (kts[k]->has_prof ? kts[k]->prof.vgpr : 0);
            if (f > top) top = f, capped = k;
        }
    }
    for (int k = 0; k < ng; ++k) {
        if (lane_of[k] < 0) continue;
        Job& j = rt->jobs.at(want[k]);
        Lane& ln = rt->lanes[lane_of[k]];
        ln.job = want[k];
        const KernelType& kt = *kts[k];
        if (solo) {
            // a co-schedule of one kernel: its residual in one launch at full
            // occupancy; the other lanes wait for it before their next launch
            sl[k] = j.fixed_slice ? j.fixed_slice : j.total - j.next;
            // a requested occupancy below the kernel's own is held by LDS
            ln.dyn_lds = j.occ > 0 && rt->cfg.lds_reserve == 2
                             ? dyn_lds_for(rt, kt, j.occ, 0, 0, true)
                             : 0;
        } else {
            int b_others = 0;
            int64_t others_lds = 0;
            for (int o = 0; o < ng; ++o) {
                if (o == k) continue;
                b_others += bw[o];
                others_lds += (int64_t)bw[o] * kts[o]->static_lds;
            }
            sl[k] = slice_size(rt, j, bw[k]);
            ln.dyn_lds = dyn_lds_for(rt, kt, bw[k], b_others, others_lds, capped == k);
        }
        ln.slice = sl[k];
        rt->cs_job[k] = want[k];
    }
    rt->cs_active = true;
    log_decision(rt, d, sl, us);
    return KL_OK;
}

// Whether job j would finish alone within the pairing threshold (such a
// job runs alone only because it is too short to pair, and need not hold
// the other lanes back).
static bool too_short_to_pair(kl_runtime* rt, const Job& j) {
    const KernelType& kt = rt->kernels[j.type];
    if (rt->cfg.min_pair_slots <= 0 || !kt.has_prof) return false;
    const double rate = wg_rate(kt.prof, rt->planner->solo(j.type), rt->cfg.n_cu);
    return rate > 0 && (double)(j.total - j.next) / rate < rt->cfg.min_pair_slots;
}

// One step of Algorithm 1: decide if needed, then fill the lanes' queues.
static kl_status markov_step(kl_runtime* rt, kl_policy policy, bool* progressed) {
    bool ended = !rt->cs_active;
    for (int k = 0; k < 3 && !ended; ++k) {
        kl_job id = rt->cs_job[k];
        if (id == KL_NO_JOB) continue;
        auto it = rt->jobs.find(id);
        if (it == rt->jobs.end() || it->second.next >= it->second.total ||
            it->second.st == J_CANCELED)
            ended = true;
    }
    if (ended) {
        if (kl_status s = decide(rt, policy)) return s;
        if (!rt->cs_active) return KL_OK;
        *progressed = true;
    }
    const bool solo = rt->cs_job[1] == KL_NO_JOB;
    for (int li = 0; li < (int)rt->lanes.size(); ++li) {
        Lane& ln = rt->lanes[li];
        if (ln.job == KL_NO_JOB) continue;
        Job& j = rt->jobs.at(ln.job);
        const bool hold_others = solo && !rt->cfg.solo_overlap &&
                                 !(j.next == 0 && too_short_to_pair(rt, j));
        while (lane_has_room(rt, ln) && j.next < j.total) {
            kl_status s = launch_slice(rt, li, j.id, ln.slice, true);
            if (s) return s;
            *progressed = true;
            if (hold_others && j.next >= j.total) {
                // later launches on the other lanes start after this run
                std::vector<int> tails;
                tails_of(j, &tails);
                for (int o = 0; o < (int)rt->lanes.size(); ++o) {
                    if (o == li) continue;
                    for (int e : tails) {
                        rt->lanes[o].barrier.push_back(e);
                        rt->pool.ref(e);
                    }
                }
            }
        }
        if (j.next >= j.total) {
            ln.job = KL_NO_JOB;
            rt->cs_active = false;  // one kernel ran out: decide again
        }
    }
    return KL_OK;
}

static bool all_launched(kl_runtime* rt) { return rt->unlaunched.empty(); }

static bool any_inflight(kl_runtime* rt) {
    for (auto& ln : rt->lanes)
        if (!ln.inflight.empty()) return true;
    return false;
}

// The dispatcher loop.  Blocking: until every job is launched.  Worker:
// until stop.
// Short waits of the dispatcher sleep for the time asked, not for the
// kernel's default timer slack (50 us), which would add that much to every
// slice a lane retires; restored on exit.
struct TimerSlack {
    int prev;
    TimerSlack() : prev(prctl(PR_GET_TIMERSLACK, 0, 0, 0, 0)) {
        prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
    }
    ~TimerSlack() {
        if (prev > 0) prctl(PR_SET_TIMERSLACK, (unsigned long)prev, 0, 0, 0);
    }
};

static kl_status dispatch(kl_runtime* rt, kl_policy policy, bool blocking,
                          bool wait_done) {
    TimerSlack slack;
    std::unique_lock<std::mutex> lk(rt->mu);
    rt->scheduling = true;
    rt->cs_active = false;
    kl_status st = KL_OK;
    while (!rt->stop.load()) {
        poll_lanes(rt);
        admit(rt);
        bool progressed = false;
        st = policy == KL_POLICY_FIFO         ? fifo_step(rt, &progressed)
             : policy == KL_POLICY_CONCURRENT ? concurrent_step(rt, &progressed)
                                              : markov_step(rt, policy, &progressed);
        if (st) break;
        if (progressed) {
            rt->cv.notify_all();
            continue;
        }
        if (blocking && all_launched(rt) && (!wait_done || !any_inflight(rt))) break;
        const bool waiting_budget = !rt->unadmitted.empty();
        if (blocking && !any_inflight(rt) && !waiting_budget) {
            // nothing in flight and nothing runnable: jobs wait on deps that
            // can never be released (e.g. a cancelled predecessor)
            bool runnable_any = false;
            for (kl_job id : rt->unlaunched) runnable_any |= runnable(rt->jobs.at(id));
            if (!runnable_any) {
                set_error("kernelet_schedule: jobs wait on dependencies that cannot finish");
                st = KL_ESTATE;
                break;
            }
        }
        // nothing to do now: wait for a slice to finish or a submission
        wait_us(rt->cv, lk, any_inflight(rt) ? 5 : 200);
    }
    poll_lanes(rt);
    rt->scheduling = false;
    rt->cv.notify_all();
    return st;
}


// ------------------------------------------------------------- submission
// Checks of one launch submitted by the caller (runtime lock held).
static kl_status check_submit(kl_runtime* rt, kl_kernel k, kl_dim3 grid, const void* args,
                              uint32_t args_bytes, uint64_t footprint, const char* fn) {
    const std::string f(fn);
    if (k < 0 || k >= (int)rt->kernels.size()) {
        set_error(f + ": unknown kernel");
        return KL_ENOTFOUND;
    }
    const KernelType& kt = rt->kernels[k];
    if (args_bytes != kt.args_bytes) {
        set_error(f + ": args_bytes differs from the registered size");
        return KL_EINVAL;
    }
    uint64_t total = (uint64_t)grid.x * grid.y * grid.z;
    if (total == 0 || total > 0xffffffffull) {
        set_error(f + ": grid must hold 1 .. 2^32-1 workgroups");
        return KL_EINVAL;
    }
    if (kt.builtin) {
        kl_dim3 need;
        std::string err;
        if (!builtin_check(kt.builtin, args, args_bytes, &need, &err)) {
            set_error(f + "(" + kt.builtin + "): " + err);
            return KL_EINVAL;
        }
        if (need.x != grid.x || need.y != grid.y || need.z != grid.z) {
            set_error(f + "(" + kt.builtin + "): grid differs from the grid the arguments need");
            return KL_EINVAL;
        }
    }
    if (rt->cfg.hbm_budget > 0 && (int64_t)footprint > rt->cfg.hbm_budget) {
        set_error(f + ": footprint exceeds the whole memory budget");
        return KL_ENOMEM;
    }
    return KL_OK;
}

static kl_status check_after(kl_runtime* rt, kl_job after, const char* fn) {
    if (after == KL_NO_JOB) return KL_OK;
    auto it = rt->jobs.find(after);
    if (it == rt->jobs.end()) {
        set_error(std::string(fn) + ": unknown `after` job");
        return KL_ENOTFOUND;
    }
    if (it->second.st == J_CANCELED) {
        set_error(std::string(fn) + ": `after` job was cancelled");
        return KL_ECANCELED;
    }
    return KL_OK;
}

// Create a checked job (runtime lock held); returns its id.
static kl_job add_job(kl_runtime* rt, kl_kernel k, kl_dim3 grid, const void* args,
                      uint32_t args_bytes, kl_job after, uint32_t client, uint64_t footprint) {
    Job j;
    j.id = rt->next_id++;
    j.type = k;
    j.grid = grid;
    j.total = (uint32_t)((uint64_t)grid.x * grid.y * grid.z);
    j.args.assign((const uint8_t*)args, (const uint8_t*)args + args_bytes);
    j.client = client;
    j.footprint = footprint;
    j.t_submit = now_ns();
    j.after = after;
    j.st = J_PENDING;
    if (after != KL_NO_JOB) {
        Job& p = rt->jobs.at(after);
        if (p.st == J_WAIT_DEP || p.st == J_PENDING) j.st = J_WAIT_DEP;
        if (p.st != J_DONE) p.dependents.push_back(j.id);
    }
    const kl_job id = j.id;
    rt->live.insert(id);
    rt->unlaunched.insert(id);
    if ((int)rt->unlaunched_by_type.size() <= k) rt->unlaunched_by_type.resize(k + 1);
    rt->unlaunched_by_type[k].insert(id);
    rt->unadmitted.insert(id);
    rt->jobs.emplace(id, std::move(j));
    rt->stats.jobs_submitted++;
    return id;
}

}  // namespace kl

using namespace kl;

// ================================================================= C ABI
extern "C" {

const char* kernelet_last_error(void) { return g_err.c_str(); }

kl_status kernelet_default_config(kl_config* cfg) {
    if (!cfg) {
        set_error("null cfg");
        return KL_EINVAL;
    }
    *cfg = defaults();
    return KL_OK;
}

kl_status kernelet_init(kl_runtime** out, int hip_device, const kl_config* cfg) {
    if (!out) {
        set_error("kernelet_init: null out");
        return KL_EINVAL;
    }
    *out = nullptr;
    kl_config c = cfg ? *cfg : defaults();
    if (kl_status s = check_cfg(c)) return s;
    if (c.group_max == 3 && c.lanes < 3) {
        set_error("kernelet_init: group_max 3 needs lanes >= 3 (one stream per kernel)");
        return KL_EINVAL;
    }
    int ndev = 0;
    KL_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev) {
        set_error("kernelet_init: no such HIP device");
        return KL_EINVAL;
    }
    KL_HIP(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    KL_HIP(hipGetDeviceProperties(&prop, hip_device));
    if (c.n_cu == 0) c.n_cu = prop.multiProcessorCount;
    auto rt = std::make_unique<kl_runtime>();
    rt->device = hip_device;
    rt->cfg = c;
    rt->planner = std::make_unique<Planner>(c);
    rt->lanes.resize(c.lanes);
    for (auto& ln : rt->lanes) {
        ln.nsub = rt->cfg.lane_streams;
        for (int b = 0; b < ln.nsub; ++b)
            KL_HIP(hipStreamCreateWithFlags(&ln.s[b], hipStreamNonBlocking));
    }
    *out = rt.release();
    return KL_OK;
}

kl_status kernelet_get_config(kl_runtime* rt, kl_config* cfg) {
    if (!rt || !cfg) {
        set_error("kernelet_get_config: null argument");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    *cfg = rt->cfg;
    return KL_OK;
}

kl_status kernelet_shutdown(kl_runtime* rt) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    rt->stop = true;
    rt->cv.notify_all();
    if (rt->worker.joinable()) rt->worker.join();
    (void)hipSetDevice(rt->device);
    for (auto& ln : rt->lanes) {
        for (hipStream_t x : ln.s)
            if (x) (void)hipStreamSynchronize(x);
    }
    for (auto& ln : rt->lanes)
        for (hipStream_t x : ln.s)
            if (x) (void)hipStreamDestroy(x);
    for (auto& ln : rt->lanes)
        for (auto& f : ln.inflight)
            if (f.start) (void)hipEventDestroy(f.start);
    rt->pool.destroy();
    for (auto e : rt->tev_free) (void)hipEventDestroy(e);
    if (rt->sur_stream) (void)hipStreamDestroy(rt->sur_stream);
    for (auto& k : rt->kernels)
        if (k.mod) (void)hipModuleUnload(k.mod);
    (void)hipFree(rt->sur_params);
    (void)hipFree(rt->sur_x);
    (void)hipFree(rt->sur_y);
    (void)hipHostFree(rt->sur_hx);
    (void)hipHostFree(rt->sur_hy);
    delete rt;
    return KL_OK;
}

// Checks shared by the two ways of registering a kernel.
static kl_status check_desc(kl_runtime* rt, const kl_kernel_desc* d, const char* who) {
    if (d->block_threads == 0 || d->block_threads % 256 || d->block_threads > 1024 ||
        d->args_bytes == 0 || d->args_bytes > 256) {
        set_error(std::string(who) + ": block_threads must be 256, 512, 768 or 1024 and "
                  "args_bytes in [1, 256]");
        return KL_EINVAL;
    }
    if (d->profile) {
        if (kl_status s = check_profile(*d->profile)) return s;
    }
    for (auto& k : rt->kernels)
        if (k.name == d->name) {
            set_error(std::string(who) + ": duplicate name " + d->name);
            return KL_EEXIST;
        }
    return KL_OK;
}

kl_status kernelet_register_image(kl_runtime* rt, const kl_kernel_desc* d, const void* image,
                                  uint64_t bytes, const char* symbol, kl_kernel* out) {
    if (!rt || !d || !out || !d->name || !image || bytes == 0 || !symbol) {
        set_error("kernelet_register_image: null argument");
        return KL_EINVAL;
    }
    if (d->host_fn) {
        set_error("kernelet_register_image: the descriptor's host_fn must be NULL");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    if (kl_status s = check_desc(rt, d, "kernelet_register_image")) return s;
    KL_HIP(hipSetDevice(rt->device));
    // the loader reads the image during the call; a copy keeps it aligned
    std::vector<uint64_t> img((bytes + 7) / 8);
    std::memcpy(img.data(), image, bytes);
    KernelType kt;
    KL_HIP(hipModuleLoadData(&kt.mod, img.data()));
    if (hipModuleGetFunction(&kt.mfn, kt.mod, symbol) != hipSuccess) {
        (void)hipModuleUnload(kt.mod);
        set_error(std::string("kernelet_register_image: no kernel ") + symbol + " in the image");
        return KL_EHIP;
    }
    int lds = 0;
    if (hipFuncGetAttribute(&lds, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, kt.mfn) == hipSuccess)
        kt.static_lds = lds;
    kt.name = d->name;
    kt.block = d->block_threads;
    kt.args_bytes = d->args_bytes;
    kt.flags = d->flags;
    if (d->profile) {
        kt.prof = *d->profile;
        kt.has_prof = true;
        rt->planner->set_type((int)rt->kernels.size(), kt.prof);
    }
    rt->kernels.push_back(kt);
    *out = (kl_kernel)(rt->kernels.size() - 1);
    return KL_OK;
}

kl_status kernelet_register(kl_runtime* rt, const kl_kernel_desc* d, kl_kernel* out) {
    if (!rt || !d || !out || !d->name || !d->host_fn) {
        set_error("kernelet_register: null argument");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    if (kl_status s = check_desc(rt, d, "kernelet_register")) return s;
    KernelType kt;
    kt.name = d->name;
    kt.fn = d->host_fn;
    kt.block = d->block_threads;
    kt.args_bytes = d->args_bytes;
    kt.flags = d->flags;
    const char* bn = nullptr;
    if (is_builtin_fn(d->host_fn, &bn)) kt.builtin = bn;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, d->host_fn) == hipSuccess)
        kt.static_lds = (int)attr.sharedSizeBytes;
    if (d->profile) {
        kt.prof = *d->profile;
        kt.has_prof = true;
        rt->planner->set_type((int)rt->kernels.size(), kt.prof);
    }
    rt->kernels.push_back(kt);
    *out = (kl_kernel)(rt->kernels.size() - 1);
    return KL_OK;
}

kl_status kernelet_kernel_info(kl_runtime* rt, kl_kernel k, int32_t* max_wg_per_cu,
                               int32_t* vgpr, int32_t* lds_bytes) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    const void* fn;
    hipFunction_t mfn;
    uint32_t block;
    {
        std::lock_guard<std::mutex> g(rt->mu);
        if (k < 0 || k >= (int)rt->kernels.size()) {
            set_error("kernelet_kernel_info: unknown kernel");
            return KL_ENOTFOUND;
        }
        fn = rt->kernels[k].fn;
        mfn = rt->kernels[k].mfn;
        block = rt->kernels[k].block;
    }
    KL_HIP(hipSetDevice(rt->device));
    if (mfn) {
        int nb = 0, regs = 0, lds = 0;
        KL_HIP(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mfn, (int)block, 0));
        KL_HIP(hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, mfn));
        KL_HIP(hipFuncGetAttribute(&lds, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, mfn));
        if (max_wg_per_cu) *max_wg_per_cu = nb;
        if (vgpr) *vgpr = regs;
        if (lds_bytes) *lds_bytes = lds;
        return KL_OK;
    }
    hipFuncAttributes attr;
    KL_HIP(hipFuncGetAttributes(&attr, fn));
    int nb = 0;
    KL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)block, 0));
    if (max_wg_per_cu) *max_wg_per_cu = nb;
    if (vgpr) *vgpr = attr.numRegs;
    if (lds_bytes) *lds_bytes = (int32_t)attr.sharedSizeBytes;
    return KL_OK;
}

kl_status kernelet_profile_from_counters(const kl_counters* c, kl_profile* out) {
    if (!c || !out) {
        set_error("kernelet_profile_from_counters: null argument");
        return KL_EINVAL;
    }
    if (!profile_from_counters(*c, out)) {
        set_error("kernelet_profile_from_counters: invalid counts, time, clock, bandwidth or "
                  "CU count");
        return KL_EINVAL;
    }
    return KL_OK;
}

kl_status kernelet_set_profile(kl_runtime* rt, kl_kernel k, const kl_profile* p) {
    if (!rt || !p) {
        set_error("kernelet_set_profile: null argument");
        return KL_EINVAL;
    }
    if (kl_status s = check_profile(*p)) return s;
    std::lock_guard<std::mutex> g(rt->mu);
    if (k < 0 || k >= (int)rt->kernels.size()) {
        set_error("kernelet_set_profile: unknown kernel");
        return KL_ENOTFOUND;
    }
    rt->kernels[k].prof = *p;
    rt->kernels[k].has_prof = true;
    rt->planner->set_type(k, *p);
    return KL_OK;
}

kl_status kernelet_get_profile(kl_runtime* rt, kl_kernel k, kl_profile* p) {
    if (!rt || !p) {
        set_error("kernelet_get_profile: null argument");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    if (k < 0 || k >= (int)rt->kernels.size() || !rt->kernels[k].has_prof) {
        set_error("kernelet_get_profile: unknown kernel or no profile");
        return KL_ENOTFOUND;
    }
    *p = rt->kernels[k].prof;
    return KL_OK;
}

kl_status kernelet_submit(kl_runtime* rt, kl_kernel k, kl_dim3 grid, const void* args,
                          uint32_t args_bytes, kl_job after, uint32_t client,
                          uint64_t footprint, kl_job* out) {
    if (!rt || !args || !out) {
        set_error("kernelet_submit: null argument");
        return KL_EINVAL;
    }
    std::unique_lock<std::mutex> lk(rt->mu);
    if (kl_status s = check_submit(rt, k, grid, args, args_bytes, footprint, "kernelet_submit"))
        return s;
    if (kl_status s = check_after(rt, after, "kernelet_submit")) return s;
    *out = add_job(rt, k, grid, args, args_bytes, after, client, footprint);
    lk.unlock();
    rt->cv.notify_all();
    return KL_OK;
}

kl_status kernelet_submit_chain(kl_runtime* rt, uint32_t n, const kl_kernel* k,
                                const kl_dim3* grid, const void* const* args,
                                const uint32_t* args_bytes, kl_job after, uint32_t client,
                                uint64_t footprint, kl_job* out) {
    if (!rt || n == 0 || !k || !grid || !args || !args_bytes || !out) {
        set_error("kernelet_submit_chain: null argument or empty chain");
        return KL_EINVAL;
    }
    std::unique_lock<std::mutex> lk(rt->mu);
    for (uint32_t i = 0; i < n; ++i) {
        if (!args[i]) {
            set_error("kernelet_submit_chain: null argument block");
            return KL_EINVAL;
        }
        if (kl_status s = check_submit(rt, k[i], grid[i], args[i], args_bytes[i],
                                       i == 0 ? footprint : 0, "kernelet_submit_chain"))
            return s;
    }
    if (kl_status s = check_after(rt, after, "kernelet_submit_chain")) return s;
    // every launch exists before the dispatcher (which needs this lock) can
    // start the first, so the footprint always travels to the last one
    kl_job prev = after;
    for (uint32_t i = 0; i < n; ++i) {
        prev = add_job(rt, k[i], grid[i], args[i], args_bytes[i], prev, client,
                       i == 0 ? footprint : 0);
        out[i] = prev;
    }
    lk.unlock();
    rt->cv.notify_all();
    return KL_OK;
}

kl_status kernelet_slice(kl_runtime* rt, kl_job jid, uint32_t wgs, uint32_t* n_slices) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    auto it = rt->jobs.find(jid);
    if (it == rt->jobs.end()) {
        set_error("kernelet_slice: unknown job");
        return KL_ENOTFOUND;
    }
    Job& j = it->second;
    if (j.next > 0 || j.st == J_LAUNCHED || j.st == J_DONE || j.st == J_CANCELED) {
        set_error("kernelet_slice: job already started");
        return KL_ESTATE;
    }
    if (wgs == 0) {
        const KernelType& kt = rt->kernels[j.type];
        wgs = kt.has_prof && kt.prof.min_slice_wgs > 0 ? (uint32_t)kt.prof.min_slice_wgs
                                                        : j.total;
    }
    j.fixed_slice = std::min(wgs, j.total);
    if (n_slices) *n_slices = (j.total + j.fixed_slice - 1) / j.fixed_slice;
    return KL_OK;
}

kl_status kernelet_job_occupancy(kl_runtime* rt, kl_job jid, int32_t wg_per_cu) {
    if (!rt || wg_per_cu < 1 || wg_per_cu > 64) {
        set_error("kernelet_job_occupancy: null runtime or occupancy outside [1, 64]");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    auto it = rt->jobs.find(jid);
    if (it == rt->jobs.end()) {
        set_error("kernelet_job_occupancy: unknown job");
        return KL_ENOTFOUND;
    }
    Job& j = it->second;
    if (j.next > 0 || j.st == J_LAUNCHED || j.st == J_DONE || j.st == J_CANCELED) {
        set_error("kernelet_job_occupancy: job already started");
        return KL_ESTATE;
    }
    j.occ = wg_per_cu;
    return KL_OK;
}

kl_status kernelet_schedule(kl_runtime* rt, kl_policy policy, uint32_t flags) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    if (policy < KL_POLICY_FIFO || policy > KL_POLICY_CONCURRENT) {
        set_error("kernelet_schedule: unknown policy");
        return KL_EINVAL;
    }
    {
        std::lock_guard<std::mutex> g(rt->mu);
        if (rt->scheduling || rt->worker_running) {
            set_error("kernelet_schedule: a scheduler is already running");
            return KL_ESTATE;
        }
        if (policy == KL_POLICY_SURROGATE && !rt->sur_params) {
            set_error("kernelet_schedule: the surrogate policy needs kernelet_set_surrogate");
            return KL_ESTATE;
        }
        if (policy == KL_POLICY_OPT && !rt->have_measures) {
            set_error("kernelet_schedule: the OPT policy needs kernelet_set_pair_measures");
            return KL_ESTATE;
        }
        if (policy != KL_POLICY_FIFO && policy != KL_POLICY_FIXED &&
            policy != KL_POLICY_CONCURRENT && !rt->cfg.auto_profile) {
            for (kl_job id : rt->live) {
                const Job& j = rt->jobs.at(id);
                if ((j.st == J_PENDING || j.st == J_WAIT_DEP) && !rt->kernels[j.type].has_prof) {
                    set_error("kernelet_schedule: kernel " + rt->kernels[j.type].name +
                              " has no profile");
                    return KL_ESTATE;
                }
            }
        }
        rt->scheduling = true;  // reserve against a concurrent call
    }
    KL_HIP(hipSetDevice(rt->device));
    if (flags & KL_BLOCKING) {
        {
            std::lock_guard<std::mutex> g(rt->mu);
            rt->scheduling = false;
        }
        return dispatch(rt, policy, true, (flags & KL_WAIT_DONE) != 0);
    }
    std::lock_guard<std::mutex> g(rt->mu);
    rt->scheduling = false;
    rt->worker_running = true;
    rt->worker_policy = policy;
    rt->worker_flags = flags;
    rt->worker = std::thread([rt, policy]() {
        (void)hipSetDevice(rt->device);
        dispatch(rt, policy, false, false);
    });
    return KL_OK;
}

kl_status kernelet_wait(kl_runtime* rt, kl_job jid, int64_t timeout_ns) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    const int64_t deadline = timeout_ns < 0 ? INT64_MAX : now_ns() + timeout_ns;
    std::unique_lock<std::mutex> lk(rt->mu);
    for (;;) {
        auto it = rt->jobs.find(jid);
        if (it == rt->jobs.end()) {
            set_error("kernelet_wait: unknown job");
            return KL_ENOTFOUND;
        }
        Job& j = it->second;
        if (j.st == J_CANCELED) {
            set_error("kernelet_wait: the job was cancelled");
            return KL_ECANCELED;
        }
        if (j.st == J_DONE) {
            if (j.error) {
                set_error("kernelet_wait: a slice of the job failed on the device");
                return KL_EHIP;
            }
            return KL_OK;
        }
        bool failed = false;
        if (j.st == J_LAUNCHED && tails_done(rt, j, &failed)) {
            mark_done(rt, j, failed || j.error);
            release_tails(rt, j);
            continue;
        }
        if (now_ns() >= deadline) {
            set_error("kernelet_wait: timed out");
            return KL_ETIMEOUT;
        }
        wait_us(rt->cv, lk, 20);
    }
}

kl_status kernelet_synchronize(kl_runtime* rt) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    KL_HIP(hipSetDevice(rt->device));
    for (auto& ln : rt->lanes)
        for (int b = 0; b < ln.nsub; ++b) KL_HIP(hipStreamSynchronize(ln.s[b]));
    std::lock_guard<std::mutex> g(rt->mu);
    poll_lanes(rt);
    // a scheduler thread may have launched more slices since the streams
    // drained: a job is done only when its own latest slices are
    const std::vector<kl_job> ids(rt->live.begin(), rt->live.end());
    for (kl_job id : ids) {
        Job& j = rt->jobs.at(id);
        bool failed = false;
        if (j.st == J_LAUNCHED && tails_done(rt, j, &failed)) {
            mark_done(rt, j, failed || j.error);
            release_tails(rt, j);
        }
    }
    return KL_OK;
}

kl_status kernelet_stream_barrier(kl_runtime* rt, void* stream) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    KL_HIP(hipSetDevice(rt->device));
    int e = rt->pool.get();
    if (e < 0) {
        set_error("hipEventCreate failed");
        return KL_EHIP;
    }
    // each wait takes the event as recorded now; the pool may reuse it later
    hipError_t r = hipEventRecord(rt->pool.ev[e], (hipStream_t)stream);
    for (size_t i = 0; r == hipSuccess && i < rt->lanes.size(); ++i)
        for (int b = 0; r == hipSuccess && b < rt->lanes[i].nsub; ++b)
            r = hipStreamWaitEvent(rt->lanes[i].s[b], rt->pool.ev[e], 0);
    rt->pool.unref(e);
    if (r != hipSuccess) {
        set_error(std::string("kernelet_stream_barrier: ") + hipGetErrorString(r));
        return KL_EHIP;
    }
    return KL_OK;
}

kl_status kernelet_cancel(kl_runtime* rt, kl_job jid) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    auto it = rt->jobs.find(jid);
    if (it == rt->jobs.end()) {
        set_error("kernelet_cancel: unknown job");
        return KL_ENOTFOUND;
    }
    Job& j = it->second;
    if (j.next > 0 || j.st == J_LAUNCHED || j.st == J_DONE) {
        set_error("kernelet_cancel: job already started");
        return KL_ESTATE;
    }
    if (j.admitted) rt->resident -= (int64_t)j.footprint;
    rt->resident -= j.carry;
    j.carry = 0;
    j.admitted = false;
    j.st = J_CANCELED;
    forget_job(rt, j);
    // dependants can never run: cancel them too
    std::vector<kl_job> todo = j.dependents;
    while (!todo.empty()) {
        kl_job d = todo.back();
        todo.pop_back();
        auto dt = rt->jobs.find(d);
        if (dt == rt->jobs.end() || dt->second.st == J_CANCELED) continue;
        if (dt->second.admitted) rt->resident -= (int64_t)dt->second.footprint;
        rt->resident -= dt->second.carry;
        dt->second.carry = 0;
        dt->second.admitted = false;
        dt->second.st = J_CANCELED;
        forget_job(rt, dt->second);
        for (kl_job x : dt->second.dependents) todo.push_back(x);
    }
    rt->cv.notify_all();
    return KL_OK;
}

kl_status kernelet_job_times(kl_runtime* rt, kl_job jid, int64_t* ts, int64_t* tb,
                             int64_t* td) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    auto it = rt->jobs.find(jid);
    if (it == rt->jobs.end()) {
        set_error("kernelet_job_times: unknown job");
        return KL_ENOTFOUND;
    }
    if (ts) *ts = it->second.t_submit;
    if (tb) *tb = it->second.t_start;
    if (td) *td = it->second.t_done;
    return KL_OK;
}

kl_status kernelet_reap(kl_runtime* rt) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    for (auto it = rt->jobs.begin(); it != rt->jobs.end();) {
        Job& j = it->second;
        if (j.st == J_DONE || j.st == J_CANCELED) {
            release_tails(rt, j);
            it = rt->jobs.erase(it);
        } else {
            ++it;
        }
    }
    return KL_OK;
}

kl_status kernelet_time_kernel(kl_runtime* rt, kl_kernel k, int32_t enable) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    if (k < 0 || k >= (int)rt->kernels.size()) {
        set_error("kernelet_time_kernel: unknown kernel");
        return KL_ENOTFOUND;
    }
    KernelType& kt = rt->kernels[k];
    kt.timed = enable != 0;
    if (kt.timed) {
        kt.time_ms = 0;
        kt.time_launches = 0;
        kt.time_wgs = 0;
    }
    return KL_OK;
}

kl_status kernelet_kernel_time(kl_runtime* rt, kl_kernel k, double* total_ms,
                               int64_t* launches, int64_t* workgroups) {
    if (!rt) {
        set_error("null runtime");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    if (k < 0 || k >= (int)rt->kernels.size()) {
        set_error("kernelet_kernel_time: unknown kernel");
        return KL_ENOTFOUND;
    }
    (void)hipSetDevice(rt->device);
    poll_lanes(rt);
    const KernelType& kt = rt->kernels[k];
    if (total_ms) *total_ms = kt.time_ms;
    if (launches) *launches = kt.time_launches;
    if (workgroups) *workgroups = kt.time_wgs;
    return KL_OK;
}

kl_status kernelet_stats(kl_runtime* rt, kl_stats* out) {
    if (!rt || !out) {
        set_error("null argument");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    *out = rt->stats;
    out->surrogate_pairs = rt->planner->scored_pairs;
    out->model_solves = rt->planner->model_solves;
    out->resident_bytes = rt->resident;
    out->resident_peak = rt->resident_peak;
    return KL_OK;
}

kl_status kernelet_set_surrogate(kl_runtime* rt, const float* params, uint32_t n_params) {
    if (!rt || !params) {
        set_error("kernelet_set_surrogate: null argument");
        return KL_EINVAL;
    }
    if (n_params != KL_MLP_PARAMS) {
        set_error("kernelet_set_surrogate: the network has KL_MLP_PARAMS parameters");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    KL_HIP(hipSetDevice(rt->device));
    if (!rt->sur_stream) KL_HIP(hipStreamCreateWithFlags(&rt->sur_stream, hipStreamNonBlocking));
    if (!rt->sur_params)
        KL_HIP(hipMalloc((void**)&rt->sur_params, KL_MLP_PARAMS * sizeof(float)));
    KL_HIP(hipMemcpyAsync(rt->sur_params, params, KL_MLP_PARAMS * sizeof(float),
                          hipMemcpyHostToDevice, rt->sur_stream));
    KL_HIP(hipStreamSynchronize(rt->sur_stream));
    rt->planner->clear_scores();
    return KL_OK;
}

// Measured co-runs by ordered type pair, each row in both orders; false
// (with the error set) for a row naming no type, one type twice, a ratio
// outside 1..8 or a rate that is not positive.
static bool measure_map(const kl_pair_measure* rows, uint32_t n, int ntypes, const char* who,
                        std::map<std::pair<int, int>, std::vector<Measure>>* out) {
    out->clear();
    for (uint32_t i = 0; i < n; ++i) {
        const kl_pair_measure& r = rows[i];
        if (r.a < 0 || r.b < 0 || r.a >= ntypes || r.b >= ntypes || r.a == r.b ||
            r.b1 < 1 || r.b1 > 8 || r.b2 < 1 || r.b2 > 8 || !(r.rel_a > 0) || !(r.rel_b > 0) ||
            !std::isfinite(r.rel_a) || !std::isfinite(r.rel_b)) {
            set_error(std::string(who) + ": bad measure row " + std::to_string(i));
            return false;
        }
        (*out)[{r.a, r.b}].push_back({r.b1, r.b2, r.rel_a, r.rel_b});
        (*out)[{r.b, r.a}].push_back({r.b2, r.b1, r.rel_b, r.rel_a});
    }
    return true;
}

kl_status kernelet_set_pair_measures(kl_runtime* rt, const kl_pair_measure* rows, uint32_t n) {
    if (!rt || (n > 0 && !rows)) {
        set_error("kernelet_set_pair_measures: null argument");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    std::map<std::pair<int, int>, std::vector<Measure>> m;
    if (!measure_map(rows, n, (int)rt->kernels.size(), "kernelet_set_pair_measures", &m))
        return KL_EINVAL;
    rt->planner->set_measures(m);
    rt->have_measures = true;
    return KL_OK;
}

kl_status kernelet_surrogate_features(const kl_config* cfg, const kl_profile* a,
                                      const kl_profile* b, int32_t b1, int32_t b2,
                                      float* out16) {
    if (!a || !b || !out16) {
        set_error("kernelet_surrogate_features: null argument");
        return KL_EINVAL;
    }
    const kl_config c = cfg ? *cfg : defaults();
    if (kl_status s = check_profile(*a)) return s;
    if (kl_status s = check_profile(*b)) return s;
    if (!ratio_feasible(*a, *b, c, b1, b2)) {
        set_error("kernelet_surrogate_features: the ratio does not fit on one CU");
        return KL_EINVAL;
    }
    surrogate_features(*a, b1, c.wmax, out16);
    surrogate_features(*b, b2, c.wmax, out16 + 8);
    return KL_OK;
}

kl_status kernelet_decisions(kl_runtime* rt, kl_decision* out, int32_t max, int32_t* n) {
    if (!rt || !n || (max > 0 && !out)) {
        set_error("null argument");
        return KL_EINVAL;
    }
    std::lock_guard<std::mutex> g(rt->mu);
    int32_t c = std::min<int32_t>(max, (int32_t)rt->declog.size());
    for (int32_t i = 0; i < c; ++i) out[i] = rt->declog[i];
    *n = c;
    rt->declog.clear();
    return KL_OK;
}

// ------------------------------------------------------------ host model
kl_status kernelet_predict(const kl_config* cfg, const kl_profile* p1, const kl_profile* p2,
                           int32_t w1, int32_t w2, double* ipc1, double* ipc2, double* cp) {
    if (!p1 || (w2 > 0 && !p2) || w1 < 0 || w2 < 0 || w1 + w2 < 1 || w1 > 16 || w2 > 16) {
        set_error("kernelet_predict: bad profile or wave counts");
        return KL_EINVAL;
    }
    kl_config c = cfg ? *cfg : defaults();
    if (kl_status s = check_cfg(c)) return s;
    if (kl_status s = check_profile(*p1)) return s;
    if (p2)
        if (kl_status s = check_profile(*p2)) return s;
    {
        KernelModel km[2] = {kernel_model(*p1, c), p2 ? kernel_model(*p2, c) : KernelModel{}};
        int w[2] = {w1, w2};
        const int n = w2 > 0 ? 2 : 1;
        if (w1 == 0) km[0] = km[1], w[0] = w2;
        if (chain_states(km, w, n) > kMaxChainStates) {
            set_error("kernelet_predict: the chain of these wave counts is too large");
            return KL_EINVAL;
        }
    }
    double out[2] = {0, 0};
    if (w2 == 0 || w1 == 0) {
        const kl_profile& p = w1 ? *p1 : *p2;
        int w = w1 ? w1 : w2;
        KernelModel km = kernel_model(p, c);
        double v;
        chain_ipc(&km, &w, 1, c.beta, c.beta_lds, &v);
        out[w1 ? 0 : 1] = v;
    } else {
        KernelModel km[2] = {kernel_model(*p1, c), kernel_model(*p2, c)};
        int w[2] = {w1, w2};
        chain_ipc(km, w, 2, c.beta, c.beta_lds, out);
    }
    if (ipc1) *ipc1 = out[0];
    if (ipc2) *ipc2 = out[1];
    if (cp) {
        double solo[2] = {solo_ipc(*p1, c), p2 ? solo_ipc(*p2, c) : 1.0};
        int n = 0;
        double ci[2], si[2];
        if (w1 > 0) ci[n] = out[0], si[n++] = solo[0];
        if (w2 > 0) ci[n] = out[1], si[n++] = solo[1];
        *cp = cp_value(ci, si, n);
    }
    return KL_OK;
}

kl_status kernelet_predict_group(const kl_config* cfg, const kl_profile* profiles,
                                 const int32_t* waves, int32_t n, double* ipc, double* cp) {
    if (!profiles || !waves || !ipc || n < 1 || n > 3) {
        set_error("kernelet_predict_group: null argument or n outside 1..3");
        return KL_EINVAL;
    }
    int total = 0;
    for (int k = 0; k < n; ++k) {
        if (waves[k] < 1 || waves[k] > 16) {
            set_error("kernelet_predict_group: wave count outside 1..16");
            return KL_EINVAL;
        }
        total += waves[k];
    }
    if (total > 24) {
        set_error("kernelet_predict_group: more than 24 waves in all");
        return KL_EINVAL;
    }
    kl_config c = cfg ? *cfg : defaults();
    if (kl_status s = check_cfg(c)) return s;
    KernelModel km[3];
    int w[3];
    double solo[3];
    for (int k = 0; k < n; ++k) {
        if (kl_status s = check_profile(profiles[k])) return s;
        km[k] = kernel_model(profiles[k], c);
        w[k] = waves[k];
    }
    if (chain_states(km, w, n) > kMaxChainStates) {
        set_error("kernelet_predict_group: the chain of these wave counts is too large");
        return KL_EINVAL;
    }
    double out[3];
    chain_ipc(km, w, n, c.beta, c.beta_lds, out);
    for (int k = 0; k < n; ++k) ipc[k] = out[k];
    if (cp) {
        for (int k = 0; k < n; ++k) solo[k] = solo_ipc(profiles[k], c);
        *cp = cp_value(out, solo, n);
    }
    return KL_OK;
}

kl_status kernelet_best_ratio(const kl_config* cfg, const kl_profile* p1, const kl_profile* p2,
                              int32_t* b1, int32_t* b2, double* value, double* c1,
                              double* c2) {
    if (!p1 || !p2) {
        set_error("kernelet_best_ratio: null profile");
        return KL_EINVAL;
    }
    kl_config c = cfg ? *cfg : defaults();
    if (kl_status s = check_cfg(c)) return s;
    if (kl_status s = check_profile(*p1)) return s;
    if (kl_status s = check_profile(*p2)) return s;
    Ratio r = best_ratio(*p1, *p2, c);
    if (!r.ok) {
        set_error("kernelet_best_ratio: no feasible ratio");
        return KL_ENOTFOUND;
    }
    if (b1) *b1 = r.b1;
    if (b2) *b2 = r.b2;
    if (value) *value = r.value;
    if (c1) *c1 = r.cipc1;
    if (c2) *c2 = r.cipc2;
    return KL_OK;
}

kl_status kernelet_simulate(const kl_config* cfg, const kl_profile* profiles,
                            int32_t n_profiles, const int32_t* job_profile,
                            const uint64_t* job_wgs, const double* job_arrival,
                            int32_t n_jobs, kl_policy policy,
                            const kl_pair_measure* measures, uint32_t n_measures,
                            kl_decision* dec, int32_t max_dec, int32_t* n_dec,
                            double* makespan, double* done) {
    if (!profiles || n_profiles < 1 || !job_profile || !job_wgs || n_jobs < 0 ||
        (n_jobs > 0 && !done) || !makespan || (n_measures > 0 && !measures)) {
        set_error("kernelet_simulate: null argument");
        return KL_EINVAL;
    }
    if (policy != KL_POLICY_FIFO && policy != KL_POLICY_MARKOV && policy != KL_POLICY_OPT &&
        policy != KL_POLICY_RANDOM) {
        set_error("kernelet_simulate: policy must be FIFO, MARKOV, OPT or RANDOM");
        return KL_EINVAL;
    }
    kl_config c = cfg ? *cfg : defaults();
    if (c.n_cu == 0) c.n_cu = 256;
    if (kl_status s = check_cfg(c)) return s;
    std::vector<kl_profile> types(profiles, profiles + n_profiles);
    for (auto& p : types)
        if (kl_status s = check_profile(p)) return s;
    for (int i = 0; i < n_jobs; ++i)
        if (job_profile[i] < 0 || job_profile[i] >= n_profiles || job_wgs[i] == 0) {
            set_error("kernelet_simulate: bad job");
            return KL_EINVAL;
        }
    Planner pl(c);
    pl.set_types(types);
    if (policy == KL_POLICY_OPT) {
        std::map<std::pair<int, int>, std::vector<Measure>> m;
        if (!measure_map(measures, n_measures, n_profiles, "kernelet_simulate", &m))
            return KL_EINVAL;
        pl.set_measures(m);
    }
    uint64_t draws = 0;
    auto arrival = [&](int i) { return job_arrival ? job_arrival[i] : 0.0; };
    int nd = 0;
    double t = 0.0;
    if (policy == KL_POLICY_FIFO) {
        for (int i = 0; i < n_jobs; ++i) {
            t = std::max(t, arrival(i));
            const kl_profile& p = types[job_profile[i]];
            t += (double)job_wgs[i] / wg_rate(p, pl.solo(job_profile[i]), c.n_cu);
            done[i] = t;
        }
        *makespan = t;
        if (n_dec) *n_dec = 0;
        return KL_OK;
    }
    const double kEps = 1e-6;
    std::vector<double> rem(n_jobs);
    std::vector<char> fin(n_jobs, 0);
    for (int i = 0; i < n_jobs; ++i) rem[i] = (double)job_wgs[i];
    int ndone = 0;
    while (ndone < n_jobs) {
        std::vector<PendingJob> pend;
        for (int i = 0; i < n_jobs; ++i)
            if (!fin[i] && arrival(i) <= t) pend.push_back({i, job_profile[i], rem[i]});
        if (pend.empty()) {
            double nt = 1e300;
            for (int i = 0; i < n_jobs; ++i)
                if (!fin[i]) nt = std::min(nt, arrival(i));
            t = nt;
            continue;
        }
        Decision d;
        if (policy == KL_POLICY_OPT) {
            d = pl.find_opt(pend);
        } else if (policy == KL_POLICY_RANDOM) {
            d = pl.find_random(pend, splitmix64(c.random_seed, 2 * draws),
                               splitmix64(c.random_seed, 2 * draws + 1));
            ++draws;
        } else {
            d = pl.find(pend);
        }
        if (dec && nd < max_dec) {
            kl_decision& x = dec[nd];
            x = kl_decision{};
            x.j1 = d.j1;
            x.j2 = d.j2;
            x.j3 = d.j3;
            x.b1 = d.b1;
            x.b2 = d.b2;
            x.b3 = d.b3;
            x.value = d.value;
            x.cipc1 = d.cipc1;
            x.cipc2 = d.cipc2;
            x.cipc3 = d.cipc3;
            x.t_us = t;
        }
        ++nd;
        int a = (int)d.j1;
        const kl_profile& pa = types[job_profile[a]];
        if (d.j2 < 0) {
            t += rem[a] / wg_rate(pa, d.cipc1, c.n_cu);
            rem[a] = 0;
            fin[a] = 1;
            done[a] = t;
            ++ndone;
            continue;
        }
        // the co-schedule runs until the first of its kernels runs out
        const int ng = d.j3 < 0 ? 2 : 3;
        const int g[3] = {a, (int)d.j2, (int)d.j3};
        const double cg[3] = {d.cipc1, d.cipc2, d.cipc3};
        double rate[3], tl[3];
        for (int k = 0; k < ng; ++k) {
            rate[k] = wg_rate(types[job_profile[g[k]]], cg[k], c.n_cu);
            tl[k] = rem[g[k]] / rate[k];
        }
        int first = 0;
        for (int k = 1; k < ng; ++k)
            if (tl[k] < tl[first]) first = k;
        const double dt = tl[first];
        t += dt;
        for (int k = 0; k < ng; ++k) {
            const int i = g[k];
            if (k != first) {
                rem[i] -= dt * rate[k];
                if (!(rem[i] <= kEps)) continue;
            }
            rem[i] = 0;
            fin[i] = 1;
            done[i] = t;
            ++ndone;
        }
    }
    *makespan = t;
    if (n_dec) *n_dec = nd;
    return KL_OK;
}

}  // extern "C"
