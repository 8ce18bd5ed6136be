/*
 * kernelet.h -- C ABI of the sliced co-execution engine (libkernelet.so).
 *
 * The engine raises the throughput of many independent GPU kernels sharing
 * one MI355X (gfx950) by the method of Kernelet (Zhong & He): every
 * submitted kernel is cut into slices (contiguous ranges of workgroup ids,
 * Section 2.2 "Problem Definition"), slices of two kernels with
 * complementary demands run at the same time (a co-schedule), and the pair
 * and its slice sizes are chosen greedily (Algorithm 1 with procedure
 * FindCoSchedule, Section 4.2) after PUR/MUR pruning (Section 4.3) by a
 * Markov-chain model of wavefront states (Section 4.4).
 *
 * Conventions for every call:
 *   - the return value is a kl_status: 0 on success, a negative KL_E* code
 *     on failure; kernelet_last_error() gives a message for the calling
 *     thread's last failure.  No C++ exception crosses this boundary.
 *   - "host" pointers point to CPU memory, "device" pointers to memory
 *     allocated on the runtime's GPU (e.g. by PyTorch).  The library never
 *     frees memory it did not allocate.
 *   - calls are thread-safe except kernelet_init / kernelet_shutdown, which
 *     must not race with any other call on the same runtime.
 */
#ifndef KERNELET_H
#define KERNELET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kl_status;
#define KL_OK 0
#define KL_EINVAL (-1)     /* bad argument, size or grid */
#define KL_ENOMEM (-2)     /* request larger than the memory budget */
#define KL_EEXIST (-3)     /* a kernel of that name is registered */
#define KL_ENOTFOUND (-4)  /* unknown kernel, job or symbol */
#define KL_ESTATE (-5)     /* call not valid in the object's state */
#define KL_ETIMEOUT (-6)   /* wait timed out; the job keeps running */
#define KL_EHIP (-7)       /* a HIP runtime call failed */
#define KL_ECANCELED (-8)  /* the job was cancelled */
#define KL_EINTERNAL (-9)

typedef struct kl_runtime kl_runtime; /* opaque; owned by the library */
typedef int32_t kl_kernel;            /* kernel type handle (>= 0) */
typedef int64_t kl_job;               /* job handle (>= 0) */
#define KL_NO_JOB ((kl_job)-1)

typedef struct {
    uint32_t x, y, z;
} kl_dim3;

/* Device-side slice descriptor.  Every sliceable kernel takes it as its
 * LAST argument and is launched on a 1-D grid of `count` workgroups; its
 * workgroup with built-in index b is workgroup offset + b of the ORIGINAL
 * grid (gx, gy, gz), linearised row-major: id = x + gx (y + gy z).  This is
 * the paper's index rectification (Section 4.1), done at source level. */
typedef struct {
    uint32_t offset; /* first original workgroup id of the slice */
    uint32_t count;  /* workgroups in the slice (= launch grid) */
    uint32_t gx, gy, gz;
    uint32_t reserved;
} kl_slice;

/* Per-kernel inputs of the performance model and of pruning (Section 4.4,
 * its paragraph on obtaining the model's inputs; PUR and MUR of Section 4.3).  The
 * Markov model runs on a virtual SIMD (the paper's virtual single-scheduler
 * SM, one of the 4 SIMDs of a CU); its time unit is one issue slot. */
typedef struct {
    double r_mem;          /* P(issued instruction stalls on memory)      */
    double mem_req;        /* memory requests held by one stalled wave     */
    double lat_mem;        /* memory-stall latency when the memory system
                              is idle, issue slots (0: the config's)       */
    double r_comp;         /* P(issued instruction stalls on compute)     */
    double lat_comp;       /* compute-stall latency, issue slots           */
    double instr_per_wave; /* instructions one wave executes (I_K)         */
    double pur, mur;       /* pipeline / memory-bandwidth utilisation     */
    double solo_ipc;       /* measured solo IPC (informational)            */
    int32_t max_wg_per_cu; /* resource-limited workgroups per CU, alone   */
    int32_t waves_per_simd;/* waves one workgroup puts on each SIMD        */
    int32_t vgpr;          /* VGPRs per lane (0: not limiting)             */
    int32_t lds_bytes;     /* static LDS bytes per workgroup               */
    int32_t min_slice_wgs; /* calibrated minimum slice (0: unknown)        */
    int32_t access;        /* dominant access pattern: 0 coalesced,
                              1 strided, 2 random (a surrogate feature)    */
    int32_t comp_pool;     /* 0: the compute stall has the fixed latency
                              lat_comp; 1: it waits on the CU's LDS, latency
                              lat_comp + beta_lds * (waves of all resident
                              kernels stalled on LDS)                      */
    int32_t reserved;
} kl_profile;

/* Hardware-counter readings of one launch of a kernel run alone, with its
 * duration: the raw material of the model inputs (Section 4.3 defines PUR
 * and MUR from instructions, DRAM traffic and time; Section 4.4 takes the
 * memory-instruction ratio from profiling the kernel).  Counts are totals
 * over the launch (rocprofv3 --pmc SQ_WAVES SQ_INSTS_* FETCH_SIZE
 * WRITE_SIZE on gfx950; FETCH_SIZE and WRITE_SIZE scaled to bytes). */
typedef struct {
    double waves;          /* waves launched (SQ_WAVES)                       */
    double valu, salu, vmem, smem, lds, branch; /* instructions issued by kind,
                              SQ_INSTS_VALU (matrix and transcendental
                              instructions included), _SALU, _VMEM, _SMEM,
                              _LDS, _BRANCH                                  */
    double mfma;           /* matrix instructions (SQ_INSTS_MFMA), of valu    */
    double trans;          /* FP32 transcendentals (SQ_INSTS_VALU_TRANS_F32),
                              of valu                                        */
    double dram_read;      /* bytes read from HBM                             */
    double dram_write;     /* bytes written to HBM                            */
    double time_s;         /* duration of the launch, seconds                 */
    double freq_hz;        /* shader clock                                    */
    double peak_bw;        /* HBM bandwidth of the roof, bytes/s              */
    int32_t n_cu;          /* compute units the launch ran on                 */
    int32_t reserved;
} kl_counters;

#define KL_KF_IDEMPOTENT 1u /* re-running a slice gives the same result */

typedef struct {
    const char* name;        /* copied; unique per runtime */
    const void* host_fn;     /* __global__ fn(ArgsT args, kl_slice s) */
    uint32_t block_threads;  /* workgroup size; a multiple of 256 */
    uint32_t args_bytes;     /* sizeof(ArgsT), <= 256 */
    uint32_t flags;          /* KL_KF_* */
    const kl_profile* profile; /* optional; copied */
} kl_kernel_desc;

typedef enum {
    KL_POLICY_FIFO = 0,    /* every job unsliced, in submission order, one stream */
    KL_POLICY_MARKOV = 1,  /* Algorithm 1 driven by the Markov model */
    KL_POLICY_SURROGATE = 2, /* Algorithm 1, pairs ranked by the surrogate
                                network, the Markov model evaluating its top k */
    KL_POLICY_FIXED = 3,   /* Algorithm 1 with explicit slice plans only */
    KL_POLICY_OPT = 4,     /* Algorithm 1 with every pair and slice ratio
                              measured beforehand (the paper's OPT baseline,
                              Section 5): the pair and ratio of highest
                              measured CP; needs kernelet_set_pair_measures */
    KL_POLICY_RANDOM = 5,  /* Algorithm 1 with the pair and slice ratio drawn
                              at random: one sample of the paper's Monte
                              Carlo baseline MC(s) (Section 5); draws from
                              SplitMix64 seeded by cfg.random_seed */
    KL_POLICY_CONCURRENT = 6 /* no model, no slicing (a baseline): each of the
                              cfg.lanes streams takes the earliest runnable
                              job not yet launched whenever its in-flight
                              window has room, and launches it whole */
} kl_policy;

#define KL_BLOCKING 1u           /* return when every pending job is launched */
#define KL_REPLAN_ON_ARRIVAL 2u  /* re-decide when a job arrives */
#define KL_WAIT_DONE 4u          /* with KL_BLOCKING: return when every job has
                                    finished (completion times are stamped by
                                    the dispatcher as slices retire) */

typedef enum {
    KL_MODE_BALANCED = 0, /* max 1 - max(T1,T2)/(T1s+T2s) over slice ratios */
    KL_MODE_CP = 1,       /* max Eq. (1) */
    KL_MODE_LITERAL = 2   /* min Delta T of Eq. (8), ties to larger CP */
} kl_ratio_mode;

typedef struct {
    int32_t n_cu;          /* compute units (0: query the device) */
    int32_t wmax;          /* wave slots per SIMD (8 on gfx950) */
    int32_t vgpr_file;     /* VGPRs per lane per SIMD (512) */
    int32_t lds_cu;        /* LDS bytes per CU (163840) */
    double alpha_p, alpha_m; /* pruning thresholds (0.4, 0.1) */
    int32_t use_prune;
    int32_t ratio_mode;    /* kl_ratio_mode (KL_MODE_CP) */
    double cp_min;         /* the best pair is taken only if its profit
                              (Eq. 1) exceeds this; else the earliest job
                              runs alone (-1: any pair not predicted to
                              halve the two kernels' throughput)          */
    double mem_latency;    /* memory latency with an idle memory system, slots */
    double beta;           /* latency added per outstanding request, slots */
    int32_t lanes;         /* co-execution streams (2) */
    int32_t inflight;      /* slices queued per lane ahead of the GPU (2) */
    int32_t lds_reserve;   /* occupancy control by LDS reservation (dynamic LDS
                              added to each workgroup of a co-schedule):
                              0 none; 1 every WG reserves LDS_CU/(b1+b2), so a
                              CU holds at most b1+b2 of them; 2 only the kernel
                              with the larger register footprint reserves just
                              over LDS_CU/(b+1), capping it at b per CU while
                              its partner fills the rest (b >= 2); default 2 */
    int32_t max_slices;    /* cap on slices per co-schedule of one kernel (0: none) */
    int64_t hbm_budget;    /* bytes of job footprint admitted at once (0: none) */
    int32_t surrogate_topk;/* pairs the Markov model re-ranks (SURROGATE);
                              0: the surrogate's best pair and ratio as is */
    uint32_t random_seed;  /* KL_POLICY_RANDOM: its k-th decision (k = 0,
                              1, ... since kernelet_init, or since the start
                              of kernelet_simulate) takes outputs 2k and
                              2k + 1 of the SplitMix64 stream whose state
                              starts at this seed (0)                      */
    int32_t solo_overlap;  /* a kernel run alone (no profitable pair, R10):
                              0 the other lanes wait for it; 1 the next
                              decision's launches may start beside it and
                              take the compute units it frees (0)         */
    int32_t pair_same_type; /* 1: the two earliest pending instances of a
                              kernel type are both candidates, so they may
                              pair (the PUR/MUR rule prunes such a pair
                              unless nothing else survives); 0: only the
                              earliest instance of each type (1)          */
    int32_t group_max;     /* kernels per co-schedule under KL_POLICY_MARKOV:
                              2 pairs (the paper's Algorithm 1); 3 the pair
                              FindCoSchedule picks may be joined by a
                              pending kernel of a third type when the
                              three-kernel model (Section 4.4) predicts a
                              larger objective for the best ratio of all
                              three than for the pair; needs lanes >= 3 (2) */
    int32_t inflight_us;   /* besides `inflight` slices, a lane keeps launching
                              while less than this many microseconds of
                              predicted work (the profile's solo rate) are
                              queued on it, up to 64 slices, so that slices
                              shorter than a launch call do not starve the
                              GPU (50; 0: the slice count alone)          */
    int32_t auto_profile;  /* 1: a model policy (MARKOV, SURROGATE, OPT, RANDOM)
                              meeting a pending job of a kernel without a
                              profile first profiles it by pre-executing
                              the job's first workgroups alone (timed, at
                              the kernel's full occupancy and at two
                              workgroups per CU held by LDS reservation;
                              they count as the job's progress) and
                              deriving the model inputs from the timings
                              and the code object's resources; 0: such a
                              schedule call fails with KL_ESTATE (1)     */
    int32_t lane_streams;  /* HIP streams per lane, 1 or 2.  With 2, the
                              model and FIXED policies alternate a job's
                              consecutive slices between the lane's two
                              streams, so that a slice's tail overlaps the
                              next slice's head (slices of one job are
                              independent, Section 2.2); LDS reservation
                              still caps the kernel per CU, a job's
                              completion is that of all its slices, and
                              each stream keeps the lane's in-flight window.
                              FIFO and CONCURRENT use one stream per lane.
                              On the MI355X mixes measured, 2 lowered the
                              gain over FIFO (1)                          */
    double beta_lds;       /* latency added per wave stalled on LDS, slots
                              (0: LDS stalls have fixed latencies)         */
    double min_pair_slots; /* a job predicted to finish alone within this
                              many issue slots is never co-scheduled
                              (0: every job may be)                        */
} kl_config;

typedef struct {
    int64_t jobs_submitted, jobs_done;
    int64_t slices_launched, decisions;
    double decision_us_total;   /* host time spent in FindCoSchedule */
    double model_us_total;      /* of which Markov solves */
    int64_t cache_hits;
    int64_t resident_bytes;     /* footprint admitted and not yet released */
    int64_t resident_peak;      /* largest resident_bytes so far */
    double surrogate_us_total;  /* host time of surrogate scoring (SURROGATE) */
    int64_t surrogate_candidates; /* (pair, ratio) candidates scored */
    int64_t surrogate_pairs;    /* pairs ranked by the surrogate */
    int64_t kernels_profiled;   /* kernel types profiled by pre-execution
                                   (kl_config.auto_profile) */
    int64_t model_solves;       /* pair (and triple) ratio searches solved by
                                   the Markov model, cache misses only */
} kl_stats;

/* One measured co-run (KL_POLICY_OPT): kernel a at b1 workgroups per CU
 * beside kernel b at b2, and each kernel's rate in the co-run relative to
 * its rate alone (cIPC / IPC, Eq. 1), so that the measured weighted speedup
 * is rel_a + rel_b and CP = 1 - 1 / (rel_a + rel_b).  a and b are kl_kernel
 * handles (kernelet_set_pair_measures) or profile indices
 * (kernelet_simulate). */
typedef struct {
    int32_t a, b;
    int32_t b1, b2;
    double rel_a, rel_b;
} kl_pair_measure;

/* One scheduling decision, as logged (Algorithm 1, one co-schedule). */
typedef struct {
    kl_job j1, j2;       /* j2 = KL_NO_JOB: kernel runs alone */
    int32_t b1, b2;      /* workgroups per CU of each slice */
    uint32_t slice1, slice2; /* slice sizes in workgroups */
    double value;        /* objective of the chosen ratio */
    double cipc1, cipc2; /* predicted co-run IPCs */
    double t_us;         /* host time of the decision since the first */
    kl_job j3;           /* a third kernel (cfg.group_max 3), else KL_NO_JOB */
    int32_t b3;          /* its workgroups per CU */
    uint32_t slice3;     /* its slice size in workgroups */
    double cipc3;        /* its predicted co-run IPC */
} kl_decision;

/* ---------------------------------------------------------------- set-up */

/* Fill *cfg with the defaults listed beside kl_config's fields. */
kl_status kernelet_default_config(kl_config* cfg);

/* Create a runtime on HIP device `hip_device`: the paper's runtime system
 * (Section 3.2: the queue of submitted kernels, the scheduler and the
 * co-execution of slices on one GPU).  `cfg` (host, may be NULL for
 * defaults) is copied.  The runtime owns its streams, events and threads.
 * Errors: KL_EINVAL (a field of cfg out of range, no such device), KL_EHIP. */
kl_status kernelet_init(kl_runtime** rt, int hip_device, const kl_config* cfg);

/* Copy the runtime's effective configuration (with n_cu filled in from the
 * device) to *cfg (host). */
kl_status kernelet_get_config(kl_runtime* rt, kl_config* cfg);

/* Wait for every launched slice, stop the scheduler thread, free all. */
kl_status kernelet_shutdown(kl_runtime* rt);

/* Message of the calling thread's last failure ("" if none); owned by the
 * library, valid until the thread's next call. */
const char* kernelet_last_error(void);

/* --------------------------------------------------------------- kernels */

/* Register a kernel type (Section 3.2: submitted kernels are kept per
 * type so that a profile and a slice size are reused).  Duplicate name:
 * KL_EEXIST.  block_threads not a positive multiple of 256 or args_bytes
 * > 256: KL_EINVAL. */
kl_status kernelet_register(kl_runtime* rt, const kl_kernel_desc* d,
                            kl_kernel* out);

/* Register a kernel type from a gfx950 code object (Section 4.1: a compiled
 * kernel made sliceable by rewriting it).  `image` (host memory, `bytes`
 * long; read during the call) holds the kernel `symbol`, which takes
 * (ArgsT args, kl_slice s) by value: the form paper_1303_5164_amd/
 * irslice.py gives a kernel written without slicing.  d->host_fn must be
 * NULL; d->name, block_threads, args_bytes (sizeof(ArgsT)), flags and
 * profile as for kernelet_register.  The code object is loaded on the
 * runtime's device and unloaded at shutdown; jobs of the type are launched
 * through it like any other.  Errors: KL_EINVAL, KL_EEXIST (duplicate
 * name), KL_EHIP (the image does not load or lacks the symbol). */
kl_status kernelet_register_image(kl_runtime* rt, const kl_kernel_desc* d,
                                  const void* image, uint64_t bytes, const char* symbol,
                                  kl_kernel* out);

/* Look up one of the library's eight workload kernels by name ("poly",
 * "gather", "sgemm", "spmv", "stencil", "bs", "hist", "lookup") and fill a
 * descriptor for kernelet_register.  The descriptor's strings are static. */
kl_status kernelet_builtin(const char* name, kl_kernel_desc* out);

/* Original grid a built-in kernel needs for the argument block `args`
 * (host, the kernel's argument struct of include/kernelet_workloads.h). */
kl_status kernelet_builtin_grid(const char* name, const void* args,
                                uint32_t args_bytes, kl_dim3* grid);

/* Resources of kernel k from its code object: workgroups one CU can hold
 * when the kernel runs alone (hipOccupancyMaxActiveBlocksPerMultiprocessor
 * with no dynamic LDS), VGPRs + AGPRs per lane, static LDS bytes per
 * workgroup.  Any output may be NULL. */
kl_status kernelet_kernel_info(kl_runtime* rt, kl_kernel k, int32_t* max_wg_per_cu,
                               int32_t* vgpr, int32_t* lds_bytes);

/* Model inputs of a kernel from the counters of a launch run alone (host;
 * no GPU).  Instructions are counted by the issue slots they hold (an FP32
 * 32x32x2 matrix instruction 16, a transcendental 4, any other 1): with S
 * slots over the launch, instr_per_wave = S / waves (I_K of Section 4.4);
 * r_mem = vmem / S, the memory-instruction ratio of Section 4.4; an LDS
 * instruction is the compute stall, r_comp = lds / S in the CU's LDS pool
 * (comp_pool 1; 0 when below 1e-4); mem_req = max(1, DRAM bytes / 64 /
 * vmem), the 64-byte requests one memory instruction holds; PUR (Section
 * 4.3) = S / (time * freq * n_cu), issue slots used over the chip's (one per
 * SIMD every four cycles), capped at 1; MUR (Section 4.3) = DRAM bytes /
 * (time * peak_bw); solo_ipc = the uncapped PUR.  The latencies
 * (lat_mem, lat_comp = 1) are left to a fit against measured occupancy
 * curves and occupancy and resource fields to the code object: out's other
 * fields are untouched.  KL_EINVAL for a count that is negative, no waves
 * or instructions, or a time, clock, bandwidth or CU count not positive. */
kl_status kernelet_profile_from_counters(const kl_counters* c, kl_profile* out);

kl_status kernelet_set_profile(kl_runtime* rt, kl_kernel k, const kl_profile* p);
kl_status kernelet_get_profile(kl_runtime* rt, kl_kernel k, kl_profile* p);

/* ------------------------------------------------------------------ jobs */

/* Submit one launch of kernel `k` over the ORIGINAL grid `grid` with
 * argument block `args` (host, args_bytes bytes, copied before return): a
 * kernel of Section 2.2's problem definition (a grid of independent thread
 * blocks), entering the pending set that Algorithm 1 re-optimises whenever
 * kernels arrive (Section 3.2).
 * Device pointers inside `args` are borrowed: the caller keeps the memory
 * alive until kernelet_wait on this job returns KL_OK.  `after` (or
 * KL_NO_JOB) names a job that must finish before this one starts.
 * `client` tags the submitting client; `footprint` is the device memory the
 * job holds (for the memory budget): it is charged when the job is admitted
 * and released when the job finishes, or, if jobs submitted `after` it
 * have yet to finish, when the last job of that chain does (an instance of
 * several dependent launches passes its footprint with the first launch).
 * A job becomes pending at once (and is scheduled by the next or the
 * running kernelet_schedule).  Errors:
 * KL_EINVAL (grid of zero workgroups or > 2^32-1, size mismatch, grid not
 * the built-in kernel's required grid), KL_ENOTFOUND (k or after),
 * KL_ENOMEM (footprint above the whole budget). */
kl_status kernelet_submit(kl_runtime* rt, kl_kernel k, kl_dim3 grid,
                          const void* args, uint32_t args_bytes, kl_job after,
                          uint32_t client, uint64_t footprint, kl_job* out);

/* Submit an instance made of `n` dependent launches at once: launch i is
 * kernel k[i] over the original grid grid[i] with argument block args[i]
 * (args_bytes[i] bytes, copied), and runs after launch i-1 (launch 0 after
 * `after`, or KL_NO_JOB).  `footprint` is charged when launch 0 is admitted
 * and released when launch n-1 finishes: the chain is created under the
 * runtime's lock, so no launch of it starts before all of them exist.
 * out[0..n-1] (host) receive the job ids.  All launches are checked first;
 * on an error none is submitted.  Errors as kernelet_submit, and KL_EINVAL
 * for n == 0. */
kl_status kernelet_submit_chain(kl_runtime* rt, uint32_t n, const kl_kernel* k,
                                const kl_dim3* grid, const void* const* args,
                                const uint32_t* args_bytes, kl_job after,
                                uint32_t client, uint64_t footprint, kl_job* out);

/* Fix the slicing plan of a job before it starts (Section 4.1: a slice is
 * a run of consecutive workgroups launched as its own kernel, the offset
 * added back to the block index on the device; Section 2.2: a slicing plan
 * cuts a kernel into slices): slices of `wgs_per_slice` workgroups (0: the
 * calibrated minimum of its kernel, else its whole grid); *n_slices
 * receives the slice count.  Used by the FIXED policy and
 * by tests.  KL_ESTATE if the job has started. */
kl_status kernelet_slice(kl_runtime* rt, kl_job j, uint32_t wgs_per_slice,
                         uint32_t* n_slices);

/* Workgroups per CU the FIXED policy runs job j at (1..64): its slices are
 * sized b * n_cu unless kernelet_slice fixed them, and LDS reservation, when
 * enabled, is computed for it.  KL_ESTATE if the job has started. */
kl_status kernelet_job_occupancy(kl_runtime* rt, kl_job j, int32_t wg_per_cu);

/* Run the scheduler with `policy` over the pending jobs (Algorithm 1:
 * FindCoSchedule picks a pair of pending kernels and their slice ratio,
 * their slices run side by side while both have workgroups left, then the
 * next decision; Section 4.2).  With KL_BLOCKING
 * the call returns once every pending job (including dependants released
 * meanwhile) has been launched; otherwise a scheduler thread keeps serving
 * submissions until kernelet_shutdown.  Launches are asynchronous: use
 * kernelet_wait for completion.  The model's policies (MARKOV, SURROGATE,
 * OPT, RANDOM) need a profile for every pending job's kernel: given at
 * registration or by kernelet_set_profile, or, with cfg.auto_profile, measured
 * from the first job's own pre-executed workgroups before its kernel is
 * first scheduled (Section 4.4, the model's inputs from a few pre-executed
 * thread blocks); FIFO, FIXED and CONCURRENT need none.  KL_ESTATE: a pending
 * kernel without a profile under a model policy when auto_profile is off,
 * SURROGATE without kernelet_set_surrogate, OPT
 * without kernelet_set_pair_measures, or a scheduler already running;
 * KL_EINVAL: an unknown policy. */
kl_status kernelet_schedule(kl_runtime* rt, kl_policy policy, uint32_t flags);

/* Block until job j has finished on the GPU, or `timeout_ns` (< 0:
 * forever) elapses (Section 2.2: kernels arrive in an order not known
 * beforehand and are throughput oriented, so a caller learns of each one's
 * completion separately).  After KL_OK the memory its argument block points
 * to may be reused.  KL_OK, KL_ETIMEOUT, KL_EHIP (device error),
 * KL_ECANCELED, KL_ENOTFOUND. */
kl_status kernelet_wait(kl_runtime* rt, kl_job j, int64_t timeout_ns);

/* Block until every launched slice has finished. */
kl_status kernelet_synchronize(kl_runtime* rt);

/* Order every later launch of the runtime after the work queued so far on
 * `stream` (a hipStream_t of the runtime's device; NULL = the null stream):
 * an event is recorded on it now and every lane waits for it before its
 * next launch.  For inputs produced asynchronously, e.g. by torch on its
 * current stream, without a host synchronisation.  KL_EHIP if the stream
 * cannot be used. */
kl_status kernelet_stream_barrier(kl_runtime* rt, void* stream);

/* Cancel a job that has not started.  KL_ESTATE once it has. */
kl_status kernelet_cancel(kl_runtime* rt, kl_job j);

/* Host timestamps (ns, steady clock) of a job: submission, first launch,
 * completion observed by the library (0 when unknown). */
kl_status kernelet_job_times(kl_runtime* rt, kl_job j, int64_t* t_submit,
                             int64_t* t_start, int64_t* t_done);

/* Forget finished jobs (their handles become unknown). */
kl_status kernelet_reap(kl_runtime* rt);

/* ----------------------------------------------------------------- model */

/* Performance model on two kernel profiles (host; no GPU needed): per-kernel
 * IPCs when w1 and w2 waves per SIMD co-run (Eqs. 5-7; w2 = 0 gives the
 * homogeneous model of Eq. 4), and CP of Eq. (1) against each kernel alone
 * at its own full occupancy.  Latency: mem_latency + beta * outstanding
 * requests (cfg may be NULL for defaults).  Any output pointer may be NULL. */
kl_status kernelet_predict(const kl_config* cfg, const kl_profile* p1,
                           const kl_profile* p2, int32_t w1, int32_t w2,
                           double* ipc1, double* ipc2, double* cp);

/* The model on n = 1..3 co-resident kernels (host): ipc[k] (host array of
 * n) is kernel k's IPC with waves[k] >= 1 waves per SIMD beside the others
 * (Eqs. 5-7 with one joint state per kernel; the paper notes its model covers
 * more than two kernels), and *cp (may be NULL) Eq. (1) over the n kernels
 * against each alone at its own full occupancy.  KL_EINVAL for n outside
 * 1..3, a wave count outside 1..16, more than 24 waves in all, or a bad
 * profile. */
kl_status kernelet_predict_group(const kl_config* cfg, const kl_profile* profiles,
                                 const int32_t* waves, int32_t n, double* ipc, double* cp);

/* Best feasible slice ratio of a pair (Section 4.4, balanced slice ratio):
 * writes b1, b2 (workgroups per CU), the objective and the two IPCs.
 * KL_ENOTFOUND when no ratio fits the CU's resources. */
kl_status kernelet_best_ratio(const kl_config* cfg, const kl_profile* p1,
                              const kl_profile* p2, int32_t* b1, int32_t* b2,
                              double* value, double* cipc1, double* cipc2);

/* Greedy co-scheduling on the virtual clock of the model (no GPU): runs
 * Algorithm 1 (or FIFO if policy == KL_POLICY_FIFO) over n jobs given by
 * kernel profile index, workgroup count and arrival time; writes up to
 * max_dec decisions (j1/j2/j3 are job indices), their count, the makespan and
 * each job's completion time (host arrays of n).  KL_POLICY_OPT takes its
 * pairs, ratios and co-run rates from `measures` (n_measures rows whose a
 * and b are profile indices; may be NULL otherwise); every other policy
 * takes co-run rates from the model; with cfg.group_max 3 the MARKOV policy
 * may co-schedule three kernels (no lanes needed here), and a co-schedule
 * runs until the first of its kernels runs out.  Used to test the
 * scheduler against the oracle and to predict a plan's gain.  KL_EINVAL for a policy other
 * than FIFO, MARKOV, OPT and RANDOM or a measure naming no profile. */
kl_status kernelet_simulate(const kl_config* cfg, const kl_profile* profiles,
                            int32_t n_profiles, const int32_t* job_profile,
                            const uint64_t* job_wgs, const double* job_arrival,
                            int32_t n_jobs, kl_policy policy,
                            const kl_pair_measure* measures, uint32_t n_measures,
                            kl_decision* decisions, int32_t max_dec,
                            int32_t* n_dec, double* makespan, double* done);

/* ------------------------------------------------------------- surrogate */
/* The learned pair ranker: a 16 -> 64 -> 64 -> 1 ReLU network (parameters
 * one device fp32 array of 5313 values: W1 [16][64], b1 [64], W2 [64][64],
 * b2 [64], W3 [64], b3) trained by mean-squared error and Adam on co-run
 * speedups.  Kernels run on `stream` (a hipStream_t; NULL = the default
 * stream) and are asynchronous.  All arrays are device memory. */

#define KL_MLP_PARAMS 5313

/* Load trained surrogate parameters (host, n_params == KL_MLP_PARAMS floats,
 * copied) into the runtime; required by KL_POLICY_SURROGATE.  In that
 * policy each decision scores every feasible slice ratio of every pair that
 * survives pruning in one batched inference on the device (its own
 * stream), keeps the cfg.surrogate_topk pairs of highest predicted weighted
 * speedup and lets the Markov model choose among them (Kernelet, Section
 * 4.3, the model of Section 4.4 deciding among the ranked pairs).  Errors: KL_EINVAL,
 * KL_EHIP. */
kl_status kernelet_set_surrogate(kl_runtime* rt, const float* params, uint32_t n_params);

/* Load measured co-runs (host array of n rows, copied; a and b are kl_kernel
 * handles of this runtime) for KL_POLICY_OPT, replacing earlier ones.  A row
 * for (a at b1, b at b2) also serves the pair in the other order.  Under
 * OPT each decision takes, over the pairs of pending kernel types with
 * rows, the ratio of highest measured CP = 1 - 1 / (rel_a + rel_b), and the
 * pair of highest such CP if it exceeds cfg.cp_min (else the earliest job
 * alone).  Errors: KL_EINVAL (unknown kernel, a == b, b1 or b2 outside
 * 1..8, a rate not positive). */
kl_status kernelet_set_pair_measures(kl_runtime* rt, const kl_pair_measure* rows, uint32_t n);

/* The 16 input features of a candidate (kernel a at b1, kernel b at b2
 * workgroups per CU; host arrays): per kernel the memory-instruction ratio
 * r_mem, log2(clamp((1 - r_mem) / r_mem, 1, 64)) / 6, lds_bytes / 65536,
 * vgpr / 256, the access one-hot (coalesced, strided, random) and
 * b / cfg->wmax (cfg NULL: defaults).  KL_EINVAL for a bad profile or a
 * ratio that does not fit on one CU. */
kl_status kernelet_surrogate_features(const kl_config* cfg, const kl_profile* a,
                                      const kl_profile* b, int32_t b1, int32_t b2,
                                      float* out16);

/* Floats of scratch a training step over `batch` samples needs. */
uint64_t kernelet_mlp_workspace_floats(uint32_t batch);

/* y[s] = net(x[s]) for s < n; x is n x 16 row-major. */
kl_status kernelet_mlp_forward(const float* params, const float* x, uint32_t n, float* y,
                               void* stream);

/* One step on the samples idx[0..batch) (idx NULL: rows 0..batch) of
 * (x, t): the gradient of mean((net(x) - t)^2) is written to grad_out (if
 * not NULL) and, when m and v (first and second moments, 5313 each) are
 * given, Adam (beta 0.9, 0.999, eps 1e-8, bias-corrected at `step` >= 1)
 * updates params in place.  workspace: kernelet_mlp_workspace_floats(batch)
 * floats. */
kl_status kernelet_mlp_train_step(float* params, float* m, float* v, const float* x,
                                  const float* t, const int32_t* idx, uint32_t batch,
                                  uint32_t step, float lr, float* grad_out, float* workspace,
                                  void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as kernelet_mlp_train_step, same kernels and results, with its
 * workspace in a static device array of the library instead of a caller
 * buffer.  batch <= kernelet_mlp_noalloc_max_batch() (4096 samples, a
 * 4.2 MB array each GPU the library runs on holds until the process
 * ends); a larger batch returns KL_EINVAL with a message.  No device
 * memory is allocated or freed.  The array is shared by every call on one
 * GPU: calls that overlap on the same GPU (on different streams or host
 * threads without ordering) race and give undefined results.  The
 * caller's stream orders the step as for the workspace variant. */
uint32_t kernelet_mlp_noalloc_max_batch(void);
kl_status kernelet_mlp_train_step_noalloc(float* params, float* m, float* v, const float* x,
                                          const float* t, const int32_t* idx, uint32_t batch,
                                          uint32_t step, float lr, float* grad_out,
                                          void* stream);

/* --------------------------------------------------------------- logging */

/* Time every launch of kernel k (enable != 0) with a pair of HIP events
 * carried by the launch itself (hipExtLaunchKernel's start and stop
 * events: the dispatch's own begin and end, no extra packets on the
 * stream).  Enabling resets the kernel's counters. */
kl_status kernelet_time_kernel(kl_runtime* rt, kl_kernel k, int32_t enable);

/* Launch timing of kernel k since it was enabled: summed GPU time of its
 * launches (ms, event to event), number of launches and workgroups.  Only
 * launches that have finished are counted (call after a synchronisation). */
kl_status kernelet_kernel_time(kl_runtime* rt, kl_kernel k, double* total_ms,
                               int64_t* launches, int64_t* workgroups);

kl_status kernelet_stats(kl_runtime* rt, kl_stats* out);

/* Copy up to `max` logged decisions of the runtime (oldest first) to
 * `out` (host); *n receives the number copied.  The log is cleared. */
kl_status kernelet_decisions(kl_runtime* rt, kl_decision* out, int32_t max,
                             int32_t* n);

#ifdef __cplusplus
}
#endif
#endif /* KERNELET_H */
