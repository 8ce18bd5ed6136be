// Markov-chain performance model, PUR/MUR pruning and greedy co-schedule
// search of the co-execution engine (host code, double precision).
//
// Model (Kernelet, Section 4.4): the state of a virtual SIMD is the number
// of stalled wavefronts of each kernel in each stall class; one Markov step
// is one round in which every ready wave issues one instruction.  A ready
// wave stalls in class c with probability r_c; a stalled wave returns with
// probability min(1, D / L_c), D = max(#ready, 1) the round length and
// L_c = base_c + beta * (outstanding memory requests) for memory classes.
// Stationary vector by a dense solve; per-kernel IPC = E[ready_k] / E[D]
// (Eqs. 4-6); CP by Eq. (1).
#pragma once

#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernelet.h"

namespace kl {

struct StallClass {
    double r;     // probability per issued instruction
    double base;  // latency with the shared resource idle (issue slots)
    double req;   // requests held in its pool while stalled (0: fixed latency)
    int pool;     // contended resource: 0 HBM, 1 the CU's LDS
};

struct KernelModel {
    int nclass = 0;
    StallClass cls[2];
};

// Profile -> stall classes: class 0 is the memory stall (always present),
// class 1 the compute stall when r_comp > 0.
KernelModel kernel_model(const kl_profile& p, const kl_config& cfg);

// Joint states of the chain of nk kernels at w[k] waves per SIMD: the
// product over kernels of their stalled-count tuples.
int64_t chain_states(const KernelModel* km, const int* w, int nk);

// Largest chain solved (its dense transition matrix holds the square of
// this many doubles, 128 MiB).
constexpr int64_t kMaxChainStates = 4096;

// Per-kernel IPCs of one to three co-resident kernels (nk), kernel k with
// w[k] >= 1 waves per SIMD.  A chain above kMaxChainStates is not solved:
// the outputs are NaN.
void chain_ipc(const KernelModel* km, const int* w, int nk, double beta_hbm,
               double beta_lds, double* ipc_out);

double cp_value(const double* cipc, const double* solo, int n);

struct Ratio {
    bool ok = false;
    int b1 = 0, b2 = 0;
    double value = 0, cipc1 = 0, cipc2 = 0;
};

double solo_ipc(const kl_profile& p, const kl_config& cfg);
Ratio best_ratio(const kl_profile& p1, const kl_profile& p2,
                 const kl_config& cfg);

// A slice ratio of three kernels (workgroups per CU of each), the objective
// of cfg.ratio_mode carried to three kernels, and the co-run IPCs.
struct Triple {
    bool ok = false;
    int b[3] = {0, 0, 0};
    double value = 0, cipc[3] = {0, 0, 0};
};

// Whether b[k] workgroups per CU of the three kernels fit on one CU
// together: wave slots per SIMD, VGPR file and LDS.
bool triple_feasible(const kl_profile* const p[3], const kl_config& cfg, const int* b);

// Best feasible (b1, b2, b3) of three kernels given their solo IPCs, in
// lexicographic order (the first maximum wins): mode CP maximises Eq. (1)
// over the three; BALANCED 1 - max_k T_k / sum_k T_k,solo; LITERAL the
// smallest spread max_k T_k - min_k T_k, ties to the larger CP.
Triple best_triple(const kl_profile* const p[3], const double* solo, const kl_config& cfg);

bool pair_pruned(const kl_profile& a, const kl_profile& b, double ap,
                 double am);

// Whether b1 and b2 workgroups per CU of two kernels fit on one CU
// together: wave slots per SIMD, VGPR file and LDS.
bool ratio_feasible(const kl_profile& p1, const kl_profile& p2, const kl_config& cfg,
                    int b1, int b2);

// The surrogate network's eight input features of one kernel at b
// workgroups per CU: memory-instruction ratio, log2(ALU instructions per
// memory instruction, clamped to [1, 64]) / 6, LDS bytes / 64 KiB,
// VGPRs / 256, access pattern one-hot (coalesced, strided, random), b / wmax.
void surrogate_features(const kl_profile& p, int b, int wmax, float* out8);

// One pending job as seen by FindCoSchedule.
struct PendingJob {
    int64_t id;        // submission order key (smaller = earlier)
    int type;          // kernel type index
    double wgs = 0.0;  // workgroups still to run
};

// A measured co-run of two kernel types: the first at b1 workgroups per CU
// beside the second at b2, and each one's co-run rate over its rate alone.
struct Measure {
    int b1 = 0, b2 = 0;
    double rel1 = 0, rel2 = 0;
};

struct Decision {
    int64_t j1 = -1, j2 = -1;  // j2 = -1: solo
    int b1 = 0, b2 = 0;
    double value = 0, cipc1 = 0, cipc2 = 0;
    int64_t j3 = -1;  // a third kernel (cfg.group_max 3); -1: none
    int b3 = 0;
    double cipc3 = 0;
};

// Caches solo IPCs and per-type-pair ratio searches; thread-safe.
class Planner {
  public:
    explicit Planner(const kl_config& cfg) : cfg_(cfg) {}
    void set_types(const std::vector<kl_profile>& t);
    void set_type(int idx, const kl_profile& p);
    const kl_config& cfg() const { return cfg_; }
    double solo(int t);
    Ratio pair(int t1, int t2);
    // best_triple of three distinct types, searched once per set of types
    // (in ascending type order) and returned in the order asked.
    Triple triple(int t1, int t2, int t3);
    // FindCoSchedule over pending jobs (any order); `only_pairs` (optional)
    // restricts the search to the listed type pairs.
    Decision find(const std::vector<PendingJob>& pending,
                  const std::vector<std::pair<int, int>>* only_pairs = nullptr);
    // Scores candidate pairs given their two profiles: the predicted
    // weighted speedup of each pair at its best slice ratio, and that ratio;
    // false if it could not (then every pair is evaluated).
    using Scorer = std::function<bool(
        const std::vector<std::pair<const kl_profile*, const kl_profile*>>&,
        std::vector<double>*, std::vector<std::pair<int, int>>*)>;
    // FindCoSchedule in which the pairs surviving pruning are ranked by
    // `score` and only the best `k` are evaluated by the Markov model; with
    // k == 0 the best-scored pair and ratio are taken as they are (a pair is
    // kept when its CP = 1 - 1/S exceeds cp_min).
    Decision find_ranked(const std::vector<PendingJob>& pending, int k, const Scorer& score);
    // Forget cached surrogate scores (new network parameters).
    void clear_scores();
    // Measured co-runs per ordered type pair (every row kept in both orders,
    // in the order given), for find_opt.
    void set_measures(const std::map<std::pair<int, int>, std::vector<Measure>>& m);
    // FindCoSchedule on measured CP (the paper's OPT baseline): over the
    // pairs of the candidates with measurements, the pair and ratio of
    // highest CP = 1 - 1/(rel1 + rel2) (first found on ties, pairs in
    // submission order); kept when CP exceeds cp_min.  Co-run IPCs are the
    // measured rates times the model's solo IPCs.  No pruning.
    Decision find_opt(const std::vector<PendingJob>& pending);
    // One random co-schedule (a sample of the paper's Monte Carlo baseline):
    // among the candidate pairs with a feasible ratio (in submission order),
    // pair r_pair mod their number; among its feasible ratios (b1 major,
    // ascending), ratio r_ratio mod their number; co-run IPCs and CP from
    // the model.  Alone only when no pair has a feasible ratio.
    Decision find_random(const std::vector<PendingJob>& pending, uint64_t r_pair,
                         uint64_t r_ratio);
    int64_t scored_pairs = 0;
    const kl_profile& prof(int t) const { return types_[t]; }
    int ntypes() const { return (int)types_.size(); }
    double model_us = 0;
    int64_t cache_hits = 0;
    int64_t model_solves = 0;   // pair and triple ratio searches run (cache misses)

  private:
    // The earliest pending job of each type (submission order) that is not
    // too short to pair, and the decision to run the earliest job alone;
    // false when fewer than two such types are pending.
    bool candidates(const std::vector<PendingJob>& pending, std::vector<PendingJob>* order,
                    Decision* solo_d);
    // cfg.group_max 3: the pair of two different types joined by the
    // candidate of a third type whose best triple ratio has the largest
    // objective, if above the pair's (submission order breaks ties).
    Decision extend(const Decision& pair, const std::vector<PendingJob>& order);
    Decision search(const std::vector<PendingJob>& pending,
                    const std::vector<std::pair<int, int>>* only_pairs, int k,
                    const Scorer* score);
    kl_config cfg_;
    std::vector<kl_profile> types_;
    std::map<int, double> solo_;
    std::map<std::pair<int, int>, Ratio> pair_;
    std::map<std::tuple<int, int, int>, Triple> triple_;
    // surrogate score and best ratio per ordered type pair
    std::map<std::pair<int, int>, std::pair<double, std::pair<int, int>>> scored_;
    std::map<std::pair<int, int>, std::vector<Measure>> meas_;
    std::mutex mu_;
};

// Workgroups per issue slot that a kernel finishes chip-wide at IPC `ipc`.
// Model inputs from the counters of a solo launch (see
// kernelet_profile_from_counters); false for invalid counts.
bool profile_from_counters(const kl_counters& c, kl_profile* out);

double wg_rate(const kl_profile& p, double ipc, int n_cu);

}  // namespace kl
