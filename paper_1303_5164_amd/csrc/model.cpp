// Markov-chain performance model, pruning and co-schedule search (host).
// See model.hpp for the model's definition.
#include "model.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace kl {

KernelModel kernel_model(const kl_profile& p, const kl_config& cfg) {
    KernelModel m;
    m.nclass = 1;
    m.cls[0] = {p.r_mem, p.lat_mem > 0 ? p.lat_mem : cfg.mem_latency, p.mem_req, 0};
    if (p.r_comp > 0) {
        m.cls[1] = {p.r_comp, p.lat_comp, p.comp_pool == 1 ? 1.0 : 0.0, 1};
        m.nclass = 2;
    }
    return m;
}

namespace {

// Binomial coefficient by the multiplicative formula (exact in double for
// every count a chain here can hold).
double choose(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    if (k > n - k) k = n - k;
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(n - k + i) / (double)i;
    return std::round(c);
}

double binom(int n, int k, double p) {
    if (k < 0 || k > n) return 0.0;
    return choose(n, k) * std::pow(p, k) * std::pow(1.0 - p, n - k);
}

// Stalled-count tuples of one kernel: (n0) or (n0, n1), sum <= w.
struct KStates {
    int nclass, w;
    std::vector<int> n0, n1;  // per state
    std::vector<int> index;   // (a * (w + 1) + b) -> state index
    int size() const { return (int)n0.size(); }
    int at(int a, int b) const { return index[a * (w + 1) + b]; }
};

KStates enumerate(int w, int nclass) {
    KStates s;
    s.nclass = nclass;
    s.w = w;
    s.index.assign((w + 1) * (w + 1), -1);
    for (int a = 0; a <= w; ++a) {
        if (nclass == 1) {
            s.index[a * (w + 1)] = s.size();
            s.n0.push_back(a);
            s.n1.push_back(0);
            continue;
        }
        for (int b = 0; a + b <= w; ++b) {
            s.index[a * (w + 1) + b] = s.size();
            s.n0.push_back(a);
            s.n1.push_back(b);
        }
    }
    return s;
}

// Solve (P^T - I) pi = 0 with the last equation replaced by sum(pi) = 1.
void stationary(const std::vector<double>& P, int N, std::vector<double>& pi) {
    std::vector<double> A((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            A[(size_t)i * N + j] = P[(size_t)j * N + i] - (i == j ? 1.0 : 0.0);
    for (int j = 0; j < N; ++j) A[(size_t)(N - 1) * N + j] = 1.0;
    pi.assign(N, 0.0);
    pi[N - 1] = 1.0;
    for (int c = 0; c < N; ++c) {  // Gaussian elimination, partial pivoting
        int piv = c;
        double best = std::fabs(A[(size_t)c * N + c]);
        for (int r = c + 1; r < N; ++r) {
            double v = std::fabs(A[(size_t)r * N + c]);
            if (v > best) best = v, piv = r;
        }
        if (piv != c) {
            for (int j = 0; j < N; ++j)
                std::swap(A[(size_t)c * N + j], A[(size_t)piv * N + j]);
            std::swap(pi[c], pi[piv]);
        }
        double d = A[(size_t)c * N + c];
        for (int r = c + 1; r < N; ++r) {
            double f = A[(size_t)r * N + c] / d;
            if (f == 0.0) continue;
            double* ar = &A[(size_t)r * N];
            const double* ac = &A[(size_t)c * N];
            for (int j = c; j < N; ++j) ar[j] -= f * ac[j];
            pi[r] -= f * pi[c];
        }
    }
    for (int c = N - 1; c >= 0; --c) {
        double s = pi[c];
        for (int j = c + 1; j < N; ++j) s -= A[(size_t)c * N + j] * pi[j];
        pi[c] = s / A[(size_t)c * N + c];
    }
}

}  // namespace

int64_t chain_states(const KernelModel* km, const int* w, int nk) {
    int64_t n = 1;
    for (int k = 0; k < nk; ++k) {
        if (w[k] < 0) return -1;
        const int64_t s = km[k].nclass == 1 ? (int64_t)w[k] + 1
                                             : ((int64_t)w[k] + 1) * ((int64_t)w[k] + 2) / 2;
        n *= s;
        if (n > (int64_t)1 << 40) return n;
    }
    return n;
}

void chain_ipc(const KernelModel* km, const int* w, int nk, double beta_hbm,
               double beta_lds, double* ipc_out) {
    if (chain_states(km, w, nk) > kMaxChainStates) {
        // the dense chain would not fit: no prediction (callers check first)
        for (int k = 0; k < nk; ++k) ipc_out[k] = std::nan("");
        return;
    }
    const double beta[2] = {beta_hbm, beta_lds};
    // kernels beyond nk have one state (no waves) and move with probability 1
    KStates ks[3];
    int S[3];
    for (int k = 0; k < 3; ++k) {
        ks[k] = enumerate(k < nk ? w[k] : 0, k < nk ? km[k].nclass : 1);
        S[k] = ks[k].size();
    }
    const int N = S[0] * S[1] * S[2];
    std::vector<double> P((size_t)N * N, 0.0);
    std::vector<double> mv[3] = {std::vector<double>(S[0]), std::vector<double>(S[1]),
                                 std::vector<double>(S[2], 1.0)};
    int ix[3];
    for (ix[0] = 0; ix[0] < S[0]; ++ix[0]) {
        for (ix[1] = 0; ix[1] < S[1]; ++ix[1]) {
            for (ix[2] = 0; ix[2] < S[2]; ++ix[2]) {
                int nst[3][2];
                int ready[3] = {0, 0, 0};
                double outst[2] = {0.0, 0.0};  // requests held in each pool
                int rtot = 0;
                for (int k = 0; k < 3; ++k) {
                    nst[k][0] = ks[k].n0[ix[k]];
                    nst[k][1] = ks[k].n1[ix[k]];
                }
                for (int k = 0; k < nk; ++k) {
                    ready[k] = w[k] - nst[k][0] - nst[k][1];
                    rtot += ready[k];
                    for (int c = 0; c < km[k].nclass; ++c)
                        outst[km[k].cls[c].pool] += nst[k][c] * km[k].cls[c].req;
                }
                double D = std::max(rtot, 1);
                for (int k = 0; k < nk; ++k) {
                    const KernelModel& m = km[k];
                    double q[2] = {0, 0};
                    for (int c = 0; c < m.nclass; ++c) {
                        const StallClass& sc = m.cls[c];
                        double lat =
                            sc.req > 0 ? sc.base + beta[sc.pool] * outst[sc.pool] : sc.base;
                        q[c] = std::min(1.0, D / lat);
                    }
                    std::vector<double>& out = mv[k];
                    std::fill(out.begin(), out.end(), 0.0);
                    int r = ready[k];
                    int n0 = nst[k][0], n1 = nst[k][1];
                    if (m.nclass == 1) {
                        for (int a = 0; a <= r; ++a) {
                            double pn = binom(r, a, m.cls[0].r);
                            if (pn == 0.0) continue;
                            for (int b = 0; b <= n0; ++b) {
                                double pb = pn * binom(n0, b, q[0]);
                                if (pb == 0.0) continue;
                                out[ks[k].at(n0 - b + a, 0)] += pb;
                            }
                        }
                    } else {
                        double p0 = m.cls[0].r, p1 = m.cls[1].r, pr = 1.0 - p0 - p1;
                        for (int a0 = 0; a0 <= r; ++a0) {
                            for (int a1 = 0; a0 + a1 <= r; ++a1) {
                                int rest = r - a0 - a1;
                                double c = choose(r, a0) * choose(r - a0, a1);
                                double pn = c * std::pow(pr, rest) * std::pow(p0, a0) *
                                            std::pow(p1, a1);
                                if (pn == 0.0) continue;
                                for (int b0 = 0; b0 <= n0; ++b0) {
                                    double pb0 = pn * binom(n0, b0, q[0]);
                                    if (pb0 == 0.0) continue;
                                    for (int b1 = 0; b1 <= n1; ++b1) {
                                        double pb = pb0 * binom(n1, b1, q[1]);
                                        if (pb == 0.0) continue;
                                        out[ks[k].at(n0 - b0 + a0, n1 - b1 + a1)] += pb;
                                    }
                                }
                            }
                        }
                    }
                }
                // independent moves given the state: the product over kernels
                double* row = &P[(size_t)((ix[0] * S[1] + ix[1]) * S[2] + ix[2]) * N];
                for (int j0 = 0; j0 < S[0]; ++j0) {
                    if (mv[0][j0] == 0.0) continue;
                    for (int j1 = 0; j1 < S[1]; ++j1) {
                        const double p01 = nk > 1 ? mv[0][j0] * mv[1][j1] : mv[0][j0];
                        if (p01 == 0.0) continue;
                        double* r2 = row + (size_t)(j0 * S[1] + j1) * S[2];
                        if (nk > 2)
                            for (int j2 = 0; j2 < S[2]; ++j2) r2[j2] = p01 * mv[2][j2];
                        else
                            r2[0] = p01;
                    }
                }
            }
        }
    }
    std::vector<double> pi;
    stationary(P, N, pi);
    double den = 0.0, num[3] = {0.0, 0.0, 0.0};
    for (ix[0] = 0; ix[0] < S[0]; ++ix[0])
        for (ix[1] = 0; ix[1] < S[1]; ++ix[1])
            for (ix[2] = 0; ix[2] < S[2]; ++ix[2]) {
                double g = pi[(ix[0] * S[1] + ix[1]) * S[2] + ix[2]];
                int r[3] = {0, 0, 0};
                for (int k = 0; k < nk; ++k)
                    r[k] = w[k] - ks[k].n0[ix[k]] - ks[k].n1[ix[k]];
                den += g * std::max(r[0] + r[1] + r[2], 1);
                for (int k = 0; k < 3; ++k) num[k] += g * r[k];
            }
    for (int k = 0; k < nk; ++k) ipc_out[k] = num[k] / den;
}

bool profile_from_counters(const kl_counters& c, kl_profile* out) {
    const double counts[] = {c.waves, c.valu, c.salu, c.vmem, c.smem, c.lds, c.branch,
                             c.mfma, c.trans, c.dram_read, c.dram_write};
    for (double v : counts)
        if (!(v >= 0.0)) return false;
    if (!(c.waves > 0.0) || !(c.time_s > 0.0) || !(c.freq_hz > 0.0) || !(c.peak_bw > 0.0) ||
        c.n_cu < 1 || c.mfma + c.trans > c.valu)
        return false;
    // issue slots: a matrix instruction holds its SIMD for 16, a
    // transcendental for 4, anything else for 1
    const double slots = (c.valu - c.mfma - c.trans) + 16.0 * c.mfma + 4.0 * c.trans + c.salu +
                         c.vmem + c.smem + c.lds + c.branch;
    if (!(slots > 0.0)) return false;
    const double dram = c.dram_read + c.dram_write;
    const double r_lds = c.lds / slots;
    const double pur = slots / (c.time_s * c.freq_hz * (double)c.n_cu);
    out->r_mem = c.vmem / slots;
    out->mem_req = c.vmem > 0.0 ? std::max(1.0, dram / 64.0 / c.vmem) : 1.0;
    out->r_comp = r_lds > 1e-4 ? r_lds : 0.0;
    out->comp_pool = r_lds > 1e-4 ? 1 : 0;
    out->lat_comp = 1.0;
    out->instr_per_wave = slots / c.waves;
    out->pur = std::min(pur, 1.0);
    out->mur = dram / (c.time_s * c.peak_bw);
    out->solo_ipc = pur;
    return true;
}

double cp_value(const double* cipc, const double* solo, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += cipc[i] / solo[i];
    return 1.0 - 1.0 / s;
}

double solo_ipc(const kl_profile& p, const kl_config& cfg) {
    int w = p.max_wg_per_cu * p.waves_per_simd;
    if (w <= 0) return 0.0;
    KernelModel km = kernel_model(p, cfg);
    double ipc;
    chain_ipc(&km, &w, 1, cfg.beta, cfg.beta_lds, &ipc);
    return ipc;
}

bool ratio_feasible(const kl_profile& p1, const kl_profile& p2, const kl_config& cfg,
                    int b1, int b2) {
    if (b1 < 1 || b2 < 1 || b1 > p1.max_wg_per_cu || b2 > p2.max_wg_per_cu) return false;
    const int w1 = b1 * p1.waves_per_simd, w2 = b2 * p2.waves_per_simd;
    if (w1 + w2 > cfg.wmax) return false;
    if (w1 * p1.vgpr + w2 * p2.vgpr > cfg.vgpr_file) return false;
    return (int64_t)b1 * p1.lds_bytes + (int64_t)b2 * p2.lds_bytes <= cfg.lds_cu;
}

void surrogate_features(const kl_profile& p, int b, int wmax, float* f) {
    const double r = p.r_mem;
    const double alu = r > 0 ? (1.0 - r) / r : 64.0;
    f[0] = (float)r;
    f[1] = (float)(std::log2(std::min(64.0, std::max(1.0, alu))) / 6.0);
    f[2] = (float)(p.lds_bytes / 65536.0);
    f[3] = (float)(p.vgpr / 256.0);
    f[4] = p.access == 0 ? 1.f : 0.f;
    f[5] = p.access == 1 ? 1.f : 0.f;
    f[6] = p.access == 2 ? 1.f : 0.f;
    f[7] = (float)b / (float)(wmax > 0 ? wmax : 8);
}

// `same`: the two are instances of one kernel type.  Identical kernels
// lump (their joint chain depends on the total only), so every split of a
// total gives the same profit; only the balanced split of each total
// (b2 - b1 in {0, 1}) is searched.
static Ratio best_ratio_with(const kl_profile& p1, const kl_profile& p2,
                             const kl_config& cfg, double s1, double s2,
                             bool same = false) {
    Ratio best;
    double bkey0 = 0, bkey1 = 0;
    KernelModel km[2] = {kernel_model(p1, cfg), kernel_model(p2, cfg)};
    for (int b1 = 1; b1 <= p1.max_wg_per_cu; ++b1) {
        for (int b2 = 1; b2 <= p2.max_wg_per_cu; ++b2) {
            if (same && (b2 < b1 || b2 > b1 + 1)) continue;
            if (!ratio_feasible(p1, p2, cfg, b1, b2)) continue;
            int w[2] = {b1 * p1.waves_per_simd, b2 * p2.waves_per_simd};
            double c[2];
            chain_ipc(km, w, 2, cfg.beta, cfg.beta_lds, c);
            double solo[2] = {s1, s2};
            double cpv = cp_value(c, solo, 2);
            double n1 = (double)w[0] * p1.instr_per_wave;
            double n2 = (double)w[1] * p2.instr_per_wave;
            double T1 = n1 / c[0], T2 = n2 / c[1];
            double T1s = n1 / s1, T2s = n2 / s2;
            double k0, k1 = 0, val;
            if (cfg.ratio_mode == KL_MODE_BALANCED) {
                k0 = 1.0 - std::max(T1, T2) / (T1s + T2s);
                val = k0;
            } else if (cfg.ratio_mode == KL_MODE_CP) {
                k0 = cpv;
                val = cpv;
            } else {
                k0 = -std::fabs(T1 - T2);
                k1 = cpv;
                val = cpv;
            }
            bool better = !best.ok || k0 > bkey0 || (k0 == bkey0 && k1 > bkey1);
            if (better) {
                best.ok = true;
                best.b1 = b1;
                best.b2 = b2;
                best.value = val;
                best.cipc1 = c[0];
                best.cipc2 = c[1];
                bkey0 = k0;
                bkey1 = k1;
            }
        }
    }
    return best;
}

Ratio best_ratio(const kl_profile& p1, const kl_profile& p2, const kl_config& cfg) {
    return best_ratio_with(p1, p2, cfg, solo_ipc(p1, cfg), solo_ipc(p2, cfg));
}

bool triple_feasible(const kl_profile* const p[3], const kl_config& cfg, const int* b) {
    int waves = 0;
    int64_t vgpr = 0, lds = 0;
    for (int k = 0; k < 3; ++k) {
        if (b[k] < 1 || b[k] > p[k]->max_wg_per_cu) return false;
        const int w = b[k] * p[k]->waves_per_simd;
        waves += w;
        vgpr += (int64_t)w * p[k]->vgpr;
        lds += (int64_t)b[k] * p[k]->lds_bytes;
    }
    return waves <= cfg.wmax && vgpr <= cfg.vgpr_file && lds <= cfg.lds_cu;
}

Triple best_triple(const kl_profile* const p[3], const double* solo, const kl_config& cfg) {
    Triple best;
    double bkey0 = 0, bkey1 = 0;
    KernelModel km[3] = {kernel_model(*p[0], cfg), kernel_model(*p[1], cfg),
                         kernel_model(*p[2], cfg)};
    int b[3];
    for (b[0] = 1; b[0] <= p[0]->max_wg_per_cu; ++b[0])
        for (b[1] = 1; b[1] <= p[1]->max_wg_per_cu; ++b[1])
            for (b[2] = 1; b[2] <= p[2]->max_wg_per_cu; ++b[2]) {
                if (!triple_feasible(p, cfg, b)) continue;
                int w[3];
                for (int k = 0; k < 3; ++k) w[k] = b[k] * p[k]->waves_per_simd;
                double c[3];
                chain_ipc(km, w, 3, cfg.beta, cfg.beta_lds, c);
                const double cpv = cp_value(c, solo, 3);
                double T[3], Ts[3];
                for (int k = 0; k < 3; ++k) {
                    const double n = (double)w[k] * p[k]->instr_per_wave;
                    T[k] = n / c[k];
                    Ts[k] = n / solo[k];
                }
                const double tmax = std::max(std::max(T[0], T[1]), T[2]);
                const double tmin = std::min(std::min(T[0], T[1]), T[2]);
                double k0, k1 = 0, val;
                if (cfg.ratio_mode == KL_MODE_BALANCED) {
                    k0 = 1.0 - tmax / (Ts[0] + Ts[1] + Ts[2]);
                    val = k0;
                } else if (cfg.ratio_mode == KL_MODE_CP) {
                    k0 = cpv;
                    val = cpv;
                } else {
                    k0 = -(tmax - tmin);
                    k1 = cpv;
                    val = cpv;
                }
                if (!best.ok || k0 > bkey0 || (k0 == bkey0 && k1 > bkey1)) {
                    best.ok = true;
                    for (int k = 0; k < 3; ++k) {
                        best.b[k] = b[k];
                        best.cipc[k] = c[k];
                    }
                    best.value = val;
                    bkey0 = k0;
                    bkey1 = k1;
                }
            }
    return best;
}

// A pair is pruned when both its PUR and MUR differences are small; a
// kernel whose MUR is unknown (negative: profiled without memory counters)
// is never pruned.
bool pair_pruned(const kl_profile& a, const kl_profile& b, double ap, double am) {
    if (a.mur < 0 || b.mur < 0) return false;
    return std::fabs(a.pur - b.pur) < ap && std::fabs(a.mur - b.mur) < am;
}

double wg_rate(const kl_profile& p, double ipc, int n_cu) {
    return (double)n_cu * ipc / ((double)p.waves_per_simd * p.instr_per_wave);
}

void Planner::set_types(const std::vector<kl_profile>& t) {
    std::lock_guard<std::mutex> g(mu_);
    types_ = t;
    solo_.clear();
    pair_.clear();
    triple_.clear();
    scored_.clear();
}

void Planner::set_type(int idx, const kl_profile& p) {
    std::lock_guard<std::mutex> g(mu_);
    if ((int)types_.size() <= idx) types_.resize(idx + 1);
    types_[idx] = p;
    solo_.clear();
    pair_.clear();
    triple_.clear();
    scored_.clear();
}

void Planner::clear_scores() {
    std::lock_guard<std::mutex> g(mu_);
    scored_.clear();
}

double Planner::solo(int t) {
    auto it = solo_.find(t);
    if (it != solo_.end()) return it->second;
    auto t0 = std::chrono::steady_clock::now();
    double v = solo_ipc(types_[t], cfg_);
    model_us += std::chrono::duration<double, std::micro>(
                    std::chrono::steady_clock::now() - t0).count();
    solo_[t] = v;
    return v;
}

Ratio Planner::pair(int t1, int t2) {
    auto key = std::make_pair(t1, t2);
    auto it = pair_.find(key);
    if (it != pair_.end()) {
        ++cache_hits;
        return it->second;
    }
    double s1 = solo(t1), s2 = solo(t2);
    ++model_solves;
    auto t0 = std::chrono::steady_clock::now();
    Ratio r = best_ratio_with(types_[t1], types_[t2], cfg_, s1, s2, t1 == t2);
    model_us += std::chrono::duration<double, std::micro>(
                    std::chrono::steady_clock::now() - t0).count();
    pair_[key] = r;
    return r;
}

Triple Planner::triple(int t1, int t2, int t3) {
    int ts[3] = {t1, t2, t3};
    int key[3] = {t1, t2, t3};
    std::sort(key, key + 3);
    auto k = std::make_tuple(key[0], key[1], key[2]);
    auto it = triple_.find(k);
    Triple r;
    if (it != triple_.end()) {
        ++cache_hits;
        r = it->second;
    } else {
        const kl_profile* p[3] = {&types_[key[0]], &types_[key[1]], &types_[key[2]]};
        double s[3] = {solo(key[0]), solo(key[1]), solo(key[2])};
        ++model_solves;
        auto t0 = std::chrono::steady_clock::now();
        r = best_triple(p, s, cfg_);
        model_us += std::chrono::duration<double, std::micro>(
                        std::chrono::steady_clock::now() - t0).count();
        triple_[k] = r;
    }
    Triple out = r;
    for (int i = 0; i < 3; ++i) {
        const int pos = (int)(std::find(key, key + 3, ts[i]) - key);
        out.b[i] = r.b[pos];
        out.cipc[i] = r.cipc[pos];
    }
    return out;
}

Decision Planner::extend(const Decision& pair, const std::vector<PendingJob>& order) {
    if (cfg_.group_max < 3 || pair.j2 < 0) return pair;
    int ta = -1, tb = -1;
    for (const auto& j : order) {
        if (j.id == pair.j1) ta = j.type;
        if (j.id == pair.j2) tb = j.type;
    }
    if (ta < 0 || tb < 0 || ta == tb) return pair;
    Decision best = pair;
    for (const auto& c : order) {
        if (c.type == ta || c.type == tb) continue;
        Triple r = triple(ta, tb, c.type);
        if (!r.ok || !(r.value > best.value)) continue;
        best = pair;
        best.b1 = r.b[0];
        best.b2 = r.b[1];
        best.b3 = r.b[2];
        best.j3 = c.id;
        best.value = r.value;
        best.cipc1 = r.cipc[0];
        best.cipc2 = r.cipc[1];
        best.cipc3 = r.cipc[2];
    }
    return best;
}

Decision Planner::find(const std::vector<PendingJob>& pending,
                       const std::vector<std::pair<int, int>>* only_pairs) {
    return search(pending, only_pairs, 0, nullptr);
}

Decision Planner::find_ranked(const std::vector<PendingJob>& pending, int k,
                              const Scorer& score) {
    return search(pending, nullptr, k, &score);
}

bool Planner::candidates(const std::vector<PendingJob>& pending, std::vector<PendingJob>* out,
                         Decision* solo_d) {
    std::vector<PendingJob> v(pending);
    std::sort(v.begin(), v.end(),
              [](const PendingJob& a, const PendingJob& b) { return a.id < b.id; });
    // the earliest job of each type, by id (the two earliest with
    // pair_same_type, so that two instances of one kernel can pair)
    std::vector<PendingJob>& order = *out;
    order.clear();
    const int per_type = cfg_.pair_same_type ? 2 : 1;
    for (const auto& j : v) {
        int seen = 0;
        for (const auto& o : order) seen += o.type == j.type;
        if (seen < per_type) order.push_back(j);
    }
    const PendingJob first = order[0];
    solo_d->j1 = first.id;
    solo_d->j2 = -1;
    solo_d->b1 = types_[first.type].max_wg_per_cu;
    solo_d->cipc1 = solo(first.type);
    if (cfg_.min_pair_slots > 0) {
        // a job that would finish alone within min_pair_slots issue slots is
        // not worth a co-schedule: it only runs alone
        std::vector<PendingJob> keep;
        for (const auto& j : order) {
            const double t = j.wgs / wg_rate(types_[j.type], solo(j.type), cfg_.n_cu);
            if (!(t < cfg_.min_pair_slots)) keep.push_back(j);
        }
        order.swap(keep);
    }
    return order.size() >= 2;
}

void Planner::set_measures(const std::map<std::pair<int, int>, std::vector<Measure>>& m) {
    std::lock_guard<std::mutex> g(mu_);
    meas_ = m;
}

Decision Planner::find_opt(const std::vector<PendingJob>& pending) {
    std::lock_guard<std::mutex> g(mu_);
    Decision solo_d;
    if (pending.empty()) return solo_d;
    std::vector<PendingJob> order;
    if (!candidates(pending, &order, &solo_d)) return solo_d;
    Decision best;
    bool have = false;
    for (size_t x = 0; x < order.size(); ++x)
        for (size_t y = x + 1; y < order.size(); ++y) {
            auto it = meas_.find({order[x].type, order[y].type});
            if (it == meas_.end()) continue;
            for (const Measure& m : it->second) {
                const double cp = 1.0 - 1.0 / (m.rel1 + m.rel2);
                if (have && !(cp > best.value)) continue;
                have = true;
                best.j1 = order[x].id;
                best.j2 = order[y].id;
                best.b1 = m.b1;
                best.b2 = m.b2;
                best.value = cp;
                best.cipc1 = m.rel1 * solo(order[x].type);
                best.cipc2 = m.rel2 * solo(order[y].type);
            }
        }
    if (!have || best.value <= cfg_.cp_min) return solo_d;
    return best;
}

Decision Planner::find_random(const std::vector<PendingJob>& pending, uint64_t r_pair,
                              uint64_t r_ratio) {
    std::lock_guard<std::mutex> g(mu_);
    Decision solo_d;
    if (pending.empty()) return solo_d;
    std::vector<PendingJob> order;
    if (!candidates(pending, &order, &solo_d)) return solo_d;
    auto ratios = [&](const kl_profile& p1, const kl_profile& p2) {
        std::vector<std::pair<int, int>> r;
        for (int b1 = 1; b1 <= p1.max_wg_per_cu; ++b1)
            for (int b2 = 1; b2 <= p2.max_wg_per_cu; ++b2)
                if (ratio_feasible(p1, p2, cfg_, b1, b2)) r.emplace_back(b1, b2);
        return r;
    };
    std::vector<std::pair<size_t, size_t>> pairs;
    for (size_t x = 0; x < order.size(); ++x)
        for (size_t y = x + 1; y < order.size(); ++y)
            if (!ratios(types_[order[x].type], types_[order[y].type]).empty())
                pairs.emplace_back(x, y);
    if (pairs.empty()) return solo_d;
    const auto pr = pairs[r_pair % pairs.size()];
    const PendingJob& a = order[pr.first];
    const PendingJob& b = order[pr.second];
    const kl_profile& p1 = types_[a.type];
    const kl_profile& p2 = types_[b.type];
    const auto rat = ratios(p1, p2);
    const auto br = rat[r_ratio % rat.size()];
    auto t0 = std::chrono::steady_clock::now();
    KernelModel km[2] = {kernel_model(p1, cfg_), kernel_model(p2, cfg_)};
    int w[2] = {br.first * p1.waves_per_simd, br.second * p2.waves_per_simd};
    double c[2];
    chain_ipc(km, w, 2, cfg_.beta, cfg_.beta_lds, c);
    model_us += std::chrono::duration<double, std::micro>(
                    std::chrono::steady_clock::now() - t0).count();
    double s[2] = {solo(a.type), solo(b.type)};
    Decision d;
    d.j1 = a.id;
    d.j2 = b.id;
    d.b1 = br.first;
    d.b2 = br.second;
    d.value = cp_value(c, s, 2);
    d.cipc1 = c[0];
    d.cipc2 = c[1];
    return d;
}

Decision Planner::search(const std::vector<PendingJob>& pending,
                         const std::vector<std::pair<int, int>>* only_pairs, int k,
                         const Scorer* score) {
    std::lock_guard<std::mutex> g(mu_);
    Decision solo_d;
    if (pending.empty()) return solo_d;
    std::vector<PendingJob> order;
    if (!candidates(pending, &order, &solo_d)) return solo_d;

    const int n = (int)order.size();
    std::vector<std::pair<int, int>> pairs;
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) pairs.emplace_back(a, b);
    if (cfg_.use_prune) {
        double ap = cfg_.alpha_p, am = cfg_.alpha_m;
        std::vector<std::pair<int, int>> keep;
        for (int it = 0; it <= 4; ++it) {
            keep.clear();
            for (auto& pr : pairs)
                if (!pair_pruned(types_[order[pr.first].type],
                                 types_[order[pr.second].type], ap, am))
                    keep.push_back(pr);
            if (!keep.empty()) break;
            ap /= 2.0;
            am /= 2.0;
        }
        if (!keep.empty()) pairs.swap(keep);
    }
    if (score && (k == 0 || (int)pairs.size() > k)) {
        // scores depend on the two types only: score the pairs not seen yet
        std::vector<std::pair<const kl_profile*, const kl_profile*>> pp;
        std::vector<size_t> todo;
        for (size_t i = 0; i < pairs.size(); ++i) {
            const int ta = order[pairs[i].first].type, tb = order[pairs[i].second].type;
            if (scored_.count({ta, tb})) continue;
            todo.push_back(i);
            pp.emplace_back(&types_[ta], &types_[tb]);
        }
        std::vector<double> sc_new;
        std::vector<std::pair<int, int>> rat_new;
        bool ok = true;
        if (!pp.empty()) {
            ok = (*score)(pp, &sc_new, &rat_new) && sc_new.size() == pp.size() &&
                 rat_new.size() == pp.size();
            if (ok) {
                scored_pairs += (int64_t)pp.size();
                for (size_t j = 0; j < todo.size(); ++j) {
                    const auto& pr = pairs[todo[j]];
                    scored_[{order[pr.first].type, order[pr.second].type}] = {sc_new[j],
                                                                              rat_new[j]};
                }
            }
        } else {
            ++cache_hits;
        }
        std::vector<double> sc(pairs.size());
        std::vector<std::pair<int, int>> rat(pairs.size());
        if (ok)
            for (size_t i = 0; i < pairs.size(); ++i) {
                const auto& e = scored_.at({order[pairs[i].first].type, order[pairs[i].second].type});
                sc[i] = e.first;
                rat[i] = e.second;
            }
        if (ok) {
            std::vector<int> idx(pairs.size());
            for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
            // best scores first; ties keep submission order
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int x, int y) { return sc[x] > sc[y]; });
            if (k == 0) {
                // the surrogate decides: its best pair at its best ratio
                const int i = idx[0];
                const double S = sc[i];
                const bool same = order[pairs[i].first].type == order[pairs[i].second].type;
                const double floor = same ? std::min(cfg_.cp_min, -1.0) : cfg_.cp_min;
                if (rat[i].first < 1 || !(S > 0) || 1.0 - 1.0 / S <= floor) return solo_d;
                Decision d;
                d.j1 = order[pairs[i].first].id;
                d.j2 = order[pairs[i].second].id;
                d.b1 = rat[i].first;
                d.b2 = rat[i].second;
                d.value = 1.0 - 1.0 / S;
                return d;
            }
            std::vector<std::pair<int, int>> top;
            for (int i = 0; i < k; ++i) top.push_back(pairs[idx[i]]);
            pairs.swap(top);
        }
    }
    Decision best;
    bool have = false;
    for (auto& pr : pairs) {
        const PendingJob& a = order[pr.first];
        const PendingJob& b = order[pr.second];
        if (only_pairs) {
            bool listed = false;
            for (auto& op : *only_pairs)
                listed |= (op.first == a.type && op.second == b.type) ||
                          (op.first == b.type && op.second == a.type);
            if (!listed) continue;
        }
        // one evaluation per unordered type pair (its lower type first), so
        // that both orders of one pair get bit-identical values
        const bool sw = a.type > b.type;
        Ratio r = sw ? pair(b.type, a.type) : pair(a.type, b.type);
        if (!r.ok) continue;
        if (sw) {
            std::swap(r.b1, r.b2);
            std::swap(r.cipc1, r.cipc2);
        }
        // a pair of two instances of one kernel (predicted profit zero:
        // identical kernels lump) is held only to min(cp_min, -1), so that a
        // positive cp_min leaves it the last resort
        const double floor = a.type != b.type ? cfg_.cp_min : std::min(cfg_.cp_min, -1.0);
        if (!(r.value > floor)) continue;
        if (!have || r.value > best.value) {
            have = true;
            best.j1 = a.id;
            best.j2 = b.id;
            best.b1 = r.b1;
            best.b2 = r.b2;
            best.value = r.value;
            best.cipc1 = r.cipc1;
            best.cipc2 = r.cipc2;
        }
    }
    if (!have) return solo_d;
    // the surrogate's policy ranks pairs only
    return score ? best : extend(best, order);
}

}  // namespace kl
