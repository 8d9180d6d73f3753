// Host-side entry points of the C ABI: build, order, plan queries, primes,
// CRT and status strings. The GPU entry points live in contract.hip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <thread>

#include "graph.hpp"
#include "internal.hpp"

namespace tn {

// randomized bisection trials of the judge: rounds of 16, one round by
// default on one host thread, kParallelRounds on several. On 1-in-3 at
// n = 300, alpha = 0.62 (six seeds, the best quarter of the trials
// reconfigured) 24 rounds give plans predicted 25 % cheaper than 8 (157
// against 211 ms), 16 rounds 15 %, 32 no more than 24; smaller instances
// stop earlier, by the time budget below.
constexpr int kTrialsPerRound = 16;
constexpr int kParallelRounds = 24;
// most rounds a caller may ask for (tn_order_rounds)
constexpr int kMaxRounds = 256;
// host microseconds of order search allowed per predicted device microsecond
constexpr double kSearchRatio = 2.0;
// predicted device microseconds above which the learned order's judged plan
// is handed to the full judge as its incumbent: a parallel round of
// bisection trials on 1-in-3 instances of n <= 250 costs at most about
// 10 ms of host time, so plans predicted above 50 ms are worth a search
constexpr double kEscalateUs = 50000.0;
// most host time spent reconfiguring plans, and its share of the predicted
// device time (measured on n = 200 cubic vertex-cover batches: 0.5 gives
// 45.1 counts/s against 44.2 at 2, 43.4 at 0.25 and 39.0 without
// reconfiguration). Every plan kept (the best quarter of the trials) is
// reconfigured within a kRefineWaves-th of that time when such a share is
// long enough for reconfiguration to settle (kSettleUs), else one plan per
// thread within the whole of it. Where a plan settles depends on the
// starting plan more than on the time given, so reconfiguring many plans
// pays (with 8 rounds, two plans per thread instead of one: predicted
// device time over six seeds 28 % lower on 1-in-3 at n = 300, alpha =
// 0.62, seed 1 and at n = 250, 7 % at n = 300, seed 4)
constexpr double kRefineCapUs = 100000.0;
constexpr double kRefineRatio = 0.5;
constexpr int kRefineWaves = 2;
// predicted device microseconds from which the judge waits for the tighter
// count bound it computes beside the trials (about 40 ms of one host thread
// at n = 300; one residue plane fewer saves a twelfth of the device time)
constexpr double kTightBoundUs = 50000.0;
// host time in which reconfiguration settles: 4-7 ms on plans of vertex
// cover n = 200, 8-11 ms on 1-in-3 n = 300; with less time per plan than
// this, one wave
constexpr double kSettleUs = 12000.0;

// Host threads for the bisection trials of one order search:
// TN_ORDER_THREADS if set, else the cores available (at most 16) less the
// one that Girvan-Newman takes beside them (on 16 cores, 15 trial threads
// finish the largest 1-in-3 search in 121 ms against 140 ms for 16).
int search_threads() {
    if (const char* e = std::getenv("TN_ORDER_THREADS")) {
        const int t = std::atoi(e);
        if (t >= 1) return std::min(t, 64);
    }
    const unsigned hw = std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    return int(hw > 2 ? hw - 1 : hw);
}

tn_status make_order(const Network& N, int32_t kind, uint64_t seed, const tn_model* model, Plan& out, int threads,
                     int rounds_asked) {
    try {
        auto plan_of = [&](int32_t k, Plan& p) -> tn_status {
            switch (k) {
                case TN_ORDER_GREEDY: return make_plan(N, order_greedy(N), k, p);
                case TN_ORDER_PARTITION: return make_plan(N, order_partition(N, seed), k, p);
                case TN_ORDER_COMMUNITY: return make_plan(N, order_community(N), k, p);
                default: return TN_EINVAL;
            }
        };
        if (kind == TN_ORDER_GREEDY || kind == TN_ORDER_PARTITION || kind == TN_ORDER_COMMUNITY)
            return plan_of(kind, out);
        if (kind == TN_ORDER_LEARNED_RAW) {
            bool ok = false;
            auto lm = order_learned(N, model, &ok);
            if (!ok) return TN_EINVAL;  // needs a model
            return make_plan(N, lm, TN_ORDER_LEARNED, out);
        }
        if (kind != TN_ORDER_BEST && kind != TN_ORDER_LEARNED) return TN_EINVAL;
        // the judge: the cheapest plan under the cost model (Sec. 4, lazy
        // evaluation); plans whose ranks exceed the cap are excluded
        bool have = false;
        tn_status last = TN_ERANK;
        if (kind == TN_ORDER_LEARNED) {
            // The learned order judged by the greedy order (Sec. 4: portfolio
            // with lazy cost prediction): both plans cost well under the
            // contraction they order, and the cheaper under the cost model is
            // kept (fallback = 1 when it is not the learned plan). When the
            // kept plan's predicted device time exceeds what a round of the
            // full judge's trials costs on the host, or neither fits the rank
            // cap, the full judge below runs with it as the incumbent.
            bool ok = false;
            auto lm = order_learned(N, model, &ok);
            Plan lp, gp;
            const bool lok = ok && make_plan(N, lm, TN_ORDER_LEARNED, lp) == TN_OK;
            const bool gok = make_plan(N, order_greedy(N), TN_ORDER_GREEDY, gp) == TN_OK;
            if (lok && (!gok || plan_cost(lp) <= plan_cost(gp))) {
                out = std::move(lp);
                have = true;
            } else if (gok) {
                out = std::move(gp);
                have = true;
            }
            if (have && plan_cost(out) <= kEscalateUs) {
                out.stats.fallback = out.stats.chosen != TN_ORDER_LEARNED;
                return TN_OK;
            }
        }
        // The tighter count bound (count_bound.cpp) of a boolean formula of
        // more than 64 bits' bound, on a thread of its own beside the
        // trials; joined (or cancelled) whatever way this function ends.
        struct TightBound {
            std::thread th;
            std::atomic<bool> cancel{false};
            int32_t bits = -1;
            std::vector<int32_t> ptr, lits;
            std::vector<uint8_t> kinds;
            void start(const Network& net) {
                if (net.f_ptr.empty() || net.n_vars <= 63 || net.count_bits <= 64) return;
                ptr = net.f_ptr;
                lits = net.f_lits;
                kinds = net.f_kinds;
                const int32_t nv = net.n_vars;
                th = std::thread([this, nv]() {
                    const tn_formula f{nv, int32_t(kinds.size()), ptr.data(), lits.data(), kinds.data()};
                    try {
                        bits = count_bound_bits_tight(&f, &cancel);
                    } catch (const std::bad_alloc&) {
                        bits = -1;  // no tighter bound: the network's stays
                    }
                });
            }
            int32_t finish(bool wait) {
                if (!th.joinable()) return -1;
                if (!wait) cancel = true;
                th.join();
                return bits;
            }
            ~TightBound() {
                if (th.joinable()) {
                    cancel = true;
                    th.join();
                }
            }
        } tight;
        // Candidates: greedy, community, and randomized recursive bisections
        // (each itself best-of-2 per level), in rounds of kTrialsPerRound
        // whatever the number of threads, so that the plan does not depend
        // on it. The cheapest `keep` of them (distinct costs, a quarter of
        // the trials) stay for reconfiguration, out being the cheapest.
        const int rounds = rounds_asked > 0 ? std::min(rounds_asked, kMaxRounds) : threads <= 1 ? 1 : kParallelRounds;
        const int trials = rounds * kTrialsPerRound;
        const size_t keep = size_t(std::max(kRefineWaves, trials / 4));
        const PartitionInput pin = partition_input(N);  // shared by every trial
        std::vector<Plan> pool;
        auto consider = [&](tn_status s2, Plan& p) {
            if (s2 != TN_OK) {
                last = s2;
                return;
            }
            const double c = plan_cost(p);
            if (!have || c < plan_cost(out)) {
                if (have) pool.push_back(std::move(out));
                out = std::move(p);
                have = true;
            } else {
                pool.push_back(std::move(p));
            }
            std::sort(pool.begin(), pool.end(), [](const Plan& x, const Plan& y) { return plan_cost(x) < plan_cost(y); });
            pool.erase(std::unique(pool.begin(), pool.end(),
                                   [](const Plan& x, const Plan& y) { return plan_cost(x) == plan_cost(y); }),
                       pool.end());
            while (!pool.empty() && plan_cost(pool.front()) == plan_cost(out)) pool.erase(pool.begin());
            if (pool.size() + 1 > keep) pool.resize(keep - 1);
        };
        // Time budget: on one thread the candidates come in increasing host
        // cost (greedy, four bisections, Girvan-Newman, more bisections), on
        // several the bisections of the first round always run; after that
        // the search stops once the host time spent on it exceeds
        // kSearchRatio times the predicted device time of the best plan so
        // far (all residue planes). The device cannot start before the first
        // plan of a batch is ready, so search time beyond the device time it
        // saves is a loss; measured on batches of n = 200 cubic vertex-cover
        // instances (small-modulus residues), two host microseconds per
        // predicted device microsecond give the shortest batch (one gives
        // worse plans, four and eight a longer wait for the first plan).
        const auto t0 = std::chrono::steady_clock::now();
        auto over_budget = [&]() {
            const double spent_us =
                std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
            if (rounds_asked > 0) return false;  // a fixed number of rounds
            return have && spent_us > kSearchRatio * plan_cost(out);
        };
        auto partition_trial = [&](int t) {
            Plan p;
            tn_status s2 = sketch_plan(N, order_partition(pin, seed * 0x9E3779B97F4A7C15ull + uint64_t(t)),
                                       TN_ORDER_PARTITION, p);
            consider(s2, p);
        };
        // trials first .. first + n - 1 on `threads` host threads; the judge sees
        // every plan, in trial order, so that which thread ran which trial
        // does not matter
        auto parallel_trials = [&](int first, int n, int at_least) {
            const int T = std::min(threads, n);
            std::vector<Plan> plans(static_cast<size_t>(n));
            std::vector<tn_status> st(static_cast<size_t>(n), TN_ERANK);
            std::atomic<int> next{0};
            // under the time budget, the threads stop taking trials (after
            // the first at_least) once the time spent exceeds kSearchRatio
            // times the cheapest plan found so far (the incumbent's or a
            // finished trial's); a trial taken always completes, so the
            // trials done are a prefix of the range
            std::atomic<bool> stop{false};
            std::mutex mu;
            double cheapest = have ? plan_cost(out) : std::numeric_limits<double>::infinity();
            auto work = [&]() {
                for (;;) {
                    if (stop.load() && next.load() >= at_least) break;
                    const int i = next.fetch_add(1);
                    if (i >= n) break;
                    Plan& p = plans[size_t(i)];
                    try {
                        st[size_t(i)] = sketch_plan(
                            N, order_partition(pin, seed * 0x9E3779B97F4A7C15ull + uint64_t(first + i)),
                            TN_ORDER_PARTITION, p);
                    } catch (const std::bad_alloc&) {
                        st[size_t(i)] = TN_ENOMEM;
                    }
                    if (rounds_asked > 0) continue;
                    double c;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        if (st[size_t(i)] == TN_OK) cheapest = std::min(cheapest, plan_cost(p));
                        c = cheapest;
                    }
                    const double spent_us =
                        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
                    if (spent_us > kSearchRatio * c) stop.store(true);
                }
            };
            std::vector<std::thread> pool;
            for (int w = 1; w < T; ++w) pool.emplace_back(work);
            work();
            for (auto& th : pool) th.join();
            const int done = std::min(n, next.load());
            for (int i = 0; i < done; ++i) consider(st[size_t(i)], plans[size_t(i)]);
        };
        if (kind != TN_ORDER_LEARNED) {
            Plan p;
            consider(plan_of(TN_ORDER_GREEDY, p), p);
        }
        if (threads <= 1) {
            partition_trial(0);
            partition_trial(1);
            for (int t = 2; t < 4 && !over_budget(); ++t) partition_trial(t);
            if (!over_budget()) {
                Plan p;
                consider(plan_of(TN_ORDER_COMMUNITY, p), p);
            }
            for (int t = 4; t < trials && !over_budget(); ++t) partition_trial(t);
        } else {
            // every trial in one pass: at least a round, then as many as the
            // time budget allows; Girvan-Newman runs beside them on a thread
            // of its own (on the largest 1-in-3 configuration it takes as
            // long as ten rounds)
            Plan gnp;
            tn_status gns = TN_EINVAL;
            std::thread gn([&]() {
                try {
                    gns = plan_of(TN_ORDER_COMMUNITY, gnp);
                } catch (const std::bad_alloc&) {
                    gns = TN_ENOMEM;
                }
            });
            tight.start(N);
            parallel_trials(0, trials, kTrialsPerRound);
            gn.join();
            consider(gns, gnp);
        }
        // local reconfiguration of the contraction trees of the winner and
        // of the runners-up kept (kRefineWaves per host thread, in
        // parallel, each with the same share of the time budget); the
        // cheapest result wins
        if (have && out.merges.size() > 2) {
            // every plan kept, each within a kRefineWaves-th of the budget,
            // when that still gives it the time to settle; else one plan per
            // thread, each within the whole budget. A fixed number of rounds
            // reconfigures every plan kept until it settles (at most six
            // sweeps), so that the plan depends on nothing else.
            const double total = std::min(kRefineCapUs, kRefineRatio * plan_cost(out));
            const bool fixed = rounds_asked > 0;
            const bool settle = fixed || total >= kRefineWaves * kSettleUs;
            const size_t ncand = settle ? keep : size_t(std::max(1, threads));
            const double budget = fixed ? std::numeric_limits<double>::infinity()
                                        : settle ? total / kRefineWaves : total;
            std::vector<const Plan*> cand{&out};
            for (const Plan& p : pool)
                if (cand.size() < ncand) cand.push_back(&p);
            std::vector<Plan> ref(cand.size());
            std::vector<tn_status> rs(cand.size(), TN_EINVAL);
            std::atomic<size_t> next{0};
            auto work = [&]() {
                for (;;) {
                    const size_t i = next.fetch_add(1);
                    if (i >= cand.size()) break;
                    try {
                        rs[i] = sketch_plan(N, refine_order(N, cand[i]->merges, budget), cand[i]->stats.chosen, ref[i]);
                    } catch (const std::bad_alloc&) {
                        rs[i] = TN_ENOMEM;
                    }
                }
            };
            std::vector<std::thread> pool_threads;
            // (with several threads, Girvan-Newman's is free again by now)
            const int T = std::min<int>(threads > 1 ? threads + 1 : 1, int(cand.size()));
            for (int t = 1; t < T; ++t) pool_threads.emplace_back(work);
            work();
            for (auto& th : pool_threads) th.join();
            int bi = -1;
            double bc = plan_cost(out);
            for (size_t i = 0; i < ref.size(); ++i)
                if (rs[i] == TN_OK && plan_cost(ref[i]) < bc) {
                    bc = plan_cost(ref[i]);
                    bi = int(i);
                }
            if (bi >= 0) {
                ref[size_t(bi)].stats.refined = 1;
                out = std::move(ref[size_t(bi)]);
            }
        }
        // trials and reconfigured plans are sketches (merges and cost): the
        // winner gets its layouts, steps and arena
        if (have && out.sketch) {
            const int32_t refined = out.stats.refined;
            const tn_status s2 = make_plan(N, out.merges, out.stats.chosen, out);
            if (s2 != TN_OK) return s2;
            out.stats.refined = refined;
        }
        // the tighter bound: waited for when the plan is costly enough for
        // a residue plane to matter (always with a fixed number of rounds,
        // so that the plan depends on nothing else), else used only if done
        {
            const bool wait = rounds_asked > 0 || (have && plan_cost(out) >= kTightBoundUs);
            const int32_t tb = tight.finish(wait);
            if (have && tb >= 0 && out.count_bits > 64 && tb < out.count_bits) {
                out.count_bits = std::max<int32_t>(64, tb);
                out.cost_us = -1;
                out.cost_us = plan_cost(out);
                out.stats.log2_cost = out.cost_us > 0 ? std::log2(out.cost_us) : 0.0;
            }
        }
        if (kind == TN_ORDER_LEARNED && have) out.stats.fallback = out.stats.chosen != TN_ORDER_LEARNED;
        return have ? TN_OK : last;
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
}

}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_build(const tn_formula* f, tn_network** out) {
    if (!f || !out) return TN_EINVAL;
    *out = nullptr;
    tn_network* h = new (std::nothrow) tn_network;
    if (!h) return TN_ENOMEM;
    tn_status st = build_network(f, h->net);
    if (st != TN_OK) {
        delete h;
        return st;
    }
    *out = h;
    return TN_OK;
}

void tn_network_free(tn_network* net) { delete net; }

tn_status tn_build_ex(const tn_formula* f, uint32_t flags, tn_network** out) {
    if (!out || (flags & ~uint32_t(TN_BUILD_RING_COPY | TN_BUILD_SPLIT_CLAUSES))) return TN_EINVAL;
    tn_status st = tn_build(f, out);
    if (st != TN_OK || !flags) return st;
    st = reduce_degree((*out)->net, flags);
    if (st != TN_OK) {
        delete *out;
        *out = nullptr;
    }
    return st;
}

tn_status tn_build_csp(const tn_csp* c, uint32_t flags, tn_network** out) {
    if (!c || !out || (flags & ~uint32_t(TN_BUILD_RING_COPY | TN_BUILD_SPLIT_CLAUSES))) return TN_EINVAL;
    *out = nullptr;
    tn_network* h = new (std::nothrow) tn_network;
    if (!h) return TN_ENOMEM;
    tn_status st = build_csp(c, h->net);
    if (st == TN_OK && flags) st = reduce_degree(h->net, flags);
    if (st != TN_OK) {
        delete h;
        return st;
    }
    *out = h;
    return TN_OK;
}

tn_status tn_network_ranks(const tn_network* net, int32_t* max_init_rank, int32_t* count_bits) {
    if (!net) return TN_EINVAL;
    int32_t r = 0;
    for (const auto& t : net->net.t) r = std::max(r, int32_t(t.bonds.size()));
    if (max_init_rank) *max_init_rank = r;
    if (count_bits) *count_bits = net->net.count_bits;
    return TN_OK;
}

tn_status tn_network_info(const tn_network* net, int32_t* n_tensors, int32_t* n_bonds) {
    if (!net) return TN_EINVAL;
    if (n_tensors) *n_tensors = int32_t(net->net.t.size());
    if (n_bonds) *n_bonds = int32_t(net->net.bond_end.size());
    return TN_OK;
}

tn_status tn_order(const tn_network* net, tn_order_kind kind, uint64_t seed, const tn_model* model,
                   tn_plan** out, tn_plan_stats* stats) {
    return tn_order_rounds(net, kind, seed, model, 0, out, stats);
}

tn_status tn_order_rounds(const tn_network* net, tn_order_kind kind, uint64_t seed, const tn_model* model,
                          int32_t rounds, tn_plan** out, tn_plan_stats* stats) {
    if (!net || !out || rounds < 0 || rounds > kMaxRounds) return TN_EINVAL;
    *out = nullptr;
    tn_plan* h = new (std::nothrow) tn_plan;
    if (!h) return TN_ENOMEM;
    tn_status st = make_order(net->net, kind, seed, model, h->plan, search_threads(), rounds);
    if (st != TN_OK) {
        delete h;
        return st;
    }
    if (stats) *stats = h->plan.stats;
    *out = h;
    return TN_OK;
}

void tn_plan_free(tn_plan* plan) { delete plan; }

tn_status tn_plan_steps(const tn_plan* plan, int32_t* pairs, int32_t cap, int32_t* n_steps) {
    if (!plan) return TN_EINVAL;
    const int32_t n = int32_t(plan->plan.merges.size());
    if (n_steps) *n_steps = n;
    if (!pairs) return TN_OK;
    if (cap < n) return TN_EBUFSIZE;
    for (int32_t k = 0; k < n; ++k) {
        pairs[2 * k] = plan->plan.merges[k].first;
        pairs[2 * k + 1] = plan->plan.merges[k].second;
    }
    return TN_OK;
}

tn_status tn_plan_verify(const tn_plan* plan) {
    if (!plan) return TN_EINVAL;
    return verify_plan(plan->plan);
}

tn_status tn_primes(int32_t k, uint32_t* out) {
    if (k < 0 || k > TN_MAX_PRIMES || (k > 0 && !out)) return TN_EINVAL;
    const auto& P = prime_table(k);
    std::copy(P.begin(), P.begin() + k, out);
    return TN_OK;
}

tn_status tn_primes_for(int32_t n_vars, int32_t* k) {
    if (n_vars < 0 || !k) return TN_EINVAL;
    const int32_t need = primes_needed(n_vars);
    if (need > TN_MAX_PRIMES) return TN_EINVAL;
    *k = need;
    return TN_OK;
}

tn_status tn_crt(const uint32_t* residues, int32_t k, uint32_t* limbs, size_t cap, size_t* n_limbs) {
    if (k <= 0 || k > TN_MAX_PRIMES || !residues || !n_limbs) return TN_EINVAL;
    const auto& P = prime_table(k);
    for (int32_t i = 0; i < k; ++i)
        if (residues[i] >= P[i]) return TN_EINVAL;
    std::vector<uint32_t> L;
    crt_limbs(residues, k, L);
    *n_limbs = L.size();
    if (!limbs || cap < L.size()) return TN_EBUFSIZE;
    std::copy(L.begin(), L.end(), limbs);
    return TN_OK;
}

tn_status tn_crt_moduli(const uint32_t* residues, const uint32_t* moduli, int32_t k, uint32_t* limbs, size_t cap,
                        size_t* n_limbs) {
    if (k <= 0 || k > 4096 || !residues || !moduli || !n_limbs) return TN_EINVAL;
    for (int32_t i = 0; i < k; ++i) {
        if (moduli[i] < 2 || residues[i] >= moduli[i]) return TN_EINVAL;
        for (int32_t j = 0; j < i; ++j) {
            uint32_t a = moduli[i], b = moduli[j];
            while (b) {
                const uint32_t t = a % b;
                a = b;
                b = t;
            }
            if (a != 1) return TN_EINVAL;  // not coprime: no unique recombination
        }
    }
    std::vector<uint32_t> L;
    try {
        crt_limbs(residues, moduli, k, L);
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    *n_limbs = L.size();
    if (!limbs || cap < L.size()) return TN_EBUFSIZE;
    std::copy(L.begin(), L.end(), limbs);
    return TN_OK;
}

const char* tn_status_str(tn_status s) {
    switch (s) {
        case TN_OK: return "ok";
        case TN_EINVAL: return "invalid argument";
        case TN_ENOMEM: return "out of host memory";
        case TN_EHIP: return "HIP runtime error";
        case TN_ETOOBIG: return "plan does not fit the workspace";
        case TN_ERANK: return "tensor rank above the supported maximum";
        case TN_EBUFSIZE: return "output buffer too small";
        case TN_EUNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char* tn_version(void) { return "tn-mi355x 0.1 (gfx950)"; }

}  // extern "C"

// ------------------------------------------------------------ learned order
#include "learned.hpp"

extern "C" {

int32_t tn_model_param_count(void) { return tn::kParams; }

tn_status tn_model_create(const float* params, tn_model** out) {
    if (!out) return TN_EINVAL;
    *out = nullptr;
    tn_model* m = new (std::nothrow) tn_model;
    if (!m) return TN_ENOMEM;
    try {
        m->params.assign(size_t(tn::kParams), 0.0f);
    } catch (const std::bad_alloc&) {
        delete m;
        return TN_ENOMEM;
    }
    if (params) std::copy(params, params + tn::kParams, m->params.begin());
    *out = m;
    return TN_OK;
}

void tn_model_free(tn_model* m) { delete m; }

tn_status tn_model_get(const tn_model* m, float* params) {
    if (!m || !params) return TN_EINVAL;
    std::copy(m->params.begin(), m->params.end(), params);
    return TN_OK;
}

tn_status tn_model_score(const tn_model* m, const float* x, int32_t n, float* y) {
    if (!m || n < 0 || (n > 0 && (!x || !y))) return TN_EINVAL;
    std::vector<float> w1t, w2t;
    tn::transpose_params(m->params.data(), w1t, w2t);
    for (int32_t i = 0; i < n; ++i)
        y[i] = tn::mlp_score_t(m->params.data(), w1t.data(), w2t.data(), x + size_t(i) * tn::kFeatures);
    return TN_OK;
}

tn_status tn_trace(const tn_network* net, const tn_plan* teacher, float* feats, uint8_t* labels, int32_t* groups,
                   int64_t cap_rows, int32_t cap_groups, int64_t* n_rows, int32_t* n_groups) {
    if (!net || !teacher || !n_rows || !n_groups) return TN_EINVAL;
    std::vector<float> f;
    std::vector<uint8_t> l;
    std::vector<int32_t> g;
    tn_status st;
    try {
        st = tn::trace_order(net->net, teacher->plan.merges, f, l, g);
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    if (st != TN_OK) return st;
    *n_rows = int64_t(l.size());
    *n_groups = int32_t(g.size()) - 1;
    if (!feats || !labels || !groups || cap_rows < int64_t(l.size()) || cap_groups < int32_t(g.size()))
        return TN_EBUFSIZE;
    std::copy(f.begin(), f.end(), feats);
    std::copy(l.begin(), l.end(), labels);
    std::copy(g.begin(), g.end(), groups);
    return TN_OK;
}

}  // extern "C"
