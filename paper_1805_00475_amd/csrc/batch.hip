// Batched counting: networks are built and ordered on host worker threads
// while the calling thread contracts the instances whose plans are ready,
// in submission order, on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "profile.hpp"

namespace tn {

namespace {

struct Slot {
    Network net;
    Plan plan;
    tn_status st = TN_OK;
    bool ready = false;
};

int worker_count(int n) {
    unsigned hw = std::thread::hardware_concurrency();
    int w = int(hw ? hw : 4);
    w = std::min(w, 16);
    return std::max(1, std::min(w, n));
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" tn_status tn_count_batch(const tn_formula* fs, int32_t n, tn_order_kind kind, uint64_t seed,
                                    const tn_contract_opts* opts, uint32_t* limbs, size_t cap_per,
                                    size_t* n_limbs, tn_plan_stats* stats) {
    if (n < 0 || (n > 0 && (!fs || !opts || !n_limbs))) return TN_EINVAL;
    if (n == 0) return TN_OK;
    std::vector<Slot> slots;
    try {
        slots.resize(size_t(n));
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    profiler().start(opts->flags & TN_FLAG_TIMING);
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        for (;;) {
            int32_t i = next.fetch_add(1);
            if (i >= n) return;
            Slot& s = slots[size_t(i)];
            s.st = build_network(&fs[i], s.net);
            if (s.st == TN_OK) s.st = make_order(s.net, kind, seed + uint64_t(i), nullptr, s.plan);
            {
                std::lock_guard<std::mutex> lk(mu);
                s.ready = true;
            }
            cv.notify_all();
        }
    };
    std::vector<std::thread> pool;
    const int W = worker_count(n);
    for (int w = 0; w < W; ++w) pool.emplace_back(work);
    tn_status first_err = TN_OK;
    for (int32_t i = 0; i < n; ++i) {
        Slot& s = slots[size_t(i)];
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return s.ready; });
        }
        tn_status st = s.st;
        std::vector<uint32_t> res, L;
        uint64_t v = 0;
        Resolved R;
        if (st == TN_OK) st = resolve(s.plan, opts, R);
        if (st == TN_OK) st = run_plan(s.net, s.plan, opts, R, res, &v);
        if (st == TN_OK) {
            if (R.u64) {
                L = {uint32_t(v), uint32_t(v >> 32)};
                while (L.size() > 1 && L.back() == 0) L.pop_back();
            } else {
                crt_limbs(res.data(), R.k, L);
            }
            n_limbs[i] = L.size();
            if (limbs && L.size() <= cap_per)
                std::copy(L.begin(), L.end(), limbs + size_t(i) * cap_per);
            else
                st = TN_EBUFSIZE;
        } else {
            n_limbs[i] = 0;
        }
        if (stats) stats[i] = s.plan.stats;
        if (st != TN_OK && first_err == TN_OK) first_err = st;
        // release the instance's memory early
        s.plan = Plan{};
        s.net = Network{};
    }
    for (auto& t : pool) t.join();
    return first_err;
}
