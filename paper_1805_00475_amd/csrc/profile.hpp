// Optional per-launch device timing with hipEvents on the caller's stream,
// accumulated per kernel class together with the algorithmic bytes and
// multiply-adds of the launched steps.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.hpp"

namespace tn {

enum KernelClass { KC_GENERIC = 0, KC_STREAM = 1, KC_ROWDOT = 2, KC_MFMA = 3, KC_BATCH = 4, KC_DOT = 5, KC_DIGITS = 6,
                  KC_NARROW = 7 };

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> cls;
    std::vector<tn_launch_record> recs;     // every launch of the record, in order
    std::vector<tn_launch_record> pending;  // shapes of launches not yet timed
    tn_kernel_profile acc[TN_KERNEL_CLASSES]{};
    // shape of the step being launched (set by the launcher)
    int32_t cur_rA = 0, cur_rB = 0, cur_s = 0, cur_rC = 0, cur_G = 0;

    hipEvent_t ev() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    // top-level calls (tn_contract, tn_count, tn_count_batch) start a record
    void start(bool enable) {
        on = enable;
        used = 0;
        cls.clear();
        recs.clear();
        pending.clear();
        for (auto& a : acc) a = tn_kernel_profile{};
    }
    void before(hipStream_t s) {
        if (!on) return;
        hipEvent_t e = ev();
        if (e) hipEventRecord(e, s);
    }
    void account(int kc, double bytes, double macs) {
        acc[kc].launches += 1;
        acc[kc].bytes += bytes;
        acc[kc].macs += macs;
        tn_launch_record r{};
        r.kernel_class = kc;
        r.rA = cur_rA;
        r.rB = cur_rB;
        r.s = cur_s;
        r.rC = cur_rC;
        r.planes = cur_G;
        pending.push_back(r);
    }
    void after(hipStream_t s, int kc, const Step& st, int G, size_t es) {
        if (!on) return;
        hipEvent_t e = ev();
        if (e) hipEventRecord(e, s);
        cls.push_back(kc);
        account(kc, double(es) * G * (std::ldexp(1.0, st.rA) + std::ldexp(1.0, st.rB) + std::ldexp(1.0, st.rC)),
                double(G) * std::ldexp(1.0, st.rA + st.rB - st.s));
    }
    void after_raw(hipStream_t s, int kc, double bytes, double macs) {
        if (!on) return;
        hipEvent_t e = ev();
        if (e) hipEventRecord(e, s);
        cls.push_back(kc);
        account(kc, bytes, macs);
    }
    // after the stream is synchronized: add the recorded launch times and
    // recycle the events (the record stays open for further launches)
    void collect() {
        if (!on) return;
        for (size_t i = 0; i < cls.size() && 2 * i + 1 < used; ++i) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, pool[2 * i], pool[2 * i + 1]) == hipSuccess) acc[cls[i]].ms += ms;
            if (i < pending.size()) {
                pending[i].ms = ms;
                if (recs.size() < (size_t(1) << 20)) recs.push_back(pending[i]);
            }
        }
        used = 0;
        cls.clear();
        pending.clear();
    }
};

Profiler& profiler();

}  // namespace tn
