// Batched counting of many formulas of uneven size.
//
// Host worker threads build and order the networks while the calling thread
// packs ready instances into sub-batches that fit the workspace. A sub-batch
// runs as a sequence of waves: wave L holds every step of level L (the
// longest chain of steps feeding it) of every instance and every residue
// plane. The small steps of a wave are tiles of one persistent launch that
// walks a device work list; the large steps of the wave get their own
// kernels (streaming, MFMA, split-K). The whole sequence is captured into a
// hipGraph and replayed once; a final gather collects every instance's
// scalar per plane for one device-to-host copy, followed by CRT per instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "profile.hpp"

namespace tn {

namespace {

// One tile of one small step of one instance in one residue plane.
struct BItem {
    const void* A;
    const void* B;
    void* C;
    uint64_t maskA, maskB;
    uint64_t c0;         // first output entry of the tile
    uint32_t p, r2;      // modulus and 2^32 mod p (RNS planes)
    uint32_t r16;        // 2^16 mod p (small moduli)
    float pinv;          // 1 / p (small moduli)
    int32_t s, tlog;     // shared bonds; log2 of the tile's outputs
    int32_t el, pad;     // element kind (kernels.hpp)
};

// Persistent wave kernel: a fixed grid walks the wave's work list; each
// wavefront takes one tile at a time, one lane per output entry (bit
// gathers), so a block serves four small tiles at once.
__global__ __launch_bounds__(256) void k_batch(const BItem* items, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = int64_t(gridDim.x) * (blockDim.x >> 6);
    for (int64_t i = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n; i += nw) {
        const BItem it = items[i];
        const uint64_t nOut = uint64_t(1) << it.tlog;
        const uint64_t K = uint64_t(1) << it.s;
        for (uint64_t t = lane; t < nOut; t += 64) {
            const uint64_t c = it.c0 + t;
            const uint64_t xa = pext64(c, it.maskA) << it.s, xb = pext64(c, it.maskB) << it.s;
            if (it.el == EL_U64) {
                const uint64_t* A = static_cast<const uint64_t*>(it.A) + xa;
                const uint64_t* B = static_cast<const uint64_t*>(it.B) + xb;
                uint64_t acc = 0;
                for (uint64_t z = 0; z < K; ++z) acc += A[z] * B[z];
                static_cast<uint64_t*>(it.C)[c] = acc;
            } else if (it.el == EL_I8) {
                const int8_t* A = static_cast<const int8_t*>(it.A) + xa;
                const int8_t* B = static_cast<const int8_t*>(it.B) + xb;
                const ModSmall ms{int32_t(it.p), it.r2, it.r16, it.pinv};
                int64_t acc = 0;
                for (uint64_t z = 0; z < K; ++z) acc += int32_t(A[z]) * int32_t(B[z]);
                static_cast<int8_t*>(it.C)[c] = int8_t(ms.center64(acc));
            } else {
                const uint32_t* A = static_cast<const uint32_t*>(it.A) + xa;
                const uint32_t* B = static_cast<const uint32_t*>(it.B) + xb;
                const ModP m{it.p, it.r2};
                uint64_t acc = 0;
                uint32_t n3 = 0;
                for (uint64_t z = 0; z < K; ++z) {
                    acc += uint64_t(A[z]) * B[z];
                    if (++n3 == 3) {
                        acc = m.fold(acc);
                        n3 = 0;
                    }
                }
                static_cast<uint32_t*>(it.C)[c] = m.finish(acc);
            }
        }
    }
}

struct GItem {
    const void* src;
    int64_t el;  // element kind
};

// int8 residues are returned sign-extended (centred)
__global__ void k_gather(const GItem* g, uint64_t* out, int64_t n) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const void* src = g[j].src;
    out[j] = g[j].el == EL_U64  ? *static_cast<const uint64_t*>(src)
             : g[j].el == EL_I8 ? uint64_t(int64_t(*static_cast<const int8_t*>(src)))
                                : *static_cast<const uint32_t*>(src);
}

struct Inst {
    Network net;
    Plan plan;
    tn_status st = TN_OK;
    bool ready = false;
    Resolved R;
    int P = 0;                // residue planes (1 for 64-bit)
    int64_t es = 4;
    int64_t init_bytes = 0, arena_bytes = 0;  // arena_bytes: the wave layout
    int64_t n_items = 0;
    int64_t init_off = 0, arena_off = 0;  // in the sub-batch layout
    std::vector<uint32_t> res;
    uint64_t u64v = 0;
    bool host_only = false;   // the count is known without device work
    std::vector<uint8_t> dig;  // per step: digit-plane bits of launch_step
    int el() const { return R.u64 ? EL_U64 : R.i8 ? EL_I8 : EL_U32; }
};

int worker_count(int n) {
    unsigned hw = std::thread::hardware_concurrency();
    int w = int(hw ? hw : 4);
    w = std::min(w, 16);
    return std::max(1, std::min(w, n));
}

constexpr int kTileLog = 8;  // outputs per wave tile (2^8, four per lane)
// milliseconds without a newly ordered instance after which the pending
// sub-batch is contracted
constexpr int kIdleFlushMs = 2;

// Steps small enough for the wave kernel; larger or wider ones get the
// shape-specific kernels of the single-instance path.
bool small_step(const Step& st) {
    return st.rC <= 14 && st.s <= 6 && st.rA <= 16 && st.rB <= 16;
}

int64_t items_of(const Plan& plan, int P) {
    int64_t n = 0;
    for (const Step& st : plan.steps)
        if (small_step(st)) n += (int64_t(1) << std::max(0, st.rC - kTileLog)) * P;
    return n;
}

struct SubBatch {
    std::vector<int32_t> ids;
    int64_t init_total = 0, arena_total = 0, items = 0, gathers = 0;
};

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Runs one sub-batch: every instance in it has a plan and fits the layout.
tn_status run_sub(std::vector<Inst>& ins, const SubBatch& sb, const tn_contract_opts* o) {
    hipStream_t stream = static_cast<hipStream_t>(o->stream);
    char* base = static_cast<char*>(o->workspace);
    const bool timing = o->flags & TN_FLAG_TIMING;
    const bool use_graph = !(o->flags & TN_FLAG_NO_GRAPH) && !timing;
    // layout: [init regions][arenas][scratch][items][gather list][results]
    int64_t off = 0;
    for (int32_t i : sb.ids) {
        ins[i].init_off = off;
        off += ins[i].init_bytes;
    }
    const int64_t init_total = off;
    for (int32_t i : sb.ids) {
        ins[i].arena_off = off;
        off += ins[i].P * ins[i].arena_bytes;
    }
    const int64_t scratch_off = off;
    off += kMaxGroup * kScratchPerPrime;
    const int64_t items_off = off;
    off += align_up(sb.items * int64_t(sizeof(BItem)), 256);
    const int64_t gather_off = off;
    off += align_up(sb.gathers * int64_t(sizeof(GItem)), 256);
    const int64_t result_off = off;
    off += align_up(sb.gathers * 8, 256);
    if (off > int64_t(o->workspace_bytes)) return TN_ETOOBIG;

    // host images of the init regions, the work list and the gather list
    std::vector<uint8_t> init(size_t(std::max<int64_t>(init_total, 1)), 0);
    int max_level = 0;
    for (int32_t i : sb.ids) {
        fill_init(ins[i].net, ins[i].plan, ins[i].el(), init.data() + ins[i].init_off);
        for (const Step& st : ins[i].plan.steps) max_level = std::max(max_level, st.level);
    }
    std::vector<std::vector<BItem>> wave_items(size_t(max_level) + 1);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> wave_big(size_t(max_level) + 1);
    std::vector<GItem> gathers;
    std::vector<std::pair<int32_t, int>> gather_of;  // (instance, plane)
    for (int32_t i : sb.ids) {
        Inst& I = ins[i];
        // digit-plane hand-over between matrix-core steps (small steps run
        // in the wave kernel)
        std::vector<KernelClass> cls(I.plan.steps.size());
        for (size_t k = 0; k < cls.size(); ++k)
            cls[k] = small_step(I.plan.steps[k]) ? KC_BATCH : choose_class(I.plan.steps[k], I.el(), o->flags);
        I.dig = digit_plan(I.plan, cls, I.el());
        char* ib = base + I.init_off;
        for (int32_t k = 0; k < int32_t(I.plan.steps.size()); ++k) {
            const Step& st = I.plan.steps[k];
            if (!small_step(st)) {
                wave_big[st.level].push_back({i, k});
                continue;
            }
            const uint64_t cmask = (uint64_t(1) << st.rC) - 1;
            const int tlog = std::min(st.rC, kTileLog);
            for (int q = 0; q < I.P; ++q) {
                char* ab = base + I.arena_off + q * I.arena_bytes;
                BItem it{};
                it.A = st.initA ? ib + st.woffA * I.es : ab + st.woffA * I.es;
                it.B = st.initB ? ib + st.woffB * I.es : ab + st.woffB * I.es;
                it.C = ab + st.woffC * I.es;
                it.maskA = st.maskA;
                it.maskB = cmask & ~st.maskA;
                it.s = st.s;
                it.tlog = tlog;
                it.el = I.el();
                if (!I.R.u64) {
                    it.p = I.R.primes[q];
                    it.r2 = uint32_t((uint64_t(1) << 32) % it.p);
                    it.r16 = uint32_t(65536u % it.p);
                    it.pinv = 1.0f / float(it.p);
                }
                for (uint64_t c0 = 0; c0 < (uint64_t(1) << st.rC); c0 += uint64_t(1) << tlog) {
                    it.c0 = c0;
                    wave_items[st.level].push_back(it);
                }
            }
        }
        const Step& last = I.plan.steps.back();
        for (int q = 0; q < I.P; ++q) {
            gathers.push_back({base + I.arena_off + q * I.arena_bytes + last.woffC * I.es, int64_t(I.el())});
            gather_of.push_back({i, q});
        }
    }
    std::vector<BItem> flat;
    flat.reserve(size_t(sb.items));
    std::vector<int64_t> wave_off(wave_items.size() + 1, 0);
    for (size_t L = 0; L < wave_items.size(); ++L) {
        wave_off[L] = int64_t(flat.size());
        flat.insert(flat.end(), wave_items[L].begin(), wave_items[L].end());
    }
    wave_off[wave_items.size()] = int64_t(flat.size());
    const BItem* d_items = reinterpret_cast<const BItem*>(base + items_off);
    auto fail = [&](tn_status s) {
        (void)hipStreamSynchronize(stream);
        return s;
    };
    if (hipMemcpyAsync(base, init.data(), size_t(init_total), hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(TN_EHIP);
    if (!flat.empty() && hipMemcpyAsync(base + items_off, flat.data(), flat.size() * sizeof(BItem),
                                        hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(TN_EHIP);
    if (!gathers.empty() && hipMemcpyAsync(base + gather_off, gathers.data(), gathers.size() * sizeof(GItem),
                                           hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(TN_EHIP);

    Profiler& prof = profiler();
    hipGraph_t graph = nullptr;
    bool capturing = use_graph && stream != nullptr;  // the null stream cannot be captured
    if (capturing && hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        capturing = false;  // launch the waves directly
    }
    hipError_t err = hipSuccess;
    for (size_t L = 1; L < wave_items.size() && err == hipSuccess; ++L) {
        const int64_t n = wave_off[L + 1] - wave_off[L];
        if (n > 0) {
            double bytes = 0, macs = 0;
            if (timing)
                for (int64_t k = wave_off[L]; k < wave_off[L + 1]; ++k) {
                    const BItem& it = flat[size_t(k)];
                    const double es = double(elem_size(it.el));
                    bytes += es * std::ldexp(1.0, it.tlog) * 1.0;  // outputs written
                    macs += std::ldexp(1.0, it.tlog + it.s);
                }
            prof.cur_rA = prof.cur_rB = prof.cur_s = prof.cur_rC = 0;
            prof.cur_G = int32_t(n);  // tiles in the wave
            prof.before(stream);
            const uint32_t grid = uint32_t(std::min<int64_t>((n + 3) / 4, 4096));
            hipLaunchKernelGGL(k_batch, dim3(grid), dim3(256), 0, stream, d_items + wave_off[L], n);
            err = hipGetLastError();
            prof.after_raw(stream, KC_BATCH, bytes, macs);
        }
        for (const auto& bk : wave_big[L]) {
            Inst& I = ins[bk.first];
            Step st = I.plan.steps[bk.second];
            st.offA = st.woffA;
            st.offB = st.woffB;
            st.offC = st.woffC;
            for (int g0 = 0; g0 < I.P && err == hipSuccess; g0 += kMaxGroup) {
                const int gn = std::min(kMaxGroup, I.P - g0);
                KernelClass kc = KC_GENERIC;
                err = launch_step(st, I.el(), o->flags, I.R.u64 ? nullptr : I.R.primes.data() + g0, gn,
                                  base + I.init_off, base + I.arena_off + g0 * I.arena_bytes, I.arena_bytes / I.es,
                                  base + scratch_off, stream, &kc, -1, I.dig[size_t(bk.second)]);
            }
        }
    }
    if (err == hipSuccess && !gathers.empty()) {
        const int64_t n = int64_t(gathers.size());
        hipLaunchKernelGGL(k_gather, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, stream,
                           reinterpret_cast<const GItem*>(base + gather_off),
                           reinterpret_cast<uint64_t*>(base + result_off), n);
        err = hipGetLastError();
    }
    if (capturing) {
        hipError_t e2 = hipStreamEndCapture(stream, &graph);
        if (err == hipSuccess) err = e2;
        if (err == hipSuccess) {
            hipGraphExec_t exec = nullptr;
            err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (err == hipSuccess) err = hipGraphLaunch(exec, stream);
            if (err == hipSuccess) err = hipStreamSynchronize(stream);
            if (exec) (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
    if (err != hipSuccess) return fail(TN_EHIP);
    std::vector<uint64_t> out(gathers.size(), 0);
    if (!out.empty() && hipMemcpyAsync(out.data(), base + result_off, out.size() * 8, hipMemcpyDeviceToHost,
                                       stream) != hipSuccess)
        return fail(TN_EHIP);
    if (hipStreamSynchronize(stream) != hipSuccess) return TN_EHIP;
    prof.collect();
    for (size_t j = 0; j < out.size(); ++j) {
        Inst& I = ins[gather_of[j].first];
        const int q = gather_of[j].second;
        if (I.R.u64) {
            I.u64v = out[j];
        } else if (I.R.i8) {
            const int64_t m = I.R.primes[size_t(q)], c = int64_t(out[j]);
            I.res[size_t(q)] = uint32_t(c < 0 ? c + m : c);
        } else {
            I.res[size_t(q)] = uint32_t(out[j]);
        }
    }
    return TN_OK;
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" tn_status tn_count_batch(const tn_formula* fs, int32_t n, tn_order_kind kind, uint64_t seed,
                                    const tn_contract_opts* opts, uint32_t* limbs, size_t cap_per,
                                    size_t* n_limbs, tn_plan_stats* stats) {
    if (n < 0 || (n > 0 && (!fs || !opts || !n_limbs || !opts->workspace))) return TN_EINVAL;
    if (n == 0) return TN_OK;
    std::vector<Inst> ins;
    try {
        ins.resize(size_t(n));
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    profiler().start(opts->flags & TN_FLAG_TIMING);
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<int32_t> next{0};
    std::vector<int32_t> done;  // instances in the order their plans were finished
    done.reserve(size_t(n));
    auto work = [&]() {
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= n) return;
            Inst& s = ins[size_t(i)];
            s.st = build_network(&fs[i], s.net);
            if (s.st == TN_OK) s.st = make_order(s.net, kind, seed + uint64_t(i), nullptr, s.plan);
            {
                std::lock_guard<std::mutex> lk(mu);
                s.ready = true;
                done.push_back(i);
            }
            cv.notify_all();
        }
    };
    std::vector<std::thread> pool;
    const int W = worker_count(n);
    for (int w = 0; w < W; ++w) pool.emplace_back(work);

    const int64_t cap = int64_t(opts->workspace_bytes) - kMaxGroup * kScratchPerPrime - (1 << 20);
    tn_status first_err = TN_OK;
    auto note = [&](tn_status s) {
        if (s != TN_OK && first_err == TN_OK) first_err = s;
    };
    SubBatch sb;
    auto flush = [&]() {
        if (sb.ids.empty()) return;
        tn_status s = run_sub(ins, sb, opts);
        for (int32_t i : sb.ids) {
            if (s != TN_OK) ins[i].st = s;
        }
        note(s);
        sb = SubBatch{};
    };
    // Instances are contracted in the order their plans become ready (order
    // searches differ in length). When no new plan arrives for a while, the
    // pending sub-batch goes to the device rather than leaving it idle.
    size_t taken = 0;
    for (int32_t got = 0; got < n; ++got) {
        int32_t i;
        {
            std::unique_lock<std::mutex> lk(mu);
            auto more = [&] { return taken < done.size(); };
            if (!sb.ids.empty() && !cv.wait_for(lk, std::chrono::milliseconds(kIdleFlushMs), more)) {
                lk.unlock();
                flush();
                lk.lock();
            }
            cv.wait(lk, more);
            i = done[taken++];
        }
        Inst& I = ins[size_t(i)];
        if (I.st != TN_OK) continue;
        I.st = resolve(I.plan, opts, I.R);
        if (I.st != TN_OK) continue;
        I.P = I.R.u64 ? 1 : I.R.k;
        I.es = I.R.es();
        I.res.assign(size_t(I.R.u64 ? 0 : I.R.k), 0);
        if (I.plan.n_init == 0 || I.plan.steps.empty()) {
            // empty network or a single scalar tensor: no device work
            uint64_t v = I.plan.n_init == 0 ? 1 : init_entry(I.net.t[size_t(I.plan.root)], {}, 0);
            I.u64v = v;
            for (int q = 0; q < int(I.res.size()); ++q) I.res[size_t(q)] = uint32_t(v % I.R.primes[size_t(q)]);
            I.host_only = true;
            continue;
        }
        I.init_bytes = align256(I.plan.init_elems * I.es);
        I.arena_bytes = align256(I.plan.warena_elems * I.es);
        I.n_items = items_of(I.plan, I.P);
        const int64_t need = I.init_bytes + I.P * I.arena_bytes + I.n_items * int64_t(sizeof(BItem)) +
                             I.P * int64_t(sizeof(GItem) + 8) + 4096;
        if (need > cap) {
            // too large to share the workspace: run alone, primes grouped as memory allows
            flush();
            std::vector<uint32_t> res;
            uint64_t v = 0;
            I.st = run_plan(I.net, I.plan, opts, I.R, res, &v);
            I.res = res;
            I.u64v = v;
            continue;
        }
        if (sb.init_total + sb.arena_total + sb.items * int64_t(sizeof(BItem)) + need > cap) flush();
        sb.ids.push_back(i);
        sb.init_total += I.init_bytes;
        sb.arena_total += I.P * I.arena_bytes;
        sb.items += I.n_items;
        sb.gathers += I.P;
    }
    flush();
    for (auto& t : pool) t.join();

    for (int32_t i = 0; i < n; ++i) {
        Inst& I = ins[size_t(i)];
        if (stats) stats[i] = I.plan.stats;
        if (I.st != TN_OK) {
            n_limbs[i] = 0;
            note(I.st);
            continue;
        }
        std::vector<uint32_t> L;
        if (I.R.u64) {
            L = {uint32_t(I.u64v), uint32_t(I.u64v >> 32)};
            while (L.size() > 1 && L.back() == 0) L.pop_back();
        } else {
            crt_limbs(I.res.data(), I.R.primes.data(), I.R.k, L);
        }
        n_limbs[i] = L.size();
        if (limbs && L.size() <= cap_per)
            std::copy(L.begin(), L.end(), limbs + size_t(i) * cap_per);
        else
            note(TN_EBUFSIZE);
    }
    return first_err;
}
