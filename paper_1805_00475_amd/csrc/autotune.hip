// Autotuner: for a grid of step shapes it times every configuration of the
// tunable kernels on the device -- the tile shape of the tiled int8
// matrix-core kernel, the B rows per thread of the streaming kernel -- with
// hipEvents on the caller's stream, keeps the fastest per shape, installs
// the table for every later launch and writes it as a JSON cache
// (tn_tune_load reads it back). Operands are zero-filled regions of the
// caller's workspace; timing does not depend on their values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "mfma.hpp"
#include "tune.hpp"

namespace tn {

namespace {

// C bits: A's two lowest first, then alternating, the rest of the larger side on top
uint64_t interleaved_mask(int fA, int fB) {
    uint64_t m = 0;
    int a = 0, b = 0, pos = 0;
    while (a < fA || b < fB) {
        const bool takeA = (a < fA) && (pos < 2 || b >= fB || (pos % 2 == 0));
        if (takeA) {
            m |= uint64_t(1) << pos;
            ++a;
        } else {
            ++b;
        }
        ++pos;
    }
    return m;
}

double time_us(hipStream_t st, int reps, const std::function<hipError_t()>& launch, bool* ok) {
    hipEvent_t e0, e1;
    *ok = false;
    if (hipEventCreate(&e0) != hipSuccess) return 0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 0;
    }
    double best = 1e30;
    bool good = launch() == hipSuccess;  // warm-up
    for (int r = 0; r < reps && good; ++r) {
        good = hipEventRecord(e0, st) == hipSuccess && launch() == hipSuccess && hipEventRecord(e1, st) == hipSuccess &&
               hipEventSynchronize(e1) == hipSuccess;
        float ms = 0;
        if (good && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, 1000.0 * ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ok = good;
    return best;
}

}  // namespace

}  // namespace tn

extern "C" tn_status tn_autotune(const char* out_path, void* workspace, size_t ws_bytes, void* stream_, int32_t reps) {
    using namespace tn;
    if (!workspace || ws_bytes < (size_t(64) << 20) || reps < 1) return TN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream_);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return TN_EHIP;
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    char* base = static_cast<char*>(workspace);
    if (hipMemsetAsync(base, 0, ws_bytes, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return TN_EHIP;
    const auto& mods = small_moduli();
    std::vector<std::string> lines;
    tune_clear();
    auto fits = [&](int fA, int fB, int s, int es, int* G) {
        const int64_t per = int64_t(es) * ((int64_t(1) << (fA + s)) + (int64_t(1) << (fB + s)) +
                                           (int64_t(1) << (fA + fB))) + kScratchPerPrime + 3 * 256;
        *G = int(std::min<int64_t>(kMaxGroup, int64_t(ws_bytes) / per));
        return *G >= 1;
    };
    auto args = [&](int fA, int fB, int s, int es, int G) {
        StepArgs a{};
        const int64_t nA = (int64_t(1) << (fA + s)), nB = (int64_t(1) << (fB + s)), nC = (int64_t(1) << (fA + fB));
        a.A = base;
        a.B = base + int64_t(G) * nA * es;
        a.C = base + int64_t(G) * (nA + nB) * es;
        a.strideA = nA;
        a.strideB = nB;
        a.strideC = nC;
        a.rC = fA + fB;
        a.s = s;
        a.fA = fA;
        a.fB = fB;
        a.maskA = interleaved_mask(fA, fB);
        a.maskB = ((uint64_t(1) << (fA + fB)) - 1) & ~a.maskA;
        fill_moduli(a, mods.data(), G);
        return a;
    };
    char buf[512];
    // tiled int8 kernel: tile shapes
    for (int s : {6, 8, 10, 12, 14, 16})
        for (int fA : {8, 10, 12, 14, 16})
            for (int fB : {6, 7, 8, 10, 12, 14, 16}) {
                if (fB > fA || fA + fB + s > 42) continue;
                int G;
                if (!fits(fA, fB, s, 1, &G)) continue;
                G = std::min(G, int(std::max<int64_t>(1, (int64_t(1) << 40) >> (fA + fB + s))));
                StepArgs a = args(fA, fB, s, 1, G);
                char* scratch = static_cast<char*>(a.C) + int64_t(G) * (int64_t(1) << (fA + fB)) + 256;
                std::vector<double> us(MFMA8_CFGS, -1.0);
                int best = -1;
                for (int cfg = 0; cfg < MFMA8_CFGS; ++cfg) {
                    if (!mfma8_cfg_fits(cfg, fA, fB)) continue;
                    bool ok;
                    const double t =
                        time_us(st, reps, [&]() { return launch_mfma8_cfg(a, G, st, scratch, kScratchPerPrime, cfg); },
                                &ok);
                    if (!ok) return TN_EHIP;
                    us[size_t(cfg)] = t / G;
                    if (best < 0 || t < us[size_t(best)] * G) best = cfg;
                }
                tune_set(TK_MFMA8, EL_I8, fA, fB, s, best);
                std::string u;
                for (int cfg = 0; cfg < MFMA8_CFGS; ++cfg)
                    if (us[size_t(cfg)] >= 0) {
                        std::snprintf(buf, sizeof buf, "%s\"%s\": %.2f", u.empty() ? "" : ", ", mfma8_cfg_name(cfg),
                                      us[size_t(cfg)]);
                        u += buf;
                    }
                std::snprintf(buf, sizeof buf,
                              "{\"kernel\": \"mfma8\", \"el\": \"i8\", \"fA\": %d, \"fB\": %d, \"s\": %d, \"choice\": %d, "
                              "\"name\": \"%s\", \"us_per_plane\": {%s}}",
                              fA, fB, s, best, mfma8_cfg_name(best), u.c_str());
                lines.push_back(buf);
            }
    // streaming kernel: B rows per thread, int8 residues and 64-bit counts
    for (int el : {int(EL_I8), int(EL_U64)})
        for (int s : {0, 1, 2, 3, 4, 5})
            for (int fA : {10, 14, 18, 22})
                for (int fB : {1, 2, 3, 4, 5, 6}) {
                    const int es = elem_size(el);
                    int G;
                    if (!fits(fA, fB, s, es, &G)) continue;
                    if (el == EL_U64) G = 1;
                    StepArgs a = args(fA, fB, s, es, G);
                    int best = -1;
                    double bt = 0;
                    std::string u;
                    for (int nb = 0; nb <= std::min(fB, 4); ++nb) {
                        bool ok;
                        const double t = time_us(st, reps, [&]() { return launch_stream_step(a, el, G, nb, st); }, &ok);
                        if (!ok) return TN_EHIP;
                        if (best < 0 || t < bt) {
                            best = nb;
                            bt = t;
                        }
                        std::snprintf(buf, sizeof buf, "%s\"%d\": %.2f", u.empty() ? "" : ", ", 1 << nb, t / G);
                        u += buf;
                    }
                    tune_set(TK_STREAM, el, fA, fB, s, best);
                    std::snprintf(buf, sizeof buf,
                                  "{\"kernel\": \"stream\", \"el\": \"%s\", \"fA\": %d, \"fB\": %d, \"s\": %d, "
                                  "\"choice\": %d, \"name\": \"%d rows\", \"us_per_plane\": {%s}}",
                                  el == EL_I8 ? "i8" : "u64", fA, fB, s, best, 1 << best, u.c_str());
                    lines.push_back(buf);
                }
    tune_publish();
    if (out_path) {
        FILE* f = std::fopen(out_path, "w");
        if (!f) return TN_EINVAL;
        std::fprintf(f, "{\"format\": \"tn-autotune-1\", \"arch\": \"%s\", \"cus\": %d, \"reps\": %d,\n \"entries\": [\n",
                     arch.c_str(), prop.multiProcessorCount, reps);
        for (size_t i = 0; i < lines.size(); ++i)
            std::fprintf(f, "  %s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
        std::fprintf(f, " ]}\n");
        std::fclose(f);
    }
    return TN_OK;
}
