// Table of autotuned launch choices: built by the autotuner or read from its
// JSON cache (tn_tune_load), consulted by the launch code. Readers take a
// snapshot of the published table; a new table replaces it whole.
#include "tune.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include "tn.h"

namespace tn {

namespace {

using Key = std::tuple<int, int, int, int, int>;  // kernel, el, fA, fB, s
struct Table {
    std::map<Key, int> choice;
};

std::mutex g_mu;
std::shared_ptr<const Table> g_table;   // published
std::shared_ptr<Table> g_building;      // being filled

std::shared_ptr<const Table> snapshot() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table;
}

}  // namespace

bool mfma8_cfg_fits(int cfg, int fA, int fB) {
    static const int wm[MFMA8_CFGS] = {8, 8, 7, 8, 7}, wn[MFMA8_CFGS] = {8, 7, 7, 6, 6};
    return cfg >= 0 && cfg < MFMA8_CFGS && fA >= wm[cfg] && fB >= wn[cfg];
}

const char* mfma8_cfg_name(int cfg) {
    static const char* names[MFMA8_CFGS] = {"256x256", "256x128", "128x128", "256x64", "128x64"};
    return cfg >= 0 && cfg < MFMA8_CFGS ? names[cfg] : "rule";
}

int tuned_choice(int kernel, int el, int fA, int fB, int s) {
    const auto t = snapshot();
    if (!t || t->choice.empty()) return -1;
    // nearest tuned shape of this kernel and element kind (squared distance
    // in free and shared bits), whose choice must also fit this shape
    int best = -1;
    long bestd = 0;
    for (const auto& kv : t->choice) {
        const auto& k = kv.first;
        if (std::get<0>(k) != kernel || std::get<1>(k) != el) continue;
        const long d = long(std::get<2>(k) - fA) * (std::get<2>(k) - fA) + long(std::get<3>(k) - fB) * (std::get<3>(k) - fB) +
                       long(std::get<4>(k) - s) * (std::get<4>(k) - s);
        if (kernel == TK_MFMA8 && !mfma8_cfg_fits(kv.second, fA, fB)) continue;
        if (kernel == TK_STREAM && kv.second > fB) continue;
        if (best < 0 || d < bestd) {
            best = kv.second;
            bestd = d;
        }
    }
    return best;
}

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_building = std::make_shared<Table>();
}

void tune_set(int kernel, int el, int fA, int fB, int s, int choice) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_building) g_building = std::make_shared<Table>();
    g_building->choice[Key(kernel, el, fA, fB, s)] = choice;
}

void tune_publish() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table = g_building ? std::shared_ptr<const Table>(g_building) : nullptr;
    g_building.reset();
}

}  // namespace tn

namespace {

// value of "key": in a line of the cache ("key": 12 or "key": "text")
bool field(const std::string& line, const char* key, std::string& out) {
    const std::string pat = std::string("\"") + key + "\":";
    size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    p += pat.size();
    while (p < line.size() && line[p] == ' ') ++p;
    if (p < line.size() && line[p] == '"') {
        const size_t e = line.find('"', p + 1);
        if (e == std::string::npos) return false;
        out = line.substr(p + 1, e - p - 1);
        return true;
    }
    size_t e = p;
    while (e < line.size() && (line[e] == '-' || (line[e] >= '0' && line[e] <= '9'))) ++e;
    out = line.substr(p, e - p);
    return !out.empty();
}

}  // namespace

extern "C" tn_status tn_tune_load(const char* path, const char* arch) {
    if (!path) {
        tn::tune_clear();
        tn::tune_publish();
        return TN_OK;
    }
    std::ifstream in(path);
    if (!in) return TN_EINVAL;
    std::string line, v;
    bool header = false;
    int n = 0;
    tn::tune_clear();
    while (std::getline(in, line)) {
        if (!header) {
            if (!field(line, "format", v) || v != "tn-autotune-1") continue;
            if (arch && field(line, "arch", v) && v != arch) return TN_EUNSUPPORTED;
            header = true;
            continue;
        }
        if (line.find("\"kernel\"") == std::string::npos) continue;
        std::string k, el, fa, fb, s, c;
        if (!field(line, "kernel", k) || !field(line, "el", el) || !field(line, "fA", fa) || !field(line, "fB", fb) ||
            !field(line, "s", s) || !field(line, "choice", c))
            return TN_EINVAL;
        const int kernel = k == "mfma8" ? tn::TK_MFMA8 : k == "stream" ? tn::TK_STREAM : -1;
        const int e = el == "u32" ? 0 : el == "u64" ? 1 : el == "i8" ? 2 : -1;
        if (kernel < 0 || e < 0) return TN_EINVAL;
        tn::tune_set(kernel, e, std::stoi(fa), std::stoi(fb), std::stoi(s), std::stoi(c));
        ++n;
    }
    if (!header) return TN_EINVAL;
    tn::tune_publish();
    return TN_OK;
}
