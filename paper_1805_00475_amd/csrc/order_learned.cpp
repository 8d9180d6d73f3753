// Learned order proposer: a 3-layer perceptron scores every connected pair
// of live tensors; the best-scoring pair is contracted next (a learned
// replacement for the "smallest rank" rule of tensor-greedy, Sec. 3.1.1).
// The scorer is trained by imitation of the orders the plain heuristics
// find (see train_order.py); the judge in make_order keeps it only when its
// plan is predicted cheaper (Sec. 4: portfolio, lazy evaluation).
//
// Features of a candidate pair (u, v), with rA >= rB the ranks, s the bonds
// shared, rC = rA + rB - 2s, dA, dB the numbers of neighbouring tensors and
// c the number of tensors adjacent to both:
//   rA/32, rB/32, s/32, rC/32, (rC - rA)/8, dA/16, dB/16, c/8,
//   (rA + rB - s)/48 (log2 of the multiply-adds), [s == rB] (B absorbed).
// They depend on u, v and their neighbourhoods only, so after a merge only
// pairs touching the new tensor or its neighbours are re-scored.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>

#include "graph.hpp"
#include "internal.hpp"
#include "learned.hpp"

namespace tn {

namespace {

// The integers the features are made of (the larger tensor first).
struct PairInts {
    int32_t ru, rv, s, du, dv, common;
};

// Common neighbours are counted against a stamp array (one entry per
// tensor id, epoch-marked) when one is given, else by search.
struct Stamps {
    std::vector<uint32_t> mark;
    uint32_t epoch = 0;
};

PairInts pair_ints(const LiveGraph& g, int32_t u, int32_t v, Stamps* st = nullptr) {
    PairInts p{g.rank[u], g.rank[v], 0, int32_t(g.nb[u].size()), int32_t(g.nb[v].size()), 0};
    if (p.rv > p.ru || (p.rv == p.ru && p.dv > p.du)) {
        std::swap(p.ru, p.rv);
        std::swap(p.du, p.dv);
        std::swap(u, v);
    }
    p.s = g.shared(u, v);
    if (st) {
        if (st->mark.size() < g.nb.size()) st->mark.resize(g.nb.size(), 0);
        const uint32_t e = ++st->epoch;
        for (const auto& b : g.nb[v]) st->mark[size_t(b.first)] = e;
        for (const auto& a : g.nb[u])
            if (a.first != v && st->mark[size_t(a.first)] == e) ++p.common;
    } else {
        for (const auto& a : g.nb[u])
            if (a.first != v && g.shared(v, a.first) > 0) ++p.common;
    }
    return p;
}

void features_of(const PairInts& p, float* f) {
    const int32_t ru = p.ru, rv = p.rv, s = p.s, du = p.du, dv = p.dv, common = p.common;
    const int32_t rc = ru + rv - 2 * s;
    f[0] = ru / 32.0f;
    f[1] = rv / 32.0f;
    f[2] = s / 32.0f;
    f[3] = rc / 32.0f;
    f[4] = (rc - ru) / 8.0f;
    f[5] = du / 16.0f;
    f[6] = dv / 16.0f;
    f[7] = common / 8.0f;
    f[8] = (ru + rv - s) / 48.0f;
    f[9] = (s == rv) ? 1.0f : 0.0f;
}

// The six integers in 10 bits each, or ~0 when one does not fit.
uint64_t pair_key(const PairInts& p) {
    const int32_t v[6] = {p.ru, p.rv, p.s, p.du, p.dv, p.common};
    uint64_t k = 0;
    for (int i = 0; i < 6; ++i) {
        if (v[i] < 0 || v[i] > 1023) return ~uint64_t(0);
        k = (k << 10) | uint64_t(v[i]);
    }
    return k;
}

}  // namespace

void pair_features(const LiveGraph& g, int32_t u, int32_t v, float* f) { features_of(pair_ints(g, u, v), f); }

// Host forward pass, float32, the same arithmetic as the GPU kernels:
// h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3. The
// transposed copies (W1t [F x H], W2t [H x H]) let every layer accumulate
// whole rows of outputs at once; inputs that the ReLU zeroed are skipped.
void transpose_params(const float* P, std::vector<float>& w1t, std::vector<float>& w2t) {
    w1t.assign(size_t(kFeatures) * kHidden, 0.0f);
    w2t.assign(size_t(kHidden) * kHidden, 0.0f);
    for (int j = 0; j < kHidden; ++j) {
        for (int k = 0; k < kFeatures; ++k) w1t[size_t(k) * kHidden + j] = P[kOffW1 + j * kFeatures + k];
        for (int k = 0; k < kHidden; ++k) w2t[size_t(k) * kHidden + j] = P[kOffW2 + j * kHidden + k];
    }
}

float mlp_score_t(const float* P, const float* w1t, const float* w2t, const float* x) {
    alignas(32) float h1[kHidden], h2[kHidden];
    for (int j = 0; j < kHidden; ++j) h1[j] = P[kOffB1 + j];
    for (int k = 0; k < kFeatures; ++k) {
        const float xk = x[k];
        const float* row = w1t + size_t(k) * kHidden;
        for (int j = 0; j < kHidden; ++j) h1[j] += row[j] * xk;
    }
    for (int j = 0; j < kHidden; ++j) h2[j] = P[kOffB2 + j];
    for (int k = 0; k < kHidden; ++k) {
        const float hk = h1[k];
        if (!(hk > 0.0f)) continue;  // relu
        const float* row = w2t + size_t(k) * kHidden;
        for (int j = 0; j < kHidden; ++j) h2[j] += row[j] * hk;
    }
    float y = P[kOffB3];
    for (int j = 0; j < kHidden; ++j) y += P[kOffW3 + j] * (h2[j] > 0.0f ? h2[j] : 0.0f);
    return y;
}

float mlp_score(const float* P, const float* x) {
    std::vector<float> w1t, w2t;
    transpose_params(P, w1t, w2t);
    return mlp_score_t(P, w1t.data(), w2t.data(), x);
}

std::vector<std::pair<int32_t, int32_t>> order_learned(const Network& net, const tn_model* model, bool* ok) {
    *ok = false;
    std::vector<std::pair<int32_t, int32_t>> merges;
    if (!model) return merges;
    const float* P = model->params.data();
    std::vector<float> w1t, w2t;
    transpose_params(P, w1t, w2t);
    LiveGraph g;
    g.init(net);
    // The score is a function of six small integers, and the same local
    // configurations recur throughout a network: scores are kept by those
    // integers (the same floats as computing them again).
    std::unordered_map<uint64_t, float> memo;
    memo.reserve(4096);
    Stamps stamps;
    float f[kFeatures];
    auto score_pair = [&](int32_t u, int32_t v) {
        const PairInts p = pair_ints(g, u, v, &stamps);
        const uint64_t key = pair_key(p);
        if (key != ~uint64_t(0)) {
            const auto it = memo.find(key);
            if (it != memo.end()) return it->second;
        }
        features_of(p, f);
        const float y = mlp_score_t(P, w1t.data(), w2t.data(), f);
        if (key != ~uint64_t(0)) memo.emplace(key, y);
        return y;
    };
    // scores of live candidate pairs
    struct Cand {
        int32_t u, v;
        float score;
    };
    std::vector<Cand> cands, keep;
    for (int32_t u = 0; u < int32_t(g.nb.size()); ++u)
        for (const auto& pr : g.nb[u])
            if (u < pr.first) cands.push_back({u, pr.first, score_pair(u, pr.first)});
    std::vector<char> touched;
    while (!cands.empty()) {
        size_t best = 0;
        for (size_t i = 1; i < cands.size(); ++i) {
            const Cand& a = cands[i];
            const Cand& b = cands[best];
            if (a.score > b.score || (a.score == b.score && (a.u < b.u || (a.u == b.u && a.v < b.v)))) best = i;
        }
        const int32_t u = cands[best].u, v = cands[best].v;
        const int32_t c = g.merge(u, v);
        merges.push_back({u, v});
        // drop pairs touching u or v; re-score pairs touching c's neighbourhood
        touched.assign(g.alive.size(), 0);
        touched[size_t(c)] = 1;
        for (const auto& pr : g.nb[size_t(c)]) touched[size_t(pr.first)] = 1;
        keep.clear();
        for (const Cand& x : cands) {
            if (x.u == u || x.v == u || x.u == v || x.v == v) continue;
            if (touched[size_t(x.u)] || touched[size_t(x.v)]) continue;  // re-scored below
            keep.push_back(x);
        }
        cands.swap(keep);
        // every live pair with an endpoint in N(c) u {c}
        auto rescore_from = [&](int32_t x) {
            for (const auto& pr : g.nb[size_t(x)]) {
                const int32_t y = pr.first;
                if (touched[size_t(y)] && y < x) continue;  // counted from y's side
                cands.push_back({std::min(x, y), std::max(x, y), score_pair(x, y)});
            }
        };
        rescore_from(c);
        for (const auto& pr : g.nb[size_t(c)])
            if (g.alive[size_t(pr.first)]) rescore_from(pr.first);
    }
    g.close_scalars(merges);
    *ok = true;
    return merges;
}

// Features and labels along a teacher's order: before every teacher merge,
// one row per connected pair of live tensors (plus the teacher's pair when it
// shares no bond), labelled 1 when that pair is a merge of the teacher whose
// two inputs are both alive at this point, else 0.
tn_status trace_order(const Network& net, const std::vector<std::pair<int32_t, int32_t>>& teacher,
                      std::vector<float>& feats, std::vector<uint8_t>& labels, std::vector<int32_t>& groups) {
    LiveGraph g;
    g.init(net);
    // teacher merges keyed by their inputs
    std::vector<std::pair<int32_t, int32_t>> tm = teacher;
    const int32_t n_init = int32_t(net.t.size());
    std::vector<int32_t> partner(n_init + tm.size(), -1);
    for (const auto& m : tm) {
        partner[m.first] = m.second;
        partner[m.second] = m.first;
    }
    groups.clear();
    groups.push_back(0);
    float f[kFeatures];
    for (size_t k = 0; k < tm.size(); ++k) {
        const int32_t a = tm[k].first, b = tm[k].second;
        if (!g.alive[a] || !g.alive[b]) return TN_EINVAL;
        size_t rows0 = labels.size();
        bool teacher_seen = false;
        for (int32_t u = 0; u < int32_t(g.nb.size()); ++u) {
            if (!g.alive[u]) continue;
            for (const auto& pr : g.nb[u]) {
                const int32_t v = pr.first;
                if (v < u) continue;
                pair_features(g, u, v, f);
                feats.insert(feats.end(), f, f + kFeatures);
                const bool pos = partner[u] == v;
                labels.push_back(pos ? 1 : 0);
                if ((u == std::min(a, b)) && (v == std::max(a, b))) teacher_seen = true;
            }
        }
        if (!teacher_seen) {
            pair_features(g, a, b, f);
            feats.insert(feats.end(), f, f + kFeatures);
            labels.push_back(1);
        }
        if (labels.size() > rows0) groups.push_back(int32_t(labels.size()));
        g.merge(a, b);
    }
    return TN_OK;
}

}  // namespace tn
