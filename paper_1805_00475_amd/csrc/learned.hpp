// The order-scoring perceptron: sizes, parameter packing and host helpers.
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace tn {

constexpr int kFeatures = 10;
constexpr int kHidden = 128;
// packed parameters: W1 [H x F], b1 [H], W2 [H x H], b2 [H], w3 [H], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kFeatures;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;
constexpr int kParams = kOffB3 + 1;

struct LiveGraph;
void pair_features(const LiveGraph& g, int32_t u, int32_t v, float* f);
float mlp_score(const float* params, const float* x);
void transpose_params(const float* params, std::vector<float>& w1t, std::vector<float>& w2t);
float mlp_score_t(const float* params, const float* w1t, const float* w2t, const float* x);
tn_status trace_order(const Network& net, const std::vector<std::pair<int32_t, int32_t>>& teacher,
                      std::vector<float>& feats, std::vector<uint8_t>& labels, std::vector<int32_t>& groups);

}  // namespace tn

struct tn_model {
    std::vector<float> params;  // kParams floats
};
