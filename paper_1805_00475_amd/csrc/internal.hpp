// Internal data structures shared by the host-side parts of libtn.
#pragma once

#include <array>
#include <atomic>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "tn.h"

namespace tn {

enum TKind : uint8_t { T_COPY = 0, T_OR = 1, T_EXONE = 2, T_XOR = 3, T_TABLE = 4 };

// A tensor of the original network (Sec. 2.1). ``bonds[k]`` is the bond on
// index k: for a COPY tensor the k-th occurrence of its variable, for a
// clause tensor its k-th literal. Bit k of ``neg`` reverses index k. A
// T_TABLE tensor lists its entries: table[x], bit k of x the value of bond k.
struct InitTensor {
    uint8_t kind = T_COPY;
    std::vector<int32_t> bonds;
    uint64_t neg = 0;
    std::vector<uint32_t> table;
};

struct Network {
    int32_t n_vars = 0;
    int32_t n_clauses = 0;
    int32_t count_bits = 0;   // the count is at most 2^count_bits
    uint64_t max_entry = 2;   // largest entry of an initial tensor
    std::vector<InitTensor> t;                   // variables first, then clauses, then split pieces
    std::vector<std::array<int32_t, 2>> bond_end;  // the two tensors of every bond
    // the formula a boolean network was built from (clause offsets,
    // literals, kinds; empty for constraint networks)
    std::vector<int32_t> f_ptr, f_lits;
    std::vector<uint8_t> f_kinds;
};

// One pairwise contraction C = A (x) B in the layout convention of the plan:
// every tensor stores its bonds sorted by the step at which they are
// contracted (earliest first, bond id breaking ties), bit 0 being the
// earliest. The s bonds shared by A and B die at this step, so they are the
// low s bits of both operands: A = [z | xA], B = [z | xB]. C's bits are the
// free bonds of A and B merged in the same sort order; bit j of ``maskA``
// says C's bit j comes from A.
struct Step {
    int32_t a = -1, b = -1, out = -1;
    int32_t rA = 0, rB = 0, s = 0, rC = 0;
    uint64_t maskA = 0;
    bool initA = false, initB = false;   // operand lives in the shared init region
    int64_t offA = 0, offB = 0, offC = 0;  // element offsets (init region or arena), plan order
    int64_t woffA = 0, woffB = 0, woffC = 0;  // the same for execution in waves (by level)
    int32_t level = 0;                   // longest chain of steps feeding this one
};

struct Plan {
    int32_t n_init = 0;
    int32_t n_vars = 0;
    int32_t count_bits = 0;   // the network's bound: the count is at most 2^count_bits
    uint64_t max_entry = 2;   // largest initial entry (above 127: initial tensors per residue plane)
    std::vector<std::pair<int32_t, int32_t>> merges;
    std::vector<Step> steps;
    std::vector<int32_t> rank;                 // per tensor id
    std::vector<std::vector<int32_t>> layout;  // per tensor id: bond on each bit
    std::vector<int64_t> init_off;             // per initial tensor, element offset
    int64_t init_elems = 0;                    // size of the init region (elements)
    int64_t arena_elems = 0;                   // arena size for one prime (elements), plan order
    int64_t warena_elems = 0;                  // arena size when steps run in waves by level
    int32_t root = -1;                         // id of the final scalar
    double cost_us = -1;                       // plan_cost, kept by make_plan (-1: not yet)
    bool sketch = false;                       // merges, cost and stats only (sketch_plan)
    tn_plan_stats stats{};
};

constexpr int64_t kAlignElems = 64;  // 256 bytes for 32-bit entries

// network.cpp
tn_status build_network(const tn_formula* f, Network& net);
tn_status build_csp(const tn_csp* c, Network& net);
tn_status reduce_degree(Network& net, uint32_t flags);

// order_*.cpp: produce merges (pairs of tensor ids; merge k creates id
// n_init + k). Every order ends with a single tensor.
struct Graph;  // adjacency of live tensors
std::vector<std::pair<int32_t, int32_t>> order_greedy(const Network& net);
std::vector<std::pair<int32_t, int32_t>> order_partition(const Network& net, uint64_t seed);
std::vector<std::pair<int32_t, int32_t>> order_community(const Network& net);
std::vector<std::pair<int32_t, int32_t>> order_learned(const Network& net, const tn_model* model,
                                                       bool* ok);

// Shared by the hierarchical orders: absorb every tensor of rank <= 2 into a
// neighbour (never raises any rank). Returns the merges done and, for every
// surviving group, its current tensor id, its rank and its bond set.
struct Reduced {
    std::vector<std::pair<int32_t, int32_t>> merges;
    std::vector<int32_t> id;                  // tensor id of each reduced vertex
    std::vector<std::vector<int32_t>> bonds;  // bonds of each reduced vertex
    int32_t next_id = 0;
};
Reduced absorb_small(const Network& net);

// plan.cpp
tn_status make_plan(const Network& net, std::vector<std::pair<int32_t, int32_t>> merges,
                    int32_t chosen, Plan& plan);
// The same checks and predicted cost as make_plan, without layouts, steps
// or arena: merges, cost_us and stats (n_steps, max_rank, log2_cost,
// chosen); make_plan of the same merges gives the full plan of equal cost.
tn_status sketch_plan(const Network& net, std::vector<std::pair<int32_t, int32_t>> merges, int32_t chosen,
                      Plan& plan);
// Residue arithmetic a contraction uses by default for counts of at most
// 2^count_bits: 64-bit wrapping counts (count_bits <= 63), small moduli
// (int8 residues) when their product holds the count, else 16-bit primes;
// and its plane count.
enum ResidueMode : int { RM_U64 = 0, RM_WIDE = 1, RM_SMALL = 2 };
int default_residue_mode(int32_t count_bits);
int32_t default_planes(int32_t count_bits);
// Predicted device time in microseconds: of a whole plan under its default
// residue mode (all planes, launches included), and of one step for one
// residue plane (launch excluded).
double plan_cost(const Plan& plan);
double step_cost_model(int rA, int rB, int s, int rC, int mode);
// order_refine.cpp: exact re-optimization of subtrees with up to 8 frontier
// nodes, sweeping the largest tensors first, within budget_us
std::vector<std::pair<int32_t, int32_t>> refine_order(const Network& net,
                                                      const std::vector<std::pair<int32_t, int32_t>>& merges,
                                                      double budget_us);
tn_status verify_plan(const Plan& plan);

// count_bound.cpp: ceil(log2) of an upper bound on the count of a boolean
// formula (mini-bucket elimination; at most n_vars; 0 when a clause is empty)
int32_t count_bound_bits(const tn_formula* f);
// a quick bound (log2, not rounded): the count of the formula kept to a
// greedy set of variable-disjoint clauses
double disjoint_clause_bound_bits(const tn_formula* f);
// the tighter, costlier variant (Hoelder norms per mini-bucket, larger
// mini-buckets, least-fill order)
// -1 when *cancel turns true before it ends
int32_t count_bound_bits_tight(const tn_formula* f, const std::atomic<bool>* cancel = nullptr);
// the elimination behind both, any mini-bucket size (checks use small ones)
int32_t count_bound_bits_with(const tn_formula* f, int ib, bool weighted, int fill_cands,
                              const std::atomic<bool>* cancel = nullptr);

// api.cpp: order of any kind (with the judge for BEST / LEARNED) + plan
// threads: host threads for the judge's randomized bisection trials (one
// order search; the batch path runs one search per thread with threads = 1);
// rounds > 0: the judge runs exactly that many rounds of trials (no time
// rule), so that the plan depends only on the seed and the thread count
tn_status make_order(const Network& N, int32_t kind, uint64_t seed, const tn_model* model, Plan& out,
                     int threads = 1, int rounds = 0);

// contract.hip
struct Resolved {
    bool u64 = false;
    bool i8 = false;  // small moduli, residues stored as centred int8
    int32_t k = 0;    // residue planes
    std::vector<uint32_t> primes;  // their moduli
    int32_t es() const { return u64 ? 8 : i8 ? 1 : 4; }
};
tn_status resolve(const Plan& plan, const tn_contract_opts* o, Resolved& r);
tn_status run_plan(const Network& net, const Plan& plan, const tn_contract_opts* o, const Resolved& R,
                   std::vector<uint32_t>& residues, uint64_t* u64v);

// crt.cpp
// primes of the residue path: the largest below kPrimeBound, descending
constexpr uint32_t kPrimeBound = 65280;
const std::vector<uint32_t>& prime_table(int32_t k);
int32_t primes_needed(int32_t n_vars);  // > TN_MAX_PRIMES when n_vars is too large
void crt_limbs(const uint32_t* residues, int32_t k, std::vector<uint32_t>& limbs);  // first k primes
void crt_limbs(const uint32_t* residues, const uint32_t* moduli, int32_t k, std::vector<uint32_t>& limbs);
// small moduli: pairwise coprime, at most kSmallModulusMax, descending
constexpr uint32_t kSmallModulusMax = 255;
const std::vector<uint32_t>& small_moduli();
int32_t small_moduli_needed(int32_t n_vars);  // 0 when they do not suffice

}  // namespace tn

struct tn_network {
    tn::Network net;
};
struct tn_plan {
    tn::Plan plan;
};
