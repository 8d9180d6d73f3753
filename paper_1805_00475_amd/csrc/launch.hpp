// Step launcher and initial-tensor helpers shared by the single-instance
// and the batched contraction paths.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.hpp"
#include "profile.hpp"

namespace tn {

// scratch per prime: partial sums of the split-K dot kernels (1024 blocks x
// 64 outputs x 8 B) and of split-K matrix-core steps (up to 2^20 residues)
constexpr int kDotBlocks = 1024;
constexpr int64_t kScratchPerPrime = int64_t(1) << 22;

int64_t align256(int64_t b);

// Chooses and launches the kernel(s) of one step for G residue planes (or
// the single 64-bit plane). Operands that are initial tensors live in the
// init region (shared by all planes); the others in the plane's arena.
// force >= 0 selects a kernel class (test hook).
hipError_t launch_step(const Step& st, bool u64, int flags, const uint32_t* primes, int G, char* init_base,
                       char* arena_base, int64_t arena_elems, char* scratch, hipStream_t stream, KernelClass* kc,
                       int force = -1);

// Entry x of an initial tensor whose bonds sit at bit positions pos.
uint64_t init_entry(const InitTensor& t, const std::vector<int32_t>& pos, uint64_t x);
// Writes every initial tensor of a plan, in plan layout, at its init offset.
void fill_init(const Network& net, const Plan& plan, bool u64, uint8_t* host);

}  // namespace tn
