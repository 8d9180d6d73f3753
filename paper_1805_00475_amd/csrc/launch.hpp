// Step launcher and initial-tensor helpers shared by the single-instance
// and the batched contraction paths.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
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
// force >= 0 selects a kernel class (test hook). dig: bit 0 / bit 1 = operand
// A / B of the plan's step is already held as digit planes (see mfma.hip),
// bit 2 = write the output as digit planes (only the matrix-core kernel
// does; the caller sets it only where choose_class says so for this step
// and for the output's consumer).
hipError_t launch_step(const Step& st, int el, int flags, const uint32_t* primes, int G, char* init_base,
                       char* arena_base, int64_t arena_elems, char* scratch, hipStream_t stream, KernelClass* kc,
                       int force = -1, unsigned dig = 0, int64_t init_stride = 0);

// The kernel class launch_step picks for a step (no launch, force < 0).
KernelClass choose_class(const Step& st, int el, int flags);

// Digit-plane hand-over between matrix-core steps: for every step, the dig
// bits of launch_step, given the class each step runs with. A tensor is
// written as digit planes when its producer and its consumer both run the
// matrix-core kernel, which then skips the digit pass on it.
std::vector<uint8_t> digit_plan(const Plan& plan, const std::vector<KernelClass>& cls, int el);

// Bytes per entry of an element kind (EL_U32, EL_U64, EL_I8 of kernels.hpp).
int elem_size(int el);
// Moduli and their reduction constants of G residue planes.
void fill_moduli(StepArgs& a, const uint32_t* primes, int G);

// The streaming kernel with 2^nb B rows per thread (autotuner launches).
hipError_t launch_stream_step(const StepArgs& a, int el, int G, int nb, hipStream_t st);

// Entry x of an initial tensor whose bonds sit at bit positions pos.
uint64_t init_entry(const InitTensor& t, const std::vector<int32_t>& pos, uint64_t x);
// Writes every initial tensor of a plan, in plan layout, at its init offset.
void fill_init(const Network& net, const Plan& plan, int el, uint8_t* host, const uint32_t* mod = nullptr);
bool init_per_plane(const Plan& plan, const Resolved& R);

}  // namespace tn
