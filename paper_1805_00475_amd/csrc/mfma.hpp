// Dense contraction steps on the int8 matrix cores (see mfma.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tn {

struct MfmaExtra {
    double inv_p[kMaxGroup];  // the double nearest 1/p, per prime
    // output tile positions 2048 q (q < 4 for 128 x 64 tiles, q < 8 for
    // 128 x 128) beyond a thread's first: C offset bits and the A-side and
    // B-side tile-local indices; dI, dJ: the indices of the word k (< 4)
    // after a position whose two lowest bits are 0
    uint64_t hiOff[8];
    uint32_t hiI[8], hiJ[8], dI[4], dJ[4];
    // 128 x 128 tiles: staging word of tile-local bit i_b / j_b (the word of
    // (i, j) is the XOR over its set bits), and the staging words of the
    // positions 2048 q and of the word k, for the C-order reads
    uint32_t phiI[7], phiJ[7], stageQ[8], stageK[4];
    uint32_t digits_out;  // 1: write C as digit planes (its consumer is a matrix-core step)
};

// A step qualifies when K = 2^s is at least 64 and the free sides give at
// least one 128 x 64 output tile (128 x 128 tiles are used when B's free
// side has at least 7 bits). The caller must also ensure that neither
// operand is a shared initial tensor: both are rewritten in place into digit
// planes.
bool mfma_eligible(const StepArgs& a);
// the same question for an element kind (EL_U32: the digit kernels above;
// EL_I8: the int8 kernel of mfma8.hip)
bool mfma_eligible(const StepArgs& a, int el);
struct Profiler;
// Digit pass on both operands, then the GEMM; each launch is bracketed by
// the profiler (no-op unless timing is on) with its algorithmic work.
// scratch: scratch_per_plane bytes for each of the G planes (split-K partials)
// dig: bit 0 / bit 1 = A / B are digit planes already (no digit pass), bit 2
// = write C as digit planes
hipError_t launch_mfma(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                       double step_macs, char* scratch, int64_t scratch_per_plane, unsigned dig = 0);
// Matrix-core step on centred int8 residues modulo small moduli (mfma8.hip):
// one int8 product per modular multiply-add, no digit pass.
hipError_t launch_mfma8(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                        double step_macs, char* scratch, int64_t scratch_per_plane);
bool mfma8_eligible(const StepArgs& a);
// The tiled int8 kernel with a given tile shape (Mfma8Cfg of tune.hpp;
// MFMA8_RULE = the built-in rule), without profiling (the autotuner's
// measurement launches).
hipError_t launch_mfma8_cfg(const StepArgs& a, int G, hipStream_t stream, char* scratch, int64_t scratch_per_plane,
                            int cfg);
// Narrow int8 matrix-core step (narrow8.hip): B side of at most 64 rows,
// K >= 64; A is read once (split K over block rows when the step has few
// row tiles, partial residues in scratch).
hipError_t launch_narrow8(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                          double step_macs, char* scratch, int64_t scratch_per_plane);
bool narrow8_eligible(const StepArgs& a);

}  // namespace tn
