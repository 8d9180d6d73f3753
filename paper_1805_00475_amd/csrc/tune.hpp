// Launch choices measured by the autotuner (autotune.hip) and consulted at
// launch time: for a kernel and a step shape, which of the kernel's
// configurations runs. Without a loaded cache (or for shapes it does not
// cover) every launch follows the built-in rules.
#pragma once

#include <cstdint>
#include <string>

namespace tn {

enum TuneKernel : int {
    TK_MFMA8 = 0,   // tiled int8 matrix-core kernel: tile shape (MFMA8_*)
    TK_STREAM = 1   // streaming kernel: B rows per thread, log2
};
enum Mfma8Cfg : int { MFMA8_RULE = -1, MFMA8_256x256 = 0, MFMA8_256x128 = 1, MFMA8_128x128 = 2, MFMA8_256x64 = 3,
                      MFMA8_128x64 = 4, MFMA8_CFGS = 5 };

// The measured choice for (kernel, element kind, free bits of A and B,
// shared bits), taken at the nearest tuned shape of that kernel and element
// kind (free and shared bits clamped to the tuned range); -1 when none.
int tuned_choice(int kernel, int el, int fA, int fB, int s);
// Replaces the table (thread-safe; launches see the old or the new one).
void tune_clear();
void tune_set(int kernel, int el, int fA, int fB, int s, int choice);
void tune_publish();
// Whether tile shape cfg can run a step with free sides fA >= fB.
bool mfma8_cfg_fits(int cfg, int fA, int fB);
const char* mfma8_cfg_name(int cfg);

}  // namespace tn
