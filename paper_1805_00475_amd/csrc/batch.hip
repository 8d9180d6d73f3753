// Batched counting: placeholder until the wave scheduler lands.
#include <hip/hip_runtime.h>

#include "internal.hpp"

extern "C" tn_status tn_count_batch(const tn_formula* fs, int32_t n, tn_order_kind kind, uint64_t seed,
                                    const tn_contract_opts* opts, uint32_t* limbs, size_t cap_per,
                                    size_t* n_limbs, tn_plan_stats* stats) {
    (void)fs; (void)n; (void)kind; (void)seed; (void)opts; (void)limbs; (void)cap_per; (void)n_limbs; (void)stats;
    return TN_EUNSUPPORTED;
}
