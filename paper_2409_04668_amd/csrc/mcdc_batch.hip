// Batched problems (placeholder until the persistent batched kernel lands).
#include "mcdc_runtime.hpp"

namespace mcdc {
void batch_destroy(mcdc_problem *) {}
}  // namespace mcdc

using namespace mcdc;

extern "C" {
int mcdc_batch_workspace_bytes(const mcdc_problem_desc *, size_t, const uint64_t *,
                               const mcdc_options *, size_t *) {
    return fail(MCDC_E_INVALID, "batched problems not available");
}
int mcdc_create_batch(const mcdc_problem_desc *, size_t, const uint64_t *, const mcdc_options *,
                      void *, size_t, mcdc_handle *) {
    return fail(MCDC_E_INVALID, "batched problems not available");
}
int mcdc_run_batch(mcdc_handle, uint64_t, void *) { return fail(MCDC_E_INVALID, "batched problems not available"); }
int mcdc_get_batch_raw(mcdc_handle, size_t, double *, size_t, void *) {
    return fail(MCDC_E_INVALID, "batched problems not available");
}
int mcdc_get_batch_counters(mcdc_handle, size_t, mcdc_counters *, void *) {
    return fail(MCDC_E_INVALID, "batched problems not available");
}
}
