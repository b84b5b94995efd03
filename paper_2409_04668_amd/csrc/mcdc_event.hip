// Event-based schedule (placeholder until the staged kernels land).
#include "mcdc_runtime.hpp"

namespace mcdc {
size_t event_workspace_bytes(const mcdc_problem_desc *, const Options &o) { return 0; }
int event_init(mcdc_problem *) { return fail(MCDC_E_INVALID, "event schedule not available"); }
int event_run_range(mcdc_problem *, const RunArgs &, hipStream_t) {
    return fail(MCDC_E_INVALID, "event schedule not available");
}
void event_destroy(mcdc_problem *) {}
}  // namespace mcdc
