// Host-side handle state shared by the runtime translation units.
#pragma once

#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "mcdc_internal.hpp"

namespace mcdc {

struct Options {
    int schedule, block, waves_per_cu, lds_tally;
    bool lead;                           // event schedule with the history-style lead stage
    int64_t event_chunk;
    int32_t tile_lo[5], tile_n[5];
    uint32_t tile_bins;                  // 0: no hot tile
    int grid;
    uint64_t n_lanes;
};

struct EventState;
struct BatchState;

}  // namespace mcdc

struct mcdc_problem {
    mcdc_problem_desc desc;
    mcdc::Options opt;
    mcdc::Layout L;
    mcdc::DevProblem P;
    char *ws = nullptr;
    uint32_t nbins = 0;
    size_t nimp = 0;
    uint64_t n_hist = 0;
    uint64_t event_iterations = 0;
    // a run taken step by step: segment by segment (resident chunks, or
    // batches), each event-schedule segment census step by census step
    bool in_run = false;
    int32_t run_steps = 0;
    uint64_t run_first = 0, run_n = 0, run_seed = 0;
    uint64_t run_seg = 0;
    int64_t batches = 0;
    mcdc_trace_rec *trace = nullptr;
    uint64_t trace_cap = 0;
    unsigned long long *trace_count = nullptr;
    double *xh_out = nullptr;
    bool is_batch = false;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    mcdc::EventState *ev = nullptr;
    mcdc::BatchState *batch = nullptr;
    // cancel word: pinned, host-coherent memory that kernels read while the
    // host may write it (cancel_dev is its device address)
    int *cancel_host = nullptr;
    int *cancel_dev = nullptr;
};

namespace mcdc {

int fail(int st, const std::string &msg);
// allocate / free the handle's cancel word; is a cancel requested?
int cancel_init(mcdc_problem *h);
void cancel_free(mcdc_problem *h);
inline bool cancel_set(const mcdc_problem *h) {
    return h->cancel_host && __atomic_load_n(h->cancel_host, __ATOMIC_ACQUIRE) != 0;
}
int hip_fail(hipError_t e, const char *where);
// kernel timing: record a start event before / a stop event after a launch
void timing_begin(mcdc_problem *h, hipStream_t s);
void timing_end(mcdc_problem *h, hipStream_t s);

// event-based schedule (mcdc_event.hip)
size_t event_workspace_bytes(const mcdc_problem_desc *d, const Options &o);
int event_init(mcdc_problem *h);
int event_run_range(mcdc_problem *h, const RunArgs &A, hipStream_t s);
uint64_t ev_resident_histories(const mcdc_problem *h);   // histories per resident chunk
// census-step control: begin (sources) and one step; `done` when the run ended
int event_begin(mcdc_problem *h, const RunArgs &A, hipStream_t s);
int event_step(mcdc_problem *h, const RunArgs &A, hipStream_t s, bool &done);
void event_destroy(mcdc_problem *h);

// batched problems (mcdc_batch.hip)
void batch_destroy(mcdc_problem *h);

// shared host helpers (mcdc_api.hip)
int validate_desc(const mcdc_problem_desc *d);
int desc_fissile(const mcdc_problem_desc *d);
uint32_t desc_nbins(const mcdc_problem_desc *d);
size_t desc_nsurf(const mcdc_problem_desc *d);
Options resolve_options(const mcdc_options *o);
void build_dev_problem(const mcdc_problem_desc *d, char *ws, const Layout &L, DevProblem &P);
std::vector<double> pack_tables(const mcdc_problem_desc *d);
void fill_counters(const DevAcc &a, mcdc_counters *o);
// the run arguments every tracking launch of the handle starts from
RunArgs base_args_for(mcdc_problem *h, uint64_t seed);

}  // namespace mcdc
