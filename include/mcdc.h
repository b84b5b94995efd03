/*
 * mcdc.h — C ABI of the MI355X (gfx950) Monte Carlo transport library.
 *
 * The library runs the fixed-source, time-dependent particle-history loop
 * (scatter + absorb, no fission) of the paper "Performant and Portable Monte
 * Carlo Neutron Transport via Numba": particles are created and transported
 * until a physical event (capture, time or space boundary), a simulation event
 * (time census) or a variance-reduction event (implicit capture, weight
 * window) ends them, and their track lengths are tallied with a statistical
 * error (Sec. "Monte Carlo Neutron Transport and MC/DC"; transport-loop
 * paragraph of Sec. "MC/DC on CPUs").  The boundary mirrors the paper's
 * problem statement: inputs are sources, materials, geometry and tallies;
 * outputs are tallies with their statistical error.
 *
 * Conventions
 *  - Every function returns an mcdc_status (0 = OK, negative = error) and on
 *    error sets a thread-local message readable with mcdc_last_error().
 *    No C++ exception crosses this boundary.
 *  - Pointers documented "device" are HIP device pointers (e.g. the data
 *    pointer of a torch tensor on cuda:0); "host" pointers are ordinary memory.
 *  - Streams are hipStream_t passed as void* (0 = the null stream).
 *  - A handle is not thread safe; distinct handles are independent.
 *  - Results are deterministic: the same problem, seed and cumulative history
 *    count give the same per-history trajectories on any schedule or stream;
 *    tally sums agree up to the order of floating-point additions.
 *  - All positions, times, weights and tallies are IEEE binary64.
 */
#ifndef MCDC_H
#define MCDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCDC_OK = 0,
    MCDC_E_INVALID = -1,     /* bad argument or problem description          */
    MCDC_E_NOMEM = -2,       /* workspace too small                          */
    MCDC_E_HIP = -3,         /* a HIP runtime call failed                    */
    MCDC_E_EVENT_CAP = -4,   /* a history exceeded max_events flights        */
    MCDC_E_CANCELLED = -5,   /* reserved                                     */
    MCDC_E_STATE = -6,       /* call not valid in the handle's current state */
    MCDC_E_STACK = -7,       /* split daughters exceeded stack_cap           */
    MCDC_E_BANK = -8,        /* event-mode particle bank overflow            */
} mcdc_status;

enum { MCDC_VACUUM = 0, MCDC_REFLECTIVE = 1 };
enum { MCDC_SRC_POINT = 0, MCDC_SRC_BOX = 1 };
/* Schedules.  HISTORY: one work-item follows a history and its split
 * daughters to the end.  EVENT: particles live in banks and move through the
 * transport loop one event class per launch.  HYBRID: one work-item follows
 * each history until its first weight-window split (or, with population
 * control or census-step control, its first census); the particles it then
 * holds go to the event banks and finish there.  HYBRID uses the EVENT
 * schedule's workspace and supports everything it does. */
enum { MCDC_SCHED_AUTO = 0, MCDC_SCHED_HISTORY = 1, MCDC_SCHED_EVENT = 2, MCDC_SCHED_HYBRID = 3 };
enum { MCDC_TALLY_MESH = 0, MCDC_TALLY_DETECTOR = 1, MCDC_TALLY_LEAKAGE = 2,
       MCDC_TALLY_COLLISION = 3, MCDC_TALLY_SURFACE = 4 };

#define MCDC_MAX_BOXES 16
#define MCDC_MAX_MAT 16
#define MCDC_MAX_G 8
#define MCDC_MAX_CENSUS 64
#define MCDC_MLP_HIDDEN 64

/* Problem description (plain data; copied by mcdc_create_problem, so the
 * caller may free it afterwards).  Array pointers are host pointers. */
typedef struct {
    double outer_lo[3], outer_hi[3];   /* outer box; +-inf allowed for slabs      */
    int32_t bc[6];                     /* faces -x,+x,-y,+y,-z,+z                 */
    int32_t n_boxes;                   /* <= MCDC_MAX_BOXES priority-ordered cells */
    const double *box_lo, *box_hi;     /* [n_boxes][3]                            */
    const int32_t *box_mat;            /* [n_boxes]                               */
    int32_t background_mat;            /* material outside every box              */
    int32_t n_mat, G;                  /* materials, energy groups                */
    const double *sigma_t;             /* [n_mat][G] total cross section, 1/cm    */
    const double *sigma_s;             /* [n_mat][G][G] scattering, row = from    */
    const double *speed;               /* [G] cm/s                                */
    int32_t src_kind;                  /* MCDC_SRC_POINT (at src_lo) or _BOX      */
    double src_lo[3], src_hi[3];
    double src_t0, src_t1;             /* birth time uniform on [t0,t1]           */
    int32_t src_isotropic;             /* else direction src_dir                  */
    double src_dir[3];
    int32_t src_group;
    double mesh_lo[4], mesh_hi[4];     /* x,y,z,t; an x/y/z axis with both bounds */
    int32_t mesh_n[4];                 /*   infinite is not cut (n must be 1)     */
    int32_t mesh_per_group;            /* tally per group or summed over groups   */
    int32_t col_tally;                 /* 1: also a collision-estimator tally on
                                          the mesh (w / Sigma_t per collision in
                                          the bin of the collision point)         */
    int32_t surf_on;                   /* 1: also a surface-current tally on the
                                          plane x[surf_axis] = surf_pos: every
                                          flight crossing it adds its weight to
                                          the bin [side][g][t][b2][b1] of the
                                          crossing (side 0: moving toward +axis;
                                          g as the mesh; t and the other two axes
                                          b1 < b2 binned as the mesh)             */
    int32_t surf_axis;                 /* 0 x, 1 y, 2 z                           */
    double surf_pos;
    int32_t pc_on;                     /* 1: population control at every
                                          intermediate census (event or hybrid
                                          schedule; event_chunk >= histories per
                                          batch):
                                          each batch's census bank is split /
                                          rouletted to round(pc_target * batch
                                          histories) particles of equal weight    */
    double pc_target;                  /* census population per source history   */
    int32_t n_census;                  /* increasing census times, last = end     */
    const double *census;
    int32_t implicit_capture;          /* 0 analog; 1 implicit with weight cutoff */
    double w_cut, w_surv;
    int32_t has_detector;              /* detector box: per-history track length  */
    double det_lo[3], det_hi[3];
    int32_t imp_on;                    /* coarse importance estimate (analog only) */
    int32_t imp_n[4];                  /* its x,y,z,t cells                        */
    int32_t n_batches;                 /* batches per run for mesh statistics     */
    int64_t max_events;                /* flights per history before an error     */
    int32_t stack_cap;                 /* split daughters held per history (history
                                          schedule: more is MCDC_E_STACK; hybrid
                                          lead stage: more go to the event banks) */
    uint32_t problem_id;               /* part of every RNG counter               */
} mcdc_problem_desc;

/* Schedule and launch knobs (0 = library default). */
typedef struct {
    int32_t schedule;                  /* MCDC_SCHED_*                            */
    int32_t block;                     /* work-items per workgroup (multiple of 64) */
    int32_t waves_per_cu;              /* persistent-grid occupancy target        */
    int32_t lds_tally;                 /* 1 allow, 0 forbid an LDS tally tile     */
    int64_t event_chunk;               /* event and hybrid schedules: histories
                                          resident at once (at most 2^26);
                                          batched runs: entries per work chunk    */
    /* History schedule and the hybrid schedule's lead stage: a sub-box of the
     * tally mesh held in LDS per workgroup (bins [tile_lo, tile_lo + tile_n)
     * along x, y, z, t, group), flushed to HBM at the end of each launch (the
     * lead stage: for the batch of the workgroup's history range); all
     * tile_n > 0 enables it (at most MCDC_MAX_TILE_BINS bins; workgroups of
     * 1024 work-items).  Place it where most track-length pieces fall (e.g.
     * from a pilot run's tally). */
    int32_t tile_lo[5], tile_n[5];
} mcdc_options;

#define MCDC_MAX_TILE_BINS 19456

/* Counters (all runs since create / reset). */
typedef struct {
    uint64_t histories, flights, pieces, collisions, absorptions, surfaces, leaks,
        census_stops, time_ends, splits, rr_kills, rr_survivals, cutoff_kills,
        cutoff_survivals, detector_hits, particles;
    double w_source, w_leak, w_absorb, w_time_end, w_gain, w_loss, path;
    double leak[6];
    double det_sum, det_sumsq;
    int64_t batches;
    uint64_t n_hist;
    int32_t status;                    /* sticky device error status             */
    uint64_t event_iterations;         /* event and hybrid schedules: stage
                                          iterations launched                     */
    uint64_t pc_kills, pc_copies;      /* population control: removed / added      */
    uint64_t surf_crossings;           /* scored surface-tally crossings          */
    uint64_t ww_plane_stops;           /* flights ended on a window grid plane    */
} mcdc_counters;

typedef struct mcdc_problem *mcdc_handle;

/* Bytes of device workspace a problem needs under the given options.  Pure. */
int mcdc_workspace_bytes(const mcdc_problem_desc *d, const mcdc_options *opt, size_t *bytes);

/* Validate and copy the description, carve the caller-owned device workspace
 * (must stay allocated until mcdc_destroy_problem) and upload the tables
 * (synchronous host-to-device copies).  Tallies start at zero. */
int mcdc_create_problem(const mcdc_problem_desc *d, const mcdc_options *opt, void *dev_workspace,
                        size_t bytes, mcdc_handle *out);

/* Transport n_histories source histories with random key `seed`, enqueued
 * asynchronously on `stream`.  History ids continue from earlier runs of the
 * handle; the run is split into n_batches equal id ranges whose tally sums
 * feed the batch statistics.  Results accumulate across runs. */
int mcdc_run(mcdc_handle h, uint64_t n_histories, uint64_t seed, void *stream);

/* A run taken census step by census step (event or hybrid schedule; all histories
 * resident: n_histories <= event_chunk; with population control, n_batches
 * must be 1).  mcdc_run_begin samples the sources and returns; each
 * mcdc_run_step transports until the next census step begins, or to the end
 * of the run (*done = 1, after which the results include the run, as after
 * mcdc_run with the same arguments).  Between steps the whole state of the
 * run lives in the caller-owned workspace and in the host record below, so a
 * run is checkpointed by copying both, and resumed by copying them into a
 * handle created from the same description and options (then
 * mcdc_set_run_state) and stepping on.  The per-history outputs of
 * mcdc_set_history_scores are written when the run ends.  Steps synchronise
 * `stream`.  MCDC_E_STATE for a step without a run in progress. */
typedef struct {
    uint64_t magic;                    /* identifies the record layout           */
    uint64_t workspace_bytes, bins;    /* of the handle that wrote it            */
    uint64_t n_hist, batches, event_iterations;
    uint64_t run_first, run_n, run_seed;
    double pc_m;
    int32_t in_run, steps;
} mcdc_run_state;
int mcdc_run_begin(mcdc_handle h, uint64_t n_histories, uint64_t seed, void *stream);
int mcdc_run_step(mcdc_handle h, int32_t *done, void *stream);
int mcdc_get_run_state(mcdc_handle h, mcdc_run_state *out);
int mcdc_set_run_state(mcdc_handle h, const mcdc_run_state *in);

/* Synchronise `stream` and copy results to the host: per-bin mean score per
 * source history divided by bin volume and time width (MCDC_TALLY_MESH,
 * n = bins; MCDC_TALLY_COLLISION the same from the collision estimator, for
 * problems created with col_tally), per surface bin the mean crossing weight
 * per source history divided by the bin's area and time width
 * (MCDC_TALLY_SURFACE, n = mcdc_surface_bins; problems created with
 * surf_on), the detector mean track length per
 * history (n = 1), or the leaked weight per face per history (n = 6);
 * rel_err may be NULL.  Returns the sticky device error status if a run
 * failed. */
int mcdc_get_tallies(mcdc_handle h, int kind, double *mean, double *rel_err, size_t n,
                     void *stream);

/* Raw accumulators (host copies): tally_sum[n] = sum of batch sums,
 * tally_sumsq[n] = sum of (batch sum)^2 / batch size; either may be NULL. */
int mcdc_get_raw(mcdc_handle h, double *tally_sum, double *tally_sumsq, size_t n, void *stream);

/* The same raw accumulators of the collision-estimator tally (problems
 * created with col_tally; MCDC_E_STATE otherwise). */
int mcdc_get_raw_collision(mcdc_handle h, double *col_sum, double *col_sumsq, size_t n,
                           void *stream);
/* The same for the surface-current tally (problems created with surf_on;
 * MCDC_E_STATE otherwise); n = mcdc_surface_bins = 2 * G_t * nt * n_b1 * n_b2. */
int mcdc_get_raw_surface(mcdc_handle h, double *surf_sum, double *surf_sumsq, size_t n,
                         void *stream);
int mcdc_surface_bins(mcdc_handle h, size_t *n);
int mcdc_get_counters(mcdc_handle h, mcdc_counters *out, void *stream);
int mcdc_reset_tallies(mcdc_handle h, void *stream);
int mcdc_tally_bins(mcdc_handle h, size_t *n);

/* Debug outputs for parity checks (device buffers owned by the caller, NULL to
 * disable): a trace of every event as mcdc_trace_rec records (appended in
 * completion order; `count` is a device uint64 the library increments), and
 * per-history results of later runs: dev_xh[2 i] = detector score and
 * dev_xh[2 i + 1] = sum of weight * flight length of history (run's first id
 * + i), both summed in the history's event order. */
typedef struct {
    uint64_t hist;
    uint32_t tag, seq;
    int32_t type, g, cell;
    uint32_t k;
    double x, y, z, t, ux, uy, uz, w, aux;
} mcdc_trace_rec;
int mcdc_set_trace(mcdc_handle h, mcdc_trace_rec *dev_buf, uint64_t cap, uint64_t *dev_count);
int mcdc_set_history_scores(mcdc_handle h, double *dev_xh);

/* Learned weight windows: copy an MLP (in = 4 + G inputs scaled to [-1,1]
 * over the outer box and [0, end time], 64 -> 64 ReLU hidden units, 1 output
 * = log importance; FP32, layout W1,b1,W2,b2,W3,b3) into the workspace and
 * turn splitting/roulette on: y = network output clamped to [ymin, ymax]
 * (the range of its training targets), target w_T = exp(logk - y), window
 * [2 w_T/(1+ratio), ratio * 2 w_T/(1+ratio)], at most n_max copies, checked
 * after every scatter and internal surface crossing.  Needs a problem created
 * with stack_cap > 0.  params == NULL turns weight windows off. */
int mcdc_set_ww_mlp(mcdc_handle h, const float *params, size_t n_params, double logk,
                    double ratio, int32_t n_max, float ymin, float ymax);

/* Weight-window map: evaluate the network set by mcdc_set_ww_mlp once at the
 * centre of every cell of a regular map, n = (nx, ny, nz, nt) cells over the
 * outer box and [0, end time] per group (centre inputs 2 (i + 1/2)/n - 1), and
 * from then on take w_T at a check from the map cell that holds the particle
 * (per axis floor(s n), s the point's fraction of the range, clamped to
 * [0, n-1]).  dev_map is caller-owned device memory of at least
 * G * nx * ny * nz * nt doubles (layout [g][t][z][y][x], filled with w_T on
 * `stream`; it must stay allocated while the map is in use).  Each n[a] lies
 * in [1, 65536] and the map holds at most 2^26 cells.  dev_map == NULL goes
 * back to evaluating the network at every check; mcdc_set_ww_mlp also does,
 * so a new network needs a new call.  MCDC_E_STATE without a network,
 * MCDC_E_NOMEM when capacity (in doubles) is too small. */
int mcdc_set_ww_map(mcdc_handle h, const int32_t n[4], double *dev_map, size_t capacity,
                    void *stream);

/* Weight-window grid planes (a reading: the paper places no window checks):
 * besides after collisions and surface crossings, the windows are checked
 * where a flight reaches an interior plane of a regular n[0] x n[1] x n[2]
 * grid over the outer box (planes lo + k (hi - lo) / n, k = 1..n-1 per axis;
 * the flight stops on the plane; ties: census, surface, plane, collision).
 * n == NULL or all zero turns the planes off.  Each n[a] lies in [1, 65536].
 * MCDC_E_STATE without a network. */
int mcdc_set_ww_grid(mcdc_handle h, const int32_t n[3]);

/* Coarse importance estimate accumulated by runs with imp_on: host copies of
 * score[c] and weight[c] for G * imp_n[0..3] cells (x fastest, then y, z, t, g). */
int mcdc_get_importance(mcdc_handle h, double *score, double *weight, size_t n, void *stream);

/* ------------------------------------------------------------------------ */
/* MLP training (log-importance regression), device buffers, FP32.          */
/* Loss = sum_i wt_i (f(x_i) - y_i)^2 / sum_i wt_i; Adam(lr, b1, b2, eps).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t steps;
    float lr, beta1, beta2, eps;
} mcdc_train_opts;

/* Forward pass: out[n] = f(X[n][in_dim]). */
int mcdc_mlp_forward(const float *dev_params, int32_t in_dim, const float *dev_X, size_t n,
                     float *dev_out, void *stream);
/* Device scratch (bytes) that mcdc_mlp_grad / mcdc_mlp_train need for n points. */
size_t mcdc_mlp_scratch_bytes(int32_t in_dim, size_t n);
/* Loss and gradient: grad[n_params] (overwritten), loss (device scalar, may be
 * NULL).  The gradient is summed over points in a fixed order. */
int mcdc_mlp_grad(const float *dev_params, int32_t in_dim, const float *dev_X, const float *dev_y,
                  const float *dev_wt, size_t n, float *dev_grad, float *dev_loss,
                  void *dev_scratch, void *stream);
/* `steps` Adam steps in place on dev_params; dev_m, dev_v (n_params each) hold
 * the moments and must start at zero; step numbering continues from
 * *step_io (host, updated).  dev_grad (may be NULL) receives the last
 * gradient; dev_loss_hist (steps floats, may be NULL) the loss before each step. */
int mcdc_mlp_train(float *dev_params, int32_t in_dim, const float *dev_X, const float *dev_y,
                   const float *dev_wt, size_t n, float *dev_m, float *dev_v, float *dev_grad,
                   const mcdc_train_opts *o, int32_t *step_io, float *dev_loss_hist,
                   void *dev_scratch, void *stream);
size_t mcdc_mlp_param_count(int32_t in_dim);

/* ------------------------------------------------------------------------ */
/* Batched problems: many independent problems in one persistent launch per  */
/* census step, census steps captured in a HIP graph.                         */
/* ------------------------------------------------------------------------ */
int mcdc_batch_workspace_bytes(const mcdc_problem_desc *ds, size_t n, const uint64_t *n_hist,
                               const mcdc_options *opt, size_t *bytes);
int mcdc_create_batch(const mcdc_problem_desc *ds, size_t n, const uint64_t *n_hist,
                      const mcdc_options *opt, void *dev_workspace, size_t bytes,
                      mcdc_handle *out);
/* One pass of every problem's histories (ids continue across passes). */
int mcdc_run_batch(mcdc_handle h, uint64_t seed, void *stream);
/* Raw mesh sums of problem p (host copy, n = its bins). */
int mcdc_get_batch_raw(mcdc_handle h, size_t p, double *tally_sum, size_t n, void *stream);
int mcdc_get_batch_counters(mcdc_handle h, size_t p, mcdc_counters *out, void *stream);
/* Per-history sum of weight * flight length of problem p for the histories of
 * the last pass, summed in event order (host copy, n = its histories). */
int mcdc_get_batch_history_path(mcdc_handle h, size_t p, double *out, size_t n, void *stream);

/* Kernel timing: with `on` = 1, later runs record a pair of HIP events on the
 * run's stream around every launch of the schedule's tracking kernel (history
 * schedule: the history kernel; event schedule: the flight stage; hybrid
 * schedule: the lead stage); mcdc_kernel_time
 * synchronises them and returns the number of launches recorded since the last
 * call and their summed duration in milliseconds (then forgets them). */
int mcdc_set_kernel_timing(mcdc_handle h, int on);
int mcdc_kernel_time(mcdc_handle h, uint64_t *launches, double *total_ms);

/* Micro-benchmarks for the measured roofline ceilings (not on the transport
 * path).  mcdc_micro_atomics: n_items work-items each add 1.0 to per_item bins
 * of dev_buf[n_bins], in runs of `run` consecutive bins starting at hashed
 * positions (run = 1: uniformly scattered).  mcdc_micro_copy: stream `bytes`
 * (a multiple of 32) from dev_src to dev_dst.  Both are asynchronous on
 * `stream`; the caller times them. */
int mcdc_micro_atomics(double *dev_buf, uint64_t n_bins, uint64_t n_items, uint32_t per_item,
                       uint32_t run, void *stream);
int mcdc_micro_copy(const void *dev_src, void *dev_dst, size_t bytes, void *stream);

void mcdc_destroy_problem(mcdc_handle h);
const char *mcdc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
