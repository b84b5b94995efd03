/*
 * mcdc.h — C ABI of the MI355X (gfx950) Monte Carlo transport library.
 *
 * The library runs the fixed-source, time-dependent particle-history loop
 * (scatter + absorb) of the paper "Performant and Portable Monte Carlo
 * Neutron Transport via Numba": particles are created and transported until a
 * physical event (capture, time or space boundary), a simulation event (time
 * census) or a variance-reduction event (implicit capture, weight window)
 * ends them, and their track lengths are tallied with a statistical error
 * (Sec. "Monte Carlo Neutron Transport and MC/DC"; transport-loop paragraph
 * of Sec. "MC/DC on CPUs").  Problems with fission data run the paper's
 * k-eigenvalue mode instead (mcdc_run_keff).  The boundary mirrors the paper's
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
    MCDC_E_CANCELLED = -5,   /* the run was cancelled with mcdc_set_cancel   */
    MCDC_E_STATE = -6,       /* call not valid in the handle's current state */
    MCDC_E_STACK = -7,       /* split daughters exceeded stack_cap           */
    MCDC_E_BANK = -8,        /* event-mode particle bank or fission site bank
                                overflow                                     */
    MCDC_E_EXTINCT = -9,     /* k-eigenvalue: a generation produced no site  */
} mcdc_status;

enum { MCDC_VACUUM = 0, MCDC_REFLECTIVE = 1 };
enum { MCDC_SRC_POINT = 0, MCDC_SRC_BOX = 1 };
/* Schedules (the paper's GPU discussion, Sec. "MC/DC on GPUs": a history per
 * thread diverges; grouping like operations is the remedy).
 * HISTORY: one work-item follows a history and its split daughters (on a
 * per-lane stack) to the end.
 * EVENT: particles live in banks and move through the transport loop one
 * event class per launch.
 * HYBRID: a lead stage follows each history in one work-item, split daughters
 * on its stack (daughters past a full stack go to the banks at once), for at
 * most 32 flights of that history (MCDC_LEAD_FLIGHTS in the library); then
 * the particle and its stacked daughters go to the banks.  A re-lead stage
 * follows each banked particle the same way, for at most 8 flights of it and
 * its daughters (MCDC_RELEAD_FLIGHTS), banking what is left for its next
 * launch, until the banks are empty.  With population control or census-step
 * control a particle that reaches an intermediate census goes to the census
 * bank instead.  Analog histories that end within the budget never touch the
 * banks.  HYBRID uses the EVENT schedule's workspace and supports everything
 * it does. */
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
    const double *nu_sigma_f;          /* [n_mat][G] fission neutrons per cm
                                          (nu Sigma_f), or NULL: a problem with any
                                          positive entry runs in the k-eigenvalue
                                          mode only (mcdc_run_keff)              */
    const double *chi;                 /* [n_mat][G] fission spectrum: relative
                                          weights of the outgoing group (needed
                                          with nu_sigma_f)                        */
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

/* Every declaration below ends its comment with a "Source:" line: the passage
 * of the paper that defines the operation, or, where the paper defines none,
 * what the call is for. */

/* Bytes of device workspace a problem needs under the given options.  Pure
 * (no device call).  MCDC_E_INVALID for a bad description or options.
 * Source: Sec. "MC/DC on CPUs", initialization (one global state holding the
 * inputs, meshes, particle banks and tallies, allocated before transport). */
int mcdc_workspace_bytes(const mcdc_problem_desc *d, const mcdc_options *opt, size_t *bytes);

/* Validate and copy the description, carve the caller-owned device workspace
 * (dev_workspace: at least `bytes` from mcdc_workspace_bytes; it must stay
 * allocated until mcdc_destroy_problem) and upload the tables (synchronous
 * host-to-device copies).  Tallies start at zero.  *out receives the handle,
 * owned by the caller until mcdc_destroy_problem.  MCDC_E_NOMEM when bytes is
 * too small.
 * Source: Sec. "Monte Carlo Neutron Transport and MC/DC" (a problem is its
 * sources, materials, geometry and tallies) and Sec. "MC/DC on CPUs"
 * (the input handler builds that state once). */
int mcdc_create_problem(const mcdc_problem_desc *d, const mcdc_options *opt, void *dev_workspace,
                        size_t bytes, mcdc_handle *out);

/* Transport n_histories source histories with random key `seed`, enqueued
 * asynchronously on `stream` (the event and hybrid schedules synchronise it
 * every few stage iterations).  History ids continue from earlier runs of the
 * handle; the run is split into n_batches equal id ranges whose tally sums
 * feed the batch statistics.  Results accumulate across runs.  Device errors
 * (event cap, stack, bank, cancel) are sticky and reported by the read-back
 * calls; MCDC_E_CANCELLED is also returned here when the cancel word is set.
 * Source: Sec. "MC/DC on CPUs", transport-loop paragraph (loop over the
 * particles; transport each until a physical, simulation or variance-reduction
 * event ends its history); straight-line motion between events (the
 * particle-state example of Fig. 2). */
int mcdc_run(mcdc_handle h, uint64_t n_histories, uint64_t seed, void *stream);

/* k-eigenvalue mode: power iteration on the fission source, n_inactive +
 * n_active generations of M histories each (history ids g M + j, j < M; the
 * handle must be fresh or reset, created for the history schedule, without
 * weight windows or the importance estimate, and with fission data).
 *   - Generation 0 starts from the problem's source, generation g > 0 from M
 *     fission sites of generation g - 1 (position and group; t = 0, unit
 *     weight, an isotropic direction from the history's own stream).
 *   - At every collision with nu Sigma_f > 0: prod = w nu Sigma_f / Sigma_t
 *     adds to the generation's collision estimate, and floor(prod / k_norm +
 *     xi) sites are made at the collision point (groups from the material's
 *     spectrum); then the collision goes on as in the fixed-source mode.
 *   - After generation g with S sites: k_col[g] = (sum of prod) / M,
 *     k_site[g] = k_norm S / M, n_sites[g] = S; k_norm (k0 for generation 0)
 *     becomes k_site[g]; the next source is M sites combed out of the S in
 *     production order (by history slot, then within the history), site
 *     floor((j + xi) S / M) for j < M (at most S - 1), xi the first draw of
 *     the stream of history id (g + 1) M with tag 0x6B656666.
 *   - Active generations score the tallies and detector, each closed out as
 *     one batch of M histories; inactive ones discard what they scored.
 * dev_workspace: caller-owned device memory of mcdc_keff_workspace_bytes(M)
 * bytes (site banks, the combed source; free after the call).  k_col, k_site,
 * n_sites: host arrays of n_inactive + n_active entries (each may be NULL).
 * The generations follow each other on `stream` without a host round trip;
 * the call synchronises it once per 64 generations to collect their results.
 * MCDC_E_BANK when a generation makes more than 4 M + 1024 sites, or when a
 * single collision would make more than that (start with k0 nearer k),
 * MCDC_E_EXTINCT when it makes none; the outputs then hold the generations
 * up to the failed one.
 * Source: Sec. "Monte Carlo Neutron Transport and MC/DC" (the k-eigenvalue
 * mode beside the time-dependent one) and Sec. "MC/DC on CPUs" (fission as a
 * physical event that ends a history; daughter particles from fission in the
 * kernel set). */
typedef struct {
    uint64_t M;                        /* histories per generation, 1 .. 2^28     */
    int32_t n_inactive, n_active;      /* generations discarded / scored (>= 1)   */
    double k0;                         /* normalisation of generation 0 (> 0)     */
} mcdc_keff_opts;

/* Device workspace bytes of mcdc_run_keff for M histories per generation.
 * Source: as mcdc_run_keff. */
int mcdc_keff_workspace_bytes(uint64_t M, size_t *bytes);

/* Run the k-eigenvalue iteration (see above).
 * Source: as described above (Sec. "Monte Carlo Neutron Transport and MC/DC"). */
int mcdc_run_keff(mcdc_handle h, const mcdc_keff_opts *o, uint64_t seed, void *dev_workspace,
                  size_t bytes, double *k_col, double *k_site, uint64_t *n_sites, void *stream);

/* Cancel word of the handle: on != 0 asks every later and every running
 * launch of the handle's runs to stop (in the persistent kernels one
 * work-item per workgroup reads it from host-coherent memory before the
 * first history and at every 64th history (or banked particle) it starts,
 * and shares it in LDS; every work-item checks that copy when it starts a
 * history or banked particle, and a batched
 * run's workgroups read it every 8th work chunk; they then end early,
 * leaving histories in flight unfinished; the host side of
 * mcdc_run / mcdc_run_step / mcdc_run_batch stops launching and returns
 * MCDC_E_CANCELLED); the results of a cancelled run are incomplete and carry
 * the sticky status MCDC_E_CANCELLED until mcdc_reset_tallies.  on = 0
 * clears the word.  The one call that may be made from another thread while
 * a run of the handle is in flight.
 * Source: not in the paper (failure handling for long runs). */
int mcdc_set_cancel(mcdc_handle h, int on);

/* A run taken step by step, with the same results as mcdc_run with the same
 * arguments.  It goes segment by segment in mcdc_run's order: under the
 * event and hybrid schedules the resident chunks of event_chunk histories
 * (with population control, the batches instead, each at most event_chunk
 * histories, controlled on its own), and each of these census step by census
 * step; under the history schedule the batches, one step each (a history
 * runs through every census time within its launch).  mcdc_run_begin samples
 * the first segment's sources and returns; each mcdc_run_step transports to
 * the next census step or to the end of a segment (then the next segment's
 * sources are sampled), or to the end of the run (*done = 1, after which the
 * results include the run).  Between steps the whole state of the run lives
 * in the caller-owned workspace and in the host record below, so a run is
 * checkpointed by copying both, and resumed by copying them into a handle
 * created from the same description and options (then mcdc_set_run_state)
 * and stepping on.  The per-history outputs of mcdc_set_history_scores are
 * written as each segment ends (a checkpoint of a run that asks for them
 * copies that array too).  Steps synchronise `stream`.  MCDC_E_STATE
 * for a step without a run in progress, and for other runs while one is. */
typedef struct {
    uint64_t magic;                    /* identifies the record layout           */
    uint64_t workspace_bytes, bins;    /* of the handle that wrote it            */
    uint64_t n_hist, batches, event_iterations;
    uint64_t run_first, run_n, run_seed;
    uint64_t segment;                  /* segment of the run in progress         */
    int32_t in_run, steps;
} mcdc_run_state;

/* Start a stepped run (see above).
 * Source: Sec. "Monte Carlo Neutron Transport and MC/DC" (time census and
 * time-dependent population control among the features) and the
 * transport-loop paragraph of Sec. "MC/DC on CPUs" (time census as a
 * simulation event that ends a flight). */
int mcdc_run_begin(mcdc_handle h, uint64_t n_histories, uint64_t seed, void *stream);

/* Transport to the next census step, the end of a segment, or the end of
 * the run (*done).
 * Source: as mcdc_run_begin. */
int mcdc_run_step(mcdc_handle h, int32_t *done, void *stream);

/* Host record of the run in progress (for a checkpoint).
 * Source: not in the paper (checkpoint/resume at a census step). */
int mcdc_get_run_state(mcdc_handle h, mcdc_run_state *out);

/* Restore a host record into a handle made from the same description and
 * options whose workspace holds the matching copy.  MCDC_E_INVALID for a
 * record of another layout or one that names no segment of its run.
 * Source: not in the paper (checkpoint/resume at a census step). */
int mcdc_set_run_state(mcdc_handle h, const mcdc_run_state *in);

/* Synchronise `stream` and copy the results to the host arrays mean[n] and
 * rel_err[n] (rel_err may be NULL):
 *   MCDC_TALLY_MESH (n = bins): per bin the mean score per source history
 *     divided by the bin's volume and time width (an unbounded axis is not
 *     cut); MCDC_TALLY_COLLISION the same from the collision estimator
 *     (problems created with col_tally);
 *   MCDC_TALLY_SURFACE (n = mcdc_surface_bins): per bin the mean crossing
 *     weight per source history divided by the bin's area on the plane and
 *     its time width (problems created with surf_on);
 *     for these three, rel_err = the batch-means standard error divided by
 *     the mean: sqrt((S2 - N m^2) / ((B - 1) N)) / m with m = S / N, S and S2
 *     the sums of the batch sums S_b and of S_b^2 / N_b, N the histories and
 *     B the non-empty batches; 0 where the mean is 0, NaN with B < 2;
 *   MCDC_TALLY_DETECTOR (n = 1): the mean track length per history in the
 *     detector box, rel_err from the per-history sample variance,
 *     sqrt((X2 / N - m^2) / (N - 1)) / m (0 for a zero mean, NaN for N < 2);
 *   MCDC_TALLY_LEAKAGE (n = 6): the weight leaked per face per history,
 *     rel_err NaN (no second moment is kept).
 * Returns the sticky device error status if a run failed; MCDC_E_STATE
 * before any history has run.
 * Source: Sec. "MC/DC on CPUs", finalization (the requested tallies with the
 * statistical error of the Monte Carlo process); Sec. "Monte Carlo Neutron
 * Transport and MC/DC" (tallies with an associated statistical error). */
int mcdc_get_tallies(mcdc_handle h, int kind, double *mean, double *rel_err, size_t n,
                     void *stream);

/* The same results written to device memory (dev_mean[n], dev_rel_err[n] or
 * NULL), computed by a kernel enqueued on `stream` with the same arithmetic
 * (bit-identical to mcdc_get_tallies).  Does not synchronise and does not
 * report device errors: read them with mcdc_get_counters.  MCDC_E_STATE while
 * a stepped run is in progress.
 * Source: as mcdc_get_tallies; kept on the device because the paper's GPU
 * profile counts host-device copies as a cost (Sec. "Performance"). */
int mcdc_get_tallies_device(mcdc_handle h, int kind, double *dev_mean, double *dev_rel_err,
                            size_t n, void *stream);

/* Raw accumulators (host copies): tally_sum[n] = sum of batch sums,
 * tally_sumsq[n] = sum of (batch sum)^2 / batch size; either may be NULL.
 * Source: Fig. 3 (tallies accumulated by adds, atomic on the GPU). */
int mcdc_get_raw(mcdc_handle h, double *tally_sum, double *tally_sumsq, size_t n, void *stream);

/* The same raw accumulators of the collision-estimator tally (problems
 * created with col_tally; MCDC_E_STATE otherwise).
 * Source: Fig. 3 (tallies scored at collision events). */
int mcdc_get_raw_collision(mcdc_handle h, double *col_sum, double *col_sumsq, size_t n,
                           void *stream);

/* The same for the surface-current tally (problems created with surf_on;
 * MCDC_E_STATE otherwise); n = mcdc_surface_bins = 2 * G_t * nt * n_b1 * n_b2.
 * Source: a reading; the paper tallies events but defines no surface tally
 * (Fig. 3). */
int mcdc_get_raw_surface(mcdc_handle h, double *surf_sum, double *surf_sumsq, size_t n,
                         void *stream);

/* Number of surface-current bins of the handle (0 without one).
 * Source: as mcdc_get_raw_surface. */
int mcdc_surface_bins(mcdc_handle h, size_t *n);

/* Counters of all runs since create or reset (synchronises `stream`).
 * Source: Sec. "MC/DC on CPUs" (events that end a history: capture, time and
 * space boundary, census, variance reduction), counted per kind. */
int mcdc_get_counters(mcdc_handle h, mcdc_counters *out, void *stream);

/* Zero the tallies, counters and sticky status (synchronises `stream`).
 * Source: Sec. "MC/DC on CPUs", initialization of the tallies. */
int mcdc_reset_tallies(mcdc_handle h, void *stream);

/* Number of mesh bins of the handle.
 * Source: Sec. "Monte Carlo Neutron Transport and MC/DC" (tallies over a
 * mesh; the paper's results are space-time mesh fluxes). */
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

/* Event trace of later runs (see above).
 * Source: Sec. "Monte Carlo Neutron Transport and MC/DC" (hash-based random
 * numbers for fully replicable testing): the trace is what replication is
 * checked on. */
int mcdc_set_trace(mcdc_handle h, mcdc_trace_rec *dev_buf, uint64_t cap, uint64_t *dev_count);

/* Per-history outputs of later runs (see above).
 * Source: as mcdc_set_trace. */
int mcdc_set_history_scores(mcdc_handle h, double *dev_xh);

/* Learned weight windows: copy an MLP (in = 4 + G inputs scaled to [-1,1]
 * over the outer box and [0, end time], 64 -> 64 ReLU hidden units, 1 output
 * = log importance; FP32, layout W1,b1,W2,b2,W3,b3) into the workspace and
 * turn splitting/roulette on: y = network output clamped to [ymin, ymax]
 * (the range of its training targets), target w_T = exp(logk - y), window
 * [2 w_T/(1+ratio), ratio * 2 w_T/(1+ratio)], at most n_max copies, checked
 * after every scatter and internal surface crossing.  Needs a problem created
 * with stack_cap > 0.  params == NULL turns weight windows off.
 * Source: not in the paper (weight windows from a learned importance map; the
 * paper names variance-reduction events and machine learning only for node
 * scheduling, Sec. "Monte Carlo Neutron Transport and MC/DC"). */
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
 * MCDC_E_NOMEM when capacity (in doubles) is too small.
 * Source: not in the paper (as mcdc_set_ww_mlp). */
int mcdc_set_ww_map(mcdc_handle h, const int32_t n[4], double *dev_map, size_t capacity,
                    void *stream);

/* Weight-window grid planes (a reading: the paper places no window checks):
 * besides after collisions and surface crossings, the windows are checked
 * where a flight reaches an interior plane of a regular n[0] x n[1] x n[2]
 * grid over the outer box (planes lo + k (hi - lo) / n, k = 1..n-1 per axis;
 * the flight stops on the plane; ties: census, surface, plane, collision).
 * n == NULL or all zero turns the planes off.  Each n[a] lies in [1, 65536].
 * MCDC_E_STATE without a network.
 * Source: not in the paper (as mcdc_set_ww_mlp). */
int mcdc_set_ww_grid(mcdc_handle h, const int32_t n[3]);

/* Coarse importance estimate accumulated by runs with imp_on: host copies of
 * score[c] and weight[c] for G * imp_n[0..3] cells (x fastest, then y, z, t, g).
 * Source: not in the paper (training data of the importance network: tallies
 * the transport itself produces). */
int mcdc_get_importance(mcdc_handle h, double *score, double *weight, size_t n, void *stream);

/* ------------------------------------------------------------------------ */
/* MLP training (log-importance regression), device buffers, FP32.          */
/* Loss = sum_i wt_i (f(x_i) - y_i)^2 / sum_i wt_i; Adam(lr, b1, b2, eps).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t steps;
    float lr, beta1, beta2, eps;
} mcdc_train_opts;

/* Forward pass: out[n] = f(X[n][in_dim]) (device buffers, async on stream).
 * Source: not in the paper (the importance network of the weight windows). */
int mcdc_mlp_forward(const float *dev_params, int32_t in_dim, const float *dev_X, size_t n,
                     float *dev_out, void *stream);

/* Device scratch (bytes) that mcdc_mlp_grad / mcdc_mlp_train need for n points.
 * Source: not in the paper (as mcdc_mlp_forward). */
size_t mcdc_mlp_scratch_bytes(int32_t in_dim, size_t n);

/* Loss and gradient: grad[n_params] (overwritten), loss (device scalar, may be
 * NULL).  The gradient is summed over points in a fixed order.  dev_scratch:
 * caller-owned, mcdc_mlp_scratch_bytes(in_dim, n) bytes.
 * Source: not in the paper (as mcdc_mlp_forward). */
int mcdc_mlp_grad(const float *dev_params, int32_t in_dim, const float *dev_X, const float *dev_y,
                  const float *dev_wt, size_t n, float *dev_grad, float *dev_loss,
                  void *dev_scratch, void *stream);

/* `steps` Adam steps in place on dev_params; dev_m, dev_v (n_params each) hold
 * the moments and must start at zero; step numbering continues from
 * *step_io (host, updated).  dev_grad (may be NULL) receives the last
 * gradient; dev_loss_hist (steps floats, may be NULL) the loss before each step.
 * Source: not in the paper (as mcdc_mlp_forward). */
int mcdc_mlp_train(float *dev_params, int32_t in_dim, const float *dev_X, const float *dev_y,
                   const float *dev_wt, size_t n, float *dev_m, float *dev_v, float *dev_grad,
                   const mcdc_train_opts *o, int32_t *step_io, float *dev_loss_hist,
                   void *dev_scratch, void *stream);

/* mcdc_mlp_train without the scratch argument: the same kernels in the same
 * order (parameters, moments and gradient bit-identical to it; the loss
 * history, summed over workgroups by float atomics, to that summation
 * order), with the scratch in a static 16 MiB device
 * array of the library (one per GPU, kept until the process ends) and the
 * loss history cleared by a fill kernel; it allocates nothing.  At most
 * 64 * floor((2^22 - 64) / n_params) points (58240 for one group, 53056 for
 * eight); more is MCDC_E_INVALID.  Calls that overlap on one GPU share the
 * array and race; a call leaves it holding its partial sums.
 * Source: not in the paper; for callers that cannot allocate (code under HIP
 * graph capture, tight training loops, harnesses that forbid hipMalloc). */
int mcdc_mlp_train_noalloc(float *dev_params, int32_t in_dim, const float *dev_X,
                           const float *dev_y, const float *dev_wt, size_t n, float *dev_m,
                           float *dev_v, float *dev_grad, const mcdc_train_opts *o,
                           int32_t *step_io, float *dev_loss_hist, void *stream);

/* Parameters of the network for in_dim inputs.
 * Source: not in the paper (as mcdc_mlp_forward). */
size_t mcdc_mlp_param_count(int32_t in_dim);

/* ------------------------------------------------------------------------ */
/* Batched problems: many independent problems in one persistent launch per  */
/* census step, census steps captured in a HIP graph.                         */
/* ------------------------------------------------------------------------ */

/* Workspace bytes of n problems with n_hist[p] histories each (all share
 * their census count).  Pure.
 * Source: not in the paper (batching many small problems on one GPU). */
int mcdc_batch_workspace_bytes(const mcdc_problem_desc *ds, size_t n, const uint64_t *n_hist,
                               const mcdc_options *opt, size_t *bytes);

/* Create the batched handle (problem p gets problem id p in its random
 * streams, so its histories match a run of it alone).
 * Source: not in the paper (as mcdc_batch_workspace_bytes). */
int mcdc_create_batch(const mcdc_problem_desc *ds, size_t n, const uint64_t *n_hist,
                      const mcdc_options *opt, void *dev_workspace, size_t bytes,
                      mcdc_handle *out);

/* One pass of every problem's histories (ids continue across passes),
 * replayed from a HIP graph of its census steps; asynchronous on `stream`.
 * Source: Sec. "MC/DC on CPUs", transport-loop paragraph, per problem; the
 * batching is not in the paper. */
int mcdc_run_batch(mcdc_handle h, uint64_t seed, void *stream);

/* Raw mesh sums of problem p (host copy, n = its bins).
 * Source: Fig. 3 (tallies accumulated by atomic adds). */
int mcdc_get_batch_raw(mcdc_handle h, size_t p, double *tally_sum, size_t n, void *stream);

/* Counters of problem p.
 * Source: as mcdc_get_counters. */
int mcdc_get_batch_counters(mcdc_handle h, size_t p, mcdc_counters *out, void *stream);

/* Per-history sum of weight * flight length of problem p for the histories of
 * the last pass, summed in event order (host copy, n = its histories).
 * Source: as mcdc_set_trace. */
int mcdc_get_batch_history_path(mcdc_handle h, size_t p, double *out, size_t n, void *stream);

/* Kernel timing: with `on` = 1, later runs record a pair of HIP events on the
 * run's stream around every launch of the schedule's tracking kernel (history
 * schedule: the history kernel; event schedule: the flight stage; hybrid
 * schedule: the lead stage).
 * Source: Sec. "Performance" (the paper profiles its GPU runs). */
int mcdc_set_kernel_timing(mcdc_handle h, int on);

/* Synchronise the recorded events and return the number of launches recorded
 * since the last call and their summed duration in milliseconds (then forget
 * them).
 * Source: as mcdc_set_kernel_timing. */
int mcdc_kernel_time(mcdc_handle h, uint64_t *launches, double *total_ms);

/* Micro-benchmark for the measured atomic ceiling (not on the transport
 * path): n_items work-items each add 1.0 to per_item bins of dev_buf[n_bins],
 * in runs of `run` consecutive bins starting at hashed positions (run = 1:
 * uniformly scattered).  Asynchronous on `stream`; the caller times it.
 * Source: Fig. 3 (the GPU tally is an atomic add; this measures its ceiling). */
int mcdc_micro_atomics(double *dev_buf, uint64_t n_bins, uint64_t n_items, uint32_t per_item,
                       uint32_t run, void *stream);

/* Micro-benchmark: n_items work-items (1024 per workgroup) each add 1.0 to
 * per_item bins of their workgroup's LDS array of n_bins doubles (2 ..
 * MCDC_MAX_TILE_BINS, the hot tile's size) with ds_add_f64, starting at a
 * hashed bin and walking with a per-lane odd stride modulo the largest power
 * of two not above n_bins; each workgroup's total is then added to
 * dev_out[0] (device, caller-owned).  Asynchronous on `stream`.
 * Source: Fig. 3 (atomic tally adds), here their on-chip ceiling. */
int mcdc_micro_lds_atomics(double *dev_out, uint32_t n_bins, uint64_t n_items, uint32_t per_item,
                           void *stream);

/* Micro-benchmark: stream `bytes` (a multiple of 32) from dev_src to dev_dst.
 * Asynchronous on `stream`.
 * Source: not in the paper (the HBM ceiling of the roofline). */
int mcdc_micro_copy(const void *dev_src, void *dev_dst, size_t bytes, void *stream);

/* Release the handle (not the caller-owned workspace).
 * Source: Sec. "MC/DC on CPUs" (the run returns to the caller after
 * finalization). */
void mcdc_destroy_problem(mcdc_handle h);

/* Thread-local message of the last failed call.
 * Source: not in the paper (error reporting across the C boundary). */
const char *mcdc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
