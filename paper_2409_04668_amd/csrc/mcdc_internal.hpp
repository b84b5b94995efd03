// Internal declarations shared by the HIP translation units of libmcdc.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mcdc.h"

namespace mcdc {

constexpr int kMaxBoxes = MCDC_MAX_BOXES;
constexpr int kMaxG = MCDC_MAX_G;
constexpr int kH = MCDC_MLP_HIDDEN;
constexpr int kImpList = 16;                 // distinct coarse cells kept per history
constexpr int kLdsTallyMaxBins = 7680;       // 60 KiB of FP64 LDS tile

// counters (device accumulator layout)
enum {
    C_HIST = 0, C_FLIGHT, C_PIECE, C_COLLISION, C_ABSORB, C_SURFACE, C_LEAK, C_CENSUS,
    C_TIME_END, C_SPLIT, C_RR_KILL, C_RR_SURVIVE, C_CUT_KILL, C_CUT_SURVIVE, C_DET_HIT,
    C_PARTICLE, C_PC_KILL, C_PC_COPY, C_SURF, C_WW_PLANE, N_CNT
};
enum { W_SOURCE = 0, W_LEAK, W_ABSORB, W_TIME_END, W_GAIN, W_LOSS, W_PATH, N_WSUM };

// trace record types
enum {
    EV_SOURCE = 0, EV_SCATTER = 1, EV_ABSORB = 2, EV_SURFACE = 3, EV_LEAK = 4, EV_CENSUS = 5,
    EV_TIME_END = 6, EV_SPLIT = 7, EV_RR_KILL = 8, EV_RR_SURVIVE = 9, EV_CUT_KILL = 10,
    EV_CUT_SURVIVE = 11, EV_PC_KILL = 12, EV_PC_KEEP = 13, EV_WW_PLANE = 14, EV_FISSION = 15,
};

struct DevAcc {
    unsigned long long cnt[N_CNT];
    double wsum[N_WSUM];
    double leak[6];
    double det[2];
    int status;
    int pad;
    double kcol;                         // k-eigenvalue: sum of w nuSigma_f / Sigma_t
                                         // over the generation's collisions
};

// Problem tables as seen by the kernels: every kernel takes them by value as
// its first argument (< 2 KiB) and reads them where the kernel-argument
// segment holds them.
struct DevProblem {
    double outer_lo[3], outer_hi[3];
    double box_lo[kMaxBoxes][3], box_hi[kMaxBoxes][3];
    int32_t box_mat[kMaxBoxes];
    int32_t bc[6];
    int32_t n_boxes, background_mat, n_mat, G;
    const double *sigma_t, *sigma_s, *speed, *census;   // device
    int32_t src_box, src_isotropic, src_group, n_census;
    double src_lo[3], src_hi[3], src_t0, src_t1, src_dir[3];
    double mesh_lo[4], mesh_delta[4], mesh_idelta[4];
    int32_t mesh_n[4], mesh_bounded[3], G_t;
    int32_t col_on;                      // collision-estimator tally
    int32_t surf_on, surf_axis;          // surface-current tally on x[axis] = pos
    double surf_pos;
    double surf_lo[2], surf_id[2];       // mesh lo and 1/delta of the in-plane axes b1 < b2
    int32_t surf_n[2], surf_bd[2];       // their bins and boundedness
    uint32_t surf_nbins;                 // 2 * G_t * nt * n_b1 * n_b2
    int32_t pc_on;                       // population control at intermediate census
    double pc_target;                    // census population per source history
    int32_t implicit_capture;
    double w_cut, w_surv;
    int32_t has_detector;
    double det_lo[3], det_hi[3];
    int32_t imp_on;
    int32_t imp_n[4];
    double imp_lo[4], imp_f[4];
    int32_t ww_on, ww_nmax;
    const float *ww_params;                               // device
    float ww_ymin, ww_ymax;                               // output clamp
    double ww_logk, ww_ratio, ww_lo[4], ww_inv[4];
    const double *ww_map;                // device w_T per map cell, or null (network per check)
    int32_t ww_map_n[4];
    int32_t ww_grid_on, ww_grid_n[3];    // window checks also on the interior planes of a
    double ww_grid_d[3], ww_grid_id[3];  // regular grid over the outer box (delta, 1/delta)
    int64_t max_events;
    int32_t stack_cap;
    uint32_t problem_id;
    uint32_t nbins;
    int32_t fis_on;                      // fission data present (k-eigenvalue mode)
    const double *nu_sigma_f, *chi;      // device [n_mat][G] each
    uint32_t hot_lo[5], hot_n[5];        // LDS hot tile (x, y, z, t, g); hot_bins 0 = off
    uint32_t hot_bins;
};

// Per-launch arguments of the tracking kernels.
struct RunArgs {
    uint64_t seed;
    uint64_t h_begin, h_end, h_run0;
    uint64_t run_n;                      // histories of the whole run (event schedule)
    uint64_t run_batches;                // batches of the run (event schedule)
    double pc_m;                         // population-control target size of this chunk
    double *tally;                       // current-batch accumulator [nbins]; event
                                         // schedule: [run_batches][nbins] slices
    double *col;                         // collision estimator, same layout as tally
    double *surf;                        // surface current; event schedule: per batch
    DevAcc *acc;
    double *imp_score, *imp_weight;
    double *xh_out;
    int32_t keep_path;                   // accumulate per-history path (an output only)
    int32_t pad_keep;
    mcdc_trace_rec *trace;
    uint64_t trace_cap;
    unsigned long long *trace_count;
    double *stk_d;                       // [8][stack_cap][n_lanes]
    int32_t *stk_i;                      // [4][stack_cap][n_lanes]
    int32_t *imp_cell;                   // [kImpList][n_lanes]
    double *imp_cnt, *imp_xsum;          // [kImpList][n_lanes]
    uint64_t n_lanes;
    const int *cancel;                   // host-coherent cancel word (may be null)
    // k-eigenvalue generation (history schedule): histories [gen_first,
    // gen_first + gen_m) start at the sites src_* (null: the problem's
    // source); fission sites go to site_* in any order with their key
    // (history slot, ordinal within the history) and hist_sites counts them
    // per slot; the collision estimate accumulates in acc->kcol
    const double *k_norm;                // site production is divided by *k_norm
    uint64_t gen_first, gen_m;
    const double *src_d;                 // [3][gen_m] positions
    const int32_t *src_g;                // [gen_m] groups
    double *site_d;                      // [3][site_cap]
    int32_t *site_g;                     // [site_cap]
    uint32_t *site_key;                  // [2][site_cap]: slot, ordinal
    uint32_t *site_n;                    // sites reserved (may pass site_cap: overflow)
    uint32_t *hist_sites;                // [gen_m]
    uint32_t site_cap;
    int32_t det_off;                     // 1: detector scores not accumulated (inactive
                                         // generation)
};

struct Layout {                          // workspace carving (byte offsets)
    size_t tables, tally_batch, tally_sum, tally_sumsq, col_batch, col_sum, col_sumsq,
        surf_batch, surf_sum, surf_sumsq, acc,
        imp_score, imp_weight, ww_params,
        stk_d, stk_i, imp_list, event, total;
};

// launch helpers implemented in the kernel translation units
hipError_t launch_history(const DevProblem &P, const RunArgs &A, int grid, int block,
                          bool lds_tally, hipStream_t s);
hipError_t launch_closeout(double *batch, double *sum, double *sumsq, uint32_t n, double nb,
                           hipStream_t s);
hipError_t launch_problem_check(const DevProblem &P, int *out, hipStream_t s);
hipError_t launch_closeout_run(double *batch, double *sum, double *sumsq, uint32_t n, uint32_t B,
                               uint64_t n_hist, hipStream_t s);
int history_grid(int block, int waves_per_cu);

}  // namespace mcdc
