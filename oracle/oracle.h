/*
 * CPU oracle for the fixed-source, time-dependent Monte Carlo transport loop
 * (scatter + absorb), and for the k-eigenvalue mode (fission source iterated
 * over generations).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the GPU path.
 *
 * The oracle is single threaded, processes histories in id order, and adds
 * every tally contribution with a plain `+=` in event order (the CPU variant of
 * the tally add in Fig. 3 of the paper).  Its per-history trajectories are the
 * definition the GPU kernels must reproduce bit for bit; its tallies are unique
 * up to summation order.
 */
#ifndef MCDC_ORACLE_H
#define MCDC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_E_INVALID = -1,
    ORC_E_EVENT_CAP = -4,
    ORC_E_STACK = -7,
    ORC_E_EXTINCT = -9,           /* k-eigenvalue: a generation produced no site */
};

/* trace record types */
enum {
    ORC_EV_SOURCE = 0,
    ORC_EV_SCATTER = 1,
    ORC_EV_ABSORB = 2,
    ORC_EV_SURFACE = 3,
    ORC_EV_LEAK = 4,
    ORC_EV_CENSUS = 5,
    ORC_EV_TIME_END = 6,
    ORC_EV_SPLIT = 7,
    ORC_EV_ROULETTE_KILL = 8,
    ORC_EV_ROULETTE_SURVIVE = 9,
    ORC_EV_CUTOFF_KILL = 10,
    ORC_EV_CUTOFF_SURVIVE = 11,
    ORC_EV_PC_KILL = 12,          /* population control at a census: removed        */
    ORC_EV_PC_KEEP = 13,          /* population control: kept as aux copies        */
    ORC_EV_WW_PLANE = 14,         /* a flight reached a weight-window grid plane   */
    ORC_EV_FISSION = 15,          /* fission sites produced at a collision (aux = n) */
};

/* counters */
enum {
    ORC_C_HIST = 0, ORC_C_FLIGHT, ORC_C_PIECE, ORC_C_COLLISION, ORC_C_ABSORB,
    ORC_C_SURFACE, ORC_C_LEAK, ORC_C_CENSUS, ORC_C_TIME_END, ORC_C_SPLIT,
    ORC_C_RR_KILL, ORC_C_RR_SURVIVE, ORC_C_CUT_KILL, ORC_C_CUT_SURVIVE,
    ORC_C_DET_HIT, ORC_C_PARTICLE, ORC_C_PC_KILL, ORC_C_PC_COPY, ORC_C_SURF_CROSS, ORC_C_WW_PLANE, ORC_NCOUNT
};
/* weight sums */
enum {
    ORC_W_SOURCE = 0, ORC_W_LEAK, ORC_W_ABSORB, ORC_W_TIME_END, ORC_W_GAIN,
    ORC_W_LOSS, ORC_W_PATH, ORC_NWSUM
};

typedef struct {
    double outer_lo[3], outer_hi[3];
    int32_t bc[6];                    /* -x,+x,-y,+y,-z,+z: 0 vacuum, 1 reflective */
    int32_t n_boxes;
    const double *box_lo, *box_hi;    /* [n_boxes][3] */
    const int32_t *box_mat;
    int32_t background_mat;
    int32_t n_mat, G;
    const double *sigma_t;            /* [n_mat][G] */
    const double *sigma_s;            /* [n_mat][G][G] from-group rows */
    const double *speed;              /* [G] */
    int32_t src_box;                  /* 0 point, 1 box */
    double src_lo[3], src_hi[3], src_t0, src_t1;
    int32_t src_isotropic;
    double src_dir[3];
    int32_t src_group;
    double mesh_lo[4], mesh_hi[4];
    int32_t mesh_n[4];
    int32_t mesh_per_group;
    int32_t n_census;
    const double *census;
    int32_t implicit_capture;
    double w_cut, w_surv;
    int32_t has_detector;
    double det_lo[3], det_hi[3];
    int32_t imp_on;
    int32_t imp_n[4];
    int32_t ww_on, ww_hidden, ww_nmax;
    const float *ww_params;
    float ww_ymin, ww_ymax;           /* network output clamped to [ymin, ymax] */
    double ww_logk, ww_ratio;
    int32_t ww_map_n[4];              /* all > 0: targets from a cell-centre map of the
                                         network, (nx, ny, nz, nt) cells; 0: network
                                         evaluated at every check */
    int32_t ww_grid_n[3];             /* all > 0: the windows are also checked where a
                                         flight reaches an interior plane of an
                                         (nx, ny, nz) grid over the outer box; 0: off */
    int32_t col_tally;                /* also a collision-estimator mesh tally */
    int32_t surf_on;                  /* also a surface-current tally on the plane
                                         x[surf_axis] = surf_pos                 */
    int32_t surf_axis;
    double surf_pos;
    int32_t pc_on;                    /* population control at every intermediate
                                         census: a batch's histories advance census
                                         step by census step together */
    double pc_target;                 /* census population per source history   */
    int32_t n_batches;
    int64_t max_events;
    int32_t stack_cap;
    uint32_t problem_id;
    const double *nu_sigma_f;         /* [n_mat][G] nu * Sigma_f, or NULL (no fission) */
    const double *chi;                /* [n_mat][G] fission spectrum (outgoing group)   */
} orc_problem;

typedef struct {
    uint64_t hist;
    uint32_t tag, seq;
    int32_t type, g, cell;
    uint32_t k;
    double x, y, z, t, ux, uy, uz, w, aux;
} orc_trace_rec;

typedef struct {
    double *tally_batch;      /* [nbins] current batch (scratch, zero on entry) */
    double *tally_sum;        /* [nbins] sum over batches of S_b              */
    double *tally_sumsq;      /* [nbins] sum over batches of S_b^2 / N_b      */
    double *col_batch, *col_sum, *col_sumsq;  /* collision estimator, same layout */
    double *surf_batch, *surf_sum, *surf_sumsq;  /* surface current, [2][G_t][nt][n_b2][n_b1] */
    double det[2];            /* sum x_h, sum x_h^2 over histories            */
    double leak[6];
    double wsum[ORC_NWSUM];
    uint64_t cnt[ORC_NCOUNT];
    double *imp_score;        /* [coarse cells] or NULL */
    double *imp_weight;
    double *hist_xh;          /* [n_hist][2] per-history (detector score, sum of w*d) or NULL */
    orc_trace_rec *trace;     /* or NULL */
    int64_t trace_cap, trace_n;
    int64_t batches_done;
    uint64_t hist_done;
} orc_result;

int orc_run(const orc_problem *P, uint64_t seed, uint64_t hist0, uint64_t n_hist,
            orc_result *R);

/* k-eigenvalue mode: power iteration on the fission source, n_inactive +
 * n_active generations of M histories (history id g * M + j for slot j of
 * generation g).  Per generation g: k_col[g] = sum over collisions of
 * w nuSigma_f / Sigma_t, divided by M; n_sites[g] = fission sites produced;
 * k_site[g] = k_norm * n_sites / M, where k_norm (k0 for the first
 * generation, then the previous k_site) divides the site production.  Only
 * the active generations score tallies, each one batch of M histories.
 * src_out (may be NULL): [M][4] (x, y, z, group) of the last combed source. */
typedef struct {
    uint64_t M;
    int32_t n_inactive, n_active;
    double k0;
    double *k_col, *k_site;   /* [n_inactive + n_active] */
    uint64_t *n_sites;        /* [n_inactive + n_active] */
    double *src_out;
} orc_keff;
int orc_run_keff(const orc_problem *P, uint64_t seed, orc_keff *K, orc_result *R);

/* primitives exposed for the pin tests */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint64_t seed, uint64_t hist, uint32_t problem, uint32_t tag, uint32_t k);
double orc_log(double x);
double orc_exp(double x);
/* n isotropic directions from one stream; returns the draws consumed */
uint32_t orc_directions(uint64_t seed, uint64_t hist, uint32_t n, double *u);
/* FP32 MLP forward as used by the weight-window check */
float orc_mlp_f32(const float *params, int32_t in_dim, int32_t hidden, const float *in);
/* weight-window map: w_T at the centre of every map cell, layout
 * [g][it][iz][iy][ix]; returns the number of cells, or -1 when the problem has
 * no map */
int64_t orc_ww_map(const orc_problem *P, double *out);
/* map cell of a point (x, y, z, t, g) under the same rules as the check */
int64_t orc_ww_map_cell(const orc_problem *P, const double p[3], double t, int32_t g);
/* track-length scoring of one straight segment into a mesh (same rules as the
 * transport loop); returns the number of scored pieces */
int64_t orc_score_segment(const orc_problem *P, const double p[3], const double u[3],
                          double t0, double d, double w, int32_t g, double *tally);

#ifdef __cplusplus
}
#endif
#endif
