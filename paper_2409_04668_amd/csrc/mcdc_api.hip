// Host runtime behind the C ABI: validation, workspace carving, table upload,
// batch loop and result read-back.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "mcdc_internal.hpp"
#include "mcdc_runtime.hpp"

namespace mcdc {

thread_local std::string g_err;

int fail(int st, const std::string &msg) {
    g_err = msg;
    return st;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(MCDC_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int cancel_init(mcdc_problem *h) {
    void *p = nullptr;
    hipError_t e = hipHostMalloc(&p, sizeof(int), hipHostMallocCoherent);
    if (e != hipSuccess) return hip_fail(e, "cancel word");
    h->cancel_host = (int *)p;
    __atomic_store_n(h->cancel_host, 0, __ATOMIC_RELEASE);
    void *d = nullptr;
    e = hipHostGetDevicePointer(&d, p, 0);
    if (e != hipSuccess) {
        cancel_free(h);
        return hip_fail(e, "cancel word device address");
    }
    h->cancel_dev = (int *)d;
    return MCDC_OK;
}

void cancel_free(mcdc_problem *h) {
    if (h->cancel_host) (void)hipHostFree(h->cancel_host);
    h->cancel_host = nullptr;
    h->cancel_dev = nullptr;
}

int validate_desc(const mcdc_problem_desc *d) {
    if (!d) return fail(MCDC_E_INVALID, "null problem description");
    if (d->G < 1 || d->G > MCDC_MAX_G) return fail(MCDC_E_INVALID, "G out of range");
    if (d->n_mat < 1 || d->n_mat > MCDC_MAX_MAT) return fail(MCDC_E_INVALID, "n_mat out of range");
    if (d->n_boxes < 0 || d->n_boxes > MCDC_MAX_BOXES) return fail(MCDC_E_INVALID, "n_boxes out of range");
    if (d->n_boxes > 0 && (!d->box_lo || !d->box_hi || !d->box_mat))
        return fail(MCDC_E_INVALID, "box arrays missing");
    for (int b = 0; b < d->n_boxes; ++b)
        if (d->box_mat[b] < 0 || d->box_mat[b] >= d->n_mat) return fail(MCDC_E_INVALID, "box material out of range");
    if (d->background_mat < 0 || d->background_mat >= d->n_mat)
        return fail(MCDC_E_INVALID, "background material out of range");
    if (!d->sigma_t || !d->sigma_s || !d->speed || !d->census) return fail(MCDC_E_INVALID, "table missing");
    for (int i = 0; i < d->n_mat * d->G; ++i)
        if (!(d->sigma_t[i] >= 0.0)) return fail(MCDC_E_INVALID, "negative sigma_t");
    for (int g = 0; g < d->G; ++g)
        if (!(d->speed[g] > 0.0)) return fail(MCDC_E_INVALID, "speed must be positive");
    if (d->src_group < 0 || d->src_group >= d->G) return fail(MCDC_E_INVALID, "source group out of range");
    if (d->n_census < 1 || d->n_census > MCDC_MAX_CENSUS) return fail(MCDC_E_INVALID, "n_census out of range");
    for (int i = 1; i < d->n_census; ++i)
        if (!(d->census[i] > d->census[i - 1])) return fail(MCDC_E_INVALID, "census times must increase");
    for (int a = 0; a < 4; ++a)
        if (d->mesh_n[a] < 1) return fail(MCDC_E_INVALID, "mesh_n must be >= 1");
    for (int a = 0; a < 3; ++a) {
        const bool unb = isinf(d->mesh_lo[a]) && isinf(d->mesh_hi[a]);
        if (unb && d->mesh_n[a] != 1) return fail(MCDC_E_INVALID, "unbounded mesh axis must have n=1");
        if (!unb && !(d->mesh_hi[a] > d->mesh_lo[a])) return fail(MCDC_E_INVALID, "mesh bounds");
    }
    if (!(d->mesh_hi[3] > d->mesh_lo[3])) return fail(MCDC_E_INVALID, "mesh time bounds");
    const double nb = (double)(d->mesh_per_group ? d->G : 1) * d->mesh_n[0] * d->mesh_n[1] *
                      d->mesh_n[2] * d->mesh_n[3];
    if (nb > 4.0e9) return fail(MCDC_E_INVALID, "tally too large (bins must fit 32 bits)");
    if (d->n_batches < 1 || d->n_batches > 65535) return fail(MCDC_E_INVALID, "n_batches must lie in [1, 65535]");
    if (d->stack_cap < 0 || d->max_events < 1) return fail(MCDC_E_INVALID, "stack_cap/max_events");
    if (d->col_tally != 0 && d->col_tally != 1) return fail(MCDC_E_INVALID, "col_tally must be 0 or 1");
    if (d->surf_on != 0 && d->surf_on != 1) return fail(MCDC_E_INVALID, "surf_on must be 0 or 1");
    if (d->surf_on && (d->surf_axis < 0 || d->surf_axis > 2 || !isfinite(d->surf_pos)))
        return fail(MCDC_E_INVALID, "surf_axis must be 0..2 and surf_pos finite");
    if (d->pc_on != 0 && d->pc_on != 1) return fail(MCDC_E_INVALID, "pc_on must be 0 or 1");
    if (d->pc_on && !(d->pc_target > 0.0 && d->pc_target <= 64.0))
        return fail(MCDC_E_INVALID, "pc_target must lie in (0, 64]");
    if (d->pc_on && d->imp_on) return fail(MCDC_E_INVALID, "population control excludes the importance estimate");
    if (d->imp_on) {
        for (int a = 0; a < 4; ++a)
            if (d->imp_n[a] < 1) return fail(MCDC_E_INVALID, "imp_n must be >= 1");
        if (d->implicit_capture) return fail(MCDC_E_INVALID, "importance estimate needs analog collisions");
    }
    if (d->imp_on || d->stack_cap > 0)
        for (int a = 0; a < 3; ++a)
            if (isinf(d->outer_lo[a]) || isinf(d->outer_hi[a]))
                return fail(MCDC_E_INVALID, "weight windows / importance need a finite outer box");
    if (d->nu_sigma_f) {
        if (!d->chi) return fail(MCDC_E_INVALID, "fission data needs the fission spectrum chi");
        for (int m = 0; m < d->n_mat; ++m) {
            double sf = 0.0, sc = 0.0;
            for (int g = 0; g < d->G; ++g) {
                const double f = d->nu_sigma_f[m * d->G + g], c = d->chi[m * d->G + g];
                if (!(f >= 0.0) || !isfinite(f) || !(c >= 0.0) || !isfinite(c))
                    return fail(MCDC_E_INVALID, "nu_sigma_f and chi must be finite and >= 0");
                sf += f;
                sc += c;
            }
            if (sf > 0.0 && !(sc > 0.0))
                return fail(MCDC_E_INVALID, "a fissile material needs a spectrum with a positive sum");
        }
    }
    return MCDC_OK;
}

// any positive nu Sigma_f: the problem runs in the k-eigenvalue mode
int desc_fissile(const mcdc_problem_desc *d) {
    if (!d->nu_sigma_f) return 0;
    for (int i = 0; i < d->n_mat * d->G; ++i)
        if (d->nu_sigma_f[i] > 0.0) return 1;
    return 0;
}

// surface-current bins: 2 sides x groups of the mesh x time bins x the mesh
// bins of the two in-plane axes
size_t desc_nsurf(const mcdc_problem_desc *d) {
    if (!d->surf_on) return 0;
    const int a = d->surf_axis, b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    return (size_t)2 * (d->mesh_per_group ? d->G : 1) * d->mesh_n[3] * d->mesh_n[b1] * d->mesh_n[b2];
}

uint32_t desc_nbins(const mcdc_problem_desc *d) {
    return (uint32_t)((d->mesh_per_group ? d->G : 1) * d->mesh_n[0] * d->mesh_n[1] * d->mesh_n[2] *
                      d->mesh_n[3]);
}

size_t desc_nimp(const mcdc_problem_desc *d) {
    return d->imp_on ? (size_t)d->G * d->imp_n[0] * d->imp_n[1] * d->imp_n[2] * d->imp_n[3] : 0;
}

Options resolve_options(const mcdc_options *o) {
    Options r;
    r.schedule = MCDC_SCHED_HISTORY;
    r.block = 256;
    r.waves_per_cu = 16;
    r.lds_tally = 1;
    r.event_chunk = 1 << 22;
    r.tile_bins = 0;
    r.lead = false;
    for (int a = 0; a < 5; ++a) r.tile_lo[a] = r.tile_n[a] = 0;
    if (o) {
        if (o->schedule) r.schedule = o->schedule;
        if (o->block) r.block = o->block;
        if (o->waves_per_cu) r.waves_per_cu = o->waves_per_cu;
        r.lds_tally = o->lds_tally;
        if (o->event_chunk) r.event_chunk = o->event_chunk;
        bool on = o->lds_tally != 0;
        uint64_t bins = 1;
        for (int a = 0; a < 5; ++a) {
            r.tile_lo[a] = o->tile_lo[a];
            r.tile_n[a] = o->tile_n[a];
            on = on && o->tile_n[a] > 0;
            bins *= (uint64_t)(o->tile_n[a] > 0 ? o->tile_n[a] : 0);
        }
        if (on) r.tile_bins = bins > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bins;
    }
    if (r.schedule == MCDC_SCHED_AUTO) r.schedule = MCDC_SCHED_HISTORY;
    // the hybrid schedule is the event schedule with a lead stage
    r.lead = r.schedule == MCDC_SCHED_HYBRID;
    if (r.lead) r.schedule = MCDC_SCHED_EVENT;
    // the hot tile runs one 1024-work-item workgroup per CU-share of LDS (the
    // history schedule, the lead and re-lead stages of the hybrid schedule,
    // the event schedule's flight stage)
    if (r.tile_bins) r.block = 1024;
    r.grid = history_grid(r.block, r.waves_per_cu);
    r.n_lanes = (uint64_t)r.grid * r.block;
    return r;
}

int check_options(const Options &o) {
    if (o.tile_bins) {
        if (o.tile_bins > MCDC_MAX_TILE_BINS) return fail(MCDC_E_INVALID, "hot tile larger than MCDC_MAX_TILE_BINS");
    } else if (o.block < 64 || o.block > 256 || o.block % 64) {
        return fail(MCDC_E_INVALID, "block must be 64..256, a multiple of 64");
    }
    if (o.waves_per_cu < 1 || o.waves_per_cu > 64) return fail(MCDC_E_INVALID, "waves_per_cu out of range");
    if (o.schedule != MCDC_SCHED_HISTORY && o.schedule != MCDC_SCHED_EVENT)
        return fail(MCDC_E_INVALID, "unknown schedule");
    return MCDC_OK;
}

Layout make_layout(const mcdc_problem_desc *d, const Options &o) {
    Layout L;
    size_t off = 0;
    const size_t n_tab = (size_t)d->n_mat * d->G + (size_t)d->n_mat * d->G * d->G + d->G + d->n_census +
                         (desc_fissile(d) ? 2 * (size_t)d->n_mat * d->G : 0);
    L.tables = off; off = align_up(off + n_tab * sizeof(double));
    const size_t nb = desc_nbins(d);
    // the event schedule keeps every batch of a run resident (one slice per
    // batch) so a run drains its particle bank once, not once per batch
    const size_t nslices = o.schedule == MCDC_SCHED_EVENT ? (size_t)d->n_batches : 1;
    L.tally_batch = off; off = align_up(off + nslices * nb * sizeof(double));
    L.tally_sum = off; off = align_up(off + nb * sizeof(double));
    L.tally_sumsq = off; off = align_up(off + nb * sizeof(double));
    const size_t nc = d->col_tally ? nb : 0;      // collision estimator, same layout
    L.col_batch = off; off = align_up(off + nslices * nc * sizeof(double));
    L.col_sum = off; off = align_up(off + nc * sizeof(double));
    L.col_sumsq = off; off = align_up(off + nc * sizeof(double));
    const size_t nsf = desc_nsurf(d);                // surface current, per batch slice
    L.surf_batch = off; off = align_up(off + nslices * nsf * sizeof(double));
    L.surf_sum = off; off = align_up(off + nsf * sizeof(double));
    L.surf_sumsq = off; off = align_up(off + nsf * sizeof(double));
    L.acc = off; off = align_up(off + sizeof(DevAcc));
    const size_t ni = desc_nimp(d);
    L.imp_score = off; off = align_up(off + ni * sizeof(double));
    L.imp_weight = off; off = align_up(off + ni * sizeof(double));
    L.ww_params = off; off = align_up(off + mcdc_mlp_param_count(4 + d->G) * sizeof(float));
    const size_t cap = (size_t)d->stack_cap;
    L.stk_d = off; off = align_up(off + 8 * cap * o.n_lanes * sizeof(double));
    L.stk_i = off; off = align_up(off + 4 * cap * o.n_lanes * sizeof(int32_t));
    L.imp_list = off;
    if (d->imp_on) off = align_up(off + (size_t)kImpList * o.n_lanes * (sizeof(int32_t) + 2 * sizeof(double)));
    L.event = off;
    off += event_workspace_bytes(d, o);
    L.total = align_up(off);
    return L;
}

void build_dev_problem(const mcdc_problem_desc *d, char *ws, const Layout &L, DevProblem &P) {
    memset(&P, 0, sizeof(P));
    for (int a = 0; a < 3; ++a) {
        P.outer_lo[a] = d->outer_lo[a];
        P.outer_hi[a] = d->outer_hi[a];
    }
    for (int f = 0; f < 6; ++f) P.bc[f] = d->bc[f];
    P.n_boxes = d->n_boxes;
    for (int b = 0; b < d->n_boxes; ++b) {
        for (int a = 0; a < 3; ++a) {
            P.box_lo[b][a] = d->box_lo[3 * b + a];
            P.box_hi[b][a] = d->box_hi[3 * b + a];
        }
        P.box_mat[b] = d->box_mat[b];
    }
    P.background_mat = d->background_mat;
    P.n_mat = d->n_mat;
    P.G = d->G;
    double *tab = (double *)(ws + L.tables);
    const size_t nst = (size_t)d->n_mat * d->G, nss = nst * d->G;
    P.sigma_t = tab;
    P.sigma_s = tab + nst;
    P.speed = tab + nst + nss;
    P.census = tab + nst + nss + d->G;
    P.fis_on = desc_fissile(d);
    if (P.fis_on) {
        P.nu_sigma_f = P.census + d->n_census;
        P.chi = P.nu_sigma_f + nst;
    }
    P.src_box = d->src_kind == MCDC_SRC_BOX;
    P.src_isotropic = d->src_isotropic;
    P.src_group = d->src_group;
    P.n_census = d->n_census;
    for (int a = 0; a < 3; ++a) {
        P.src_lo[a] = d->src_lo[a];
        P.src_hi[a] = d->src_hi[a];
        P.src_dir[a] = d->src_dir[a];
    }
    P.src_t0 = d->src_t0;
    P.src_t1 = d->src_t1;
    for (int a = 0; a < 4; ++a) {
        P.mesh_n[a] = d->mesh_n[a];
        P.mesh_lo[a] = d->mesh_lo[a];
        if (a < 3 && isinf(d->mesh_lo[a]) && isinf(d->mesh_hi[a])) {
            P.mesh_bounded[a] = 0;
            P.mesh_delta[a] = HUGE_VAL;
            P.mesh_idelta[a] = 0.0;
        } else {
            if (a < 3) P.mesh_bounded[a] = 1;
            P.mesh_delta[a] = (d->mesh_hi[a] - d->mesh_lo[a]) / (double)d->mesh_n[a];
            P.mesh_idelta[a] = 1.0 / P.mesh_delta[a];
        }
    }
    P.G_t = d->mesh_per_group ? d->G : 1;
    P.col_on = d->col_tally;
    P.surf_on = d->surf_on;
    if (d->surf_on) {
        const int a = d->surf_axis, b[2] = {a == 0 ? 1 : 0, a == 2 ? 1 : 2};
        P.surf_axis = a;
        P.surf_pos = d->surf_pos;
        for (int k = 0; k < 2; ++k) {
            P.surf_lo[k] = P.mesh_lo[b[k]];
            P.surf_id[k] = P.mesh_idelta[b[k]];
            P.surf_n[k] = P.mesh_n[b[k]];
            P.surf_bd[k] = P.mesh_bounded[b[k]];
        }
        P.surf_nbins = (uint32_t)desc_nsurf(d);
    }
    P.pc_on = d->pc_on;
    P.pc_target = d->pc_target;
    P.implicit_capture = d->implicit_capture;
    P.w_cut = d->w_cut;
    P.w_surv = d->w_surv;
    P.has_detector = d->has_detector;
    for (int a = 0; a < 3; ++a) {
        P.det_lo[a] = d->det_lo[a];
        P.det_hi[a] = d->det_hi[a];
    }
    const double t_end = d->census[d->n_census - 1];
    P.imp_on = d->imp_on;
    for (int a = 0; a < 4; ++a) {
        P.imp_n[a] = d->imp_n[a] < 1 ? 1 : d->imp_n[a];
        const double lo = a < 3 ? d->outer_lo[a] : 0.0;
        const double hi = a < 3 ? d->outer_hi[a] : t_end;
        P.imp_lo[a] = lo;
        P.imp_f[a] = (double)P.imp_n[a] / (hi - lo);
    }
    P.ww_on = 0;
    P.ww_params = (const float *)(ws + L.ww_params);
    for (int a = 0; a < 3; ++a) {
        P.ww_lo[a] = d->outer_lo[a];
        P.ww_inv[a] = 1.0 / (d->outer_hi[a] - d->outer_lo[a]);
    }
    P.ww_lo[3] = 0.0;
    P.ww_inv[3] = 1.0 / t_end;
    P.max_events = d->max_events;
    P.stack_cap = d->stack_cap;
    P.problem_id = d->problem_id;
    P.nbins = desc_nbins(d);
}

void timing_begin(mcdc_problem *h, hipStream_t s) {
    if (!h->timing) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(a, s);
    h->events.push_back({a, b});
}

void timing_end(mcdc_problem *h, hipStream_t s) {
    if (!h->timing || h->events.empty()) return;
    (void)hipEventRecord(h->events.back().second, s);
}

static void timing_clear(mcdc_problem *h) {
    for (auto &p : h->events) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    h->events.clear();
}

std::vector<double> pack_tables(const mcdc_problem_desc *d) {
    std::vector<double> t;
    const size_t nst = (size_t)d->n_mat * d->G, nss = nst * d->G;
    t.insert(t.end(), d->sigma_t, d->sigma_t + nst);
    t.insert(t.end(), d->sigma_s, d->sigma_s + nss);
    t.insert(t.end(), d->speed, d->speed + d->G);
    t.insert(t.end(), d->census, d->census + d->n_census);
    if (desc_fissile(d)) {
        t.insert(t.end(), d->nu_sigma_f, d->nu_sigma_f + nst);
        t.insert(t.end(), d->chi, d->chi + nst);
    }
    return t;
}

}  // namespace mcdc

using namespace mcdc;

extern "C" {

const char *mcdc_last_error(void) { return g_err.c_str(); }

size_t mcdc_mlp_param_count(int32_t in_dim) {
    const size_t H = kH;
    return H * (size_t)in_dim + H + H * H + H + H + 1;
}

int mcdc_workspace_bytes(const mcdc_problem_desc *d, const mcdc_options *opt, size_t *bytes) {
    int st = validate_desc(d);
    if (st) return st;
    Options o = resolve_options(opt);
    if ((st = check_options(o))) return st;
    if (d->pc_on && o.schedule != MCDC_SCHED_EVENT)
        return fail(MCDC_E_INVALID, "population control runs in the event schedule");
    if (!bytes) return fail(MCDC_E_INVALID, "null bytes");
    *bytes = make_layout(d, o).total;
    return MCDC_OK;
}

int mcdc_create_problem(const mcdc_problem_desc *d, const mcdc_options *opt, void *dev_ws,
                        size_t bytes, mcdc_handle *out) {
    int st = validate_desc(d);
    if (st) return st;
    if (!out || !dev_ws) return fail(MCDC_E_INVALID, "null workspace or handle");
    Options o = resolve_options(opt);
    if ((st = check_options(o))) return st;
    if (d->pc_on && o.schedule != MCDC_SCHED_EVENT)
        return fail(MCDC_E_INVALID, "population control runs in the event schedule");
    Layout L = make_layout(d, o);
    if (bytes < L.total) return fail(MCDC_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
    auto *h = new mcdc_problem();
    h->desc = *d;
    h->opt = o;
    h->L = L;
    h->ws = (char *)dev_ws;
    h->nbins = desc_nbins(d);
    h->nimp = desc_nimp(d);
    build_dev_problem(d, h->ws, L, h->P);
    if (o.tile_bins) {
        // the hot tile must lie inside the mesh (x, y, z, t, group)
        const int32_t ext[5] = {d->mesh_n[0], d->mesh_n[1], d->mesh_n[2], d->mesh_n[3],
                                d->mesh_per_group ? d->G : 1};
        for (int a = 0; a < 5; ++a) {
            if (o.tile_lo[a] < 0 || o.tile_lo[a] + o.tile_n[a] > ext[a]) {
                delete h;
                return fail(MCDC_E_INVALID, "hot tile outside the mesh");
            }
            h->P.hot_lo[a] = (uint32_t)o.tile_lo[a];
            h->P.hot_n[a] = (uint32_t)o.tile_n[a];
        }
        h->P.hot_bins = o.tile_bins;
    }
    std::vector<double> tab = pack_tables(d);
    hipError_t e = hipMemcpy(h->ws + L.tables, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->ws + L.tally_batch, 0, L.ww_params - L.tally_batch);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "create_problem upload");
    }
    {
        // the kernels find the description at the start of their argument
        // segment: check that once (scratch word: the accumulator's padding)
        int *flag = &((DevAcc *)(h->ws + L.acc))->pad;
        int ok = 0;
        e = launch_problem_check(h->P, flag, 0);
        if (e == hipSuccess) e = hipMemcpy(&ok, flag, sizeof(int), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemset(flag, 0, sizeof(int));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "create_problem check");
        }
        if (!ok) {
            delete h;
            return fail(MCDC_E_HIP, "kernel argument layout differs from the problem description");
        }
    }
    if ((st = cancel_init(h))) {
        delete h;
        return st;
    }
    if (o.schedule == MCDC_SCHED_EVENT && (st = event_init(h))) {
        cancel_free(h);
        delete h;
        return st;
    }
    *out = h;
    return MCDC_OK;
}

int mcdc_set_kernel_timing(mcdc_handle h, int on) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    h->timing = on != 0;
    return MCDC_OK;
}

int mcdc_kernel_time(mcdc_handle h, uint64_t *launches, double *total_ms) {
    if (!h || !launches || !total_ms) return fail(MCDC_E_INVALID, "null argument");
    double ms = 0.0;
    for (auto &p : h->events) {
        hipError_t e = hipEventSynchronize(p.second);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, p.first, p.second);
        if (e != hipSuccess) {
            timing_clear(h);
            return hip_fail(e, "kernel_time");
        }
        ms += t;
    }
    *launches = h->events.size();
    *total_ms = ms;
    timing_clear(h);
    return MCDC_OK;
}

void mcdc_destroy_problem(mcdc_handle h) {
    if (!h) return;
    timing_clear(h);
    event_destroy(h);
    batch_destroy(h);
    cancel_free(h);
    delete h;
}

int mcdc_set_cancel(mcdc_handle h, int on) {
    if (!h || !h->cancel_host) return fail(MCDC_E_INVALID, "null handle");
    __atomic_store_n(h->cancel_host, on ? 1 : 0, __ATOMIC_RELEASE);
    return MCDC_OK;
}

int mcdc_set_trace(mcdc_handle h, mcdc_trace_rec *buf, uint64_t cap, uint64_t *count) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (buf && !count) return fail(MCDC_E_INVALID, "trace needs a device counter");
    h->trace = buf;
    h->trace_cap = buf ? cap : 0;
    h->trace_count = (unsigned long long *)count;
    return MCDC_OK;
}

int mcdc_set_history_scores(mcdc_handle h, double *dev_xh) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    h->xh_out = dev_xh;
    return MCDC_OK;
}

int mcdc_set_ww_mlp(mcdc_handle h, const float *params, size_t n, double logk, double ratio,
                    int32_t n_max, float ymin, float ymax) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (!params) {
        h->P.ww_on = 0;
        h->P.ww_map = nullptr;
        h->P.ww_grid_on = 0;
        return MCDC_OK;
    }
    if (h->desc.stack_cap < 1) return fail(MCDC_E_STATE, "problem was created with stack_cap = 0");
    if (h->P.fis_on) return fail(MCDC_E_STATE, "weight windows are not combined with the k-eigenvalue mode");
    if (h->desc.imp_on) return fail(MCDC_E_STATE, "weight windows and the importance estimate exclude each other");
    if (n != mcdc_mlp_param_count(4 + h->desc.G)) return fail(MCDC_E_INVALID, "wrong parameter count");
    if (!(ratio >= 1.0) || n_max < 2) return fail(MCDC_E_INVALID, "ratio >= 1 and n_max >= 2 required");
    if (!(ymin <= ymax)) return fail(MCDC_E_INVALID, "ymin must not exceed ymax");
    hipError_t e = hipMemcpy(h->ws + h->L.ww_params, params, n * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "set_ww_mlp");
    h->P.ww_on = 1;
    h->P.ww_map = nullptr;                // a new network invalidates any baked map
    for (int a = 0; a < 4; ++a) h->P.ww_map_n[a] = 0;
    h->P.ww_logk = logk;
    h->P.ww_ratio = ratio;
    h->P.ww_nmax = n_max;
    h->P.ww_ymin = ymin;
    h->P.ww_ymax = ymax;
    return MCDC_OK;
}

int mcdc_set_ww_grid(mcdc_handle h, const int32_t n[3]) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle has no weight windows");
    if (!n || (n[0] == 0 && n[1] == 0 && n[2] == 0)) {
        h->P.ww_grid_on = 0;
        return MCDC_OK;
    }
    if (!h->P.ww_on) return fail(MCDC_E_STATE, "set the network with mcdc_set_ww_mlp first");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > (1 << 16)) return fail(MCDC_E_INVALID, "grid planes: n must lie in [1, 65536]");
    for (int a = 0; a < 3; ++a) {
        h->P.ww_grid_n[a] = n[a];
        h->P.ww_grid_d[a] = (h->desc.outer_hi[a] - h->desc.outer_lo[a]) / (double)n[a];
        h->P.ww_grid_id[a] = 1.0 / h->P.ww_grid_d[a];
    }
    h->P.ww_grid_on = 1;
    return MCDC_OK;
}

static RunArgs base_args(mcdc_handle h, uint64_t seed) {
    RunArgs A;
    memset(&A, 0, sizeof(A));
    A.seed = seed;
    A.tally = (double *)(h->ws + h->L.tally_batch);
    A.col = h->desc.col_tally ? (double *)(h->ws + h->L.col_batch) : nullptr;
    A.surf = h->desc.surf_on ? (double *)(h->ws + h->L.surf_batch) : nullptr;
    A.acc = (DevAcc *)(h->ws + h->L.acc);
    A.imp_score = (double *)(h->ws + h->L.imp_score);
    A.imp_weight = (double *)(h->ws + h->L.imp_weight);
    A.xh_out = h->xh_out;
    A.keep_path = h->xh_out != nullptr;
    A.trace = h->trace;
    A.trace_cap = h->trace_cap;
    A.trace_count = h->trace_count;
    A.stk_d = (double *)(h->ws + h->L.stk_d);
    A.stk_i = (int32_t *)(h->ws + h->L.stk_i);
    const uint64_t Ln = h->opt.n_lanes;
    A.imp_cell = (int32_t *)(h->ws + h->L.imp_list);
    A.imp_cnt = (double *)(h->ws + h->L.imp_list + align_up(kImpList * Ln * sizeof(int32_t)));
    A.imp_xsum = A.imp_cnt + kImpList * Ln;
    A.n_lanes = Ln;
    A.cancel = h->cancel_dev;
    return A;
}

}  // extern "C"

RunArgs mcdc::base_args_for(mcdc_problem *h, uint64_t seed) { return base_args(h, seed); }

extern "C" {

// Batch close-outs of an event- or hybrid-schedule run of n histories: every
// per-batch slice in one launch per tally.
static int close_event_run(mcdc_handle h, uint64_t n, hipStream_t s) {
    const uint32_t B = (uint32_t)h->desc.n_batches;
    hipError_t e = launch_closeout_run((double *)(h->ws + h->L.tally_batch),
                                       (double *)(h->ws + h->L.tally_sum),
                                       (double *)(h->ws + h->L.tally_sumsq), h->nbins, B, n, s);
    if (e == hipSuccess && h->desc.col_tally)
        e = launch_closeout_run((double *)(h->ws + h->L.col_batch), (double *)(h->ws + h->L.col_sum),
                                (double *)(h->ws + h->L.col_sumsq), h->nbins, B, n, s);
    if (e == hipSuccess && h->desc.surf_on)
        e = launch_closeout_run((double *)(h->ws + h->L.surf_batch), (double *)(h->ws + h->L.surf_sum),
                                (double *)(h->ws + h->L.surf_sumsq), h->P.surf_nbins, B, n, s);
    if (e != hipSuccess) return hip_fail(e, "run launch");
    for (uint64_t b = 0; b < B; ++b)
        if (((b + 1) * n) / B != (b * n) / B) h->batches += 1;
    h->n_hist += n;
    return MCDC_OK;
}

// One batch of the history schedule: histories [A.h_begin, A.h_end) in one
// launch, then the batch close-out of every tally.
static int history_batch(mcdc_handle h, const RunArgs &A, hipStream_t s) {
    const double nb = (double)(A.h_end - A.h_begin);
    const bool lds = h->opt.lds_tally && h->nbins <= (uint32_t)kLdsTallyMaxBins;
    timing_begin(h, s);
    hipError_t e = launch_history(h->P, A, h->opt.grid, h->opt.block, lds, s);
    timing_end(h, s);
    if (e == hipSuccess)
        e = launch_closeout((double *)(h->ws + h->L.tally_batch), (double *)(h->ws + h->L.tally_sum),
                            (double *)(h->ws + h->L.tally_sumsq), h->nbins, nb, s);
    if (e == hipSuccess && h->desc.col_tally)
        e = launch_closeout((double *)(h->ws + h->L.col_batch), (double *)(h->ws + h->L.col_sum),
                            (double *)(h->ws + h->L.col_sumsq), h->nbins, nb, s);
    if (e == hipSuccess && h->desc.surf_on)
        e = launch_closeout((double *)(h->ws + h->L.surf_batch), (double *)(h->ws + h->L.surf_sum),
                            (double *)(h->ws + h->L.surf_sumsq), h->P.surf_nbins, nb, s);
    if (e != hipSuccess) return hip_fail(e, "run launch");
    h->batches += 1;
    if (cancel_set(h)) return fail(MCDC_E_CANCELLED, "run cancelled");
    return MCDC_OK;
}

int mcdc_run(mcdc_handle h, uint64_t n, uint64_t seed, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle: use mcdc_run_batch");
    if (h->P.fis_on) return fail(MCDC_E_STATE, "a problem with fission runs in the k-eigenvalue mode (mcdc_run_keff)");
    if (h->in_run) return fail(MCDC_E_STATE, "a stepped run is in progress");
    if (h->n_hist + n >= (1ull << 48)) return fail(MCDC_E_INVALID, "history ids exhausted (2^48)");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t B = (uint64_t)h->desc.n_batches;
    const uint64_t h0 = h->n_hist;
    RunArgs A = base_args(h, seed);
    A.h_run0 = h0;
    if (h->opt.schedule == MCDC_SCHED_EVENT) {
        // one pass over all histories of the run; each particle scores into
        // the slice of its history's batch; then every batch is closed out
        if (n == 0) return MCDC_OK;
        A.run_n = n;
        A.run_batches = B;
        if (h->desc.pc_on) {
            // population control synchronises the histories of one batch:
            // each batch is one resident chunk, controlled on its own
            if ((n + B - 1) / B > ev_resident_histories(h))
                return fail(MCDC_E_INVALID, "population control needs event_chunk >= histories per batch");
            for (uint64_t b = 0; b < B; ++b) {
                const uint64_t lo = (b * n) / B, hi = ((b + 1) * n) / B;
                if (hi == lo) continue;
                A.h_begin = h0 + lo;
                A.h_end = h0 + hi;
                double m = floor(h->desc.pc_target * (double)(hi - lo) + 0.5);
                A.pc_m = m < 1.0 ? 1.0 : m;
                int st = event_run_range(h, A, s);
                if (st) return st;
            }
        } else {
            A.h_begin = h0;
            A.h_end = h0 + n;
            int st = event_run_range(h, A, s);
            if (st) return st;
        }
        return close_event_run(h, n, s);
    }
    for (uint64_t b = 0; b < B; ++b) {
        const uint64_t lo = (b * n) / B, hi = ((b + 1) * n) / B;
        if (hi == lo) continue;
        A.h_begin = h0 + lo;
        A.h_end = h0 + hi;
        int st = history_batch(h, A, s);
        if (st) return st;
    }
    h->n_hist += n;
    return MCDC_OK;
}

// ---- census-step control ----------------------------------------------------
//
// A stepped run is taken segment by segment, in the order mcdc_run takes the
// same histories, so that it ends with the same results:
//   event or hybrid schedule, no population control: the resident chunks;
//   event or hybrid schedule with population control: the batches (each one
//     resident chunk, controlled on its own);
//   history schedule: the batches (one launch each).
// An event-schedule segment takes one step per census step; a
// history-schedule segment one step (a history runs through every census
// time within its launch).

static const uint64_t kRunStateMagic = 0x6D636463'72756E32ull;   // "mcdcrun2"

static bool seg_by_batch(const mcdc_problem *h) {
    return h->opt.schedule == MCDC_SCHED_HISTORY || h->desc.pc_on;
}

// Segments of a run of n histories.
static uint64_t seg_count(const mcdc_problem *h, uint64_t n) {
    if (seg_by_batch(h)) return (uint64_t)h->desc.n_batches;
    const uint64_t c = ev_resident_histories(h);
    return c ? (n + c - 1) / c : 0;
}

static void seg_range(const mcdc_problem *h, uint64_t k, uint64_t &lo, uint64_t &hi) {
    if (seg_by_batch(h)) {
        const uint64_t B = (uint64_t)h->desc.n_batches;
        lo = (k * h->run_n) / B;
        hi = ((k + 1) * h->run_n) / B;
    } else {
        const uint64_t c = ev_resident_histories(h);
        lo = k * c;
        hi = lo + c < h->run_n ? lo + c : h->run_n;
    }
}

// The first non-empty segment at or after k (seg_count when none is left).
static uint64_t seg_next(const mcdc_problem *h, uint64_t k) {
    const uint64_t K = seg_count(h, h->run_n);
    for (; k < K; ++k) {
        uint64_t lo, hi;
        seg_range(h, k, lo, hi);
        if (hi > lo) break;
    }
    return k;
}

static RunArgs stepped_args(mcdc_handle h) {
    uint64_t lo, hi;
    seg_range(h, h->run_seg, lo, hi);
    RunArgs A = base_args(h, h->run_seed);
    A.h_run0 = h->run_first;
    A.h_begin = h->run_first + lo;
    A.h_end = h->run_first + hi;
    A.run_n = h->run_n;
    A.run_batches = (uint64_t)h->desc.n_batches;
    const double m = floor(h->desc.pc_target * (double)(hi - lo) + 0.5);
    A.pc_m = m < 1.0 ? 1.0 : m;
    A.keep_path = 1;                     // outputs may be asked for before the last step
    return A;
}

int mcdc_run_begin(mcdc_handle h, uint64_t n, uint64_t seed, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle: use mcdc_run_batch");
    if (h->P.fis_on) return fail(MCDC_E_STATE, "a problem with fission runs in the k-eigenvalue mode (mcdc_run_keff)");
    if (h->in_run) return fail(MCDC_E_STATE, "a stepped run is in progress");
    if (n == 0) return fail(MCDC_E_INVALID, "empty run");
    const uint64_t B = (uint64_t)h->desc.n_batches;
    if (h->opt.schedule == MCDC_SCHED_EVENT && h->desc.pc_on && (n + B - 1) / B > ev_resident_histories(h))
        return fail(MCDC_E_INVALID, "population control needs event_chunk >= histories per batch");
    if (h->n_hist + n >= (1ull << 48)) return fail(MCDC_E_INVALID, "history ids exhausted (2^48)");
    h->run_first = h->n_hist;
    h->run_n = n;
    h->run_seed = seed;
    h->run_steps = 0;
    h->run_seg = seg_next(h, 0);
    if (h->opt.schedule == MCDC_SCHED_EVENT) {
        int st = event_begin(h, stepped_args(h), (hipStream_t)stream);
        if (st) return st;
    }
    h->in_run = true;
    return MCDC_OK;
}

int mcdc_run_step(mcdc_handle h, int32_t *done, void *stream) {
    if (!h || !done) return fail(MCDC_E_INVALID, "null argument");
    if (!h->in_run) return fail(MCDC_E_STATE, "no stepped run in progress");
    *done = 0;
    hipStream_t s = (hipStream_t)stream;
    const bool ev = h->opt.schedule == MCDC_SCHED_EVENT;
    bool seg_done = true;
    int st = ev ? event_step(h, stepped_args(h), s, seg_done) : history_batch(h, stepped_args(h), s);
    if (st) return st;
    if (!ev) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "run step");
    }
    h->run_steps += 1;
    if (!seg_done) return MCDC_OK;
    h->run_seg = seg_next(h, h->run_seg + 1);
    if (h->run_seg < seg_count(h, h->run_n))
        return ev ? event_begin(h, stepped_args(h), s) : MCDC_OK;
    h->in_run = false;
    *done = 1;
    if (ev) return close_event_run(h, h->run_n, s);
    h->n_hist += h->run_n;
    return MCDC_OK;
}

int mcdc_get_run_state(mcdc_handle h, mcdc_run_state *o) {
    if (!h || !o) return fail(MCDC_E_INVALID, "null argument");
    memset(o, 0, sizeof(*o));
    o->magic = kRunStateMagic;
    o->workspace_bytes = h->L.total;
    o->bins = h->nbins;
    o->n_hist = h->n_hist;
    o->batches = (uint64_t)h->batches;
    o->event_iterations = h->event_iterations;
    o->run_first = h->run_first;
    o->run_n = h->run_n;
    o->run_seed = h->run_seed;
    o->segment = h->run_seg;
    o->in_run = h->in_run ? 1 : 0;
    o->steps = h->run_steps;
    return MCDC_OK;
}

int mcdc_set_run_state(mcdc_handle h, const mcdc_run_state *in) {
    if (!h || !in) return fail(MCDC_E_INVALID, "null argument");
    if (in->magic != kRunStateMagic) return fail(MCDC_E_INVALID, "not a run-state record");
    if (in->workspace_bytes != h->L.total || in->bins != h->nbins)
        return fail(MCDC_E_INVALID, "run state of a handle with another description or options");
    if (in->in_run && h->is_batch) return fail(MCDC_E_STATE, "batched handle: use mcdc_run_batch");
    if (in->in_run && (in->run_n == 0 || in->segment >= seg_count(h, in->run_n)))
        return fail(MCDC_E_INVALID, "run-state record names no segment of its run");
    h->n_hist = in->n_hist;
    h->batches = (int64_t)in->batches;
    h->event_iterations = in->event_iterations;
    h->run_first = in->run_first;
    h->run_n = in->run_n;
    h->run_seed = in->run_seed;
    h->run_seg = in->segment;
    h->in_run = in->in_run != 0;
    h->run_steps = in->steps;
    return MCDC_OK;
}

static int read_acc(mcdc_handle h, DevAcc &acc, hipStream_t s) {
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&acc, h->ws + h->L.acc, sizeof(DevAcc), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read accumulators");
    if (acc.status != 0) return fail(acc.status, "a run failed on the device (status " + std::to_string(acc.status) + ")");
    return MCDC_OK;
}

int mcdc_tally_bins(mcdc_handle h, size_t *n) {
    if (!h || !n) return fail(MCDC_E_INVALID, "null argument");
    *n = h->nbins;
    return MCDC_OK;
}

int mcdc_get_raw(mcdc_handle h, double *tsum, double *tsumsq, size_t n, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (n != h->nbins) return fail(MCDC_E_INVALID, "wrong bin count");
    DevAcc acc;
    int st = read_acc(h, acc, (hipStream_t)stream);
    if (st) return st;
    hipError_t e = hipSuccess;
    if (tsum) e = hipMemcpy(tsum, h->ws + h->L.tally_sum, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && tsumsq)
        e = hipMemcpy(tsumsq, h->ws + h->L.tally_sumsq, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_raw");
    return MCDC_OK;
}

int mcdc_get_raw_collision(mcdc_handle h, double *csum, double *csumsq, size_t n, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->is_batch || !h->desc.col_tally)
        return fail(MCDC_E_STATE, "problem created without the collision estimator");
    if (n != h->nbins) return fail(MCDC_E_INVALID, "wrong bin count");
    DevAcc acc;
    int st = read_acc(h, acc, (hipStream_t)stream);
    if (st) return st;
    hipError_t e = hipSuccess;
    if (csum) e = hipMemcpy(csum, h->ws + h->L.col_sum, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && csumsq)
        e = hipMemcpy(csumsq, h->ws + h->L.col_sumsq, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_raw_collision");
    return MCDC_OK;
}

int mcdc_surface_bins(mcdc_handle h, size_t *n) {
    if (!h || !n) return fail(MCDC_E_INVALID, "null argument");
    *n = h->is_batch ? 0 : desc_nsurf(&h->desc);
    return MCDC_OK;
}

int mcdc_get_raw_surface(mcdc_handle h, double *ssum, double *ssumsq, size_t n, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->is_batch || !h->desc.surf_on)
        return fail(MCDC_E_STATE, "problem created without the surface-current tally");
    if (n != desc_nsurf(&h->desc)) return fail(MCDC_E_INVALID, "wrong surface bin count");
    DevAcc acc;
    int st = read_acc(h, acc, (hipStream_t)stream);
    if (st) return st;
    hipError_t e = hipSuccess;
    if (ssum) e = hipMemcpy(ssum, h->ws + h->L.surf_sum, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && ssumsq)
        e = hipMemcpy(ssumsq, h->ws + h->L.surf_sumsq, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_raw_surface");
    return MCDC_OK;
}

}  // extern "C"

void mcdc::fill_counters(const DevAcc &a, mcdc_counters *o) {
    const unsigned long long *c = a.cnt;
    o->histories = c[C_HIST]; o->flights = c[C_FLIGHT]; o->pieces = c[C_PIECE];
    o->collisions = c[C_COLLISION]; o->absorptions = c[C_ABSORB]; o->surfaces = c[C_SURFACE];
    o->leaks = c[C_LEAK]; o->census_stops = c[C_CENSUS]; o->time_ends = c[C_TIME_END];
    o->splits = c[C_SPLIT]; o->rr_kills = c[C_RR_KILL]; o->rr_survivals = c[C_RR_SURVIVE];
    o->cutoff_kills = c[C_CUT_KILL]; o->cutoff_survivals = c[C_CUT_SURVIVE];
    o->detector_hits = c[C_DET_HIT]; o->particles = c[C_PARTICLE];
    o->pc_kills = c[C_PC_KILL]; o->pc_copies = c[C_PC_COPY];
    o->surf_crossings = c[C_SURF];
    o->ww_plane_stops = c[C_WW_PLANE];
    o->w_source = a.wsum[W_SOURCE]; o->w_leak = a.wsum[W_LEAK]; o->w_absorb = a.wsum[W_ABSORB];
    o->w_time_end = a.wsum[W_TIME_END]; o->w_gain = a.wsum[W_GAIN]; o->w_loss = a.wsum[W_LOSS];
    o->path = a.wsum[W_PATH];
    for (int f = 0; f < 6; ++f) o->leak[f] = a.leak[f];
    o->det_sum = a.det[0];
    o->det_sumsq = a.det[1];
    o->status = a.status;
}

extern "C" {

int mcdc_get_counters(mcdc_handle h, mcdc_counters *out, void *stream) {
    if (!h || !out) return fail(MCDC_E_INVALID, "null argument");
    DevAcc acc;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipMemcpy(&acc, h->ws + h->L.acc, sizeof(DevAcc), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_counters");
    memset(out, 0, sizeof(*out));
    fill_counters(acc, out);
    out->batches = h->batches;
    out->n_hist = h->n_hist;
    out->event_iterations = h->event_iterations;
    return MCDC_OK;
}

}  // extern "C"

namespace mcdc {

// What a run reports (the finalization step: tallies with their statistical
// error).  One definition serves the host read-back and the device kernel, so
// both give the same bits.
//   mesh-type bin: mean = S / N / size, with S the sum of the batch sums, N
//   the source histories and size the bin's volume (area on a surface) times
//   its time width; rel = standard error / (S / N) from the batch means,
//   sqrt((S2 - N m^2) / ((B - 1) N)) / m with S2 = sum of S_b^2 / N_b (the
//   weighted form, exact for equal batches too); 0 for a zero mean; NaN with
//   fewer than two batches.
//   detector: mean = X / N; rel = sqrt((X2 / N - m^2) / (N - 1)) / m from the
//   per-history scores (0 for a zero mean, NaN with fewer than two histories).
__host__ __device__ inline void bin_result(double s, double s2, double N, double B, double size,
                                           double &mean, double &rel) {
    const double m = s / N;
    mean = m / size;
    if (B < 2.0) {
        rel = NAN;
    } else if (m <= 0.0) {
        rel = 0.0;
    } else {
        const double var = (s2 - N * m * m) / ((B - 1.0) * N);
        rel = sqrt(var > 0.0 ? var : 0.0) / m;
    }
}

__host__ __device__ inline void detector_result(double x, double x2, double N, double &mean,
                                                double &rel) {
    const double m = x / N;
    mean = m;
    if (N < 2.0) {
        rel = NAN;
    } else if (m <= 0.0) {
        rel = 0.0;
    } else {
        const double var = (x2 / N - m * m) / (N - 1.0);
        rel = sqrt(var > 0.0 ? var : 0.0) / m;
    }
}

__global__ void k_bin_results(const double *__restrict__ s, const double *__restrict__ s2,
                              uint32_t n, double N, double B, double size, double *__restrict__ mean,
                              double *__restrict__ rel) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double m, r;
        bin_result(s[i], s2[i], N, B, size, m, r);
        mean[i] = m;
        if (rel) rel[i] = r;
    }
}

// kind: 1 detector (one value), 2 leakage (six values)
__global__ void k_scalar_results(const DevAcc *__restrict__ acc, int kind, double N,
                                 double *__restrict__ mean, double *__restrict__ rel) {
    const int i = threadIdx.x;
    if (kind == MCDC_TALLY_DETECTOR) {
        if (i != 0) return;
        double m, r;
        detector_result(acc->det[0], acc->det[1], N, m, r);
        mean[0] = m;
        if (rel) rel[0] = r;
    } else if (i < 6) {
        mean[i] = acc->leak[i] / N;
        if (rel) rel[i] = NAN;
    }
}

// Checks shared by both read-backs; on success the sum / sum-of-squares
// offsets and the bin size of a mesh-type kind.
static int tally_kind(mcdc_handle h, int kind, size_t n, size_t &o1, size_t &o2, double &size) {
    if (h->n_hist == 0) return fail(MCDC_E_STATE, "no histories run yet");
    if (kind == MCDC_TALLY_DETECTOR) {
        if (n != 1) return fail(MCDC_E_INVALID, "detector tally has 1 value");
        return MCDC_OK;
    }
    if (kind == MCDC_TALLY_LEAKAGE) {
        if (n != 6) return fail(MCDC_E_INVALID, "leakage tally has 6 values");
        return MCDC_OK;
    }
    if (kind != MCDC_TALLY_MESH && kind != MCDC_TALLY_COLLISION && kind != MCDC_TALLY_SURFACE)
        return fail(MCDC_E_INVALID, "unknown tally kind");
    if (kind == MCDC_TALLY_COLLISION && !h->desc.col_tally)
        return fail(MCDC_E_STATE, "problem created without the collision estimator");
    if (kind == MCDC_TALLY_SURFACE && !h->desc.surf_on)
        return fail(MCDC_E_STATE, "problem created without the surface-current tally");
    const bool surf = kind == MCDC_TALLY_SURFACE;
    if (n != (surf ? desc_nsurf(&h->desc) : (size_t)h->nbins)) return fail(MCDC_E_INVALID, "wrong bin count");
    o1 = surf ? h->L.surf_sum : (kind == MCDC_TALLY_MESH ? h->L.tally_sum : h->L.col_sum);
    o2 = surf ? h->L.surf_sumsq : (kind == MCDC_TALLY_MESH ? h->L.tally_sumsq : h->L.col_sumsq);
    // mesh bins: volume times time width; surface bins: area on the plane
    // times time width; an unbounded axis is not cut
    size = 1.0;
    for (int a = 0; a < 4; ++a)
        if ((a == 3 || h->P.mesh_bounded[a]) && !(surf && a == h->desc.surf_axis))
            size *= h->P.mesh_delta[a];
    return MCDC_OK;
}

}  // namespace mcdc

extern "C" {

int mcdc_get_tallies(mcdc_handle h, int kind, double *mean, double *rel, size_t n, void *stream) {
    if (!h || !mean) return fail(MCDC_E_INVALID, "null argument");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle: use mcdc_get_batch_raw");
    DevAcc acc;
    int st = read_acc(h, acc, (hipStream_t)stream);
    if (st) return st;
    size_t o1 = 0, o2 = 0;
    double size = 1.0;
    if ((st = tally_kind(h, kind, n, o1, o2, size))) return st;
    const double N = (double)h->n_hist;
    if (kind == MCDC_TALLY_DETECTOR) {
        double r;
        detector_result(acc.det[0], acc.det[1], N, mean[0], r);
        if (rel) rel[0] = r;
        return MCDC_OK;
    }
    if (kind == MCDC_TALLY_LEAKAGE) {
        for (int f = 0; f < 6; ++f) {
            mean[f] = acc.leak[f] / N;
            if (rel) rel[f] = NAN;
        }
        return MCDC_OK;
    }
    std::vector<double> s(n), s2(n);
    hipError_t e = hipMemcpy(s.data(), h->ws + o1, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(s2.data(), h->ws + o2, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_tallies");
    const double B = (double)h->batches;
    for (size_t i = 0; i < n; ++i) {
        double r;
        bin_result(s[i], s2[i], N, B, size, mean[i], r);
        if (rel) rel[i] = r;
    }
    return MCDC_OK;
}

int mcdc_get_tallies_device(mcdc_handle h, int kind, double *dev_mean, double *dev_rel, size_t n,
                            void *stream) {
    if (!h || !dev_mean) return fail(MCDC_E_INVALID, "null argument");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle: use mcdc_get_batch_raw");
    if (h->in_run) return fail(MCDC_E_STATE, "a stepped run is in progress");
    size_t o1 = 0, o2 = 0;
    double size = 1.0;
    int st = tally_kind(h, kind, n, o1, o2, size);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const double N = (double)h->n_hist;
    if (kind == MCDC_TALLY_DETECTOR || kind == MCDC_TALLY_LEAKAGE) {
        hipLaunchKernelGGL(k_scalar_results, dim3(1), dim3(64), 0, s,
                           (const DevAcc *)(h->ws + h->L.acc), kind, N, dev_mean, dev_rel);
    } else {
        const int block = 256;
        int grid = (int)((n + block - 1) / block);
        if (grid > 65536) grid = 65536;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(k_bin_results, dim3(grid), dim3(block), 0, s,
                           (const double *)(h->ws + o1), (const double *)(h->ws + o2), (uint32_t)n,
                           N, (double)h->batches, size, dev_mean, dev_rel);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "get_tallies_device");
    return MCDC_OK;
}

int mcdc_reset_tallies(mcdc_handle h, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (h->in_run) return fail(MCDC_E_STATE, "a stepped run is in progress");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemset(h->ws + h->L.tally_batch, 0, h->L.ww_params - h->L.tally_batch);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "reset_tallies");
    h->batches = 0;
    h->n_hist = 0;
    return MCDC_OK;
}

int mcdc_get_importance(mcdc_handle h, double *score, double *weight, size_t n, void *stream) {
    if (!h) return fail(MCDC_E_INVALID, "null handle");
    if (!h->desc.imp_on || n != h->nimp) return fail(MCDC_E_INVALID, "importance not enabled or wrong size");
    DevAcc acc;
    int st = read_acc(h, acc, (hipStream_t)stream);
    if (st) return st;
    hipError_t e = hipSuccess;
    if (score) e = hipMemcpy(score, h->ws + h->L.imp_score, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && weight)
        e = hipMemcpy(weight, h->ws + h->L.imp_weight, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_importance");
    return MCDC_OK;
}

}  // extern "C"
