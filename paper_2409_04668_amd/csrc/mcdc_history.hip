// History-based tracking kernel: one work-item carries one history (its source
// particle and, with weight windows, its split daughters on a LIFO stack) from
// birth to the end, flight by flight.  The grid is persistent (a fixed number
// of workgroups sized to the chip) and work-items stride over history ids, so
// a work-item whose history ends starts its next history in the same loop
// iteration instead of idling until the wave drains.
//
// Tallies: track-length pieces go to FP64 atomics, either straight into the
// batch accumulator in HBM or, when the whole mesh fits, into an LDS tile per
// workgroup that is flushed with one global atomic per touched bin at the end.
#include "transport_device.hpp"

namespace mcdc {

struct Shared {
    unsigned long long cnt[N_CNT];
    double wsum[N_WSUM];
    double leak[6];
};

MCDC_DEV void trace_rec(const RunArgs &A, uint64_t hist, Part &q, int type, double aux) {
    const uint32_t seq = q.seq;
    q.seq += 1u;
    if (A.trace == nullptr) return;
    const unsigned long long i = atomicAdd(A.trace_count, 1ull);
    if (i >= A.trace_cap) return;
    mcdc_trace_rec r;
    r.hist = hist;
    r.tag = q.tag;
    r.seq = seq;
    r.type = type;
    r.g = q.g;
    r.cell = q.cell;
    r.k = q.k;
    r.x = q.x[0]; r.y = q.x[1]; r.z = q.x[2]; r.t = q.t;
    r.ux = q.u[0]; r.uy = q.u[1]; r.uz = q.u[2]; r.w = q.w;
    r.aux = aux;
    A.trace[i] = r;
}

MCDC_DEV void set_status(const RunArgs &A, int st) { atomicMin(&A.acc->status, st); }

// Per-work-item history context.
struct Hist {
    uint64_t id;
    double xh, path;
    int64_t events;
    int sp;
    int n_imp;
};

// outer boundary after a surface crossing; returns the leak face or -1
MCDC_DEV int boundary(const DevProblem &P, Part &q) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (axis_in(P.outer_lo[a], P.outer_hi[a], q.x[a], q.u[a])) continue;
        const int side = q.x[a] >= P.outer_hi[a] ? 1 : 0;
        const int face = 2 * a + side;
        if (P.bc[face] == MCDC_REFLECTIVE) {
            q.x[a] = side ? P.outer_hi[a] : P.outer_lo[a];
            q.u[a] = -q.u[a];
        } else {
            return face;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (axis_in(P.outer_lo[a], P.outer_hi[a], q.x[a], q.u[a])) continue;
        return 2 * a + (q.x[a] >= P.outer_hi[a] ? 1 : 0);
    }
    return -1;
}

MCDC_DEV void leak(Shared &S, Part &q, int face) {
    atomicAdd(&S.leak[face], q.w);
    atomicAdd(&S.wsum[W_LEAK], q.w);
    atomicAdd(&S.cnt[C_LEAK], 1ull);
    q.alive = false;
}

// stack storage: SoA [field][depth][lane]
MCDC_DEV void push(const RunArgs &A, uint64_t lane, int cap, int depth, const Part &q) {
    const uint64_t L = A.n_lanes;
    const uint64_t o = (uint64_t)depth * L + lane;
    const uint64_t F = (uint64_t)cap * L;
    A.stk_d[0 * F + o] = q.x[0];
    A.stk_d[1 * F + o] = q.x[1];
    A.stk_d[2 * F + o] = q.x[2];
    A.stk_d[3 * F + o] = q.u[0];
    A.stk_d[4 * F + o] = q.u[1];
    A.stk_d[5 * F + o] = q.u[2];
    A.stk_d[6 * F + o] = q.t;
    A.stk_d[7 * F + o] = q.w;
    A.stk_i[0 * F + o] = q.g;
    A.stk_i[1 * F + o] = q.cell;
    A.stk_i[2 * F + o] = q.ci;
    A.stk_i[3 * F + o] = (int32_t)q.tag;
}

MCDC_DEV void pop(const RunArgs &A, uint64_t lane, int cap, int depth, Part &q) {
    const uint64_t L = A.n_lanes;
    const uint64_t o = (uint64_t)depth * L + lane;
    const uint64_t F = (uint64_t)cap * L;
    q.x[0] = A.stk_d[0 * F + o];
    q.x[1] = A.stk_d[1 * F + o];
    q.x[2] = A.stk_d[2 * F + o];
    q.u[0] = A.stk_d[3 * F + o];
    q.u[1] = A.stk_d[4 * F + o];
    q.u[2] = A.stk_d[5 * F + o];
    q.t = A.stk_d[6 * F + o];
    q.w = A.stk_d[7 * F + o];
    q.g = A.stk_i[0 * F + o];
    q.cell = A.stk_i[1 * F + o];
    q.ci = A.stk_i[2 * F + o];
    q.tag = (uint32_t)A.stk_i[3 * F + o];
    q.k = 0;
    q.seq = 0;
    q.alive = true;
}

// Weight-window check (learned importance): split above the window into
// n = min(ceil(w / w_T), n_max) copies (daughters pushed LIFO with tags from
// one parent Philox block), roulette below it, nothing (and no draw) inside.
MCDC_DEV void ww_check(const DevProblem &P, const RunArgs &A, Shared &S, uint64_t lane, Hist &H,
                       Part &q) {
    float in[4 + kMaxG];
#pragma unroll
    for (int a = 0; a < 3; ++a) in[a] = (float)(2.0 * ((q.x[a] - P.ww_lo[a]) * P.ww_inv[a]) - 1.0);
    in[3] = (float)(2.0 * ((q.t - P.ww_lo[3]) * P.ww_inv[3]) - 1.0);
#pragma unroll
    for (int g = 0; g < kMaxG; ++g) in[4 + g] = g == q.g ? 1.0f : 0.0f;
    const float y = mlp_infer(P.ww_params, 4 + P.G, in);
    const double wt = own_exp(P.ww_logk - (double)y);
    const double wl = (2.0 * wt) / (1.0 + P.ww_ratio);
    const double wu = P.ww_ratio * wl;
    if (q.w > wu) {
        const double ratio = q.w / wt;
        const int n = ratio >= (double)P.ww_nmax ? P.ww_nmax : (int)ceil(ratio);
        if (n < 2) return;
        Rng r = make_rng(A.seed, H.id, P.problem_id, q.tag, q.k);
        uint32_t blk[4];
        rng_block(r, blk);
        q.k = r.k;
        const double wn = q.w / (double)n;
        q.w = wn;
        for (int i = 1; i < n; ++i) {
            if (H.sp >= P.stack_cap) {
                set_status(A, MCDC_E_STACK);
                return;
            }
            Part d = q;
            d.tag = blk[0] + (uint32_t)i * 0x9E3779B9u;
            push(A, lane, P.stack_cap, H.sp, d);
            H.sp += 1;
        }
        atomicAdd(&S.cnt[C_SPLIT], (unsigned long long)(n - 1));
        atomicAdd(&S.cnt[C_PARTICLE], (unsigned long long)(n - 1));
        trace_rec(A, H.id, q, EV_SPLIT, (double)n);
    } else if (q.w < wl) {
        Rng r = make_rng(A.seed, H.id, P.problem_id, q.tag, q.k);
        const double xi = rng_uniform(r);
        q.k = r.k;
        if (xi * wt < q.w) {
            atomicAdd(&S.wsum[W_GAIN], wt - q.w);
            q.w = wt;
            atomicAdd(&S.cnt[C_RR_SURVIVE], 1ull);
            trace_rec(A, H.id, q, EV_RR_SURVIVE, 0.0);
        } else {
            atomicAdd(&S.wsum[W_LOSS], q.w);
            atomicAdd(&S.cnt[C_RR_KILL], 1ull);
            q.alive = false;
            trace_rec(A, H.id, q, EV_RR_KILL, 0.0);
        }
    }
}

MCDC_DEV void imp_point(const DevProblem &P, const RunArgs &A, uint64_t lane, Hist &H,
                        const Part &q) {
    int ix[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double x = a < 3 ? q.x[a] : q.t;
        const double f = (x - P.imp_lo[a]) * P.imp_f[a];
        int i = (int)floor(f);
        if (i < 0) i = 0;
        if (i > P.imp_n[a] - 1) i = P.imp_n[a] - 1;
        ix[a] = i;
    }
    int c = q.g;
    c = c * P.imp_n[3] + ix[3];
    c = c * P.imp_n[2] + ix[2];
    c = c * P.imp_n[1] + ix[1];
    c = c * P.imp_n[0] + ix[0];
    const uint64_t L = A.n_lanes;
    for (int i = 0; i < H.n_imp; ++i) {
        if (A.imp_cell[i * L + lane] == c) {
            A.imp_cnt[i * L + lane] += 1.0;
            A.imp_xsum[i * L + lane] += H.xh;
            return;
        }
    }
    if (H.n_imp < kImpList) {
        A.imp_cell[H.n_imp * L + lane] = c;
        A.imp_cnt[H.n_imp * L + lane] = 1.0;
        A.imp_xsum[H.n_imp * L + lane] = H.xh;
        H.n_imp += 1;
    }
}

// One flight: census / surface / collision distances, the event (ties: census,
// then surface, then collision), scoring, the move, and the event itself.
template <class T, bool WW, bool IMP>
MCDC_DEV void flight(const DevProblem &P, const RunArgs &A, Shared &S, const T &tally,
                     uint64_t lane, Hist &H, Part &q, uint32_t &n_flight, uint32_t &n_piece,
                     double &path) {
    H.events += 1;
    if (H.events > P.max_events) {
        set_status(A, MCDC_E_EVENT_CAP);
        q.alive = false;
        H.sp = 0;
        return;
    }
    n_flight += 1;
    if (IMP) imp_point(P, A, lane, H, q);

    const int mat = q.cell >= 0 ? P.box_mat[q.cell] : P.background_mat;
    const double sig_t = P.sigma_t[mat * P.G + q.g];
    const double v = P.speed[q.g];
    double iu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) iu[a] = q.u[a] != 0.0 ? 1.0 / q.u[a] : 0.0;

    const double tc = P.census[q.ci];
    const double d_t = (tc - q.t) * v;
    int sax;
    double spl;
    const double d_s = dist_surface(P, q.x, q.u, iu, sax, spl);
    double d_c = kInf;
    Rng r = make_rng(A.seed, H.id, P.problem_id, q.tag, q.k);
    if (sig_t > 0.0) {
        const double xi = rng_uniform(r);
        d_c = (-own_log(xi)) / sig_t;
    }
    q.k = r.k;

    int ev;
    double d;
    if (d_t <= d_s && d_t <= d_c) { ev = EV_CENSUS; d = d_t; }
    else if (d_s <= d_c) { ev = EV_SURFACE; d = d_s; }
    else { ev = EV_SCATTER; d = d_c; }

    n_piece += score_mesh(P, q.x, q.u, iu, q.t, v, d, q.w, q.g, tally);
    if (P.has_detector) {
        const double l = detector_len(P, q.x, q.u, iu, d);
        if (l > 0.0) H.xh += q.w * l;
    }
    path += q.w * d;
    H.path += q.w * d;

    q.x[0] = q.x[0] + q.u[0] * d;
    q.x[1] = q.x[1] + q.u[1] * d;
    q.x[2] = q.x[2] + q.u[2] * d;

    if (ev == EV_CENSUS) {
        q.t = tc;
        if (q.ci == P.n_census - 1) {
            atomicAdd(&S.wsum[W_TIME_END], q.w);
            atomicAdd(&S.cnt[C_TIME_END], 1ull);
            q.alive = false;
            trace_rec(A, H.id, q, EV_TIME_END, d);
        } else {
            q.ci += 1;
            atomicAdd(&S.cnt[C_CENSUS], 1ull);
            trace_rec(A, H.id, q, EV_CENSUS, d);
        }
        return;
    }
    q.t = q.t + d / v;

    if (ev == EV_SURFACE) {
        // snap the crossing coordinate onto the plane (select, no dynamic index)
        if (sax == 0) q.x[0] = spl;
        else if (sax == 1) q.x[1] = spl;
        else if (sax == 2) q.x[2] = spl;
        atomicAdd(&S.cnt[C_SURFACE], 1ull);
        const int face = boundary(P, q);
        if (face >= 0) {
            leak(S, q, face);
            trace_rec(A, H.id, q, EV_LEAK, d);
            return;
        }
        q.cell = locate(P, q.x, q.u);
        trace_rec(A, H.id, q, EV_SURFACE, d);
        if (WW) ww_check(P, A, S, lane, H, q);
        return;
    }

    atomicAdd(&S.cnt[C_COLLISION], 1ull);
    const double *ss_row = P.sigma_s + (mat * P.G + q.g) * P.G;
    double sig_s = 0.0;
    for (int h = 0; h < P.G; ++h) sig_s = sig_s + ss_row[h];
    r = make_rng(A.seed, H.id, P.problem_id, q.tag, q.k);
    if (!P.implicit_capture) {
        const double xi = rng_uniform(r);
        q.k = r.k;
        if (!(xi * sig_t < sig_s)) {
            atomicAdd(&S.wsum[W_ABSORB], q.w);
            atomicAdd(&S.cnt[C_ABSORB], 1ull);
            q.alive = false;
            trace_rec(A, H.id, q, EV_ABSORB, d);
            return;
        }
    } else {
        const double c = sig_s / sig_t;
        const double wn = q.w * c;
        atomicAdd(&S.wsum[W_ABSORB], q.w - wn);
        q.w = wn;
        if (q.w < P.w_cut) {
            const double xi = rng_uniform(r);
            q.k = r.k;
            if (xi * P.w_surv < q.w) {
                atomicAdd(&S.wsum[W_GAIN], P.w_surv - q.w);
                q.w = P.w_surv;
                atomicAdd(&S.cnt[C_CUT_SURVIVE], 1ull);
            } else {
                atomicAdd(&S.wsum[W_LOSS], q.w);
                atomicAdd(&S.cnt[C_CUT_KILL], 1ull);
                q.alive = false;
                trace_rec(A, H.id, q, EV_CUT_KILL, d);
                return;
            }
        }
    }
    if (P.G > 1) {
        const double xi = rng_uniform(r);
        const double target = xi * sig_s;
        double cum = 0.0;
        int gn = -1, last = 0;
        for (int h = 0; h < P.G; ++h) {
            cum = cum + ss_row[h];
            if (ss_row[h] > 0.0) last = h;
            if (gn < 0 && target < cum) gn = h;
        }
        q.g = gn >= 0 ? gn : last;
    }
    iso_direction(r, q.u[0], q.u[1], q.u[2]);
    q.k = r.k;
    trace_rec(A, H.id, q, EV_SCATTER, d);
    if (WW) ww_check(P, A, S, lane, H, q);
}

// Source particle: position, birth time, direction, group, unit weight, cell;
// leaks at once when born on the outer boundary moving out.
MCDC_DEV void source(const DevProblem &P, const RunArgs &A, Shared &S, Hist &H, Part &q) {
    q.tag = 0;
    q.k = 0;
    q.seq = 0;
    Rng r = make_rng(A.seed, H.id, P.problem_id, 0u, 0u);
    if (P.src_box) {
#pragma unroll
        for (int a = 0; a < 3; ++a) q.x[a] = P.src_lo[a] + rng_uniform(r) * (P.src_hi[a] - P.src_lo[a]);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) q.x[a] = P.src_lo[a];
    }
    q.t = P.src_t0;
    if (P.src_t1 > P.src_t0) q.t = P.src_t0 + rng_uniform(r) * (P.src_t1 - P.src_t0);
    if (P.src_isotropic) {
        iso_direction(r, q.u[0], q.u[1], q.u[2]);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) q.u[a] = P.src_dir[a];
    }
    q.g = P.src_group;
    q.w = 1.0;
    q.k = r.k;
    q.alive = true;
    q.ci = 0;
    while (q.ci < P.n_census && !(P.census[q.ci] > q.t)) q.ci += 1;
    atomicAdd(&S.cnt[C_PARTICLE], 1ull);
    atomicAdd(&S.wsum[W_SOURCE], q.w);
    q.cell = locate(P, q.x, q.u);
    if (q.ci >= P.n_census) {
        atomicAdd(&S.wsum[W_TIME_END], q.w);
        atomicAdd(&S.cnt[C_TIME_END], 1ull);
        q.alive = false;
        trace_rec(A, H.id, q, EV_TIME_END, 0.0);
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!axis_in(P.outer_lo[a], P.outer_hi[a], q.x[a], q.u[a])) {
            leak(S, q, 2 * a + (q.x[a] >= P.outer_hi[a] ? 1 : 0));
            trace_rec(A, H.id, q, EV_LEAK, 0.0);
            return;
        }
    }
    trace_rec(A, H.id, q, EV_SOURCE, 0.0);
}

MCDC_DEV void finish_history(const DevProblem &P, const RunArgs &A, Shared &S, uint64_t lane,
                             const Hist &H) {
    if (H.xh != 0.0) {
        unsafeAtomicAdd(&A.acc->det[0], H.xh);
        unsafeAtomicAdd(&A.acc->det[1], H.xh * H.xh);
    }
    if (H.xh > 0.0) atomicAdd(&S.cnt[C_DET_HIT], 1ull);
    if (A.xh_out) {
        A.xh_out[2 * (H.id - A.h_run0)] = H.xh;
        A.xh_out[2 * (H.id - A.h_run0) + 1] = H.path;
    }
    if (P.imp_on) {
        const uint64_t L = A.n_lanes;
        for (int i = 0; i < H.n_imp; ++i) {
            const int c = A.imp_cell[i * L + lane];
            const double cnt = A.imp_cnt[i * L + lane];
            unsafeAtomicAdd(&A.imp_score[c], cnt * H.xh - A.imp_xsum[i * L + lane]);
            unsafeAtomicAdd(&A.imp_weight[c], cnt);
        }
    }
}

template <bool LDS, bool WW, bool IMP>
__global__ void __launch_bounds__(256) k_history(DevProblem P, RunArgs A) {
    extern __shared__ double s_tile[];
    __shared__ Shared S;
    for (int i = threadIdx.x; i < N_CNT; i += blockDim.x) S.cnt[i] = 0ull;
    for (int i = threadIdx.x; i < N_WSUM; i += blockDim.x) S.wsum[i] = 0.0;
    for (int i = threadIdx.x; i < 6; i += blockDim.x) S.leak[i] = 0.0;
    if (LDS)
        for (uint32_t i = threadIdx.x; i < P.nbins; i += blockDim.x) s_tile[i] = 0.0;
    __syncthreads();

    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = A.n_lanes;
    uint64_t next = A.h_begin + lane;
    uint32_t n_flight = 0, n_piece = 0, n_hist = 0;
    double path = 0.0;
    Part q;
    q.alive = false;
    Hist H;
    H.sp = 0;
    H.id = 0;
    bool in_hist = false;
    typename std::conditional<LDS, LdsTally, GlobalTally>::type tally{LDS ? s_tile : A.tally};

    for (;;) {
        if (!q.alive) {
            if (WW && H.sp > 0) {
                H.sp -= 1;
                pop(A, lane, P.stack_cap, H.sp, q);
            } else {
                if (in_hist) {
                    finish_history(P, A, S, lane, H);
                    in_hist = false;
                }
                if (next >= A.h_end) break;
                H.id = next;
                next += stride;
                H.xh = 0.0;
                H.path = 0.0;
                H.events = 0;
                H.sp = 0;
                H.n_imp = 0;
                in_hist = true;
                n_hist += 1;
                source(P, A, S, H, q);
                if (!q.alive) continue;
            }
        }
        flight<decltype(tally), WW, IMP>(P, A, S, tally, lane, H, q, n_flight, n_piece, path);
    }

    atomicAdd(&S.cnt[C_HIST], (unsigned long long)n_hist);
    atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
    atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
    atomicAdd(&S.wsum[W_PATH], path);
    __syncthreads();
    if (LDS) {
        for (uint32_t i = threadIdx.x; i < P.nbins; i += blockDim.x) {
            const double v = s_tile[i];
            if (v != 0.0) unsafeAtomicAdd(&A.tally[i], v);
        }
    }
    for (int i = threadIdx.x; i < N_CNT; i += blockDim.x)
        if (S.cnt[i]) atomicAdd(&A.acc->cnt[i], S.cnt[i]);
    for (int i = threadIdx.x; i < N_WSUM; i += blockDim.x)
        if (S.wsum[i] != 0.0) unsafeAtomicAdd(&A.acc->wsum[i], S.wsum[i]);
    for (int i = threadIdx.x; i < 6; i += blockDim.x)
        if (S.leak[i] != 0.0) unsafeAtomicAdd(&A.acc->leak[i], S.leak[i]);
}

// Batch close-out: per bin, sum += S_b, sumsq += S_b^2 / N_b, S_b = 0.
__global__ void k_closeout(double *__restrict__ batch, double *__restrict__ sum,
                           double *__restrict__ sumsq, uint32_t n, double nb) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double sb = batch[i];
        if (sb != 0.0) {
            sum[i] = sum[i] + sb;
            sumsq[i] = sumsq[i] + sb * sb / nb;
            batch[i] = 0.0;
        }
    }
}

int history_grid(int block, int waves_per_cu) {
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
    }
    const int waves_per_block = block / 64;
    int g = n_cu * waves_per_cu / waves_per_block;
    return g < 1 ? 1 : g;
}

hipError_t launch_history(const DevProblem &P, const RunArgs &A, int grid, int block,
                          bool lds_tally, hipStream_t s) {
    const size_t shm = lds_tally ? (size_t)P.nbins * sizeof(double) : 0;
    const bool ww = P.ww_on != 0, imp = P.imp_on != 0;
#define MCDC_LAUNCH(L, W, I) \
    hipLaunchKernelGGL((k_history<L, W, I>), dim3(grid), dim3(block), shm, s, P, A)
    if (lds_tally) {
        if (ww) MCDC_LAUNCH(true, true, false);
        else if (imp) MCDC_LAUNCH(true, false, true);
        else MCDC_LAUNCH(true, false, false);
    } else {
        if (ww) MCDC_LAUNCH(false, true, false);
        else if (imp) MCDC_LAUNCH(false, false, true);
        else MCDC_LAUNCH(false, false, false);
    }
#undef MCDC_LAUNCH
    return hipGetLastError();
}

hipError_t launch_closeout(double *batch, double *sum, double *sumsq, uint32_t n, double nb,
                           hipStream_t s) {
    const int block = 256;
    int grid = (int)((n + block - 1) / block);
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_closeout, dim3(grid), dim3(block), 0, s, batch, sum, sumsq, n, nb);
    return hipGetLastError();
}

}  // namespace mcdc
