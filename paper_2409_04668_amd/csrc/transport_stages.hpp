// The transport loop split into stages: source, flight (distances, event
// selection, scoring, move, census), surface crossing, collision, weight-window
// check.  The history-based kernel and the hybrid lead stage call them back
// to back for one particle; the event-based kernels call each stage over a
// compacted bank of particles.  A context object supplies what belongs to the
// particle's history (its id for the random streams, its detector score, its
// flight count, where split daughters go, its tally slices), so every schedule
// shares one definition of the arithmetic.
#pragma once

#include "transport_device.hpp"

namespace mcdc {

struct Shared {
    unsigned long long cnt[N_CNT];
    double wsum[N_WSUM];
    double leak[6];
    double kcol;
};

MCDC_DEV void shared_zero(Shared &S) {
    for (int i = threadIdx.x; i < N_CNT; i += blockDim.x) S.cnt[i] = 0ull;
    for (int i = threadIdx.x; i < N_WSUM; i += blockDim.x) S.wsum[i] = 0.0;
    for (int i = threadIdx.x; i < 6; i += blockDim.x) S.leak[i] = 0.0;
    if (threadIdx.x == 0) S.kcol = 0.0;
}

// after a __syncthreads(): one global atomic per non-zero entry
MCDC_DEV void shared_flush(const Shared &S, DevAcc *acc) {
    for (int i = threadIdx.x; i < N_CNT; i += blockDim.x)
        if (S.cnt[i]) atomicAdd(&acc->cnt[i], S.cnt[i]);
    for (int i = threadIdx.x; i < N_WSUM; i += blockDim.x)
        if (S.wsum[i] != 0.0) unsafeAtomicAdd(&acc->wsum[i], S.wsum[i]);
    for (int i = threadIdx.x; i < 6; i += blockDim.x)
        if (S.leak[i] != 0.0) unsafeAtomicAdd(&acc->leak[i], S.leak[i]);
    if (threadIdx.x == 0 && S.kcol != 0.0) unsafeAtomicAdd(&acc->kcol, S.kcol);
}

// Reserve n consecutive entries of *count for every active lane with one
// atomic per wave: a wave-uniform loop over the active lanes (ascending) sums
// their counts and hands each lane its offset.
MCDC_DEV uint32_t wave_reserve_n(uint32_t *count, uint32_t n) {
    const uint64_t act = __ballot(true);
    uint64_t m = act;
    const int lane = (int)__lane_id();
    uint32_t total = 0, mine = 0;
    while (m) {
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        const uint32_t nl = (uint32_t)__builtin_amdgcn_readlane((int)n, l);
        if (lane == l) mine = total;
        total += nl;
    }
    const int leader = __ffsll((long long)act) - 1;
    uint32_t base = 0;
    if (lane == leader && total) base = atomicAdd(count, total);
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    return base + mine;
}

// One entry of *count for every active lane with one atomic per wave; the
// active lanes take consecutive entries in ascending lane order.
MCDC_DEV uint32_t wave_reserve_one(uint32_t *count) {
    const uint64_t act = __ballot(true);
    const int leader = __ffsll((long long)act) - 1;
    uint32_t base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(act));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    return base + __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
}

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

// The host's cancel word, read past every cache (it lives in host memory and
// the host writes it while kernels run).  A read of host memory is slow and
// many at once queue on the link (every lane reading it at its own history
// starts made the lead stage 2.3x slower; one read per wave every 256 flights
// still cost 4%), so the persistent tracking kernels read it from one
// work-item per workgroup (before the first history, then at every
// kCancelPoll-th history that work-item starts) and publish it in LDS, where
// every work-item looks at each history start.
constexpr uint32_t kCancelPoll = 64;
MCDC_DEV bool cancel_requested(const int *flag) {
    return flag != nullptr &&
           __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// The workgroup's copy of the cancel word (LDS).
struct CancelSeen {
    uint32_t *lds;
    // before the workgroup's first history (a __syncthreads() must follow)
    MCDC_DEV void init(const int *flag) const {
        if (threadIdx.x == 0) *(volatile uint32_t *)lds = cancel_requested(flag) ? 1u : 0u;
    }
    // at a history start: work-item 0 reads the host word again every
    // kCancelPoll-th of its histories; every work-item reads the copy
    MCDC_DEV bool check(const int *flag, uint32_t started) const {
        if (threadIdx.x == 0 && started % kCancelPoll == kCancelPoll - 1 && cancel_requested(flag))
            *(volatile uint32_t *)lds = 1u;
        return *(volatile uint32_t *)lds != 0u;
    }
};

// outer boundary after a surface crossing; returns the leak face or -1
MCDC_DEV int boundary(CP &P, Part &q) {
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

// Weight-window check: split above the window into n = min(ceil(w / w_T),
// n_max) copies (daughters get stream tags from one parent Philox block),
// roulette below it, nothing (and no draw) inside.  w_T comes from the
// network at the particle's point, or from the map cell that holds it.
template <class Ctx>
MCDC_DEV void ww_check(CP &P, const RunArgs &A, Shared &S, Ctx &C, Part &q) {
    double wt;
    if (Ctx::kWWMap) {
        wt = P.ww_map[ww_map_cell(P, q)];
    } else {
        float xt[4];
#pragma unroll
        for (int a = 0; a < 3; ++a) xt[a] = (float)(2.0 * ((q.x[a] - P.ww_lo[a]) * P.ww_inv[a]) - 1.0);
        xt[3] = (float)(2.0 * ((q.t - P.ww_lo[3]) * P.ww_inv[3]) - 1.0);
        wt = ww_net_target(P, C.mlp_params(P), xt, q.g);
    }
    const double wl = (2.0 * wt) / (1.0 + P.ww_ratio);
    const double wu = P.ww_ratio * wl;
    if (q.w > wu) {
        const double ratio = q.w / wt;
        const int n = ratio >= (double)P.ww_nmax ? P.ww_nmax : (int)ceil(ratio);
        if (n < 2) return;
        Rng r = make_rng(A.seed, C.hist(), P.problem_id, q.tag, q.k);
        uint32_t blk[4];
        rng_block(r, blk);
        q.k = r.k;
        const double wn = q.w / (double)n;
        q.w = wn;
        // daughters i = 1..n-1: the parent's state with tag blk[0] + i * golden,
        // fresh counter and sequence (the context stores or defers them)
        if (!C.push_daughters(q, blk[0], n)) return;
        atomicAdd(&S.cnt[C_SPLIT], (unsigned long long)(n - 1));
        atomicAdd(&S.cnt[C_PARTICLE], (unsigned long long)(n - 1));
        trace_rec(A, C.hist(), q, EV_SPLIT, (double)n);
    } else if (q.w < wl) {
        Rng r = make_rng(A.seed, C.hist(), P.problem_id, q.tag, q.k);
        const double xi = rng_uniform(r);
        q.k = r.k;
        if (xi * wt < q.w) {
            atomicAdd(&S.wsum[W_GAIN], wt - q.w);
            q.w = wt;
            atomicAdd(&S.cnt[C_RR_SURVIVE], 1ull);
            trace_rec(A, C.hist(), q, EV_RR_SURVIVE, 0.0);
        } else {
            atomicAdd(&S.wsum[W_LOSS], q.w);
            atomicAdd(&S.cnt[C_RR_KILL], 1ull);
            q.alive = false;
            trace_rec(A, C.hist(), q, EV_RR_KILL, 0.0);
        }
    }
}

// Source particle of the context's history: position, birth time, direction,
// group, unit weight, cell; leaks at once when born on the outer boundary
// moving out.
template <class Ctx>
MCDC_DEV void stage_source(CP &P, const RunArgs &A, Shared &S, Ctx &C, Part &q) {
    q.tag = 0;
    q.k = 0;
    q.seq = 0;
    Rng r = make_rng(A.seed, C.hist(), P.problem_id, 0u, 0u);
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
        trace_rec(A, C.hist(), q, EV_TIME_END, 0.0);
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!axis_in(P.outer_lo[a], P.outer_hi[a], q.x[a], q.u[a])) {
            leak(S, q, 2 * a + (q.x[a] >= P.outer_hi[a] ? 1 : 0));
            trace_rec(A, C.hist(), q, EV_LEAK, 0.0);
            return;
        }
    }
    trace_rec(A, C.hist(), q, EV_SOURCE, 0.0);
}

// Source particle of a k-eigenvalue generation after the first: born at
// fission site j of the combed source (its position and group) at t = 0 with
// unit weight and an isotropic direction from the history's own stream; then
// the same checks as the problem's source.
template <class Ctx>
MCDC_DEV void stage_source_site(CP &P, const RunArgs &A, Shared &S, Ctx &C, Part &q, uint64_t j) {
    q.tag = 0;
    q.k = 0;
    q.seq = 0;
    Rng r = make_rng(A.seed, C.hist(), P.problem_id, 0u, 0u);
    q.x[0] = A.src_d[j];
    q.x[1] = A.src_d[A.gen_m + j];
    q.x[2] = A.src_d[2 * A.gen_m + j];
    q.t = 0.0;
    iso_direction(r, q.u[0], q.u[1], q.u[2]);
    q.g = A.src_g[j];
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
        trace_rec(A, C.hist(), q, EV_TIME_END, 0.0);
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!axis_in(P.outer_lo[a], P.outer_hi[a], q.x[a], q.u[a])) {
            leak(S, q, 2 * a + (q.x[a] >= P.outer_hi[a] ? 1 : 0));
            trace_rec(A, C.hist(), q, EV_LEAK, 0.0);
            return;
        }
    }
    trace_rec(A, C.hist(), q, EV_SOURCE, 0.0);
}

// Contexts that carry fission sites (the k-eigenvalue mode) declare kFis.
template <class C, class = void>
struct fis_ctx : std::false_type {};
template <class C>
struct fis_ctx<C, std::void_t<decltype(C::kFis)>> : std::integral_constant<bool, C::kFis> {};

// Contexts whose kernels sit at their register limit declare kTightRegs.
template <class C, class = void>
struct tight_regs : std::false_type {};
template <class C>
struct tight_regs<C, std::void_t<decltype(C::kTightRegs)>>
    : std::integral_constant<bool, C::kTightRegs> {};

// Flight: census, surface, weight-window grid plane (windows with a grid) and
// collision distances; the event (ties: census, then surface, then grid
// plane, then collision); track-length scoring; straight-line motion; census
// and end-of-time handling.  Returns EV_CENSUS (particle continues), EV_TIME_END or
// -1 (particle ended), EV_SURFACE or EV_SCATTER (the surface or collision
// stage comes next), EV_WW_PLANE (the window check comes next); `d` is the
// flight length.
template <class T, class Ctx>
MCDC_DEV int stage_flight(CP &P, const RunArgs &A, Shared &S, const T &tally, Ctx &C,
                          Part &q, double &d, uint32_t &n_piece, double &path) {
    if (!C.count_flight()) {
        set_status(A, MCDC_E_EVENT_CAP);
        q.alive = false;
        return -1;
    }
    C.imp_point(P, q);
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
    Rng r = make_rng(A.seed, C.hist(), P.problem_id, q.tag, q.k);
    if (sig_t > 0.0) {
        const double xi = rng_uniform(r);
        d_c = (-own_log(xi)) / sig_t;
    }
    q.k = r.k;

    // weight-window grid plane (windows with a grid only)
    int wax = -1;
    double wpl = 0.0, d_w = kInf;
    if (Ctx::kWW && P.ww_grid_on) d_w = dist_ww_plane(P, q.x, q.u, iu, wax, wpl);

    // ties: census, surface, grid plane, collision
    int ev;
    if (d_t <= d_s && d_t <= d_w && d_t <= d_c) { ev = EV_CENSUS; d = d_t; }
    else if (d_s <= d_w && d_s <= d_c) { ev = EV_SURFACE; d = d_s; }
    else if (wax >= 0 && d_w <= d_c) { ev = EV_WW_PLANE; d = d_w; }
    else { ev = EV_SCATTER; d = d_c; }

    // the weight-window kernels and those that declare tight registers
    // recompute the walk's crossing steps
    n_piece += score_mesh<!Ctx::kWW && !tight_regs<Ctx>::value>(P, q.x, q.u, iu, q.t, v, d, q.w,
                                                                 q.g, tally);
    if (P.has_detector) {
        const double l = detector_len(P, q.x, q.u, iu, d);
        if (l > 0.0) C.add_score(q.w * l);
    }
    const double wd = q.w * d;
    path += wd;
    C.add_path(wd);
    if (P.surf_on && score_surface(P, q.x, q.u, iu, q.t, v, d, q.w, q.g, C.surf_tally()))
        atomicAdd(&S.cnt[C_SURF], 1ull);

    // straight-line motion: each coordinate by its direction cosine times d;
    // the time by d / v below, unless the flight ends at a census
#pragma unroll
    for (int a = 0; a < 3; ++a) q.x[a] += q.u[a] * d;

    if (ev == EV_CENSUS) {
        q.t = tc;
        if (q.ci == P.n_census - 1) {
            atomicAdd(&S.wsum[W_TIME_END], q.w);
            atomicAdd(&S.cnt[C_TIME_END], 1ull);
            q.alive = false;
            trace_rec(A, C.hist(), q, EV_TIME_END, d);
            return EV_TIME_END;
        }
        q.ci += 1;
        atomicAdd(&S.cnt[C_CENSUS], 1ull);
        trace_rec(A, C.hist(), q, EV_CENSUS, d);
        return EV_CENSUS;
    }
    q.t = q.t + d / v;
    if (Ctx::kWW && ev == EV_WW_PLANE) {
        // on the plane exactly (select, no dynamic index); the window check
        // comes next
        if (wax == 0) q.x[0] = wpl;
        else if (wax == 1) q.x[1] = wpl;
        else q.x[2] = wpl;
        atomicAdd(&S.cnt[C_WW_PLANE], 1ull);
        trace_rec(A, C.hist(), q, EV_WW_PLANE, d);
        return EV_WW_PLANE;
    }
    if (ev == EV_SURFACE) {
        // snap the crossing coordinate onto the plane (select, no dynamic index)
        if (sax == 0) q.x[0] = spl;
        else if (sax == 1) q.x[1] = spl;
        else if (sax == 2) q.x[2] = spl;
    }
    return ev;
}

// Surface crossing: outer boundary (leak / reflect), new cell.  Returns true
// when a weight-window check is due (the caller runs ww_check before the
// particle moves again, possibly batched with other lanes).
template <class Ctx>
MCDC_DEV bool stage_surface(CP &P, const RunArgs &A, Shared &S, Ctx &C, Part &q,
                            double d) {
    atomicAdd(&S.cnt[C_SURFACE], 1ull);
    const int face = boundary(P, q);
    if (face >= 0) {
        leak(S, q, face);
        trace_rec(A, C.hist(), q, EV_LEAK, d);
        return false;
    }
    q.cell = locate(P, q.x, q.u);
    trace_rec(A, C.hist(), q, EV_SURFACE, d);
    return Ctx::kWW && P.ww_on;
}

// Collision: analog absorption or implicit capture with weight cutoff, then
// the outgoing group (cumulative row) and an isotropic direction.  Returns
// true when a weight-window check is due.
template <class Ctx>
MCDC_DEV bool stage_collision(CP &P, const RunArgs &A, Shared &S, Ctx &C, Part &q,
                              double d) {
    atomicAdd(&S.cnt[C_COLLISION], 1ull);
    const int mat = q.cell >= 0 ? P.box_mat[q.cell] : P.background_mat;
    const double sig_t = P.sigma_t[mat * P.G + q.g];
    if (P.col_on) {                      // collision estimator: w / Sigma_t at the point
        const int64_t b = mesh_point_bin(P, q.x, q.t, q.g);
        if (b >= 0) unsafeAtomicAdd(C.col_tally() + b, q.w / sig_t);
    }
    const double *ss_row = P.sigma_s + (mat * P.G + q.g) * P.G;
    double sig_s = 0.0;
    for (int h = 0; h < P.G; ++h) sig_s = sig_s + ss_row[h];
    Rng r = make_rng(A.seed, C.hist(), P.problem_id, q.tag, q.k);
    if constexpr (fis_ctx<Ctx>::value) {
        // k-eigenvalue mode: w nuSigma_f / Sigma_t is this collision's
        // expected fission neutrons (its collision estimate of k); divided by
        // the generation's k_norm it is the expected number of sites, made as
        // floor(. + xi) sites (one draw) at the collision point, each with an
        // outgoing group from the material's spectrum (first g' with xi times
        // the spectrum's sum below the ascending cumulative spectrum; one draw
        // per site when G > 1).  Fission is part of the absorption: the
        // collision then goes on as in the fixed-source mode.
        const double nusf = P.nu_sigma_f[mat * P.G + q.g];
        if (nusf > 0.0) {
            const double prod = q.w * nusf / sig_t;
            atomicAdd(&S.kcol, prod);
            const double xi = rng_uniform(r);
            const double nf = floor(prod / C.k_norm + xi);
            // more sites than the whole bank holds (a normalisation far below
            // k, or none after a failed generation) fail the generation at
            // once rather than looping over sites that cannot be kept
            uint32_t n = 0;
            if (nf <= (double)A.site_cap) n = (uint32_t)nf;
            else set_status(A, MCDC_E_BANK);
            const double *chi = P.chi + mat * P.G;
            double chi_sum = 0.0;
            for (int h = 0; h < P.G; ++h) chi_sum = chi_sum + chi[h];
            uint32_t pos = wave_reserve_n(A.site_n, n);
            for (uint32_t i = 0; i < n; ++i, ++pos) {
                int gs = 0;
                if (P.G > 1) {
                    const double target = rng_uniform(r) * chi_sum;
                    double cum = 0.0;
                    int gn = -1, last = 0;
                    for (int h = 0; h < P.G; ++h) {
                        cum = cum + chi[h];
                        if (chi[h] > 0.0) last = h;
                        if (gn < 0 && target < cum) gn = h;
                    }
                    gs = gn >= 0 ? gn : last;
                }
                C.put_site(q, gs, pos);
            }
            q.k = r.k;
            if (n > 0) trace_rec(A, C.hist(), q, EV_FISSION, (double)n);
        }
    }
    if (!P.implicit_capture) {
        const double xi = rng_uniform(r);
        q.k = r.k;
        if (!(xi * sig_t < sig_s)) {
            atomicAdd(&S.wsum[W_ABSORB], q.w);
            atomicAdd(&S.cnt[C_ABSORB], 1ull);
            q.alive = false;
            trace_rec(A, C.hist(), q, EV_ABSORB, d);
            return false;
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
                trace_rec(A, C.hist(), q, EV_CUT_KILL, d);
                return false;
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
    trace_rec(A, C.hist(), q, EV_SCATTER, d);
    return Ctx::kWW && P.ww_on;
}

}  // namespace mcdc
