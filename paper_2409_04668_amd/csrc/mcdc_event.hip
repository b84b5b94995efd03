// Event-based schedule: particles live in an SoA bank in HBM and are moved
// through the transport loop one event class at a time, each class a launch
// over a compacted queue of bank indices:
//   flight    (all live particles)  -> surface queue | collision queue |
//                                        census queue | ended
//   interact  (surface + collision queues, one launch) -> next active
//             queue | ended; its last workgroup advances the queue roles
// Queues are appended with one atomic per wavefront: __ballot of the
// predicate, popcount for the wave's total, mbcnt for each lane's offset.
// When the active queue drains, the census queue becomes the active queue
// (the next census step); when both are empty the chunk of histories is done.
// Queue roles live in device memory, so every launch of an iteration has fixed
// arguments (graph-capturable); kernels with an empty input queue exit at once.
#include "mcdc_runtime.hpp"
#include "transport_stages.hpp"

namespace mcdc {

enum { Q_A = 0, Q_B = 1, Q_C = 2 };     // three physical active/census buffers

struct EvCtl {
    uint32_t n_act[3];                   // entries in the three active/census buffers
    uint32_t n_surf, n_coll;
    uint32_t cur, nxt, cen;              // roles: current active, next active, census
    uint32_t bank_n;                     // bank entries in use
    uint32_t done;
    uint32_t blocks_done;                // completion count of the interaction launch
    uint32_t pad[5];
};

struct EvBank {
    double *d;                           // [9][cap]: x y z ux uy uz t w dist
    uint32_t *i;                         // [7][cap]: g cell ci tag k seq slot
    uint32_t *q;                         // [3][cap] active/census queues
    uint32_t *qs, *qc;                   // [cap] surface, collision queues
    double *xh, *path;                   // [chunk] per-history
    uint32_t *events;                    // [chunk]
    EvCtl *ctl;
    uint32_t cap, chunk;
};

}  // namespace mcdc

namespace mcdc {

struct EventState {
    EvBank B;
    uint32_t *host_done;                 // pinned
    int grid, block;
};

MCDC_DEV void bank_load(const EvBank &B, uint32_t j, Part &q, double &d, uint32_t &slot) {
    const size_t c = B.cap;
    q.x[0] = B.d[0 * c + j]; q.x[1] = B.d[1 * c + j]; q.x[2] = B.d[2 * c + j];
    q.u[0] = B.d[3 * c + j]; q.u[1] = B.d[4 * c + j]; q.u[2] = B.d[5 * c + j];
    q.t = B.d[6 * c + j]; q.w = B.d[7 * c + j]; d = B.d[8 * c + j];
    q.g = (int32_t)B.i[0 * c + j]; q.cell = (int32_t)B.i[1 * c + j]; q.ci = (int32_t)B.i[2 * c + j];
    q.tag = B.i[3 * c + j]; q.k = B.i[4 * c + j]; q.seq = B.i[5 * c + j]; slot = B.i[6 * c + j];
    q.alive = true;
}

MCDC_DEV void bank_store(const EvBank &B, uint32_t j, const Part &q, double d, uint32_t slot) {
    const size_t c = B.cap;
    B.d[0 * c + j] = q.x[0]; B.d[1 * c + j] = q.x[1]; B.d[2 * c + j] = q.x[2];
    B.d[3 * c + j] = q.u[0]; B.d[4 * c + j] = q.u[1]; B.d[5 * c + j] = q.u[2];
    B.d[6 * c + j] = q.t; B.d[7 * c + j] = q.w; B.d[8 * c + j] = d;
    B.i[0 * c + j] = (uint32_t)q.g; B.i[1 * c + j] = (uint32_t)q.cell; B.i[2 * c + j] = (uint32_t)q.ci;
    B.i[3 * c + j] = q.tag; B.i[4 * c + j] = q.k; B.i[5 * c + j] = q.seq; B.i[6 * c + j] = slot;
}

// Wavefront-aggregated append: one atomic per wave on the queue tail.
MCDC_DEV void wave_append(uint32_t *queue, uint32_t *count, uint32_t value, bool pred) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return;
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (pred) {
        const uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        queue[base + off] = value;
    }
}

// Per-history context of a banked particle.
template <int WW>
struct EvCtx {
    static constexpr bool kWW = WW != 0;
    static constexpr bool kWWMap = WW == 2;
    const DevProblem &P;
    const RunArgs &A;
    const EvBank &B;
    uint32_t slot;
    MCDC_DEV uint64_t hist() const { return A.h_begin + slot; }
    // batch b of the history (run-relative id r) holds ids
    // [floor(b n / B), floor((b+1) n / B)): b = floor(((r+1) B - 1) / n)
    MCDC_DEV uint64_t batch() const {
        const uint64_t r = A.h_begin + slot - A.h_run0;
        return ((r + 1) * A.run_batches - 1) / A.run_n;
    }
    MCDC_DEV double *col_tally() const { return A.col + batch() * (uint64_t)P.nbins; }
    MCDC_DEV const float *mlp_params(const DevProblem &Pp) const { return Pp.ww_params; }
    MCDC_DEV bool count_flight() {
        uint32_t e;
        if (WW) e = atomicAdd(&B.events[slot], 1u) + 1u;
        else e = (B.events[slot] += 1u);
        return (int64_t)e <= P.max_events;
    }
    MCDC_DEV void add_score(double v) {
        if (WW) unsafeAtomicAdd(&B.xh[slot], v);
        else B.xh[slot] += v;
    }
    MCDC_DEV void add_path(double v) {
        if (!A.xh_out) return;           // the per-history path is an output only
        if (WW) unsafeAtomicAdd(&B.path[slot], v);
        else B.path[slot] += v;
    }
    MCDC_DEV void imp_point(const DevProblem &, const Part &) {}
    // daughters are only recorded here: the interaction kernel allocates
    // bank entries and queue places for a whole wave at once
    uint32_t split_n = 0, split_tag0 = 0;
    MCDC_DEV bool push_daughters(const Part &, uint32_t tag0, int n) {
        split_n = (uint32_t)n;
        split_tag0 = tag0;
        return true;
    }
};

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active).
MCDC_DEV uint32_t wave_scan_incl(uint32_t x) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Write the recorded daughters of every lane of the wave: one atomic per wave
// on the bank size and one on the next active queue, then each lane writes
// its n-1 daughters (the parent state with tag0 + i * golden, k = seq = 0)
// at its offset.  Entries past the bank capacity are dropped with an error.
MCDC_DEV void wave_write_daughters(const RunArgs &A, const EvBank &B, const Part &q, uint32_t slot,
                                   uint32_t nd, uint32_t tag0) {
    const uint32_t incl = wave_scan_incl(nd);
    const uint32_t total = __shfl(incl, 63);
    if (total == 0) return;
    const int lane = (int)__lane_id();
    const uint32_t nx = B.ctl->nxt;
    uint32_t jb = 0, qb = 0;
    if (lane == 0) {
        jb = atomicAdd(&B.ctl->bank_n, total);
        qb = atomicAdd(&B.ctl->n_act[nx], total);
    }
    jb = __shfl(jb, 0);
    qb = __shfl(qb, 0);
    const uint32_t off = incl - nd;
    for (uint32_t i = 0; i < nd; ++i) {
        const uint64_t j = (uint64_t)jb + off + i;
        if (j >= B.cap) {
            set_status(A, MCDC_E_BANK);
            break;
        }
        Part d = q;
        d.tag = tag0 + (i + 1u) * 0x9E3779B9u;
        d.k = 0;
        d.seq = 0;
        bank_store(B, (uint32_t)j, d, 0.0, slot);
        B.q[(size_t)nx * B.cap + qb + off + i] = (uint32_t)j;
    }
}

template <bool WW>
__global__ void __launch_bounds__(256) k_ev_source(DevProblem P, RunArgs A, EvBank B, uint32_t n) {
    __shared__ Shared S;
    shared_zero(S);
    __syncthreads();
    const uint32_t cur = B.ctl->cur;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s - threadIdx.x < n;
         s += gridDim.x * blockDim.x) {
        const bool valid = s < n;
        bool alive = false;
        if (valid) {
            B.xh[s] = 0.0;
            B.path[s] = 0.0;
            B.events[s] = 0u;
            EvCtx<WW> C{P, A, B, s};
            Part q;
            stage_source(P, A, S, C, q);
            alive = q.alive;
            if (alive) bank_store(B, s, q, 0.0, s);
        }
        wave_append(B.q + (size_t)cur * B.cap, &B.ctl->n_act[cur], s, valid && alive);
    }
    __syncthreads();
    shared_flush(S, A.acc);
}

template <bool WW>
__global__ void __launch_bounds__(256) k_ev_flight(DevProblem P, RunArgs A, EvBank B) {
    __shared__ Shared S;
    shared_zero(S);
    __syncthreads();
    const uint32_t cur = B.ctl->cur, cen = B.ctl->cen;
    const uint32_t n = B.ctl->n_act[cur];
    const uint32_t *in = B.q + (size_t)cur * B.cap;
    uint32_t n_piece = 0, n_flight = 0;
    double path = 0.0;
    for (uint32_t j0 = blockIdx.x * blockDim.x; j0 < n; j0 += gridDim.x * blockDim.x) {
        const uint32_t jj = j0 + threadIdx.x;
        const bool valid = jj < n;
        int ev = -1;
        uint32_t j = 0;
        if (valid) {
            j = in[jj];
            Part q;
            double d;
            uint32_t slot;
            bank_load(B, j, q, d, slot);
            EvCtx<WW> C{P, A, B, slot};
            GlobalTally tally{A.tally + C.batch() * (uint64_t)P.nbins};
            ev = stage_flight(P, A, S, tally, C, q, d, n_piece, path);
            if (ev >= 0) n_flight += 1;
            if (q.alive) bank_store(B, j, q, d, slot);
            else ev = -1;
        }
        wave_append(B.qs, &B.ctl->n_surf, j, ev == EV_SURFACE);
        wave_append(B.qc, &B.ctl->n_coll, j, ev == EV_SCATTER);
        wave_append(B.q + (size_t)cen * B.cap, &B.ctl->n_act[cen], j, ev == EV_CENSUS);
    }
    atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
    atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
    atomicAdd(&S.wsum[W_PATH], path);
    __syncthreads();
    shared_flush(S, A.acc);
}

// Queue roles for the next iteration.  Reads the counters with atomics so
// that the values other workgroups appended are seen.
MCDC_DEV void ev_advance(EvCtl *c) {
    const uint32_t cur = c->cur, nxt = c->nxt, cen = c->cen;
    const uint32_t n_nxt = atomicAdd(&c->n_act[nxt], 0u);
    const uint32_t n_cen = atomicAdd(&c->n_act[cen], 0u);
    c->n_act[cur] = 0;
    c->n_surf = 0;
    c->n_coll = 0;
    if (n_nxt > 0) {
        c->cur = nxt;
        c->nxt = cur;
    } else if (n_cen > 0) {                  // next census step
        c->cur = cen;
        c->cen = nxt;
        c->nxt = cur;
    } else {
        c->done = 1;
    }
}

// Surface and collision stages in one launch: entries [0, n_surf) of the
// combined range come from the surface queue, the rest from the collision
// queue.  The last workgroup to finish advances the queue roles.  WW: 0 none,
// 1 network at each check, 2 baked window map.
template <int WW>
__global__ void __launch_bounds__(256) k_ev_interact(DevProblem P, RunArgs A, EvBank B) {
    __shared__ Shared S;
    __shared__ bool s_last;
    shared_zero(S);
    __syncthreads();
    const uint32_t nxt = B.ctl->nxt;
    const uint32_t ns = B.ctl->n_surf, nc = B.ctl->n_coll;
    const uint32_t n = ns + nc;
    for (uint32_t j0 = blockIdx.x * blockDim.x; j0 < n; j0 += gridDim.x * blockDim.x) {
        const uint32_t jj = j0 + threadIdx.x;
        const bool valid = jj < n;
        bool alive = false;
        uint32_t j = 0;
        uint32_t nd = 0, tag0 = 0, dslot = 0;     // recorded daughters of this lane
        Part dq;
        if (valid) {
            const bool surf = jj < ns;
            j = surf ? B.qs[jj] : B.qc[jj - ns];
            Part q;
            double d;
            uint32_t slot;
            bank_load(B, j, q, d, slot);
            EvCtx<WW> C{P, A, B, slot};
            const bool due = surf ? stage_surface(P, A, S, C, q, d) : stage_collision(P, A, S, C, q, d);
            if (WW != 0 && due) ww_check(P, A, S, C, q);
            alive = q.alive;
            if (alive) bank_store(B, j, q, d, slot);
            if (WW != 0 && C.split_n > 1) {
                nd = C.split_n - 1;
                tag0 = C.split_tag0;
                dq = q;
                dslot = slot;
            }
        }
        if (WW != 0) wave_write_daughters(A, B, dq, dslot, nd, tag0);
        wave_append(B.q + (size_t)nxt * B.cap, &B.ctl->n_act[nxt], j, valid && alive);
    }
    __syncthreads();
    shared_flush(S, A.acc);
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&B.ctl->blocks_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        ev_advance(B.ctl);
        B.ctl->blocks_done = 0;
    }
}

// End of a chunk: per-history detector statistics and optional outputs.
__global__ void __launch_bounds__(256) k_ev_finish(RunArgs A, EvBank B, uint32_t n) {
    __shared__ unsigned long long hits;
    if (threadIdx.x == 0) hits = 0;
    __syncthreads();
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        const double xh = B.xh[s];
        if (xh != 0.0) {
            unsafeAtomicAdd(&A.acc->det[0], xh);
            unsafeAtomicAdd(&A.acc->det[1], xh * xh);
        }
        if (xh > 0.0) atomicAdd(&hits, 1ull);
        if (A.xh_out) {
            const uint64_t o = A.h_begin + s - A.h_run0;
            A.xh_out[2 * o] = xh;
            A.xh_out[2 * o + 1] = B.path[s];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (hits) atomicAdd(&A.acc->cnt[C_DET_HIT], hits);
    }
}

__global__ void k_ev_reset(EvBank B, uint32_t n_hist) {
    EvCtl *c = B.ctl;
    for (int i = 0; i < 3; ++i) c->n_act[i] = 0;
    c->n_surf = c->n_coll = 0;
    c->cur = Q_A;
    c->nxt = Q_B;
    c->cen = Q_C;
    c->bank_n = n_hist;
    c->done = 0;
    c->blocks_done = 0;
}

__global__ void k_ev_count_hist(DevAcc *acc, uint64_t n) { atomicAdd(&acc->cnt[C_HIST], (unsigned long long)n); }

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static uint32_t ev_chunk(const mcdc_problem_desc *d, const Options &o) {
    int64_t c = o.event_chunk > 0 ? o.event_chunk : (1 << 22);
    if (c > (1 << 26)) c = 1 << 26;
    (void)d;
    return (uint32_t)c;
}

static uint32_t ev_cap(const mcdc_problem_desc *d, const Options &o) {
    const uint64_t chunk = ev_chunk(d, o);
    const uint64_t f = d->stack_cap > 0 ? 4 : 1;
    uint64_t cap = chunk * f;
    if (cap > 0xF0000000ull) cap = 0xF0000000ull;
    return (uint32_t)cap;
}

size_t event_workspace_bytes(const mcdc_problem_desc *d, const Options &o) {
    if (o.schedule != MCDC_SCHED_EVENT) return 0;
    const size_t cap = ev_cap(d, o), chunk = ev_chunk(d, o);
    size_t b = al(9 * cap * sizeof(double)) + al(7 * cap * sizeof(uint32_t)) +
               al(3 * cap * sizeof(uint32_t)) + 2 * al(cap * sizeof(uint32_t)) +
               2 * al(chunk * sizeof(double)) + al(chunk * sizeof(uint32_t)) + al(sizeof(EvCtl));
    return b;
}

int event_init(mcdc_problem *h) {
    if (h->desc.imp_on) return fail(MCDC_E_INVALID, "the importance estimate runs in the history schedule only");
    auto *E = new EventState();
    const size_t cap = ev_cap(&h->desc, h->opt), chunk = ev_chunk(&h->desc, h->opt);
    char *p = h->ws + h->L.event;
    EvBank &B = E->B;
    B.cap = (uint32_t)cap;
    B.chunk = (uint32_t)chunk;
    B.d = (double *)p; p += al(9 * cap * sizeof(double));
    B.i = (uint32_t *)p; p += al(7 * cap * sizeof(uint32_t));
    B.q = (uint32_t *)p; p += al(3 * cap * sizeof(uint32_t));
    B.qs = (uint32_t *)p; p += al(cap * sizeof(uint32_t));
    B.qc = (uint32_t *)p; p += al(cap * sizeof(uint32_t));
    B.xh = (double *)p; p += al(chunk * sizeof(double));
    B.path = (double *)p; p += al(chunk * sizeof(double));
    B.events = (uint32_t *)p; p += al(chunk * sizeof(uint32_t));
    B.ctl = (EvCtl *)p;
    hipError_t e = hipHostMalloc((void **)&E->host_done, sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete E;
        return hip_fail(e, "event_init");
    }
    E->block = 256;
    E->grid = history_grid(256, 16);
    h->ev = E;
    return MCDC_OK;
}

void event_destroy(mcdc_problem *h) {
    if (!h->ev) return;
    if (h->ev->host_done) (void)hipHostFree(h->ev->host_done);
    delete h->ev;
    h->ev = nullptr;
}

// Transport histories [A.h_begin, A.h_end) chunk by chunk.
int event_run_range(mcdc_problem *h, const RunArgs &A0, hipStream_t s) {
    EventState *E = h->ev;
    if (!E) return fail(MCDC_E_STATE, "event schedule not initialised");
    const DevProblem &P = h->P;
    const EvBank &B = E->B;
    const int grid = E->grid, block = E->block;
    for (uint64_t c0 = A0.h_begin; c0 < A0.h_end; c0 += B.chunk) {
        const uint64_t c1 = c0 + B.chunk < A0.h_end ? c0 + B.chunk : A0.h_end;
        const uint32_t n = (uint32_t)(c1 - c0);
        RunArgs A = A0;
        A.h_begin = c0;
        A.h_end = c1;
        hipLaunchKernelGGL(k_ev_reset, dim3(1), dim3(1), 0, s, B, n);
        hipLaunchKernelGGL(k_ev_count_hist, dim3(1), dim3(1), 0, s, A.acc, (uint64_t)n);
        int sg = (int)((n + block - 1) / block);
        if (sg > grid) sg = grid;
        const bool ww = P.ww_on != 0;
        if (ww) hipLaunchKernelGGL((k_ev_source<true>), dim3(sg), dim3(block), 0, s, P, A, B, n);
        else hipLaunchKernelGGL((k_ev_source<false>), dim3(sg), dim3(block), 0, s, P, A, B, n);
        for (int iter = 0;; ++iter) {
            const int K = 8;
            h->event_iterations += K;
            for (int k = 0; k < K; ++k) {
                timing_begin(h, s);
                if (ww) hipLaunchKernelGGL((k_ev_flight<true>), dim3(grid), dim3(block), 0, s, P, A, B);
                else hipLaunchKernelGGL((k_ev_flight<false>), dim3(grid), dim3(block), 0, s, P, A, B);
                timing_end(h, s);
                if (!ww) hipLaunchKernelGGL((k_ev_interact<0>), dim3(grid), dim3(block), 0, s, P, A, B);
                else if (P.ww_map) hipLaunchKernelGGL((k_ev_interact<2>), dim3(grid), dim3(block), 0, s, P, A, B);
                else hipLaunchKernelGGL((k_ev_interact<1>), dim3(grid), dim3(block), 0, s, P, A, B);
            }
            hipError_t e = hipMemcpyAsync(E->host_done, &B.ctl->done, sizeof(uint32_t),
                                          hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "event loop");
            if (*E->host_done) break;
            if (iter > 1000000) return fail(MCDC_E_EVENT_CAP, "event loop did not drain");
        }
        const int fg = (int)((n + block - 1) / block) < grid ? (int)((n + block - 1) / block) : grid;
        hipLaunchKernelGGL(k_ev_finish, dim3(fg), dim3(block), 0, s, A, B, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "event launch");
    }
    return MCDC_OK;
}

}  // namespace mcdc
