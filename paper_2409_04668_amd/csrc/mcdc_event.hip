// Event-based schedule: particles live in SoA banks in HBM and are moved
// through the transport loop one event class at a time.  A stage reads its
// input bank contiguously and copies every particle it keeps into the bank of
// the next stage at a wave-reserved position, so reads and writes are
// coalesced and no index queues are gathered through:
//   flight    (active bank)      -> interaction bank (surface entries from the
//                                   front, collision entries from the back) |
//                                   census bank | ended
//   interact  (interaction bank) -> next active bank (+ split daughters) |
//                                   ended; its last workgroup advances the
//                                   bank roles
//   control   (census bank, only with population control at census)
//                                -> next active bank
// Positions come from one atomic per wavefront: __ballot of the predicate,
// popcount for the wave's total, mbcnt for each lane's offset.  When the
// active bank drains, the census bank becomes the active bank (the next census
// step); when both are empty the chunk of histories is done.  Bank roles and
// counts live in device memory, so every launch of an iteration has fixed
// arguments; a kernel whose input is empty exits at once.
//
// Hybrid schedule: a lead stage replaces the source stage.  One work-item
// follows each history in registers, as the history schedule does, with its
// split daughters on a per-work-item stack, until the history ends or has
// taken MCDC_LEAD_FLIGHTS flights (or, with population control or
// census-step control, a particle reaches a census); what is left then goes
// to the banks.  In place of the flight and interaction stages, a re-lead
// stage then runs the same loop over the banked particles, MCDC_RELEAD_FLIGHTS
// flights each before what is left is banked again, until the banks are
// empty.  Short histories never touch the banks; long split chains, which
// would serialise on one work-item, are spread over the grid.
#include "lane_stack.hpp"
#include "mcdc_runtime.hpp"
#include "transport_stages.hpp"

namespace mcdc {

// One bank: 9 FP64 fields (x y z ux uy uz t w dist) and 7 u32 fields
// (g cell ci tag k seq slot), `cap` entries each.
struct Bank {
    double *d;
    uint32_t *i;
};

enum { R_A = 0, R_B = 1, R_C = 2, R_X = 3 };   // three role banks, interaction bank
constexpr uint32_t kPlaneMark = 0x80000000u;     // interaction entry: a grid-plane stop

struct EvCtl {
    uint32_t n_act[3];                   // particles in the three role banks
    uint32_t n_surf, n_coll;             // interaction bank: [0, n_surf), [cap - n_coll, cap)
    uint32_t cur, nxt, cen;              // roles: current active, next active, census
    uint32_t done;
    uint32_t paused;                     // a census step began; launches are no-ops
                                         // (read by the host together with `done`)
    uint32_t blocks_done;                // last-workgroup hand-over within a launch
    uint32_t pc_stage;                   // population control: 0 idle, 1 sum, 2 apply
    unsigned long long pc_wq;            // census-bank weight in units of 2^-32
    uint32_t pause_at_census;            // census-step control: stop at the next census step
};
static_assert(offsetof(EvCtl, paused) == offsetof(EvCtl, done) + sizeof(uint32_t),
              "the host reads done and paused as one pair");

struct EvBank {
    Bank b[4];
    double *xh, *path;                   // [chunk] per-history
    uint32_t *events;                    // [chunk]
    EvCtl *ctl;
    uint32_t cap, chunk;
};

struct EventState {
    EvBank B;
    uint32_t *host_done;                 // pinned: done, paused
    int grid, block;
};

MCDC_DEV void bank_load(const Bank &K, size_t c, uint32_t j, Part &q, double &d, uint32_t &slot) {
    q.x[0] = K.d[0 * c + j]; q.x[1] = K.d[1 * c + j]; q.x[2] = K.d[2 * c + j];
    q.u[0] = K.d[3 * c + j]; q.u[1] = K.d[4 * c + j]; q.u[2] = K.d[5 * c + j];
    q.t = K.d[6 * c + j]; q.w = K.d[7 * c + j]; d = K.d[8 * c + j];
    q.g = (int32_t)K.i[0 * c + j]; q.cell = (int32_t)K.i[1 * c + j]; q.ci = (int32_t)K.i[2 * c + j];
    q.tag = K.i[3 * c + j]; q.k = K.i[4 * c + j]; q.seq = K.i[5 * c + j]; slot = K.i[6 * c + j];
    q.alive = true;
}

MCDC_DEV void bank_store(const Bank &K, size_t c, uint32_t j, const Part &q, double d, uint32_t slot) {
    K.d[0 * c + j] = q.x[0]; K.d[1 * c + j] = q.x[1]; K.d[2 * c + j] = q.x[2];
    K.d[3 * c + j] = q.u[0]; K.d[4 * c + j] = q.u[1]; K.d[5 * c + j] = q.u[2];
    K.d[6 * c + j] = q.t; K.d[7 * c + j] = q.w; K.d[8 * c + j] = d;
    K.i[0 * c + j] = (uint32_t)q.g; K.i[1 * c + j] = (uint32_t)q.cell; K.i[2 * c + j] = (uint32_t)q.ci;
    K.i[3 * c + j] = q.tag; K.i[4 * c + j] = q.k; K.i[5 * c + j] = q.seq; K.i[6 * c + j] = slot;
}

// Wavefront-aggregated reservation: the lanes with `pred` get consecutive
// positions from one atomic per wave on *count; returns the lane's position.
MCDC_DEV uint32_t wave_reserve(uint32_t *count, bool pred) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return 0;
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    return base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

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

// Copy a particle into bank K at a reserved position; past the capacity the
// particle is dropped and the run reports a bank overflow.
MCDC_DEV void bank_put(const RunArgs &A, const EvBank &B, const Bank &K, uint32_t pos, const Part &q,
                       double d, uint32_t slot) {
    if (pos >= B.cap) {
        set_status(A, MCDC_E_BANK);
        return;
    }
    bank_store(K, B.cap, pos, q, d, slot);
}

// Write the recorded copies of every lane of the wave into bank K: one atomic
// per wave on *count, then each lane writes its nd copies (the parent state
// with tag tag0 + i * golden, i = 1..nd, counter and sequence 0).
MCDC_DEV void wave_write_copies(const RunArgs &A, const EvBank &B, const Bank &K, uint32_t *count,
                                const Part &q, uint32_t slot, uint32_t nd, uint32_t tag0) {
    const uint32_t incl = wave_scan_incl(nd);
    const uint32_t total = __shfl(incl, 63);
    if (total == 0) return;
    uint32_t base = 0;
    if (__lane_id() == 0) base = atomicAdd(count, total);
    base = __shfl(base, 0);
    const uint32_t off = incl - nd;
    for (uint32_t i = 0; i < nd; ++i) {
        const uint64_t j = (uint64_t)base + off + i;
        if (j >= B.cap) {
            set_status(A, MCDC_E_BANK);
            break;
        }
        Part d = q;
        d.tag = tag0 + (i + 1u) * 0x9E3779B9u;
        d.k = 0;
        d.seq = 0;
        bank_store(K, B.cap, (uint32_t)j, d, 0.0, slot);
    }
}

// Per-history context of a banked particle.  WW: 0 no weight windows,
// 1 network at each check, 2 baked window map.
template <int WW>
struct EvCtx {
    static constexpr bool kWW = WW != 0;
    static constexpr bool kWWMap = WW == 2;
    CP &P;
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
    MCDC_DEV double *surf_tally() const { return A.surf + batch() * (uint64_t)P.surf_nbins; }
    MCDC_DEV const float *mlp_params(CP &Pp) const { return Pp.ww_params; }
    // several particles of one history can be in flight at once when they
    // split (weight windows, population control): their sums are atomic
    MCDC_DEV bool count_flight() {
        uint32_t e;
        if (WW || P.pc_on) e = atomicAdd(&B.events[slot], 1u) + 1u;
        else e = (B.events[slot] += 1u);
        return (int64_t)e <= P.max_events;
    }
    MCDC_DEV void add_score(double v) {
        if (WW || P.pc_on) unsafeAtomicAdd(&B.xh[slot], v);
        else B.xh[slot] += v;
    }
    MCDC_DEV void add_path(double v) {
        if (!A.keep_path) return;        // the per-history path is an output only
        if (WW || P.pc_on) unsafeAtomicAdd(&B.path[slot], v);
        else B.path[slot] += v;
    }
    MCDC_DEV void imp_point(CP &, const Part &) {}
    // split daughters are only recorded here: the interaction kernel writes
    // them for a whole wave at once
    uint32_t split_n = 0, split_tag0 = 0;
    MCDC_DEV bool push_daughters(const Part &, uint32_t tag0, int n) {
        split_n = (uint32_t)n;
        split_tag0 = tag0;
        return true;
    }
};

template <bool WW>
__global__ void __launch_bounds__(256) k_ev_source(DevProblem, RunArgs A, EvBank B, uint32_t n) {
    CP &P = kernel_problem();
    __shared__ Shared S;
    shared_zero(S);
    __syncthreads();
    const uint32_t cur = B.ctl->cur;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s - threadIdx.x < n;
         s += gridDim.x * blockDim.x) {
        const bool valid = s < n;
        bool alive = false;
        Part q;
        if (valid) {
            B.xh[s] = 0.0;
            B.path[s] = 0.0;
            B.events[s] = 0u;
            EvCtx<WW> C{P, A, B, s};
            stage_source(P, A, S, C, q);
            alive = q.alive;
        }
        const uint32_t pos = wave_reserve(&B.ctl->n_act[cur], valid && alive);
        if (valid && alive) bank_put(A, B, B.b[cur], pos, q, 0.0, s);
    }
    __syncthreads();
    shared_flush(S, A.acc);
}

// Lead-stage flights per history (its particles together) before the rest of
// the history is handed to the banks: short histories finish in the lead,
// long split chains are spread over the grid instead of holding one
// work-item.  The re-lead stage's budget counts the flights of one banked
// particle and its daughters.  Measured on the learned-window duct (lead /
// re-lead budget, histories/s with the window map and with the network at
// every check): 64/64 4.95e8 and 3.23e8, 32/16 5.37e8 and 3.86e8, 32/8
// 5.41e8 and 3.98e8, 16/8 5.33e8 and 3.97e8, 8/8 5.21e8 and 3.93e8.
#ifndef MCDC_LEAD_FLIGHTS
#define MCDC_LEAD_FLIGHTS 32
#endif
#ifndef MCDC_RELEAD_FLIGHTS
#define MCDC_RELEAD_FLIGHTS 8
#endif

// Context of a history in the lead stage: one work-item owns the history (its
// banked particles, if any, move only after the lead stage), so its sums stay
// in registers and are stored to the per-history arrays when the lead ends.
// In the re-lead stage (BANK) a work-item follows one banked particle of a
// history whose other particles may be in flight on other work-items, so the
// sums are atomic adds to the per-history arrays.  Split daughters go onto the
// work-item's stack while it has room, else into bank `cur` (the active bank
// after the lead stage; the next active bank in the re-lead stage).
template <int WW, bool BANK = false>
struct LeadCtx {
    static constexpr bool kWW = WW != 0;
    static constexpr bool kWWMap = WW == 2;
    CP &P;
    const RunArgs &A;
    const EvBank &B;
    uint64_t lane;
    uint32_t cur;
    uint32_t slot;
    double xh, path;
    // flights of the history: the lead stage's own count; in the re-lead
    // stage the history's count when the particle was taken (ev0) plus this
    // work-item's flights since, added to the per-history count when the
    // work-item moves on (so a flight does not wait on a returning atomic;
    // the event cap of a history split over several work-items can then
    // trigger a few flights late)
    uint32_t events;
    int sp;
    uint32_t ev0 = 0;
    MCDC_DEV uint64_t hist() const { return A.h_begin + slot; }
    MCDC_DEV uint64_t batch() const {
        const uint64_t r = A.h_begin + slot - A.h_run0;
        return ((r + 1) * A.run_batches - 1) / A.run_n;
    }
    MCDC_DEV double *col_tally() const { return A.col + batch() * (uint64_t)P.nbins; }
    MCDC_DEV double *surf_tally() const { return A.surf + batch() * (uint64_t)P.surf_nbins; }
    MCDC_DEV const float *mlp_params(CP &Pp) const { return Pp.ww_params; }
    MCDC_DEV bool count_flight() {
        events += 1u;
        return (int64_t)events <= P.max_events;
    }
    // re-lead stage: take over the history of bank slot s / hand back the
    // flights counted since
    MCDC_DEV void take(uint32_t s) {
        slot = s;
        ev0 = events = B.events[s];
    }
    MCDC_DEV void flush_events() const {
        if (events != ev0)
            __hip_atomic_fetch_add(&B.events[slot], events - ev0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    MCDC_DEV void add_score(double v) {
        if constexpr (BANK) unsafeAtomicAdd(&B.xh[slot], v);
        else xh += v;
    }
    MCDC_DEV void add_path(double v) {
        if (!A.keep_path) return;
        if constexpr (BANK) unsafeAtomicAdd(&B.path[slot], v);
        else path += v;
    }
    MCDC_DEV void imp_point(CP &, const Part &) {}
    // copy a particle ready for its next flight into bank `cur`
    MCDC_DEV void to_bank(const Part &q, uint32_t pos) const {
        bank_put(A, B, B.b[cur], pos, q, 0.0, slot);
    }
    // daughters i = 1..n-1 (tag tag0 + i * golden, counter and sequence 0)
    MCDC_DEV bool push_daughters(const Part &q, uint32_t tag0, int n) {
        const int room = P.stack_cap - sp;
        const int spill = n - 1 > room ? n - 1 - room : 0;
        // the lanes splitting together reserve their spills with one atomic
        uint32_t base = 0u;
        if (__ballot(spill != 0)) base = wave_reserve_n(&B.ctl->n_act[cur], (uint32_t)spill);
        for (int i = 1; i < n; ++i) {
            Part d = q;
            d.tag = tag0 + (uint32_t)i * 0x9E3779B9u;
            d.k = 0;
            d.seq = 0;
            if (i <= room) {
                stack_push(A, lane, P.stack_cap, sp, d);
                sp += 1;
            } else {
                to_bank(d, base + (uint32_t)(i - 1 - room));
            }
        }
        return true;
    }
};

// Tally target of the lead stage: HBM atomics into the history's batch slice,
// or (LDS == 2) a hot tile in LDS for the workgroup's batch with the rest of
// the mesh, and every other batch, in HBM.
template <int LDS>
struct LeadTally {
    GlobalTally t;
    MCDC_DEV void init(CP &, double *) {}
    MCDC_DEV void select(CP &P, const RunArgs &A, uint64_t b, uint64_t) {
        t.base = A.tally + b * (uint64_t)P.nbins;
    }
};
template <>
struct LeadTally<2> {
    HotTileTally t;
    MCDC_DEV void init(CP &P, double *lds) {
        t.lds = (lds_f64 *)lds;
        t.prob = &P;
        t.n0 = P.hot_n[0];
    }
    // the tile holds batch b_tile only: an empty x extent sends every update
    // of another batch to HBM
    MCDC_DEV void select(CP &P, const RunArgs &A, uint64_t b, uint64_t b_tile) {
        t.glob = (hbm_f64 *)(A.tally + b * (uint64_t)P.nbins);
        t.n0 = b == b_tile ? P.hot_n[0] : 0u;
    }
};

MCDC_DEV uint64_t batch_of(const RunArgs &A, uint32_t slot) {
    const uint64_t r = A.h_begin + slot - A.h_run0;
    return ((r + 1) * A.run_batches - 1) / A.run_n;
}

// Work-items per workgroup of the lead and re-lead stages.  With the hot
// tile, one workgroup per compute unit: 1024 work-items (16 waves, up to 128
// VGPRs), or 768 (12 waves, up to 168 VGPRs) when every window check
// evaluates the network: its values on top of the particle's spill at 128
// VGPRs, and the extra registers gain more than the four waves of latency
// hiding (7% on the duct's network-per-check run; the analog and window-map
// stages lose 14% and 3% at 768).
constexpr int kNetTileThreads = 768;
constexpr int tile_threads(int LDS, int WW) { return LDS != 2 ? 256 : WW == 1 ? kNetTileThreads : 1024; }

// One loop turn of the lead and re-lead stages for the live particle q: once
// `flights` reaches the budget, hand the particle and the stacked daughters
// over to bank C.cur; else one flight and the event that ends it.  A
// window-map check (WW 2) is made at once; a network check (WW 1) is
// returned as due, for the caller to run in a wave-level batch.
template <int WW, uint32_t BUDGET, class Ctx, class Tally>
MCDC_DEV bool lead_turn(CP &PL, const RunArgs &A, const EvBank &B, Shared &S, const Tally &tally,
                        Ctx &C, Part &q, uint32_t &flights, uint32_t &n_flight, uint32_t &n_piece,
                        double &path, bool stop_at_census, uint32_t cen) {
    if (WW != 0 && flights >= BUDGET) {
        // one atomic for the lanes of the wave that hand over together
        const uint32_t base = wave_reserve_n(&B.ctl->n_act[C.cur], (uint32_t)C.sp + 1u);
        C.to_bank(q, base);
        for (int i = 0; i < C.sp; ++i) {
            Part r;
            stack_pop(A, C.lane, PL.stack_cap, i, r);
            C.to_bank(r, base + 1u + (uint32_t)i);
        }
        C.sp = 0;
        q.alive = false;
        return false;
    }
    flights += 1;
    double d = 0.0;
    const int ev = stage_flight(PL, A, S, tally, C, q, d, n_piece, path);
    if (ev >= 0) n_flight += 1;
    if (!q.alive) {
        if (ev < 0) C.sp = 0;               // event cap: the history is abandoned
        return false;
    }
    bool due = false;
    if (ev == EV_SURFACE) {
        due = stage_surface(PL, A, S, C, q, d);
    } else if (ev == EV_SCATTER) {
        due = stage_collision(PL, A, S, C, q, d);
    } else if (ev == EV_WW_PLANE) {
        due = true;
    } else if (ev == EV_CENSUS && stop_at_census) {
        bank_put(A, B, B.b[cen], wave_reserve_one(&B.ctl->n_act[cen]), q, d, C.slot);
        q.alive = false;
        return false;
    }
    if (WW == 2 && due) ww_check(PL, A, S, C, q);
    return WW == 1 && due;
}

// Network checks (WW 1) run in wave-level batches, as in the history kernel:
// a lane whose check is due waits (its particle does not move) until at
// least half of the wave's active lanes wait, then they evaluate the network
// together; the check sees exactly the state it would have seen at once.
// Returns true when this loop turn was spent on (or waiting for) checks.
template <int WW, class Ctx>
MCDC_DEV bool batched_check(CP &PL, const RunArgs &A, Shared &S, Ctx &C, Part &q, bool &due) {
    if constexpr (WW != 1) return false;
    const uint64_t waiting = __ballot(due);
    if (waiting && 2 * __popcll(waiting) >= __popcll(__ballot(true))) {
        if (due) {
            ww_check(PL, A, S, C, q);
            due = false;
        }
        return true;
    }
    return due;
}

// Lead stage (hybrid schedule).  Workgroup w takes the contiguous slots
// [w n / G, (w+1) n / G) (so its LDS tile, if any, sees one batch apart from
// at most one boundary); its work-items take the next slot from a counter in
// LDS and run one flight per loop turn, as the history schedule does: the
// particle, then the daughters on the stack, then the next slot.  After
// MCDC_LEAD_FLIGHTS flights of one history its particle and stacked daughters
// go into the active bank; with population control or census-step control a
// particle that reaches a census goes into the census bank.  The re-lead
// stage finishes what was banked.  LDS: 0 tally in HBM, 2 hot tile in LDS.
template <int LDS, int WW>
__global__ void __launch_bounds__(tile_threads(LDS, WW)) k_ev_lead(DevProblem, RunArgs A, EvBank B,
                                                                  uint32_t n) {
    CP &P = kernel_problem();
    extern __shared__ double s_tile[];
    __shared__ Shared S;
    __shared__ uint32_t s_next, s_cancel;
    const CancelSeen cancel{&s_cancel};
    shared_zero(S);
    cancel.init(A.cancel);
    const uint32_t r0 = (uint32_t)((uint64_t)blockIdx.x * n / gridDim.x);
    const uint32_t r1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * n / gridDim.x);
    if (threadIdx.x == 0) s_next = r0;
    if (LDS == 2)
        for (uint32_t i = threadIdx.x; i < P.hot_bins; i += blockDim.x) s_tile[i] = 0.0;
    __syncthreads();
    const uint64_t b_tile = batch_of(A, r0);
    const uint32_t cur = B.ctl->cur, cen = B.ctl->cen;
    const bool stop_at_census = P.pc_on || B.ctl->pause_at_census;
    // analog histories that cannot stop at a census never reach the banks:
    // the lead stage closes their statistics itself (lead_finalizes)
    const bool finalize = WW == 0 && !stop_at_census;
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n_flight = 0, n_piece = 0, lead_flights = 0, n_hit = 0;
    double path = 0.0;
    LeadCtx<WW> C{P, A, B, lane, cur, 0u, 0.0, 0.0, 0u, 0};
    LeadTally<LDS> tally;
    tally.init(P, s_tile);
    Part q;
    q.alive = false;
    bool in_hist = false;
    bool ww_due = false;
    uint32_t n_started = 0;
    for (;;) {
        CP &PL = problem_reload(P);
        if (batched_check<WW>(PL, A, S, C, q, ww_due)) continue;
        if (!q.alive) {
            if (WW != 0 && C.sp > 0) {
                C.sp -= 1;
                stack_pop(A, lane, PL.stack_cap, C.sp, q);
            } else {
                if (in_hist) {
                    if (finalize) {
                        // nothing of the history was banked: its statistics
                        // are final (what the finish kernel does otherwise)
                        if (C.xh != 0.0) {
                            unsafeAtomicAdd(&A.acc->det[0], C.xh);
                            unsafeAtomicAdd(&A.acc->det[1], C.xh * C.xh);
                        }
                        if (C.xh > 0.0) n_hit += 1;
                        if (A.xh_out) {
                            const uint64_t o = A.h_begin + C.slot - A.h_run0;
                            A.xh_out[2 * o] = C.xh;
                            A.xh_out[2 * o + 1] = C.path;
                        }
                    } else {
                        B.xh[C.slot] = C.xh;
                        B.path[C.slot] = C.path;
                        B.events[C.slot] = C.events;
                    }
                    in_hist = false;
                }
                if (cancel.check(A.cancel, n_started++)) {
                    set_status(A, MCDC_E_CANCELLED);
                    break;
                }
                const uint32_t s = atomicAdd(&s_next, 1u);
                if (s >= r1) break;
                C.slot = s;
                C.xh = 0.0;
                C.path = 0.0;
                C.events = 0u;
                C.sp = 0;
                lead_flights = 0;
                in_hist = true;
                tally.select(PL, A, batch_of(A, s), b_tile);
                stage_source(PL, A, S, C, q);
                if (!q.alive) continue;
            }
        }
        // the rest of the history is handed over after MCDC_LEAD_FLIGHTS flights
        ww_due = lead_turn<WW, MCDC_LEAD_FLIGHTS>(PL, A, B, S, tally.t, C, q, lead_flights,
                                                  n_flight, n_piece, path, stop_at_census, cen);
    }
    atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
    atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
    if (n_hit) atomicAdd(&S.cnt[C_DET_HIT], (unsigned long long)n_hit);
    atomicAdd(&S.wsum[W_PATH], path);
    __syncthreads();
    if (LDS == 2 && r0 < r1) hot_tile_flush(P, s_tile, A.tally + b_tile * (uint64_t)P.nbins);
    shared_flush(S, A.acc);
}

// Flight stage.  LDS 0: tally updates to HBM atomics, the workgroups stride
// over the active bank.  LDS 2: workgroup w takes the contiguous entries
// [w n / G, (w+1) n / G) (particles stay near the order of their histories,
// so a range holds few batches) and keeps the hot tile of its first
// particle's batch in LDS, as the lead stage does.
template <bool WW, int LDS>
__global__ void __launch_bounds__(LDS == 2 ? 1024 : 256) k_ev_flight(DevProblem, RunArgs A, EvBank B) {
    CP &P = kernel_problem();
    extern __shared__ double s_tile[];
    __shared__ Shared S;
    if (B.ctl->paused) return;
    shared_zero(S);
    const uint32_t cur = B.ctl->cur, cen = B.ctl->cen;
    const uint32_t n = min(B.ctl->n_act[cur], B.cap);   // counts can pass cap on overflow
    uint32_t r0 = blockIdx.x * blockDim.x, r1 = n, stride = gridDim.x * blockDim.x;
    if (LDS == 2) {
        r0 = (uint32_t)((uint64_t)blockIdx.x * n / gridDim.x);
        r1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * n / gridDim.x);
        stride = blockDim.x;
        if (r0 < r1)
            for (uint32_t i = threadIdx.x; i < P.hot_bins; i += blockDim.x) s_tile[i] = 0.0;
    }
    __syncthreads();
    const Bank in = B.b[cur], X = B.b[R_X], CB = B.b[cen];
    const uint64_t b_tile = LDS == 2 && r0 < r1 ? batch_of(A, in.i[6 * (size_t)B.cap + r0]) : 0;
    LeadTally<LDS> tally;
    tally.init(P, s_tile);
    uint32_t n_piece = 0, n_flight = 0;
    double path = 0.0;
    for (uint32_t j0 = r0; j0 < r1; j0 += stride) {
        CP &PL = problem_reload(P);
        const uint32_t jj = j0 + threadIdx.x;
        const bool valid = jj < r1;
        int ev = -1;
        Part q;
        double d = 0.0;
        uint32_t slot = 0;
        if (valid) {
            bank_load(in, B.cap, jj, q, d, slot);
            EvCtx<WW> C{PL, A, B, slot};
            tally.select(PL, A, C.batch(), b_tile);
            ev = stage_flight(PL, A, S, tally.t, C, q, d, n_piece, path);
            if (ev >= 0) n_flight += 1;
            if (!q.alive) ev = -1;
        }
        // grid-plane stops go to the front of the interaction bank with the
        // surfaces, marked in the slot's top bit (slots are below 2^26)
        const bool front = ev == EV_SURFACE || ev == EV_WW_PLANE;
        const uint32_t ps = wave_reserve(&B.ctl->n_surf, front);
        const uint32_t pc = wave_reserve(&B.ctl->n_coll, ev == EV_SCATTER);
        const uint32_t pn = wave_reserve(&B.ctl->n_act[cen], ev == EV_CENSUS);
        if (front) bank_put(A, B, X, ps, q, d, ev == EV_WW_PLANE ? slot | kPlaneMark : slot);
        else if (ev == EV_SCATTER) bank_put(A, B, X, B.cap - 1u - pc, q, d, slot);
        else if (ev == EV_CENSUS) bank_put(A, B, CB, pn, q, d, slot);
    }
    atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
    atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
    atomicAdd(&S.wsum[W_PATH], path);
    __syncthreads();
    if (LDS == 2 && r0 < r1) hot_tile_flush(P, s_tile, A.tally + b_tile * (uint64_t)P.nbins);
    shared_flush(S, A.acc);
}

// Bank roles for the next iteration.  Reads the counts with atomics so that
// what other workgroups reserved is seen.  With population control a census
// switch first runs the control (the sum and apply launches of the same
// iteration), which then rotates the roles.
MCDC_DEV void ev_advance(EvCtl *c, bool pc) {
    const uint32_t cur = c->cur, nxt = c->nxt, cen = c->cen;
    const uint32_t n_nxt = atomicAdd(&c->n_act[nxt], 0u);
    const uint32_t n_cen = atomicAdd(&c->n_act[cen], 0u);
    c->n_act[cur] = 0;
    c->n_surf = 0;
    c->n_coll = 0;
    if (n_nxt > 0) {
        c->cur = nxt;
        c->nxt = cur;
    } else if (n_cen > 0) {
        if (pc) {
            c->pc_wq = 0ull;
            c->pc_stage = 1;
        } else {                         // next census step
            c->cur = cen;
            c->cen = nxt;
            c->nxt = cur;
            if (c->pause_at_census) c->paused = 1;
        }
    } else {
        c->done = 1;
    }
}

// Is this workgroup the last of the launch to finish?  (after its last
// global write; resets the count for the next launch)
MCDC_DEV bool last_block(EvCtl *c, bool &s_last) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&c->blocks_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        c->blocks_done = 0;
    }
    return s_last;
}

// Surface and collision stages in one launch: entries [0, n_surf) of the
// combined range are the surface entries at the front of the interaction
// bank, the rest the collision entries at its back.  WW: 0 none, 1 network
// at each check, 2 baked window map.
template <int WW>
__global__ void __launch_bounds__(256) k_ev_interact(DevProblem, RunArgs A, EvBank B) {
    CP &P = kernel_problem();
    __shared__ Shared S;
    __shared__ bool s_last;
    if (B.ctl->paused) return;
    shared_zero(S);
    __syncthreads();
    const uint32_t nxt = B.ctl->nxt;
    const uint32_t ns = min(B.ctl->n_surf, B.cap);
    const uint32_t nc = min(B.ctl->n_coll, B.cap - ns);
    const uint32_t n = ns + nc;
    const Bank X = B.b[R_X], out = B.b[nxt];
    for (uint32_t j0 = blockIdx.x * blockDim.x; j0 < n; j0 += gridDim.x * blockDim.x) {
        CP &PL = problem_reload(P);
        const uint32_t jj = j0 + threadIdx.x;
        const bool valid = jj < n;
        bool alive = false;
        uint32_t nd = 0, tag0 = 0, slot = 0;
        Part q;
        double d = 0.0;
        if (valid) {
            const bool surf = jj < ns;
            bank_load(X, B.cap, surf ? jj : B.cap - 1u - (jj - ns), q, d, slot);
            const bool plane = surf && (slot & kPlaneMark) != 0u;   // grid-plane stop
            slot &= ~kPlaneMark;
            EvCtx<WW> C{PL, A, B, slot};
            const bool due = plane ? true
                                   : (surf ? stage_surface(PL, A, S, C, q, d)
                                           : stage_collision(PL, A, S, C, q, d));
            if (WW != 0 && due) ww_check(PL, A, S, C, q);
            alive = q.alive;
            if (WW != 0 && C.split_n > 1) {
                nd = C.split_n - 1;
                tag0 = C.split_tag0;
            }
        }
        const uint32_t pos = wave_reserve(&B.ctl->n_act[nxt], alive);
        if (alive) bank_put(A, B, out, pos, q, d, slot);
        if (WW != 0) wave_write_copies(A, B, out, &B.ctl->n_act[nxt], q, slot, nd, tag0);
    }
    __syncthreads();
    shared_flush(S, A.acc);
    if (last_block(B.ctl, s_last) && threadIdx.x == 0) ev_advance(B.ctl, P.pc_on != 0);
}

// Re-lead stage (hybrid schedule): the lead stage's loop run over the
// particles of the active bank instead of new histories, in place of the
// flight and interaction stages.  Workgroup w takes the bank entries
// [w n / G, (w+1) n / G); a work-item follows each particle it takes, with its
// split daughters on the work-item's stack, for MCDC_RELEAD_FLIGHTS flights and
// hands what is left to the next active bank (a census stop, with population
// control or census-step control, to the census bank).  The tally target is
// the lead stage's, its LDS tile holding the batch of the workgroup's first
// particle.  The last workgroup to finish advances the bank roles as the
// interaction stage does.
template <int LDS, int WW>
__global__ void __launch_bounds__(tile_threads(LDS, WW)) k_ev_relead(DevProblem, RunArgs A, EvBank B) {
    CP &P = kernel_problem();
    extern __shared__ double s_tile[];
    __shared__ Shared S;
    __shared__ uint32_t s_next, s_cancel;
    __shared__ bool s_last;
    if (B.ctl->paused) return;
    const CancelSeen cancel{&s_cancel};
    shared_zero(S);
    cancel.init(A.cancel);
    const uint32_t cur = B.ctl->cur, nxt = B.ctl->nxt, cen = B.ctl->cen;
    const uint32_t n = min(B.ctl->n_act[cur], B.cap);   // counts can pass cap on overflow
    const uint32_t r0 = (uint32_t)((uint64_t)blockIdx.x * n / gridDim.x);
    const uint32_t r1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * n / gridDim.x);
    if (threadIdx.x == 0) s_next = r0;
    if (LDS == 2 && r0 < r1)
        for (uint32_t i = threadIdx.x; i < P.hot_bins; i += blockDim.x) s_tile[i] = 0.0;
    __syncthreads();
    const Bank in = B.b[cur];
    const uint64_t b_tile = r0 < r1 ? batch_of(A, in.i[6 * (size_t)B.cap + r0]) : 0;
    const bool stop_at_census = P.pc_on || B.ctl->pause_at_census;
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n_flight = 0, n_piece = 0, flights = 0;
    double path = 0.0;
    LeadCtx<WW, true> C{P, A, B, lane, nxt, 0u, 0.0, 0.0, 0u, 0};
    LeadTally<LDS> tally;
    tally.init(P, s_tile);
    Part q;
    q.alive = false;
    bool ww_due = false;
    uint32_t n_started = 0;
    for (;;) {
        CP &PL = problem_reload(P);
        if (batched_check<WW>(PL, A, S, C, q, ww_due)) continue;
        if (!q.alive) {
            if (WW != 0 && C.sp > 0) {
                C.sp -= 1;
                stack_pop(A, lane, PL.stack_cap, C.sp, q);
            } else {
                if (cancel.check(A.cancel, n_started++)) {
                    set_status(A, MCDC_E_CANCELLED);
                    break;
                }
                const uint32_t j = atomicAdd(&s_next, 1u);
                if (j >= r1) break;
                double d0;
                uint32_t slot;
                bank_load(in, B.cap, j, q, d0, slot);
                C.flush_events();
                C.take(slot);
                flights = 0;
                tally.select(PL, A, batch_of(A, slot), b_tile);
            }
        }
        ww_due = lead_turn<WW, MCDC_RELEAD_FLIGHTS>(PL, A, B, S, tally.t, C, q, flights, n_flight,
                                                    n_piece, path, stop_at_census, cen);
    }
    C.flush_events();
    atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
    atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
    atomicAdd(&S.wsum[W_PATH], path);
    __syncthreads();
    if (LDS == 2 && r0 < r1) hot_tile_flush(P, s_tile, A.tally + b_tile * (uint64_t)P.nbins);
    shared_flush(S, A.acc);
    if (last_block(B.ctl, s_last) && threadIdx.x == 0) ev_advance(B.ctl, P.pc_on != 0);
}

// Population control, step 1: the census bank's total weight, summed exactly
// as integers floor(w * 2^32).
__global__ void __launch_bounds__(256) k_ev_pc_sum(EvBank B) {
    __shared__ unsigned long long s_sum;
    __shared__ bool s_last;
    if (B.ctl->pc_stage != 1) return;
    if (threadIdx.x == 0) s_sum = 0ull;
    __syncthreads();
    const uint32_t cen = B.ctl->cen;
    const uint32_t n = min(B.ctl->n_act[cen], B.cap);
    const double *w = B.b[cen].d + 7 * (size_t)B.cap;
    unsigned long long part = 0ull;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        part += (unsigned long long)floor(w[j] * 4294967296.0);
    if (part) atomicAdd(&s_sum, part);
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicAdd(&B.ctl->pc_wq, s_sum);
    if (last_block(B.ctl, s_last) && threadIdx.x == 0) B.ctl->pc_stage = 2;
}

// Population control, step 2: splitting-roulette of every census particle to
// the target weight w_T = (sum * 2^-32) / M.  One draw xi from the particle's
// stream: below w_T it survives iff xi * w_T < w, at weight w_T; otherwise it
// becomes n = floor(w / w_T + xi) particles of weight w_T, the copies taking
// stream tags from one further block.  Survivors and copies go to the next
// active bank, which then becomes the active bank.
__global__ void __launch_bounds__(256) k_ev_pc_apply(DevProblem, RunArgs A, EvBank B) {
    CP &P = kernel_problem();
    __shared__ Shared S;
    __shared__ bool s_last;
    if (B.ctl->pc_stage != 2) return;
    shared_zero(S);
    __syncthreads();
    const uint32_t cen = B.ctl->cen, nxt = B.ctl->nxt;
    const uint32_t n = min(B.ctl->n_act[cen], B.cap);
    const double wt = ((double)B.ctl->pc_wq * 0x1p-32) / A.pc_m;
    const bool on = wt > 0.0;              // a bank of negligible weight is left as it is
    const Bank in = B.b[cen], out = B.b[nxt];
    for (uint32_t j0 = blockIdx.x * blockDim.x; j0 < n; j0 += gridDim.x * blockDim.x) {
        const uint32_t jj = j0 + threadIdx.x;
        const bool valid = jj < n;
        bool keep = false;
        uint32_t nd = 0, tag0 = 0, slot = 0;
        Part q;
        double d = 0.0;
        if (valid) {
            bank_load(in, B.cap, jj, q, d, slot);
            keep = true;
            if (on) {
                const uint64_t hist = A.h_begin + slot;
                Rng r = make_rng(A.seed, hist, P.problem_id, q.tag, q.k);
                const double xi = rng_uniform(r);
                const double w = q.w;
                if (w < wt) {
                    q.k = r.k;
                    if (xi * wt < w) {
                        atomicAdd(&S.wsum[W_GAIN], wt - w);
                        q.w = wt;
                        trace_rec(A, hist, q, EV_PC_KEEP, 1.0);
                    } else {
                        atomicAdd(&S.wsum[W_LOSS], w);
                        atomicAdd(&S.cnt[C_PC_KILL], 1ull);
                        trace_rec(A, hist, q, EV_PC_KILL, 0.0);
                        keep = false;
                    }
                } else {
                    const double nf = floor(w / wt + xi);
                    const double tot = nf * wt;
                    if (tot > w) atomicAdd(&S.wsum[W_GAIN], tot - w);
                    else atomicAdd(&S.wsum[W_LOSS], w - tot);
                    const uint32_t nn = (uint32_t)nf;
                    if (nn >= 2) {
                        uint32_t blk[4];
                        rng_block(r, blk);
                        tag0 = blk[0];
                        nd = nn - 1u;
                        atomicAdd(&S.cnt[C_PC_COPY], (unsigned long long)nd);
                        atomicAdd(&S.cnt[C_PARTICLE], (unsigned long long)nd);
                    }
                    q.k = r.k;
                    q.w = wt;
                    trace_rec(A, hist, q, EV_PC_KEEP, nf);
                }
            }
        }
        const uint32_t pos = wave_reserve(&B.ctl->n_act[nxt], keep);
        if (keep) bank_put(A, B, out, pos, q, d, slot);
        wave_write_copies(A, B, out, &B.ctl->n_act[nxt], q, slot, nd, tag0);
    }
    __syncthreads();
    shared_flush(S, A.acc);
    if (last_block(B.ctl, s_last) && threadIdx.x == 0) {
        EvCtl *c = B.ctl;
        const uint32_t cur = c->cur;     // drained
        c->n_act[cen] = 0;
        c->cur = nxt;
        c->nxt = cen;
        c->cen = cur;
        c->pc_stage = 0;
        if (atomicAdd(&c->n_act[nxt], 0u) == 0u) c->done = 1;
        else if (c->pause_at_census) c->paused = 1;
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

__global__ void k_ev_reset(EvBank B) {
    EvCtl *c = B.ctl;
    for (int i = 0; i < 3; ++i) c->n_act[i] = 0;
    c->n_surf = c->n_coll = 0;
    c->cur = R_A;
    c->nxt = R_B;
    c->cen = R_C;
    c->done = 0;
    c->blocks_done = 0;
    c->pc_stage = 0;
    c->pc_wq = 0ull;
    c->pause_at_census = 0;
    c->paused = 0;
}

__global__ void k_ev_set_pause(EvBank B, uint32_t pause) {
    B.ctl->pause_at_census = pause;
    B.ctl->paused = 0;
}

__global__ void k_ev_count_hist(DevAcc *acc, uint64_t n) { atomicAdd(&acc->cnt[C_HIST], (unsigned long long)n); }

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static uint32_t ev_chunk(const mcdc_problem_desc *d, const Options &o) {
    int64_t c = o.event_chunk > 0 ? o.event_chunk : (1 << 22);
    if (c > (1 << 26)) c = 1 << 26;
    (void)d;
    return (uint32_t)c;
}

// Bank capacity: the live population, not the particles ever made (every
// stage compacts): the resident histories, times 4 with weight windows, plus
// room for the population-control target.
static uint32_t ev_cap(const mcdc_problem_desc *d, const Options &o) {
    const uint64_t chunk = ev_chunk(d, o);
    uint64_t f = d->stack_cap > 0 ? 4 : 1;
    if (d->pc_on) f += (uint64_t)ceil(d->pc_target) + 1;
    uint64_t cap = chunk * f;
    if (cap > 0xF0000000ull) cap = 0xF0000000ull;
    return (uint32_t)cap;
}

static size_t bank_bytes(size_t cap) { return al(9 * cap * sizeof(double)) + al(7 * cap * sizeof(uint32_t)); }

size_t event_workspace_bytes(const mcdc_problem_desc *d, const Options &o) {
    if (o.schedule != MCDC_SCHED_EVENT) return 0;
    const size_t cap = ev_cap(d, o), chunk = ev_chunk(d, o);
    return 4 * bank_bytes(cap) + 2 * al(chunk * sizeof(double)) + al(chunk * sizeof(uint32_t)) +
           al(sizeof(EvCtl));
}

uint64_t ev_resident_histories(const mcdc_problem *h) { return h->ev ? h->ev->B.chunk : 0; }

int event_init(mcdc_problem *h) {
    if (h->desc.imp_on) return fail(MCDC_E_INVALID, "the importance estimate runs in the history schedule only");
    auto *E = new EventState();
    const size_t cap = ev_cap(&h->desc, h->opt), chunk = ev_chunk(&h->desc, h->opt);
    char *p = h->ws + h->L.event;
    EvBank &B = E->B;
    B.cap = (uint32_t)cap;
    B.chunk = (uint32_t)chunk;
    for (int k = 0; k < 4; ++k) {
        B.b[k].d = (double *)p;
        p += al(9 * cap * sizeof(double));
        B.b[k].i = (uint32_t *)p;
        p += al(7 * cap * sizeof(uint32_t));
    }
    B.xh = (double *)p; p += al(chunk * sizeof(double));
    B.path = (double *)p; p += al(chunk * sizeof(double));
    B.events = (uint32_t *)p; p += al(chunk * sizeof(uint32_t));
    B.ctl = (EvCtl *)p;
    hipError_t e = hipHostMalloc((void **)&E->host_done, 2 * sizeof(uint32_t), hipHostMallocDefault);
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

static void ev_launch_source(mcdc_problem *h, const RunArgs &A, hipStream_t s, uint32_t n) {
    EventState *E = h->ev;
    const EvBank &B = E->B;
    int sg = (int)((n + E->block - 1) / E->block);
    if (sg > E->grid) sg = E->grid;
    hipLaunchKernelGGL(k_ev_count_hist, dim3(1), dim3(1), 0, s, A.acc, (uint64_t)n);
    if (h->opt.lead) {
        // the lead grid is the history schedule's (block, grid), with 768
        // work-items per workgroup for tiled network checks: work-item i owns
        // stack lane i, and A.n_lanes = grid * block lanes exist
        const DevProblem &P = h->P;
        const int ww = P.ww_on ? (P.ww_map ? 2 : 1) : 0;
        const int lb = P.hot_bins && ww == 1 ? kNetTileThreads : h->opt.block;
        int lg = (int)((n + lb - 1) / lb);
        if (lg > h->opt.grid) lg = h->opt.grid;
        if (lg < 1) lg = 1;
        const size_t shm = P.hot_bins ? (size_t)P.hot_bins * sizeof(double) : 0;
#define MCDC_LEAD(L, W)                                                                        \
    do {                                                                                       \
        if (shm > 65536)                                                                       \
            (void)hipFuncSetAttribute((const void *)k_ev_lead<L, W>,                           \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);   \
        hipLaunchKernelGGL((k_ev_lead<L, W>), dim3(lg), dim3(lb), shm, s, P, A, B, n);         \
    } while (0)
        timing_begin(h, s);
        if (P.hot_bins) {
            if (ww == 2) MCDC_LEAD(2, 2);
            else if (ww == 1) MCDC_LEAD(2, 1);
            else MCDC_LEAD(2, 0);
        } else {
            if (ww == 2) MCDC_LEAD(0, 2);
            else if (ww == 1) MCDC_LEAD(0, 1);
            else MCDC_LEAD(0, 0);
        }
#undef MCDC_LEAD
        timing_end(h, s);
        return;
    }
    if (h->P.ww_on) hipLaunchKernelGGL((k_ev_source<true>), dim3(sg), dim3(E->block), 0, s, h->P, A, B, n);
    else hipLaunchKernelGGL((k_ev_source<false>), dim3(sg), dim3(E->block), 0, s, h->P, A, B, n);
}

// The re-lead stage on the lead stage's grid and block (work-item i owns
// stack lane i); every workgroup reads the bank count on the device.
static void ev_launch_relead(mcdc_problem *h, const RunArgs &A, hipStream_t s) {
    const DevProblem &P = h->P;
    const EvBank &B = h->ev->B;
    const int ww = P.ww_on ? (P.ww_map ? 2 : 1) : 0;
    const dim3 grid(h->opt.grid), block(P.hot_bins && ww == 1 ? kNetTileThreads : h->opt.block);
    const size_t shm = P.hot_bins ? (size_t)P.hot_bins * sizeof(double) : 0;
#define MCDC_RELEAD(L, W)                                                                      \
    do {                                                                                       \
        if (shm > 65536)                                                                       \
            (void)hipFuncSetAttribute((const void *)k_ev_relead<L, W>,                         \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);   \
        hipLaunchKernelGGL((k_ev_relead<L, W>), grid, block, shm, s, P, A, B);                 \
    } while (0)
    if (P.hot_bins) {
        if (ww == 2) MCDC_RELEAD(2, 2);
        else if (ww == 1) MCDC_RELEAD(2, 1);
        else MCDC_RELEAD(2, 0);
    } else {
        if (ww == 2) MCDC_RELEAD(0, 2);
        else if (ww == 1) MCDC_RELEAD(0, 1);
        else MCDC_RELEAD(0, 0);
    }
#undef MCDC_RELEAD
}

// The flight stage: with a hot tile on the options' grid of 1024-work-item
// workgroups and the tile in dynamic LDS, else on the event grid.
static void ev_launch_flight(mcdc_problem *h, const RunArgs &A, hipStream_t s) {
    const DevProblem &P = h->P;
    const EventState *E = h->ev;
    const bool ww = P.ww_on != 0;
    if (P.hot_bins) {
        const size_t shm = (size_t)P.hot_bins * sizeof(double);
        const void *k = ww ? (const void *)k_ev_flight<true, 2> : (const void *)k_ev_flight<false, 2>;
        if (shm > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (ww) hipLaunchKernelGGL((k_ev_flight<true, 2>), dim3(h->opt.grid), dim3(h->opt.block), shm, s, P, A, E->B);
        else hipLaunchKernelGGL((k_ev_flight<false, 2>), dim3(h->opt.grid), dim3(h->opt.block), shm, s, P, A, E->B);
    } else {
        if (ww) hipLaunchKernelGGL((k_ev_flight<true, 0>), dim3(E->grid), dim3(E->block), 0, s, P, A, E->B);
        else hipLaunchKernelGGL((k_ev_flight<false, 0>), dim3(E->grid), dim3(E->block), 0, s, P, A, E->B);
    }
}

// Iterate the stages of the resident chunk until it ends (or, under
// census-step control, a census step begins): K iterations per host check.
// An iteration is the flight and interaction stages, or in the hybrid
// schedule the re-lead stage; then, with population control, the control
// launches.
static int ev_iterate(mcdc_problem *h, const RunArgs &A, hipStream_t s, bool &done) {
    EventState *E = h->ev;
    const DevProblem &P = h->P;
    const EvBank &B = E->B;
    const int grid = E->grid, block = E->block;
    const bool ww = P.ww_on != 0, pc = P.pc_on != 0, lead = h->opt.lead;
    for (int iter = 0;; ++iter) {
        // after a lead stage the banks are often empty: check after one
        // iteration first, then every four (a re-lead iteration finishes most
        // of what it takes); every eight in the event schedule
        const int K = lead ? (iter == 0 ? 1 : 4) : 8;
        h->event_iterations += K;
        for (int k = 0; k < K; ++k) {
            if (lead) {
                ev_launch_relead(h, A, s);
            } else {
                // timed stage: the flight stage (the lead stage in the hybrid schedule)
                timing_begin(h, s);
                ev_launch_flight(h, A, s);
                timing_end(h, s);
                if (!ww) hipLaunchKernelGGL((k_ev_interact<0>), dim3(grid), dim3(block), 0, s, P, A, B);
                else if (P.ww_map) hipLaunchKernelGGL((k_ev_interact<2>), dim3(grid), dim3(block), 0, s, P, A, B);
                else hipLaunchKernelGGL((k_ev_interact<1>), dim3(grid), dim3(block), 0, s, P, A, B);
            }
            if (pc) {
                hipLaunchKernelGGL(k_ev_pc_sum, dim3(grid), dim3(block), 0, s, B);
                hipLaunchKernelGGL(k_ev_pc_apply, dim3(grid), dim3(block), 0, s, P, A, B);
            }
        }
        hipError_t e = hipMemcpyAsync(E->host_done, &B.ctl->done, 2 * sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "event loop");
        if (cancel_set(h)) return fail(MCDC_E_CANCELLED, "run cancelled");
        if (E->host_done[0]) {
            done = true;
            return MCDC_OK;
        }
        if (E->host_done[1]) {
            done = false;
            return MCDC_OK;
        }
        if (iter > 1000000) return fail(MCDC_E_EVENT_CAP, "event loop did not drain");
    }
}

// Does the lead stage close the statistics of every history itself?  (The
// same condition as `finalize` in k_ev_lead, for a run without census-step
// control: then it banks nothing either.)
static bool lead_finalizes(const mcdc_problem *h) {
    return h->opt.lead && !h->P.ww_on && !h->P.pc_on;
}

static int ev_finish_chunk(mcdc_problem *h, const RunArgs &A, hipStream_t s, uint32_t n) {
    EventState *E = h->ev;
    const int fg = (int)((n + E->block - 1) / E->block) < E->grid ? (int)((n + E->block - 1) / E->block)
                                                                : E->grid;
    hipLaunchKernelGGL(k_ev_finish, dim3(fg), dim3(E->block), 0, s, A, E->B, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "event launch");
    return MCDC_OK;
}

// Transport histories [A.h_begin, A.h_end) chunk by chunk.
int event_run_range(mcdc_problem *h, const RunArgs &A0, hipStream_t s) {
    EventState *E = h->ev;
    if (!E) return fail(MCDC_E_STATE, "event schedule not initialised");
    const EvBank &B = E->B;
    for (uint64_t c0 = A0.h_begin; c0 < A0.h_end; c0 += B.chunk) {
        const uint64_t c1 = c0 + B.chunk < A0.h_end ? c0 + B.chunk : A0.h_end;
        const uint32_t n = (uint32_t)(c1 - c0);
        RunArgs A = A0;
        A.h_begin = c0;
        A.h_end = c1;
        hipLaunchKernelGGL(k_ev_reset, dim3(1), dim3(1), 0, s, B);
        ev_launch_source(h, A, s, n);
        if (lead_finalizes(h)) {
            // the lead stage banked nothing and closed every history itself:
            // no re-lead launch and no host check of the banks (the host
            // stays ahead of the GPU, as in the history schedule)
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "event launch");
            if (cancel_set(h)) return fail(MCDC_E_CANCELLED, "run cancelled");
            continue;
        }
        bool done = false;
        int st = ev_iterate(h, A, s, done);
        if (st) return st;
        if ((st = ev_finish_chunk(h, A, s, n))) return st;
    }
    return MCDC_OK;
}

// Census-step control: the run's histories form one resident chunk.
int event_begin(mcdc_problem *h, const RunArgs &A, hipStream_t s) {
    EventState *E = h->ev;
    if (!E) return fail(MCDC_E_STATE, "event schedule not initialised");
    const uint32_t n = (uint32_t)(A.h_end - A.h_begin);
    hipLaunchKernelGGL(k_ev_reset, dim3(1), dim3(1), 0, s, E->B);
    hipLaunchKernelGGL(k_ev_set_pause, dim3(1), dim3(1), 0, s, E->B, 1u);
    ev_launch_source(h, A, s, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "run_begin");
    return MCDC_OK;
}

int event_step(mcdc_problem *h, const RunArgs &A, hipStream_t s, bool &done) {
    EventState *E = h->ev;
    if (!E) return fail(MCDC_E_STATE, "event schedule not initialised");
    hipLaunchKernelGGL(k_ev_set_pause, dim3(1), dim3(1), 0, s, E->B, 1u);
    int st = ev_iterate(h, A, s, done);
    if (st) return st;
    if (done) return ev_finish_chunk(h, A, s, (uint32_t)(A.h_end - A.h_begin));
    return MCDC_OK;
}

}  // namespace mcdc
