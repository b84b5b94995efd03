// Batched problems: many independent problems of uneven size in one
// persistent launch per census step, the census steps of a pass captured once
// in a HIP graph and replayed.
//
// Per census step s:
//   k_b_plan       one workgroup: per-problem work = histories (step 0) or
//                  particles that reached the previous census; chunk counts and
//                  their prefix sum form the step's work queue; queue roles swap.
//   k_b_persistent grid sized to the chip; each workgroup pops chunks
//                  (problem p, entry range) from the device work queue until it
//                  is empty.  A chunk belongs to one problem, so the problem's
//                  description is wave-uniform (scalar loads).  Within a chunk
//                  each work-item takes the next entry when its particle ends
//                  and runs one flight per loop turn.  Particles fly
//                  until they end or reach the census time of step s; those
//                  that reach it are appended (one atomic per wave) to the
//                  problem's queue for step s+1.  Tally pieces in the step's
//                  time bin go to an LDS tile of that time slice, flushed to HBM
//                  when the workgroup moves to another problem; the rest (only
//                  possible at bin edges) go straight to HBM atomics.
// After the last step: batch close-out of every problem's tally and the
// history-id bases advance, all inside the graph.  Seeds, step index and
// history bases live in device memory so the graph's kernel arguments never
// change; nothing is memset inside the graph.
#include "mcdc_runtime.hpp"
#include "transport_stages.hpp"

namespace mcdc {

constexpr int kBatchMaxProblems = 4096;
constexpr int kTileBins = 8192;               // 64 KiB LDS time-slice tile

struct BProb {
    DevProblem P;
    uint64_t tally_off;                       // doubles into the batch tally arrays
    uint64_t bank_off;                        // first bank slot
    uint32_t n_hist;                          // histories per pass
    uint32_t slice;                           // bins in one time slice (x*y*z), 0 = no tile
};

struct BCtl {
    uint64_t seed;
    uint32_t step, total_chunks, chunk_next;
    uint32_t pad[3];
};

struct BDev {
    BProb *probs;
    uint32_t n_prob, chunk, n_steps;
    double *tally, *tsum, *tsumsq;
    DevAcc *acc;                              // [n_prob]
    double *bd;                               // [10][cap]: x y z ux uy uz t w path (spare)
    uint32_t *bi;                             // [7][cap]: g cell ci tag k seq flights
    uint32_t *q;                              // [2][cap] queues (problem-local entries)
    uint32_t *nq;                             // [2][n_prob] queue counts
    uint32_t *chunk_off;                      // [n_prob + 1]
    uint64_t *hist_base;                      // [n_prob]
    BCtl *ctl;
    const int *cancel;                        // host-coherent cancel word
    uint64_t cap;
    uint64_t total_bins;
};

}  // namespace mcdc

namespace mcdc {

struct BatchState {
    BDev D;
    std::vector<BProb> host_probs;
    std::vector<uint64_t> n_hist;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int grid = 0, block = 256;
    uint64_t passes = 0;
    double *host_seed = nullptr;              // pinned staging for the seed
};

struct BatchCtx {
    static constexpr bool kWW = false;
    static constexpr bool kWWMap = false;
    // the persistent batch kernel sits at its register limit
    static constexpr bool kTightRegs = true;
    MCDC_DEV double *col_tally() const { return nullptr; }
    MCDC_DEV double *surf_tally() const { return nullptr; }
    CP &P;
    const RunArgs &A;
    const BDev &D;
    uint64_t hist_id;
    uint64_t slot;
    MCDC_DEV uint64_t hist() const { return hist_id; }
    MCDC_DEV const float *mlp_params(CP &Pp) const { return Pp.ww_params; }
    // one particle per history (no weight windows in batched runs): the
    // history's flight count lives in the particle's bank slot
    MCDC_DEV bool count_flight() {
        const uint32_t e = (D.bi[6 * D.cap + slot] += 1u);
        return (int64_t)e <= P.max_events;
    }
    MCDC_DEV void add_score(double) {}
    MCDC_DEV void add_path(double v) { D.bd[8 * D.cap + slot] += v; }
    MCDC_DEV void imp_point(CP &, const Part &) {}
    MCDC_DEV bool push_daughters(const Part &, uint32_t, int) { return false; }
};

// LDS tile for one time slice of one problem; other bins go to HBM.
struct TileTally {
    lds_f64 *lds;
    hbm_f64 *glob;
    uint32_t lo, hi;
    MCDC_DEV void add(uint32_t i, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, double v) const {
        if (i >= lo && i < hi) lds_add(lds + (i - lo), v);
        else hbm_add(glob + i, v);
    }
};

MCDC_DEV void bload(const BDev &D, uint64_t j, Part &q) {
    const uint64_t c = D.cap;
    q.x[0] = D.bd[0 * c + j]; q.x[1] = D.bd[1 * c + j]; q.x[2] = D.bd[2 * c + j];
    q.u[0] = D.bd[3 * c + j]; q.u[1] = D.bd[4 * c + j]; q.u[2] = D.bd[5 * c + j];
    q.t = D.bd[6 * c + j]; q.w = D.bd[7 * c + j];
    q.g = (int32_t)D.bi[0 * c + j]; q.cell = (int32_t)D.bi[1 * c + j]; q.ci = (int32_t)D.bi[2 * c + j];
    q.tag = D.bi[3 * c + j]; q.k = D.bi[4 * c + j]; q.seq = D.bi[5 * c + j];
    q.alive = true;
}

MCDC_DEV void bstore(const BDev &D, uint64_t j, const Part &q) {
    const uint64_t c = D.cap;
    D.bd[0 * c + j] = q.x[0]; D.bd[1 * c + j] = q.x[1]; D.bd[2 * c + j] = q.x[2];
    D.bd[3 * c + j] = q.u[0]; D.bd[4 * c + j] = q.u[1]; D.bd[5 * c + j] = q.u[2];
    D.bd[6 * c + j] = q.t; D.bd[7 * c + j] = q.w;
    D.bi[0 * c + j] = (uint32_t)q.g; D.bi[1 * c + j] = (uint32_t)q.cell; D.bi[2 * c + j] = (uint32_t)q.ci;
    D.bi[3 * c + j] = q.tag; D.bi[4 * c + j] = q.k; D.bi[5 * c + j] = q.seq;
}

// Plan step `step`: per-problem chunk counts and prefix sums (one workgroup).
// Step s reads queue buffer s % 2 (written by step s-1) and appends census
// survivors to buffer (s + 1) % 2; step 0 reads the histories themselves.
__global__ void __launch_bounds__(1024) k_b_plan(BDev D, uint32_t step) {
    __shared__ uint32_t scan[1024];
    __shared__ uint32_t carry;
    BCtl *c = D.ctl;
    const uint32_t cur = step & 1u;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < D.n_prob; base += blockDim.x) {
        const uint32_t p = base + threadIdx.x;
        uint32_t n = 0;
        if (p < D.n_prob) n = step == 0 ? D.probs[p].n_hist : D.nq[cur * D.n_prob + p];
        const uint32_t ch = (n + D.chunk - 1) / D.chunk;
        scan[threadIdx.x] = ch;
        __syncthreads();
        for (uint32_t off = 1; off < blockDim.x; off <<= 1) {
            const uint32_t v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0u;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        if (p < D.n_prob) D.chunk_off[p] = carry + scan[threadIdx.x] - ch;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += scan[threadIdx.x];
        __syncthreads();
    }
    // next-step queue (the other buffer) starts empty
    for (uint32_t p = threadIdx.x; p < D.n_prob; p += blockDim.x) D.nq[(cur ^ 1u) * D.n_prob + p] = 0u;
    if (threadIdx.x == 0) {
        D.chunk_off[D.n_prob] = carry;
        c->total_chunks = carry;
        c->chunk_next = 0;
        c->step = step;
    }
}

// Four waves per SIMD (at most 128 VGPRs): with three, the 256-problem batch
// runs at 2.07e9 histories/s instead of 2.70e9.
template <bool TILE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_b_persistent(BDev D) {
    extern __shared__ double s_tile[];
    __shared__ Shared S;
    __shared__ uint32_t s_chunk, s_cancel, s_entry;
    const BCtl *c = D.ctl;
    const uint32_t step = c->step, cur = step & 1u, total = c->total_chunks;
    RunArgs A{};
    A.seed = c->seed;
    int tile_p = -1;
    shared_zero(S);
    if (threadIdx.x == 0) s_cancel = 0u;
    __syncthreads();
    for (uint32_t fetch = 0;; ++fetch) {
        if (threadIdx.x == 0) {
            // the host's cancel word, every eighth chunk of this workgroup
            if (fetch % 8u == 0u && cancel_requested(D.cancel)) s_cancel = 1u;
            s_chunk = s_cancel ? total : atomicAdd(&D.ctl->chunk_next, 1u);
        }
        __syncthreads();
        const uint32_t ch = s_chunk;
        __syncthreads();
        if (ch >= total) break;
        // problem of this chunk: last p with chunk_off[p] <= ch (uniform)
        uint32_t lo = 0, hi = D.n_prob;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (D.chunk_off[mid] <= ch) lo = mid; else hi = mid;
        }
        const int p = __builtin_amdgcn_readfirstlane((int)lo);
        const BProb &BP = D.probs[p];
        // the problem array is not written during the launch
        CP &P = *(CP *)(uintptr_t)&BP.P;
        if (p != tile_p) {
            if (tile_p >= 0) {
                __syncthreads();
                const BProb &OP = D.probs[tile_p];
                if (TILE && OP.slice) {
                    double *g = D.tally + OP.tally_off + (uint64_t)step * OP.slice;
                    for (uint32_t i = threadIdx.x; i < OP.slice; i += blockDim.x) {
                        const double v = s_tile[i];
                        if (v != 0.0) unsafeAtomicAdd(g + i, v);
                    }
                }
                shared_flush(S, &D.acc[tile_p]);
                __syncthreads();
                shared_zero(S);
            }
            if (TILE && BP.slice)
                for (uint32_t i = threadIdx.x; i < BP.slice; i += blockDim.x) s_tile[i] = 0.0;
            tile_p = p;
            __syncthreads();
        }
        A.acc = &D.acc[p];
        const uint32_t n = step == 0 ? BP.n_hist : D.nq[cur * D.n_prob + p];
        const uint32_t e0 = (ch - D.chunk_off[p]) * D.chunk;
        const uint32_t e1 = e0 + D.chunk < n ? e0 + D.chunk : n;
        TileTally tally{(lds_f64 *)s_tile, (hbm_f64 *)(D.tally + BP.tally_off),
                        TILE && BP.slice ? step * BP.slice : 0u,
                        TILE && BP.slice ? (step + 1) * BP.slice : 0u};
        uint32_t n_flight = 0, n_piece = 0, n_new = 0;
        double path = 0.0;
        // work-items take the chunk's entries one at a time from a counter in
        // LDS and run one flight per loop turn: a lane whose particle ends (or
        // reaches the census) takes the next entry while the others fly on,
        // instead of the wave waiting for its longest history per entry
        if (threadIdx.x == 0) s_entry = e0;
        __syncthreads();
        const uint32_t nxt = cur ^ 1u;
        Part q;
        q.alive = false;
        uint32_t local = 0;
        for (;;) {
            if (!q.alive) {
                const uint32_t e = atomicAdd(&s_entry, 1u);
                if (e >= e1) break;
                if (step == 0) {
                    local = e;
                    BatchCtx C{P, A, D, D.hist_base[p] + local, BP.bank_off + local};
                    D.bd[8 * D.cap + C.slot] = 0.0;
                    D.bi[6 * D.cap + C.slot] = 0u;
                    n_new += 1;
                    stage_source(P, A, S, C, q);
                    if (!q.alive) continue;
                } else {
                    local = D.q[(uint64_t)cur * D.cap + BP.bank_off + e];
                    bload(D, BP.bank_off + local, q);
                }
            }
            BatchCtx C{P, A, D, D.hist_base[p] + local, BP.bank_off + local};
            double d;
            const int ev = stage_flight(P, A, S, tally, C, q, d, n_piece, path);
            if (ev >= 0) n_flight += 1;
            if (!q.alive) continue;
            if (ev == EV_SURFACE) {
                stage_surface(P, A, S, C, q, d);
            } else if (ev == EV_SCATTER) {
                stage_collision(P, A, S, C, q, d);
            } else if (ev == EV_CENSUS) {
                // census survivor: its problem-local index into the next queue
                bstore(D, BP.bank_off + local, q);
                const uint32_t pos = wave_reserve_one(&D.nq[nxt * D.n_prob + p]);
                D.q[(uint64_t)nxt * D.cap + BP.bank_off + pos] = local;
                q.alive = false;
            }
        }
        __syncthreads();                      // the chunk's entries are done before s_entry is reused
        if (n_new) atomicAdd(&S.cnt[C_HIST], (unsigned long long)n_new);
        atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
        atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
        atomicAdd(&S.wsum[W_PATH], path);
    }
    __syncthreads();
    if (tile_p >= 0) {
        const BProb &OP = D.probs[tile_p];
        if (TILE && OP.slice) {
            double *g = D.tally + OP.tally_off + (uint64_t)step * OP.slice;
            for (uint32_t i = threadIdx.x; i < OP.slice; i += blockDim.x) {
                const double v = s_tile[i];
                if (v != 0.0) unsafeAtomicAdd(g + i, v);
            }
        }
        shared_flush(S, &D.acc[tile_p]);
    }
    if (s_cancel)
        for (uint32_t i = threadIdx.x; i < D.n_prob; i += blockDim.x)
            atomicMin(&D.acc[i].status, (int)MCDC_E_CANCELLED);
}

// close-out of one pass (one batch per problem): flattened over all bins
__global__ void k_b_closeout(BDev D) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D.total_bins; i += stride) {
        const double sb = D.tally[i];
        if (sb == 0.0) continue;
        uint32_t lo = 0, hi = D.n_prob;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (D.probs[mid].tally_off <= i) lo = mid; else hi = mid;
        }
        const double nb = (double)D.probs[lo].n_hist;
        D.tsum[i] = D.tsum[i] + sb;
        D.tsumsq[i] = D.tsumsq[i] + sb * sb / nb;
        D.tally[i] = 0.0;
    }
}

__global__ void k_b_advance(BDev D) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < D.n_prob; p += gridDim.x * blockDim.x) {
        D.hist_base[p] += D.probs[p].n_hist;
    }
}

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct BLayout {
    size_t probs, tables, tally, tsum, tsumsq, acc, bd, bi, q, nq, chunk_off, hist_base, ctl, total;
};

static BLayout blayout(const mcdc_problem_desc *ds, size_t n, const uint64_t *nh) {
    BLayout L;
    size_t off = 0, ntab = 0, nbins = 0;
    uint64_t cap = 0;
    for (size_t p = 0; p < n; ++p) {
        const mcdc_problem_desc *d = &ds[p];
        ntab += (size_t)d->n_mat * d->G + (size_t)d->n_mat * d->G * d->G + d->G + d->n_census;
        nbins += (size_t)(d->mesh_per_group ? d->G : 1) * d->mesh_n[0] * d->mesh_n[1] * d->mesh_n[2] * d->mesh_n[3];
        cap += nh[p];
    }
    L.probs = off; off = al(off + n * sizeof(BProb));
    L.tables = off; off = al(off + ntab * sizeof(double));
    L.tally = off; off = al(off + nbins * sizeof(double));
    L.tsum = off; off = al(off + nbins * sizeof(double));
    L.tsumsq = off; off = al(off + nbins * sizeof(double));
    L.acc = off; off = al(off + n * sizeof(DevAcc));
    L.bd = off; off = al(off + 10 * cap * sizeof(double));
    L.bi = off; off = al(off + 7 * cap * sizeof(uint32_t));
    L.q = off; off = al(off + 2 * cap * sizeof(uint32_t));
    L.nq = off; off = al(off + 2 * n * sizeof(uint32_t));
    L.chunk_off = off; off = al(off + (n + 1) * sizeof(uint32_t));
    L.hist_base = off; off = al(off + n * sizeof(uint64_t));
    L.ctl = off; off = al(off + sizeof(BCtl));
    L.total = off;
    return L;
}

static int bvalidate(const mcdc_problem_desc *ds, size_t n, const uint64_t *nh) {
    if (!ds || !nh || n == 0) return fail(MCDC_E_INVALID, "empty batch");
    if (n > (size_t)kBatchMaxProblems) return fail(MCDC_E_INVALID, "too many problems in a batch");
    const int nc = ds[0].n_census;
    uint64_t cap = 0;
    for (size_t p = 0; p < n; ++p) {
        int st = validate_desc(&ds[p]);
        if (st) return fail(st, "problem " + std::to_string(p) + ": " + mcdc_last_error());
        if (ds[p].n_census != nc) return fail(MCDC_E_INVALID, "all batched problems need the same number of census steps");
        if (ds[p].imp_on || ds[p].stack_cap > 0) return fail(MCDC_E_INVALID, "batched problems run analog/implicit transport without weight windows");
        if (ds[p].has_detector) return fail(MCDC_E_INVALID, "batched problems have no detector tally");
        if (ds[p].col_tally) return fail(MCDC_E_INVALID, "batched problems have no collision-estimator tally");
        if (ds[p].surf_on) return fail(MCDC_E_INVALID, "batched problems have no surface-current tally");
        if (desc_fissile(&ds[p])) return fail(MCDC_E_INVALID, "batched problems have no fission (k-eigenvalue runs one problem)");
        if (ds[p].pc_on) return fail(MCDC_E_INVALID, "batched problems run without population control");
        if (nh[p] > 0xFFFFFFF0ull) return fail(MCDC_E_INVALID, "too many histories in one problem");
        cap += nh[p];
    }
    if (cap > 0xFFFFFFF0ull) return fail(MCDC_E_INVALID, "too many histories in the batch");
    return MCDC_OK;
}

}  // namespace mcdc

using namespace mcdc;

extern "C" {

int mcdc_batch_workspace_bytes(const mcdc_problem_desc *ds, size_t n, const uint64_t *nh,
                               const mcdc_options *opt, size_t *bytes) {
    int st = bvalidate(ds, n, nh);
    if (st) return st;
    if (!bytes) return fail(MCDC_E_INVALID, "null bytes");
    (void)opt;
    *bytes = blayout(ds, n, nh).total;
    return MCDC_OK;
}

int mcdc_create_batch(const mcdc_problem_desc *ds, size_t n, const uint64_t *nh,
                      const mcdc_options *opt, void *ws, size_t bytes, mcdc_handle *out) {
    int st = bvalidate(ds, n, nh);
    if (st) return st;
    if (!ws || !out) return fail(MCDC_E_INVALID, "null workspace or handle");
    BLayout L = blayout(ds, n, nh);
    if (bytes < L.total) return fail(MCDC_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
    Options o = resolve_options(opt);
    auto *h = new mcdc_problem();
    h->is_batch = true;
    h->desc = ds[0];
    h->opt = o;
    h->ws = (char *)ws;
    auto *B = new BatchState();
    h->batch = B;
    char *w = (char *)ws;
    BDev &D = B->D;
    D.probs = (BProb *)(w + L.probs);
    D.n_prob = (uint32_t)n;
    // histories (or census particles) per work-queue chunk
    D.chunk = (opt && opt->event_chunk > 0) ? (uint32_t)std::min<int64_t>(opt->event_chunk, 1 << 20) : 2048u;
    D.n_steps = (uint32_t)ds[0].n_census;
    D.tally = (double *)(w + L.tally);
    D.tsum = (double *)(w + L.tsum);
    D.tsumsq = (double *)(w + L.tsumsq);
    D.acc = (DevAcc *)(w + L.acc);
    D.bd = (double *)(w + L.bd);
    D.bi = (uint32_t *)(w + L.bi);
    D.q = (uint32_t *)(w + L.q);
    D.nq = (uint32_t *)(w + L.nq);
    D.chunk_off = (uint32_t *)(w + L.chunk_off);
    D.hist_base = (uint64_t *)(w + L.hist_base);
    D.ctl = (BCtl *)(w + L.ctl);
    if ((st = cancel_init(h))) {
        mcdc_destroy_problem(h);
        return st;
    }
    D.cancel = h->cancel_dev;
    std::vector<double> tables;
    uint64_t tally_off = 0, bank_off = 0;
    Layout dummy{};
    for (size_t p = 0; p < n; ++p) {
        const mcdc_problem_desc *d = &ds[p];
        BProb bp;
        memset(&bp, 0, sizeof(bp));
        mcdc_problem_desc dp = *d;
        dp.problem_id = (uint32_t)p;
        dummy.tables = L.tables + tables.size() * sizeof(double);
        dummy.ww_params = 0;
        build_dev_problem(&dp, w, dummy, bp.P);
        std::vector<double> t = pack_tables(&dp);
        tables.insert(tables.end(), t.begin(), t.end());
        bp.tally_off = tally_off;
        bp.bank_off = bank_off;
        bp.n_hist = (uint32_t)nh[p];
        const uint32_t slice = (uint32_t)d->mesh_n[0] * d->mesh_n[1] * d->mesh_n[2];
        // the LDS tile covers time bin s during census step s: only when the
        // time bins are the census steps and the tally is not per group
        bool tile = !d->mesh_per_group && d->mesh_n[3] == d->n_census && slice <= (uint32_t)kTileBins &&
                    d->mesh_lo[3] == 0.0;
        for (int k = 0; tile && k < d->n_census; ++k) {
            const double e = d->mesh_lo[3] + (double)(k + 1) * ((d->mesh_hi[3] - d->mesh_lo[3]) / d->mesh_n[3]);
            if (fabs(e - d->census[k]) > 1e-9 * fabs(d->census[k])) tile = false;
        }
        bp.slice = tile ? slice : 0u;
        tally_off += bp.P.nbins;
        bank_off += nh[p];
        B->host_probs.push_back(bp);
        B->n_hist.push_back(nh[p]);
    }
    D.cap = bank_off;
    D.total_bins = tally_off;
    hipError_t e = hipMemcpy(w + L.probs, B->host_probs.data(), n * sizeof(BProb), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w + L.tables, tables.data(), tables.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(w + L.tally, 0, L.bd - L.tally);
    if (e == hipSuccess) e = hipMemset(w + L.nq, 0, L.total - L.nq);
    if (e == hipSuccess) e = hipHostMalloc((void **)&B->host_seed, sizeof(double) * 2, hipHostMallocDefault);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mcdc_destroy_problem(h);
        return hip_fail(e, "create_batch");
    }
    // 512 work-items per workgroup: with the 64 KiB time-slice tile two
    // workgroups (16 waves) fit one CU's 160 KiB of LDS
    B->block = 512;
    B->grid = history_grid(512, o.waves_per_cu);
    *out = h;
    return MCDC_OK;
}

}  // extern "C"

namespace mcdc {

static hipError_t enqueue_pass(BatchState *B, hipStream_t s) {
    const BDev &D = B->D;
    bool any_tile = false;
    for (auto &bp : B->host_probs) any_tile |= bp.slice != 0;
    const size_t shm = any_tile ? (size_t)kTileBins * sizeof(double) : 0;
    for (uint32_t step = 0; step < D.n_steps; ++step) {
        hipLaunchKernelGGL(k_b_plan, dim3(1), dim3(1024), 0, s, D, step);
        if (any_tile) hipLaunchKernelGGL((k_b_persistent<true>), dim3(B->grid), dim3(B->block), shm, s, D);
        else hipLaunchKernelGGL((k_b_persistent<false>), dim3(B->grid), dim3(B->block), 0, s, D);
    }
    int cg = (int)((D.total_bins + 255) / 256);
    if (cg > 8192) cg = 8192;
    hipLaunchKernelGGL(k_b_closeout, dim3(cg < 1 ? 1 : cg), dim3(256), 0, s, D);
    hipLaunchKernelGGL(k_b_advance, dim3((D.n_prob + 255) / 256), dim3(256), 0, s, D);
    return hipGetLastError();
}

void batch_destroy(mcdc_problem *h) {
    if (!h->batch) return;
    BatchState *B = h->batch;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->host_seed) (void)hipHostFree(B->host_seed);
    delete B;
    h->batch = nullptr;
}

}  // namespace mcdc

extern "C" {

int mcdc_run_batch(mcdc_handle h, uint64_t seed, void *stream) {
    if (!h || !h->is_batch || !h->batch) return fail(MCDC_E_STATE, "not a batched handle");
    BatchState *B = h->batch;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    // the seed reaches the graph through device memory
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "run_batch");
    memcpy(B->host_seed, &seed, sizeof(seed));
    e = hipMemcpyAsync(&B->D.ctl->seed, B->host_seed, sizeof(uint64_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "run_batch seed");
    if (!B->exec) {
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "run_batch capture stream");
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t el = enqueue_pass(B, cs);
            e = hipStreamEndCapture(cs, &B->graph);
            if (e == hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return hip_fail(e, "run_batch graph capture");
    }
    e = hipGraphLaunch(B->exec, s);
    if (e != hipSuccess) return hip_fail(e, "run_batch graph launch");
    B->passes += 1;
    if (cancel_set(h)) return fail(MCDC_E_CANCELLED, "run cancelled");
    return MCDC_OK;
}

static int batch_check(mcdc_handle h, size_t p) {
    if (!h || !h->is_batch || !h->batch) return fail(MCDC_E_STATE, "not a batched handle");
    if (p >= h->batch->D.n_prob) return fail(MCDC_E_INVALID, "problem index out of range");
    return MCDC_OK;
}

int mcdc_get_batch_raw(mcdc_handle h, size_t p, double *tsum, size_t n, void *stream) {
    int st = batch_check(h, p);
    if (st) return st;
    BatchState *B = h->batch;
    const BProb &bp = B->host_probs[p];
    if (n != bp.P.nbins) return fail(MCDC_E_INVALID, "wrong bin count");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpy(tsum, B->D.tsum + bp.tally_off, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_batch_raw");
    return MCDC_OK;
}

int mcdc_get_batch_counters(mcdc_handle h, size_t p, mcdc_counters *out, void *stream) {
    int st = batch_check(h, p);
    if (st) return st;
    if (!out) return fail(MCDC_E_INVALID, "null counters");
    BatchState *B = h->batch;
    DevAcc acc;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipMemcpy(&acc, B->D.acc + p, sizeof(DevAcc), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_batch_counters");
    memset(out, 0, sizeof(*out));
    fill_counters(acc, out);
    out->batches = (int64_t)B->passes;
    out->n_hist = B->passes * B->n_hist[p];
    return MCDC_OK;
}

// Per-history sum of w*d of problem p for the histories of the last pass.
int mcdc_get_batch_history_path(mcdc_handle h, size_t p, double *out, size_t n, void *stream) {
    int st = batch_check(h, p);
    if (st) return st;
    BatchState *B = h->batch;
    const BProb &bp = B->host_probs[p];
    if (n != bp.n_hist) return fail(MCDC_E_INVALID, "wrong history count");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpy(out, B->D.bd + 8 * B->D.cap + bp.bank_off, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "get_batch_history_path");
    return MCDC_OK;
}

}  // extern "C"
