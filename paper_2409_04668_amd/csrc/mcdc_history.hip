// History-based tracking kernel: one work-item carries one history (its source
// particle and, with weight windows, its split daughters on a LIFO stack) from
// birth to the end, flight by flight.  The grid is persistent (a fixed number
// of workgroups sized to the chip); each workgroup takes a contiguous range of
// the launch's history ids and its work-items take the next one from a
// counter in LDS, so a work-item whose history ends starts its next history
// in the same loop iteration instead of idling until the wave drains, and a
// long history holds up no other history.
//
// Tallies: track-length pieces go to FP64 atomics, either straight into the
// batch accumulator in HBM or, when the whole mesh fits, into an LDS tile per
// workgroup that is flushed with one global atomic per touched bin at the end.
#include "lane_stack.hpp"
#include "transport_stages.hpp"

namespace mcdc {

// Per-work-item history context (registers).  WW: 0 no weight windows,
// 1 network evaluated at each check, 2 baked window map.  FIS: a generation
// of the k-eigenvalue mode (fission sites recorded with their history slot
// and ordinal).
template <int WW, bool IMP, bool FIS = false>
struct HistCtx {
    static constexpr bool kWW = WW != 0;
    static constexpr bool kWWMap = WW == 2;
    static constexpr bool kFis = FIS;
    // the fission variants sit at their register limit
    static constexpr bool kTightRegs = FIS;
    CP &P;
    const RunArgs &A;
    uint64_t lane;
    uint64_t id;
    double xh, path;
    int64_t events;
    int sp, n_imp;
    uint32_t n_site;
    double k_norm = 0.0;                 // the generation's normalisation (fission variants)

    // fission site `pos` of the generation's bank (in reservation order;
    // past the capacity it is dropped and the host reports the overflow)
    MCDC_DEV void put_site(const Part &q, int g, uint32_t pos) {
        const uint32_t ord = n_site;
        n_site += 1;
        if (pos >= A.site_cap) return;
        const uint64_t c = A.site_cap;
        A.site_d[pos] = q.x[0];
        A.site_d[c + pos] = q.x[1];
        A.site_d[2 * c + pos] = q.x[2];
        A.site_g[pos] = g;
        A.site_key[pos] = (uint32_t)(id - A.gen_first);
        A.site_key[c + pos] = ord;
    }

    MCDC_DEV uint64_t hist() const { return id; }
    MCDC_DEV double *col_tally() const { return A.col; }
    MCDC_DEV double *surf_tally() const { return A.surf; }
    MCDC_DEV const float *mlp_params(CP &Pp) const { return Pp.ww_params; }
    MCDC_DEV bool count_flight() {
        events += 1;
        return events <= P.max_events;
    }
    MCDC_DEV void add_score(double v) { xh += v; }
    MCDC_DEV void add_path(double v) { path += v; }
    MCDC_DEV bool push_daughters(const Part &q, uint32_t tag0, int n) {
        for (int i = 1; i < n; ++i) {
            if (sp >= P.stack_cap) {
                set_status(A, MCDC_E_STACK);
                return false;
            }
            Part d = q;
            d.tag = tag0 + (uint32_t)i * 0x9E3779B9u;
            d.k = 0;
            d.seq = 0;
            stack_push(A, lane, P.stack_cap, sp, d);
            sp += 1;
        }
        return true;
    }
    // forward importance estimate: record the score so far at each flight
    // start, per distinct coarse cell (at most kImpList cells per history)
    MCDC_DEV void imp_point(CP &Pp, const Part &q) {
        if (!IMP) return;
        int ix[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double x = a < 3 ? q.x[a] : q.t;
            const double f = (x - Pp.imp_lo[a]) * Pp.imp_f[a];
            int i = (int)floor(f);
            if (i < 0) i = 0;
            if (i > Pp.imp_n[a] - 1) i = Pp.imp_n[a] - 1;
            ix[a] = i;
        }
        int c = q.g;
        c = c * Pp.imp_n[3] + ix[3];
        c = c * Pp.imp_n[2] + ix[2];
        c = c * Pp.imp_n[1] + ix[1];
        c = c * Pp.imp_n[0] + ix[0];
        const uint64_t L = A.n_lanes;
        for (int i = 0; i < n_imp; ++i) {
            if (A.imp_cell[i * L + lane] == c) {
                A.imp_cnt[i * L + lane] += 1.0;
                A.imp_xsum[i * L + lane] += xh;
                return;
            }
        }
        if (n_imp < kImpList) {
            A.imp_cell[n_imp * L + lane] = c;
            A.imp_cnt[n_imp * L + lane] = 1.0;
            A.imp_xsum[n_imp * L + lane] = xh;
            n_imp += 1;
        }
    }
};

template <int WW, bool IMP, bool FIS>
MCDC_DEV void finish_history(const RunArgs &A, Shared &S, const HistCtx<WW, IMP, FIS> &H) {
    if (FIS) A.hist_sites[H.id - A.gen_first] = H.n_site;
    if (FIS && A.det_off) {
        // an inactive generation: its detector scores are discarded
    } else {
        if (H.xh != 0.0) {
            unsafeAtomicAdd(&A.acc->det[0], H.xh);
            unsafeAtomicAdd(&A.acc->det[1], H.xh * H.xh);
        }
        if (H.xh > 0.0) atomicAdd(&S.cnt[C_DET_HIT], 1ull);
    }
    if (A.xh_out) {
        A.xh_out[2 * (H.id - A.h_run0)] = H.xh;
        A.xh_out[2 * (H.id - A.h_run0) + 1] = H.path;
    }
    if (IMP) {
        const uint64_t L = A.n_lanes;
        for (int i = 0; i < H.n_imp; ++i) {
            const int c = A.imp_cell[i * L + H.lane];
            const double cnt = A.imp_cnt[i * L + H.lane];
            unsafeAtomicAdd(&A.imp_score[c], cnt * H.xh - A.imp_xsum[i * L + H.lane]);
            unsafeAtomicAdd(&A.imp_weight[c], cnt);
        }
    }
}

// LDS modes: 0 = tally in HBM, 1 = whole mesh in LDS, 2 = hot tile in LDS.
template <int LDS>
struct TallyFor { using type = GlobalTally; };
template <>
struct TallyFor<1> { using type = LdsTally; };
template <>
struct TallyFor<2> { using type = HotTileTally; };

MCDC_DEV GlobalTally make_tally(GlobalTally *, CP &, const RunArgs &A, double *) {
    return GlobalTally{A.tally};
}
MCDC_DEV LdsTally make_tally(LdsTally *, CP &, const RunArgs &, double *lds) {
    return LdsTally{(lds_f64 *)lds};
}
MCDC_DEV HotTileTally make_tally(HotTileTally *, CP &P, const RunArgs &A, double *lds) {
    HotTileTally t;
    t.lds = (lds_f64 *)lds;
    t.glob = (hbm_f64 *)A.tally;
    t.prob = &P;
    t.n0 = P.hot_n[0];
    return t;
}

template <int LDS, int WW, bool IMP, bool FIS>
__global__ void __launch_bounds__(LDS == 2 ? 1024 : 256) k_history(DevProblem, RunArgs A) {
    CP &P = kernel_problem();
    // a k-eigenvalue generation after a failed one (its source would come from
    // sites that were never made) transports nothing
    if (FIS && A.acc->status != 0) return;
    extern __shared__ double s_tile[];
    __shared__ Shared S;
    __shared__ uint32_t s_cancel;
    __shared__ unsigned long long s_next;
    const CancelSeen cancel{&s_cancel};
    shared_zero(S);
    cancel.init(A.cancel);
    const uint32_t tile_bins = LDS == 1 ? P.nbins : (LDS == 2 ? P.hot_bins : 0u);
    for (uint32_t i = threadIdx.x; i < tile_bins; i += blockDim.x) s_tile[i] = 0.0;
    // workgroup w takes the contiguous histories [w n / G, (w+1) n / G) of
    // the launch; its work-items take the next one from a counter in LDS as
    // their histories end, so a long history delays no other work-item's next
    // (floor(b n / G) = b q + floor(b r / G) with n = q G + r, without overflow)
    const uint64_t n_all = A.h_end - A.h_begin;
    const uint64_t q_all = n_all / gridDim.x, r_all = n_all % gridDim.x;
    const uint64_t b1 = blockIdx.x + 1u;
    const uint64_t h1 = A.h_begin + b1 * q_all + (b1 * r_all) / gridDim.x;
    if (threadIdx.x == 0)
        s_next = A.h_begin + blockIdx.x * q_all + ((uint64_t)blockIdx.x * r_all) / gridDim.x;
    __syncthreads();

    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n_flight = 0, n_piece = 0, n_hist = 0;
    double path = 0.0;
    Part q;
    q.alive = false;
    HistCtx<WW, IMP, FIS> H{P, A, lane, 0, 0.0, 0.0, 0, 0, 0, 0u};
    // read once: the kernel's own writes could otherwise alias it at every use
    if constexpr (FIS) H.k_norm = *A.k_norm;
    bool in_hist = false;
    using Tally = typename TallyFor<LDS>::type;
    const Tally tally = make_tally((Tally *)nullptr, P, A, s_tile);

    bool ww_due = false;                    // a weight-window check waits for this lane
    for (;;) {
        CP &PL = problem_reload(P);
        if (WW == 1) {
            // Weight-window checks run batched: a lane that needs one waits
            // (its particle does not move) until at least half of the wave's
            // active lanes wait, then they evaluate the network together.
            // The check sees exactly the state it would have seen at once.
            const uint64_t due = __ballot(ww_due);
            if (due && 2 * __popcll(due) >= __popcll(__ballot(true))) {
                if (ww_due) {
                    ww_check(PL, A, S, H, q);
                    ww_due = false;
                }
                continue;
            }
            if (ww_due) continue;
        }
        if (!q.alive) {
            if (WW && H.sp > 0) {
                H.sp -= 1;
                stack_pop(A, lane, PL.stack_cap, H.sp, q);
            } else {
                if (in_hist) {
                    finish_history(A, S, H);
                    in_hist = false;
                }
                if (cancel.check(A.cancel, n_hist)) {
                    set_status(A, MCDC_E_CANCELLED);
                    break;
                }
                const uint64_t next = atomicAdd(&s_next, 1ull);
                if (next >= h1) break;
                H.id = next;
                H.xh = 0.0;
                H.path = 0.0;
                H.events = 0;
                H.sp = 0;
                H.n_imp = 0;
                H.n_site = 0;
                in_hist = true;
                n_hist += 1;
                if (FIS && A.src_d != nullptr) stage_source_site(PL, A, S, H, q, H.id - A.gen_first);
                else stage_source(PL, A, S, H, q);
                if (!q.alive) continue;
            }
        }
        double d;
        const int ev = stage_flight(PL, A, S, tally, H, q, d, n_piece, path);
        if (ev == EV_SURFACE) {
            ww_due = stage_surface(PL, A, S, H, q, d);
        } else if (ev == EV_SCATTER) {
            ww_due = stage_collision(PL, A, S, H, q, d);
        } else if (ev == EV_WW_PLANE) {
            ww_due = true;
        } else if (ev < 0) {
            H.sp = 0;                       // event cap: the history is abandoned
        }
        if (WW == 2 && ww_due) {            // a map read is cheap: check at once
            ww_check(PL, A, S, H, q);
            ww_due = false;
        }
        if (ev >= 0) n_flight += 1;
    }

    atomicAdd(&S.cnt[C_HIST], (unsigned long long)n_hist);
    atomicAdd(&S.cnt[C_FLIGHT], (unsigned long long)n_flight);
    atomicAdd(&S.cnt[C_PIECE], (unsigned long long)n_piece);
    atomicAdd(&S.wsum[W_PATH], path);
    __syncthreads();
    if (LDS == 1) {
        for (uint32_t i = threadIdx.x; i < P.nbins; i += blockDim.x) {
            const double v = s_tile[i];
            if (v != 0.0) unsafeAtomicAdd(&A.tally[i], v);
        }
    } else if (LDS == 2) {
        hot_tile_flush(P, s_tile, A.tally);
    }
    shared_flush(S, A.acc);
}

// Close-out of every batch slice of a run of n histories in B batches at
// once: per bin, for b = 0, 1, ..., B-1, sum += S_b, sumsq += S_b^2 / N_b,
// S_b = 0, with N_b the histories of batch b (empty batches skipped): the
// additions, in the same order, of B single-slice close-outs.
__global__ void k_closeout_run(double *__restrict__ batch, double *__restrict__ sum,
                               double *__restrict__ sumsq, uint32_t n, uint32_t B,
                               uint64_t n_hist) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s = sum[i], s2 = sumsq[i];
        bool touched = false;
        for (uint32_t b = 0; b < B; ++b) {
            const uint64_t lo = (b * n_hist) / B, hi = ((b + 1) * n_hist) / B;
            double *slot = batch + (uint64_t)b * n + i;
            const double sb = *slot;
            if (sb == 0.0 || hi == lo) continue;
            s = s + sb;
            s2 = s2 + sb * sb / (double)(hi - lo);
            *slot = 0.0;
            touched = true;
        }
        if (touched) {
            sum[i] = s;
            sumsq[i] = s2;
        }
    }
}

hipError_t launch_closeout_run(double *batch, double *sum, double *sumsq, uint32_t n, uint32_t B,
                               uint64_t n_hist, hipStream_t s) {
    const int block = 256;
    int grid = (int)((n + block - 1) / block);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_closeout_run, dim3(grid), dim3(block), 0, s, batch, sum, sumsq, n, B, n_hist);
    return hipGetLastError();
}

// The kernels read the problem description through kernel_problem(), the
// address of their first argument in the kernel-argument segment.  This
// kernel reads a few fields by name and through that address: *out = 1 when
// they agree (checked once per handle).
__global__ void k_problem_check(DevProblem P, int *out) {
    CP &K = kernel_problem();
    *out = (K.problem_id == P.problem_id && K.nbins == P.nbins && K.n_census == P.n_census &&
            K.G == P.G && K.mesh_n[3] == P.mesh_n[3] && K.max_events == P.max_events &&
            K.hot_bins == P.hot_bins) ? 1 : 0;
}

hipError_t launch_problem_check(const DevProblem &P, int *out, hipStream_t s) {
    hipLaunchKernelGGL(k_problem_check, dim3(1), dim3(1), 0, s, P, out);
    return hipGetLastError();
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

// Each workgroup of the history kernel takes a fixed contiguous range of
// histories, so workgroups beyond those the GPU holds at once would run
// their whole ranges in a second, partly filled round: the grid is capped at
// the workgroups of this kernel that are resident together (its occupancy,
// which its registers and LDS set, times the compute units).
static int resident_grid(const void *k, int grid, int block, size_t shm) {
    int dev = 0, per_cu = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, shm) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return grid;
    }
    const int cap = per_cu * n_cu;
    return cap > 0 && cap < grid ? cap : grid;
}

hipError_t launch_history(const DevProblem &P, const RunArgs &A, int grid, int block,
                          bool lds_tally, hipStream_t s) {
    const int mode = P.hot_bins ? 2 : (lds_tally ? 1 : 0);
    const size_t shm = mode == 2 ? (size_t)P.hot_bins * sizeof(double)
                                 : (mode == 1 ? (size_t)P.nbins * sizeof(double) : 0);
    const int ww = P.ww_on ? (P.ww_map ? 2 : 1) : 0;
    const bool imp = P.imp_on != 0;
#define MCDC_LAUNCH_F(L, W, I, F)                                                              \
    do {                                                                                       \
        const void *kf = (const void *)k_history<L, W, I, F>;                                  \
        if (shm > 65536)                                                                       \
            (void)hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm); \
        const int g = resident_grid(kf, grid, block, shm);                                     \
        hipLaunchKernelGGL((k_history<L, W, I, F>), dim3(g), dim3(block), shm, s, P, A);       \
    } while (0)
#define MCDC_LAUNCH(L, W, I) MCDC_LAUNCH_F(L, W, I, false)
    if (P.fis_on) {
        // a k-eigenvalue generation (no weight windows, no importance estimate)
        if (mode == 2) MCDC_LAUNCH_F(2, 0, false, true);
        else if (mode == 1) MCDC_LAUNCH_F(1, 0, false, true);
        else MCDC_LAUNCH_F(0, 0, false, true);
    } else if (mode == 2) {
        if (ww == 2) MCDC_LAUNCH(2, 2, false);
        else if (ww == 1) MCDC_LAUNCH(2, 1, false);
        else if (imp) MCDC_LAUNCH(2, 0, true);
        else MCDC_LAUNCH(2, 0, false);
    } else if (mode == 1) {
        if (ww == 2) MCDC_LAUNCH(1, 2, false);
        else if (ww == 1) MCDC_LAUNCH(1, 1, false);
        else if (imp) MCDC_LAUNCH(1, 0, true);
        else MCDC_LAUNCH(1, 0, false);
    } else {
        if (ww == 2) MCDC_LAUNCH(0, 2, false);
        else if (ww == 1) MCDC_LAUNCH(0, 1, false);
        else if (imp) MCDC_LAUNCH(0, 0, true);
        else MCDC_LAUNCH(0, 0, false);
    }
#undef MCDC_LAUNCH
#undef MCDC_LAUNCH_F
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
