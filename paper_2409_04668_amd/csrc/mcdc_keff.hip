// k-eigenvalue mode: power iteration on the fission source (the paper's second
// simulation mode beside the time-dependent one; fission as a physical event
// and daughter particles from fission in its kernel set).
//
// One generation of M histories is one launch of the history kernel in its
// fission variant.  A fission collision reserves its sites with one atomic
// per wave and writes them in any order, each with its key (history slot,
// ordinal within the history); the history's site count goes to hist_sites.
// The production order the comb needs (by history slot, then in the order a
// history made them) is restored without a sort: an exclusive scan of the
// per-slot counts gives every slot its first position, and each site moves to
// slot offset + ordinal.  The comb then picks M sites with one random offset;
// its index arithmetic is the definition's, so the next generation starts
// from exactly the sites a serial implementation picks.
//
// The normalisation k_norm, the site count and the per-generation estimates
// stay on the device (k_keff_gen_end), so generations follow each other
// without a host round trip; the host reads a block of kGenBlock generations'
// results at a time.
#include <string>

#include "mcdc_runtime.hpp"
#include "transport_device.hpp"

namespace mcdc {

constexpr uint32_t kCombTag = 0x6B656666u;       // stream tag of the comb's draw
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                     // counts per work-item
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr uint64_t kKeffMaxM = 1ull << 28;
constexpr int kGenBlock = 64;                    // generations per host read-back

// per generation, written by k_keff_gen_end
struct KeffOut {
    double k_col, k_site;
    uint64_t n_sites;
    int32_t status;                              // the run's status after the generation
    int32_t pad;
};

struct KeffCtl {
    uint32_t site_n;                             // sites reserved by the generation
    uint32_t stop;                               // a generation failed: order and comb do nothing
    uint64_t total;                              // sum of the per-slot counts
    double k_norm;                               // normalisation of the running generation
    uint64_t pad2;
    KeffOut out[kGenBlock];                      // generation g at out[g % kGenBlock]
};

struct KeffLayout {
    size_t site_d, site_g, site_key, ord_d, ord_g, src_d, src_g, hist_sites, hist_off, bsum, ctl,
        total;
    uint64_t cap, nblk;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static KeffLayout keff_layout(uint64_t M) {
    KeffLayout L;
    L.cap = 4 * M + 1024;
    L.nblk = (M + kScanTile - 1) / kScanTile;
    size_t off = 0;
    L.site_d = off; off = al256(off + 3 * L.cap * sizeof(double));
    L.site_g = off; off = al256(off + L.cap * sizeof(int32_t));
    L.site_key = off; off = al256(off + 2 * L.cap * sizeof(uint32_t));
    L.ord_d = off; off = al256(off + 3 * L.cap * sizeof(double));
    L.ord_g = off; off = al256(off + L.cap * sizeof(int32_t));
    L.src_d = off; off = al256(off + 3 * M * sizeof(double));
    L.src_g = off; off = al256(off + M * sizeof(int32_t));
    L.hist_sites = off; off = al256(off + M * sizeof(uint32_t));
    L.hist_off = off; off = al256(off + M * sizeof(uint32_t));
    L.bsum = off; off = al256(off + L.nblk * sizeof(uint32_t));
    L.ctl = off; off = al256(off + sizeof(KeffCtl));
    L.total = off;
    return L;
}

// start of a run: the first generation's normalisation
__global__ void k_keff_run_begin(KeffCtl *ctl, double k0) {
    if (threadIdx.x == 0) {
        ctl->k_norm = k0;
        ctl->stop = 0u;
    }
}

// start of a generation: no sites yet, collision estimate zero
__global__ void k_keff_gen_begin(KeffCtl *ctl, DevAcc *acc) {
    if (threadIdx.x == 0) {
        ctl->site_n = 0u;
        acc->kcol = 0.0;
    }
}

// end of generation g (after the site-count scan): its estimates
// k_col = (sum of w nuSigma_f / Sigma_t) / M and k_site = k_norm S / M, its
// site count S and the run's status after it, and the next generation's
// normalisation k_site.  A generation with more sites than the bank holds,
// or with none, sets the status unless an earlier failure did; after any
// failure the normalisation is infinite, so later generations make no sites
// (the host reports the first failure at its next read-back).
__global__ void k_keff_gen_end(KeffCtl *ctl, DevAcc *acc, uint64_t M, uint64_t cap, uint32_t g) {
    if (threadIdx.x != 0) return;
    const uint64_t S = ctl->total;
    KeffOut &o = ctl->out[g % kGenBlock];
    o.k_col = acc->kcol / (double)M;
    o.k_site = ctl->k_norm * (double)S / (double)M;
    o.n_sites = S;
    int st = acc->status;
    if (st == 0) {
        if (ctl->site_n > cap || S > cap) st = MCDC_E_BANK;
        else if (S != ctl->site_n) st = MCDC_E_HIP;
        else if (S == 0) st = MCDC_E_EXTINCT;
        if (st != 0) atomicMin(&acc->status, st);
    }
    o.status = st;
    ctl->k_norm = st == 0 ? o.k_site : __builtin_inf();
    // a generation whose history launch stopped early (or never ran) left
    // site keys and counts that are not its own
    if (st != 0) ctl->stop = 1u;
}

__global__ void k_fill_zero(double *__restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

// sum of each tile of kScanTile counts
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const uint32_t *__restrict__ cnt,
                                                             uint64_t n, uint32_t *__restrict__ bsum) {
    __shared__ uint32_t red[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + threadIdx.x + (uint64_t)k * kScanThreads;
        if (i < n) s += cnt[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kScanThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// exclusive scan of the tile sums in place (one workgroup, 1024 at a time),
// the grand total to ctl->total
__global__ void __launch_bounds__(1024) k_scan_top(uint32_t *__restrict__ bsum, uint64_t nblk,
                                                   KeffCtl *ctl) {
    __shared__ uint64_t buf[1024];
    __shared__ uint64_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint64_t c0 = 0; c0 < nblk; c0 += 1024) {
        const uint64_t i = c0 + t;
        const uint64_t v = i < nblk ? bsum[i] : 0u;
        buf[t] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const uint64_t x = t >= o ? buf[t - o] : 0u;
            __syncthreads();
            buf[t] += x;
            __syncthreads();
        }
        if (i < nblk) bsum[i] = (uint32_t)(carry + buf[t] - v);
        __syncthreads();
        if (t == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (t == 0) ctl->total = carry;
}

// per slot: the tile's offset plus the exclusive scan within the tile
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t *__restrict__ cnt,
                                                             uint64_t n,
                                                             const uint32_t *__restrict__ bsum,
                                                             uint32_t *__restrict__ off) {
    __shared__ uint32_t buf[kScanThreads];
    const int t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)t * kScanPer;
    uint32_t loc[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + k;
        loc[k] = s;
        s += i < n ? cnt[i] : 0u;
    }
    buf[t] = s;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint32_t x = t >= o ? buf[t - o] : 0u;
        __syncthreads();
        buf[t] += x;
        __syncthreads();
    }
    const uint32_t excl = bsum[blockIdx.x] + buf[t] - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + k;
        if (i < n) off[i] = excl + loc[k];
    }
}

// every site to its place in production order: slot offset + ordinal (the
// generation's S sites; nothing after a failed generation, and no key or
// place outside the arrays)
__global__ void k_site_order(const double *__restrict__ sd, const int32_t *__restrict__ sg,
                             const uint32_t *__restrict__ key, const uint32_t *__restrict__ off,
                             uint64_t cap, uint64_t M, const KeffCtl *ctl, double *__restrict__ od,
                             int32_t *__restrict__ og) {
    if (ctl->stop) return;
    const uint64_t n = ctl->total < cap ? ctl->total : cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t slot = key[i];
        if (slot >= M) continue;
        const uint64_t dst = (uint64_t)off[slot] + key[cap + i];
        if (dst >= cap) continue;
        od[dst] = sd[i];
        od[cap + dst] = sd[cap + i];
        od[2 * cap + dst] = sd[2 * cap + i];
        og[dst] = sg[i];
    }
}

// the comb: source j of the next generation is site floor((j + xi) S / M)
// (at most S - 1) of S in production order, xi the first draw of the stream
// (seed, history id of the next generation's first history, tag kCombTag)
__global__ void k_site_comb(uint64_t seed, uint64_t comb_hist, uint32_t problem,
                            const double *__restrict__ od, const int32_t *__restrict__ og,
                            uint64_t cap, const KeffCtl *ctl, uint64_t M, double *__restrict__ src_d,
                            int32_t *__restrict__ src_g) {
    if (ctl->stop) return;                       // a failed generation: no next source
    const uint64_t S = ctl->total < cap ? (ctl->total > 0 ? ctl->total : 1) : cap;
    Rng r = make_rng(seed, comb_hist, problem, kCombTag, 0u);
    const double xi = rng_uniform(r);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += stride) {
        uint64_t idx = (uint64_t)floor(((double)j + xi) * (double)S / (double)M);
        if (idx > S - 1) idx = S - 1;
        src_d[j] = od[idx];
        src_d[M + j] = od[cap + idx];
        src_d[2 * M + j] = od[2 * cap + idx];
        src_g[j] = og[idx];
    }
}

static int grid_for(uint64_t n, int block, int max_grid) {
    uint64_t g = (n + block - 1) / block;
    if (g > (uint64_t)max_grid) g = max_grid;
    return g < 1 ? 1 : (int)g;
}

}  // namespace mcdc

using namespace mcdc;

extern "C" {

int mcdc_keff_workspace_bytes(uint64_t M, size_t *bytes) {
    if (!bytes) return fail(MCDC_E_INVALID, "null bytes");
    if (M < 1 || M > kKeffMaxM) return fail(MCDC_E_INVALID, "M must lie in [1, 2^28]");
    *bytes = keff_layout(M).total;
    return MCDC_OK;
}

int mcdc_run_keff(mcdc_handle h, const mcdc_keff_opts *o, uint64_t seed, void *ws, size_t bytes,
                  double *k_col, double *k_site, uint64_t *n_sites, void *stream) {
    if (!h || !o || !ws) return fail(MCDC_E_INVALID, "null argument");
    if (h->is_batch) return fail(MCDC_E_STATE, "batched handle has no k-eigenvalue mode");
    if (!h->P.fis_on) return fail(MCDC_E_STATE, "the problem has no fission data");
    if (h->opt.schedule != MCDC_SCHED_HISTORY)
        return fail(MCDC_E_STATE, "the k-eigenvalue mode runs in the history schedule");
    if (h->P.ww_on || h->desc.imp_on || h->desc.pc_on)
        return fail(MCDC_E_STATE, "the k-eigenvalue mode runs without weight windows, importance "
                                  "estimate or population control");
    if (h->in_run) return fail(MCDC_E_STATE, "a stepped run is in progress");
    if (h->n_hist != 0 || h->batches != 0)
        return fail(MCDC_E_STATE, "the k-eigenvalue mode needs a fresh or reset handle");
    const uint64_t M = o->M;
    if (M < 1 || M > kKeffMaxM) return fail(MCDC_E_INVALID, "M must lie in [1, 2^28]");
    if (o->n_inactive < 0 || o->n_active < 1) return fail(MCDC_E_INVALID, "n_inactive >= 0, n_active >= 1");
    if (!(o->k0 > 0.0) || !isfinite(o->k0)) return fail(MCDC_E_INVALID, "k0 must be positive and finite");
    const int n_gen = o->n_inactive + o->n_active;
    if ((double)n_gen * (double)M >= 0x1p48) return fail(MCDC_E_INVALID, "history ids exhausted (2^48)");
    const KeffLayout K = keff_layout(M);
    if (bytes < K.total) return fail(MCDC_E_NOMEM, "keff workspace too small: need " + std::to_string(K.total));
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    KeffCtl *ctl = (KeffCtl *)(w + K.ctl);
    double *site_d = (double *)(w + K.site_d);
    int32_t *site_g = (int32_t *)(w + K.site_g);
    uint32_t *site_key = (uint32_t *)(w + K.site_key);
    double *ord_d = (double *)(w + K.ord_d);
    int32_t *ord_g = (int32_t *)(w + K.ord_g);
    double *src_d = (double *)(w + K.src_d);
    int32_t *src_g = (int32_t *)(w + K.src_g);
    uint32_t *hist_sites = (uint32_t *)(w + K.hist_sites);
    uint32_t *hist_off = (uint32_t *)(w + K.hist_off);
    uint32_t *bsum = (uint32_t *)(w + K.bsum);
    DevAcc *acc = (DevAcc *)(h->ws + h->L.acc);

    RunArgs A = base_args_for(h, seed);
    A.h_run0 = 0;
    A.gen_m = M;
    A.site_d = site_d;
    A.site_g = site_g;
    A.site_key = site_key;
    A.site_n = &ctl->site_n;
    A.hist_sites = hist_sites;
    A.site_cap = (uint32_t)K.cap;
    double *batch = (double *)(h->ws + h->L.tally_batch);
    double *sum = (double *)(h->ws + h->L.tally_sum);
    double *sumsq = (double *)(h->ws + h->L.tally_sumsq);
    const bool col = h->desc.col_tally != 0, surf = h->desc.surf_on != 0;
    const bool lds = h->opt.lds_tally && h->nbins <= (uint32_t)kLdsTallyMaxBins;
    const int fg = history_grid(256, 8);
    A.k_norm = &ctl->k_norm;
    hipLaunchKernelGGL(k_keff_run_begin, dim3(1), dim3(64), 0, s, ctl, o->k0);
    for (int g = 0; g < n_gen; ++g) {
        const bool score = g >= o->n_inactive;
        A.gen_first = (uint64_t)g * M;
        A.h_begin = A.gen_first;
        A.h_end = A.gen_first + M;
        A.src_d = g > 0 ? src_d : nullptr;
        A.src_g = g > 0 ? src_g : nullptr;
        A.det_off = score ? 0 : 1;
        hipLaunchKernelGGL(k_keff_gen_begin, dim3(1), dim3(64), 0, s, ctl, acc);
        timing_begin(h, s);
        hipError_t e = launch_history(h->P, A, h->opt.grid, h->opt.block, lds, s);
        timing_end(h, s);
        if (e != hipSuccess) return hip_fail(e, "keff generation launch");
        if (score) {
            e = launch_closeout(batch, sum, sumsq, h->nbins, (double)M, s);
            if (e == hipSuccess && col)
                e = launch_closeout((double *)(h->ws + h->L.col_batch), (double *)(h->ws + h->L.col_sum),
                                    (double *)(h->ws + h->L.col_sumsq), h->nbins, (double)M, s);
            if (e == hipSuccess && surf)
                e = launch_closeout((double *)(h->ws + h->L.surf_batch), (double *)(h->ws + h->L.surf_sum),
                                    (double *)(h->ws + h->L.surf_sumsq), h->P.surf_nbins, (double)M, s);
        } else {
            // an inactive generation discards what it scored
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(h->nbins, 256, 8192)), dim3(256), 0, s, batch,
                               (uint64_t)h->nbins);
            if (col)
                hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(h->nbins, 256, 8192)), dim3(256), 0, s,
                                   (double *)(h->ws + h->L.col_batch), (uint64_t)h->nbins);
            if (surf)
                hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(h->P.surf_nbins, 256, 8192)), dim3(256), 0,
                                   s, (double *)(h->ws + h->L.surf_batch), (uint64_t)h->P.surf_nbins);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return hip_fail(e, "keff close-out");
        // production order: per-slot offsets from the site counts
        hipLaunchKernelGGL(k_scan_tiles, dim3((uint32_t)K.nblk), dim3(kScanThreads), 0, s, hist_sites, M,
                           bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, K.nblk, ctl);
        hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)K.nblk), dim3(kScanThreads), 0, s, hist_sites, M,
                           bsum, hist_off);
        hipLaunchKernelGGL(k_keff_gen_end, dim3(1), dim3(64), 0, s, ctl, acc, M, K.cap, (uint32_t)g);
        if (g + 1 < n_gen) {
            hipLaunchKernelGGL(k_site_order, dim3(grid_for(K.cap, 256, 16384)), dim3(256), 0, s, site_d,
                               site_g, site_key, hist_off, K.cap, M, ctl, ord_d, ord_g);
            hipLaunchKernelGGL(k_site_comb, dim3(grid_for(M, 256, fg)), dim3(256), 0, s, seed,
                               (uint64_t)(g + 1) * M, h->P.problem_id, ord_d, ord_g, K.cap, ctl, M, src_d,
                               src_g);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "keff generation");
        // a block of generations done (or the last one): read their results
        if ((g + 1) % kGenBlock != 0 && g + 1 != n_gen && !cancel_set(h)) continue;
        const int g0 = g - g % kGenBlock;
        KeffOut res[kGenBlock];
        e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipMemcpy(res, ctl->out, sizeof(res), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "keff generation read-back");
        for (int j = g0; j <= g; ++j) {
            const KeffOut &r = res[j % kGenBlock];
            if (k_col) k_col[j] = r.k_col;
            if (k_site) k_site[j] = r.k_site;
            if (n_sites) n_sites[j] = r.n_sites;
            // the first generation that failed names the error
            const std::string gen = "generation " + std::to_string(j);
            if (r.status == MCDC_E_BANK)
                return fail(MCDC_E_BANK, gen + " made more than " + std::to_string(K.cap) +
                                             " fission sites (start with k0 nearer k)");
            if (r.status == MCDC_E_EXTINCT) return fail(MCDC_E_EXTINCT, gen + " made no fission site");
            if (r.status != 0)
                return fail(r.status, gen + " failed on the device (status " + std::to_string(r.status) + ")");
            if (j >= o->n_inactive) {
                h->batches += 1;
                h->n_hist += M;
            }
        }
        if (cancel_set(h)) return fail(MCDC_E_CANCELLED, "run cancelled");
    }
    return MCDC_OK;
}

}  // extern "C"
