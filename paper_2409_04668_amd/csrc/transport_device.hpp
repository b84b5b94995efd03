// Device-side transport arithmetic for gfx950.
//
// Every routine here is written so that, compiled with -ffp-contract=off and
// IEEE binary64 division/sqrt, it rounds exactly as the definition of the
// method does: the same operations on the same operands in the same order.
// That makes each history's trajectory reproducible bit for bit on any
// schedule.  Sources of the definitions:
//  - straight-line motion between events: position advances by direction
//    times distance, time by distance over speed (the particle-state example
//    of the paper's Fig. 2);
//  - the events that end a flight or a particle: capture, time or space
//    boundary, time census, implicit capture (paper, Sec. "MC/DC on CPUs",
//    transport-loop paragraph);
//  - tallies accumulated by atomic adds on the GPU (paper, Fig. 3);
//  - counter-based random numbers (paper, Sec. "Monte Carlo Neutron Transport
//    and MC/DC", list of developments): Philox4x32-10 of Salmon et al. (SC'11).
#pragma once

#include "mcdc_internal.hpp"

namespace mcdc {

#define MCDC_DEV __device__ __forceinline__

// The problem description as the kernels read it: in the constant address
// space, so that its fields (the same for every lane) come through uniform
// scalar loads.  Every kernel that takes the description by value takes it
// as its first argument, at offset 0 of the kernel-argument segment, and
// reads it there.
typedef const __attribute__((address_space(4))) DevProblem CP;

MCDC_DEV CP &kernel_problem() { return *(CP *)__builtin_amdgcn_kernarg_segment_ptr(); }

// An opaque copy of the description's address, taken once per turn of a
// long transport loop: the compiler then loads each field where it is used
// (scalar-cache hits) instead of hoisting every field out of the loop into
// SGPRs, which overflow and spill to VGPR lanes (one v_readlane per 32 bits
// at every use).
MCDC_DEV CP &problem_reload(CP &P) {
    CP *p = &P;
    asm volatile("" : "+s"(p));
    return *p;
}

constexpr double kInf = __builtin_huge_val();

// ---------------------------------------------------------------------------
// Philox4x32-10 and the per-particle stream.
// counter = (k, tag, hist low 32, hist bits 32..47 | problem << 16), key = seed.
// ---------------------------------------------------------------------------
struct Rng {
    uint32_t key0, key1, tag, c2, c3, k;
};

MCDC_DEV void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                       uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // each 32x32 -> 64-bit product in one v_mad_u64_u32
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

MCDC_DEV Rng make_rng(uint64_t seed, uint64_t hist, uint32_t problem, uint32_t tag, uint32_t k) {
    Rng r;
    r.key0 = (uint32_t)seed;
    r.key1 = (uint32_t)(seed >> 32);
    r.tag = tag;
    r.c2 = (uint32_t)hist;
    r.c3 = (uint32_t)((hist >> 32) & 0xFFFFu) | (problem << 16);
    r.k = k;
    return r;
}

MCDC_DEV void rng_block(Rng &r, uint32_t out[4]) {
    uint32_t c0 = r.k, c1 = r.tag, c2 = r.c2, c3 = r.c3;
    philox10(c0, c1, c2, c3, r.key0, r.key1);
    r.k += 1u;
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// xi = ((u >> 12) + 0.5) * 2^-52, u = (r1 << 32) | r0  -> exact, in (0,1)
MCDC_DEV double rng_uniform(Rng &r) {
    uint32_t c0 = r.k, c1 = r.tag, c2 = r.c2, c3 = r.c3;
    philox10(c0, c1, c2, c3, r.key0, r.key1);
    r.k += 1u;
    const uint64_t u = ((uint64_t)c1 << 32) | (uint64_t)c0;
    return ((double)(u >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// Natural log and exp built from +,-,*,/ only (Cody-Waite reduction with a
// split ln 2; odd atanh series through f^21; Taylor degree 13), so that the
// result does not depend on the device math library.
// ---------------------------------------------------------------------------
constexpr double kLn2Hi = 0x1.62e42feep-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kInvLn2 = 1.4426950408889634;
constexpr double kSqrt2 = 1.4142135623730951;

MCDC_DEV double own_log(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    int e = (int)((b >> 52) & 0x7FFu) - 1023;
    double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (m > kSqrt2) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double s = f * f;
    double p = 1.0 / 21.0;
    p = p * s + 1.0 / 19.0;
    p = p * s + 1.0 / 17.0;
    p = p * s + 1.0 / 15.0;
    p = p * s + 1.0 / 13.0;
    p = p * s + 1.0 / 11.0;
    p = p * s + 1.0 / 9.0;
    p = p * s + 1.0 / 7.0;
    p = p * s + 1.0 / 5.0;
    p = p * s + 1.0 / 3.0;
    const double lm = 2.0 * f + (2.0 * f) * (s * p);
    const double de = (double)e;
    return de * kLn2Hi + (de * kLn2Lo + lm);
}

MCDC_DEV double own_exp(double x) {
    if (x > 700.0) x = 700.0;
    if (x < -700.0) x = -700.0;
    const double n = floor(x * kInvLn2 + 0.5);
    const double r = (x - n * kLn2Hi) - n * kLn2Lo;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    const long long ni = (long long)n;
    const double scale = __longlong_as_double((ni + 1023) << 52);
    return p * scale;
}

// Isotropic direction by Marsaglia's (1972) rejection method.
MCDC_DEV void iso_direction(Rng &r, double &ux, double &uy, double &uz) {
    double a, b, s;
    for (;;) {
        a = 2.0 * rng_uniform(r) - 1.0;
        b = 2.0 * rng_uniform(r) - 1.0;
        s = a * a + b * b;
        if (s < 1.0 && s > 0.0) break;
    }
    const double q = __builtin_sqrt(1.0 - s);
    ux = (2.0 * a) * q;
    uy = (2.0 * b) * q;
    uz = 1.0 - 2.0 * s;
}

// ---------------------------------------------------------------------------
// Particle state in registers.
// ---------------------------------------------------------------------------
struct Part {
    double x[3], u[3], t, w;
    int32_t g, cell, ci;
    uint32_t tag, k, seq;
    bool alive;
};

// ---------------------------------------------------------------------------
// Geometry: priority-ordered boxes, direction-aware containment per axis:
// inside iff lo < p < hi, or p == lo with u >= 0, or p == hi with u < 0.
// ---------------------------------------------------------------------------
MCDC_DEV bool axis_in(double lo, double hi, double p, double u) {
    return (lo < p && p < hi) || (p == lo && u >= 0.0) || (p == hi && p != lo && u < 0.0);
}

typedef const __attribute__((address_space(4))) double cdouble_t;   // a field of CP

MCDC_DEV bool box_in(cdouble_t *lo, cdouble_t *hi, const double p[3], const double u[3]) {
    return axis_in(lo[0], hi[0], p[0], u[0]) && axis_in(lo[1], hi[1], p[1], u[1]) &&
           axis_in(lo[2], hi[2], p[2], u[2]);
}

// The first box containing the point (every box is tested, so the lanes of a
// wave leave the loop together), or -1 for the background.
MCDC_DEV int locate(CP &P, const double p[3], const double u[3]) {
    int cell = -1;
    for (int b = 0; b < P.n_boxes; ++b) {
        const bool in = box_in(P.box_lo[b], P.box_hi[b], p, u);
        cell = (cell < 0 && in) ? b : cell;
    }
    return cell;
}

// Next surface along u: outer-box exit, then per box its exit (inside) or
// slab-test entry (0 <= entry < exit).  First strict minimum wins in the order
// outer box, boxes ascending, axes x,y,z; negative exits clamp to 0.
MCDC_DEV double dist_surface(CP &P, const double p[3], const double u[3],
                             const double iu[3], int &axis, double &plane) {
    double best = kInf;
    int bax = -1;
    double bpl = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (u[a] == 0.0) continue;
        const double pl = u[a] > 0.0 ? P.outer_hi[a] : P.outer_lo[a];
        double s = (pl - p[a]) * iu[a];
        if (!(s > 0.0)) s = 0.0;
        if (s < best) { best = s; bax = a; bpl = pl; }
    }
    // Per box, the slab distances to its two faces on each axis serve both
    // cases: inside, the far face is the exit; outside, the near faces give
    // the entry.  Both candidates are formed and kept by select, so lanes
    // inside and outside a box run the same instructions.
    for (int b = 0; b < P.n_boxes; ++b) {
        cdouble_t *lo = P.box_lo[b];
        cdouble_t *hi = P.box_hi[b];
        const bool inside = box_in(lo, hi, p, u);
        double tn = -kInf, tf = kInf, tpl = 0.0;
        int ta = -1;
        bool miss = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool up = u[a] > 0.0;
            const double s1 = (lo[a] - p[a]) * iu[a];
            const double s2 = (hi[a] - p[a]) * iu[a];
            const double nr = up ? s1 : s2;
            const double fr = up ? s2 : s1;
            const bool moving = u[a] != 0.0;
            // inside: exit through the far face (negative distances clamp to 0)
            const double se = fr > 0.0 ? fr : 0.0;
            const bool take = inside && moving && se < best;
            best = take ? se : best;
            bax = take ? a : bax;
            bpl = take ? (up ? hi[a] : lo[a]) : bpl;
            // outside: slab test
            miss = miss || (!moving && !axis_in(lo[a], hi[a], p[a], 0.0));
            const bool nearer = moving && nr > tn;
            tn = nearer ? nr : tn;
            ta = nearer ? a : ta;
            tpl = nearer ? (up ? lo[a] : hi[a]) : tpl;
            tf = (moving && fr < tf) ? fr : tf;
        }
        const bool enter = !inside && !miss && ta >= 0 && tn < tf && tn >= 0.0 && tn < best;
        best = enter ? tn : best;
        bax = enter ? ta : bax;
        bpl = enter ? tpl : bpl;
    }
    axis = bax;
    plane = bpl;
    return best;
}

// Part of [0,d] inside the detector box.
MCDC_DEV double detector_len(CP &P, const double p[3], const double u[3],
                             const double iu[3], double d) {
    double si = 0.0, so = d;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (u[a] == 0.0) {
            if (!(P.det_lo[a] <= p[a] && p[a] <= P.det_hi[a])) return 0.0;
            continue;
        }
        const double s1 = (P.det_lo[a] - p[a]) * iu[a];
        const double s2 = (P.det_hi[a] - p[a]) * iu[a];
        const double nr = u[a] > 0.0 ? s1 : s2;
        const double fr = u[a] > 0.0 ? s2 : s1;
        if (nr > si) si = nr;
        if (fr < so) so = fr;
    }
    return so > si ? so - si : 0.0;
}

// ---------------------------------------------------------------------------
// Tally targets: FP64 atomics into global memory, or into an LDS tile that
// the kernel flushes to global memory when it ends.
// ---------------------------------------------------------------------------
// add(flat bin, g, t, z, y, x indices, value)
struct GlobalTally {
    double *base;
    MCDC_DEV void add(uint32_t i, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, double v) const {
        unsafeAtomicAdd(base + i, v);
    }
};
// LDS and HBM tally targets carry their address space in the pointer type, so
// an update is a ds_add_f64 or a global_atomic_add_f64; through generic
// pointers the two branches of a tile test fold into one flat atomic.
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(1))) double hbm_f64;

MCDC_DEV void lds_add(lds_f64 *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
MCDC_DEV void hbm_add(hbm_f64 *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LdsTally {
    lds_f64 *base;
    MCDC_DEV void add(uint32_t i, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, double v) const {
        lds_add(base + i, v);
    }
};
// A sub-box of the (g, t, z, y, x) mesh privatised in LDS (the bins that take
// most of the updates); every other bin goes to HBM atomics.  The box's
// corner and extents are read from the problem description at each update
// (scalar loads) rather than held in SGPRs for the whole kernel; `n0` is the
// x extent, zero while the workgroup scores a batch the tile does not hold.
struct HotTileTally {
    lds_f64 *lds;
    hbm_f64 *glob;
    CP *prob;
    uint32_t n0;
    MCDC_DEV void add(uint32_t i, uint32_t g, uint32_t t, uint32_t z, uint32_t y, uint32_t x,
                      double v) const {
        CP &Q = problem_reload(*prob);
        uint32_t l0 = Q.hot_lo[0], l1 = Q.hot_lo[1], l2 = Q.hot_lo[2], l3 = Q.hot_lo[3],
                 l4 = Q.hot_lo[4], n1 = Q.hot_n[1], n2 = Q.hot_n[2], n3 = Q.hot_n[3],
                 n4 = Q.hot_n[4];
        // all nine fields loaded before the test (no load sinks into one of
        // its branches), so the test is one compare per axis and mask ANDs
        asm volatile("" : "+s"(l0), "+s"(l1), "+s"(l2), "+s"(l3), "+s"(l4), "+s"(n1), "+s"(n2),
                          "+s"(n3), "+s"(n4));
        const uint32_t dx = x - l0, dy = y - l1, dz = z - l2, dt = t - l3, dg = g - l4;
        if (dx < n0 && dy < n1 && dz < n2 && dt < n3 && dg < n4) {
            const uint32_t j = (((dg * n3 + dt) * n2 + dz) * n1 + dy) * n0 + dx;
            lds_add(lds + j, v);
        } else {
            hbm_add(glob + i, v);
        }
    }
};

// Add a workgroup's hot tile (LDS, x fastest over the tile box) into the mesh
// tally at `out`: one HBM atomic per touched bin.
MCDC_DEV void hot_tile_flush(CP &P, const double *tile, double *out) {
    const uint32_t nx = P.hot_n[0], ny = P.hot_n[1], nz = P.hot_n[2], nt = P.hot_n[3];
    const uint32_t mx = P.mesh_n[0], my = P.mesh_n[1], mz = P.mesh_n[2], mt = P.mesh_n[3];
    for (uint32_t j = threadIdx.x; j < P.hot_bins; j += blockDim.x) {
        const double v = tile[j];
        if (v == 0.0) continue;
        uint32_t r = j;
        const uint32_t x = r % nx + P.hot_lo[0]; r /= nx;
        const uint32_t y = r % ny + P.hot_lo[1]; r /= ny;
        const uint32_t z = r % nz + P.hot_lo[2]; r /= nz;
        const uint32_t t = r % nt + P.hot_lo[3]; r /= nt;
        const uint32_t g = r + P.hot_lo[4];
        const uint32_t b = (((g * mt + t) * mz + z) * my + y) * mx + x;
        unsafeAtomicAdd(&out[b], v);
    }
}

// Minimum of two doubles that are never NaN: one v_min_f64, without the
// quieting of signalling NaNs the compiler adds in front of fmin.
MCDC_DEV double min_f64(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Track-length scoring of the segment p + s u, s in [0,d], from time t0 at
// speed v: the segment is cut at every mesh plane and time edge it crosses
// (edges lo + k*delta); each in-mesh piece of positive length adds
// w * length to tally[g][it][iz][iy][ix].  Returns the pieces.
//
// Crossing distances: the first on each axis from the segment start,
// (edge - p) * (1/u) (time: (edge - t0) * v); each later one adds the axis's
// step delta * |1/u| (time: delta * v) to the one before; all axes at the
// minimum advance together.  The walk ends at d or at the far mesh edge of a
// bounded axis in the direction of travel or the last time edge, each
// computed from the segment start, whichever comes first.  A piece is in the
// mesh when all four indices are (the accumulated crossings and the end
// distance come from different formulas, so the indices decide).
// kKeepSteps: the four crossing steps are held in registers for the walk;
// without it (kernels at their register limit) each step is recomputed from
// the same operands where it is added, to the same value.
template <bool kKeepSteps, class T>
MCDC_DEV uint32_t score_mesh(CP &P, const double p[3], const double u[3],
                             double iu[3], double t0, double v, double d, double w, int g,
                             const T &tally) {
    if (!(d > 0.0)) return 0;
    int idx[4];
    double s[4];
    double dd = d;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!P.mesh_bounded[a]) { idx[a] = 0; s[a] = kInf; continue; }
        if (u[a] != 0.0) {
            const int k = u[a] > 0.0 ? P.mesh_n[a] : 0;
            const double se = (P.mesh_lo[a] + (double)k * P.mesh_delta[a] - p[a]) * iu[a];
            if (se < dd) dd = se;
        }
        const double q = (p[a] - P.mesh_lo[a]) * P.mesh_idelta[a];
        double fq = floor(q);
        if (fq < -1.0) fq = -1.0;
        if (fq > (double)P.mesh_n[a]) fq = (double)P.mesh_n[a];
        int i = (int)fq;
        if (q == fq && u[a] < 0.0) i = i - 1;
        if (i < -1) i = -1;
        idx[a] = i;
        if (u[a] > 0.0) {
            if (i >= P.mesh_n[a]) return 0;
            const double e = P.mesh_lo[a] + (double)(i + 1) * P.mesh_delta[a];
            s[a] = (e - p[a]) * iu[a];
        } else if (u[a] < 0.0) {
            if (i < 0) return 0;
            const double e = P.mesh_lo[a] + (double)i * P.mesh_delta[a];
            s[a] = (e - p[a]) * iu[a];
        } else {
            if (i < 0 || i >= P.mesh_n[a]) return 0;
            s[a] = kInf;
        }
    }
    {
        const double q = (t0 - P.mesh_lo[3]) * P.mesh_idelta[3];
        double fq = floor(q);
        if (fq < -1.0) fq = -1.0;
        if (fq > (double)P.mesh_n[3]) fq = (double)P.mesh_n[3];
        const int i = (int)fq;
        if (i >= P.mesh_n[3]) return 0;
        idx[3] = i;
        const double e = P.mesh_lo[3] + (double)(i + 1) * P.mesh_delta[3];
        s[3] = (e - t0) * v;
        const double se = (P.mesh_lo[3] + (double)P.mesh_n[3] * P.mesh_delta[3] - t0) * v;
        if (se < dd) dd = se;
    }
    const uint32_t n0 = P.mesh_n[0], n1 = P.mesh_n[1], n2 = P.mesh_n[2], n3 = P.mesh_n[3];
    const uint32_t gt = (uint32_t)(P.G_t > 1 ? g : 0);
    const uint32_t gbase = gt * n3;
    // Per-axis index step and crossing step.  The advance below computes every
    // axis's candidate and keeps it by select, so lanes with different
    // direction signs or tie patterns run the same instructions (the values
    // are those of advancing axis by axis); an axis that is not cut keeps an
    // infinite distance.
    int step[3];
    double ds[4];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        step[a] = u[a] > 0.0 ? 1 : -1;
        if constexpr (kKeepSteps) ds[a] = P.mesh_delta[a] * fabs(iu[a]);
    }
    if constexpr (kKeepSteps) ds[3] = P.mesh_delta[3] * v;
    uint32_t pieces = 0;
    double sp = 0.0;
    for (;;) {
        // the nearest of the walk's end and the four next crossings (no NaN
        // occurs; +0 and -0, the only values min may order either way,
        // compare equal in every later test and give the same differences)
        const double sn = min_f64(min_f64(dd, s[0]), min_f64(min_f64(s[1], s[2]), s[3]));
        if (sn > sp) {
            const bool in = (uint32_t)idx[0] < n0 && (uint32_t)idx[1] < n1 &&
                            (uint32_t)idx[2] < n2 && (uint32_t)idx[3] < n3;
            if (in) {
                const uint32_t b =
                    (((gbase + (uint32_t)idx[3]) * n2 + (uint32_t)idx[2]) * n1 + (uint32_t)idx[1]) *
                        n0 + (uint32_t)idx[0];
                tally.add(b, gt, (uint32_t)idx[3], (uint32_t)idx[2], (uint32_t)idx[1],
                          (uint32_t)idx[0], w * (sn - sp));
                pieces += 1;
            }
        }
        if (sn >= dd) break;
        if constexpr (!kKeepSteps) {
            // the operands look changed on every turn, so the products are
            // formed here rather than hoisted out of the loop into registers
            asm volatile("" : "+v"(iu[0]), "+v"(iu[1]), "+v"(iu[2]), "+v"(v));
#pragma unroll
            for (int a = 0; a < 3; ++a) ds[a] = P.mesh_delta[a] * fabs(iu[a]);
            ds[3] = P.mesh_delta[3] * v;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool adv = s[a] == sn;
            idx[a] = adv ? idx[a] + step[a] : idx[a];
            s[a] = adv ? s[a] + ds[a] : s[a];
        }
        {
            const bool adv = s[3] == sn;
            idx[3] = adv ? idx[3] + 1 : idx[3];
            s[3] = adv ? s[3] + ds[3] : s[3];
        }
        sp = sn;
    }
    return pieces;
}

// ---------------------------------------------------------------------------
// FP32 log-importance MLP: in -> 64 -> 64 -> 1, ReLU; each neuron starts from
// its bias and adds weight*input products for ascending inputs, as separate
// float multiplies and adds.  Layout W1[64][in], b1, W2[64][64], b2, W3, b3.
// The weights are the same for every lane and read-only during a launch, so
// they are read through the constant address space: uniform scalar loads
// into SGPRs that the vector multiplies take as operands, with no LDS copy
// and no per-lane vector loads.  `prm` must point to global memory.
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) float cfloat_t;

MCDC_DEV float mlp_infer(const float *__restrict__ gprm, int in_dim, const float in[4 + kMaxG]) {
    cfloat_t *prm = (cfloat_t *)(uintptr_t)gprm;
    cfloat_t *W1 = prm;
    cfloat_t *b1 = W1 + kH * in_dim;
    cfloat_t *W2 = b1 + kH;
    cfloat_t *b2 = W2 + kH * kH;
    cfloat_t *W3 = b2 + kH;
    cfloat_t *b3 = W3 + kH;
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = b1[j];
#pragma unroll
        for (int i = 0; i < 4 + kMaxG; ++i) {
            if (i < in_dim) {
                const float prod = W1[j * in_dim + i] * in[i];
                acc = acc + prod;
            }
        }
        h1[j] = acc > 0.0f ? acc : 0.0f;
    }
    float out = b3[0];
    for (int j = 0; j < kH; ++j) {
        float acc = b2[j];
        cfloat_t *row = W2 + j * kH;
#pragma unroll
        for (int i = 0; i < kH; ++i) {
            const float prod = row[i] * h1[i];
            acc = acc + prod;
        }
        const float h2 = acc > 0.0f ? acc : 0.0f;
        const float prod = W3[j] * h2;
        out = out + prod;
    }
    return out;
}

// Weight-window grid planes: the interior planes lo + k delta (k = 1..n-1) of
// a regular grid over the outer box, per axis.  Distance along u to the next
// one ahead of p: moving up k = floor((p - lo) / delta) + 1, moving down the
// plane at or below p (one lower when p is on it); then one further while
// (plane - p) * iu is not positive, so a particle on a plane moves off it.
// First strict minimum in axis order; +inf (axis -1) when none lies ahead.
MCDC_DEV double dist_ww_plane(CP &P, const double p[3], const double u[3], const double iu[3],
                              int &axis, double &plane) {
    double best = kInf;
    int bax = -1;
    double bpl = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (u[a] == 0.0) continue;
        const double lo = P.outer_lo[a], dl = P.ww_grid_d[a];
        const double q = (p[a] - lo) * P.ww_grid_id[a];
        const double f = floor(q);
        const bool up = u[a] > 0.0;
        double k = up ? f + 1.0 : (q == f ? f - 1.0 : f);
        double pl = lo + k * dl;
        double s = (pl - p[a]) * iu[a];
        for (int it = 0; it < 4 && !(s > 0.0); ++it) {
            k = up ? k + 1.0 : k - 1.0;
            pl = lo + k * dl;
            s = (pl - p[a]) * iu[a];
        }
        if (!(s > 0.0) || k < 1.0 || k > (double)(P.ww_grid_n[a] - 1)) continue;
        if (s < best) { best = s; bax = a; bpl = pl; }
    }
    axis = bax;
    plane = bpl;
    return best;
}

// Surface-current tally on the plane x[a] = c (a = P.surf_axis, c =
// P.surf_pos): a flight p + s u, s in (0, d], crosses it at
// s* = (c - p[a]) * iu[a] when 0 < s* <= d and adds its weight w to the bin
// [side][g][t][b2][b1] of the crossing: side 0 when u[a] > 0, the group as
// the mesh, the time bin of t0 + s*/v and the mesh bins of the two other axes
// (b1 < b2) at p + s* u.  A crossing outside the mesh is not scored; a flight
// that starts on the plane does not cross it.  Returns 1 when it scored.
MCDC_DEV uint32_t score_surface(CP &P, const double p[3], const double u[3], const double iu[3],
                                double t0, double v, double d, double w, int g, double *out) {
    const int a = P.surf_axis;
    const double ua = a == 0 ? u[0] : (a == 1 ? u[1] : u[2]);
    if (ua == 0.0) return 0;
    const double pa = a == 0 ? p[0] : (a == 1 ? p[1] : p[2]);
    const double iua = a == 0 ? iu[0] : (a == 1 ? iu[1] : iu[2]);
    const double sx = (P.surf_pos - pa) * iua;
    if (!(sx > 0.0 && sx <= d)) return 0;
    // in-plane axes b1 < b2
    const double p1 = a == 0 ? p[1] : p[0], u1 = a == 0 ? u[1] : u[0];
    const double p2 = a == 2 ? p[1] : p[2], u2 = a == 2 ? u[1] : u[2];
    int32_t i1 = 0, i2 = 0;
    if (P.surf_bd[0]) {
        const double f = floor((p1 + u1 * sx - P.surf_lo[0]) * P.surf_id[0]);
        if (f < 0.0 || f >= (double)P.surf_n[0]) return 0;
        i1 = (int32_t)f;
    }
    if (P.surf_bd[1]) {
        const double f = floor((p2 + u2 * sx - P.surf_lo[1]) * P.surf_id[1]);
        if (f < 0.0 || f >= (double)P.surf_n[1]) return 0;
        i2 = (int32_t)f;
    }
    const double ft = floor((t0 + sx / v - P.mesh_lo[3]) * P.mesh_idelta[3]);
    if (ft < 0.0 || ft >= (double)P.mesh_n[3]) return 0;
    const uint32_t side = ua > 0.0 ? 0u : 1u;
    const uint32_t gg = P.G_t > 1 ? (uint32_t)g : 0u;
    const uint32_t bin = (((side * (uint32_t)P.G_t + gg) * (uint32_t)P.mesh_n[3] + (uint32_t)ft) *
                              (uint32_t)P.surf_n[1] + (uint32_t)i2) * (uint32_t)P.surf_n[0] + (uint32_t)i1;
    unsafeAtomicAdd(out + bin, w);
    return 1;
}

// Mesh bin holding a point (x, y, z, t) in group g, for the collision
// estimator: per axis floor((p - lo) / delta); -1 outside the mesh (an
// unbounded axis is one bin).
MCDC_DEV int64_t mesh_point_bin(CP &P, const double p[3], double t, int g) {
    int64_t c = P.G_t > 1 ? g : 0;
#pragma unroll
    for (int a = 3; a >= 0; --a) {
        int64_t i = 0;
        if (a == 3 || P.mesh_bounded[a]) {
            const double v = a == 3 ? t : (a == 2 ? p[2] : (a == 1 ? p[1] : p[0]));
            const double f = floor((v - P.mesh_lo[a]) * P.mesh_idelta[a]);
            if (f < 0.0 || f >= (double)P.mesh_n[a]) return -1;
            i = (int64_t)f;
        }
        c = c * P.mesh_n[a] + i;
    }
    return c;
}

// Map cell of a point for the weight-window map: per axis floor(s n) of the
// fraction s of the outer box (of the last census time), clamped to [0, n-1];
// layout [g][t][z][y][x].
MCDC_DEV int64_t ww_map_cell(CP &P, const Part &q) {
    int64_t c = q.g;
#pragma unroll
    for (int a = 3; a >= 0; --a) {
        const double v = a == 3 ? q.t : (a == 2 ? q.x[2] : (a == 1 ? q.x[1] : q.x[0]));
        const double sa = (v - P.ww_lo[a]) * P.ww_inv[a];
        const double f = floor(sa * (double)P.ww_map_n[a]);
        const int64_t i = f < 0.0 ? 0 : (f >= (double)P.ww_map_n[a] ? P.ww_map_n[a] - 1 : (int64_t)f);
        c = c * P.ww_map_n[a] + i;
    }
    return c;
}

// Window target from the network: output y at the normalised point (2 s - 1
// per axis, group one-hot), clamped to its training-target range, and
// w_T = exp(log K - y).
MCDC_DEV double ww_net_target(CP &P, const float *prm, const float xt[4], int g) {
    float in[4 + kMaxG];
#pragma unroll
    for (int a = 0; a < 4; ++a) in[a] = xt[a];
#pragma unroll
    for (int j = 0; j < kMaxG; ++j) in[4 + j] = j == g ? 1.0f : 0.0f;
    float y = mlp_infer(prm, 4 + P.G, in);
    if (y < P.ww_ymin) y = P.ww_ymin;
    if (y > P.ww_ymax) y = P.ww_ymax;
    return own_exp(P.ww_logk - (double)y);
}

}  // namespace mcdc
