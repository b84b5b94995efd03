/*
 * CPU oracle — TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain C99, built with -O2 -ffp-contract=off -fno-fast-math on x86-64 (SSE2
 * binary64, round to nearest even, no FMA).  Every arithmetic expression is
 * written in the order that defines the method; the GPU kernels follow the same
 * definition from their own source.
 *
 * What the paper fixes and where:
 *  - particle histories driven by pseudorandom numbers, material data and
 *    geometry, tallied with a statistical error: Sec. "Monte Carlo Neutron
 *    Transport and MC/DC";
 *  - the fixed-source loop that transports each particle until a physical
 *    event (capture, time or space boundary), a simulation event (time census)
 *    or a variance-reduction event (implicit capture) ends it: Sec. "MC/DC on
 *    CPUs", transport-loop paragraph;
 *  - straight-line motion between events: position advances by direction
 *    times distance and time by distance over speed (the particle-state
 *    example of Fig. 2);
 *  - tally accumulation by a plain add on the CPU, an atomic add on the GPU:
 *    Fig. 3;
 *  - hash-based (counter-based) random numbers for replicable testing: Sec.
 *    "Monte Carlo Neutron Transport and MC/DC", list of novel developments;
 *  - the k-eigenvalue mode beside the time-dependent one, fission as a
 *    physical event that ends a history, and the generation of daughter
 *    particles from fission in the kernel set: Sec. "Monte Carlo Neutron
 *    Transport and MC/DC" (feature list) and Sec. "MC/DC on CPUs".
 * Everything else (RNG algorithm, sampling formulas, estimator, tie rules,
 * weight windows, population control) is a reading of this implementation,
 * stated in the comments below.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define O_INF HUGE_VAL

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).     */
/* Ten rounds; each round multiplies words 0 and 2 by the two Philox         */
/* multipliers, and the key is bumped by the two Weyl constants between      */
/* rounds.                                                                   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One random stream per particle: key = seed, counter = (k, tag, history low
 * word, history high 16 bits | problem << 16).  Each draw uses one Philox
 * block and advances k. */
typedef struct {
    uint32_t key[2];
    uint32_t tag, c2, c3;
    uint32_t k;
} o_stream;

static o_stream o_stream_make(uint64_t seed, uint64_t hist, uint32_t problem, uint32_t tag)
{
    o_stream s;
    s.key[0] = (uint32_t)seed;
    s.key[1] = (uint32_t)(seed >> 32);
    s.tag = tag;
    s.c2 = (uint32_t)hist;
    s.c3 = (uint32_t)((hist >> 32) & 0xFFFFu) | (problem << 16);
    s.k = 0;
    return s;
}

static void o_block(o_stream *s, uint32_t out[4])
{
    uint32_t ctr[4] = {s->k, s->tag, s->c2, s->c3};
    orc_philox4x32_10(ctr, s->key, out);
    s->k += 1u;
}

/* xi = ((u >> 12) + 0.5) * 2^-52 with u = (r1 << 32) | r0: exact, in (0,1). */
static double o_draw(o_stream *s)
{
    uint32_t r[4];
    o_block(s, r);
    uint64_t u = ((uint64_t)r[1] << 32) | (uint64_t)r[0];
    return ((double)(u >> 12) + 0.5) * 0x1p-52;
}

double orc_uniform(uint64_t seed, uint64_t hist, uint32_t problem, uint32_t tag, uint32_t k)
{
    o_stream s = o_stream_make(seed, hist, problem, tag);
    s.k = k;
    return o_draw(&s);
}

/* ------------------------------------------------------------------------ */
/* Own natural log and exp, so that both implementations round identically. */
/* log: Cody-Waite style reduction x = 2^e * m with m in [sqrt(1/2),sqrt(2)), */
/* log m = 2 atanh(f), f = (m-1)/(m+1), odd series through f^21 (|f|<0.1716).*/
/* exp: n = floor(x/ln2 + 1/2), r = (x - n ln2_hi) - n ln2_lo, Taylor        */
/* polynomial of degree 13 in Horner form, times 2^n built from exponent bits.*/
/* ln2_hi = ln 2 rounded to 32 significant bits, ln2_lo = the remainder.     */
/* ------------------------------------------------------------------------ */
static const double O_LN2_HI = 0x1.62e42feep-1;          /* 6.93147180369123816490e-01 */
static const double O_LN2_LO = 0x1.a39ef35793c76p-33;    /* 1.90821492927058770002e-10 */
static const double O_INV_LN2 = 1.4426950408889634;
static const double O_SQRT2 = 1.4142135623730951;

static uint64_t o_bits(double x) { uint64_t b; memcpy(&b, &x, 8); return b; }
static double o_from_bits(uint64_t b) { double x; memcpy(&x, &b, 8); return x; }

double orc_log(double x)
{
    /* domain: positive normal numbers (the transport loop only takes logs of
     * numbers in (0,1) that are multiples of 2^-53) */
    uint64_t b = o_bits(x);
    int e = (int)((b >> 52) & 0x7FFu) - 1023;
    double m = o_from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > O_SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = (m - 1.0) / (m + 1.0);
    double s = f * f;
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
    double lm = 2.0 * f + (2.0 * f) * (s * p);
    double de = (double)e;
    return de * O_LN2_HI + (de * O_LN2_LO + lm);
}

double orc_exp(double x)
{
    if (x > 700.0) x = 700.0;
    if (x < -700.0) x = -700.0;
    double n = floor(x * O_INV_LN2 + 0.5);
    double r = (x - n * O_LN2_HI) - n * O_LN2_LO;
    double p = 1.0 / 6227020800.0;        /* 1/13! */
    p = p * r + 1.0 / 479001600.0;        /* 1/12! */
    p = p * r + 1.0 / 39916800.0;         /* 1/11! */
    p = p * r + 1.0 / 3628800.0;          /* 1/10! */
    p = p * r + 1.0 / 362880.0;           /* 1/9!  */
    p = p * r + 1.0 / 40320.0;            /* 1/8!  */
    p = p * r + 1.0 / 5040.0;             /* 1/7!  */
    p = p * r + 1.0 / 720.0;              /* 1/6!  */
    p = p * r + 1.0 / 120.0;              /* 1/5!  */
    p = p * r + 1.0 / 24.0;               /* 1/4!  */
    p = p * r + 1.0 / 6.0;                /* 1/3!  */
    p = p * r + 0.5;                      /* 1/2!  */
    p = p * r + 1.0;                      /* 1/1!  */
    p = p * r + 1.0;                      /* 1/0!  */
    int64_t ni = (int64_t)n;
    double scale = o_from_bits((uint64_t)(ni + 1023) << 52);
    return p * scale;
}

/* Isotropic direction, Marsaglia (1972): draw a = 2 xi1 - 1, b = 2 xi2 - 1
 * until 0 < s = a^2 + b^2 < 1; then u = (2a sqrt(1-s), 2b sqrt(1-s), 1 - 2s). */
static void o_direction(o_stream *st, double u[3])
{
    double a, b, s;
    for (;;) {
        a = 2.0 * o_draw(st) - 1.0;
        b = 2.0 * o_draw(st) - 1.0;
        s = a * a + b * b;
        if (s < 1.0 && s > 0.0) break;
    }
    double r = sqrt(1.0 - s);
    u[0] = (2.0 * a) * r;
    u[1] = (2.0 * b) * r;
    u[2] = 1.0 - 2.0 * s;
}

uint32_t orc_directions(uint64_t seed, uint64_t hist, uint32_t n, double *u)
{
    o_stream s = o_stream_make(seed, hist, 0, 0);
    for (uint32_t i = 0; i < n; ++i) o_direction(&s, u + 3 * i);
    return s.k;
}

/* ------------------------------------------------------------------------ */
/* FP32 MLP forward (log-importance): inputs -> H -> H -> 1 with ReLU.       */
/* Parameter layout: W1[H][in], b1[H], W2[H][H], b2[H], W3[H], b3.           */
/* Each neuron: acc = bias, then acc = acc + w_i * x_i for i ascending, as   */
/* separate float multiply and add.                                          */
/* ------------------------------------------------------------------------ */
float orc_mlp_f32(const float *prm, int32_t in_dim, int32_t H, const float *in)
{
    const float *W1 = prm;
    const float *b1 = W1 + (size_t)H * in_dim;
    const float *W2 = b1 + H;
    const float *b2 = W2 + (size_t)H * H;
    const float *W3 = b2 + H;
    const float *b3 = W3 + H;
    float h1[256], h2[256];
    for (int j = 0; j < H; ++j) {
        float acc = b1[j];
        for (int i = 0; i < in_dim; ++i) {
            float prod = W1[(size_t)j * in_dim + i] * in[i];
            acc = acc + prod;
        }
        h1[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int j = 0; j < H; ++j) {
        float acc = b2[j];
        for (int i = 0; i < H; ++i) {
            float prod = W2[(size_t)j * H + i] * h1[i];
            acc = acc + prod;
        }
        h2[j] = acc > 0.0f ? acc : 0.0f;
    }
    float out = b3[0];
    for (int i = 0; i < H; ++i) {
        float prod = W3[i] * h2[i];
        out = out + prod;
    }
    return out;
}

/* ------------------------------------------------------------------------ */
/* Geometry: priority-ordered axis-aligned boxes inside an outer box.        */
/* A point belongs to the first box that contains it, else to the background */
/* material.  Containment is decided per axis and is direction aware: inside */
/* iff lo < p < hi, or p == lo moving in (u >= 0 at lo), or p == hi moving  */
/* in (u < 0).                                                               */
/* ------------------------------------------------------------------------ */
static int o_axis_in(double lo, double hi, double p, double u)
{
    if (lo < p && p < hi) return 1;
    if (p == lo) return u >= 0.0;
    if (p == hi) return u < 0.0;
    return 0;
}

static int o_box_in(const double *lo, const double *hi, const double p[3], const double u[3])
{
    return o_axis_in(lo[0], hi[0], p[0], u[0]) && o_axis_in(lo[1], hi[1], p[1], u[1]) &&
           o_axis_in(lo[2], hi[2], p[2], u[2]);
}

static int o_locate(const orc_problem *P, const double p[3], const double u[3])
{
    for (int b = 0; b < P->n_boxes; ++b)
        if (o_box_in(P->box_lo + 3 * b, P->box_hi + 3 * b, p, u)) return b;
    return -1;
}

static int o_material(const orc_problem *P, int cell)
{
    return cell >= 0 ? P->box_mat[cell] : P->background_mat;
}

/* Distance to the next surface along u (1/u precomputed, unused where u == 0):
 * exit of the outer box, and for every box either its exit (point inside) or
 * its entry (slab test, entry >= 0 and entry < exit).  Strict '<' keeps the
 * first candidate in the order outer box, boxes ascending, axes x,y,z.
 * Negative exit distances (a point a rounding error outside) become 0. */
static double o_dist_surface(const orc_problem *P, const double p[3], const double u[3],
                             const double iu[3], int *axis, double *plane)
{
    double best = O_INF;
    int bax = -1;
    double bpl = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (u[a] == 0.0) continue;
        double pl = u[a] > 0.0 ? P->outer_hi[a] : P->outer_lo[a];
        double s = (pl - p[a]) * iu[a];
        if (!(s > 0.0)) s = 0.0;
        if (s < best) { best = s; bax = a; bpl = pl; }
    }
    for (int b = 0; b < P->n_boxes; ++b) {
        const double *lo = P->box_lo + 3 * b, *hi = P->box_hi + 3 * b;
        if (o_box_in(lo, hi, p, u)) {
            for (int a = 0; a < 3; ++a) {
                if (u[a] == 0.0) continue;
                double pl = u[a] > 0.0 ? hi[a] : lo[a];
                double s = (pl - p[a]) * iu[a];
                if (!(s > 0.0)) s = 0.0;
                if (s < best) { best = s; bax = a; bpl = pl; }
            }
        } else {
            double tn = -O_INF, tf = O_INF, tpl = 0.0;
            int ta = -1, miss = 0;
            for (int a = 0; a < 3; ++a) {
                if (u[a] == 0.0) {
                    if (!o_axis_in(lo[a], hi[a], p[a], 0.0)) miss = 1;
                    continue;
                }
                double s1 = (lo[a] - p[a]) * iu[a];
                double s2 = (hi[a] - p[a]) * iu[a];
                double nr = u[a] > 0.0 ? s1 : s2;
                double fr = u[a] > 0.0 ? s2 : s1;
                if (nr > tn) { tn = nr; ta = a; tpl = u[a] > 0.0 ? lo[a] : hi[a]; }
                if (fr < tf) tf = fr;
            }
            if (!miss && ta >= 0 && tn < tf && tn >= 0.0 && tn < best) {
                best = tn; bax = ta; bpl = tpl;
            }
        }
    }
    *axis = bax;
    *plane = bpl;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Track-length estimator: a straight segment p + s u, s in [0,d], starting  */
/* at time t0 with speed v, is cut at every mesh plane and time-bin edge it  */
/* crosses; each piece adds w * length to tally[g][it][iz][iy][ix].  Edges   */
/* are lo + k*delta with delta = (hi-lo)/n.  The first crossing of an axis   */
/* is (edge - p) / u from the segment start (time: (edge - t0) v); each      */
/* later crossing of that axis is the previous one plus delta / |u| (time:   */
/* delta v); all axes that reach the minimum advance together.  The walk     */
/* ends at d or where the segment leaves the mesh: the far edge of a bounded */
/* axis in the direction of travel, or the last time edge, each taken from   */
/* the segment start, whichever comes first.  Pieces of zero or negative     */
/* length and pieces whose bin lies outside the mesh are not scored.  An     */
/* axis with infinite bounds is not cut.  (A reading: the paper names the    */
/* estimator, not how the crossings are computed.)                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n[4], bounded[3];
    double lo[4], delta[4], idelta[4];
    int G_t;                                /* groups in the tally (1 or G) */
} o_mesh;

static o_mesh o_mesh_make(const orc_problem *P)
{
    o_mesh M;
    for (int a = 0; a < 4; ++a) {
        M.n[a] = P->mesh_n[a];
        M.lo[a] = P->mesh_lo[a];
        if (a < 3 && isinf(P->mesh_lo[a]) && isinf(P->mesh_hi[a])) {
            M.bounded[a] = 0;
            M.delta[a] = O_INF;
            M.idelta[a] = 0.0;
        } else {
            if (a < 3) M.bounded[a] = 1;
            M.delta[a] = (P->mesh_hi[a] - P->mesh_lo[a]) / (double)P->mesh_n[a];
            M.idelta[a] = 1.0 / M.delta[a];
        }
    }
    M.G_t = P->mesh_per_group ? P->G : 1;
    return M;
}

/* mesh bin holding a point (x, y, z, t) in group g: per axis floor((p - lo) /
 * delta); -1 when the point lies outside the mesh (an unbounded axis is one
 * bin) */
static int64_t o_point_bin(const o_mesh *M, const double p[3], double t, int g)
{
    int64_t c = M->G_t > 1 ? g : 0;
    for (int a = 3; a >= 0; --a) {
        int64_t i = 0;
        if (a == 3 || M->bounded[a]) {
            double v = a == 3 ? t : p[a];
            double f = floor((v - M->lo[a]) * M->idelta[a]);
            if (f < 0.0 || f >= (double)M->n[a]) return -1;
            i = (int64_t)f;
        }
        c = c * M->n[a] + i;
    }
    return c;
}

/* Surface-current tally (a reading; the paper names tallies but defines no
 * surface estimator): the plane x[a] = c of one axis.  A flight p + s u,
 * s in (0, d], crosses it at s* = (c - p[a]) * (1 / u[a]) when 0 < s* <= d,
 * and adds its weight w to the bin of the crossing: side (0 when u[a] > 0,
 * 1 when u[a] < 0), group (per-group meshes), the time bin of t + s* / v and
 * the mesh bins of the two other axes at p + s* u (the lower axis fastest);
 * a crossing outside the mesh is not scored.  A flight that ends on the plane
 * counts there; the next one, starting on it, does not.  The number of
 * surface bins is 2 G_t nt n_b1 n_b2.  Returns 1 when it scored. */
static int o_score_surface(const o_mesh *M, int a, double c, const double p[3],
                           const double u[3], const double iu[3], double t0, double v,
                           double d, double w, int g, double *out)
{
    if (u[a] == 0.0) return 0;
    double sx = (c - p[a]) * iu[a];
    if (!(sx > 0.0 && sx <= d)) return 0;
    int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    int64_t i1 = 0, i2 = 0, it;
    if (M->bounded[b1]) {
        double f = floor((p[b1] + u[b1] * sx - M->lo[b1]) * M->idelta[b1]);
        if (f < 0.0 || f >= (double)M->n[b1]) return 0;
        i1 = (int64_t)f;
    }
    if (M->bounded[b2]) {
        double f = floor((p[b2] + u[b2] * sx - M->lo[b2]) * M->idelta[b2]);
        if (f < 0.0 || f >= (double)M->n[b2]) return 0;
        i2 = (int64_t)f;
    }
    {
        double f = floor((t0 + sx / v - M->lo[3]) * M->idelta[3]);
        if (f < 0.0 || f >= (double)M->n[3]) return 0;
        it = (int64_t)f;
    }
    int64_t side = u[a] > 0.0 ? 0 : 1;
    int64_t gg = M->G_t > 1 ? g : 0;
    int64_t bin = (((side * M->G_t + gg) * M->n[3] + it) * M->n[b2] + i2) * M->n[b1] + i1;
    out[bin] += w;
    return 1;
}

/* returns pieces scored; tally may be NULL (count only) */
static int64_t o_score_mesh(const o_mesh *M, const double p[3], const double u[3],
                            const double iu[3], double t0, double v, double d, double w,
                            int g, double *tally)
{
    int idx[4];
    double s[4], ds[4];
    int64_t pieces = 0;
    if (!(d > 0.0)) return 0;
    double end = d;
    for (int a = 0; a < 3; ++a) {
        if (!M->bounded[a]) { idx[a] = 0; s[a] = O_INF; ds[a] = O_INF; continue; }
        if (u[a] > 0.0) {
            double far = (M->lo[a] + (double)M->n[a] * M->delta[a] - p[a]) * iu[a];
            if (far < end) end = far;
        } else if (u[a] < 0.0) {
            double far = (M->lo[a] - p[a]) * iu[a];
            if (far < end) end = far;
        }
        double q = (p[a] - M->lo[a]) * M->idelta[a];
        double fq = floor(q);
        if (fq < -1.0) fq = -1.0;
        if (fq > (double)M->n[a]) fq = (double)M->n[a];
        int i = (int)fq;
        if (q == fq && u[a] < 0.0) i = i - 1;          /* on an edge moving down */
        if (i < -1) i = -1;
        idx[a] = i;
        if (u[a] > 0.0) {
            if (i >= M->n[a]) return 0;                /* beyond and moving away */
            double e = M->lo[a] + (double)(i + 1) * M->delta[a];
            s[a] = (e - p[a]) * iu[a];
            ds[a] = M->delta[a] * fabs(iu[a]);
        } else if (u[a] < 0.0) {
            if (i < 0) return 0;
            double e = M->lo[a] + (double)i * M->delta[a];
            s[a] = (e - p[a]) * iu[a];
            ds[a] = M->delta[a] * fabs(iu[a]);
        } else {
            if (i < 0 || i >= M->n[a]) return 0;
            s[a] = O_INF;
            ds[a] = O_INF;
        }
    }
    {
        double q = (t0 - M->lo[3]) * M->idelta[3];
        double fq = floor(q);
        if (fq < -1.0) fq = -1.0;
        if (fq > (double)M->n[3]) fq = (double)M->n[3];
        int i = (int)fq;
        if (i >= M->n[3]) return 0;
        idx[3] = i;
        double e = M->lo[3] + (double)(i + 1) * M->delta[3];
        s[3] = (e - t0) * v;
        ds[3] = M->delta[3] * v;
        double far = (M->lo[3] + (double)M->n[3] * M->delta[3] - t0) * v;
        if (far < end) end = far;
    }
    double sp = 0.0;
    for (;;) {
        double sn = end;
        for (int a = 0; a < 4; ++a)
            if (s[a] < sn) sn = s[a];
        if (sn > sp) {
            int in = 1;
            for (int a = 0; a < 4; ++a)
                if (idx[a] < 0 || idx[a] >= M->n[a]) in = 0;
            if (in) {
                int gt = M->G_t > 1 ? g : 0;
                size_t b = ((((size_t)gt * M->n[3] + idx[3]) * M->n[2] + idx[2]) * M->n[1] + idx[1]) *
                               M->n[0] + idx[0];
                if (tally) tally[b] += w * (sn - sp);
                pieces += 1;
            }
        }
        if (sn >= end) break;
        for (int a = 0; a < 4; ++a) {
            if (s[a] != sn) continue;
            idx[a] += (a == 3 || u[a] > 0.0) ? 1 : -1;
            s[a] = s[a] + ds[a];
        }
        sp = sn;
    }
    return pieces;
}

/* part of the segment inside the detector box (box clip of [0,d]) */
static double o_detector_len(const orc_problem *P, const double p[3], const double u[3],
                             const double iu[3], double d)
{
    double si = 0.0, so = d;
    for (int a = 0; a < 3; ++a) {
        if (u[a] == 0.0) {
            if (!(P->det_lo[a] <= p[a] && p[a] <= P->det_hi[a])) return 0.0;
            continue;
        }
        double s1 = (P->det_lo[a] - p[a]) * iu[a];
        double s2 = (P->det_hi[a] - p[a]) * iu[a];
        double nr = u[a] > 0.0 ? s1 : s2;
        double fr = u[a] > 0.0 ? s2 : s1;
        if (nr > si) si = nr;
        if (fr < so) so = fr;
    }
    return so > si ? so - si : 0.0;
}

int64_t orc_score_segment(const orc_problem *P, const double p[3], const double u[3],
                          double t0, double d, double w, int32_t g, double *tally)
{
    o_mesh M = o_mesh_make(P);
    double iu[3];
    for (int a = 0; a < 3; ++a) iu[a] = u[a] != 0.0 ? 1.0 / u[a] : 0.0;
    return o_score_mesh(&M, p, u, iu, t0, P->speed[g], d, w, g, tally);
}

/* ------------------------------------------------------------------------ */
/* Particle state and the per-history loop                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double p[3], u[3], t, w;
    int g, cell, ci;
    uint32_t tag, k, seq;
    int alive;
} o_part;

typedef struct {
    const orc_problem *P;
    o_mesh M;
    orc_result *R;
    uint64_t seed, hist;
    double xh, path_h;
    int64_t events;
    o_part *stack;
    int sp;
    int status;
    /* importance list: distinct coarse cells visited at flight starts */
    int n_imp;
    int64_t imp_cell[16];
    double imp_cnt[16], imp_xsum[16];
    double ww_lo[4], ww_inv[4];
    double *ww_map;           /* window map (NULL: network at every check) */
    int wwg_on;               /* weight-window grid planes */
    double wwg_d[3], wwg_id[3];
    int census_hit;           /* the last flight stopped at an intermediate census */
    /* k-eigenvalue mode (NULL fis: fixed-source run, no fission) */
    struct o_sites *fis;      /* sites produced in this generation, in history order */
    double k_norm;            /* site production is divided by this */
    double kcol;              /* sum of w nuSigma_f / Sigma_t over collisions */
} o_ctx;

/* Fission sites of one generation: position and outgoing group. */
typedef struct { double p[3]; int g; } o_site;
typedef struct o_sites { o_site *s; size_t n, cap; } o_sites;

static void o_site_push(o_sites *b, const double p[3], int g)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->s = (o_site *)realloc(b->s, b->cap * sizeof(o_site));
    }
    for (int a = 0; a < 3; ++a) b->s[b->n].p[a] = p[a];
    b->s[b->n].g = g;
    b->n += 1;
}

static void o_trace(o_ctx *C, o_part *q, int type, double aux)
{
    orc_result *R = C->R;
    uint32_t seq = q->seq;
    q->seq += 1u;
    if (!R->trace || R->trace_n >= R->trace_cap) return;
    orc_trace_rec *r = &R->trace[R->trace_n++];
    r->hist = C->hist;
    r->tag = q->tag;
    r->seq = seq;
    r->type = type;
    r->g = q->g;
    r->cell = q->cell;
    r->k = q->k;
    r->x = q->p[0]; r->y = q->p[1]; r->z = q->p[2]; r->t = q->t;
    r->ux = q->u[0]; r->uy = q->u[1]; r->uz = q->u[2]; r->w = q->w;
    r->aux = aux;
}

static o_stream o_part_stream(o_ctx *C, const o_part *q)
{
    o_stream s = o_stream_make(C->seed, C->hist, C->P->problem_id, q->tag);
    s.k = q->k;
    return s;
}

/* Outer boundary after a surface crossing: every axis on which the point is
 * outside (direction aware) is handled in x,y,z order: reflective faces put
 * the point on the face and reverse that direction component, vacuum faces
 * leak the particle.  A point still outside after that leaks through its first
 * failing face.  Returns the leak face or -1. */
static int o_boundary(const orc_problem *P, o_part *q)
{
    for (int a = 0; a < 3; ++a) {
        if (o_axis_in(P->outer_lo[a], P->outer_hi[a], q->p[a], q->u[a])) continue;
        int side = q->p[a] >= P->outer_hi[a] ? 1 : 0;
        int face = 2 * a + side;
        if (P->bc[face] == 1) {
            q->p[a] = side ? P->outer_hi[a] : P->outer_lo[a];
            q->u[a] = -q->u[a];
        } else {
            return face;
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (o_axis_in(P->outer_lo[a], P->outer_hi[a], q->p[a], q->u[a])) continue;
        return 2 * a + (q->p[a] >= P->outer_hi[a] ? 1 : 0);
    }
    return -1;
}

static void o_leak(o_ctx *C, o_part *q, int face)
{
    C->R->leak[face] += q->w;
    C->R->wsum[ORC_W_LEAK] += q->w;
    C->R->cnt[ORC_C_LEAK] += 1;
    q->alive = 0;
}

/* Window target from the network: y = network output at the normalised point
 * (2 s - 1 per axis, s the fraction of the outer box / of the last census
 * time, group one-hot), clamped to the range [ymin, ymax] of its training
 * targets; w_T = exp(log K - y). */
static double o_ww_net(const orc_problem *P, const float *in_xt, int32_t g)
{
    float in[4 + 16];
    for (int a = 0; a < 4; ++a) in[a] = in_xt[a];
    for (int j = 0; j < P->G; ++j) in[4 + j] = j == g ? 1.0f : 0.0f;
    float y = orc_mlp_f32(P->ww_params, 4 + P->G, P->ww_hidden, in);
    if (y < P->ww_ymin) y = P->ww_ymin;
    if (y > P->ww_ymax) y = P->ww_ymax;
    return orc_exp(P->ww_logk - (double)y);
}

static int o_has_map(const orc_problem *P)
{
    return P->ww_on && P->ww_map_n[0] > 0 && P->ww_map_n[1] > 0 && P->ww_map_n[2] > 0 &&
           P->ww_map_n[3] > 0;
}

static void o_ww_norm(const orc_problem *P, double lo[4], double inv[4])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = P->outer_lo[a];
        inv[a] = 1.0 / (P->outer_hi[a] - P->outer_lo[a]);
    }
    lo[3] = 0.0;
    inv[3] = 1.0 / P->census[P->n_census - 1];
}

/* map cell: per axis i = floor(s n) clamped to [0, n-1] */
static int64_t o_map_cell(const orc_problem *P, const double lo[4], const double inv[4],
                          const double p[3], double t, int32_t g)
{
    int64_t c = g;
    for (int a = 3; a >= 0; --a) {
        double v = a < 3 ? p[a] : t;
        double sa = (v - lo[a]) * inv[a];
        double f = floor(sa * (double)P->ww_map_n[a]);
        int64_t i = f < 0.0 ? 0 : (f >= (double)P->ww_map_n[a] ? P->ww_map_n[a] - 1 : (int64_t)f);
        c = c * P->ww_map_n[a] + i;
    }
    return c;
}

int64_t orc_ww_map(const orc_problem *P, double *out)
{
    if (!o_has_map(P)) return -1;
    const int32_t *n = P->ww_map_n;
    int64_t c = 0;
    for (int32_t g = 0; g < P->G; ++g)
        for (int32_t it = 0; it < n[3]; ++it)
            for (int32_t iz = 0; iz < n[2]; ++iz)
                for (int32_t iy = 0; iy < n[1]; ++iy)
                    for (int32_t ix = 0; ix < n[0]; ++ix) {
                        const int32_t idx[4] = {ix, iy, iz, it};
                        float in[4];
                        for (int a = 0; a < 4; ++a)
                            in[a] = (float)(2.0 * (((double)idx[a] + 0.5) / (double)n[a]) - 1.0);
                        out[c++] = o_ww_net(P, in, g);
                    }
    return c;
}

int64_t orc_ww_map_cell(const orc_problem *P, const double p[3], double t, int32_t g)
{
    if (!o_has_map(P)) return -1;
    double lo[4], inv[4];
    o_ww_norm(P, lo, inv);
    return o_map_cell(P, lo, inv, p, t, g);
}

/* Weight-window check: target w_T from the network at the particle's point
 * (or, with a map, at the centre of its map cell), window [w_L, w_U] with
 * w_L = 2 w_T / (1 + r), w_U = r w_L.  Above: split into
 * n = min(ceil(w / w_T), n_max) copies of weight w/n; the n-1 daughters go on
 * the LIFO stack with stream tags derived from one parent block.  Below:
 * roulette, survive iff xi * w_T < w with weight w_T.  No draw otherwise. */
static void o_ww(o_ctx *C, o_part *q)
{
    const orc_problem *P = C->P;
    double wt;
    if (C->ww_map) {
        wt = C->ww_map[o_map_cell(P, C->ww_lo, C->ww_inv, q->p, q->t, q->g)];
    } else {
        float in[4];
        for (int a = 0; a < 3; ++a)
            in[a] = (float)(2.0 * ((q->p[a] - C->ww_lo[a]) * C->ww_inv[a]) - 1.0);
        in[3] = (float)(2.0 * ((q->t - C->ww_lo[3]) * C->ww_inv[3]) - 1.0);
        wt = o_ww_net(P, in, q->g);
    }
    double wl = (2.0 * wt) / (1.0 + P->ww_ratio);
    double wu = P->ww_ratio * wl;
    if (q->w > wu) {
        double ratio = q->w / wt;
        int n = ratio >= (double)P->ww_nmax ? P->ww_nmax : (int)ceil(ratio);
        if (n < 2) return;
        o_stream s = o_part_stream(C, q);
        uint32_t blk[4];
        o_block(&s, blk);
        q->k = s.k;
        double wn = q->w / (double)n;
        q->w = wn;
        for (int i = 1; i < n; ++i) {
            if (C->sp >= P->stack_cap) { C->status = ORC_E_STACK; return; }
            o_part *d = &C->stack[C->sp++];
            *d = *q;
            d->tag = blk[0] + (uint32_t)i * 0x9E3779B9u;
            d->k = 0;
            d->seq = 0;
        }
        C->R->cnt[ORC_C_SPLIT] += (uint64_t)(n - 1);
        C->R->cnt[ORC_C_PARTICLE] += (uint64_t)(n - 1);
        o_trace(C, q, ORC_EV_SPLIT, (double)n);
    } else if (q->w < wl) {
        o_stream s = o_part_stream(C, q);
        double xi = o_draw(&s);
        q->k = s.k;
        if (xi * wt < q->w) {
            C->R->wsum[ORC_W_GAIN] += wt - q->w;
            q->w = wt;
            C->R->cnt[ORC_C_RR_SURVIVE] += 1;
            o_trace(C, q, ORC_EV_ROULETTE_SURVIVE, 0.0);
        } else {
            C->R->wsum[ORC_W_LOSS] += q->w;
            C->R->cnt[ORC_C_RR_KILL] += 1;
            q->alive = 0;
            o_trace(C, q, ORC_EV_ROULETTE_KILL, 0.0);
        }
    }
}

/* coarse space-time(-group) cell of a point, for the importance estimate */
static int64_t o_imp_cell(o_ctx *C, const o_part *q)
{
    const orc_problem *P = C->P;
    int ix[4];
    for (int a = 0; a < 4; ++a) {
        double x = a < 3 ? q->p[a] : q->t;
        double lo = a < 3 ? P->outer_lo[a] : 0.0;
        double hi = a < 3 ? P->outer_hi[a] : P->census[P->n_census - 1];
        double f = (x - lo) * ((double)P->imp_n[a] / (hi - lo));
        int i = (int)floor(f);
        if (i < 0) i = 0;
        if (i > P->imp_n[a] - 1) i = P->imp_n[a] - 1;
        ix[a] = i;
    }
    int64_t c = q->g;
    c = c * P->imp_n[3] + ix[3];
    c = c * P->imp_n[2] + ix[2];
    c = c * P->imp_n[1] + ix[1];
    c = c * P->imp_n[0] + ix[0];
    return c;
}

/* Forward importance estimate: every flight start in coarse cell c records
 * the detector score reached so far; at the end of the history, cell c gains
 * (final score - score at the point) per point and one unit of weight per
 * point (analog runs: all weights are 1).  At most 16 distinct cells per
 * history are kept; later new cells are dropped. */
static void o_imp_point(o_ctx *C, const o_part *q)
{
    int64_t c = o_imp_cell(C, q);
    for (int i = 0; i < C->n_imp; ++i) {
        if (C->imp_cell[i] == c) {
            C->imp_cnt[i] += 1.0;
            C->imp_xsum[i] += C->xh;
            return;
        }
    }
    if (C->n_imp < 16) {
        C->imp_cell[C->n_imp] = c;
        C->imp_cnt[C->n_imp] = 1.0;
        C->imp_xsum[C->n_imp] = C->xh;
        C->n_imp += 1;
    }
}

/* Weight-window grid (a reading: besides collisions and surface crossings,
 * the windows are checked where a flight reaches a plane of a regular grid
 * over the outer box).  Interior planes lo + k (hi - lo) / n, k = 1..n-1, per
 * axis.  Distance along u to the next plane ahead of p: moving up,
 * k = floor((p - lo) / delta) + 1; moving down, the plane at or below p, one
 * lower when p lies on it; then one further while the distance
 * (plane - p) * (1 / u) is not positive, so a particle standing on a plane
 * moves off it.  The first strict minimum in axis order x, y, z wins;
 * returns +inf when no interior plane lies ahead. */
static double o_dist_wwplane(const o_ctx *C, const double p[3], const double u[3],
                             const double iu[3], int *axis, double *plane)
{
    const orc_problem *P = C->P;
    double best = O_INF;
    int bax = -1;
    double bpl = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (u[a] == 0.0) continue;
        const double lo = P->outer_lo[a], dl = C->wwg_d[a];
        const double q = (p[a] - lo) * C->wwg_id[a];
        const double f = floor(q);
        double k = u[a] > 0.0 ? f + 1.0 : (q == f ? f - 1.0 : f);
        const double step = u[a] > 0.0 ? 1.0 : -1.0;
        double pl = lo + k * dl;
        double s = (pl - p[a]) * iu[a];
        for (int it = 0; it < 4 && !(s > 0.0); ++it) {
            k = k + step;
            pl = lo + k * dl;
            s = (pl - p[a]) * iu[a];
        }
        if (!(s > 0.0) || k < 1.0 || k > (double)(P->ww_grid_n[a] - 1)) continue;
        if (s < best) { best = s; bax = a; bpl = pl; }
    }
    *axis = bax;
    *plane = bpl;
    return best;
}

/* One flight of particle q: the candidate distances (census, surface, the
 * next weight-window grid plane when windows and a grid are on, collision),
 * the event with the tie order census < surface < grid plane < collision,
 * track-length scoring of the flight, the straight-line motion, and the event. */
static void o_flight(o_ctx *C, o_part *q)
{
    const orc_problem *P = C->P;
    orc_result *R = C->R;
    C->events += 1;
    if (C->events > P->max_events) { C->status = ORC_E_EVENT_CAP; q->alive = 0; return; }
    R->cnt[ORC_C_FLIGHT] += 1;
    if (P->imp_on) o_imp_point(C, q);

    int mat = o_material(P, q->cell);
    double sig_t = P->sigma_t[mat * P->G + q->g];
    double v = P->speed[q->g];
    double iu[3];
    for (int a = 0; a < 3; ++a) iu[a] = q->u[a] != 0.0 ? 1.0 / q->u[a] : 0.0;

    double tc = P->census[q->ci];
    double d_t = (tc - q->t) * v;
    int sax;
    double spl;
    double d_s = o_dist_surface(P, q->p, q->u, iu, &sax, &spl);
    double d_c = O_INF;
    o_stream st = o_part_stream(C, q);
    if (sig_t > 0.0) {
        double xi = o_draw(&st);
        d_c = (-orc_log(xi)) / sig_t;
    }
    q->k = st.k;

    /* weight-window grid plane (only with windows and a grid) */
    int wax = -1;
    double wpl = 0.0;
    double d_w = O_INF;
    if (C->wwg_on) d_w = o_dist_wwplane(C, q->p, q->u, iu, &wax, &wpl);

    /* ties: census, then surface, then grid plane, then collision */
    int ev;
    double d;
    if (d_t <= d_s && d_t <= d_w && d_t <= d_c) { ev = ORC_EV_CENSUS; d = d_t; }
    else if (d_s <= d_w && d_s <= d_c) { ev = ORC_EV_SURFACE; d = d_s; }
    else if (wax >= 0 && d_w <= d_c) { ev = ORC_EV_WW_PLANE; d = d_w; }
    else { ev = ORC_EV_SCATTER; d = d_c; }

    /* track-length scoring of [0, d] */
    R->cnt[ORC_C_PIECE] += (uint64_t)o_score_mesh(&C->M, q->p, q->u, iu, q->t, v, d, q->w, q->g,
                                                  R->tally_batch);
    if (P->has_detector) {
        double l = o_detector_len(P, q->p, q->u, iu, d);
        if (l > 0.0) C->xh += q->w * l;
    }
    R->wsum[ORC_W_PATH] += q->w * d;
    C->path_h += q->w * d;
    if (P->surf_on)
        R->cnt[ORC_C_SURF_CROSS] += (uint64_t)o_score_surface(&C->M, P->surf_axis, P->surf_pos, q->p,
                                                              q->u, iu, q->t, v, d, q->w, q->g,
                                                              R->surf_batch);

    /* straight-line motion over the flight: every coordinate advances by its
     * direction cosine times the distance (the time advances below, by
     * distance over speed, unless the flight ends at a census) */
    for (int a = 0; a < 3; ++a) q->p[a] += q->u[a] * d;

    if (ev == ORC_EV_CENSUS) {
        q->t = tc;
        if (q->ci == P->n_census - 1) {
            R->wsum[ORC_W_TIME_END] += q->w;
            R->cnt[ORC_C_TIME_END] += 1;
            q->alive = 0;
            o_trace(C, q, ORC_EV_TIME_END, d);
        } else {
            q->ci += 1;
            R->cnt[ORC_C_CENSUS] += 1;
            C->census_hit = 1;
            o_trace(C, q, ORC_EV_CENSUS, d);
        }
        return;
    }
    q->t = q->t + d / v;

    if (ev == ORC_EV_WW_PLANE) {
        q->p[wax] = wpl;                 /* on the plane exactly */
        R->cnt[ORC_C_WW_PLANE] += 1;
        o_trace(C, q, ORC_EV_WW_PLANE, d);
        o_ww(C, q);
        return;
    }

    if (ev == ORC_EV_SURFACE) {
        q->p[sax] = spl;
        R->cnt[ORC_C_SURFACE] += 1;
        int face = o_boundary(P, q);
        if (face >= 0) {
            o_leak(C, q, face);
            o_trace(C, q, ORC_EV_LEAK, d);
            return;
        }
        q->cell = o_locate(P, q->p, q->u);
        o_trace(C, q, ORC_EV_SURFACE, d);
        if (P->ww_on) o_ww(C, q);
        return;
    }

    /* collision; the collision estimator scores w / Sigma_t (weight before
     * the collision) into the bin of the collision point: its expectation is
     * the track length the bin receives */
    R->cnt[ORC_C_COLLISION] += 1;
    if (P->col_tally) {
        int64_t b = o_point_bin(&C->M, q->p, q->t, q->g);
        if (b >= 0) R->col_batch[b] += q->w / sig_t;
    }
    const double *ss_row = P->sigma_s + ((size_t)mat * P->G + q->g) * P->G;
    double sig_s = 0.0;
    for (int h = 0; h < P->G; ++h) sig_s = sig_s + ss_row[h];
    st = o_part_stream(C, q);
    /* k-eigenvalue mode: fission sites for the next generation.  The
     * expected number of fission neutrons from this collision, w nuSigma_f /
     * Sigma_t, is the collision estimate of the multiplication; divided by
     * the generation's normalisation k_norm it is the expected number of
     * sites, n = floor(w nuSigma_f / Sigma_t / k_norm + xi) of them (one
     * draw), each at the collision point with an outgoing group drawn from
     * the material's fission spectrum (first g' with xi sum(chi) below the
     * ascending cumulative chi; one draw per site when G > 1).  Fission is
     * part of the absorption, so the collision then goes on as before. */
    if (C->fis) {
        const double nusf = P->nu_sigma_f[mat * P->G + q->g];
        if (nusf > 0.0) {
            const double prod = q->w * nusf / sig_t;
            C->kcol += prod;
            const double xi = o_draw(&st);
            const int64_t n = (int64_t)floor(prod / C->k_norm + xi);
            const double *chi = P->chi + (size_t)mat * P->G;
            double chi_sum = 0.0;
            for (int h = 0; h < P->G; ++h) chi_sum = chi_sum + chi[h];
            for (int64_t i = 0; i < n; ++i) {
                int gs = 0;
                if (P->G > 1) {
                    const double target = o_draw(&st) * chi_sum;
                    double cum = 0.0;
                    int gn = -1, last = 0;
                    for (int h = 0; h < P->G; ++h) {
                        cum = cum + chi[h];
                        if (chi[h] > 0.0) last = h;
                        if (gn < 0 && target < cum) gn = h;
                    }
                    gs = gn >= 0 ? gn : last;
                }
                o_site_push(C->fis, q->p, gs);
            }
            q->k = st.k;
            if (n > 0) o_trace(C, q, ORC_EV_FISSION, (double)n);
        }
    }
    if (!P->implicit_capture) {
        double xi = o_draw(&st);
        q->k = st.k;
        if (!(xi * sig_t < sig_s)) {
            R->wsum[ORC_W_ABSORB] += q->w;
            R->cnt[ORC_C_ABSORB] += 1;
            q->alive = 0;
            o_trace(C, q, ORC_EV_ABSORB, d);
            return;
        }
    } else {
        double c = sig_s / sig_t;
        double wn = q->w * c;
        R->wsum[ORC_W_ABSORB] += q->w - wn;
        q->w = wn;
        if (q->w < P->w_cut) {
            double xi = o_draw(&st);
            q->k = st.k;
            if (xi * P->w_surv < q->w) {
                R->wsum[ORC_W_GAIN] += P->w_surv - q->w;
                q->w = P->w_surv;
                R->cnt[ORC_C_CUT_SURVIVE] += 1;
            } else {
                R->wsum[ORC_W_LOSS] += q->w;
                R->cnt[ORC_C_CUT_KILL] += 1;
                q->alive = 0;
                o_trace(C, q, ORC_EV_CUTOFF_KILL, d);
                return;
            }
        }
    }
    /* scatter: outgoing group by the cumulative row (first g' with
     * xi * Sigma_s,g < C_g'), then an isotropic direction */
    if (P->G > 1) {
        double xi = o_draw(&st);
        double target = xi * sig_s;
        double cum = 0.0;
        int gn = -1, last = 0;
        for (int h = 0; h < P->G; ++h) {
            cum = cum + ss_row[h];
            if (ss_row[h] > 0.0) last = h;
            if (gn < 0 && target < cum) gn = h;
        }
        q->g = gn >= 0 ? gn : last;
    }
    o_direction(&st, q->u);
    q->k = st.k;
    o_trace(C, q, ORC_EV_SCATTER, d);
    if (P->ww_on) o_ww(C, q);
}

/* Source particle of history h: position (box: lo + xi (hi-lo) per axis x,y,z),
 * time (t0 + xi (t1-t0) when t1 > t0), direction (isotropic or fixed), group,
 * unit weight; then the cell, and an immediate leak when the point lies on
 * the outer boundary moving out. */
static void o_source(o_ctx *C, o_part *q)
{
    const orc_problem *P = C->P;
    memset(q, 0, sizeof(*q));
    q->tag = 0;
    q->k = 0;
    q->seq = 0;
    o_stream st = o_part_stream(C, q);
    if (P->src_box) {
        for (int a = 0; a < 3; ++a) q->p[a] = P->src_lo[a] + o_draw(&st) * (P->src_hi[a] - P->src_lo[a]);
    } else {
        for (int a = 0; a < 3; ++a) q->p[a] = P->src_lo[a];
    }
    q->t = P->src_t0;
    if (P->src_t1 > P->src_t0) q->t = P->src_t0 + o_draw(&st) * (P->src_t1 - P->src_t0);
    if (P->src_isotropic) o_direction(&st, q->u);
    else for (int a = 0; a < 3; ++a) q->u[a] = P->src_dir[a];
    q->g = P->src_group;
    q->w = 1.0;
    q->k = st.k;
    q->alive = 1;
    q->ci = 0;
    while (q->ci < P->n_census && !(P->census[q->ci] > q->t)) q->ci += 1;
    C->R->cnt[ORC_C_PARTICLE] += 1;
    C->R->wsum[ORC_W_SOURCE] += q->w;
    q->cell = o_locate(P, q->p, q->u);
    if (q->ci >= P->n_census) {               /* born after the end time */
        C->R->wsum[ORC_W_TIME_END] += q->w;
        C->R->cnt[ORC_C_TIME_END] += 1;
        q->alive = 0;
        o_trace(C, q, ORC_EV_TIME_END, 0.0);
        return;
    }
    for (int a = 0; a < 3; ++a) {
        if (!o_axis_in(P->outer_lo[a], P->outer_hi[a], q->p[a], q->u[a])) {
            o_leak(C, q, 2 * a + (q->p[a] >= P->outer_hi[a] ? 1 : 0));
            o_trace(C, q, ORC_EV_LEAK, 0.0);
            return;
        }
    }
    o_trace(C, q, ORC_EV_SOURCE, 0.0);
}

static int o_history(o_ctx *C, uint64_t h, uint64_t slot)
{
    orc_result *R = C->R;
    C->hist = h;
    C->xh = 0.0;
    C->path_h = 0.0;
    C->events = 0;
    C->sp = 0;
    C->n_imp = 0;
    R->cnt[ORC_C_HIST] += 1;
    o_part q;
    o_source(C, &q);
    for (;;) {
        while (q.alive && C->status == ORC_OK) o_flight(C, &q);
        if (C->status != ORC_OK) return C->status;
        if (C->sp == 0) break;
        q = C->stack[--C->sp];
        q.alive = 1;
    }
    R->det[0] += C->xh;
    R->det[1] += C->xh * C->xh;
    if (C->xh > 0.0) R->cnt[ORC_C_DET_HIT] += 1;
    if (R->hist_xh) {
        R->hist_xh[2 * slot] = C->xh;
        R->hist_xh[2 * slot + 1] = C->path_h;
    }
    if (C->P->imp_on) {
        for (int i = 0; i < C->n_imp; ++i) {
            R->imp_score[C->imp_cell[i]] += C->imp_cnt[i] * C->xh - C->imp_xsum[i];
            R->imp_weight[C->imp_cell[i]] += C->imp_cnt[i];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Population control at census (census-synchronised batches).               */
/* ------------------------------------------------------------------------ */

typedef struct {
    o_part *p;
    uint64_t *slot;            /* history index within the batch */
    size_t n, cap;
} o_bank;

static void o_bank_push(o_bank *b, const o_part *q, uint64_t slot)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->p = (o_part *)realloc(b->p, b->cap * sizeof(o_part));
        b->slot = (uint64_t *)realloc(b->slot, b->cap * sizeof(uint64_t));
    }
    b->p[b->n] = *q;
    b->slot[b->n] = slot;
    b->n += 1;
}

/* Transport one banked particle (and the weight-window daughters it makes)
 * until each dies or stops at the next intermediate census, where it is
 * banked for the next step.  The history's running sums live in per-slot
 * arrays between the particle's visits. */
static int o_pc_transport(o_ctx *C, o_part q, uint64_t slot, uint64_t hist_first, o_bank *next,
                          double *xh, double *ph, int64_t *ev)
{
    C->hist = hist_first + slot;
    C->xh = xh[slot];
    C->path_h = ph[slot];
    C->events = ev[slot];
    C->sp = 0;
    for (;;) {
        while (q.alive && C->status == ORC_OK) {
            C->census_hit = 0;
            o_flight(C, &q);
            if (C->census_hit) {
                o_bank_push(next, &q, slot);
                q.alive = 0;
            }
        }
        if (C->status != ORC_OK) break;
        if (C->sp == 0) break;
        q = C->stack[--C->sp];
        q.alive = 1;
    }
    xh[slot] = C->xh;
    ph[slot] = C->path_h;
    ev[slot] = C->events;
    return C->status;
}

/* Splitting-roulette population control of a census bank to M particles,
 * M = round(pc_target * histories of the batch).  The bank's total weight is
 * summed exactly as integers floor(w * 2^32); the target weight is
 * w_T = (sum * 2^-32) / M.  Each particle draws one xi from its own stream:
 * below w_T it survives with probability w / w_T (xi * w_T < w) at weight
 * w_T; otherwise it becomes n = floor(w / w_T + xi) >= 1 particles of weight
 * w_T, the n - 1 copies taking stream tags from one further block of its
 * stream (tag + i * golden ratio, as for splits).  The expected weight of
 * every particle is kept, so tallies stay unbiased. */
static void o_pc_apply(o_ctx *C, o_bank *b, uint64_t n_batch_hist, uint64_t hist_first)
{
    const orc_problem *P = C->P;
    orc_result *R = C->R;
    if (b->n == 0) return;
    uint64_t wq = 0;
    for (size_t i = 0; i < b->n; ++i) wq += (uint64_t)floor(b->p[i].w * 4294967296.0);
    double M = floor(P->pc_target * (double)n_batch_hist + 0.5);
    if (M < 1.0) M = 1.0;
    const double wt = ((double)wq * 0x1p-32) / M;
    if (!(wt > 0.0)) return;
    o_bank out = {0};
    for (size_t i = 0; i < b->n; ++i) {
        o_part q = b->p[i];
        const uint64_t slot = b->slot[i];
        C->hist = hist_first + slot;
        o_stream st = o_part_stream(C, &q);
        const double xi = o_draw(&st);
        const double w = q.w;
        if (w < wt) {
            q.k = st.k;
            if (xi * wt < w) {
                R->wsum[ORC_W_GAIN] += wt - w;
                q.w = wt;
                o_trace(C, &q, ORC_EV_PC_KEEP, 1.0);
                o_bank_push(&out, &q, slot);
            } else {
                R->wsum[ORC_W_LOSS] += w;
                R->cnt[ORC_C_PC_KILL] += 1;
                o_trace(C, &q, ORC_EV_PC_KILL, 0.0);
            }
            continue;
        }
        const double nf = floor(w / wt + xi);
        const int64_t n = (int64_t)nf;
        const double tot = nf * wt;
        if (tot > w) R->wsum[ORC_W_GAIN] += tot - w;
        else R->wsum[ORC_W_LOSS] += w - tot;
        uint32_t blk[4] = {0, 0, 0, 0};
        if (n >= 2) o_block(&st, blk);
        q.k = st.k;
        q.w = wt;
        o_trace(C, &q, ORC_EV_PC_KEEP, nf);
        o_bank_push(&out, &q, slot);
        for (int64_t m = 1; m < n; ++m) {
            o_part d = q;
            d.tag = blk[0] + (uint32_t)m * 0x9E3779B9u;
            d.k = 0;
            d.seq = 0;
            o_bank_push(&out, &d, slot);
        }
        if (n >= 2) {
            R->cnt[ORC_C_PC_COPY] += (uint64_t)(n - 1);
            R->cnt[ORC_C_PARTICLE] += (uint64_t)(n - 1);
        }
    }
    free(b->p);
    free(b->slot);
    *b = out;
}

/* One batch [lo, hi) of the run, census step by census step: transport every
 * particle of the bank to death or the next intermediate census, apply
 * population control to the new census bank, repeat; then the per-history
 * detector statistics. */
static int o_batch_pc(o_ctx *C, uint64_t hist0, uint64_t lo, uint64_t hi)
{
    orc_result *R = C->R;
    const uint64_t nb = hi - lo;
    const uint64_t first = hist0 + lo;
    double *xh = (double *)calloc(nb, sizeof(double));
    double *ph = (double *)calloc(nb, sizeof(double));
    int64_t *ev = (int64_t *)calloc(nb, sizeof(int64_t));
    o_bank bank = {0}, next = {0};
    int st = ORC_OK;
    for (uint64_t j = 0; j < nb; ++j) {
        C->hist = first + j;
        R->cnt[ORC_C_HIST] += 1;
        o_part q;
        o_source(C, &q);
        if (q.alive) o_bank_push(&bank, &q, j);
    }
    while (bank.n > 0 && st == ORC_OK) {
        next.n = 0;
        for (size_t i = 0; i < bank.n && st == ORC_OK; ++i)
            st = o_pc_transport(C, bank.p[i], bank.slot[i], first, &next, xh, ph, ev);
        if (st != ORC_OK) break;
        o_pc_apply(C, &next, nb, first);
        o_bank tmp = bank;
        bank = next;
        next = tmp;
    }
    if (st == ORC_OK) {
        for (uint64_t j = 0; j < nb; ++j) {
            R->det[0] += xh[j];
            R->det[1] += xh[j] * xh[j];
            if (xh[j] > 0.0) R->cnt[ORC_C_DET_HIT] += 1;
            if (R->hist_xh) {
                R->hist_xh[2 * (lo + j)] = xh[j];
                R->hist_xh[2 * (lo + j) + 1] = ph[j];
            }
        }
    }
    free(bank.p); free(bank.slot); free(next.p); free(next.slot);
    free(xh); free(ph); free(ev);
    return st;
}

static int o_validate(const orc_problem *P)
{
    if (P->G < 1 || P->G > 16 || P->n_mat < 1 || P->n_census < 1) return ORC_E_INVALID;
    if (P->src_group < 0 || P->src_group >= P->G) return ORC_E_INVALID;
    for (int a = 0; a < 4; ++a)
        if (P->mesh_n[a] < 1) return ORC_E_INVALID;
    for (int i = 1; i < P->n_census; ++i)
        if (!(P->census[i] > P->census[i - 1])) return ORC_E_INVALID;
    if (P->n_batches < 1 || P->stack_cap < 0) return ORC_E_INVALID;
    if (P->ww_on && (P->ww_hidden < 1 || P->ww_hidden > 256 || P->ww_nmax < 2 || !P->ww_params))
        return ORC_E_INVALID;
    if ((P->ww_on || P->imp_on) && (isinf(P->outer_lo[0]) || isinf(P->outer_lo[1]) ||
                                    isinf(P->outer_lo[2]) || isinf(P->outer_hi[0]) ||
                                    isinf(P->outer_hi[1]) || isinf(P->outer_hi[2])))
        return ORC_E_INVALID;
    if (P->imp_on && (P->ww_on || P->implicit_capture)) return ORC_E_INVALID;
    if (P->pc_on && (P->imp_on || !(P->pc_target > 0.0))) return ORC_E_INVALID;
    if (P->surf_on && (P->surf_axis < 0 || P->surf_axis > 2 || !isfinite(P->surf_pos)))
        return ORC_E_INVALID;
    {
        int gpos = 0, gzero = 0;
        for (int a = 0; a < 3; ++a) {
            if (P->ww_grid_n[a] > 0 && P->ww_grid_n[a] <= 65536) ++gpos;
            if (P->ww_grid_n[a] == 0) ++gzero;
        }
        if (!(gpos == 3 || gzero == 3)) return ORC_E_INVALID;
        if (gpos == 3 && !P->ww_on) return ORC_E_INVALID;
    }
    if (P->ww_on) {
        int pos = 0, zero = 0;
        for (int a = 0; a < 4; ++a) {
            if (P->ww_map_n[a] > 0) ++pos;
            if (P->ww_map_n[a] == 0) ++zero;
        }
        if (!(pos == 4 || zero == 4)) return ORC_E_INVALID;
        if (pos == 4 && (double)P->ww_map_n[0] * P->ww_map_n[1] * P->ww_map_n[2] *
                                    P->ww_map_n[3] * P->G > (double)(1 << 26))
            return ORC_E_INVALID;
    }
    return ORC_OK;
}

/* 1 when any material has nuSigma_f > 0 */
static int o_fissile(const orc_problem *P)
{
    if (!P->nu_sigma_f) return 0;
    for (int i = 0; i < P->n_mat * P->G; ++i)
        if (P->nu_sigma_f[i] > 0.0) return 1;
    return 0;
}

/* Batch close-out: per bin, sum += S_b, sumsq += S_b^2 / N_b, S_b = 0, for
 * every mesh-type tally of the problem. */
static void o_closeout(o_ctx *C, size_t nbins, double nb)
{
    const orc_problem *P = C->P;
    orc_result *R = C->R;
    for (size_t i = 0; i < nbins; ++i) {
        double sb = R->tally_batch[i];
        if (sb != 0.0) {
            R->tally_sum[i] += sb;
            R->tally_sumsq[i] += sb * sb / nb;
            R->tally_batch[i] = 0.0;
        }
        if (P->col_tally) {
            double cb = R->col_batch[i];
            if (cb != 0.0) {
                R->col_sum[i] += cb;
                R->col_sumsq[i] += cb * cb / nb;
                R->col_batch[i] = 0.0;
            }
        }
    }
    if (P->surf_on) {
        int a = P->surf_axis, b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
        size_t ns = (size_t)2 * C->M.G_t * P->mesh_n[3] * P->mesh_n[b1] * P->mesh_n[b2];
        for (size_t i = 0; i < ns; ++i) {
            double sb = R->surf_batch[i];
            if (sb != 0.0) {
                R->surf_sum[i] += sb;
                R->surf_sumsq[i] += sb * sb / nb;
                R->surf_batch[i] = 0.0;
            }
        }
    }
}

int orc_run(const orc_problem *P, uint64_t seed, uint64_t hist0, uint64_t n_hist, orc_result *R)
{
    int st = o_validate(P);
    if (st != ORC_OK) return st;
    if (o_fissile(P)) return ORC_E_INVALID;     /* fission runs in k-eigenvalue mode */
    if (P->col_tally && (!R->col_batch || !R->col_sum || !R->col_sumsq)) return ORC_E_INVALID;
    if (P->surf_on && (!R->surf_batch || !R->surf_sum || !R->surf_sumsq)) return ORC_E_INVALID;
    o_ctx C;
    memset(&C, 0, sizeof(C));
    C.P = P;
    C.M = o_mesh_make(P);
    C.R = R;
    C.seed = seed;
    C.status = ORC_OK;
    C.stack = (o_part *)malloc(sizeof(o_part) * (size_t)(P->stack_cap > 0 ? P->stack_cap : 1));
    o_ww_norm(P, C.ww_lo, C.ww_inv);
    C.wwg_on = P->ww_on && P->ww_grid_n[0] > 0;
    for (int a = 0; a < 3 && C.wwg_on; ++a) {
        C.wwg_d[a] = (P->outer_hi[a] - P->outer_lo[a]) / (double)P->ww_grid_n[a];
        C.wwg_id[a] = 1.0 / C.wwg_d[a];
    }
    if (o_has_map(P)) {
        size_t cells = (size_t)P->G * P->ww_map_n[0] * P->ww_map_n[1] * P->ww_map_n[2] *
                       P->ww_map_n[3];
        C.ww_map = (double *)malloc(sizeof(double) * cells);
        orc_ww_map(P, C.ww_map);
    }
    size_t nbins = (size_t)C.M.G_t * P->mesh_n[0] * P->mesh_n[1] * P->mesh_n[2] * P->mesh_n[3];
    const uint64_t B = (uint64_t)P->n_batches;
    for (uint64_t b = 0; b < B; ++b) {
        uint64_t lo = (b * n_hist) / B, hi = ((b + 1) * n_hist) / B;
        if (hi == lo) continue;
        if (P->pc_on) {
            st = o_batch_pc(&C, hist0, lo, hi);
            if (st != ORC_OK) { free(C.stack); free(C.ww_map); return st; }
        } else {
            for (uint64_t i = lo; i < hi; ++i) {
                st = o_history(&C, hist0 + i, i);
                if (st != ORC_OK) { free(C.stack); free(C.ww_map); return st; }
            }
        }
        o_closeout(&C, nbins, (double)(hi - lo));
        R->batches_done += 1;
    }
    R->hist_done += n_hist;
    free(C.stack);
    free(C.ww_map);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* k-eigenvalue mode: power iteration on the fission source.                 */
/* ------------------------------------------------------------------------ */

/* Source particle of a generation after the first: born at a fission site
 * of the previous generation (its position and group), at t = 0 (the mode is
 * steady state), with unit weight and an isotropic direction drawn from the
 * history's own stream; then the same checks as a fixed source. */
static void o_source_site(o_ctx *C, o_part *q, const o_site *site)
{
    const orc_problem *P = C->P;
    memset(q, 0, sizeof(*q));
    o_stream st = o_part_stream(C, q);
    for (int a = 0; a < 3; ++a) q->p[a] = site->p[a];
    q->t = 0.0;
    o_direction(&st, q->u);
    q->g = site->g;
    q->w = 1.0;
    q->k = st.k;
    q->alive = 1;
    q->ci = 0;
    while (q->ci < P->n_census && !(P->census[q->ci] > q->t)) q->ci += 1;
    C->R->cnt[ORC_C_PARTICLE] += 1;
    C->R->wsum[ORC_W_SOURCE] += q->w;
    q->cell = o_locate(P, q->p, q->u);
    if (q->ci >= P->n_census) {
        C->R->wsum[ORC_W_TIME_END] += q->w;
        C->R->cnt[ORC_C_TIME_END] += 1;
        q->alive = 0;
        o_trace(C, q, ORC_EV_TIME_END, 0.0);
        return;
    }
    for (int a = 0; a < 3; ++a) {
        if (!o_axis_in(P->outer_lo[a], P->outer_hi[a], q->p[a], q->u[a])) {
            o_leak(C, q, 2 * a + (q->p[a] >= P->outer_hi[a] ? 1 : 0));
            o_trace(C, q, ORC_EV_LEAK, 0.0);
            return;
        }
    }
    o_trace(C, q, ORC_EV_SOURCE, 0.0);
}

/* One history of a generation; its detector score counts only when the
 * generation scores (an active one). */
static int o_keff_history(o_ctx *C, uint64_t h, uint64_t slot, const o_site *site, int score)
{
    orc_result *R = C->R;
    C->hist = h;
    C->xh = 0.0;
    C->path_h = 0.0;
    C->events = 0;
    C->sp = 0;
    R->cnt[ORC_C_HIST] += 1;
    o_part q;
    if (site) o_source_site(C, &q, site);
    else o_source(C, &q);
    while (q.alive && C->status == ORC_OK) o_flight(C, &q);
    if (C->status != ORC_OK) return C->status;
    if (score) {
        R->det[0] += C->xh;
        R->det[1] += C->xh * C->xh;
        if (C->xh > 0.0) R->cnt[ORC_C_DET_HIT] += 1;
    }
    if (R->hist_xh) {
        R->hist_xh[2 * slot] = C->xh;
        R->hist_xh[2 * slot + 1] = C->path_h;
    }
    return ORC_OK;
}

/* Stream tag of the draw that places a generation's comb ("keff" in ASCII). */
#define O_COMB_TAG 0x6B656666u

/* Generation g (ids g M .. g M + M - 1): the first takes the problem's
 * source, later ones the combed sites of the one before.  After the
 * generation: k_col = (sum of w nuSigma_f / Sigma_t) / M; S sites; the
 * site-count estimate k_site = k_norm S / M becomes the next k_norm, so the
 * expected population stays near M; the next source is M sites taken from
 * the S in production order by a comb with one random offset xi (drawn from
 * the stream of the next generation's first history id with tag "keff"):
 * site floor((j + xi) S / M) for j = 0..M-1 (at most S - 1), each of unit
 * weight.  An active generation closes out as one tally batch of M
 * histories; an inactive one discards what it scored. */
int orc_run_keff(const orc_problem *P, uint64_t seed, orc_keff *K, orc_result *R)
{
    int st = o_validate(P);
    if (st != ORC_OK) return st;
    if (!o_fissile(P) || !P->chi || K->M < 1 || K->M > ((uint64_t)1 << 32) || K->n_inactive < 0 ||
        K->n_active < 1 || !(K->k0 > 0.0) || P->ww_on || P->pc_on || P->imp_on)
        return ORC_E_INVALID;
    for (int m = 0; m < P->n_mat; ++m) {
        double sum = 0.0, sf = 0.0;
        for (int g = 0; g < P->G; ++g) {
            if (P->chi[m * P->G + g] < 0.0 || P->nu_sigma_f[m * P->G + g] < 0.0) return ORC_E_INVALID;
            sum += P->chi[m * P->G + g];
            sf += P->nu_sigma_f[m * P->G + g];
        }
        if (sf > 0.0 && !(sum > 0.0)) return ORC_E_INVALID;
    }
    if (P->col_tally && (!R->col_batch || !R->col_sum || !R->col_sumsq)) return ORC_E_INVALID;
    if (P->surf_on && (!R->surf_batch || !R->surf_sum || !R->surf_sumsq)) return ORC_E_INVALID;
    o_ctx C;
    memset(&C, 0, sizeof(C));
    C.P = P;
    C.M = o_mesh_make(P);
    C.R = R;
    C.seed = seed;
    C.status = ORC_OK;
    C.stack = (o_part *)malloc(sizeof(o_part));
    o_sites sites = {0};
    C.fis = &sites;
    C.k_norm = K->k0;
    const uint64_t M = K->M;
    o_site *src = NULL;
    size_t nbins = (size_t)C.M.G_t * P->mesh_n[0] * P->mesh_n[1] * P->mesh_n[2] * P->mesh_n[3];
    const int n_gen = K->n_inactive + K->n_active;
    for (int g = 0; g < n_gen && st == ORC_OK; ++g) {
        const int score = g >= K->n_inactive;
        sites.n = 0;
        C.kcol = 0.0;
        for (uint64_t j = 0; j < M; ++j) {
            st = o_keff_history(&C, (uint64_t)g * M + j, (uint64_t)g * M + j, src ? &src[j] : NULL,
                                score);
            if (st != ORC_OK) break;
        }
        if (st != ORC_OK) break;
        const uint64_t S = sites.n;
        K->k_col[g] = C.kcol / (double)M;
        K->k_site[g] = C.k_norm * (double)S / (double)M;
        K->n_sites[g] = S;
        if (score) {
            o_closeout(&C, nbins, (double)M);
            R->batches_done += 1;
            R->hist_done += M;
        } else {
            memset(R->tally_batch, 0, nbins * sizeof(double));
            if (P->col_tally) memset(R->col_batch, 0, nbins * sizeof(double));
            if (P->surf_on) {
                int a = P->surf_axis, b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
                size_t ns = (size_t)2 * C.M.G_t * P->mesh_n[3] * P->mesh_n[b1] * P->mesh_n[b2];
                memset(R->surf_batch, 0, ns * sizeof(double));
            }
        }
        if (S == 0) { st = ORC_E_EXTINCT; break; }
        o_stream cs = o_stream_make(seed, (uint64_t)(g + 1) * M, P->problem_id, O_COMB_TAG);
        const double xi = o_draw(&cs);
        if (!src) src = (o_site *)malloc(M * sizeof(o_site));
        for (uint64_t j = 0; j < M; ++j) {
            uint64_t idx = (uint64_t)floor(((double)j + xi) * (double)S / (double)M);
            if (idx > S - 1) idx = S - 1;
            src[j] = sites.s[idx];
        }
        C.k_norm = K->k_site[g];
    }
    if (st == ORC_OK && K->src_out)
        for (uint64_t j = 0; j < M; ++j) {
            for (int a = 0; a < 3; ++a) K->src_out[4 * j + a] = src[j].p[a];
            K->src_out[4 * j + 3] = (double)src[j].g;
        }
    free(sites.s);
    free(src);
    free(C.stack);
    return st;
}
