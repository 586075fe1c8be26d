/*
 * rmp_oracle.c -- plain, slow, float64 CPU reference for the raycast-and-policy pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it computes (Pantic et al., "Obstacle avoidance using raycasting and Riemannian
 * Motion Policies at kHz rates for MAVs"):
 *   - ray directions from a 2-D Halton sequence, bases 2 and 3     (Sec. III-E, Eq. 10)
 *   - the distance along each ray to the first occupied voxel       (Sec. III-E, R(x, r))
 *   - one obstacle policy (f_rep + f_damp, A_obs) per hit ray       (Sec. III-C, Eqs. 4-9)
 *   - the metric-weighted combination  f = (sum A_i)^+ sum A_i f_i  (Sec. III-A, Eq. 1;
 *                                                                    Sec. III-E, Eq. 11)
 *   - the LiDAR variant that takes beam direction and range directly (Sec. III-G)
 *
 * Readings where the paper is silent or garbled (each listed with its reason in the
 * project's design notes):
 *   R1  the exponent of the soft normalisation uses the norm: exp(-2 c |v|);
 *   R2  the obstacle unit vector is n = -r_i (the ray points toward the obstacle, the
 *       policy's vector points away from it);
 *   R3  w_r is the printed polynomial d^2/r^2 - 2d/r + 1 on [0, r], 0 beyond;
 *   R4  epsilon is a parameter (default 1e-3);
 *   R5  N rays are Halton indices 0..N-1; base 2 drives the polar angle, base 3 azimuth;
 *   R6  the ray distance is where the ray enters the first occupied voxel (3-D DDA of
 *       Amanatides & Woo 1987), on the float32 start point and float32 directions;
 *   R7  a voxel is occupied when its stored TSDF value is <= 0 (uint8 maps: != 0);
 *   R8  the pseudo-inverse drops eigenvalues <= rank_tol * lambda_max;
 *   R9  nothing within max_range, or leaving the grid, is a miss and contributes 0;
 *   R14 exact DDA ties step the lowest axis index; near-ties (< 1e-5 voxel) are flagged
 *       and both orders are enumerated into an admissible set;
 *   R21 the ESDF is the exact centre-to-centre Euclidean distance transform of the occupancy;
 *   R22 the ESDF policy reads the distance of x's voxel and central differences of its six
 *       neighbours, and evaluates the obstacle policy once for that (direction, distance);
 *   R20 optional sub-voxel distance: one secant step on the trilinearly interpolated TSDF
 *       across the entry point of the hit voxel (the paper's raycaster steps a continuous
 *       distance field; the walk's voxel-face distance is its voxel-exact stand-in).
 *
 * Parity unpinned: the constants epsilon, rank_tol and min_range, and readings R1-R3,
 * which nothing printed in the paper can confirm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------------- */
/* types                                                                               */
/* ---------------------------------------------------------------------------------- */

typedef struct {
    int32_t nx, ny, nz;
    int32_t dtype;        /* 0: float32 TSDF, 1: float16 TSDF (binary16 bits), 2: uint8 occupancy */
    double h;             /* voxel edge length, metres */
    double origin[3];     /* world coordinate of the grid's minimum corner */
    const void *data;     /* x fastest: lin = i + nx*(j + ny*k) */
} orc_map;

typedef struct {
    double c, eta_rep, nu_rep, eta_damp, nu_damp, radius;   /* Table I columns */
    double eps, max_range, rank_tol, min_range;             /* readings R4, R9, R8, R11 */
    double subvoxel;      /* non-zero: refine each hit distance (R20) before the policy */
} orc_params;

typedef struct {
    double S[9];          /* sum_i A_i, row major */
    double b[3];          /* sum_i A_i (f_rep,i + f_damp,i) */
    double f[3];          /* resolved acceleration S^+ b */
    double lam[3];        /* eigenvalues of S, ascending */
    int32_t rank;
    int32_t n_hit;        /* rays that hit an occupied voxel within range */
    int32_t n_contrib;    /* hits with d < radius and xdot . r > 0: non-zero metric */
    int32_t n_tie;        /* rays carrying the TIE flag */
    uint32_t flags;       /* query flags: ORC_Q_* */
    int32_t pad;
    int64_t visits;       /* voxels read, summed over rays */
} orc_result;

enum {
    ORC_TIE = 1u,             /* a near-tie between two axis crossings on the path */
    ORC_RANGE_TIE = 2u,       /* termination within 1e-5 voxel of max_range */
    ORC_START_FACE = 4u,      /* start coordinate within 1e-5 of a voxel face */
    ORC_IN_COLLISION = 8u     /* start voxel occupied */
};
enum { ORC_Q_ILL = 1u, ORC_Q_IN_COLLISION = 2u, ORC_Q_TIE = 4u };

#define ORC_TIE_BAND 1e-5
#define ORC_MAX_ALT 16
#define ORC_MAX_BRANCH_DEPTH 3

/* ---------------------------------------------------------------------------------- */
/* Halton directions (Sec. III-E, Eq. 10)                                              */
/* ---------------------------------------------------------------------------------- */

/* Radical inverse of i in base b: the base-b digits of i mirrored about the radix point. */
double orc_radical_inverse(uint64_t i, uint32_t base)
{
    double r = 0.0;
    double f = 1.0 / (double)base;
    while (i > 0) {
        r += f * (double)(i % base);
        i /= base;
        f /= (double)base;
    }
    return r;
}

/* Ray i: polar angle phi = acos(1 - 2 H(i,2)), azimuth theta = 2 pi H(i,3), and
 * r = (sin phi cos theta, sin phi sin theta, cos phi), each component rounded to float32.
 * sin(acos z) = sqrt(1 - z^2) on [0, pi], so the acos is not evaluated. */
void orc_directions(int32_t n, float *out)
{
    for (int32_t i = 0; i < n; ++i) {
        double u = orc_radical_inverse((uint64_t)i, 2);
        double w = orc_radical_inverse((uint64_t)i, 3);
        double z = 1.0 - 2.0 * u;
        double s = 1.0 - z * z;
        double rho = sqrt(s > 0.0 ? s : 0.0);
        double th = 2.0 * M_PI * w;
        out[3 * i + 0] = (float)(rho * cos(th));
        out[3 * i + 1] = (float)(rho * sin(th));
        out[3 * i + 2] = (float)z;
    }
}

/* ---------------------------------------------------------------------------------- */
/* map access (reading R7)                                                             */
/* ---------------------------------------------------------------------------------- */

static double half_to_double(uint16_t hb)
{
    int sign = (hb >> 15) & 1;
    int e = (hb >> 10) & 0x1f;
    int m = hb & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);                 /* zero or subnormal */
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(m + 1024), e - 25);
    return sign ? -v : v;
}

static int occupied(const orc_map *m, int64_t lin)
{
    switch (m->dtype) {
    case 0: return ((const float *)m->data)[lin] <= 0.0f;
    case 1: return half_to_double(((const uint16_t *)m->data)[lin]) <= 0.0;
    default: return ((const uint8_t *)m->data)[lin] != 0;
    }
}

static int64_t lin_index(const orc_map *m, const int32_t v[3])
{
    return (int64_t)v[0] + (int64_t)m->nx * ((int64_t)v[1] + (int64_t)m->ny * (int64_t)v[2]);
}

static int inside(const orc_map *m, const int32_t v[3])
{
    return v[0] >= 0 && v[1] >= 0 && v[2] >= 0 && v[0] < m->nx && v[1] < m->ny && v[2] < m->nz;
}

/* Grid-space start g = fp32((x - origin) / h), each component in float64 then rounded once.
 * Returns 0 when the start lies outside [0, n) on some axis. */
int orc_grid_start(const orc_map *m, const double x[3], float g[3])
{
    const int32_t n[3] = {m->nx, m->ny, m->nz};
    for (int a = 0; a < 3; ++a) {
        g[a] = (float)((x[a] - m->origin[a]) / m->h);
        if (!(g[a] >= 0.0f) || !(g[a] < (float)n[a]))
            return 0;
    }
    return 1;
}

/* ---------------------------------------------------------------------------------- */
/* voxel traversal: Amanatides & Woo 3-D DDA on float32 inputs in float64 (R6, R14)     */
/* ---------------------------------------------------------------------------------- */

typedef struct {
    const orc_map *m;
    double g[3];          /* start, voxel units (exact float32 values) */
    double r[3];          /* direction (exact float32 values, not renormalised) */
    double max_range;
    /* primary outcome */
    int32_t hit;
    double d;
    uint32_t flags;
    int32_t visits;
    /* admissible outcomes, primary first */
    int32_t n_alt;
    int32_t alt_hit[ORC_MAX_ALT];
    double alt_d[ORC_MAX_ALT];
} trace_ctx;

static void add_alt(trace_ctx *tc, int32_t hit, double d)
{
    for (int k = 0; k < tc->n_alt; ++k)
        if (tc->alt_hit[k] == hit && (tc->alt_d[k] == d || (isinf(d) && isinf(tc->alt_d[k]))))
            return;
    if (tc->n_alt < ORC_MAX_ALT) {
        tc->alt_hit[tc->n_alt] = hit;
        tc->alt_d[tc->n_alt] = d;
        tc->n_alt++;
    }
}

/* Crossing parameter of the next face along axis a, measured from the start point and
 * always computed from the integer boundary (never accumulated). */
static double crossing(const trace_ctx *tc, const int32_t v[3], int a)
{
    if (tc->r[a] > 0.0) return ((double)(v[a] + 1) - tc->g[a]) / tc->r[a];
    if (tc->r[a] < 0.0) return ((double)v[a] - tc->g[a]) / tc->r[a];
    return INFINITY;
}

/*
 * Walk from voxel v.  `forced` >= 0 makes the first step go along that axis (used to
 * enumerate the other order at a near-tie); `skip_range` ignores the range test once (the
 * other outcome of a range near-tie).  Only the primary walk (primary = 1) records the
 * ray's outcome, flags and visit count; every walk adds its outcome to the admissible set.
 */
static void walk(trace_ctx *tc, int32_t v0[3], int forced, int skip_range, int depth, int primary)
{
    const orc_map *m = tc->m;
    int32_t v[3] = {v0[0], v0[1], v0[2]};
    for (;;) {
        double T[3];
        for (int a = 0; a < 3; ++a) T[a] = crossing(tc, v, a);
        int a = 0;                                  /* argmin, lowest axis on exact ties */
        if (T[1] < T[a]) a = 1;
        if (T[2] < T[a]) a = 2;
        if (forced >= 0) {
            a = forced;
            forced = -1;
        } else {
            for (int bax = 0; bax < 3; ++bax) {
                if (bax == a || !(T[bax] - T[a] < ORC_TIE_BAND)) continue;
                if (primary) tc->flags |= ORC_TIE;
                if (depth < ORC_MAX_BRANCH_DEPTH)
                    walk(tc, v, bax, 0, depth + 1, 0);
            }
        }
        double t = T[a];
        double dist = t * m->h;
        int beyond = dist > tc->max_range;
        if (fabs(dist - tc->max_range) < ORC_TIE_BAND * m->h) {
            if (primary) tc->flags |= ORC_RANGE_TIE;
            if (depth < ORC_MAX_BRANCH_DEPTH) {
                if (beyond && !skip_range)
                    walk(tc, v, a, 1, depth + 1, 0);       /* the ray reaches this face */
                else if (!beyond)
                    add_alt(tc, -1, INFINITY);              /* the ray stops short */
            }
        }
        if (beyond && !skip_range) {                        /* R9: nothing within range */
            if (primary) { tc->hit = -1; tc->d = INFINITY; }
            add_alt(tc, -1, INFINITY);
            return;
        }
        skip_range = 0;
        v[a] += tc->r[a] > 0.0 ? 1 : -1;
        if (!inside(m, v)) {                                /* R9: leaving the grid */
            if (primary) { tc->hit = -1; tc->d = INFINITY; }
            add_alt(tc, -1, INFINITY);
            return;
        }
        if (primary) tc->visits++;
        int64_t lin = lin_index(m, v);
        if (occupied(m, lin)) {
            if (primary) { tc->hit = (int32_t)lin; tc->d = dist; }
            add_alt(tc, (int32_t)lin, dist);
            return;
        }
    }
}

/* Trace one ray from grid start g along r.  The start voxel is assumed free. */
static void trace_one(trace_ctx *tc, const float g[3], const float r[3])
{
    for (int a = 0; a < 3; ++a) {
        tc->g[a] = (double)g[a];
        tc->r[a] = (double)r[a];
    }
    tc->hit = -1;
    tc->d = INFINITY;
    tc->flags = 0;
    tc->visits = 1;                  /* the start voxel */
    tc->n_alt = 0;
    for (int a = 0; a < 3; ++a) {
        double fr = tc->g[a] - floor(tc->g[a]);
        if (fr < ORC_TIE_BAND || 1.0 - fr < ORC_TIE_BAND) tc->flags |= ORC_START_FACE;
    }
    int32_t v0[3] = {(int32_t)floor(tc->g[0]), (int32_t)floor(tc->g[1]), (int32_t)floor(tc->g[2])};
    int32_t alt_hit[ORC_MAX_ALT];
    double alt_d[ORC_MAX_ALT];
    walk(tc, v0, -1, 0, 0, 1);
    /* put the primary outcome first in the admissible list */
    int n = 0;
    alt_hit[n] = tc->hit; alt_d[n] = tc->d; n++;
    for (int k = 0; k < tc->n_alt; ++k) {
        if (tc->alt_hit[k] == tc->hit && (tc->alt_d[k] == tc->d || (isinf(tc->d) && isinf(tc->alt_d[k]))))
            continue;
        if (n < ORC_MAX_ALT) { alt_hit[n] = tc->alt_hit[k]; alt_d[n] = tc->alt_d[k]; n++; }
    }
    memcpy(tc->alt_hit, alt_hit, sizeof(alt_hit));
    memcpy(tc->alt_d, alt_d, sizeof(alt_d));
    tc->n_alt = n;
}

/*
 * Trace rays dirs[0..n) from grid start g.  Per-ray outputs (any may be NULL):
 *   hit[n]   linear index of the first occupied voxel, -1 on a miss
 *   d[n]     distance in metres to where the ray enters it (+inf on a miss)
 *   flags[n] ORC_* flags
 *   visits[n] voxels read (start voxel included)
 *   alt_n[n], alt_hit[n*16], alt_d[n*16]  admissible outcomes, primary first
 * Returns the number of rays traced, or -1 if g is outside the grid.
 */
int32_t orc_trace(const orc_map *m, const float g[3], const float *dirs, int32_t n, double max_range,
                  int32_t *hit, double *d, uint32_t *flags, int32_t *visits,
                  int32_t *alt_n, int32_t *alt_hit, double *alt_d, int32_t nthreads)
{
    const int32_t nn[3] = {m->nx, m->ny, m->nz};
    for (int a = 0; a < 3; ++a)
        if (!(g[a] >= 0.0f) || !(g[a] < (float)nn[a])) return -1;
    int32_t v0[3] = {(int32_t)floorf(g[0]), (int32_t)floorf(g[1]), (int32_t)floorf(g[2])};
    int64_t lin0 = lin_index(m, v0);
    int in_coll = occupied(m, lin0);
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int32_t i = 0; i < n; ++i) {
        trace_ctx tc;
        memset(&tc, 0, sizeof tc);
        tc.m = m;
        tc.max_range = max_range;
        if (in_coll) {                              /* R10: every ray hits at distance 0 */
            tc.hit = (int32_t)lin0; tc.d = 0.0; tc.flags = ORC_IN_COLLISION; tc.visits = 1;
            tc.n_alt = 1; tc.alt_hit[0] = tc.hit; tc.alt_d[0] = 0.0;
        } else {
            trace_one(&tc, g, dirs + 3 * (int64_t)i);
        }
        if (hit) hit[i] = tc.hit;
        if (d) d[i] = tc.d;
        if (flags) flags[i] = tc.flags;
        if (visits) visits[i] = tc.visits;
        if (alt_n) alt_n[i] = tc.n_alt;
        if (alt_hit)
            for (int k = 0; k < ORC_MAX_ALT; ++k) alt_hit[(int64_t)i * ORC_MAX_ALT + k] = k < tc.n_alt ? tc.alt_hit[k] : -2;
        if (alt_d)
            for (int k = 0; k < ORC_MAX_ALT; ++k) alt_d[(int64_t)i * ORC_MAX_ALT + k] = k < tc.n_alt ? tc.alt_d[k] : NAN;
    }
    return n;
}

/* ---------------------------------------------------------------------------------- */
/* sub-voxel hit distance (reading R20)                                                 */
/* ---------------------------------------------------------------------------------- */

/* Stored TSDF value of voxel (i, j, k), indices clamped into the grid, as float64. */
static double stored_value(const orc_map *m, int64_t i, int64_t j, int64_t k)
{
    i = i < 0 ? 0 : (i >= m->nx ? m->nx - 1 : i);
    j = j < 0 ? 0 : (j >= m->ny ? m->ny - 1 : j);
    k = k < 0 ? 0 : (k >= m->nz ? m->nz - 1 : k);
    const int64_t lin = i + (int64_t)m->nx * (j + (int64_t)m->ny * k);
    if (m->dtype == 0) return (double)((const float *)m->data)[lin];
    return half_to_double(((const uint16_t *)m->data)[lin]);
}

/* The continuous field: trilinear interpolation of the stored values, which sit at the voxel
 * centres (grid coordinates i + 1/2).  p is in grid coordinates. */
double orc_field(const orc_map *m, const double p[3])
{
    double u[3], f[3];
    int64_t i0[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = p[a] - 0.5;
        i0[a] = (int64_t)floor(u[a]);
        f[a] = u[a] - (double)i0[a];
    }
    double c[2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
            const double a0 = stored_value(m, i0[0], i0[1] + dy, i0[2] + dz);
            const double a1 = stored_value(m, i0[0] + 1, i0[1] + dy, i0[2] + dz);
            c[dz][dy] = a0 + f[0] * (a1 - a0);          /* along x */
        }
    const double e0 = c[0][0] + f[1] * (c[0][1] - c[0][0]);   /* along y, z = 0 */
    const double e1 = c[1][0] + f[1] * (c[1][1] - c[1][0]);   /* along y, z = 1 */
    return e0 + f[2] * (e1 - e0);                              /* along z */
}

/*
 * Refined distance of a hit (R20).  d is the exact walk's distance in metres to where the ray
 * from grid start g along r enters its first occupied voxel.  With t = d / h (grid units), the
 * field is sampled along the ray at t_k = max(t + k/2 - 3/2, 0), k = 0..7 (from 1.5 voxels
 * before the entry to 2 voxels after it, a window that held the field's zero crossing for
 * every ray measured on an oblique plane).  At the first k with phi_k > 0 >= phi_k+1 one secant
 * step gives t* = t_k + (t_k+1 - t_k) phi_k / (phi_k - phi_k+1), and the result is t* h.
 * Without such a sign change (and for misses and d = 0) d is returned unchanged.
 */
double orc_subvoxel(const orc_map *m, const float g[3], const float r[3], double d)
{
    if (!(d > 0.0) || isinf(d) || m->dtype == 2) return d;
    const double t = d / m->h;
    double tk[8], phi[8];
    for (int k = 0; k < 8; ++k) {
        const double s = t + 0.5 * (double)k - 1.5;
        tk[k] = s > 0.0 ? s : 0.0;
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = (double)g[a] + tk[k] * (double)r[a];
        phi[k] = orc_field(m, p);
    }
    for (int k = 0; k < 7; ++k)
        if (phi[k] > 0.0 && phi[k + 1] <= 0.0) {
            const double ts = tk[k] + (tk[k + 1] - tk[k]) * (phi[k] / (phi[k] - phi[k + 1]));
            return ts * m->h;
        }
    return d;
}

/* ---------------------------------------------------------------------------------- */
/* exact Euclidean distance transform of the occupancy (the ESDF of Sec. III-D, R21)    */
/* ---------------------------------------------------------------------------------- */

/*
 * out[lin] = min over occupied voxels o of |c(lin) - c(o)|^2 in voxel units (centre to
 * centre, an integer), 0 on occupied voxels, -1 everywhere when no voxel is occupied.  The
 * squared distance separates over the axes: first the distance to the nearest occupied voxel
 * of the same x row, then min over j of (g_j + (i - j)^2) along y and along z, each minimum
 * taken over every j of the line (no envelope tricks).
 */
int32_t orc_edt(const orc_map *m, int32_t *out)
{
    const int64_t nx = m->nx, ny = m->ny, nz = m->nz, n = nx * ny * nz;
    const int64_t INF = (int64_t)1 << 40;
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *line = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz)));
    if (!g || !line) { free(g); free(line); return -1; }
    int any = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j) {
            const int64_t row = nx * (j + ny * k);
            for (int64_t i = 0; i < nx; ++i) {
                int64_t best = INF;
                for (int64_t o = 0; o < nx; ++o)
                    if (occupied(m, row + o)) {
                        const int64_t dd = (i - o) * (i - o);
                        if (dd < best) best = dd;
                    }
                g[row + i] = best;
                any |= best == 0;
            }
        }
    /* along y, then along z */
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t len = pass == 0 ? ny : nz, stride = pass == 0 ? nx : nx * ny;
        const int64_t n_lines = n / len;
        for (int64_t l = 0; l < n_lines; ++l) {
            /* line l: base index of its first element */
            const int64_t base = pass == 0 ? (l % nx) + nx * ny * (l / nx) : l;
            for (int64_t i = 0; i < len; ++i) line[i] = g[base + i * stride];
            for (int64_t i = 0; i < len; ++i) {
                int64_t best = INF;
                for (int64_t j2 = 0; j2 < len; ++j2) {
                    if (line[j2] >= INF) continue;
                    const int64_t v = line[j2] + (i - j2) * (i - j2);
                    if (v < best) best = v;
                }
                g[base + i * stride] = best;
            }
        }
    }
    for (int64_t q = 0; q < n; ++q) out[q] = any ? (int32_t)g[q] : -1;
    free(g);
    free(line);
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* per-ray obstacle policy (Sec. III-C, Eqs. 4-9; readings R1-R4)                      */
/* ---------------------------------------------------------------------------------- */

/* Soft normalisation s(v) = v / (|v| + c log(1 + exp(-2 c |v|)))   (Eq. 4, reading R1). */
void orc_soft_normalize(const double v[3], double c, double out[3])
{
    double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double den = nv + c * log1p(exp(-2.0 * c * nv));
    for (int k = 0; k < 3; ++k) out[k] = v[k] / den;
}

/* Distance weight w_r(d) = d^2/r^2 - 2 d / r + 1 on [0, r], 0 beyond (Eq. 9, reading R3). */
double orc_weight(double d, double r)
{
    if (d > r) return 0.0;
    return d * d / (r * r) - 2.0 * d / r + 1.0;
}

/*
 * One obstacle policy for a ray with direction rhat (toward the obstacle) and distance d,
 * robot velocity v.  Writes A_obs (3x3, row major) and b = A_obs (f_rep + f_damp).
 *   n      = -rhat                                   unit vector away from the obstacle (R2)
 *   f_rep  = eta_rep exp(-d / nu_rep) n              (Eq. 6)
 *   g_obs  = max(0, -v.n)^2 n                        (Eq. 7)
 *   f_damp = eta_damp / (d / nu_damp + eps) g_obs    (Eq. 8)
 *   A_obs  = w_r(d) s(f_damp) s(f_damp)^T            (Eq. 9)
 */
void orc_rmp_ray(const orc_params *p, const double rhat[3], double d, const double v[3],
                 double A[9], double b[3])
{
    double n[3] = {-rhat[0], -rhat[1], -rhat[2]};
    double erep = p->eta_rep * exp(-d / p->nu_rep);
    double f_rep[3] = {erep * n[0], erep * n[1], erep * n[2]};
    double vn = -(v[0] * n[0] + v[1] * n[1] + v[2] * n[2]);
    double mx = vn > 0.0 ? vn : 0.0;
    double g_obs[3] = {mx * mx * n[0], mx * mx * n[1], mx * mx * n[2]};
    double kd = p->eta_damp / (d / p->nu_damp + p->eps);
    double f_damp[3] = {kd * g_obs[0], kd * g_obs[1], kd * g_obs[2]};
    double s[3];
    orc_soft_normalize(f_damp, p->c, s);
    double w = orc_weight(d, p->radius);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[3 * i + j] = w * s[i] * s[j];
    double f_obs[3] = {f_rep[0] + f_damp[0], f_rep[1] + f_damp[1], f_rep[2] + f_damp[2]};
    for (int i = 0; i < 3; ++i)
        b[i] = A[3 * i + 0] * f_obs[0] + A[3 * i + 1] * f_obs[1] + A[3 * i + 2] * f_obs[2];
}

/* ---------------------------------------------------------------------------------- */
/* resolve: f = S^+ b (Eq. 1, reading R8)                                              */
/* ---------------------------------------------------------------------------------- */

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: S = Q diag(lam) Q^T,
 * columns of Q are eigenvectors, eigenvalues returned ascending. */
void orc_sym3_eig(const double S_in[9], double lam[3], double Q[9])
{
    double S[3][3], V[3][3];
    double frob = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            S[i][j] = 0.5 * (S_in[3 * i + j] + S_in[3 * j + i]);
            V[i][j] = i == j ? 1.0 : 0.0;
            frob += S[i][j] * S[i][j];
        }
    frob = sqrt(frob);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = sqrt(S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2]);
        if (off <= 1e-15 * frob || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (S[p][q] == 0.0) continue;
                /* rotation angle that zeroes S[p][q] */
                double theta = (S[q][q] - S[p][p]) / (2.0 * S[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                for (int k = 0; k < 3; ++k) {          /* S <- S J  */
                    double skp = S[k][p], skq = S[k][q];
                    S[k][p] = c * skp - s * skq;
                    S[k][q] = s * skp + c * skq;
                }
                for (int k = 0; k < 3; ++k) {          /* S <- J^T S */
                    double spk = S[p][k], sqk = S[q][k];
                    S[p][k] = c * spk - s * sqk;
                    S[q][k] = s * spk + c * sqk;
                }
                for (int k = 0; k < 3; ++k) {          /* V <- V J  */
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int idx[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)                         /* sort ascending */
        for (int j = i + 1; j < 3; ++j)
            if (S[idx[j]][idx[j]] < S[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
    for (int k = 0; k < 3; ++k) {
        lam[k] = S[idx[k]][idx[k]];
        for (int i = 0; i < 3; ++i) Q[3 * i + k] = V[i][idx[k]];
    }
}

/* f = sum over kept eigenpairs of q_j (q_j . b) / lam_j, keeping lam_j > rank_tol * lam_max.
 * ILL when an eigenvalue lies within a factor 10 of the cut, or the kept condition
 * number exceeds 1e3. */
void orc_resolve(const double S[9], const double b[3], double rank_tol, double f[3],
                 double lam[3], int32_t *rank, uint32_t *qflags)
{
    double Q[9];
    orc_sym3_eig(S, lam, Q);
    f[0] = f[1] = f[2] = 0.0;
    *rank = 0;
    double lmax = lam[2];
    if (!(lmax > 0.0)) return;
    double tau = rank_tol * lmax;
    double lmin_kept = lmax;
    for (int j = 0; j < 3; ++j) {
        if (lam[j] >= 0.1 * tau && lam[j] <= 10.0 * tau) *qflags |= ORC_Q_ILL;
        if (!(lam[j] > tau)) continue;
        (*rank)++;
        if (lam[j] < lmin_kept) lmin_kept = lam[j];
        double qb = Q[0 * 3 + j] * b[0] + Q[1 * 3 + j] * b[1] + Q[2 * 3 + j] * b[2];
        for (int i = 0; i < 3; ++i) f[i] += Q[i * 3 + j] * qb / lam[j];
    }
    if (lmax / lmin_kept > 1e3) *qflags |= ORC_Q_ILL;
}

/* ---------------------------------------------------------------------------------- */
/* compensated sums (Neumaier) and the combination of Eq. 11                           */
/* ---------------------------------------------------------------------------------- */

typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/*
 * Combine per-ray outcomes into one policy.  rhat[n*3] (float64 copies of the directions),
 * d[n] distances (+inf or a negative hit flag marks a miss: hit[i] < 0).
 */
void orc_combine(const orc_params *p, const double *rhat, const double *d, const int32_t *hit,
                 int32_t n, const double v[3], orc_result *out)
{
    nsum SA[9], sb[3];
    memset(SA, 0, sizeof SA);
    memset(sb, 0, sizeof sb);
    int32_t n_hit = 0, n_contrib = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (hit[i] < 0) continue;                 /* a miss contributes nothing (R9) */
        n_hit++;
        double A[9], b[3];
        const double *rh = rhat + 3 * (int64_t)i;
        orc_rmp_ray(p, rh, d[i], v, A, b);
        for (int k = 0; k < 9; ++k) nadd(&SA[k], A[k]);
        for (int k = 0; k < 3; ++k) nadd(&sb[k], b[k]);
        /* the metric is non-zero exactly when w_r(d) > 0 and g_obs != 0 */
        double vn = -(v[0] * -rh[0] + v[1] * -rh[1] + v[2] * -rh[2]);
        n_contrib += d[i] < p->radius && vn > 0.0;
    }
    for (int k = 0; k < 9; ++k) out->S[k] = SA[k].s + SA[k].c;
    for (int k = 0; k < 3; ++k) out->b[k] = sb[k].s + sb[k].c;
    out->n_hit = n_hit;
    out->n_contrib = n_contrib;
    orc_resolve(out->S, out->b, p->rank_tol, out->f, out->lam, &out->rank, &out->flags);
}

/*
 * The full map query: start from world position x, cast the first n Halton rays
 * (dirs = orc_directions output), evaluate one policy per hit, combine and resolve.
 * Returns 0, or -1 when x is outside the grid.
 */
int32_t orc_query(const orc_map *m, const double x[3], const double v[3], int32_t n,
                  const float *dirs, const orc_params *p, int32_t nthreads, orc_result *out)
{
    memset(out, 0, sizeof *out);
    float g[3];
    if (!orc_grid_start(m, x, g)) return -1;
    int32_t *hit = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    uint32_t *fl = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int32_t *vis = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *rh = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_trace(m, g, dirs, n, p->max_range, hit, d, fl, vis, NULL, NULL, NULL, nthreads);
    if (p->subvoxel != 0.0)
        for (int32_t i = 0; i < n; ++i) d[i] = orc_subvoxel(m, g, dirs + 3 * (int64_t)i, d[i]);
    int64_t visits = 0;
    int32_t n_tie = 0;
    for (int32_t i = 0; i < n; ++i) {
        visits += vis[i];
        n_tie += (fl[i] & ORC_TIE) != 0;
        for (int k = 0; k < 3; ++k) rh[3 * i + k] = (double)dirs[3 * i + k];
    }
    orc_combine(p, rh, d, hit, n, v, out);
    out->visits = visits;
    out->n_tie = n_tie;
    if (n_tie) out->flags |= ORC_Q_TIE;
    if (n > 0 && (fl[0] & ORC_IN_COLLISION)) out->flags |= ORC_Q_IN_COLLISION;
    free(hit); free(d); free(fl); free(vis); free(rh);
    return 0;
}

/*
 * LiDAR scan policy (Sec. III-G, reading R11): each point p, robot-relative in a
 * world-aligned frame, gives direction p/|p| and distance |p|.  Non-finite points and
 * points closer than min_range (dropouts encoded as the origin, returns from the vehicle)
 * are skipped.
 */
int32_t orc_scan(const float *pts, int32_t n, const double v[3], const orc_params *p, orc_result *out)
{
    memset(out, 0, sizeof *out);
    double *rh = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t *hit = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        double q[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
        double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        int ok = isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && nq >= p->min_range;
        hit[i] = ok ? i : -1;
        d[i] = ok ? nq : INFINITY;
        for (int k = 0; k < 3; ++k) rh[3 * i + k] = ok ? q[k] / nq : 0.0;
    }
    orc_combine(p, rh, d, hit, n, v, out);
    free(rh); free(d); free(hit);
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* single-lookup ESDF policy (Sec. III-D, reading R22)                                 */
/* ---------------------------------------------------------------------------------- */

/* Distance in metres at voxel (i, j, k) (indices clamped into the grid) from the squared
 * distance transform sq; -1 when the grid holds no occupied voxel. */
static double esdf_at(const orc_map *m, const int32_t *sq, int64_t i, int64_t j, int64_t k)
{
    i = i < 0 ? 0 : (i >= m->nx ? m->nx - 1 : i);
    j = j < 0 ? 0 : (j >= m->ny ? m->ny - 1 : j);
    k = k < 0 ? 0 : (k >= m->nz ? m->nz - 1 : k);
    const int32_t q = sq[i + (int64_t)m->nx * (j + (int64_t)m->ny * k)];
    return q < 0 ? -1.0 : m->h * sqrt((double)q);
}

/*
 * The ESDF policy at x: d = the distance stored for x's voxel, its gradient by central
 * differences over the six neighbour voxels (clamped at the grid edge, divided by 2h), the
 * obstacle direction r = -grad / |grad|, and the obstacle policy of Eqs. 4-9 for that one
 * (r, d), resolved like a query.  No occupied voxel in the grid, or a zero gradient: no
 * policy (all sums zero).  An occupied voxel at x sets ORC_Q_IN_COLLISION.
 */
int32_t orc_esdf_query(const orc_map *m, const int32_t *sq, const double x[3], const double v[3],
                       const orc_params *p, orc_result *out)
{
    memset(out, 0, sizeof *out);
    float g[3];
    if (!orc_grid_start(m, x, g)) return -1;
    const int64_t c[3] = {(int64_t)floorf(g[0]), (int64_t)floorf(g[1]), (int64_t)floorf(g[2])};
    const double d = esdf_at(m, sq, c[0], c[1], c[2]);
    if (d < 0.0) return 0;
    if (d == 0.0) out->flags |= ORC_Q_IN_COLLISION;
    double grad[3];
    for (int a = 0; a < 3; ++a) {
        int64_t hi[3] = {c[0], c[1], c[2]}, lo[3] = {c[0], c[1], c[2]};
        hi[a] += 1;
        lo[a] -= 1;
        grad[a] = (esdf_at(m, sq, hi[0], hi[1], hi[2]) - esdf_at(m, sq, lo[0], lo[1], lo[2])) / (2.0 * m->h);
    }
    const double gn = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    if (!(gn > 0.0)) return 0;
    const double rhat[3] = {-grad[0] / gn, -grad[1] / gn, -grad[2] / gn};
    double A[9], b[3];
    orc_rmp_ray(p, rhat, d, v, A, b);
    memcpy(out->S, A, sizeof A);
    memcpy(out->b, b, sizeof b);
    out->n_hit = 1;
    out->n_contrib = d < p->radius && (v[0] * rhat[0] + v[1] * rhat[1] + v[2] * rhat[2]) > 0.0;
    orc_resolve(out->S, out->b, p->rank_tol, out->f, out->lam, &out->rank, &out->flags);
    return 0;
}
