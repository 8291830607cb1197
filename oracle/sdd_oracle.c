/*
 * sdd_oracle.c -- plain FP64 CPU oracle for the Monte-Carlo Feynman-Kac
 * evaluation of the 2-D TE magnetotelluric equation at interface nodes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link,
 * load or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * constant with the GPU library: it is written from the paper, one rule per
 * function, in the paper's order, for a reader to check by eye.
 *
 * Paper: Bihlo, Farquharson, Haynes, Loredo-Osti, "Stochastic domain
 * decomposition for the solution of the two-dimensional magnetotelluric
 * problem" (arXiv:1603.09311).
 *
 * What it computes (Sec. 2.2, Eqs. 5a/5b and 7-8; Sec. 3.1):
 *   TE mode, Eq. (1):  div((i w mu)^-1 grad E) - sigma E = 0, i.e. in model
 *   length units L,  Laplace(E) = i alpha E  with  alpha = w mu0 sigma L^2.
 *   With standard Brownian motion X (generator Laplace/2) the Feynman-Kac
 *   formula (Eq. 5a) gives
 *       E(x) = Exp[ g(X_tau) exp(-i S) ],   S = (1/2) int_0^tau alpha(X_s) ds,
 *   a pure phase: lambda = i alpha / 2 is the killing rate of Eq. (7) with
 *   kappa = 1.  The walk is the modified Euler-Maruyama scheme of Sec. 3.1
 *   (Eq. 13) with the Brownian-bridge first-hitting test (Eq. 14) applied to
 *   the rectangular outer boundary (end of Sec. 3.1), and the occupation times
 *   of the MC estimator (the sum over regions at the end of Sec. 3.1) folded
 *   into the phase S.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - mu0 = 4 pi 1e-7 H/m (the paper's value lacks the pi);
 *   - equal-kappa interfaces (TE): the step's phase goes to the region of the
 *     proposed point (Sec. 3.1, last rule for kappa_i = kappa_j);
 *   - a bridge exit ends at the nearer wall, tangential coordinate
 *     interpolated at f = t/dt; on an exit step the partial phase uses the
 *     region of the last inside point;
 *   - uniforms (w + 1/2) 2^-32; Box-Muller normals; Philox4x32-10 streams
 *     keyed by (seed) with counter (step pair, path, node, 2 stream + domain).
 *
 * Build: gcc -O2 -ffp-contract=off -std=c11 -fPIC -shared -lm -lpthread
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Problem and result records (this file's own definitions).                 */
/* ------------------------------------------------------------------------ */

enum { ORC_HALF_Z_LT = 0, ORC_HALF_Y_LT = 1, ORC_BOX = 2, ORC_TRIANGLE = 3 };

enum {
    ORC_OK = 0,
    ORC_E_INVALID = -1,
    ORC_E_NOMEM = -2
};

typedef struct {
    /* Omega = [y_lo, y_hi] x [z_lo, z_hi]; y to the right, z downward. */
    double y_lo, y_hi, z_lo, z_hi;
    /* Conductivity model (Sec. 2.2: piecewise-constant sub-domains):
       ordered primitives, the first one containing the point wins, else the
       background. */
    int32_t n_regions;
    const int32_t *region_kind;   /* n_regions */
    const double *region_param;   /* n_regions x 6 */
    const double *region_sigma;   /* n_regions, S/m (or relative) */
    double sigma_background;
    double length_unit_m;         /* metres per model length unit */
    double freq_hz;               /* > 0: alpha = (2 pi f) mu0 sigma L^2 */
    double alpha_direct;          /* freq_hz == 0: alpha = alpha_direct sigma */
    /* Dirichlet data g on the four walls, order top, right, bottom, left;
       each wall g_samples = M+1 equispaced complex samples (re, im). */
    int32_t g_samples;
    const double *g;
    /* Interface nodes and, per node, the range of path indices to walk. */
    int32_t n_nodes;
    const double *nodes;          /* n_nodes x (y, z) */
    const uint32_t *path_begin;   /* n_nodes */
    const uint32_t *path_count;   /* n_nodes */
    double dt;                    /* Euler-Maruyama time step */
    uint64_t seed;                /* Philox key */
    uint32_t stream;              /* Philox counter word 3 = 2 stream + domain */
    uint32_t max_steps;           /* proposals per path before giving up */
    int32_t naive_exit;           /* 1: exit on a crossing only (no bridge test) */
} orc_problem;

typedef struct {
    double w_re, w_im;   /* g(X_tau) exp(-i S) */
    double S;            /* phase integral (1/2) int alpha ds */
    double tau;          /* exit-time estimate (n + f) dt */
    double exit_t;       /* tangential coordinate of the exit point */
    uint32_t steps;      /* proposals drawn */
    int32_t wall;        /* 0 top, 1 right, 2 bottom, 3 left; -1 unfinished */
} orc_path;

typedef struct {
    double mean_re, mean_im;
    double var_re, var_im, cov;
    double se_re, se_im, se;
    double mean_exit_time;
    uint64_t paths_done, steps, unfinished;
} orc_node;

/* ------------------------------------------------------------------------ */
/* Random numbers.                                                           */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
   Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
   two 32x32->64 multiplications with a Weyl-sequence key schedule. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A 32-bit word as a uniform in the open interval (0, 1): (w + 1/2) 2^-32,
   exact in FP64, so log(u) is always finite. */
double orc_u01(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/* Box-Muller: two uniforms to two independent standard normals, the
   W ~ N(0, I_2) of the Euler-Maruyama step (Sec. 3.1, Eq. 13). */
void orc_box_muller(double ua, double ub, double out[2])
{
    const double two_pi = 6.283185307179586476925286766559;
    double r = sqrt(-2.0 * log(ua));
    double theta = two_pi * ub;
    out[0] = r * cos(theta);
    out[1] = r * sin(theta);
}

static void key_of(const orc_problem *P, uint32_t key[2])
{
    key[0] = (uint32_t)(P->seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(P->seed >> 32);
}

/* The normal pair of step n of path p at node j.  One Philox call serves two
   steps: words 0,1 for even n and 2,3 for odd n, counter (n/2, p, j, 2s). */
static void step_normals(const orc_problem *P, int j, uint32_t p, uint32_t n,
                         double out[2])
{
    uint32_t key[2], ctr[4], w[4];
    key_of(P, key);
    ctr[0] = n >> 1;
    ctr[1] = p;
    ctr[2] = (uint32_t)j;
    ctr[3] = 2u * P->stream + 0u;
    orc_philox4x32_10(ctr, key, w);
    if ((n & 1u) == 0u)
        orc_box_muller(orc_u01(w[0]), orc_u01(w[1]), out);
    else
        orc_box_muller(orc_u01(w[2]), orc_u01(w[3]), out);
}

/* The bridge uniform U of Eq. (14) for axis a (0 = y, 1 = z) at step n:
   word a of the Philox call with counter (n, p, j, 2s + 1). */
static double bridge_uniform(const orc_problem *P, int j, uint32_t p,
                             uint32_t n, int axis)
{
    uint32_t key[2], ctr[4], w[4];
    key_of(P, key);
    ctr[0] = n;
    ctr[1] = p;
    ctr[2] = (uint32_t)j;
    ctr[3] = 2u * P->stream + 1u;
    orc_philox4x32_10(ctr, key, w);
    return orc_u01(w[axis]);
}

/* ------------------------------------------------------------------------ */
/* Model: conductivity regions and the per-step phase increments.            */
/* ------------------------------------------------------------------------ */

static int in_primitive(int kind, const double *v, double y, double z)
{
    switch (kind) {
    case ORC_HALF_Z_LT:          /* z < v0 (air above the surface) */
        return z < v[0];
    case ORC_HALF_Y_LT:          /* y < v0 */
        return y < v[0];
    case ORC_BOX:                /* v0 <= y < v1 and v2 <= z < v3 */
        return (y >= v[0]) && (y < v[1]) && (z >= v[2]) && (z < v[3]);
    case ORC_TRIANGLE: {         /* vertices a=(v0,v1) b=(v2,v3) c=(v4,v5) */
        double e0 = (v[2] - v[0]) * (z - v[1]) - (v[3] - v[1]) * (y - v[0]);
        double e1 = (v[4] - v[2]) * (z - v[3]) - (v[5] - v[3]) * (y - v[2]);
        double e2 = (v[0] - v[4]) * (z - v[5]) - (v[1] - v[5]) * (y - v[4]);
        int all_nonneg = (e0 >= 0.0) && (e1 >= 0.0) && (e2 >= 0.0);
        int all_nonpos = (e0 <= 0.0) && (e1 <= 0.0) && (e2 <= 0.0);
        return all_nonneg || all_nonpos;
    }
    default:
        return 0;
    }
}

/* Index of the sub-domain containing (y, z): the first primitive in list
   order, else n_regions for the background. */
int orc_region(const orc_problem *P, double y, double z)
{
    for (int r = 0; r < P->n_regions; ++r)
        if (in_primitive(P->region_kind[r], P->region_param + 6 * r, y, z))
            return r;
    return P->n_regions;
}

/* alpha = w mu0 sigma L^2 (TE mode of Eq. 1 in model length units). */
static double alpha_of_sigma(const orc_problem *P, double sigma)
{
    const double pi = 3.14159265358979323846264338327950288;
    if (P->freq_hz > 0.0) {
        double omega = 2.0 * pi * P->freq_hz;
        double mu0 = 4.0e-7 * pi;
        double L = P->length_unit_m;
        return omega * mu0 * sigma * (L * L);
    }
    return P->alpha_direct * sigma;
}

/* Phase increment of one full step spent in region r: c_r = alpha_r dt / 2,
   i.e. lambda_r T with lambda = i alpha/2 and T = dt (Sec. 3.1, estimator). */
static void phase_increments(const orc_problem *P, double *c)
{
    for (int r = 0; r < P->n_regions; ++r)
        c[r] = alpha_of_sigma(P, P->region_sigma[r]) * P->dt / 2.0;
    c[P->n_regions] = alpha_of_sigma(P, P->sigma_background) * P->dt / 2.0;
}

/* ------------------------------------------------------------------------ */
/* Boundary data.                                                            */
/* ------------------------------------------------------------------------ */

/* g on wall `wall` at tangential coordinate t, by linear interpolation in the
   equispaced table (top/bottom run along y, left/right along z). */
void orc_table_g(const orc_problem *P, int wall, double t, double out[2])
{
    int M = P->g_samples - 1;
    double t0, t1;
    if (wall == 0 || wall == 2) { t0 = P->y_lo; t1 = P->y_hi; }
    else                        { t0 = P->z_lo; t1 = P->z_hi; }
    double h = (t1 - t0) / (double)M;
    double u = (t - t0) / h;
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i > M - 1) i = M - 1;
    double lam = u - (double)i;
    const double *gw = P->g + (size_t)wall * (size_t)P->g_samples * 2;
    out[0] = (1.0 - lam) * gw[2 * i] + lam * gw[2 * i + 2];
    out[1] = (1.0 - lam) * gw[2 * i + 1] + lam * gw[2 * i + 3];
}

/* ------------------------------------------------------------------------ */
/* One realisation of the discretised process (Sec. 3.1).                   */
/* ------------------------------------------------------------------------ */

int orc_walk_path(const orc_problem *P, int j, uint32_t p, orc_path *out)
{
    double c[64];
    if (P->n_regions > 63) return ORC_E_INVALID;
    phase_increments(P, c);

    const double s = sqrt(P->dt);
    double y = P->nodes[2 * j], z = P->nodes[2 * j + 1];
    double S = 0.0;
    const double lo[2] = {P->y_lo, P->z_lo};
    const double hi[2] = {P->y_hi, P->z_hi};

    for (uint32_t n = 0; n < P->max_steps; ++n) {
        /* Provisional position, Eq. (13) with kappa = 1. */
        double N[2];
        step_normals(P, j, p, n, N);
        double yn = y + s * N[0];
        double zn = z + s * N[1];

        /* The outer boundary is checked first (Sec. 3.1).  Per axis, the
           nearer wall; crossed -> linear fraction (Eq. 14, second case);
           same side -> Brownian-bridge test, hit iff t_gamma <= dt with
           t_gamma = -2 d0 d1 / log U (Eq. 14, first case, kappa = 1). */
        const double x[2] = {y, z};
        const double xn[2] = {yn, zn};
        int hit[2] = {0, 0}, upper[2] = {0, 0};
        double f[2] = {0.0, 0.0};
        for (int a = 0; a < 2; ++a) {
            double dlo = x[a] - lo[a];
            double dhi = hi[a] - x[a];
            upper[a] = !(dlo <= dhi);          /* a tie goes to the lower wall */
            double d0 = upper[a] ? dhi : dlo;
            double d1 = upper[a] ? (hi[a] - xn[a]) : (xn[a] - lo[a]);
            if (d1 <= 0.0) {
                hit[a] = 1;
                f[a] = d0 / (d0 - d1);
            } else if (!P->naive_exit) {
                double q = (2.0 * d0) * d1;
                double L = -log(bridge_uniform(P, j, p, n, a));
                if (q <= P->dt * L) {
                    hit[a] = 1;
                    f[a] = q / (P->dt * L);
                }
            }
        }
        if (hit[0] || hit[1]) {
            /* The earlier of the two hits ends the path; a tie goes to y. */
            int a = (hit[0] && (!hit[1] || f[0] <= f[1])) ? 0 : 1;
            double fr = f[a];
            double t;
            int wall;
            if (a == 0) {
                wall = upper[0] ? 1 : 3;
                t = z + fr * (zn - z);
                if (t < P->z_lo) t = P->z_lo;
                if (t > P->z_hi) t = P->z_hi;
            } else {
                wall = upper[1] ? 2 : 0;
                t = y + fr * (yn - y);
                if (t < P->y_lo) t = P->y_lo;
                if (t > P->y_hi) t = P->y_hi;
            }
            /* Partial step: the fraction fr of dt spent where the walk was. */
            S += c[orc_region(P, y, z)] * fr;
            double g[2];
            orc_table_g(P, wall, t, g);
            double cs = cos(S), sn = sin(S);
            out->w_re = g[0] * cs + g[1] * sn;    /* g exp(-i S) */
            out->w_im = g[1] * cs - g[0] * sn;
            out->S = S;
            out->tau = ((double)n + fr) * P->dt;
            out->exit_t = t;
            out->steps = n + 1;
            out->wall = wall;
            return ORC_OK;
        }
        /* No exit: keep the proposal; the step's occupation time goes to the
           region where the proposed point lies (equal-kappa interface rule). */
        S += c[orc_region(P, yn, zn)];
        y = yn;
        z = zn;
    }
    out->w_re = 0.0;
    out->w_im = 0.0;
    out->S = S;
    out->tau = -1.0;
    out->exit_t = 0.0;
    out->steps = P->max_steps;
    out->wall = -1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-node estimator (Sec. 3.1: u = (1/N) sum_r g(beta_r) exp(-sum lambda T)) */
/* ------------------------------------------------------------------------ */

int orc_node_stats(const orc_path *paths, uint64_t n, orc_node *out)
{
    uint64_t done = 0, steps = 0, unfinished = 0;
    double sre = 0.0, sim = 0.0, stau = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        steps += paths[i].steps;
        if (paths[i].wall < 0) { ++unfinished; continue; }
        ++done;
        sre += paths[i].w_re;
        sim += paths[i].w_im;
        stau += paths[i].tau;
    }
    out->paths_done = done;
    out->steps = steps;
    out->unfinished = unfinished;
    double N = (double)done;
    out->mean_re = sre / N;
    out->mean_im = sim / N;
    out->mean_exit_time = stau / N;
    double qrr = 0.0, qii = 0.0, qri = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        if (paths[i].wall < 0) continue;
        double dr = paths[i].w_re - out->mean_re;
        double di = paths[i].w_im - out->mean_im;
        qrr += dr * dr;
        qii += di * di;
        qri += dr * di;
    }
    out->var_re = qrr / (N - 1.0);
    out->var_im = qii / (N - 1.0);
    out->cov = qri / (N - 1.0);
    out->se_re = sqrt(out->var_re / N);
    out->se_im = sqrt(out->var_im / N);
    out->se = sqrt((out->var_re + out->var_im) / N);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Validation.                                                               */
/* ------------------------------------------------------------------------ */

int orc_validate(const orc_problem *P)
{
    if (!(P->y_lo < P->y_hi) || !(P->z_lo < P->z_hi)) return ORC_E_INVALID;
    if (!(P->dt > 0.0) || !isfinite(P->dt)) return ORC_E_INVALID;
    /* A step never exceeds 6.8 sqrt(dt) per axis (|N| <= sqrt(-2 log 2^-33));
       keeping it under half the shorter side means only the nearer wall can
       be crossed in one step. */
    double half = 0.5 * fmin(P->y_hi - P->y_lo, P->z_hi - P->z_lo);
    if (!(7.0 * sqrt(P->dt) < half)) return ORC_E_INVALID;
    if (P->g_samples < 2 || P->g == NULL) return ORC_E_INVALID;
    if (P->n_regions < 0 || P->n_regions > 63) return ORC_E_INVALID;
    if (P->n_nodes < 0) return ORC_E_INVALID;
    if (P->stream >= 0x80000000u) return ORC_E_INVALID;
    if (P->max_steps == 0) return ORC_E_INVALID;
    if (!(P->sigma_background >= 0.0) || !isfinite(P->sigma_background))
        return ORC_E_INVALID;
    for (int r = 0; r < P->n_regions; ++r) {
        if (!(P->region_sigma[r] >= 0.0) || !isfinite(P->region_sigma[r]))
            return ORC_E_INVALID;
        if (P->region_kind[r] < 0 || P->region_kind[r] > 3) return ORC_E_INVALID;
    }
    if (P->freq_hz > 0.0 && !(P->length_unit_m > 0.0)) return ORC_E_INVALID;
    for (int j = 0; j < P->n_nodes; ++j) {
        double y = P->nodes[2 * j], z = P->nodes[2 * j + 1];
        if (!(y > P->y_lo && y < P->y_hi && z > P->z_lo && z < P->z_hi))
            return ORC_E_INVALID;
        if (P->path_count[j] < 1) return ORC_E_INVALID;
        if ((uint64_t)P->path_begin[j] + P->path_count[j] > 0x100000000ull)
            return ORC_E_INVALID;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole problem: walk every (node, path), then reduce per node in path order. */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_problem *P;
    orc_path *recs;
    const uint64_t *rec_off;      /* n_nodes + 1 */
    uint64_t n_items;             /* work items of BLOCK paths */
    const uint64_t *item_off;     /* n_nodes + 1: first item of node j */
    uint64_t next;                /* shared item counter */
} orc_work;

#define ORC_BLOCK 256u

static void *worker(void *arg)
{
    orc_work *W = (orc_work *)arg;
    const orc_problem *P = W->P;
    for (;;) {
        uint64_t item = __atomic_fetch_add(&W->next, 1, __ATOMIC_RELAXED);
        if (item >= W->n_items) break;
        int j = 0;
        while (W->item_off[j + 1] <= item) ++j;
        uint64_t k0 = (item - W->item_off[j]) * ORC_BLOCK;
        uint64_t k1 = k0 + ORC_BLOCK;
        if (k1 > P->path_count[j]) k1 = P->path_count[j];
        for (uint64_t k = k0; k < k1; ++k)
            orc_walk_path(P, j, P->path_begin[j] + (uint32_t)k,
                          W->recs + W->rec_off[j] + k);
    }
    return NULL;
}

int orc_solve(const orc_problem *P, int n_threads, orc_node *out_nodes,
              orc_path *out_paths)
{
    int rc = orc_validate(P);
    if (rc != ORC_OK) return rc;
    int n = P->n_nodes;
    uint64_t *rec_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    uint64_t *item_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!rec_off || !item_off) { free(rec_off); free(item_off); return ORC_E_NOMEM; }
    for (int j = 0; j < n; ++j) {
        rec_off[j + 1] = rec_off[j] + P->path_count[j];
        item_off[j + 1] = item_off[j] + (P->path_count[j] + ORC_BLOCK - 1) / ORC_BLOCK;
    }
    orc_path *recs = out_paths;
    if (recs == NULL && rec_off[n] > 0) {
        recs = (orc_path *)malloc((size_t)rec_off[n] * sizeof(orc_path));
        if (!recs) { free(rec_off); free(item_off); return ORC_E_NOMEM; }
    }
    orc_work W = {P, recs, rec_off, item_off[n], item_off, 0};
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 512) n_threads = 512;
    pthread_t tid[512];
    int started = 0;
    for (int t = 1; t < n_threads; ++t)
        if (pthread_create(&tid[started], NULL, worker, &W) == 0) ++started;
    worker(&W);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    for (int j = 0; j < n; ++j)
        orc_node_stats(recs + rec_off[j], P->path_count[j], out_nodes + j);
    if (recs != out_paths) free(recs);
    free(rec_off);
    free(item_off);
    return ORC_OK;
}

/* ======================================================================== */
/* Discontinuous kappa: the interface scheme of Secs. 2.2 and 3.1.          */
/* ======================================================================== */
/*
 * (1/2) div(kappa grad u) - lambda u = 0 (Eq. 9) with kappa and lambda
 * constant on each side of one vertical interface y = y_if (the case the
 * paper derives, Eqs. 10-12), u = g on the rectangle's boundary.  In each
 * side the process is sqrt(kappa_i) times Brownian motion (Eq. 10); a step
 * that reaches the interface (crossing, or a bridge hit, Eq. 14 with
 * kappa_i) resumes inside a disc of radius h on the side drawn with the
 * probabilities of Eq. 12, and the step's time is split between the two
 * occupation times as Sec. 3.1 describes.  The estimator is
 * g(beta(tau)) exp(-(lambda_0 T_0 + lambda_1 T_1)).
 *
 * Readings (also in the design notes): both discs have the radius
 * h = sqrt(kappa_i dt) of the step that reached the interface (kappa_i of the
 * side it started on), so that the probabilities of Eq. (12), which hold for
 * equal radii, are the consistent ones (with unequal radii they would make
 * every visit of the interface O(h) wrong and the walk's limit biased); for
 * the side change the second share is
 * (1/2)(dt - t_gamma)(2 - p_j), so that the two shares sum to the step (the
 * printed (1 + p_j) sums to dt only when p_j = 1/2); the interface point is
 * the step's point at t_gamma (linear in the step); a point on the interface
 * belongs to side 1; the disc of side i touches the interface from side i;
 * a disc point outside the rectangle ends the walk at the nearest boundary
 * point with f = 1; equal kappa: the proposal is kept and the step's time
 * goes to the side of the proposal.
 * The split of an interface step's time between the two sides (the
 * (1/2)(dt - t_gamma) p terms) changes only the constant of the scheme's
 * O(sqrt(dt)) bias (an interface is visited O(1/sqrt(dt)) times per path),
 * so no continuum closed form separates it; it is pinned against the exact
 * expectation of this discrete scheme at a finite dt on a strip, where the
 * walk is a one-dimensional Markov chain evaluated without sampling
 * (tests/kappa_chain.py).
 * Random numbers: counter (n/2, p, j, 4s) -> the normals of steps n, n+1
 * (words 0,1 / 2,3); (n, p, j, 4s+1) -> outer bridge uniforms (words 0, 1),
 * the interface bridge uniform (word 2), the side uniform (word 3);
 * (n, p, j, 4s+2) -> the disc point (radius word 0, angle word 1).
 */

typedef struct {
    double y_lo, y_hi, z_lo, z_hi;
    double y_if;                  /* interface y = y_if */
    double kappa[2];              /* side 0: y < y_if, side 1: y >= y_if */
    double lambda_re[2], lambda_im[2];
    int32_t g_samples;
    const double *g;              /* 4 walls x g_samples x (re, im) */
    int32_t n_nodes;
    const double *nodes;
    const uint32_t *path_begin;
    const uint32_t *path_count;
    double dt;
    uint64_t seed;
    uint32_t stream;
    uint32_t max_steps;
} orc_kproblem;

static void kwords(const orc_kproblem *P, uint32_t c0, uint32_t p, int j,
                   uint32_t domain, uint32_t w[4])
{
    uint32_t key[2] = {(uint32_t)(P->seed & 0xFFFFFFFFu), (uint32_t)(P->seed >> 32)};
    uint32_t ctr[4] = {c0, p, (uint32_t)j, 4u * P->stream + domain};
    orc_philox4x32_10(ctr, key, w);
}

static void ktable_g(const orc_kproblem *P, int wall, double t, double out[2])
{
    orc_problem Q;
    memset(&Q, 0, sizeof(Q));
    Q.y_lo = P->y_lo; Q.y_hi = P->y_hi; Q.z_lo = P->z_lo; Q.z_hi = P->z_hi;
    Q.g_samples = P->g_samples;
    Q.g = P->g;
    orc_table_g(&Q, wall, t, out);
}

static void kfinish(const orc_kproblem *P, const double T[2], int wall, double t,
                    double tau, uint32_t steps, orc_path *out)
{
    double g[2];
    ktable_g(P, wall, t, g);
    /* exp(-(lambda_0 T_0 + lambda_1 T_1)) */
    double er = -(P->lambda_re[0] * T[0] + P->lambda_re[1] * T[1]);
    double ei = -(P->lambda_im[0] * T[0] + P->lambda_im[1] * T[1]);
    double m = exp(er);
    double cr = m * cos(ei), ci = m * sin(ei);
    out->w_re = g[0] * cr - g[1] * ci;
    out->w_im = g[0] * ci + g[1] * cr;
    out->S = -ei;
    out->tau = tau;
    out->exit_t = t;
    out->steps = steps;
    out->wall = wall;
}

/* The wall point nearest to (y, z) (outside or on the rectangle). */
static void nearest_wall(const orc_kproblem *P, double y, double z, int *wall, double *t)
{
    double dl = y - P->y_lo, dr = P->y_hi - y, dt_ = z - P->z_lo, db = P->z_hi - z;
    double m = dl; *wall = 3;
    if (dr < m) { m = dr; *wall = 1; }
    if (dt_ < m) { m = dt_; *wall = 0; }
    if (db < m) { m = db; *wall = 2; }
    double yy = fmin(fmax(y, P->y_lo), P->y_hi), zz = fmin(fmax(z, P->z_lo), P->z_hi);
    *t = (*wall == 0 || *wall == 2) ? yy : zz;
}

int orc_kwalk_path(const orc_kproblem *P, int j, uint32_t p, orc_path *out)
{
    double y = P->nodes[2 * j], z = P->nodes[2 * j + 1];
    double T[2] = {0.0, 0.0};
    const double lo[2] = {P->y_lo, P->z_lo};
    const double hi[2] = {P->y_hi, P->z_hi};
    const double dt = P->dt;

    for (uint32_t n = 0; n < P->max_steps; ++n) {
        int si = (y < P->y_if) ? 0 : 1;           /* side of the current point */
        double ki = P->kappa[si];
        uint32_t w[4], u[4];
        kwords(P, n >> 1, p, j, 0u, w);
        double N[2];
        if ((n & 1u) == 0u) orc_box_muller(orc_u01(w[0]), orc_u01(w[1]), N);
        else                orc_box_muller(orc_u01(w[2]), orc_u01(w[3]), N);
        double s = sqrt(ki * dt);                 /* Eq. (13) with kappa_i */
        double yn = y + s * N[0], zn = z + s * N[1];
        kwords(P, n, p, j, 1u, u);

        /* outer boundary first: nearer wall per axis, crossing or bridge
           (Eq. 14 with kappa_i) */
        const double x[2] = {y, z}, xn[2] = {yn, zn};
        int hit[2] = {0, 0}, upper[2] = {0, 0};
        double f[2] = {0.0, 0.0};
        for (int a = 0; a < 2; ++a) {
            double dlo = x[a] - lo[a], dhi = hi[a] - x[a];
            upper[a] = !(dlo <= dhi);
            double d0 = upper[a] ? dhi : dlo;
            double d1 = upper[a] ? (hi[a] - xn[a]) : (xn[a] - lo[a]);
            if (d1 <= 0.0) {
                hit[a] = 1;
                f[a] = d0 / (d0 - d1);
            } else {
                double q = (2.0 * d0) * d1;
                double L = -log(orc_u01(u[a]));
                if (q <= ki * dt * L) { hit[a] = 1; f[a] = q / (ki * dt * L); }
            }
        }
        if (hit[0] || hit[1]) {
            int a = (hit[0] && (!hit[1] || f[0] <= f[1])) ? 0 : 1;
            double fr = f[a], t;
            int wall;
            if (a == 0) {
                wall = upper[0] ? 1 : 3;
                t = fmin(fmax(z + fr * (zn - z), P->z_lo), P->z_hi);
            } else {
                wall = upper[1] ? 2 : 0;
                t = fmin(fmax(y + fr * (yn - y), P->y_lo), P->y_hi);
            }
            T[si] += fr * dt;
            kfinish(P, T, wall, t, ((double)n + fr) * dt, n + 1, out);
            return ORC_OK;
        }

        /* the interface */
        int sn = (yn < P->y_if) ? 0 : 1;
        if (P->kappa[0] == P->kappa[1]) {
            T[sn] += dt;                          /* no regime change */
            y = yn; z = zn;
            continue;
        }
        double d0 = fabs(y - P->y_if);
        double tg;
        int reached;
        if (sn != si) {                           /* crossed: Eq. 14, 2nd case */
            tg = dt * fabs(d0 / (yn - y));
            reached = 1;
        } else {                                  /* same side: bridge test */
            double d1 = fabs(yn - P->y_if);
            tg = -2.0 * d0 * d1 / (ki * log(orc_u01(u[2])));
            reached = tg <= dt;
        }
        if (!reached) {
            T[si] += dt;
            y = yn; z = zn;
            continue;
        }
        int sj = 1 - si;
        double kj = P->kappa[sj];
        /* Eq. (12): the probabilities of Eq. (11) for equal radii; both discs
           get the radius of the step that reached the interface */
        double pi_ = ki / (ki + kj), pj = 1.0 - pi_;
        double h = sqrt(ki * dt);
        double zg = z + (tg / dt) * (zn - z);            /* interface point */
        double towards = (si == 0) ? 1.0 : -1.0;         /* c_ij(h) / h */
        double cy;
        if (orc_u01(u[3]) < pi_) {                       /* resume on side i */
            cy = P->y_if - towards * h;
            T[si] += dt - 0.5 * (dt - tg) * pi_;
            T[sj] += 0.5 * (dt - tg) * pi_;
        } else {                                         /* resume on side j */
            cy = P->y_if + towards * h;
            T[si] += tg + 0.5 * (dt - tg) * pj;
            T[sj] += 0.5 * (dt - tg) * (2.0 - pj);
        }
        uint32_t d[4];
        kwords(P, n, p, j, 2u, d);
        const double two_pi = 6.283185307179586476925286766559;
        double r = h * sqrt(orc_u01(d[0])), th = two_pi * orc_u01(d[1]);
        y = cy + r * cos(th);
        z = zg + r * sin(th);
        if (!(y > P->y_lo && y < P->y_hi && z > P->z_lo && z < P->z_hi)) {
            int wall;
            double t;
            nearest_wall(P, y, z, &wall, &t);
            kfinish(P, T, wall, t, ((double)n + 1.0) * dt, n + 1, out);
            return ORC_OK;
        }
    }
    out->w_re = 0.0;
    out->w_im = 0.0;
    out->S = 0.0;
    out->tau = -1.0;
    out->exit_t = 0.0;
    out->steps = P->max_steps;
    out->wall = -1;
    return ORC_OK;
}

int orc_kvalidate(const orc_kproblem *P)
{
    if (!(P->y_lo < P->y_if && P->y_if < P->y_hi) || !(P->z_lo < P->z_hi)) return ORC_E_INVALID;
    if (!(P->dt > 0.0) || !isfinite(P->dt)) return ORC_E_INVALID;
    for (int i = 0; i < 2; ++i) {
        if (!(P->kappa[i] > 0.0) || !isfinite(P->kappa[i])) return ORC_E_INVALID;
        if (!(P->lambda_re[i] >= 0.0) || !isfinite(P->lambda_re[i]) || !isfinite(P->lambda_im[i]))
            return ORC_E_INVALID;
    }
    double kmax = fmax(P->kappa[0], P->kappa[1]);
    double half = 0.5 * fmin(P->y_hi - P->y_lo, P->z_hi - P->z_lo);
    if (!(7.0 * sqrt(kmax * P->dt) < half)) return ORC_E_INVALID;
    if (P->g_samples < 2 || P->g == NULL || P->n_nodes < 0 || P->max_steps == 0) return ORC_E_INVALID;
    if (P->stream >= 0x40000000u) return ORC_E_INVALID;
    for (int j = 0; j < P->n_nodes; ++j) {
        double y = P->nodes[2 * j], z = P->nodes[2 * j + 1];
        if (!(y > P->y_lo && y < P->y_hi && z > P->z_lo && z < P->z_hi)) return ORC_E_INVALID;
        if (P->path_count[j] < 1) return ORC_E_INVALID;
        if ((uint64_t)P->path_begin[j] + P->path_count[j] > 0x100000000ull) return ORC_E_INVALID;
    }
    return ORC_OK;
}

typedef struct {
    const orc_kproblem *P;
    orc_path *recs;
    const uint64_t *rec_off;
    uint64_t n_items;
    const uint64_t *item_off;
    uint64_t next;
} orc_kwork;

static void *kworker(void *arg)
{
    orc_kwork *W = (orc_kwork *)arg;
    const orc_kproblem *P = W->P;
    for (;;) {
        uint64_t item = __atomic_fetch_add(&W->next, 1, __ATOMIC_RELAXED);
        if (item >= W->n_items) break;
        int j = 0;
        while (W->item_off[j + 1] <= item) ++j;
        uint64_t k0 = (item - W->item_off[j]) * ORC_BLOCK;
        uint64_t k1 = k0 + ORC_BLOCK;
        if (k1 > P->path_count[j]) k1 = P->path_count[j];
        for (uint64_t k = k0; k < k1; ++k)
            orc_kwalk_path(P, j, P->path_begin[j] + (uint32_t)k, W->recs + W->rec_off[j] + k);
    }
    return NULL;
}

int orc_ksolve(const orc_kproblem *P, int n_threads, orc_node *out_nodes, orc_path *out_paths)
{
    int rc = orc_kvalidate(P);
    if (rc != ORC_OK) return rc;
    int n = P->n_nodes;
    uint64_t *rec_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    uint64_t *item_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!rec_off || !item_off) { free(rec_off); free(item_off); return ORC_E_NOMEM; }
    for (int j = 0; j < n; ++j) {
        rec_off[j + 1] = rec_off[j] + P->path_count[j];
        item_off[j + 1] = item_off[j] + (P->path_count[j] + ORC_BLOCK - 1) / ORC_BLOCK;
    }
    orc_path *recs = out_paths;
    if (recs == NULL && rec_off[n] > 0) {
        recs = (orc_path *)malloc((size_t)rec_off[n] * sizeof(orc_path));
        if (!recs) { free(rec_off); free(item_off); return ORC_E_NOMEM; }
    }
    orc_kwork W = {P, recs, rec_off, item_off[n], item_off, 0};
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 512) n_threads = 512;
    pthread_t tid[512];
    int started = 0;
    for (int t = 1; t < n_threads; ++t)
        if (pthread_create(&tid[started], NULL, kworker, &W) == 0) ++started;
    kworker(&W);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    for (int j = 0; j < n; ++j)
        orc_node_stats(recs + rec_off[j], P->path_count[j], out_nodes + j);
    if (recs != out_paths) free(recs);
    free(rec_off);
    free(item_off);
    return ORC_OK;
}
