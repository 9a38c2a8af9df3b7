/*
 * FP64 CPU oracle for the multilevel summation method (MSM).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the package smoke check
 * and the CPU-baseline leg of the benchmark, never by the product path. It
 * shares no code with the HIP library. Each function follows one passage of
 * the paper (Pazurikova & Matyska, "Parallel-in-time method for calculation of
 * long-range electrostatic interactions", Section 3) and is written for
 * reading, not speed: sums are direct, and OpenMP only splits loops whose
 * iterations write disjoint outputs.
 *
 * Readings of the paper that this file depends on (the paper is silent):
 *  - Phi is the C1 cubic numerical Hermite interpolant of the cardinal data
 *    (1 at node 0, 0 elsewhere) with central-difference slopes.
 *  - Grid origin of every level is the domain's lower corner; level k nodes
 *    sit at lo + 2^k h i. The level-0 index range is [-1, floor(L/h) + 2]
 *    (every node within reach of an atom in [lo, hi]) and
 *    level k+1 covers [ceil((i0-3)/2), floor((i1+3)/2)] of level k's [i0, i1],
 *    which keeps every non-zero term of the nested sums.
 *  - The number of grids l is the smallest with ceil(L_d / (2^(l-1) h)) <= 4
 *    on every axis, unless given.
 *  - Energy U = 1/2 sum_i q_i phi_i with phi_i = ke (u_short + u_long -
 *    q_i gamma(0)/a); the subtracted term removes the smooth self-interaction
 *    that the grids include.
 */
#include "msm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Threads the OpenMP loops of this library use. */
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ---- Section 3, smoothing function gamma of degree 2m: for rho < 1 the
 *      Taylor polynomial of (rho^2)^(-1/2) about rho^2 = 1 up to the
 *      (rho^2 - 1)^m term, which joins 1/rho with m continuous derivatives;
 *      1/rho beyond. m = 2 is the even quartic the paper selects. ---- */
static double binom_mhalf(int k)   /* binomial coefficient (-1/2 choose k) */
{
    double c = 1.0;
    for (int i = 0; i < k; i++) c *= (-0.5 - i) / (i + 1);
    return c;
}

double orc_gamma_m(double rho, int m)
{
    if (rho >= 1.0) return 1.0 / rho;
    double s = rho * rho - 1.0, term = 1.0, acc = 0.0;
    for (int k = 0; k <= m; k++) {
        acc += binom_mhalf(k) * term;
        term *= s;
    }
    return acc;
}

double orc_dgamma_m(double rho, int m)
{
    if (rho >= 1.0) return -1.0 / (rho * rho);
    /* d/drho (rho^2 - 1)^k = 2 k rho (rho^2 - 1)^(k-1) */
    double s = rho * rho - 1.0, term = 1.0, acc = 0.0;
    for (int k = 1; k <= m; k++) {
        acc += binom_mhalf(k) * k * term;
        term *= s;
    }
    return 2.0 * rho * acc;
}

double orc_gamma(double rho) { return orc_gamma_m(rho, 2); }
double orc_dgamma(double rho) { return orc_dgamma_m(rho, 2); }

static int smooth_of(const orc_params *p) { return p->smoothing > 0 ? p->smoothing : 2; }

/* ---- Section 3, nodal basis Phi of degree p: the Hermite interpolant of the
 *      cardinal data c(n) = [n == 0] whose node derivatives are central
 *      differences of the data. p = 3 (the paper's cubic numerical Hermite
 *      interpolant): slopes (c(n+1) - c(n-1)) / 2, support |t| < 2.
 *      p = 5 (a reading of "degree p" for the quintic): first and second
 *      derivatives from the five-point central differences, support |t| < 3;
 *      C2, and it reproduces polynomials up to degree 4. ---- */
static double card(long n) { return n == 0 ? 1.0 : 0.0; }
static double card_slope(long n) { return 0.5 * (card(n + 1) - card(n - 1)); }
static double card_d1_5(long n) { return (card(n - 2) - 8 * card(n - 1) + 8 * card(n + 1) - card(n + 2)) / 12.0; }
static double card_d2_5(long n)
{
    return (-card(n - 2) + 16 * card(n - 1) - 30 * card(n) + 16 * card(n + 1) - card(n + 2)) / 12.0;
}

static double phi3(double t, int deriv)
{
    double f = floor(t);
    long n = (long)f;
    double s = t - f;
    if (!deriv) {
        double h00 = 2 * s * s * s - 3 * s * s + 1;
        double h10 = s * s * s - 2 * s * s + s;
        double h01 = -2 * s * s * s + 3 * s * s;
        double h11 = s * s * s - s * s;
        return card(n) * h00 + card_slope(n) * h10 + card(n + 1) * h01 + card_slope(n + 1) * h11;
    }
    double d00 = 6 * s * s - 6 * s;
    double d10 = 3 * s * s - 4 * s + 1;
    double d01 = -6 * s * s + 6 * s;
    double d11 = 3 * s * s - 2 * s;
    return card(n) * d00 + card_slope(n) * d10 + card(n + 1) * d01 + card_slope(n + 1) * d11;
}

/* quintic Hermite basis on [0, 1]: value, first and second derivative at 0
 * (e0, e1, e2) and at 1 (f0, f1, f2), or their derivatives in s */
static double phi5(double t, int deriv)
{
    double f = floor(t);
    long n = (long)f;
    double s = t - f, s2 = s * s, s3 = s2 * s, s4 = s3 * s, s5 = s4 * s;
    double e0, e1, e2, f0, f1, f2;
    if (!deriv) {
        e0 = 1 - 10 * s3 + 15 * s4 - 6 * s5;
        e1 = s - 6 * s3 + 8 * s4 - 3 * s5;
        e2 = 0.5 * s2 - 1.5 * s3 + 1.5 * s4 - 0.5 * s5;
        f0 = 10 * s3 - 15 * s4 + 6 * s5;
        f1 = -4 * s3 + 7 * s4 - 3 * s5;
        f2 = 0.5 * s3 - s4 + 0.5 * s5;
    } else {
        e0 = -30 * s2 + 60 * s3 - 30 * s4;
        e1 = 1 - 18 * s2 + 32 * s3 - 15 * s4;
        e2 = s - 4.5 * s2 + 6 * s3 - 2.5 * s4;
        f0 = 30 * s2 - 60 * s3 + 30 * s4;
        f1 = -12 * s2 + 28 * s3 - 15 * s4;
        f2 = 1.5 * s2 - 4 * s3 + 2.5 * s4;
    }
    return card(n) * e0 + card_d1_5(n) * e1 + card_d2_5(n) * e2 + card(n + 1) * f0 + card_d1_5(n + 1) * f1 +
           card_d2_5(n + 1) * f2;
}

double orc_Phi_p(double t, int p) { return p == 5 ? phi5(t, 0) : phi3(t, 0); }
double orc_dPhi_p(double t, int p) { return p == 5 ? phi5(t, 1) : phi3(t, 1); }
double orc_Phi(double t) { return phi3(t, 0); }
double orc_dPhi(double t) { return phi3(t, 1); }

static int basis_of(const orc_params *p) { return p->basis == 5 ? 5 : 3; }
/* half-width S of the support of Phi: |t| < S, S = (p + 1) / 2 */
static int support_of(const orc_params *p) { return (basis_of(p) + 1) / 2; }

/* ---- Section 3, kernel splitting 1/r = g* + g^0 + ... + g^{l-1}. ---- */
double orc_gstar_m(double r, double a, int m) { return 1.0 / r - orc_gamma_m(r / a, m) / a; }

double orc_dgstar_m(double r, double a, int m) { return -1.0 / (r * r) - orc_dgamma_m(r / a, m) / (a * a); }

double orc_glevel_m(double r, double a, int k, int l, int m)
{
    double ak = ldexp(a, k);
    if (k == l - 1) return orc_gamma_m(r / ak, m) / ak;
    double ak1 = ldexp(a, k + 1);
    return orc_gamma_m(r / ak, m) / ak - orc_gamma_m(r / ak1, m) / ak1;
}

double orc_gstar(double r, double a) { return orc_gstar_m(r, a, 2); }
double orc_dgstar(double r, double a) { return orc_dgstar_m(r, a, 2); }
double orc_glevel(double r, double a, int k, int l) { return orc_glevel_m(r, a, k, l, 2); }

/* ---- grids ---- */
int orc_levels(const orc_params *p)
{
    if (p->levels > 0) return p->levels;
    for (int l = 1; l <= ORC_MAXLEV; l++) {
        int ok = 1;
        for (int d = 0; d < 3; d++) {
            double len = p->hi[d] - p->lo[d];
            if (ceil(len / (ldexp(p->h, l - 1))) > 4.0) ok = 0;
        }
        if (ok) return l;
    }
    return ORC_MAXLEV;
}

static long floordiv2(long v) { return (v >= 0) ? v / 2 : -((-v + 1) / 2); }
static long ceildiv2(long v) { return -floordiv2(-v); }

int orc_grid_shape(const orc_params *p, int level, int org[3], int dim[3])
{
    int l = orc_levels(p);
    if (level < 0 || level >= l) return -1;
    /* level 0: every node an atom in [lo, hi] reaches, base - (S-1) .. base + S;
     * level k+1: every node whose restriction window 2 mu -+ (2S-1) meets level k */
    const long S = support_of(p), W = 2 * S - 1;
    for (int d = 0; d < 3; d++) {
        long i0 = -(S - 1);
        long i1 = (long)floor((p->hi[d] - p->lo[d]) / p->h) + S;
        for (int k = 0; k < level; k++) {
            i0 = ceildiv2(i0 - W);
            i1 = floordiv2(i1 + W);
        }
        org[d] = (int)i0;
        dim[d] = (int)(i1 - i0 + 1);
    }
    return 0;
}

typedef struct {
    int l;
    int p, S;   /* basis degree and support half-width */
    int org[ORC_MAXLEV][3];
    int dim[ORC_MAXLEV][3];
    int64_t size[ORC_MAXLEV];
} plan_t;

static void make_plan(const orc_params *p, plan_t *pl)
{
    pl->l = orc_levels(p);
    pl->p = basis_of(p);
    pl->S = support_of(p);
    for (int k = 0; k < pl->l; k++) {
        orc_grid_shape(p, k, pl->org[k], pl->dim[k]);
        pl->size[k] = (int64_t)pl->dim[k][0] * pl->dim[k][1] * pl->dim[k][2];
    }
}

static int64_t gidx(const plan_t *pl, int k, long ix, long iy, long iz)
{
    long x = ix - pl->org[k][0], y = iy - pl->org[k][1], z = iz - pl->org[k][2];
    if (x < 0 || y < 0 || z < 0 || x >= pl->dim[k][0] || y >= pl->dim[k][1] || z >= pl->dim[k][2])
        return -1;
    return ((int64_t)z * pl->dim[k][1] + y) * pl->dim[k][0] + x;
}

/* Neumaier compensated sum. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}

static int check_inputs(const orc_params *p, int64_t n, const double *xyz, const double *q)
{
    if (!p || n < 0 || (n > 0 && (!xyz || !q))) return -1;
    if (!(p->a > 0) || !(p->h > 0)) return -1;
    for (int d = 0; d < 3; d++)
        if (!(p->hi[d] > p->lo[d])) return -1;
    for (int64_t i = 0; i < n; i++) {
        for (int d = 0; d < 3; d++) {
            double x = xyz[3 * i + d];
            if (!isfinite(x)) return -3;
            if (x < p->lo[d] || x > p->hi[d]) return -2;
        }
        if (!isfinite(q[i])) return -3;
    }
    return 0;
}

/* ---- Section 3: short-range part u_i^short = sum_{j != i, r_ij < a} g*(r_ij) q_j,
 *      and its gradient. A plain cell list (cells no smaller than a) only
 *      restricts the j loop to candidates; every pair is tested. ---- */
static void short_range(const orc_params *p, int64_t n, const double *xyz, const double *q,
                        double *u, double *f)
{
    int nc[3];
    double cs[3];
    for (int d = 0; d < 3; d++) {
        double len = p->hi[d] - p->lo[d];
        nc[d] = (int)floor(len / (p->a * 1.000001)); /* cells strictly wider than a */
        if (nc[d] < 1) nc[d] = 1;
        cs[d] = len / nc[d];
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = malloc(sizeof(int64_t) * ncell);
    int64_t *next = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int *cell = malloc(sizeof(int) * 3 * (n > 0 ? n : 1));
    for (int64_t c = 0; c < ncell; c++) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; i--) {
        int c3[3];
        for (int d = 0; d < 3; d++) {
            int c = (int)floor((xyz[3 * i + d] - p->lo[d]) / cs[d]);
            if (c >= nc[d]) c = nc[d] - 1;
            if (c < 0) c = 0;
            c3[d] = c;
            cell[3 * i + d] = c;
        }
        int64_t cid = ((int64_t)c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
        next[i] = head[cid];
        head[cid] = i;
    }
    double a = p->a;
    const int m = smooth_of(p);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double ui = 0, fx = 0, fy = 0, fz = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int cx = cell[3 * i] + dx, cy = cell[3 * i + 1] + dy, cz = cell[3 * i + 2] + dz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= nc[0] || cy >= nc[1] || cz >= nc[2]) continue;
                    for (int64_t j = head[((int64_t)cz * nc[1] + cy) * nc[0] + cx]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        double rx = xyz[3 * i] - xyz[3 * j];
                        double ry = xyz[3 * i + 1] - xyz[3 * j + 1];
                        double rz = xyz[3 * i + 2] - xyz[3 * j + 2];
                        double r = sqrt(rx * rx + ry * ry + rz * rz);
                        if (!(r < a)) continue;
                        ui += orc_gstar_m(r, a, m) * q[j];
                        double s = -orc_dgstar_m(r, a, m) / r * q[j];
                        fx += s * rx;
                        fy += s * ry;
                        fz += s * rz;
                    }
                }
        u[i] = ui;
        f[3 * i] = fx;
        f[3 * i + 1] = fy;
        f[3 * i + 2] = fz;
    }
    free(head);
    free(next);
    free(cell);
}

/* ---- Section 3, anterpolation: q^0_mu = sum_j phi^0_mu(r_j) q_j, written as a
 *      scatter from each atom to the (2S)^3 nodes around it. ---- */
static void anterpolate(const orc_params *p, const plan_t *pl, int64_t n, const double *xyz,
                        const double *q, double *q0)
{
    memset(q0, 0, sizeof(double) * pl->size[0]);
    for (int64_t j = 0; j < n; j++) {
        double t[3];
        long base[3];
        for (int d = 0; d < 3; d++) {
            t[d] = (xyz[3 * j + d] - p->lo[d]) / p->h;
            base[d] = (long)floor(t[d]);
        }
        const long S = pl->S;
        for (long mz = base[2] - (S - 1); mz <= base[2] + S; mz++)
            for (long my = base[1] - (S - 1); my <= base[1] + S; my++)
                for (long mx = base[0] - (S - 1); mx <= base[0] + S; mx++) {
                    double w = orc_Phi_p(t[0] - mx, pl->p) * orc_Phi_p(t[1] - my, pl->p) * orc_Phi_p(t[2] - mz, pl->p);
                    if (w == 0.0) continue;
                    int64_t g = gidx(pl, 0, mx, my, mz);
                    q0[g] += w * q[j];
                }
    }
}

/* ---- Section 3, restriction: q^{k+1}_mu = sum_nu phi^{k+1}_mu(r^k_nu) q^k_nu.
 *      A level-k node nu sits at half-integer coarse coordinates nu/2, so its
 *      weight is prod_d Phi((nu_d - 2 mu_d)/2); the sum runs directly over the
 *      3-D window where that product can be non-zero. ---- */
static void restrict_level(const plan_t *pl, int k, const double *qk, double *qk1)
{
    const int *oc = pl->org[k + 1], *dc = pl->dim[k + 1];
#pragma omp parallel for collapse(2)
    for (long cz = 0; cz < dc[2]; cz++)
        for (long cy = 0; cy < dc[1]; cy++)
            for (long cx = 0; cx < dc[0]; cx++) {
                long mx = cx + oc[0], my = cy + oc[1], mz = cz + oc[2];
                double acc = 0;
                const long W = 2 * pl->S - 1;
                for (long nz = 2 * mz - W; nz <= 2 * mz + W; nz++)
                    for (long ny = 2 * my - W; ny <= 2 * my + W; ny++)
                        for (long nx = 2 * mx - W; nx <= 2 * mx + W; nx++) {
                            int64_t g = gidx(pl, k, nx, ny, nz);
                            if (g < 0) continue;
                            double w = orc_Phi_p((nx - 2.0 * mx) / 2.0, pl->p) * orc_Phi_p((ny - 2.0 * my) / 2.0, pl->p) *
                                       orc_Phi_p((nz - 2.0 * mz) / 2.0, pl->p);
                            acc += w * qk[g];
                        }
                qk1[(cz * dc[1] + cy) * dc[0] + cx] = acc;
            }
}

/* ---- Section 3, lattice cutoff at level k < l-1 (g^k vanishes beyond 2^{k+1} a)
 *      and the top level k = l-1 (all node pairs):
 *      u_mu = sum_nu g^k(|r^k_mu - r^k_nu|) q^k_nu. ---- */
static void level_potential(const orc_params *p, const plan_t *pl, int k, const double *qk, double *uk)
{
    const int *o = pl->org[k], *dm = pl->dim[k];
    double hk = ldexp(p->h, k);
    int top = (k == pl->l - 1);
    long reach = top ? (long)(dm[0] > dm[1] ? (dm[0] > dm[2] ? dm[0] : dm[2]) : (dm[1] > dm[2] ? dm[1] : dm[2]))
                     : (long)ceil(2.0 * p->a / p->h);
    double rcut = ldexp(2.0 * p->a, k);
    /* g^k at every node offset the sum visits, evaluated once (the values and
     * the order of the terms are those of evaluating g^k per node pair); an
     * offset at or beyond 2^{k+1} a below the top level is not a term */
    const long side = 2 * reach + 1;
    double *gt = malloc(sizeof(double) * side * side * side);
    unsigned char *term = malloc((size_t)(side * side * side));
    for (long dz = -reach; dz <= reach; dz++)
        for (long dy = -reach; dy <= reach; dy++)
            for (long dx = -reach; dx <= reach; dx++) {
                const long t = ((dz + reach) * side + (dy + reach)) * side + (dx + reach);
                double rx = dx * hk, ry = dy * hk, rz = dz * hk;
                double r = sqrt(rx * rx + ry * ry + rz * rz);
                term[t] = top || r < rcut;
                gt[t] = term[t] ? orc_glevel_m(r, p->a, k, pl->l, smooth_of(p)) : 0.0;
            }
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (long z = 0; z < dm[2]; z++)
        for (long y = 0; y < dm[1]; y++)
            for (long x = 0; x < dm[0]; x++) {
                long mx = x + o[0], my = y + o[1], mz = z + o[2];
                ksum acc = {0, 0};
                for (long nz = mz - reach; nz <= mz + reach; nz++)
                    for (long ny = my - reach; ny <= my + reach; ny++)
                        for (long nx = mx - reach; nx <= mx + reach; nx++) {
                            int64_t g = gidx(pl, k, nx, ny, nz);
                            if (g < 0 || qk[g] == 0.0) continue;
                            const long t = ((nz - mz + reach) * side + (ny - my + reach)) * side + (nx - mx + reach);
                            if (!term[t]) continue;
                            kadd(&acc, gt[t] * qk[g]);
                        }
                uk[(z * dm[1] + y) * dm[0] + x] = acc.s + acc.c;
            }
    free(gt);
    free(term);
}

/* ---- Section 3, prolongation: u^k_mu = u^{k,cutoff}_mu + sum_nu phi^{k+1}_nu(r^k_mu) u^{k+1}_nu,
 *      with phi^{k+1}_nu(r^k_mu) = prod_d Phi((mu_d - 2 nu_d)/2). ---- */
static void prolong_level(const plan_t *pl, int k, const double *uk1, double *uk)
{
    const int *o = pl->org[k], *dm = pl->dim[k];
#pragma omp parallel for collapse(2)
    for (long z = 0; z < dm[2]; z++)
        for (long y = 0; y < dm[1]; y++)
            for (long x = 0; x < dm[0]; x++) {
                long mx = x + o[0], my = y + o[1], mz = z + o[2];
                double acc = 0;
                const long W = 2 * pl->S - 1;
                for (long nz = floordiv2(mz - W); nz <= floordiv2(mz + W) + 1; nz++)
                    for (long ny = floordiv2(my - W); ny <= floordiv2(my + W) + 1; ny++)
                        for (long nx = floordiv2(mx - W); nx <= floordiv2(mx + W) + 1; nx++) {
                            double w = orc_Phi_p((mx - 2.0 * nx) / 2.0, pl->p) * orc_Phi_p((my - 2.0 * ny) / 2.0, pl->p) *
                                       orc_Phi_p((mz - 2.0 * nz) / 2.0, pl->p);
                            if (w == 0.0) continue;
                            int64_t g = gidx(pl, k + 1, nx, ny, nz);
                            /* every node with a non-zero weight lies in the coarse range */
                            if (g < 0) continue;
                            acc += w * uk1[g];
                        }
                uk[(z * dm[1] + y) * dm[0] + x] += acc;
            }
}

/* ---- Section 3, interpolation u_i^long = sum_mu phi^0_mu(r_i) u^0_mu and its gradient. ---- */
static void interpolate(const orc_params *p, const plan_t *pl, int64_t n, const double *xyz,
                        const double *u0, double *ul, double *gl)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double t[3];
        long base[3];
        for (int d = 0; d < 3; d++) {
            t[d] = (xyz[3 * i + d] - p->lo[d]) / p->h;
            base[d] = (long)floor(t[d]);
        }
        double u = 0, gx = 0, gy = 0, gz = 0;
        const long S = pl->S;
        const int pd = pl->p;
        for (long mz = base[2] - (S - 1); mz <= base[2] + S; mz++)
            for (long my = base[1] - (S - 1); my <= base[1] + S; my++)
                for (long mx = base[0] - (S - 1); mx <= base[0] + S; mx++) {
                    int64_t g = gidx(pl, 0, mx, my, mz);
                    double px = orc_Phi_p(t[0] - mx, pd), py = orc_Phi_p(t[1] - my, pd), pz = orc_Phi_p(t[2] - mz, pd);
                    double dx = orc_dPhi_p(t[0] - mx, pd) / p->h, dy = orc_dPhi_p(t[1] - my, pd) / p->h,
                           dz = orc_dPhi_p(t[2] - mz, pd) / p->h;
                    double v = u0[g];
                    u += px * py * pz * v;
                    gx += dx * py * pz * v;
                    gy += px * dy * pz * v;
                    gz += px * py * dz * v;
                }
        ul[i] = u;
        gl[3 * i] = gx;
        gl[3 * i + 1] = gy;
        gl[3 * i + 2] = gz;
    }
}

int orc_msm(const orc_params *p, int64_t n, const double *xyz, const double *q,
            double *energy, double *forces, double *pot, orc_stages *st)
{
    int rc = check_inputs(p, n, xyz, q);
    if (rc) return rc;
    plan_t pl;
    make_plan(p, &pl);
    if (pl.l < 1 || pl.l > ORC_MAXLEV) return -1;
    int l = pl.l;
    size_t nn = (size_t)(n > 0 ? n : 1);

    double *us = malloc(sizeof(double) * nn), *fs = malloc(sizeof(double) * 3 * nn);
    double *ul = malloc(sizeof(double) * nn), *gl = malloc(sizeof(double) * 3 * nn);
    double *qg[ORC_MAXLEV], *ug[ORC_MAXLEV];
    for (int k = 0; k < l; k++) {
        qg[k] = malloc(sizeof(double) * pl.size[k]);
        ug[k] = malloc(sizeof(double) * pl.size[k]);
    }

    /* ORC_PROGRESS set: a line on stderr after each step of a long evaluation */
    const int progress = getenv("ORC_PROGRESS") != NULL;
    /* step 1: short-range part */
    short_range(p, n, xyz, q, us, fs);
    if (progress) fprintf(stderr, "oracle: short-range part of %lld atoms done\n", (long long)n);
    /* step 2: anterpolation */
    anterpolate(p, &pl, n, xyz, q, qg[0]);
    if (progress) fprintf(stderr, "oracle: anterpolation done\n");
    /* steps 3-4: restriction and lattice cutoff on levels 0 .. l-2 */
    for (int k = 0; k + 1 < l; k++) restrict_level(&pl, k, qg[k], qg[k + 1]);
    /* steps 3-5: lattice cutoff on every level, the top level over all pairs */
    for (int k = 0; k < l; k++) {
        level_potential(p, &pl, k, qg[k], ug[k]);
        if (progress) fprintf(stderr, "oracle: level %d of %d done\n", k, l);
    }
    if (st)
        for (int k = 0; k < l; k++) {
            if (st->q_grid[k]) memcpy(st->q_grid[k], qg[k], sizeof(double) * pl.size[k]);
            if (st->ucut_grid[k]) memcpy(st->ucut_grid[k], ug[k], sizeof(double) * pl.size[k]);
        }
    /* steps 6-7: prolongation, coarse to fine */
    for (int k = l - 2; k >= 0; k--) prolong_level(&pl, k, ug[k + 1], ug[k]);
    /* step 8: interpolation */
    interpolate(p, &pl, n, xyz, ug[0], ul, gl);

    /* step 9: combination into per-atom potentials, energy and forces */
    double self = orc_gamma_m(0.0, smooth_of(p)) / p->a;
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; i++) {
        double phi = p->ke * (us[i] + ul[i] - q[i] * self);
        if (pot) pot[i] = phi;
        kadd(&e, q[i] * phi);
        if (forces)
            for (int d = 0; d < 3; d++) forces[3 * i + d] = p->ke * q[i] * (fs[3 * i + d] - gl[3 * i + d]);
    }
    if (energy) *energy = 0.5 * (e.s + e.c);

    if (st) {
        if (st->u_short) memcpy(st->u_short, us, sizeof(double) * n);
        if (st->f_short) memcpy(st->f_short, fs, sizeof(double) * 3 * n);
        if (st->u_long) memcpy(st->u_long, ul, sizeof(double) * n);
        if (st->g_long) memcpy(st->g_long, gl, sizeof(double) * 3 * n);
        for (int k = 0; k < l; k++)
            if (st->u_grid[k]) memcpy(st->u_grid[k], ug[k], sizeof(double) * pl.size[k]);
    }
    free(us);
    free(fs);
    free(ul);
    free(gl);
    for (int k = 0; k < l; k++) {
        free(qg[k]);
        free(ug[k]);
    }
    return 0;
}

/* ---- Section 3, short-range part of selected atoms only, by a direct loop
 *      over every other atom (for spot checks of very large systems). ---- */
int orc_short_subset(const orc_params *p, int64_t n, const double *xyz, const double *q, int64_t nsel,
                     const int64_t *sel, double *u, double *f)
{
    if (!p || n < 0 || nsel < 0 || (nsel > 0 && (!sel || !u || !f))) return -1;
    double a = p->a;
    const int m = smooth_of(p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nsel; s++) {
        int64_t i = sel[s];
        double ui = 0, fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double rx = xyz[3 * i] - xyz[3 * j], ry = xyz[3 * i + 1] - xyz[3 * j + 1], rz = xyz[3 * i + 2] - xyz[3 * j + 2];
            double r2 = rx * rx + ry * ry + rz * rz;
            if (!(r2 < a * a)) continue;
            double r = sqrt(r2);
            ui += orc_gstar_m(r, a, m) * q[j];
            double sc = -orc_dgstar_m(r, a, m) / r * q[j];
            fx += sc * rx;
            fy += sc * ry;
            fz += sc * rz;
        }
        u[s] = ui;
        f[3 * s] = fx;
        f[3 * s + 1] = fy;
        f[3 * s + 2] = fz;
    }
    return 0;
}

/* ---- Section 2, Coulomb's law, summed directly over every pair i < j. ---- */
int orc_coulomb(int64_t n, const double *xyz, const double *q, double ke,
                double *energy, double *forces, double *pot)
{
    if (n < 0 || (n > 0 && (!xyz || !q))) return -1;
    double *phi = malloc(sizeof(double) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double u = 0, fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double rx = xyz[3 * i] - xyz[3 * j], ry = xyz[3 * i + 1] - xyz[3 * j + 1],
                   rz = xyz[3 * i + 2] - xyz[3 * j + 2];
            double r2 = rx * rx + ry * ry + rz * rz;
            double r = sqrt(r2);
            u += q[j] / r;
            double s = q[j] / (r2 * r);
            fx += s * rx;
            fy += s * ry;
            fz += s * rz;
        }
        phi[i] = ke * u;
        if (forces) {
            forces[3 * i] = ke * q[i] * fx;
            forces[3 * i + 1] = ke * q[i] * fy;
            forces[3 * i + 2] = ke * q[i] * fz;
        }
    }
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; i++) kadd(&e, q[i] * phi[i]);
    if (energy) *energy = 0.5 * (e.s + e.c);
    if (pot) memcpy(pot, phi, sizeof(double) * n);
    free(phi);
    return 0;
}

/* ---- Section 5: the simple cutoff method ---- */
int orc_cutoff(int64_t n, const double *xyz, const double *q, const int32_t *molid, double rc, double ke,
               double *energy, double *forces, double *pot)
{
    if (n < 0 || (n > 0 && (!xyz || !q)) || !(rc > 0)) return -1;
    double *phi = malloc(sizeof(double) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double u = 0, fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i || (molid && molid[j] == molid[i])) continue;
            double rx = xyz[3 * i] - xyz[3 * j], ry = xyz[3 * i + 1] - xyz[3 * j + 1],
                   rz = xyz[3 * i + 2] - xyz[3 * j + 2];
            double r = sqrt(rx * rx + ry * ry + rz * rz);
            if (!(r < rc)) continue;
            u += q[j] / r;
            /* -d(q_j/r)/dr_i = q_j (r_i - r_j) / r^3 */
            fx += q[j] * rx / (r * r * r);
            fy += q[j] * ry / (r * r * r);
            fz += q[j] * rz / (r * r * r);
        }
        phi[i] = ke * u;
        if (forces) {
            forces[3 * i] = ke * q[i] * fx;
            forces[3 * i + 1] = ke * q[i] * fy;
            forces[3 * i + 2] = ke * q[i] * fz;
        }
    }
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; i++) kadd(&e, q[i] * phi[i]);
    if (energy) *energy = 0.5 * (e.s + e.c);
    if (pot) memcpy(pot, phi, sizeof(double) * n);
    free(phi);
    return 0;
}

/* ---- Section 5: Wolf summation ---- */
int orc_wolf(int64_t n, const double *xyz, const double *q, const int32_t *molid, double rc, double alpha, double ke,
             double *energy, double *forces, double *pot)
{
    if (n < 0 || (n > 0 && (!xyz || !q)) || !(rc > 0) || !(alpha >= 0)) return -1;
    const double shift = erfc(alpha * rc) / rc;
    const double sqrt_pi = sqrt(acos(-1.0));
    const double self = erfc(alpha * rc) / (2.0 * rc) + alpha / sqrt_pi;
    double *phi = malloc(sizeof(double) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double u = 0, fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i || (molid && molid[j] == molid[i])) continue;
            double rx = xyz[3 * i] - xyz[3 * j], ry = xyz[3 * i + 1] - xyz[3 * j + 1],
                   rz = xyz[3 * i + 2] - xyz[3 * j + 2];
            double r = sqrt(rx * rx + ry * ry + rz * rz);
            if (!(r < rc)) continue;
            u += q[j] * (erfc(alpha * r) / r - shift);
            /* -d/dr (erfc(alpha r)/r) = erfc(alpha r)/r^2 + (2 alpha / sqrt(pi)) exp(-alpha^2 r^2) / r */
            double g = (erfc(alpha * r) / (r * r) + 2.0 * alpha / sqrt_pi * exp(-alpha * alpha * r * r) / r) / r;
            fx += q[j] * g * rx;
            fy += q[j] * g * ry;
            fz += q[j] * g * rz;
        }
        phi[i] = ke * (u - 2.0 * self * q[i]);
        if (forces) {
            forces[3 * i] = ke * q[i] * fx;
            forces[3 * i + 1] = ke * q[i] * fy;
            forces[3 * i + 2] = ke * q[i] * fz;
        }
    }
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; i++) kadd(&e, q[i] * phi[i]);
    if (energy) *energy = 0.5 * (e.s + e.c);
    if (pot) memcpy(pot, phi, sizeof(double) * n);
    free(phi);
    return 0;
}

int orc_cutoff_subset(int64_t n, const double *xyz, const double *q, const int32_t *molid, double rc, double ke,
                      int64_t nsel, const int64_t *sel, double *forces, double *pot)
{
    if (n < 0 || nsel < 0 || !(rc > 0) || (nsel > 0 && (!xyz || !q || !sel))) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < nsel; s++) {
        const int64_t i = sel[s];
        double u = 0, fx = 0, fy = 0, fz = 0;
        if (i < 0 || i >= n) continue;
        for (int64_t j = 0; j < n; j++) {
            if (j == i || (molid && molid[j] == molid[i])) continue;
            double rx = xyz[3 * i] - xyz[3 * j], ry = xyz[3 * i + 1] - xyz[3 * j + 1],
                   rz = xyz[3 * i + 2] - xyz[3 * j + 2];
            double r = sqrt(rx * rx + ry * ry + rz * rz);
            if (!(r < rc)) continue;
            u += q[j] / r;
            fx += q[j] * rx / (r * r * r);
            fy += q[j] * ry / (r * r * r);
            fz += q[j] * rz / (r * r * r);
        }
        if (pot) pot[s] = ke * u;
        if (forces) {
            forces[3 * s] = ke * q[i] * fx;
            forces[3 * s + 1] = ke * q[i] * fy;
            forces[3 * s + 2] = ke * q[i] * fz;
        }
    }
    return 0;
}
