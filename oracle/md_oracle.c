/*
 * FP64 CPU oracle for velocity-Verlet dynamics on the multilevel summation
 * method and for the parareal iteration over it.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the package smoke check
 * and the CPU-baseline leg of the benchmark. Shares no code with the HIP
 * library.
 *
 * The paper (Section 2) moves particles under F = -dU_all/dr with velocity
 * Verlet or leapfrog, U_all including bonded, van der Waals and Coulomb terms;
 * it gives no force field. The model here (a reading): rigid three-site
 * molecules held by RATTLE (Andersen 1983), Coulomb by MSM (or, for a
 * context with method ORC_METHOD_CUTOFF or ORC_METHOD_WOLF, by the simple
 * cutoff method or Wolf summation of Section 5) with the pairs inside one
 * molecule excluded, and Lennard-Jones
 * with Lorentz-Berthelot mixing, cut and shifted at the cutoff a.
 * Parareal follows Section 4: lambda_{n+1}^{k+1} = G(lambda_n^{k+1}) +
 * F(lambda_n^k) - G(lambda_n^k), started from a coarse sweep; for rigid
 * molecules each corrected state is projected back onto the constraints.
 */
#include "md_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- Coulomb pairs inside one molecule: remove k q_i q_j / r from the MSM
 * result, which includes every pair (atoms of a molecule are contiguous) ---- */
static void exclusions(const orc_params *p, const orc_model *m, int64_t n, const double *xyz, const double *q,
                       double *e, double *f)
{
    if (!m->molid) return;
    double acc = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n && m->molid[j] == m->molid[i]; j++) {
            double d[3], r2 = 0;
            for (int c = 0; c < 3; c++) {
                d[c] = xyz[3 * i + c] - xyz[3 * j + c];
                r2 += d[c] * d[c];
            }
            double r = sqrt(r2);
            double u = p->ke * q[i] * q[j] / r;
            acc += u;
            for (int c = 0; c < 3; c++) {
                double fc = u / r2 * d[c];      /* force of the pair on i */
                f[3 * i + c] -= fc;
                f[3 * j + c] += fc;
            }
        }
    *e -= acc;
}

/* ---- Lennard-Jones 4 eps ((s/r)^12 - (s/r)^6), shifted to zero at the cutoff a ---- */
static double lj_pair(double s, double eps, double r2, double rc2, double *fscal)
{
    double sr2 = s * s / r2, sr6 = sr2 * sr2 * sr2;
    double sc2 = s * s / rc2, sc6 = sc2 * sc2 * sc2;
    *fscal = 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / r2;   /* F_i = fscal (r_i - r_j) */
    return 4.0 * eps * (sr6 * sr6 - sr6) - 4.0 * eps * (sc6 * sc6 - sc6);
}

static void lennard_jones(const orc_params *p, const orc_model *m, int64_t n, const double *xyz, double *e, double *f)
{
    if (!m->lj || n == 0) return;
    double rc = p->a, rc2 = rc * rc;
    int nc[3];
    double cs[3];
    for (int d = 0; d < 3; d++) {
        double len = p->hi[d] - p->lo[d];
        nc[d] = (int)floor(len / (rc * 1.000001));
        if (nc[d] < 1) nc[d] = 1;
        cs[d] = len / nc[d];
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = malloc(sizeof(int64_t) * ncell), *next = malloc(sizeof(int64_t) * n);
    int *cell = malloc(sizeof(int) * 3 * n);
    for (int64_t c = 0; c < ncell; c++) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; i--) {
        int c3[3];
        for (int d = 0; d < 3; d++) {
            int c = (int)floor((xyz[3 * i + d] - p->lo[d]) / cs[d]);
            c3[d] = c < 0 ? 0 : (c >= nc[d] ? nc[d] - 1 : c);
            cell[3 * i + d] = c3[d];
        }
        int64_t id = ((int64_t)c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
        next[i] = head[id];
        head[id] = i;
    }
    double *ei = calloc(n, sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        if (m->lj[2 * i + 1] == 0.0) continue;
        double fx = 0, fy = 0, fz = 0, u = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int cx = cell[3 * i] + dx, cy = cell[3 * i + 1] + dy, cz = cell[3 * i + 2] + dz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= nc[0] || cy >= nc[1] || cz >= nc[2]) continue;
                    for (int64_t j = head[((int64_t)cz * nc[1] + cy) * nc[0] + cx]; j >= 0; j = next[j]) {
                        if (j == i || m->lj[2 * j + 1] == 0.0) continue;
                        if (m->molid && m->molid[i] == m->molid[j]) continue;
                        double d[3], r2 = 0;
                        for (int c = 0; c < 3; c++) {
                            d[c] = xyz[3 * i + c] - xyz[3 * j + c];
                            r2 += d[c] * d[c];
                        }
                        if (!(r2 < rc2)) continue;
                        double s = 0.5 * (m->lj[2 * i] + m->lj[2 * j]);
                        double eps = sqrt(m->lj[2 * i + 1] * m->lj[2 * j + 1]);
                        double fs;
                        u += lj_pair(s, eps, r2, rc2, &fs);
                        fx += fs * d[0];
                        fy += fs * d[1];
                        fz += fs * d[2];
                    }
                }
        f[3 * i] += fx;
        f[3 * i + 1] += fy;
        f[3 * i + 2] += fz;
        ei[i] = u;
    }
    double acc = 0;
    for (int64_t i = 0; i < n; i++) acc += ei[i];
    *e += 0.5 * acc;
    free(ei);
    free(head);
    free(next);
    free(cell);
}

int orc_md_forces(const orc_params *p, const orc_model *m, int64_t n, const double *xyz, const double *q,
                  double *epot, double *forces)
{
    double e = 0;
    if (p->method == ORC_METHOD_CUTOFF) {
        /* simple cutoff at a, intramolecular pairs left out of the sum */
        int rc = orc_cutoff(n, xyz, q, m->molid, p->a, p->ke, &e, forces, NULL);
        if (rc) return rc;
    } else if (p->method == ORC_METHOD_WOLF) {
        /* Wolf summation at a with damping alpha, intramolecular pairs left out */
        int rc = orc_wolf(n, xyz, q, m->molid, p->a, p->alpha, p->ke, &e, forces, NULL);
        if (rc) return rc;
    } else {
        int rc = orc_msm(p, n, xyz, q, &e, forces, NULL, NULL);
        if (rc) return rc;
        exclusions(p, m, n, xyz, q, &e, forces);
    }
    lennard_jones(p, m, n, xyz, &e, forces);
    if (epot) *epot = e;
    return 0;
}

/* ---- RATTLE (Andersen 1983) for rigid triples ---- */
static const int tri_a[3] = {0, 0, 1}, tri_b[3] = {1, 2, 2};

/* positions: bring |r'_a - r'_b| to d along the previous bond vectors, and
 * carry the same displacement into the half-step velocities */
static void rattle_positions(const orc_model *m, int64_t n, const double *xold, double *x, double *v, double dt)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n / 3; t++) {
        for (int it = 0; it < 1000; it++) {
            int done = 1;
            for (int c = 0; c < 3; c++) {
                int64_t a = 3 * t + tri_a[c], b = 3 * t + tri_b[c];
                double d = m->tri[c];
                double s[3], r[3], ss = 0, sr = 0;
                for (int k = 0; k < 3; k++) {
                    s[k] = x[3 * a + k] - x[3 * b + k];
                    r[k] = xold[3 * a + k] - xold[3 * b + k];
                    ss += s[k] * s[k];
                    sr += s[k] * r[k];
                }
                double diff = d * d - ss;
                if (fabs(diff) <= 2.0 * m->tol * d * d) continue;
                done = 0;
                double ia = 1.0 / m->mass[a], ib = 1.0 / m->mass[b];
                double g = diff / (2.0 * sr * (ia + ib));
                for (int k = 0; k < 3; k++) {
                    x[3 * a + k] += g * ia * r[k];
                    x[3 * b + k] -= g * ib * r[k];
                    v[3 * a + k] += g * ia * r[k] / dt;
                    v[3 * b + k] -= g * ib * r[k] / dt;
                }
            }
            if (done) break;
        }
    }
}

/* velocities: remove the relative velocity along every bond */
static void rattle_velocities(const orc_model *m, int64_t n, const double *x, double *v)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n / 3; t++) {
        for (int it = 0; it < 1000; it++) {
            int done = 1;
            for (int c = 0; c < 3; c++) {
                int64_t a = 3 * t + tri_a[c], b = 3 * t + tri_b[c];
                double d = m->tri[c];
                double r[3], w[3], rw = 0;
                for (int k = 0; k < 3; k++) {
                    r[k] = x[3 * a + k] - x[3 * b + k];
                    w[k] = v[3 * a + k] - v[3 * b + k];
                    rw += r[k] * w[k];
                }
                double ia = 1.0 / m->mass[a], ib = 1.0 / m->mass[b];
                double kk = rw / ((ia + ib) * d * d);
                if (fabs(rw) <= m->tol * d * d) continue;
                done = 0;
                for (int k = 0; k < 3; k++) {
                    v[3 * a + k] -= kk * ia * r[k];
                    v[3 * b + k] += kk * ib * r[k];
                }
            }
            if (done) break;
        }
    }
}

/* ---- Section 2: velocity Verlet ---- */
int orc_vv(const orc_params *p, const orc_model *m, int64_t n, double *xyz, double *v, const double *q,
           double dt, int nsteps, double *epot, double *ekin)
{
    double *f = malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double *xold = malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double e = 0;
    int rc = orc_md_forces(p, m, n, xyz, q, &e, f);
    for (int s = 0; rc == 0 && s < nsteps; s++) {
        memcpy(xold, xyz, sizeof(double) * 3 * n);
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < 3; k++) {
                v[3 * i + k] += 0.5 * dt * f[3 * i + k] / m->mass[i];
                xyz[3 * i + k] += dt * v[3 * i + k];
            }
        if (m->rigid) rattle_positions(m, n, xold, xyz, v, dt);
        rc = orc_md_forces(p, m, n, xyz, q, &e, f);
        if (rc) break;
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < 3; k++) v[3 * i + k] += 0.5 * dt * f[3 * i + k] / m->mass[i];
        if (m->rigid) rattle_velocities(m, n, xyz, v);
    }
    if (epot) *epot = e;
    if (ekin) {
        double k = 0;
        for (int64_t i = 0; i < n; i++)
            k += 0.5 * m->mass[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
        *ekin = k;
    }
    free(f);
    free(xold);
    return rc;
}

/* ---- Multiple time steps (Section 5 names them as a further improvement) ----
 * The MSM force splits into a fast part, the short-range pairs (g* for every
 * pair inside a, Coulomb removed again for the excluded pairs) plus
 * Lennard-Jones, and a slow part, the grid potential's gradient; the smooth
 * self term is constant and goes with the slow energy. */
int orc_md_forces_split(const orc_params *p, const orc_model *m, int64_t n, const double *xyz, const double *q,
                        double *e_fast, double *f_fast, double *e_slow, double *f_slow)
{
    if (p->method != ORC_METHOD_MSM) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *us = malloc(sizeof(double) * nn), *fs = malloc(sizeof(double) * 3 * nn);
    double *ul = malloc(sizeof(double) * nn), *gl = malloc(sizeof(double) * 3 * nn);
    orc_stages st;
    memset(&st, 0, sizeof(st));
    st.u_short = us;
    st.f_short = fs;
    st.u_long = ul;
    st.g_long = gl;
    double etot = 0;
    int rc = orc_msm(p, n, xyz, q, &etot, NULL, NULL, &st);
    if (!rc) {
        const double self = orc_gamma_m(0.0, p->smoothing > 0 ? p->smoothing : 2) / p->a;
        double ef = 0, es = 0;
        for (int64_t i = 0; i < n; i++) {
            ef += 0.5 * p->ke * q[i] * us[i];
            es += 0.5 * p->ke * q[i] * (ul[i] - q[i] * self);
            for (int k = 0; k < 3; k++) {
                f_fast[3 * i + k] = p->ke * q[i] * fs[3 * i + k];
                f_slow[3 * i + k] = -p->ke * q[i] * gl[3 * i + k];
            }
        }
        exclusions(p, m, n, xyz, q, &ef, f_fast);
        lennard_jones(p, m, n, xyz, &ef, f_fast);
        *e_fast = ef;
        *e_slow = es;
    }
    free(us);
    free(fs);
    free(ul);
    free(gl);
    return rc;
}

/* Impulse multiple-time-step velocity Verlet (r-RESPA, Tuckerman et al.
 * 1992): every outer step of dt is a half kick with the slow force, ninner
 * velocity-Verlet steps of dt/ninner with the fast force (RATTLE for rigid
 * triples), the slow force at the new positions and a second slow half kick
 * (followed by the velocity constraints). */
int orc_vv_mts(const orc_params *p, const orc_model *m, int64_t n, double *xyz, double *v, const double *q,
               double dt, int ninner, int nouter, double *epot, double *ekin)
{
    if (ninner < 1 || nouter < 0) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *ff = malloc(sizeof(double) * 3 * nn), *fsl = malloc(sizeof(double) * 3 * nn);
    double *xold = malloc(sizeof(double) * 3 * nn);
    double ef = 0, es = 0;
    const double di = dt / ninner;
    int rc = orc_md_forces_split(p, m, n, xyz, q, &ef, ff, &es, fsl);
    for (int o = 0; rc == 0 && o < nouter; o++) {
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < 3; k++) v[3 * i + k] += 0.5 * dt * fsl[3 * i + k] / m->mass[i];
        if (m->rigid) rattle_velocities(m, n, xyz, v);
        for (int s = 0; rc == 0 && s < ninner; s++) {
            memcpy(xold, xyz, sizeof(double) * 3 * n);
            for (int64_t i = 0; i < n; i++)
                for (int k = 0; k < 3; k++) {
                    v[3 * i + k] += 0.5 * di * ff[3 * i + k] / m->mass[i];
                    xyz[3 * i + k] += di * v[3 * i + k];
                }
            if (m->rigid) rattle_positions(m, n, xold, xyz, v, di);
            /* both parts at the new positions; the inner step uses the fast
             * one, and after the last inner step fsl is the slow force for
             * the closing slow kick */
            rc = orc_md_forces_split(p, m, n, xyz, q, &ef, ff, &es, fsl);
            if (rc) break;
            for (int64_t i = 0; i < n; i++)
                for (int k = 0; k < 3; k++) v[3 * i + k] += 0.5 * di * ff[3 * i + k] / m->mass[i];
            if (m->rigid) rattle_velocities(m, n, xyz, v);
        }
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < 3; k++) v[3 * i + k] += 0.5 * dt * fsl[3 * i + k] / m->mass[i];
        if (m->rigid) rattle_velocities(m, n, xyz, v);
    }
    if (epot) *epot = ef + es;
    if (ekin) {
        double kk = 0;
        for (int64_t i = 0; i < n; i++)
            kk += 0.5 * m->mass[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
        *ekin = kk;
    }
    free(ff);
    free(fsl);
    free(xold);
    return rc;
}

/* ---- Section 4: parareal ---- */

/* Project a corrected state (n x 6) of rigid triples back onto the
 * constraints (a reading; the paper is silent on constraints): positions move
 * along their own bond vectors until every bond has its length, then
 * velocities lose their relative component along every bond. A state that
 * already satisfies the constraints is left unchanged. */
static void project_triples(const orc_model *m, int64_t n, double *st)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n / 3; t++) {
        for (int it = 0; it < 1000; it++) {
            int done = 1;
            for (int c = 0; c < 3; c++) {
                int64_t a = 3 * t + tri_a[c], b = 3 * t + tri_b[c];
                double d = m->tri[c];
                double s[3], ss = 0;
                for (int k = 0; k < 3; k++) {
                    s[k] = st[6 * a + k] - st[6 * b + k];
                    ss += s[k] * s[k];
                }
                double diff = d * d - ss;
                if (fabs(diff) <= 2.0 * m->tol * d * d) continue;
                done = 0;
                double ia = 1.0 / m->mass[a], ib = 1.0 / m->mass[b];
                double g = diff / (2.0 * ss * (ia + ib));
                for (int k = 0; k < 3; k++) {
                    st[6 * a + k] += g * ia * s[k];
                    st[6 * b + k] -= g * ib * s[k];
                }
            }
            if (done) break;
        }
        for (int it = 0; it < 1000; it++) {
            int done = 1;
            for (int c = 0; c < 3; c++) {
                int64_t a = 3 * t + tri_a[c], b = 3 * t + tri_b[c];
                double d = m->tri[c];
                double r[3], w[3], rw = 0;
                for (int k = 0; k < 3; k++) {
                    r[k] = st[6 * a + k] - st[6 * b + k];
                    w[k] = st[6 * a + 3 + k] - st[6 * b + 3 + k];
                    rw += r[k] * w[k];
                }
                if (fabs(rw) <= m->tol * d * d) continue;
                done = 0;
                double ia = 1.0 / m->mass[a], ib = 1.0 / m->mass[b];
                double kk = rw / ((ia + ib) * d * d);
                for (int k = 0; k < 3; k++) {
                    st[6 * a + 3 + k] -= kk * ia * r[k];
                    st[6 * b + 3 + k] += kk * ib * r[k];
                }
            }
            if (done) break;
        }
    }
}
static int propagate(const orc_params *p, const orc_model *m, int64_t n, const double *q, const double *in,
                     double *out, int steps, double dt, double *x, double *v)
{
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < 3; k++) {
            x[3 * i + k] = in[6 * i + k];
            v[3 * i + k] = in[6 * i + 3 + k];
        }
    int rc = orc_vv(p, m, n, x, v, q, dt, steps, NULL, NULL);
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < 3; k++) {
            out[6 * i + k] = x[3 * i + k];
            out[6 * i + 3 + k] = v[3 * i + k];
        }
    return rc;
}

int orc_parareal(const orc_params *pf, const orc_params *pg, const orc_model *m, int64_t n, const double *q,
                 const double *state0, int nslices, int steps_f, double dt_f, int steps_g, double dt_g, int kmax,
                 double tol, double *lambda, int *iters, double *resid)
{
    if (nslices < 1 || kmax < 0 || n < 0) return -1;
    const size_t S = (size_t)6 * n;
    double *gold = malloc(sizeof(double) * S * (nslices + 1));
    double *fout = malloc(sizeof(double) * S * (nslices + 1));
    double *gnew = malloc(sizeof(double) * S);
    double *corr = malloc(sizeof(double) * S);
    double *x = malloc(sizeof(double) * 3 * (n > 0 ? n : 1)), *v = malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    int rc = 0, done = 0;
    memcpy(lambda, state0, sizeof(double) * S);
    /* initial coarse sweep: lambda^0_{n+1} = G(lambda^0_n) */
    for (int s = 0; s < nslices && !rc; s++) {
        rc = propagate(pg, m, n, q, lambda + S * s, lambda + S * (s + 1), steps_g, dt_g, x, v);
        memcpy(gold + S * (s + 1), lambda + S * (s + 1), sizeof(double) * S);
    }
    *iters = 0;
    for (int k = 0; k < kmax && !rc && !done; k++) {
        /* fine propagator on every slice not yet exact (slices < k are) */
        for (int s = k; s < nslices && !rc; s++)
            rc = propagate(pf, m, n, q, lambda + S * s, fout + S * (s + 1), steps_f, dt_f, x, v);
        /* serial correction sweep: lambda_{s+1} = F(lambda^k_s) + (G(lambda^{k+1}_s) - G(lambda^k_s)) */
        double change = 0;
        for (int s = k; s < nslices && !rc; s++) {
            rc = propagate(pg, m, n, q, lambda + S * s, gnew, steps_g, dt_g, x, v);
            double *lam = lambda + S * (s + 1), *fo = fout + S * (s + 1), *go = gold + S * (s + 1);
            for (size_t e = 0; e < S; e++) {
                corr[e] = fo[e] + (gnew[e] - go[e]);
                go[e] = gnew[e];
            }
            if (m->rigid) project_triples(m, n, corr);
            for (size_t e = 0; e < S; e++) {
                if (e % 6 < 3) {
                    double c = fabs(corr[e] - lam[e]);
                    if (c != c) c = INFINITY;
                    if (c > change) change = c;
                }
                lam[e] = corr[e];
            }
        }
        resid[k] = change;
        *iters = k + 1;
        if (change < tol || k + 1 >= nslices) done = 1;
    }
    free(gold);
    free(fout);
    free(gnew);
    free(corr);
    free(x);
    free(v);
    if (rc) return rc;
    return done ? 0 : 1;
}

/* Parareal over a computational window that slides along the time axis
 * (Section 4). The states lambda_{start+1} .. lambda_{start+We} (We =
 * min(width, nslices - start)) are iterated with the update of Section 4
 * while lambda_0 .. lambda_start are final. After an iteration the first open
 * state is exact (its fine run started from a final state), and each further
 * leading state whose positions moved by less than tol is accepted too; the
 * window then starts at the last accepted state and its new tail states get
 * the coarse prediction. */
int orc_parareal_window(const orc_params *pf, const orc_params *pg, const orc_model *m, int64_t n, const double *q,
                        int nslices, int width, int steps_f, double dt_f, int steps_g, double dt_g, double tol,
                        int max_iters, double *lambda, double *ring, orc_window_state *st)
{
    if (nslices < 1 || width < 1 || n < 0 || max_iters < 0 || !st) return -1;
    if (st->start < 0 || st->start > nslices) return -1;
    const size_t S = (size_t)6 * n;
    double *fout = malloc(sizeof(double) * S * width);
    double *gnew = malloc(sizeof(double) * S);
    double *corr = malloc(sizeof(double) * S);
    double *chg = malloc(sizeof(double) * width);
    double *x = malloc(sizeof(double) * 3 * (n > 0 ? n : 1)), *v = malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    int rc = 0, done_here = 0;
#define LAM(s) (lambda + S * (size_t)(s))
#define RING(s) (ring + S * (size_t)((s) % width))
    int b = st->start;
    int end = b + (width < nslices - b ? width : nslices - b);   /* last state of the window */
    if (!st->window_valid) {
        /* coarse prediction of the window: lambda_{s+1} = G(lambda_s), kept as G(lambda_s) */
        for (int s = b; s < end && !rc; s++) {
            rc = propagate(pg, m, n, q, LAM(s), LAM(s + 1), steps_g, dt_g, x, v);
            memcpy(RING(s), LAM(s + 1), sizeof(double) * S);
            st->coarse_slices++;
        }
        st->window_valid = 1;
    }
    while (!rc && b < nslices && (max_iters == 0 || done_here < max_iters)) {
        const int we = end - b;
        /* fine propagator on every open slice */
        for (int j = 0; j < we && !rc; j++)
            rc = propagate(pf, m, n, q, LAM(b + j), fout + S * j, steps_f, dt_f, x, v);
        st->fine_slices += we;
        /* serial sweep: lambda_{s+1} = F(lambda^k_s) + (G(lambda^{k+1}_s) - G(lambda^k_s)) */
        for (int j = 0; j < we && !rc; j++) {
            const int s = b + j;
            rc = propagate(pg, m, n, q, LAM(s), gnew, steps_g, dt_g, x, v);
            double *lam = LAM(s + 1), *go = RING(s), *fo = fout + S * j;
            for (size_t e = 0; e < S; e++) {
                corr[e] = fo[e] + (gnew[e] - go[e]);
                go[e] = gnew[e];
            }
            if (m->rigid) project_triples(m, n, corr);
            double change = 0;
            for (size_t e = 0; e < S; e++) {
                if (e % 6 < 3) {
                    double c = fabs(corr[e] - lam[e]);
                    if (c != c) c = INFINITY;
                    if (c > change) change = c;
                }
                lam[e] = corr[e];
            }
            chg[j] = change;
        }
        st->coarse_slices += we;
        if (rc) break;
        /* the first open state is exact; accept the following ones that moved less than tol */
        int acc = 1;
        while (acc < we && chg[acc] < tol) acc++;
        double worst = 0;
        for (int j = 0; j < we; j++)
            if (chg[j] > worst) worst = chg[j];
        st->last_accepted = acc;
        st->last_change = worst;
        st->iterations++;
        done_here++;
        b += acc;
        /* slide: coarse predictions for the states that enter the window */
        const int new_end = b + (width < nslices - b ? width : nslices - b);
        for (int s = end; s < new_end && !rc; s++) {
            rc = propagate(pg, m, n, q, LAM(s), LAM(s + 1), steps_g, dt_g, x, v);
            memcpy(RING(s), LAM(s + 1), sizeof(double) * S);
            st->coarse_slices++;
        }
        end = new_end;
    }
#undef LAM
#undef RING
    st->start = b;
    free(fout);
    free(gnew);
    free(corr);
    free(chg);
    free(x);
    free(v);
    if (rc) return rc;
    return b == nslices ? 0 : 1;
}
