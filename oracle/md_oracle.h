/*
 * FP64 CPU oracle for velocity-Verlet dynamics driven by the multilevel
 * summation method, and for the parareal iteration over it.
 *
 * TEST INFRASTRUCTURE ONLY (see msm_oracle.h).
 */
#ifndef MD_ORACLE_H
#define MD_ORACLE_H
#include <stdint.h>

#include "msm_oracle.h"

/* Molecular model of a run. Atoms of one molecule are contiguous. */
typedef struct {
    const double *mass;     /* n */
    const int32_t *molid;   /* n, or NULL: no excluded pairs */
    const double *lj;       /* n x 2 (sigma, epsilon), Lorentz-Berthelot mixing, cut and
                               shifted to zero at the MSM cutoff a; NULL: none */
    int rigid;              /* 1: atoms (3m, 3m+1, 3m+2) keep fixed mutual distances */
    double tri[3];          /* |r0-r1|, |r0-r2|, |r1-r2| of every rigid triple */
    double tol;             /* relative tolerance of the constraint iteration */
} orc_model;

/* Potential energy and forces: Coulomb by MSM (p->method ORC_METHOD_MSM), by
 * the simple cutoff at p->a (ORC_METHOD_CUTOFF) or by Wolf summation at p->a
 * with damping p->alpha (ORC_METHOD_WOLF), intramolecular pairs excluded,
 * plus Lennard-Jones. */
int orc_md_forces(const orc_params *p, const orc_model *m, int64_t n, const double *xyz, const double *q,
                  double *epot, double *forces);

/* The MSM model force split for multiple time steps: fast = the short-range
 * pairs (g* for every pair inside a, Coulomb removed again for excluded
 * pairs) plus Lennard-Jones; slow = the grid potential's gradient (the smooth
 * self term goes with the slow energy). fast + slow = orc_md_forces. MSM only. */
int orc_md_forces_split(const orc_params *p, const orc_model *m, int64_t n, const double *xyz, const double *q,
                        double *e_fast, double *f_fast, double *e_slow, double *f_slow);

/* nouter impulse multiple-time-step steps of dt (r-RESPA): slow half kick,
 * ninner velocity-Verlet steps of dt/ninner with the fast force, slow half
 * kick; RATTLE for rigid triples. epot/ekin after the last step. */
int orc_vv_mts(const orc_params *p, const orc_model *m, int64_t n, double *xyz, double *v, const double *q,
               double dt, int ninner, int nouter, double *epot, double *ekin);

/* nsteps of velocity Verlet (with RATTLE for rigid triples) in place.
 * epot/ekin receive the energies after the last step (may be NULL). */
int orc_vv(const orc_params *p, const orc_model *m, int64_t n, double *xyz, double *v, const double *q,
           double dt, int nsteps, double *epot, double *ekin);

/* Parareal (Section 4) over nslices slices of the fine propagator
 * (pf, steps_f x dt_f) with the coarse one (pg, steps_g x dt_g). With rigid
 * triples every corrected state is projected back onto the constraints
 * (positions along their bond vectors, then velocities).
 * state0: n x 6 (x y z vx vy vz). lambda: (nslices+1) x n x 6, out.
 * Stops at the first iteration whose largest position change is below tol
 * or after kmax iterations; *iters receives the number done and resid[k]
 * the position change of iteration k (kmax entries). Returns 0, 1 when not
 * converged, or a negative error. */
int orc_parareal(const orc_params *pf, const orc_params *pg, const orc_model *m, int64_t n, const double *q,
                 const double *state0, int nslices, int steps_f, double dt_f, int steps_g, double dt_g, int kmax,
                 double tol, double *lambda, int *iters, double *resid);

/* Resumable state of a sliding-window parareal run: a checkpoint is this
 * struct with lambda and the coarse ring. A new run starts from zeros. */
typedef struct {
    int start;              /* lambda_0 .. lambda_start are final */
    int window_valid;       /* 1: the window's states and the ring hold iterates;
                               0: the window is predicted from lambda_start */
    int iterations;         /* iterations so far */
    int last_accepted;      /* states accepted by the last iteration */
    int64_t fine_slices;    /* fine-propagator slice runs so far */
    int64_t coarse_slices;  /* coarse-propagator slice runs so far */
    double last_change;     /* largest position change of the last iteration */
} orc_window_state;

/* Parareal with a sliding computational window (Section 4) over nslices
 * slices, width slices iterated at once. After each iteration the first open
 * state is exact and the following states that moved by less than tol (nm)
 * are accepted; the window moves past the accepted states and the states
 * entering it get the coarse prediction. tol = 0 accepts exact states only,
 * which gives the serial fine trajectory bitwise.
 * lambda: (nslices+1) x n x 6, lambda_0 in, every state out;
 * ring: width x n x 6, G(lambda_s) of the window's slice s at slot s % width.
 * Runs at most max_iters iterations (0: no limit). Returns 0 when every slice
 * is final, 1 when stopped early (resume by calling again with the same
 * lambda, ring and state), or a negative error. */
int orc_parareal_window(const orc_params *pf, const orc_params *pg, const orc_model *m, int64_t n, const double *q,
                        int nslices, int width, int steps_f, double dt_f, int steps_g, double dt_g, double tol,
                        int max_iters, double *lambda, double *ring, orc_window_state *st);

#endif
