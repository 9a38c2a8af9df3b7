/*
 * FP64 CPU oracle for the multilevel summation method (MSM) and the
 * velocity-Verlet / parareal integration that uses it.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load or call this library. It
 * shares no code, header, table or constant generator with the HIP library;
 * it is written to be read against the paper, not to be fast.
 *
 * Units: nm, e, kJ/mol (with ke = 1/(4 pi eps0) = 138.935458 kJ mol^-1 nm e^-2),
 * or ke = 1 for unit tests. Arrays are row-major; positions are (n, 3).
 * Return codes: 0 ok, -1 bad argument, -2 atom outside the domain,
 * -3 non-finite input.
 */
#ifndef MSM_ORACLE_H
#define MSM_ORACLE_H
#include <stdint.h>

#define ORC_MAXLEV 16

#define ORC_METHOD_MSM 0
#define ORC_METHOD_CUTOFF 1
#define ORC_METHOD_WOLF 2

typedef struct {
    double a;          /* short-range cutoff (the cutoff radius for ORC_METHOD_CUTOFF) */
    double h;          /* finest grid spacing */
    int levels;        /* number of grids l; 0 = choose from the domain */
    double lo[3];      /* domain lower corner (grid origin of every level) */
    double hi[3];      /* domain upper corner */
    double ke;         /* Coulomb constant */
    int method;        /* ORC_METHOD_MSM, or ORC_METHOD_CUTOFF: the simple cutoff
                          method of Section 5 (used by the dynamics oracle) */
    int smoothing;     /* order m of the smoothing function (degree 2m); 0 = 2 */
    int basis;         /* degree p of the nodal basis Phi: 3 (0 means 3) or 5 */
    double alpha;      /* damping of the Wolf method (1/nm), ORC_METHOD_WOLF only */
} orc_params;

/* Optional per-stage outputs; any pointer may be NULL. Grid arrays are
 * x-fastest over the level's node range (see orc_grid_shape). */
typedef struct {
    double *u_short;               /* n: sum_j g*(r_ij) q_j */
    double *f_short;               /* n*3: -sum_j q_j (dg^*(r)/dr) (r_i - r_j) / r_ij */
    double *q_grid[ORC_MAXLEV];    /* grid charges q^k */
    double *ucut_grid[ORC_MAXLEV]; /* lattice-cutoff potentials u^{k,cutoff} (top: u^{l-1}) */
    double *u_grid[ORC_MAXLEV];    /* prolongated potentials u^k */
    double *u_long;                /* n: sum_mu phi_mu(r_i) u^0_mu */
    double *g_long;                /* n*3: sum_mu grad phi_mu(r_i) u^0_mu */
} orc_stages;

int orc_threads(void);
/* OpenMP threads of the parallel loops that follow (n > 0). */
void orc_set_threads(int n);
/* gamma of order m (degree 2m) and its derivative; the unsuffixed forms are m = 2 */
double orc_gamma_m(double rho, int m);
double orc_dgamma_m(double rho, int m);
double orc_gamma(double rho);
double orc_dgamma(double rho);
double orc_Phi(double t);
double orc_Phi_p(double t, int p);
double orc_dPhi_p(double t, int p);
double orc_dPhi(double t);
double orc_gstar(double r, double a);
double orc_dgstar(double r, double a);
double orc_glevel(double r, double a, int k, int l);
double orc_gstar_m(double r, double a, int m);
double orc_dgstar_m(double r, double a, int m);
double orc_glevel_m(double r, double a, int k, int l, int m);

int orc_levels(const orc_params *p);
int orc_grid_shape(const orc_params *p, int level, int org[3], int dim[3]);

int orc_msm(const orc_params *p, int64_t n, const double *xyz, const double *q,
            double *energy, double *forces, double *pot, orc_stages *st);

/* u_short and the short-range force bracket (as in orc_stages) of the atoms
 * listed in sel, each by a direct loop over all atoms. */
int orc_short_subset(const orc_params *p, int64_t n, const double *xyz, const double *q, int64_t nsel,
                     const int64_t *sel, double *u, double *f);

int orc_coulomb(int64_t n, const double *xyz, const double *q, double ke,
                double *energy, double *forces, double *pot);

/* Simple cutoff method (Section 5, the coarse propagator the paper proposes):
 * Coulomb's law between every pair closer than rc and nothing beyond,
 * phi_i = ke sum_{j != i, r_ij < rc} q_j / r_ij, U = 1/2 sum_i q_i phi_i and
 * F_i = -dU/dr_i away from the cutoff sphere. molid (may be NULL) removes the
 * pairs of equal molecule id. Direct double loop over all pairs. */
int orc_cutoff(int64_t n, const double *xyz, const double *q, const int32_t *molid, double rc, double ke,
               double *energy, double *forces, double *pot);

/* Wolf summation (Section 5 names it as a coarse propagator; Wolf et al.
 * 1999): damped, shifted pair potential below rc,
 *   phi_i = ke [ sum_{j != i, r_ij < rc} q_j (erfc(alpha r)/r - erfc(alpha rc)/rc) - 2 C q_i ],
 *   C = erfc(alpha rc)/(2 rc) + alpha/sqrt(pi),
 * U = 1/2 sum_i q_i phi_i, F_i = -dU/dr_i (the shift and the self term are
 * constant in the positions). molid (may be NULL) removes the pairs of equal
 * molecule id. Direct double loop over all pairs. */
int orc_wolf(int64_t n, const double *xyz, const double *q, const int32_t *molid, double rc, double alpha, double ke,
             double *energy, double *forces, double *pot);

/* The potentials and forces of orc_cutoff for the atoms listed in sel only,
 * each by a direct loop over all atoms (spot checks of very large systems). */
int orc_cutoff_subset(int64_t n, const double *xyz, const double *q, const int32_t *molid, double rc, double ke,
                      int64_t nsel, const int64_t *sel, double *forces, double *pot);

#endif
