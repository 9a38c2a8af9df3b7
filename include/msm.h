/*
 * msmx: multilevel summation electrostatics and parareal velocity Verlet on
 * one AMD Instinct MI355X (gfx950).
 *
 * C ABI of libmsmx.so. Method: J. Pazurikova and L. Matyska, "Parallel-in-time
 * method for calculation of long-range electrostatic interactions"
 * (arXiv:1309.1889). Section 2 states the problem (charges q_i, positions r_i,
 * velocities v_i in; potential energy U and forces F_i = -dU/dr_i out),
 * Section 3 the multilevel summation method (MSM) that evaluates U, and
 * Section 4 the parareal iteration that uses a fine and a coarse propagator,
 * and Section 5 the combination, with the simple cutoff method as the coarse
 * propagator.
 *
 * Conventions
 *  - Units: nm, e, amu, ps, kJ/mol; coulomb_k = 1/(4 pi eps0) = 138.935458
 *    kJ mol^-1 nm e^-2 (or 1.0 for unit tests).
 *  - Every pointer whose name ends in _dev is a device pointer (HBM of the
 *    context's GPU) owned by the caller; _host pointers are host memory owned
 *    by the caller. The library owns its workspace, allocated in msm_setup and
 *    freed in msm_destroy; the evaluation and integration calls allocate no
 *    memory.
 *  - Calls are asynchronous on the stream given at setup: they return once
 *    the work is enqueued. Results are valid after the stream synchronises.
 *    Conditions only the device can see (an atom outside the domain, a
 *    non-finite value) set a status word that msm_get_status reads.
 *  - Precision: MSM_FP64 runs every step in double. MSM_FP32 runs pair, grid
 *    and stencil arithmetic in float and keeps the energy reduction (and the
 *    parareal correction) in double. Positions/charges, forces and potentials
 *    are float or double accordingly.
 *  - Return value: MSM_OK (0), MSM_NOT_CONVERGED (1) or a negative MSM_ERR_*.
 *  - A context is used by one host thread at a time.
 */
#ifndef MSMX_MSM_H
#define MSMX_MSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MSM_OK = 0,
    MSM_NOT_CONVERGED = 1,      /* parareal stopped at kmax above tolerance */
    MSM_ERR_ARG = -1,           /* invalid argument */
    MSM_ERR_DOMAIN = -2,        /* an atom lies outside its system's domain */
    MSM_ERR_NONFINITE = -3,     /* a position or charge is NaN or infinite */
    MSM_ERR_CAPACITY = -4,      /* more atoms/systems or a larger domain than set up for */
    MSM_ERR_HIP = -5,           /* a HIP runtime call failed */
    MSM_ERR_UNSUPPORTED = -6,   /* parameters outside what the kernels are built for */
    MSM_ERR_CONSTRAINT = -7     /* the constraint iteration of a rigid molecule stopped at its
                                   cap (500 steps) without meeting the tolerance */
};

enum { MSM_FP64 = 0, MSM_FP32 = 1 };

/* How the Coulomb interaction is evaluated. MSM_METHOD_MSM: multilevel
 * summation (Section 3). MSM_METHOD_CUTOFF: the simple cutoff method the
 * paper chooses for the coarse parareal propagator (Section 5): Coulomb's law
 * between the pairs closer than a and nothing beyond. MSM_METHOD_WOLF: Wolf
 * summation, which Section 5 proposes as its refinement (Wolf et al. 1999):
 * the damped, shifted pair potential erfc(alpha r)/r - erfc(alpha a)/a below
 * a and the self term -(erfc(alpha a)/(2a) + alpha/sqrt(pi)) q_i^2. Neither
 * builds grids: h is only the edge of the cells of the pair search and
 * levels, smoothing and basis are ignored. */
enum { MSM_METHOD_MSM = 0, MSM_METHOD_CUTOFF = 1, MSM_METHOD_WOLF = 2 };

typedef struct msm_ctx msm_ctx;   /* opaque; owned by the library */

/* Method parameters (Section 3): cutoff a, finest spacing h, number of grids
 * l, the order m of the smoothing function, the degree p of the nodal basis,
 * and the domain. p = 3 (the C1 cubic numerical Hermite interpolant) with
 * m = 2 (the C2 even quartic) is the pair the paper selects for accuracy and
 * cost; higher orders trade cost for accuracy. */
typedef struct {
    double a;              /* short-range cutoff (nm), > 0 */
    double h;              /* finest grid spacing (nm), > 0; a/h <= 6 */
    int levels;            /* number of grids l; 0 = smallest l with the coarsest
                              grid spanning at most 4 spacings per axis */
    int precision;         /* MSM_FP64 or MSM_FP32 */
    double lo[3], hi[3];   /* non-periodic domain; its extent bounds every system's */
    double coulomb_k;      /* prefactor of the potential */
    int64_t max_atoms;     /* capacity: atoms summed over a batch */
    int max_systems;       /* capacity: systems per batch */
    int method;            /* MSM_METHOD_MSM or MSM_METHOD_CUTOFF */
    int smoothing;         /* order m of gamma (Section 3: degree 2m), 1 .. 3; 0 = 2.
                              For rho < 1 gamma is the Taylor polynomial of
                              (rho^2)^(-1/2) about rho^2 = 1 up to (rho^2 - 1)^m,
                              which joins 1/rho with m continuous derivatives */
    int basis;             /* degree p of the nodal basis Phi (Section 3), 3 or 5;
                              0 = 3. p = 5: the quintic Hermite interpolant of the
                              cardinal data with five-point central differences
                              for the node first and second derivatives (C2,
                              support |t| < 3: 6 nodes per axis per atom) */
    double alpha;          /* Wolf damping alpha (1/nm), >= 0; MSM_METHOD_WOLF only */
} msm_params;

/* Create a context: validates the parameters, builds the stencil weights and
 * allocates the workspace for max_atoms atoms in up to max_systems systems
 * whose domains are no larger than [lo, hi]. stream is a hipStream_t (NULL:
 * the null stream). On success *out owns the context. */
int msm_setup(const msm_params *params, void *stream, msm_ctx **out);

/* Release the context and its workspace (synchronises its stream). NULL is a no-op. */
void msm_destroy(msm_ctx *ctx);

/* Change the stream later calls are enqueued on. */
int msm_set_stream(msm_ctx *ctx, void *stream);

/* Energy, forces and per-atom potentials of nsys independent systems
 * (Section 3: short-range part, anterpolation, restriction, lattice cutoff,
 * top level, prolongation, interpolation, and the combination
 * U_i = k (u_i^short + u_i^long); Section 2: F_i = -dU/dr_i).
 *
 *  offsets_host   nsys+1 increasing int64; system s owns atoms
 *                 [offsets[s], offsets[s+1]) of the arrays below;
 *                 offsets[0] = 0 and offsets[nsys] <= max_atoms.
 *  domains_host   NULL (every system uses the context's domain) or nsys*6
 *                 doubles lo_x lo_y lo_z hi_x hi_y hi_z, each extent no
 *                 larger than the context's.
 *  xyzq_dev       N x 4 (x, y, z, q), float or double per the precision.
 *  energy_dev     nsys doubles: U = 1/2 sum_i q_i phi_i per system, where phi_i
 *                 excludes the atom's own charge (the smooth self term
 *                 q_i gamma(0)/a is removed). May be NULL. With
 *                 MSM_METHOD_CUTOFF, phi_i = k sum_{j != i, r_ij < a} q_j / r_ij;
 *                 with MSM_METHOD_WOLF, phi_i = k (sum_{j != i, r_ij < a}
 *                 q_j (erfc(alpha r)/r - erfc(alpha a)/a) - 2 C q_i),
 *                 C = erfc(alpha a)/(2a) + alpha/sqrt(pi).
 *  forces_dev     N x 3, F_i = -dU/dr_i. May be NULL.
 *  potentials_dev N, phi_i = dU/dq_i. May be NULL.
 * Outputs are in the caller's atom order. Results for a system with an atom
 * outside its domain or a non-finite input are undefined; the status word
 * reports it. Two atoms at the same position are not allowed. */
int msm_energy_forces(msm_ctx *ctx, int nsys, const int64_t *offsets_host,
                      const double *domains_host, const void *xyzq_dev,
                      double *energy_dev, void *forces_dev, void *potentials_dev);

/* Allocation-free evaluation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): msm_energy_forces for one system of natoms atoms on the
 * current device, without a context. Every work array (cells, sorted atoms,
 * all grids, the stencil and plan tables) lives in one static device array
 * of MSM_NOALLOC_SCRATCH_MIB MiB per device, which the library holds from
 * the first call on that device until the process ends; the call allocates
 * no device or pinned memory (the first call on a device looks the array up
 * and reserves the host bookkeeping once).
 *  params     as for msm_setup; max_atoms and max_systems are ignored.
 *             At most MSM_NOALLOC_MAX_LEVELS grids.
 *  stream     hipStream_t the work is enqueued on (NULL: the null stream).
 *  xyzq_dev, energy_dev (1 double), forces_dev, potentials_dev: as for
 *             msm_energy_forces with one system; outputs may be NULL.
 *  status_dev NULL or one int32 that receives, when the work has run,
 *             MSM_OK, MSM_ERR_DOMAIN or MSM_ERR_NONFINITE (msm_get_status's
 *             codes for this evaluation).
 * Returns MSM_ERR_CAPACITY when the system's work arrays and tables do not
 * fit the array (a 99,999-atom water box at h = 0.25 nm fits in both
 * precisions), MSM_ERR_ARG/UNSUPPORTED as msm_setup, MSM_ERR_HIP.
 * Results equal msm_energy_forces with the default launch configuration.
 * Every call on a device uses the same array and clears it first: calls that
 * overlap on one device (on different streams, or from different host
 * threads before the earlier work has run) race and give undefined results;
 * the host side of concurrent calls is serialised. */
#define MSM_NOALLOC_SCRATCH_MIB 64
#define MSM_NOALLOC_MAX_LEVELS 8
int msm_energy_forces_noalloc(const msm_params *params, void *stream, int64_t natoms,
                              const void *xyzq_dev, double *energy_dev, void *forces_dev,
                              void *potentials_dev, int32_t *status_dev);

/* Launch configuration of the two heaviest kernels, and of the stream use of
 * an evaluation. Every configuration is deterministic, but pair_waves and
 * stencil_threads add the same terms in different orders, so results of
 * different values agree to rounding, not bitwise (contexts that must agree
 * bitwise, e.g. a parareal pair and its serial reference, should share one
 * configuration); concurrent changes no result bit. Defaults: the cluster form (2), 1024
 * threads, concurrent, the grid cells (pair_cell 1). */
typedef struct {
    int pair_waves;        /* short-range sum: 4, 8 or 16 waves share one 64-atom group, one
                              lane per atom; 1: each wave owns 16 atoms, four lanes per atom;
                              2: each of 8 waves owns an 8-atom cluster of the group, eight
                              lanes per atom, and evaluates only the candidates within the
                              cutoff of the cluster's bounding box; 3: as 2, but each of 4 waves
                              takes two clusters and lays out one candidate stream for both
                              (same terms in the same order as 2, so the same bits); 5 and 6:
                              as 2 with 16-atom clusters, four lanes per atom (5), or 32-atom
                              clusters, two lanes per atom (6); 7 and 9: as 2, but the 8
                              clusters of a 64-atom group (7; one workgroup of 8 waves) or the
                              4 of half a group (9) share one candidate stream, built and
                              loaded once by the workgroup (same terms in the same order as
                              2, so the same bits); 10 (single precision only, not for
                              msm_energy_forces_noalloc): as 2, but each pair inside the
                              cutoff is evaluated once (Newton's third law, Section 3's
                              short-range sum) and the candidate's share is added to 64-bit
                              fixed-point accumulators (unit 2^-32 of the force bracket and
                              potential, |share| < 2^31 per block of candidates); setting it
                              allocates those accumulators (32 bytes per atom of max_atoms).
                              Integer sums are exact, so this form too gives the same bits
                              in every run, but other bits than 2 */
    int stencil_threads;   /* threads per lattice-cutoff tile: 256 or 1024 */
    int concurrent;        /* 1: the short-range sum runs on a second stream of the context,
                              concurrently with the grid stages (forked after binning,
                              joined before interpolation; HIP graphs capture both branches);
                              2: as 1, but forked after anterpolation, which first runs
                              alone (its LDS-heavy tiles are not starved by the pair
                              workgroups; better for large systems);
                              0: every stage on the context stream in turn. Stage timing
                              always runs the stages in turn. */
    int pair_cell;         /* cells of the short-range pair search: 1, the cells of edge h
                              that anterpolation walks; 2 or 3, cells of edge h/2 or h/3,
                              into which the atoms are binned a second time (for a coarse
                              h, whose cells hold many atoms outside the cutoff of a
                              cluster). Setting 2 or 3 allocates those cells' arrays
                              (MSM_ERR_CAPACITY beyond 2^31 cells; MSM_ERR_UNSUPPORTED for
                              msm_energy_forces_noalloc) */
} msm_tuning;

int msm_get_tuning(const msm_ctx *ctx, msm_tuning *out);
int msm_set_tuning(msm_ctx *ctx, const msm_tuning *tuning);

/* Autotuner: time whole evaluations (launched eagerly; with concurrent stages
 * on, for both fork points 1 and 2) for every pair_waves (10 in single
 * precision only) and stencil_threads candidate,
 * reps evaluations each, on the caller's own batch (arguments as for
 * msm_energy_forces; no outputs are written), then the chosen ones with
 * pair_cell 2 and 3; keep the fastest and report it in *chosen (may be
 * NULL). Synchronous; may allocate the pair cells' arrays. */
int msm_autotune(msm_ctx *ctx, int nsys, const int64_t *offsets_host, const double *domains_host,
                 const void *xyzq_dev, int reps, msm_tuning *chosen);

/* Replay captured HIP graphs for evaluations (enable != 0) or launch every
 * kernel eagerly (0, the default). With graphs on, the first evaluation of a
 * batch shape and set of buffers is captured and later ones with the same
 * plan and pointers replay it (a new shape or pointer captures again; up to
 * four captures are kept per context). Results are identical either way;
 * stage timing always runs eagerly. */
int msm_set_graphs(msm_ctx *ctx, int enable);

/* Synchronise the stream, return and clear the device status word:
 * MSM_OK, or the first applicable of the conditions seen since the last
 * call: MSM_ERR_DOMAIN (an atom left its domain; what follows from it is not
 * reported separately), MSM_ERR_NONFINITE (a non-finite position or charge,
 * or a constraint iteration that met a non-finite value and stopped there),
 * MSM_ERR_CONSTRAINT; or MSM_ERR_HIP. */
int msm_get_status(msm_ctx *ctx);

/* Text for a status code. */
const char *msm_status_string(int code);

/* Grid geometry of one system (context domain when domain_host is NULL):
 * returns the number of grids and fills, per level k < 16, the first node
 * index org[3k..3k+2] and node counts dim[3k..3k+2]. Level k node (i, j, l)
 * sits at lo + 2^k h (i, j, l). */
int msm_grid_shape(const msm_ctx *ctx, const double *domain_host, int *org, int *dim);

/* Copy intermediate results of the last msm_energy_forces call for system
 * `sys` into caller device buffers (any may be NULL), converted to double:
 * u_short (N_s), f_short (N_s x 3, the bracket of the short-range force
 * before the factor k q_i; with a molecular model bound, with the excluded
 * pairs taken out and without Lennard-Jones), per-level grids q^k and u^k (prolongated; the
 * lattice-cutoff part for `ucut`) in x-fastest order of msm_grid_shape.
 * Grid pointers are arrays of `levels` device pointers in host memory.
 * Atom arrays are in the caller's order. u_short is zero when that call asked
 * for neither energy nor potentials. For tests. */
int msm_debug_stages(msm_ctx *ctx, int sys, double *u_short_dev, double *f_short_dev,
                     double *const *q_grid_dev, double *const *ucut_grid_dev,
                     double *const *u_grid_dev);

/* ---- Dynamics (Section 2: move particles under F = -dU/dr) ----
 * The paper names bonded, van der Waals and Coulomb terms but gives no force
 * field. The model here: Coulomb by this library's MSM with the pairs inside
 * one molecule excluded, Lennard-Jones between atoms of different molecules
 * (Lorentz-Berthelot mixing, cut and shifted to zero at the cutoff a), and
 * optionally rigid three-site molecules held by RATTLE (Andersen 1983). */
typedef struct {
    int64_t period;              /* entries of the per-atom arrays; batch atom i uses
                                    entry i % period (period = atoms of one system) */
    const int32_t *molid_dev;    /* period molecule ids, or NULL (no exclusions); the atoms of a
                                    molecule lie within one system and closer than a, at most
                                    1024 atoms per molecule (MSM_ERR_ARG otherwise) */
    const double *lj_dev;        /* period x 2 (sigma nm, epsilon kJ/mol), or NULL */
    int rigid_triples;           /* 1: atoms 3m, 3m+1, 3m+2 of every system are rigid; system
                                    offsets must then be multiples of 3 */
    double tri_len[3];           /* distances 0-1, 0-2, 1-2 of each rigid triple (nm) */
    double constraint_tol;       /* relative tolerance of the constraints (0: 1e-10), in FP64:
                                    RATTLE's position stage takes Newton steps on a triple's
                                    three bond conditions until each is within it, the velocity
                                    stage solves its three linear conditions directly, and a
                                    triple already within it is left unchanged by both */
} msm_md_model;

/* Copy a molecular model into the context and allocate the dynamics
 * workspace (forces, propagator state and parareal arrays for max_atoms
 * atoms). Must precede msm_vv_run and parareal_run; a later call replaces the
 * model. With a model bound, msm_energy_forces also applies it: the pair sum
 * runs as without a model, a per-atom pass takes each molecule's excluded
 * pairs out of it, and Lennard-Jones runs over the atoms with epsilon > 0
 * only. */
int msm_md_bind(msm_ctx *ctx, const msm_md_model *model);

/* nsteps velocity-Verlet steps of dt ps (Section 2), in place, on nsys
 * systems (offsets and domains as for msm_energy_forces):
 *  xyzq_dev  N x 4 doubles: positions and charges;
 *  vel_dev   N x 4 doubles: velocities (nm/ps) and inverse masses (1/amu).
 * The integrator state and the constraints are FP64 in both precisions; an
 * FP32 context evaluates the forces from an FP32 copy of the positions.
 * Each step: half kick, drift, RATTLE positions, forces, half kick, RATTLE
 * velocities; forces are evaluated nsteps + 1 times. epot_dev / ekin_dev
 * (nsys doubles, may be NULL) receive the potential and kinetic energy at the
 * end. Domain exits are reported through msm_get_status. */
int msm_vv_run(msm_ctx *ctx, int nsys, const int64_t *offsets_host, const double *domains_host, void *xyzq_dev,
               void *vel_dev, int nsteps, double dt, double *epot_dev, double *ekin_dev);

/* Multiple time steps (Section 5 names them as an improvement): nouter steps
 * of dt ps of impulse multiple-time-step velocity Verlet (r-RESPA), in place,
 * arguments as for msm_vv_run. The force splits into a fast part, the
 * short-range pairs (with the excluded pairs' smooth correction and the
 * model's Lennard-Jones), and a slow part, the grid (long-range) part with the
 * smooth self term. Each outer step: half kick with the slow force, ninner
 * velocity-Verlet steps of dt/ninner with the fast force (RATTLE positions
 * and velocities), the slow force at the new positions, half kick with it
 * (then RATTLE velocities). The grid part is evaluated nouter + 1 times, the
 * pairs nouter * ninner + 1 times; epot_dev gets a full evaluation at the
 * end. MSM contexts only (MSM_ERR_UNSUPPORTED for the cutoff methods). */
int msm_vv_mts_run(msm_ctx *ctx, int nsys, const int64_t *offsets_host, const double *domains_host,
                   void *xyzq_dev, void *vel_dev, int nouter, int ninner, double dt, double *epot_dev,
                   double *ekin_dev);

typedef struct {
    int nslices;        /* time slices N (window of the iteration) */
    int kmax;           /* at most this many iterations (iterations == nslices is exact) */
    double tol;         /* stop when no position changed by more than tol (nm) */
    int steps_f;        /* fine propagator: steps_f velocity-Verlet steps of dt_f (fine context) */
    double dt_f;
    int steps_g;        /* coarse propagator: steps_g steps of dt_g (coarse context) */
    double dt_g;
} parareal_params;

typedef struct {
    int iterations;         /* iterations done */
    int converged;          /* 1 when the tolerance was met or every slice is exact */
    double residual[64];    /* largest position change of iteration k (first 64) */
    double seconds;         /* wall time of the call, including the final synchronisation */
} parareal_report;

/* Parareal (Section 4) for one system of natoms atoms in the domain of both
 * contexts:
 *   lambda^0_{n+1} = G(lambda^0_n), then for k = 0, 1, ...:
 *   lambda^{k+1}_{n+1} = F(lambda^k_n) + (G(lambda^{k+1}_n) - G(lambda^k_n)),
 * with F and G velocity Verlet on the fine and coarse context. The fine
 * propagator of all slices that are not yet exact runs as one batch of
 * systems; the coarse sweep is serial. The correction and the iterates are
 * FP64. When both contexts hold rigid triples, each corrected state is
 * projected back onto the constraints (positions along their own bond
 * vectors, then velocities, with the fine model's tolerance); states that
 * satisfy them already, as every propagator output does, are unchanged.
 * After k iterations slices 0..k equal the serial fine trajectory bitwise.
 *  charges_dev, invmass_dev  natoms doubles;
 *  state0_dev                natoms x 6 (x y z vx vy vz);
 *  lambda_dev                (nslices+1) x natoms x 6, out: every slice.
 * The fine context needs max_atoms >= nslices*natoms and max_systems >=
 * nslices, the coarse one natoms and 1; both need a bound model and the
 * same stream. Returns MSM_OK when converged, MSM_NOT_CONVERGED after kmax
 * iterations, or an error (MSM_ERR_DOMAIN/NONFINITE if a state left the
 * domain). Synchronises once per iteration to read the residual. */
int parareal_run(msm_ctx *fine, msm_ctx *coarse, const parareal_params *params, int64_t natoms,
                 const double *charges_dev, const double *invmass_dev, const double *state0_dev,
                 double *lambda_dev, parareal_report *report);

typedef struct {
    int nslices;        /* slices of the whole run */
    int width;          /* slices iterated at once: the computational window */
    int max_iters;      /* return after this many iterations of this call (0: run to the end) */
    int pipeline;       /* 0: one fine batch over the window before each coarse sweep;
                           1: fine batches start as soon as the sweep has produced their
                           states, overlapping the sweep (fine and coarse contexts on
                           different streams) */
    int chunk;          /* pipelined mode: slices per fine batch (0: width/4 rounded up) */
    double tol;         /* accept a state whose positions moved by less than tol (nm);
                           0 accepts exact states only */
    int steps_f;        /* fine propagator: steps_f velocity-Verlet steps of dt_f (fine context) */
    double dt_f;
    int steps_g;        /* coarse propagator: steps_g steps of dt_g (coarse context) */
    double dt_g;
} parareal_window_params;

/* Resumable state of a sliding-window run, kept by the caller between calls.
 * All zeros starts a new run. Together with lambda and the coarse ring it is
 * a checkpoint: copying the three away and back and calling again continues
 * the run bitwise as if it had not stopped. */
typedef struct {
    int start;              /* lambda_0 .. lambda_start are final */
    int window_valid;       /* 1: the window's states and the ring hold iterates;
                               0: the window is predicted by the coarse propagator
                               from lambda_start (a restart from the window edge) */
    int iterations;         /* iterations so far, over all calls */
    int last_accepted;      /* states accepted by the last iteration */
    int64_t fine_slices;    /* fine-propagator slice runs so far (pipelined runs count
                               the speculative ones too) */
    int64_t coarse_slices;  /* coarse-propagator slice runs so far */
    double last_change;     /* largest position change of the last iteration (nm) */
    double seconds;         /* wall time over all calls */
} parareal_window_state;

/* Parareal with a sliding computational window (Section 4: converged early
 * time points let the window move on along the time axis). The states
 * lambda_{start+1} .. lambda_{start+We}, We = min(width, nslices - start),
 * are iterated with the update of parareal_run while lambda_0 .. lambda_start
 * are final. After each iteration the first open state is exact (its fine run
 * started from a final state), and each further leading state whose
 * positions moved by less than tol is accepted; the window moves past the
 * accepted states and the states entering it get the coarse prediction.
 * With tol = 0 the result is the serial fine trajectory bitwise; with width
 * = nslices and tol = 0, k iterations leave every state equal to
 * parareal_run's after k iterations.
 *  charges_dev, invmass_dev  natoms doubles;
 *  lambda_dev   (nslices+1) x natoms x 6 (x y z vx vy vz): lambda_0 in, every state out;
 *  ring_dev     width x natoms x 6: G(lambda_s) of the window's slice s at slot s % width;
 *  state        host, in and out.
 * The fine context needs max_atoms >= width*natoms and max_systems >= width,
 * the coarse one natoms and 1; both need a bound model on the same device.
 * Their streams may differ (the pipelined mode overlaps only then); the call
 * orders its work across them with events and returns with both idle.
 * Returns MSM_OK when every slice is final, MSM_NOT_CONVERGED when it stopped
 * after max_iters iterations (call again to resume), or an error
 * (MSM_ERR_DOMAIN/NONFINITE if a state left the domain; the buffers are then
 * no valid checkpoint). Synchronises once per iteration to read the changes. */
int parareal_window_run(msm_ctx *fine, msm_ctx *coarse, const parareal_window_params *params, int64_t natoms,
                        const double *charges_dev, const double *invmass_dev, double *lambda_dev, double *ring_dev,
                        parareal_window_state *state);

/* Stages of one evaluation, for msm_stage_timing. */
enum {
    MSM_STAGE_BIN = 0,       /* counting sort of atoms into cells */
    MSM_STAGE_SHORT = 1,     /* short-range pair sum */
    MSM_STAGE_ANTERP = 2,    /* anterpolation to the finest grid */
    MSM_STAGE_RESTRICT = 3,  /* restriction, all levels */
    MSM_STAGE_CUTOFF = 4,    /* lattice cutoff stencils, all levels below the top */
    MSM_STAGE_TOP = 5,       /* top-level all-pairs sum */
    MSM_STAGE_PROLONG = 6,   /* prolongation, all levels */
    MSM_STAGE_INTERP = 7,    /* interpolation, combination and energy reduction */
    MSM_NSTAGES = 8
};

/* Benchmark instrumentation: while enabled, every evaluation records HIP
 * events on the context stream around each stage and waits for the last one
 * before returning (so enabled calls are synchronous). msm_stage_timing
 * returns the summed milliseconds per stage (MSM_NSTAGES doubles) and the
 * number of evaluations since the last reset; reset != 0 clears them. */
int msm_enable_stage_timing(msm_ctx *ctx, int enable);
int msm_stage_timing(msm_ctx *ctx, double *ms_out, int64_t *evaluations, int reset);

#ifdef __cplusplus
}
#endif
#endif
