// Launchers of the dynamics kernels (velocity Verlet with RATTLE, parareal state handling).
#pragma once

#include "launch.h"

namespace msmx {

// Largest molecule of a bound model (its excluded pairs are listed per atom).
constexpr int kMaxMoleculeAtoms = 1024;

// Rigid triples: atoms 3m, 3m+1, 3m+2 at distances len[0] (0-1), len[1] (0-2), len[2] (1-2).
struct TriModel {
    double len[3];
    double tol;        // relative tolerance on the squared bond length / bond velocity
    int max_iter;
    int *status;       // the context's status word: kStatusConstraint when an iteration
                       // stops at max_iter, kStatusNonFinite when it meets a non-finite value
};

// T is the precision of the forces (the context's); the state is FP64.
template <typename T> struct MdLaunch {
    static hipError_t kick_drift(hipStream_t s, int64_t n, double4 *x, double4 *v, const T *f, double dt,
                                 const TriModel *tm, vec4_t<T> *xe);
    static hipError_t kick(hipStream_t s, int64_t n, const double4 *x, double4 *v, const T *f, double dt,
                           const TriModel *tm);
    static hipError_t to_eval(hipStream_t s, int64_t n, const double4 *x, vec4_t<T> *xe);
};

hipError_t md_kinetic(hipStream_t s, const DevPlan &p, const double4 *v, double *parts, double *ekin);
hipError_t md_state_in(hipStream_t s, int64_t natoms, int64_t count, const double *lam, const double *q,
                       const double *invm, double4 *x, double4 *v);
hipError_t md_state_out(hipStream_t s, int64_t count, const double4 *x, const double4 *v, double *out);

// Per-system sums of the per-block partials of the plan's interpolation
// blocks, times `scale`, into out[nsys].
hipError_t reduce_blocks(hipStream_t s, const DevPlan &p, const double *parts, double *out, double scale);
hipError_t parareal_correct(hipStream_t s, int64_t count6, double *lam, const double *fout, const double *gnew,
                            double *gold, unsigned long long *change);
// The correction for rigid triples (natoms a multiple of 3), followed by the
// projection of each corrected triple back onto its constraints.
hipError_t parareal_correct_rigid(hipStream_t s, int64_t natoms, double *lam, const double *fout, const double *gnew,
                                  double *gold, const double *invm, const TriModel &tm, unsigned long long *change);
hipError_t copy_f64(hipStream_t s, const double *src, double *dst, int64_t n);
// Clear n words (a fill kernel, so it may sit in a captured graph).
hipError_t zero_u64(hipStream_t s, unsigned long long *p, int n = 1);

}  // namespace msmx
