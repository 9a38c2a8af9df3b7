// Launchers of the dynamics kernels (velocity Verlet with RATTLE, parareal state handling).
#pragma once

#include "launch.h"

namespace msmx {

// Rigid triples: atoms 3m, 3m+1, 3m+2 at distances len[0] (0-1), len[1] (0-2), len[2] (1-2).
struct TriModel {
    double len[3];
    double tol;        // relative tolerance on the squared bond length / bond velocity
    int max_iter;
};

template <typename T> struct MdLaunch {
    static hipError_t kick_drift(hipStream_t s, int64_t n, vec4_t<T> *x, vec4_t<T> *v, const T *f, double dt,
                                 const TriModel *tm);
    static hipError_t kick(hipStream_t s, int64_t n, const vec4_t<T> *x, vec4_t<T> *v, const T *f, double dt,
                           const TriModel *tm);
    static hipError_t kinetic(hipStream_t s, const DevPlan &p, const vec4_t<T> *v, double *parts, double *ekin);
    static hipError_t state_in(hipStream_t s, int64_t natoms, int64_t count, const double *lam, const double *q,
                               const double *invm, vec4_t<T> *x, vec4_t<T> *v);
    static hipError_t state_out(hipStream_t s, int64_t count, const vec4_t<T> *x, const vec4_t<T> *v, double *out);
};

// Per-system sums of the per-block partials of the plan's interpolation
// blocks, times `scale`, into out[nsys].
hipError_t reduce_blocks(hipStream_t s, const DevPlan &p, const double *parts, double *out, double scale);
hipError_t parareal_correct(hipStream_t s, int64_t count6, double *lam, const double *fout, const double *gnew,
                            double *gold, unsigned long long *change);
hipError_t copy_f64(hipStream_t s, const double *src, double *dst, int64_t n);
hipError_t zero_u64(hipStream_t s, unsigned long long *p);

}  // namespace msmx
