// Kernels of the dynamics built on the multilevel summation forces:
// velocity Verlet (Section 2) with RATTLE for rigid three-site molecules
// (Andersen 1983), kinetic energy, and the parareal state handling of
// Section 4 (conversion between the FP64 iterates and the propagator state,
// and the correction lambda_{n+1} = F(lambda^k_n) + (G(lambda^{k+1}_n) - G(lambda^k_n))).
//
// Propagator state (mixed precision): x = (x, y, z, q) and v = (vx, vy, vz,
// 1/m) in FP64 for both context precisions, so that positions far from the
// origin and the constraint iteration keep full resolution; the forces come
// from the evaluation in the context's precision T (N x 3), and for T = float
// an FP32 copy of x feeds that evaluation.
#include "device_util.h"
#include "md.h"

namespace msmx {

namespace {

template <typename T> struct V3 {
    T x, y, z;
};
template <typename T> __device__ inline V3<T> sub(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T> __device__ inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__constant__ int kTriA[3] = {0, 0, 1};
__constant__ int kTriB[3] = {1, 2, 2};

// Bond c of a triple: s = r_a - r_b and the squared-length residual
// diff = len^2 - |s|^2; true when |diff| is within the tolerance. One
// function for every constraint test, so that a state one stage accepted is
// accepted by every other stage too.
__device__ inline bool bond_within(const V3<double> r[3], int c, const TriModel &tm, V3<double> &s, double &diff)
{
    const double d2 = tm.len[c] * tm.len[c];
    s = sub(r[kTriA[c]], r[kTriB[c]]);
    diff = d2 - dot(s, s);
    return fabs(diff) <= 2.0 * tm.tol * d2;
}

// Outcome of a constraint iteration: 0 (every bond within the tolerance),
// kStatusNonFinite (it met a non-finite value and stopped there) or
// kStatusConstraint (max_iter sweeps without meeting the tolerance); a
// non-zero outcome is or-ed into the status word.
__device__ inline void report_constraint(const TriModel &tm, int outcome)
{
    if (outcome && tm.status) atomicOr(tm.status, outcome);
}

// RATTLE's velocity stage: velocities with no relative component along any
// bond. A triple whose bonds are all within the tolerance is left unchanged.
// Otherwise the three conditions, linear in the bond multipliers mu_c
// (v_x -= im_x sum_c mu_c sgn(c, x) r_c, r_c = r_a(c) - r_b(c), sgn +1 for
// a(c), -1 for b(c)), are solved at once: M mu = w with
// w_c = r_c . (v_a(c) - v_b(c)) and M_cd = (r_c . r_d) K_cd, K the inverse-mass
// coupling of the bonds (symmetric), by Cramer's rule. This is the point the
// iteration of the velocity stage converges to, reached to rounding.
__device__ inline int constrain_velocities(const V3<double> r[3], V3<double> vel[3], const double im[3],
                                           const TriModel &tm)
{
    V3<double> rr[3];
    double w[3];
    bool done = true;
    for (int c = 0; c < 3; c++) {
        const int a = kTriA[c], b = kTriB[c];
        rr[c] = sub(r[a], r[b]);
        w[c] = dot(rr[c], sub(vel[a], vel[b]));
        if (!isfinite(w[c])) return kStatusNonFinite;
        if (fabs(w[c]) > tm.tol * tm.len[c] * tm.len[c]) done = false;
    }
    if (done) return 0;
    // bonds 0 = (0, 1), 1 = (0, 2), 2 = (1, 2)
    const double m00 = dot(rr[0], rr[0]) * (im[0] + im[1]), m11 = dot(rr[1], rr[1]) * (im[0] + im[2]);
    const double m22 = dot(rr[2], rr[2]) * (im[1] + im[2]);
    const double m01 = dot(rr[0], rr[1]) * im[0], m02 = -dot(rr[0], rr[2]) * im[1], m12 = dot(rr[1], rr[2]) * im[2];
    const double a00 = m11 * m22 - m12 * m12, a01 = m02 * m12 - m01 * m22, a02 = m01 * m12 - m02 * m11;
    const double a11 = m00 * m22 - m02 * m02, a12 = m01 * m02 - m00 * m12, a22 = m00 * m11 - m01 * m01;
    const double idet = 1.0 / (m00 * a00 + m01 * a01 + m02 * a02);
    const double mu0 = (a00 * w[0] + a01 * w[1] + a02 * w[2]) * idet;
    const double mu1 = (a01 * w[0] + a11 * w[1] + a12 * w[2]) * idet;
    const double mu2 = (a02 * w[0] + a12 * w[1] + a22 * w[2]) * idet;
    if (!isfinite(mu0) || !isfinite(mu1) || !isfinite(mu2)) return kStatusNonFinite;
    const double k0 = im[0], k1 = im[1], k2 = im[2];
    vel[0] = {vel[0].x - k0 * (mu0 * rr[0].x + mu1 * rr[1].x), vel[0].y - k0 * (mu0 * rr[0].y + mu1 * rr[1].y),
              vel[0].z - k0 * (mu0 * rr[0].z + mu1 * rr[1].z)};
    vel[1] = {vel[1].x - k1 * (mu2 * rr[2].x - mu0 * rr[0].x), vel[1].y - k1 * (mu2 * rr[2].y - mu0 * rr[0].y),
              vel[1].z - k1 * (mu2 * rr[2].z - mu0 * rr[0].z)};
    vel[2] = {vel[2].x + k2 * (mu1 * rr[1].x + mu2 * rr[2].x), vel[2].y + k2 * (mu1 * rr[1].y + mu2 * rr[2].y),
              vel[2].z + k2 * (mu1 * rr[1].z + mu2 * rr[2].z)};
    return 0;
}

// Half kick and drift of one atom (no constraints). The state is FP64; the
// forces come in the evaluation precision T; `xe` (may be null) receives the
// new positions and charges in T for the next force evaluation.
template <typename T>
__global__ void k_kick_drift(int64_t n, double4 *__restrict__ x, double4 *__restrict__ v, const T *__restrict__ f,
                             double dt, vec4_t<T> *__restrict__ xe)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 vi = v[i], xi = x[i];
    const double h = 0.5 * dt * vi.w;
    vi.x += h * (double)f[3 * i];
    vi.y += h * (double)f[3 * i + 1];
    vi.z += h * (double)f[3 * i + 2];
    xi.x += dt * vi.x;
    xi.y += dt * vi.y;
    xi.z += dt * vi.z;
    v[i] = vi;
    x[i] = xi;
    if (xe) {
        vec4_t<T> o;
        o.x = T(xi.x);
        o.y = T(xi.y);
        o.z = T(xi.z);
        o.w = T(xi.w);
        xe[i] = o;
    }
}

// Molecules per workgroup of k_kick_rattle. A thread owns one triple (96
// bytes of positions and 96 of velocities); the workgroup moves its atoms
// between HBM and LDS as contiguous runs, so every global access is
// coalesced, and each thread reads and writes its own triple in LDS.
constexpr int kTriWg = 128;

template <typename T> struct TriLds {
    double4 x[3 * kTriWg];
    double4 v[3 * kTriWg];
    T f[9 * kTriWg];
};

// Load the workgroup's atoms (positions, velocities) and their forces.
template <typename T>
__device__ inline void tri_stage_in(TriLds<T> &L, int64_t a0, int na, const double4 *__restrict__ x,
                                    const double4 *__restrict__ v, const T *__restrict__ f)
{
    for (int k = threadIdx.x; k < na; k += kTriWg) {
        L.x[k] = x[a0 + k];
        L.v[k] = v[a0 + k];
    }
    for (int k = threadIdx.x; k < 3 * na; k += kTriWg) L.f[k] = f[3 * a0 + k];
    __syncthreads();
}

// Half kick, drift, then RATTLE's position stage for one rigid triple: the
// drifted atoms are moved along the old bond vectors ro_d, atom x by
// im_x sum_d lambda_d sgn(d, x) ro_d, until every bond has its length, and
// the same displacement over dt is added to the velocities. The multipliers
// come from Newton's method on the three conditions |s_c|^2 = len_c^2 (the
// Jacobian is J_cd = 2 K_cd (s_c . ro_d) with K the inverse-mass coupling of
// the bonds), solved by Cramer's rule: three or four steps to the tolerance,
// where a sweep bond by bond (the same solution) takes several dozen.
template <typename T>
__global__ void k_kick_drift_rattle(int64_t ntri, double4 *__restrict__ x, double4 *__restrict__ v,
                                    const T *__restrict__ f, double dt, TriModel tm, vec4_t<T> *__restrict__ xe)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntri) return;
    V3<double> r[3], vel[3], ro[3];
    double im[3], q[3];
    for (int a = 0; a < 3; a++) {
        const int64_t i = 3 * t + a;
        const double4 xs = x[i];
        const double4 vi = v[i];
        q[a] = xs.w;
        im[a] = vi.w;
        const double h = 0.5 * dt * vi.w;
        vel[a] = {vi.x + h * (double)f[3 * i], vi.y + h * (double)f[3 * i + 1], vi.z + h * (double)f[3 * i + 2]};
        r[a] = {xs.x, xs.y, xs.z};
    }
    for (int c = 0; c < 3; c++) ro[c] = sub(r[kTriA[c]], r[kTriB[c]]);
    for (int a = 0; a < 3; a++) r[a] = {r[a].x + dt * vel[a].x, r[a].y + dt * vel[a].y, r[a].z + dt * vel[a].z};
    // bonds 0 = (0, 1), 1 = (0, 2), 2 = (1, 2)
    const double k00 = im[0] + im[1], k11 = im[0] + im[2], k22 = im[1] + im[2];
    const double k01 = im[0], k02 = -im[1], k12 = im[2];
    const double inv_dt = 1.0 / dt;
    int outcome = kStatusConstraint;
    for (int it = 0; it < tm.max_iter; it++) {
        V3<double> sb[3];
        double d[3];
        bool done = true;
        for (int c = 0; c < 3; c++)
            if (!bond_within(r, c, tm, sb[c], d[c])) done = false;
        if (done) {
            outcome = 0;
            break;
        }
        const double j00 = 2.0 * k00 * dot(sb[0], ro[0]), j01 = 2.0 * k01 * dot(sb[0], ro[1]);
        const double j02 = 2.0 * k02 * dot(sb[0], ro[2]), j10 = 2.0 * k01 * dot(sb[1], ro[0]);
        const double j11 = 2.0 * k11 * dot(sb[1], ro[1]), j12 = 2.0 * k12 * dot(sb[1], ro[2]);
        const double j20 = 2.0 * k02 * dot(sb[2], ro[0]), j21 = 2.0 * k12 * dot(sb[2], ro[1]);
        const double j22 = 2.0 * k22 * dot(sb[2], ro[2]);
        const double c00 = j11 * j22 - j12 * j21, c01 = j12 * j20 - j10 * j22, c02 = j10 * j21 - j11 * j20;
        const double c10 = j02 * j21 - j01 * j22, c11 = j00 * j22 - j02 * j20, c12 = j01 * j20 - j00 * j21;
        const double c20 = j01 * j12 - j02 * j11, c21 = j02 * j10 - j00 * j12, c22 = j00 * j11 - j01 * j10;
        const double idet = 1.0 / (j00 * c00 + j01 * c01 + j02 * c02);
        const double l0 = (c00 * d[0] + c10 * d[1] + c20 * d[2]) * idet;
        const double l1 = (c01 * d[0] + c11 * d[1] + c21 * d[2]) * idet;
        const double l2 = (c02 * d[0] + c12 * d[1] + c22 * d[2]) * idet;
        if (!isfinite(l0) || !isfinite(l1) || !isfinite(l2)) {
            outcome = kStatusNonFinite;
            break;
        }
        const V3<double> dr[3] = {
            {im[0] * (l0 * ro[0].x + l1 * ro[1].x), im[0] * (l0 * ro[0].y + l1 * ro[1].y),
             im[0] * (l0 * ro[0].z + l1 * ro[1].z)},
            {im[1] * (l2 * ro[2].x - l0 * ro[0].x), im[1] * (l2 * ro[2].y - l0 * ro[0].y),
             im[1] * (l2 * ro[2].z - l0 * ro[0].z)},
            {-im[2] * (l1 * ro[1].x + l2 * ro[2].x), -im[2] * (l1 * ro[1].y + l2 * ro[2].y),
             -im[2] * (l1 * ro[1].z + l2 * ro[2].z)}};
        for (int a = 0; a < 3; a++) {
            r[a] = {r[a].x + dr[a].x, r[a].y + dr[a].y, r[a].z + dr[a].z};
            vel[a] = {vel[a].x + inv_dt * dr[a].x, vel[a].y + inv_dt * dr[a].y, vel[a].z + inv_dt * dr[a].z};
        }
    }
    report_constraint(tm, outcome);
    for (int a = 0; a < 3; a++) {
        const int64_t i = 3 * t + a;
        x[i] = make_double4(r[a].x, r[a].y, r[a].z, q[a]);
        v[i] = make_double4(vel[a].x, vel[a].y, vel[a].z, im[a]);
        if (xe) {
            vec4_t<T> o;
            o.x = T(r[a].x);
            o.y = T(r[a].y);
            o.z = T(r[a].z);
            o.w = T(q[a]);
            xe[i] = o;
        }
    }
}

template <typename T>
__global__ void k_kick(int64_t n, double4 *__restrict__ v, const T *__restrict__ f, double dt)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 vi = v[i];
    const double h = 0.5 * dt * vi.w;
    vi.x += h * (double)f[3 * i];
    vi.y += h * (double)f[3 * i + 1];
    vi.z += h * (double)f[3 * i + 2];
    v[i] = vi;
}

// Second half kick, then RATTLE's velocity stage.
template <typename T>
__global__ __launch_bounds__(kTriWg) void k_kick_rattle(int64_t ntri, const double4 *__restrict__ x,
                                                        double4 *__restrict__ v, const T *__restrict__ f, double dt,
                                                        TriModel tm)
{
    __shared__ TriLds<T> L;
    const int64_t t0 = blockIdx.x * (int64_t)kTriWg, a0 = 3 * t0;
    const int na = 3 * (int)min((int64_t)kTriWg, ntri - t0);
    tri_stage_in(L, a0, na, x, v, f);
    const int tl = threadIdx.x;
    if (3 * tl < na) {
        V3<double> r[3], vel[3];
        double im[3];
        for (int a = 0; a < 3; a++) {
            const int i = 3 * tl + a;
            const double4 xi = L.x[i], vi = L.v[i];
            im[a] = vi.w;
            const double h = 0.5 * dt * vi.w;
            vel[a] = {vi.x + h * (double)L.f[3 * i], vi.y + h * (double)L.f[3 * i + 1],
                      vi.z + h * (double)L.f[3 * i + 2]};
            r[a] = {xi.x, xi.y, xi.z};
        }
        report_constraint(tm, constrain_velocities(r, vel, im, tm));
        for (int a = 0; a < 3; a++) L.v[3 * tl + a] = make_double4(vel[a].x, vel[a].y, vel[a].z, im[a]);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < na; k += kTriWg) v[a0 + k] = L.v[k];
}

// Positions and charges in the evaluation precision.
template <typename T>
__global__ void k_to_eval(int64_t n, const double4 *__restrict__ x, vec4_t<T> *__restrict__ xe)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 xi = x[i];
    vec4_t<T> o;
    o.x = T(xi.x);
    o.y = T(xi.y);
    o.z = T(xi.z);
    o.w = T(xi.w);
    xe[i] = o;
}

// Kinetic energy 1/2 sum m v^2 per interpolation-sized block of each system.
__global__ __launch_bounds__(256) void k_kinetic(DevPlan p, const double4 *__restrict__ v, double *__restrict__ parts)
{
    __shared__ double wpart[256 / 64];
    const int64_t blk = blockIdx.x;
    const int s = find_segment(p.iblk_prefix, p.nsys, blk);
    const SysPlan &P = p.sys[s];
    const int64_t i = P.atom0 + (blk - p.iblk_prefix[s]) * 256 + threadIdx.x;
    double e = 0;
    if (i < P.atom0 + P.natoms) {
        const double4 vi = v[i];
        e = 0.5 * (vi.x * vi.x + vi.y * vi.y + vi.z * vi.z) / vi.w;
    }
    e = block_sum<256>(e, wpart);
    if (threadIdx.x == 0) parts[blk] = e;
}

// Propagator state of consecutive slices from the FP64 iterates:
// lambda (slice-major, n x 6 per slice) -> x (positions, charge), v (velocity, 1/m).
__global__ void k_state_in(int64_t natoms, int64_t count, const double *__restrict__ lam, const double *__restrict__ q,
                           const double *__restrict__ invm, double4 *__restrict__ x, double4 *__restrict__ v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t a = i % natoms;
    const double *l = lam + 6 * i;
    x[i] = make_double4(l[0], l[1], l[2], q[a]);
    v[i] = make_double4(l[3], l[4], l[5], invm[a]);
}

__global__ void k_state_out(int64_t count, const double4 *__restrict__ x, const double4 *__restrict__ v,
                            double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double4 xi = x[i], vi = v[i];
    double *o = out + 6 * i;
    o[0] = xi.x;
    o[1] = xi.y;
    o[2] = xi.z;
    o[3] = vi.x;
    o[4] = vi.y;
    o[5] = vi.z;
}

// Parareal correction (Section 4), in FP64:
// lambda_{n+1} = F(lambda^k_n) + (G(lambda^{k+1}_n) - G(lambda^k_n)); the old
// coarse value is replaced by the new one, and the largest position change is
// folded into *change (max of non-negative doubles, order-independent).
__global__ __launch_bounds__(256) void k_correct(int64_t count6, double *__restrict__ lam,
                                                 const double *__restrict__ fout, const double *__restrict__ gnew,
                                                 double *__restrict__ gold, unsigned long long *__restrict__ change)
{
    __shared__ double wpart[256 / 64];
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double c = 0;
    if (e < count6) {
        const double g = gnew[e];
        const double nv = fout[e] + (g - gold[e]);
        if (e % 6 < 3) c = fabs(nv - lam[e]);
        if (!(c == c)) c = __longlong_as_double(0x7ff0000000000000LL);   // NaN -> +inf
        lam[e] = nv;
        gold[e] = g;
    }
    c = block_max<256>(c, wpart);
    if (threadIdx.x == 0) atomicMax(change, (unsigned long long)__double_as_longlong(c));
}

// The same correction for rigid triples (a reading: Section 4 is silent on
// constraints). A linear combination of three constrained states is not
// constrained, and molecules bent by it can stop the next propagator's
// constraint iteration from converging, so the corrected state of each triple
// is projected back: positions along their own bond vectors until every bond
// has its length, then velocities by RATTLE's velocity stage. A state that
// already satisfies the constraints (any propagator output, so every slice
// that is already exact) passes both tests unchanged.
__global__ __launch_bounds__(256) void k_correct_rigid(int64_t ntri, double *__restrict__ lam,
                                                       const double *__restrict__ fout,
                                                       const double *__restrict__ gnew, double *__restrict__ gold,
                                                       const double *__restrict__ invm, TriModel tm,
                                                       unsigned long long *__restrict__ change)
{
    __shared__ double wpart[256 / 64];
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double ch = 0;
    if (t < ntri) {
        V3<double> r[3], vel[3];
        double im[3];
        for (int a = 0; a < 3; a++) {
            const int64_t e = 6 * (3 * t + a);
            double nv[6];
            for (int c = 0; c < 6; c++) {
                const double g = gnew[e + c];
                nv[c] = fout[e + c] + (g - gold[e + c]);
                gold[e + c] = g;
            }
            r[a] = {nv[0], nv[1], nv[2]};
            vel[a] = {nv[3], nv[4], nv[5]};
            im[a] = invm[3 * t + a];
        }
        int outcome = kStatusConstraint;
        for (int it = 0; it < tm.max_iter && outcome == kStatusConstraint; it++) {
            bool done = true;
            for (int c = 0; c < 3; c++) {
                const int a = kTriA[c], b = kTriB[c];
                V3<double> s;
                double diff;
                if (bond_within(r, c, tm, s, diff)) continue;
                done = false;
                const double g = diff / (2.0 * dot(s, s) * (im[a] + im[b]));
                if (!isfinite(g)) {
                    outcome = kStatusNonFinite;
                    break;
                }
                const double ga = g * im[a], gb = g * im[b];
                r[a] = {r[a].x + ga * s.x, r[a].y + ga * s.y, r[a].z + ga * s.z};
                r[b] = {r[b].x - gb * s.x, r[b].y - gb * s.y, r[b].z - gb * s.z};
            }
            if (done && outcome == kStatusConstraint) outcome = 0;
        }
        report_constraint(tm, outcome);
        if (!outcome) report_constraint(tm, constrain_velocities(r, vel, im, tm));
        for (int a = 0; a < 3; a++) {
            double *l = lam + 6 * (3 * t + a);
            const double rv[3] = {r[a].x, r[a].y, r[a].z}, vv[3] = {vel[a].x, vel[a].y, vel[a].z};
            for (int c = 0; c < 3; c++) {
                double d = fabs(rv[c] - l[c]);
                if (!(d == d)) d = __longlong_as_double(0x7ff0000000000000LL);   // NaN -> +inf
                ch = fmax(ch, d);
                l[c] = rv[c];
                l[3 + c] = vv[c];
            }
        }
    }
    ch = block_max<256>(ch, wpart);
    if (threadIdx.x == 0) atomicMax(change, (unsigned long long)__double_as_longlong(ch));
}

__global__ void k_copy_f64(int64_t n, const double *__restrict__ src, double *__restrict__ dst)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_zero_u64(int n, unsigned long long *p)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

template <typename T>
hipError_t MdLaunch<T>::kick_drift(hipStream_t s, int64_t n, double4 *x, double4 *v, const T *f, double dt,
                                   const TriModel *tm, vec4_t<T> *xe)
{
    if (n == 0) return hipSuccess;
    if (tm)
        hipLaunchKernelGGL(k_kick_drift_rattle<T>, dim3(nblocks(n / 3, 128)), dim3(128), 0, s, n / 3, x, v, f, dt, *tm,
                           xe);
    else
        hipLaunchKernelGGL(k_kick_drift<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, n, x, v, f, dt, xe);
    return hipGetLastError();
}

template <typename T>
hipError_t MdLaunch<T>::kick(hipStream_t s, int64_t n, const double4 *x, double4 *v, const T *f, double dt,
                             const TriModel *tm)
{
    if (n == 0) return hipSuccess;
    if (tm)
        hipLaunchKernelGGL(k_kick_rattle<T>, dim3(nblocks(n / 3, kTriWg)), dim3(kTriWg), 0, s, n / 3, x, v, f, dt,
                           *tm);
    else
        hipLaunchKernelGGL(k_kick<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, n, v, f, dt);
    return hipGetLastError();
}

template <typename T> hipError_t MdLaunch<T>::to_eval(hipStream_t s, int64_t n, const double4 *x, vec4_t<T> *xe)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_eval<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, n, x, xe);
    return hipGetLastError();
}

hipError_t md_kinetic(hipStream_t s, const DevPlan &p, const double4 *v, double *parts, double *ekin)
{
    if (p.niblk > 0) hipLaunchKernelGGL(k_kinetic, dim3((unsigned)p.niblk), dim3(256), 0, s, p, v, parts);
    return reduce_blocks(s, p, parts, ekin, 1.0);
}

hipError_t md_state_in(hipStream_t s, int64_t natoms, int64_t count, const double *lam, const double *q,
                       const double *invm, double4 *x, double4 *v)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_state_in, dim3(nblocks(count, 256)), dim3(256), 0, s, natoms, count, lam, q, invm, x, v);
    return hipGetLastError();
}

hipError_t md_state_out(hipStream_t s, int64_t count, const double4 *x, const double4 *v, double *out)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_state_out, dim3(nblocks(count, 256)), dim3(256), 0, s, count, x, v, out);
    return hipGetLastError();
}

hipError_t parareal_correct(hipStream_t s, int64_t count6, double *lam, const double *fout, const double *gnew,
                            double *gold, unsigned long long *change)
{
    if (count6 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_correct, dim3(nblocks(count6, 256)), dim3(256), 0, s, count6, lam, fout, gnew, gold, change);
    return hipGetLastError();
}

hipError_t parareal_correct_rigid(hipStream_t s, int64_t natoms, double *lam, const double *fout, const double *gnew,
                                  double *gold, const double *invm, const TriModel &tm, unsigned long long *change)
{
    const int64_t ntri = natoms / 3;
    if (ntri == 0) return hipSuccess;
    hipLaunchKernelGGL(k_correct_rigid, dim3(nblocks(ntri, 256)), dim3(256), 0, s, ntri, lam, fout, gnew, gold, invm,
                       tm, change);
    return hipGetLastError();
}

hipError_t copy_f64(hipStream_t s, const double *src, double *dst, int64_t n)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f64, dim3(nblocks(n, 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t zero_u64(hipStream_t s, unsigned long long *p, int n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, n, p);
    return hipGetLastError();
}

template struct MdLaunch<float>;
template struct MdLaunch<double>;

}  // namespace msmx
