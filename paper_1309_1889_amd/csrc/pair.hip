// The short-range pair kernel of the multilevel summation method (Section 3),
// also the whole pair sum of the simple cutoff method and of Wolf summation
// (Section 5), templated on the arithmetic type T (float or double).
#include <cmath>

#include "device_util.h"
#include "launch.h"

namespace msmx {

namespace {

// ---------------------------------------------------------------------------
// Short-range part (Section 3): u_i^short = sum_{j != i, r < a} g*(r_ij) q_j with
// g*(r) = 1/r - gamma(r/a)/a, and the force bracket
// b_i = sum_j q_j (-dg*/dr / r)(r_i - r_j) = sum_j q_j (1/r^3 - (5/2 - 3/2 rho^2)/a^3)(r_i - r_j),
// so that F_i^short = k q_i b_i.
//
// A workgroup owns 64 consecutive sorted atoms (a compact group, one per
// lane of each of its waves). Its waves walk the cell rows that intersect the
// group's bounding box grown by a, each row clipped to the chord the cutoff
// sphere leaves it, and read the candidate j atoms by broadcast: each lane
// tests its own pair. Every pair is evaluated from both sides, so no atomics
// are needed and the summation order is fixed. With a zero smoothing
// polynomial the same kernel sums Coulomb's law below the cutoff, which is
// the simple cutoff method.
// ---------------------------------------------------------------------------
template <typename T> struct PairK {
    T a2;               // a^2
    T reach;            // a plus a rounding margin, for the row search
    T inv_a2;           // 1/a^2
    T c0, c1, c2, c3;   // gamma(r/a)/a = c0 + c1 r^2 + c2 r^4 (+ c3 r^6 for m = 3)
    T d0, d1, d2;       // -(d/dr)(gamma(r/a)/a) / r = d0 + d1 r^2 (+ d2 r^4 for m = 3)
    T alpha, alpha2;    // Wolf damping alpha and alpha^2
    T wshift, wexp;     // erfc(alpha a)/a and 2 alpha / sqrt(pi)
    const float4 *wtab; // single precision: the Wolf table (kWolfPieces pieces of E and D)
    float wscale;       // kWolfPieces / a
    T ke;               // Coulomb constant (dynamics forms: forces leave in final units)
    // kLJ1: s^2, 4 eps, 24 eps, 48 eps and the energy at r = a, 4 eps ((s/a)^12 - (s/a)^6)
    T lj_s2, lj_e4, lj_e24, lj_e48, lj_shift;
};

// Wolf summation in single precision: E(r) = erfc(alpha r) and the force
// numerator D(r) = E(r) + (2 alpha r / sqrt(pi)) exp(-alpha^2 r^2) from the
// cubic pieces staged in LDS, so that
// erfc(alpha r)/r - erfc(alpha a)/a = E rinv - wshift and
// -(d/dr)(erfc(alpha r)/r) / r = D rinv^3.
__device__ inline void wolf_lookup(const float4 *__restrict__ tab, float r, float scale, float &E, float &D)
{
    const float x = r * scale;
    const int k = min((int)x, kWolfPieces - 1);
    const float u = x - float(k);
    const float4 ce = tab[2 * k], cd = tab[2 * k + 1];
    E = ce.x + u * (ce.y + u * (ce.z + u * ce.w));
    D = cd.x + u * (cd.y + u * (cd.z + u * cd.w));
}

// The table of a workgroup in LDS (all threads take part; one barrier).
template <typename T, int KIND> struct WolfLds {
    float4 t[1];
    __device__ void load(const PairK<T> &) {}
    __device__ const float4 *ptr() const { return nullptr; }
};
template <> struct WolfLds<float, 2> {
    float4 t[2 * kWolfPieces];
    __device__ void load(const PairK<float> &k)
    {
        for (int e = threadIdx.x; e < 2 * kWolfPieces; e += blockDim.x) t[e] = k.wtab[e];
        __syncthreads();
    }
    __device__ const float4 *ptr() const { return t; }
};

// Pair kernel forms: the smoothing polynomial of degree at most 4 (MSM with
// m <= 2, and the simple cutoff method with a zero polynomial), of degree 6
// (m = 3), Wolf's damped, shifted Coulomb (Section 5), and the dynamics
// model's Lennard-Jones term, which runs over the atoms that carry one: in
// general (kLJ, per-atom parameters and molecules read from the aux records)
// or for a model with one Lennard-Jones type and at most one such atom per
// molecule (kLJ1, the parameters constant, no record read).
enum PairKind { kPoly = 0, kPolyHigh = 1, kWolf = 2, kLJ = 3, kLJ1 = 4 };

#ifndef MSMX_PAIR_UNROLL
#define MSMX_PAIR_UNROLL 8
#endif
constexpr int kPairUnroll = MSMX_PAIR_UNROLL;   // staged candidates read per step

// Half-width of the chord a row of cells leaves inside the cutoff sphere
// around a box. The search reach carries a relative margin of 1e-5, far above
// the error of the hardware square root, so the chord still covers every
// candidate within the cutoff (a candidate it might lose lies beyond a and
// contributes nothing).
__device__ inline float chord_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double chord_sqrt(double x) { return sqrt(x); }

// molecule id stored in the first component of an aux record
__device__ inline int mol_of(const float4 &v) { return __float_as_int(v.x); }
__device__ inline int mol_of(const double4 &v) { return (int)__double_as_longlong(v.x); }

// the three used components of an aux record (molecule id, s/2, sqrt(eps))
// read from LDS, the fourth known to be zero, so no register holds it
template <typename T> __device__ inline vec4_t<T> aux3(const vec4_t<T> &r)
{
    vec4_t<T> v;
    v.x = r.x;
    v.y = r.y;
    v.z = r.z;
    v.w = T(0);
    return v;
}

// Per-wave LDS: the flattened candidate stream of the wave's 64 current work
// items and the staged chunk of 64 candidate atoms.
template <typename T, bool MD> struct PairLds {
    int pre[kWave + 1];                // start of each item's atoms in the stream
    int first[kWave];                  // first atom of each item
    vec4_t<T> atom[kWave];             // staged candidates
    vec4_t<T> aux[MD ? kWave : 1];
};

// POT = false: forces only (no potential or energy sums), for evaluations
// that are asked for neither. KIND: one of PairKind. MD: the candidates carry
// aux records (molecule id bits, s/2, sqrt(eps), 0), which the Lennard-Jones
// kind reads: 4 eps ((s/r)^12 - (s/r)^6), shifted to zero at r = a, between
// atoms of different molecules, with s = s_i/2 + s_j/2 and
// eps = sqrt(eps_i) sqrt(eps_j); u then sums the pair energies of atom i.
// The one-type kind kLJ1 takes s and eps from the constants; with at most
// one Lennard-Jones atom per molecule the only pair inside a molecule is an
// atom with itself, which r^2 > 0 leaves out.
template <typename T, bool MD, bool POT, int KIND>
__device__ inline void pair_term(const vec4_t<T> &ai, const vec4_t<T> &xi, const vec4_t<T> &aj, const vec4_t<T> &xj,
                                 const PairK<T> &k, T &fx, T &fy, T &fz, T &u, const float4 *wtab = nullptr)
{
    const T dx = ai.x - aj.x, dy = ai.y - aj.y, dz = ai.z - aj.z;
    const T r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < k.a2 && r2 > T(0)) {
        T t;
        if constexpr (KIND == kLJ1) {
            const T ir2 = rcp_t(r2);
            const T sr2 = k.lj_s2 * ir2, sr6 = sr2 * sr2 * sr2;
            if (POT) u += k.lj_e4 * (sr6 * sr6 - sr6) - k.lj_shift;
            t = sr6 * (k.lj_e48 * sr6 - k.lj_e24) * ir2;
        } else if constexpr (KIND == kLJ) {
            const T rinv = rsqrt_t(r2);
            static_assert(MD, "the Lennard-Jones kind reads the aux records");
            const T eps = mol_of(xi) == mol_of(xj) ? T(0) : xi.z * xj.z;
            const T sg = xi.y + xj.y;
            const T s2 = sg * sg, ir2 = rinv * rinv;
            const T sr2 = s2 * ir2, sr6 = sr2 * sr2 * sr2;
            if (POT) {
                const T sc2 = s2 * k.inv_a2, sc6 = sc2 * sc2 * sc2;
                u += T(4) * eps * ((sr6 * sr6 - sr6) - (sc6 * sc6 - sc6));
            }
            t = T(24) * eps * (T(2) * sr6 * sr6 - sr6) * ir2;
        } else {
            const T rinv = rsqrt_t(r2);
            T br;
            if (KIND == kWolf && sizeof(T) == 4) {
                // single precision: the tabulated E and D
                const T r = r2 * rinv;
                float E, D;
                wolf_lookup(wtab, float(r), k.wscale, E, D);
                br = T(D) * rinv * rinv * rinv;
                if (POT) u += aj.w * (T(E) * rinv - k.wshift);
            } else if (KIND == kWolf) {
                // erfc(alpha r)/r - erfc(alpha a)/a, and -(d/dr)(erfc(alpha r)/r)/r
                // = (erfc(alpha r)/r + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)) / r^2
                const T r = r2 * rinv;
                const T er = erfc(k.alpha * r);
                br = (er * rinv + k.wexp * exp(-k.alpha2 * r2)) * rinv * rinv;
                if (POT) u += aj.w * (er * rinv - k.wshift);
            } else if (KIND == kPolyHigh) {
                br = rinv * rinv * rinv - (k.d0 + r2 * (k.d1 + r2 * k.d2));
                if (POT) u += aj.w * (rinv - (k.c0 + r2 * (k.c1 + r2 * (k.c2 + r2 * k.c3))));
            } else {
                br = rinv * rinv * rinv - (k.d0 + k.d1 * r2);
                if (POT) u += aj.w * (rinv - (k.c0 + r2 * (k.c1 + r2 * k.c2)));
            }
            t = aj.w * br;
        }
        fx += t * dx;
        fy += t * dy;
        fz += t * dz;
    }
}

// Work layout: a workgroup of kPairWaves waves owns one group of 64
// consecutive sorted atoms (one per lane). The work items are the pieces of
// cell rows (cy, cz) inside one brick column that can reach the group's
// bounding box; each is clipped to the chord the cutoff sphere leaves its
// row and is one contiguous run of sorted atoms. Items are dealt round-robin
// to the waves. A wave lays 64 items at a time out as one stream of
// candidate atoms, stages the stream 64 atoms at a time in LDS with one
// coalesced load (the next chunk is fetched while the current one is used),
// and every lane reads each staged atom by broadcast and evaluates its own
// pair. The waves' partial sums are added in a fixed order at the end.
template <typename T, bool MD, bool POT, int KIND, int kPairWaves>
__global__ __launch_bounds__(kPairWaves * kWave) void k_pair(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                              const int *__restrict__ cstart,
                                                              vec4_t<T> *__restrict__ out, PairK<T> k,
                                                              const vec4_t<T> *__restrict__ saux)
{
    __shared__ PairLds<T, MD> lds[kPairWaves];
    __shared__ vec4_t<T> red[kPairWaves][kWave];
    __shared__ WolfLds<T, KIND> wl;
    if (eval_failed(p)) return;
    wl.load(k);
    const float4 *wtab = wl.ptr();
    const int64_t g = blockIdx.x;
    const int s = find_segment(p.group_prefix, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int64_t first = P.atom0 + (g - p.group_prefix[s]) * kWave;
    const int64_t end = P.atom0 + P.natoms;
    const int lane = threadIdx.x % kWave;
    const int wv = uni((int)(threadIdx.x / kWave));
    PairLds<T, MD> &L = lds[wv];
    const int64_t i = first + lane;
    const bool valid = i < end;
    const vec4_t<T> ai = sx[valid ? i : first];
    vec4_t<T> xi;
    if (MD) xi = saux[valid ? i : first];

    const T bminx = uni(wave_min(ai.x)), bmaxx = uni(wave_max(ai.x));
    const T bminy = uni(wave_min(ai.y)), bmaxy = uni(wave_max(ai.y));
    const T bminz = uni(wave_min(ai.z)), bmaxz = uni(wave_max(ai.z));
    const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]);
    const T inv_h = T(P.inv_h), h = T(1.0 / P.inv_h);
    const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
    const T reach = k.reach, reach2 = k.reach * k.reach;
    const int cy0 = clampi((int)floor((bminy - loy - reach) * inv_h), 0, ncy - 1);
    const int cy1 = clampi((int)floor((bmaxy - loy + reach) * inv_h), 0, ncy - 1);
    const int cz0 = clampi((int)floor((bminz - loz - reach) * inv_h), 0, ncz - 1);
    const int cz1 = clampi((int)floor((bmaxz - loz + reach) * inv_h), 0, ncz - 1);
    const int bx0 = clampi((int)floor((bminx - lox - reach) * inv_h), 0, ncx - 1) / kBrick;
    const int bx1 = clampi((int)floor((bmaxx - lox + reach) * inv_h), 0, ncx - 1) / kBrick;
    const int nbx = bx1 - bx0 + 1, ny = cy1 - cy0 + 1;
    const int nitems = nbx * ny * (cz1 - cz0 + 1);

    // The polynomial addends that meet a scalar multiplier in the Horner
    // chains are kept in vector registers: an FMA takes one scalar operand,
    // so as kernel arguments they would be copied to vector registers again
    // for every candidate.
    if (KIND == kPolyHigh)
        asm volatile("" : "+v"(k.c2), "+v"(k.d1));
    else if (KIND == kPoly)
        asm volatile("" : "+v"(k.c1), "+v"(k.d0));
    T fx = 0, fy = 0, fz = 0, u = 0;
    // items wv, wv + W, wv + 2W, ..., 64 per batch
    for (int ib = wv; ib < nitems; ib += kPairWaves * kWave) {
        const int q = ib + kPairWaves * lane;            // this lane's item
        int len = 0, jb = 0;
        if (q < nitems) {
            const int bx = bx0 + q % nbx, row = q / nbx;
            const int cy = cy0 + row % ny, cz = cz0 + row / ny;
            const T z0 = loz + T(cz) * h, y0 = loy + T(cy) * h;
            const T dz = fmax(T(0), fmax(z0 - bmaxz, bminz - (z0 + h)));
            const T dy = fmax(T(0), fmax(y0 - bmaxy, bminy - (y0 + h)));
            const T rem = reach2 - dy * dy - dz * dz;
            if (rem > T(0)) {
                const T wdt = chord_sqrt(rem);
                const int cx0 = clampi((int)floor((bminx - lox - wdt) * inv_h), 0, ncx - 1);
                const int cx1 = clampi((int)floor((bmaxx - lox + wdt) * inv_h), 0, ncx - 1);
                const int ca = max(cx0, bx * kBrick), cb = min(cx1, bx * kBrick + kBrick - 1);
                if (ca <= cb) {
                    const int r0 = (int)P.cell0 + cell_rank32(P, ca, cy, cz);
                    jb = cstart[r0];
                    len = cstart[r0 + (cb - ca) + 1] - jb;
                }
            }
        }
        // exclusive prefix of the item lengths across the wave
        const int incl = wave_incl_scan(len);
        L.pre[lane] = incl - len;
        L.first[lane] = jb;
        const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
        if (lane == 0) L.pre[kWave] = total;
        // the wave's own LDS writes are seen by its later reads (one wave, in
        // order); the barrier only keeps the compiler from moving them
        __builtin_amdgcn_wave_barrier();
        // stream position -> sorted atom index
        auto locate = [&](int pos) -> int {
            int lo_ = 0, hi_ = kWave;       // pre[lo_] <= pos < pre[hi_]
            while (hi_ - lo_ > 1) {
                const int mid = (lo_ + hi_) >> 1;
                if (L.pre[mid] <= pos) lo_ = mid; else hi_ = mid;
            }
            return L.first[lo_] + (pos - L.pre[lo_]);
        };
        vec4_t<T> pa, px;
        if (lane < total) {
            const int j = locate(lane);
            pa = sx[j];
            if (MD) px = saux[j];
        }
        for (int c0 = 0; c0 < total; c0 += kWave) {
            __builtin_amdgcn_wave_barrier();
            L.atom[lane] = pa;
            if (MD) L.aux[lane] = px;
            __builtin_amdgcn_wave_barrier();
            const int nxt = c0 + kWave + lane;
            if (nxt < total) {
                const int j = locate(nxt);
                pa = sx[j];
                if (MD) px = saux[j];
            }
            const int cnt = uni(min(kWave, total - c0));
            int t = 0;
            // unrolled so that several broadcast reads are in flight at once
            for (; t + kPairUnroll <= cnt; t += kPairUnroll) {
                vec4_t<T> aj[kPairUnroll], xj[kPairUnroll];
#pragma unroll
                for (int v = 0; v < kPairUnroll; ++v) {
                    aj[v] = L.atom[t + v];
                    xj[v] = MD ? aux3<T>(L.aux[t + v]) : aj[v];
                }
#pragma unroll
                for (int v = 0; v < kPairUnroll; ++v)
                    pair_term<T, MD, POT, KIND>(ai, xi, aj[v], xj[v], k, fx, fy, fz, u, wtab);
            }
            for (; t < cnt; ++t) {
                const vec4_t<T> aj = L.atom[t];
                const vec4_t<T> xj = MD ? aux3<T>(L.aux[t]) : aj;
                pair_term<T, MD, POT, KIND>(ai, xi, aj, xj, k, fx, fy, fz, u, wtab);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    vec4_t<T> o;
    o.x = fx;
    o.y = fy;
    o.z = fz;
    o.w = u;
    red[wv][lane] = o;
    __syncthreads();
    if (wv == 0 && valid) {
        vec4_t<T> acc = red[0][lane];
        for (int w = 1; w < kPairWaves; ++w) {   // fixed order: deterministic
            const vec4_t<T> v = red[w][lane];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        out[i] = acc;
    }
}

// Sub-group form (pair_waves = 1): each wave of a 4-wave workgroup owns 16
// of the group's 64 atoms, four lanes per atom. The candidate region of 16
// atoms is smaller than that of 64 (about 0.7 times the candidates per atom
// at the default water density), and the lanes of one atom read four
// consecutive candidates of the stream at a time, so a wave still evaluates
// 64 pairs per step. The four partial sums of an atom are added across its
// lanes in a fixed order; the waves share nothing, so there is no barrier.
constexpr int kSub = 16;                 // atoms per wave
constexpr int kSubLanes = kWave / kSub;  // lanes per atom
constexpr int kSubUnroll = 4;            // steps of kSubLanes candidates read at once

template <typename T> __device__ inline T sum_lanes(T v)
{
    v += __shfl_xor(v, kSub, kWave);
    v += __shfl_xor(v, 2 * kSub, kWave);
    return v;
}

template <typename T, bool MD, bool POT, int KIND>
__global__ __launch_bounds__(kSubLanes * kWave) void k_pair_sub(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                                const int *__restrict__ cstart,
                                                                vec4_t<T> *__restrict__ out, PairK<T> k,
                                                                const vec4_t<T> *__restrict__ saux)
{
    __shared__ PairLds<T, MD> lds[kWave / kSub];
    __shared__ WolfLds<T, KIND> wl;
    if (eval_failed(p)) return;
    wl.load(k);
    const float4 *wtab = wl.ptr();
    const int64_t g = blockIdx.x;
    const int s = find_segment(p.group_prefix, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int lane = threadIdx.x % kWave;
    const int wv = uni((int)(threadIdx.x / kWave));
    PairLds<T, MD> &L = lds[wv];
    const int64_t first = P.atom0 + (g - p.group_prefix[s]) * kWave + wv * kSub;
    const int64_t end = P.atom0 + P.natoms;
    if (first >= end) return;   // the whole wave: no atoms in this sub-group
    const int me = lane % kSub, slot = lane / kSub;   // the lane's atom and candidate slot
    const int64_t i = first + me;
    const bool valid = i < end;
    const vec4_t<T> ai = sx[valid ? i : first];
    vec4_t<T> xi;
    if (MD) xi = saux[valid ? i : first];

    const T bminx = uni(wave_min(ai.x)), bmaxx = uni(wave_max(ai.x));
    const T bminy = uni(wave_min(ai.y)), bmaxy = uni(wave_max(ai.y));
    const T bminz = uni(wave_min(ai.z)), bmaxz = uni(wave_max(ai.z));
    const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]);
    const T inv_h = T(P.inv_h), h = T(1.0 / P.inv_h);
    const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
    const T reach = k.reach, reach2 = k.reach * k.reach;
    const int cy0 = clampi((int)floor((bminy - loy - reach) * inv_h), 0, ncy - 1);
    const int cy1 = clampi((int)floor((bmaxy - loy + reach) * inv_h), 0, ncy - 1);
    const int cz0 = clampi((int)floor((bminz - loz - reach) * inv_h), 0, ncz - 1);
    const int cz1 = clampi((int)floor((bmaxz - loz + reach) * inv_h), 0, ncz - 1);
    const int bx0 = clampi((int)floor((bminx - lox - reach) * inv_h), 0, ncx - 1) / kBrick;
    const int bx1 = clampi((int)floor((bmaxx - lox + reach) * inv_h), 0, ncx - 1) / kBrick;
    const int nbx = bx1 - bx0 + 1, ny = cy1 - cy0 + 1;
    const int nitems = nbx * ny * (cz1 - cz0 + 1);

    if (KIND == kPolyHigh)
        asm volatile("" : "+v"(k.c2), "+v"(k.d1));
    else if (KIND == kPoly)
        asm volatile("" : "+v"(k.c1), "+v"(k.d0));
    T fx = 0, fy = 0, fz = 0, u = 0;
    for (int ib = 0; ib < nitems; ib += kWave) {
        const int q = ib + lane;   // this lane's item
        int len = 0, jb = 0;
        if (q < nitems) {
            const int bx = bx0 + q % nbx, row = q / nbx;
            const int cy = cy0 + row % ny, cz = cz0 + row / ny;
            const T z0 = loz + T(cz) * h, y0 = loy + T(cy) * h;
            const T dz = fmax(T(0), fmax(z0 - bmaxz, bminz - (z0 + h)));
            const T dy = fmax(T(0), fmax(y0 - bmaxy, bminy - (y0 + h)));
            const T rem = reach2 - dy * dy - dz * dz;
            if (rem > T(0)) {
                const T wdt = chord_sqrt(rem);
                const int cx0 = clampi((int)floor((bminx - lox - wdt) * inv_h), 0, ncx - 1);
                const int cx1 = clampi((int)floor((bmaxx - lox + wdt) * inv_h), 0, ncx - 1);
                const int ca = max(cx0, bx * kBrick), cb = min(cx1, bx * kBrick + kBrick - 1);
                if (ca <= cb) {
                    const int r0 = (int)P.cell0 + cell_rank32(P, ca, cy, cz);
                    jb = cstart[r0];
                    len = cstart[r0 + (cb - ca) + 1] - jb;
                }
            }
        }
        const int incl = wave_incl_scan(len);
        L.pre[lane] = incl - len;
        L.first[lane] = jb;
        const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
        if (lane == 0) L.pre[kWave] = total;
        __builtin_amdgcn_wave_barrier();
        auto locate = [&](int pos) -> int {
            int lo_ = 0, hi_ = kWave;
            while (hi_ - lo_ > 1) {
                const int mid = (lo_ + hi_) >> 1;
                if (L.pre[mid] <= pos) lo_ = mid; else hi_ = mid;
            }
            return L.first[lo_] + (pos - L.pre[lo_]);
        };
        vec4_t<T> pa, px;
        if (lane < total) {
            const int j = locate(lane);
            pa = sx[j];
            if (MD) px = saux[j];
        }
        for (int c0 = 0; c0 < total; c0 += kWave) {
            __builtin_amdgcn_wave_barrier();
            L.atom[lane] = pa;
            if (MD) L.aux[lane] = px;
            __builtin_amdgcn_wave_barrier();
            const int nxt = c0 + kWave + lane;
            if (nxt < total) {
                const int j = locate(nxt);
                pa = sx[j];
                if (MD) px = saux[j];
            }
            const int cnt = uni(min(kWave, total - c0));
            int t = 0;
            constexpr int step = kSubLanes * kSubUnroll;
            for (; t + step <= cnt; t += step) {
                vec4_t<T> aj[kSubUnroll], xj[kSubUnroll];
#pragma unroll
                for (int v = 0; v < kSubUnroll; ++v) {
                    aj[v] = L.atom[t + kSubLanes * v + slot];
                    xj[v] = MD ? aux3<T>(L.aux[t + kSubLanes * v + slot]) : aj[v];
                }
#pragma unroll
                for (int v = 0; v < kSubUnroll; ++v)
                    pair_term<T, MD, POT, KIND>(ai, xi, aj[v], xj[v], k, fx, fy, fz, u, wtab);
            }
            for (; t < cnt; t += kSubLanes) {
                const int tj = t + slot;
                if (tj < cnt) {
                    const vec4_t<T> aj = L.atom[tj];
                    const vec4_t<T> xj = MD ? aux3<T>(L.aux[tj]) : aj;
                    pair_term<T, MD, POT, KIND>(ai, xi, aj, xj, k, fx, fy, fz, u, wtab);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    fx = sum_lanes(fx);
    fy = sum_lanes(fy);
    fz = sum_lanes(fz);
    if (POT) u = sum_lanes(u);
    if (slot == 0 && valid) {
        vec4_t<T> o;
        o.x = fx;
        o.y = fy;
        o.z = fz;
        o.w = u;
        out[i] = o;
    }
}

// Cluster form (pair_waves = 2, 3, 5, 6), in two kernels, for clusters of
// CA = 8, 16 or 32 atoms.
//
// k_clusters: one wave per 64-atom group splits the group into 64 / CA
// clusters of CA atoms by median cuts (k-d order: halve along the longest
// extent of the group, then of each half, and so on), which gives compact
// boxes whatever the group's shape, and writes the cluster order.
//
// k_pair_cl: one wave per cluster, 64 / CA lanes per atom (lane = CA slot +
// atom). The wave lays out the cell-row pieces that can reach its cluster's
// box (each clipped to the chord the cutoff sphere leaves its row) as one
// stream, 64 pieces at a time, with a table in LDS from stream position to
// atom; it loads the stream 64 candidates at a time (the next chunk is in
// flight while the current one is used), keeps those whose distance to the
// box is below the cutoff (a ballot and a prefix count give each its place in
// a ring in LDS), and evaluates the ring 64 / CA candidates per step, one per
// slot, whenever it holds four steps' worth. With 8-atom clusters more than
// half of the evaluated lane pairs are inside the cutoff, against a fifth in
// the forms above; larger clusters keep more candidates per box but share the
// cost of building the stream among more atoms. The waves share nothing. The
// partial sums of an atom are added across its lanes in a fixed order.
constexpr int kClUnroll = 4;                   // steps per evaluated block
#ifndef MSMX_CL_UNROLL_MD
#define MSMX_CL_UNROLL_MD 4
#endif
// steps per evaluated block of the dynamics forms (their pair term holds more registers)
template <bool MD> constexpr int cl_unroll() { return MD ? MSMX_CL_UNROLL_MD : kClUnroll; }
constexpr int kClRing = 128;                   // ring capacity (a multiple of kBlock, power of two)
constexpr int kClMap = 512;                    // stream positions with a table entry
constexpr int kClWgWaves = 4;                  // waves per workgroup (independent)
#ifndef MSMX_CL_PREFETCH
#define MSMX_CL_PREFETCH 1
#endif
constexpr int kClPrefetch = MSMX_CL_PREFETCH;  // stream chunks in flight ahead of the one in use

template <int CA, typename T> __device__ inline T sum_slots(T v)
{
#pragma unroll
    for (int off = CA; off < kWave; off <<= 1) v += xor_lane(v, off);
    return v;
}

// min / max over aligned segments of n lanes
template <typename T> __device__ inline T seg_min(T v, int n)
{
#pragma unroll
    for (int off = 1; off < n; off <<= 1) v = fmin(v, xor_lane(v, off));
    return v;
}
template <typename T> __device__ inline T seg_max(T v, int n)
{
#pragma unroll
    for (int off = 1; off < n; off <<= 1) v = fmax(v, xor_lane(v, off));
    return v;
}

// One median cut of every aligned segment of n lanes: lane l holds group
// position pos; each segment is sorted ascending (bitonic network) by the
// coordinate along its longest extent, ties by position. Positions at or
// beyond natoms are absent atoms and sort last.
template <typename T>
__device__ inline int kd_cut(const vec4_t<T> *grp, int pos, int natoms, int n, int lane)
{
    const vec4_t<T> a = grp[pos];
    const bool real = pos < natoms;
    const T inf = T(1e30);
    const T ex = seg_max(real ? a.x : -inf, n) - seg_min(real ? a.x : inf, n);
    const T ey = seg_max(real ? a.y : -inf, n) - seg_min(real ? a.y : inf, n);
    const T ez = seg_max(real ? a.z : -inf, n) - seg_min(real ? a.z : inf, n);
    const int axis = (ex >= ey && ex >= ez) ? 0 : (ey >= ez ? 1 : 2);
    T key = real ? (axis == 0 ? a.x : (axis == 1 ? a.y : a.z)) : inf;
    int p = pos;
#pragma unroll
    for (int kk = 2; kk <= n; kk <<= 1)
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            const T ok = xor_lane(key, j);
            const int op = xor_lane(p, j);
            const bool up = kk == n || (lane & kk) == 0;   // every segment ascending
            const bool lower = (lane & j) == 0;
            const bool less = ok < key || (ok == key && op < p);   // the partner comes first
            if (less == (lower == up)) {
                key = ok;
                p = op;
            }
        }
    return p;
}

template <typename T, int CA>
__global__ __launch_bounds__(kWave) void k_clusters(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                    int *__restrict__ cluster)
{
    __shared__ vec4_t<T> grp[kWave];
    if (eval_failed(p)) return;
    const int64_t g = blockIdx.x;
    const int s = find_segment(p.group_prefix, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int64_t first = P.atom0 + (g - p.group_prefix[s]) * kWave;
    const int natoms = (int)min((int64_t)kWave, P.atom0 + P.natoms - first);
    const int lane = threadIdx.x;
    grp[lane] = sx[first + min(lane, natoms - 1)];
    __syncthreads();
    int pos = lane;
#pragma unroll
    for (int n = kWave; n > CA; n >>= 1) pos = kd_cut<T>(grp, pos, natoms, n, lane);
    cluster[g * kWave + lane] = pos < natoms ? (int)(first + pos) : -1;
}

template <typename T, bool MD, int NSUB> struct ClLds {
    vec4_t<T> ring[kClWgWaves][NSUB][kClRing];
    vec4_t<T> raux[MD ? kClWgWaves : 1][NSUB][MD ? kClRing : 1];
    int map[kClWgWaves][kClMap];        // stream position -> sorted atom
    int pre[kClWgWaves][kWave + 1];     // item stream offsets (positions beyond the table)
    int first[kClWgWaves][kWave];       // first atom of each item
};

// NSUB = 2: a wave takes the two clusters of one 16-atom k-d half-quarter,
// lays out one candidate stream for their common box and keeps each
// candidate for each cluster whose box is within the cutoff (a ring per
// cluster): the stream's cost is shared, and each cluster's evaluations stay
// those of its own box.
template <typename T, bool MD, bool POT, int KIND, int NSUB, int CA>
__global__ __launch_bounds__(kClWgWaves * kWave) void k_pair_cl(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                                const int *__restrict__ cstart,
                                                                const int *__restrict__ cluster,
                                                                vec4_t<T> *__restrict__ out, PairK<T> k,
                                                                const vec4_t<T> *__restrict__ saux)
{
    constexpr int kSlots = kWave / CA;          // candidates per step
    constexpr int kU = cl_unroll<MD>(), kBlock = kSlots * kU;  // candidates per evaluated block
    __shared__ ClLds<T, MD, NSUB> L;
    __shared__ WolfLds<T, KIND> wl;
    if (eval_failed(p)) return;
    wl.load(k);   // before any wave of the workgroup can leave
    const float4 *wtab = wl.ptr();
    const int lane = threadIdx.x % kWave;
    const int wv = uni((int)(threadIdx.x / kWave));
    // clusters of neighbouring groups share candidates: keep them on one XCD's L2
    const int64_t c = (xcd_remap(blockIdx.x, gridDim.x) * kClWgWaves + wv) * NSUB;   // first cluster
    if (c >= p.ngroups * (kWave / CA)) return;
    const int me = lane % CA, slot = lane / CA;
    const int m0 = uni(cluster[c * CA]);
    if (m0 < 0) return;   // clusters of absent atoms (the last group of a system)
    const int64_t g = c / (kWave / CA);
    const int s = find_segment(p.group_prefix, p.nsys, g);
    const SysPlan &P = p.sys[s];
    bool on[NSUB], valid[NSUB];
    int64_t i[NSUB];
    vec4_t<T> ai[NSUB], xi[NSUB];
    T bx_lo[NSUB], bx_hi[NSUB], by_lo[NSUB], by_hi[NSUB], bz_lo[NSUB], bz_hi[NSUB];
#pragma unroll
    for (int sc = 0; sc < NSUB; ++sc) {
        const int first = uni(cluster[(c + sc) * CA]);
        on[sc] = first >= 0;   // uniform
        const int mi = cluster[(c + sc) * CA + me];
        valid[sc] = mi >= 0;
        i[sc] = valid[sc] ? mi : (on[sc] ? first : m0);
        ai[sc] = sx[i[sc]];
        if (MD) xi[sc] = saux[i[sc]];
        bx_lo[sc] = uni(seg_min(ai[sc].x, CA)), bx_hi[sc] = uni(seg_max(ai[sc].x, CA));
        by_lo[sc] = uni(seg_min(ai[sc].y, CA)), by_hi[sc] = uni(seg_max(ai[sc].y, CA));
        bz_lo[sc] = uni(seg_min(ai[sc].z, CA)), bz_hi[sc] = uni(seg_max(ai[sc].z, CA));
    }
    // the stream covers the box of the clusters together
    T bminx = bx_lo[0], bmaxx = bx_hi[0], bminy = by_lo[0], bmaxy = by_hi[0], bminz = bz_lo[0], bmaxz = bz_hi[0];
#pragma unroll
    for (int sc = 1; sc < NSUB; ++sc)
        if (on[sc]) {
            bminx = fmin(bminx, bx_lo[sc]), bmaxx = fmax(bmaxx, bx_hi[sc]);
            bminy = fmin(bminy, by_lo[sc]), bmaxy = fmax(bmaxy, by_hi[sc]);
            bminz = fmin(bminz, bz_lo[sc]), bmaxz = fmax(bmaxz, bz_hi[sc]);
        }
    const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]);
    const T inv_h = T(P.inv_h), h = T(1.0 / P.inv_h);
    const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
    const T reach = k.reach, reach2 = k.reach * k.reach;
    const int cy0 = clampi((int)floor((bminy - loy - reach) * inv_h), 0, ncy - 1);
    const int cy1 = clampi((int)floor((bmaxy - loy + reach) * inv_h), 0, ncy - 1);
    const int cz0 = clampi((int)floor((bminz - loz - reach) * inv_h), 0, ncz - 1);
    const int cz1 = clampi((int)floor((bmaxz - loz + reach) * inv_h), 0, ncz - 1);
    const int bx0 = clampi((int)floor((bminx - lox - reach) * inv_h), 0, ncx - 1) / kBrick;
    const int bx1 = clampi((int)floor((bmaxx - lox + reach) * inv_h), 0, ncx - 1) / kBrick;
    const int nbx = bx1 - bx0 + 1, ny = cy1 - cy0 + 1;
    const int nitems = nbx * ny * (cz1 - cz0 + 1);

    if (KIND == kPolyHigh)
        asm volatile("" : "+v"(k.c2), "+v"(k.d1));
    else if (KIND == kPoly)
        asm volatile("" : "+v"(k.c1), "+v"(k.d0));
    T fx[NSUB], fy[NSUB], fz[NSUB], u[NSUB];
#pragma unroll
    for (int sc = 0; sc < NSUB; ++sc) fx[sc] = fy[sc] = fz[sc] = u[sc] = T(0);
    int *map = L.map[wv], *pre = L.pre[wv], *fst = L.first[wv];
    int head[NSUB], tail[NSUB];   // ring positions (uniform; taken modulo the capacity)
#pragma unroll
    for (int sc = 0; sc < NSUB; ++sc) head[sc] = tail[sc] = 0;
    auto eval_block = [&](int sc) {
        // a block starts at a multiple of its size, so it does not wrap
        const vec4_t<T> *ring = L.ring[wv][sc];
        const vec4_t<T> *raux = L.raux[MD ? wv : 0][MD ? sc : 0];
        const int e0 = (head[sc] & (kClRing - 1)) + slot;
        vec4_t<T> aj[kU], xj[kU];
#pragma unroll
        for (int v = 0; v < kU; ++v) {
            aj[v] = ring[e0 + kSlots * v];
            xj[v] = MD ? aux3<T>(raux[MD ? e0 + kSlots * v : 0]) : aj[v];
        }
#pragma unroll
        for (int v = 0; v < kU; ++v)
            pair_term<T, MD, POT, KIND>(ai[sc], xi[sc], aj[v], xj[v], k, fx[sc], fy[sc], fz[sc], u[sc], wtab);
        head[sc] += kBlock;
    };
    for (int ib = 0; ib < nitems; ib += kWave) {
        const int q = ib + lane;   // this lane's item
        int len = 0, jb = 0;
        if (q < nitems) {
            const int bx = bx0 + q % nbx, row = q / nbx;
            const int cy = cy0 + row % ny, cz = cz0 + row / ny;
            const T z0 = loz + T(cz) * h, y0 = loy + T(cy) * h;
            const T dz = fmax(T(0), fmax(z0 - bmaxz, bminz - (z0 + h)));
            const T dy = fmax(T(0), fmax(y0 - bmaxy, bminy - (y0 + h)));
            const T rem = reach2 - dy * dy - dz * dz;
            if (rem > T(0)) {
                const T wdt = chord_sqrt(rem);
                const int cx0 = clampi((int)floor((bminx - lox - wdt) * inv_h), 0, ncx - 1);
                const int cx1 = clampi((int)floor((bmaxx - lox + wdt) * inv_h), 0, ncx - 1);
                const int ca = max(cx0, bx * kBrick), cb = min(cx1, bx * kBrick + kBrick - 1);
                if (ca <= cb) {
                    const int r0 = (int)P.cell0 + cell_rank32(P, ca, cy, cz);
                    jb = cstart[r0];
                    len = cstart[r0 + (cb - ca) + 1] - jb;
                }
            }
        }
        const int incl = wave_incl_scan(len);
        const int start = incl - len;
        pre[lane] = start;
        fst[lane] = jb;
        const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
        if (lane == 0) pre[kWave] = total;
        // table of the first kClMap stream positions
        // (a per-lane loop: a wave-wide bound would hold cross-lane
        // addresses in registers the kernel cannot spare)
        for (int t = 0; t < len && start + t < kClMap; ++t) map[start + t] = jb + t;
        __builtin_amdgcn_wave_barrier();
        auto atom_at = [&](int pos) -> int {
            if (pos < kClMap) return map[pos];
            int lo_ = 0, hi_ = kWave;   // pre[lo_] <= pos < pre[hi_]
            while (hi_ - lo_ > 1) {
                const int mid = (lo_ + hi_) >> 1;
                if (pre[mid] <= pos) lo_ = mid; else hi_ = mid;
            }
            return fst[lo_] + (pos - pre[lo_]);
        };
        // chunks c0 + kWave * d (d < kClPrefetch) are in flight
        vec4_t<T> pa[kClPrefetch], px[kClPrefetch];
#pragma unroll
        for (int d = 0; d < kClPrefetch; ++d)
            if (kWave * d + lane < total) {
                const int j = atom_at(kWave * d + lane);
                pa[d] = sx[j];
                if (MD) px[d] = saux[j];
            }
        for (int c0 = 0; c0 < total; c0 += kWave) {
            const bool have = c0 + lane < total;
            const vec4_t<T> ca = pa[0];
            vec4_t<T> cx;
            if (MD) cx = px[0];
#pragma unroll
            for (int d = 0; d + 1 < kClPrefetch; ++d) {
                pa[d] = pa[d + 1];
                if (MD) px[d] = px[d + 1];
            }
            const int nxt = c0 + kWave * kClPrefetch + lane;   // the chunk that joins the pipeline
            if (nxt < total) {
                const int j = atom_at(nxt);
                pa[kClPrefetch - 1] = sx[j];
                if (MD) px[kClPrefetch - 1] = saux[j];
            }
#pragma unroll
            for (int sc = 0; sc < NSUB; ++sc) {
                const T ddx = fmax(T(0), fmax(bx_lo[sc] - ca.x, ca.x - bx_hi[sc]));
                const T ddy = fmax(T(0), fmax(by_lo[sc] - ca.y, ca.y - by_hi[sc]));
                const T ddz = fmax(T(0), fmax(bz_lo[sc] - ca.z, ca.z - bz_hi[sc]));
                const bool keep = on[sc] && have && ddx * ddx + ddy * ddy + ddz * ddz < reach2;
                const uint64_t m = __ballot(keep);
                if (keep) {
                    const int e = (tail[sc] + (int)__builtin_amdgcn_mbcnt_hi(
                                                  (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))) &
                                  (kClRing - 1);
                    L.ring[wv][sc][e] = ca;
                    if (MD) L.raux[MD ? wv : 0][MD ? sc : 0][MD ? e : 0] = cx;
                }
                tail[sc] += __popcll(m);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int sc = 0; sc < NSUB; ++sc)
                while (tail[sc] - head[sc] >= kBlock) eval_block(sc);
            __builtin_amdgcn_wave_barrier();
        }
    }
#pragma unroll
    for (int sc = 0; sc < NSUB; ++sc) {
        if (tail[sc] > head[sc]) {   // the last partial block, padded with a far-away atom
            if (lane < head[sc] + kBlock - tail[sc]) {
                vec4_t<T> far;
                far.x = far.y = far.z = T(1e18);
                far.w = T(0);
                L.ring[wv][sc][(tail[sc] + lane) & (kClRing - 1)] = far;
                if (MD) L.raux[MD ? wv : 0][MD ? sc : 0][MD ? (tail[sc] + lane) & (kClRing - 1) : 0] = far;
            }
            __builtin_amdgcn_wave_barrier();
            eval_block(sc);
        }
        fx[sc] = sum_slots<CA>(fx[sc]);
        fy[sc] = sum_slots<CA>(fy[sc]);
        fz[sc] = sum_slots<CA>(fz[sc]);
        if (POT) u[sc] = sum_slots<CA>(u[sc]);
        if (slot == 0 && valid[sc]) {
            vec4_t<T> o;
            o.x = fx[sc];
            o.y = fy[sc];
            o.z = fz[sc];
            o.w = u[sc];
            out[i[sc]] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// Newton's third law form (pair_waves 10, single precision): each pair inside
// the cutoff is evaluated once. The wave of an 8-atom cluster of group G
// takes from its candidate stream only the atoms sorted after G (the clusters
// of a later group would otherwise meet the pair again), and from G itself the
// atoms of its own and of later clusters in the group's k-d order (inside its
// own cluster the later ones). A lane holds one candidate j; the wave walks the
// cluster's 8 atoms i, wave-uniform, and the lane adds q_j b (r_i - r_j) and
// q_j g to its partial sums of atom i, and q_i b (r_j - r_i) and q_i g to
// those of its candidate (b: the force bracket, g: the pair potential, both
// of r_ij). After a block of 64 candidates each lane adds its candidate's sums
// to the candidate's 64-bit accumulators in fixed point (unit 2^-32): integer
// addition is associative, so the totals do not depend on the order in which
// waves reach them, and the results are the same bits in every run. The
// partial sums of the cluster's atoms are added across the lanes at the end
// (a fixed butterfly) and stored; k_n3_combine then adds each atom's
// accumulators to its stored sums and clears them for the next evaluation.
// Every term is the one the full-list forms compute for the pair, from its
// either side; only the grouping of the sums differs.
// ---------------------------------------------------------------------------
constexpr double kFixScale = 4294967296.0;   // 2^32
constexpr double kFixUnit = 1.0 / kFixScale;

__device__ inline unsigned long long to_fixed(float v)
{
    return (unsigned long long)(long long)((double)v * kFixScale);
}

__device__ inline void acc_add(unsigned long long *a, unsigned long long v)
{
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the force bracket b and (POT) the potential g of a pair at r^2 (the terms of pair_term)
template <bool POT, int KIND>
__device__ inline void pair_bg(float r2, const PairK<float> &k, const float4 *wtab, float &br, float &g)
{
    const float rinv = rsqrt_t(r2);
    if constexpr (KIND == kWolf) {
        const float r = r2 * rinv;
        float E, D;
        wolf_lookup(wtab, r, k.wscale, E, D);
        br = D * rinv * rinv * rinv;
        if (POT) g = E * rinv - k.wshift;
    } else if constexpr (KIND == kPolyHigh) {
        br = rinv * rinv * rinv - (k.d0 + r2 * (k.d1 + r2 * k.d2));
        if (POT) g = rinv - (k.c0 + r2 * (k.c1 + r2 * (k.c2 + r2 * k.c3)));
    } else {
        br = rinv * rinv * rinv - (k.d0 + k.d1 * r2);
        if (POT) g = rinv - (k.c0 + r2 * (k.c1 + r2 * k.c2));
    }
}

constexpr int kN3Cl = 8;   // atoms per cluster

// One exchange of the lane sums: of the values v[0, 2N) a lane keeps the
// lower half (bit OFF of its lane clear) or the upper half, adds its partner's
// copy of that half and leaves it in v[0, N).
template <int N, int OFF> __device__ inline void halve(float (&v)[32], int lane)
{
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        const float send = up ? v[t] : v[t + N];
        const float keep = up ? v[t + N] : v[t];
        v[t] = keep + __shfl_xor(send, OFF, kWave);
    }
}

struct N3Lds {
    float4 ring[kClWgWaves][kClRing];   // kept candidates
    int ridx[kClWgWaves][kClRing];      // their sorted indices
    int map[kClWgWaves][kClMap];        // stream position -> sorted atom
    int pre[kClWgWaves][kWave + 1];
    int first[kClWgWaves][kWave];
};

template <bool POT, int KIND>
__global__ __launch_bounds__(kClWgWaves * kWave) void k_pair_n3(DevPlan p, const float4 *__restrict__ sx,
                                                                const int *__restrict__ cstart,
                                                                const int *__restrict__ cluster,
                                                                float4 *__restrict__ out,
                                                                unsigned long long *__restrict__ acc,
                                                                int64_t stride, PairK<float> k)
{
    constexpr int CA = kN3Cl;
    __shared__ N3Lds L;
    __shared__ WolfLds<float, KIND> wl;
    if (eval_failed(p)) return;
    wl.load(k);   // before any wave of the workgroup can leave
    const float4 *wtab = wl.ptr();
    const int lane = threadIdx.x % kWave;
    const int wv = uni((int)(threadIdx.x / kWave));
    const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * kClWgWaves + wv;
    if (c >= p.ngroups * (kWave / CA)) return;
    const int m0 = uni(cluster[c * CA]);
    if (m0 < 0) return;   // a cluster of absent atoms (the last group of a system)
    const int64_t g = c / (kWave / CA);
    const int base = (int)(c % (kWave / CA)) * CA;   // the cluster's first place in the group's k-d order
    const int s = find_segment(p.group_prefix, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int gend = (int)min(P.atom0 + (g - p.group_prefix[s] + 1) * kWave, P.atom0 + P.natoms);
    const int me = lane % CA;
    const int mi = cluster[c * CA + me];
    const float4 ai = sx[mi >= 0 ? mi : m0];
    const float bx_lo = uni(seg_min(ai.x, CA)), bx_hi = uni(seg_max(ai.x, CA));
    const float by_lo = uni(seg_min(ai.y, CA)), by_hi = uni(seg_max(ai.y, CA));
    const float bz_lo = uni(seg_min(ai.z, CA)), bz_hi = uni(seg_max(ai.z, CA));
    // the cluster's atoms, wave-uniform (an absent one carries no charge)
    const float qme = mi >= 0 ? ai.w : 0.f;
    float xi[CA], yi[CA], zi[CA], qi[CA];
#pragma unroll
    for (int ia = 0; ia < CA; ++ia) {
        xi[ia] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ai.x), ia));
        yi[ia] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ai.y), ia));
        zi[ia] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ai.z), ia));
        qi[ia] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qme), ia));
    }
    float fx[CA], fy[CA], fz[CA], u[CA];
#pragma unroll
    for (int ia = 0; ia < CA; ++ia) fx[ia] = fy[ia] = fz[ia] = u[ia] = 0.f;

    // one candidate per lane (jj < 0: none); INTRA: only places after the pair's atom i
    auto eval64 = [&](const float4 aj, const int jj, const bool intra) {
        float gx = 0.f, gy = 0.f, gz = 0.f, gu = 0.f;
#pragma unroll
        for (int ia = 0; ia < CA; ++ia) {
            const float dx = xi[ia] - aj.x, dy = yi[ia] - aj.y, dz = zi[ia] - aj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            bool in = r2 < k.a2 && r2 > 0.f;
            if (intra) in = in && lane > base + ia;
            if (in) {
                float br, pg;
                pair_bg<POT, KIND>(r2, k, wtab, br, pg);
                const float ti = aj.w * br, tj = qi[ia] * br;
                fx[ia] += ti * dx;
                fy[ia] += ti * dy;
                fz[ia] += ti * dz;
                gx -= tj * dx;
                gy -= tj * dy;
                gz -= tj * dz;
                if (POT) {
                    u[ia] += aj.w * pg;
                    gu += qi[ia] * pg;
                }
            }
        }
        if (jj >= 0) {
            acc_add(acc + jj, to_fixed(gx));
            acc_add(acc + stride + jj, to_fixed(gy));
            acc_add(acc + 2 * stride + jj, to_fixed(gz));
            if (POT) acc_add(acc + 3 * stride + jj, to_fixed(gu));
        }
    };

    // pairs inside the group: the places from the cluster's own on
    {
        const int jj0 = cluster[g * kWave + lane];
        const int jj = lane > base ? jj0 : -1;
        float4 aj;
        if (jj >= 0) aj = sx[jj];
        else aj.x = aj.y = aj.z = 1e18f, aj.w = 0.f;
        eval64(aj, jj, true);
    }

    // candidates sorted after the group
    const float lox = float(P.lo[0]), loy = float(P.lo[1]), loz = float(P.lo[2]);
    const float inv_h = float(P.inv_h), h = float(1.0 / P.inv_h);
    const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
    const float reach = k.reach, reach2 = k.reach * k.reach;
    const int cy0 = clampi((int)floorf((by_lo - loy - reach) * inv_h), 0, ncy - 1);
    const int cy1 = clampi((int)floorf((by_hi - loy + reach) * inv_h), 0, ncy - 1);
    const int cz0 = clampi((int)floorf((bz_lo - loz - reach) * inv_h), 0, ncz - 1);
    const int cz1 = clampi((int)floorf((bz_hi - loz + reach) * inv_h), 0, ncz - 1);
    const int bx0 = clampi((int)floorf((bx_lo - lox - reach) * inv_h), 0, ncx - 1) / kBrick;
    const int bx1 = clampi((int)floorf((bx_hi - lox + reach) * inv_h), 0, ncx - 1) / kBrick;
    const int nbx = bx1 - bx0 + 1, ny = cy1 - cy0 + 1;
    const int nitems = nbx * ny * (cz1 - cz0 + 1);
    int *map = L.map[wv], *pre = L.pre[wv], *fst = L.first[wv];
    float4 *ring = L.ring[wv];
    int *ridx = L.ridx[wv];
    int head = 0, tail = 0;   // ring positions (uniform; taken modulo the capacity)
    auto eval_block = [&]() {
        const int e = (head + lane) & (kClRing - 1);
        eval64(ring[e], ridx[e], false);
        head += kWave;
    };
    for (int ib = 0; ib < nitems; ib += kWave) {
        const int q = ib + lane;   // this lane's item
        int len = 0, jb = 0;
        if (q < nitems) {
            const int bx = bx0 + q % nbx, row = q / nbx;
            const int cy = cy0 + row % ny, cz = cz0 + row / ny;
            const float z0 = loz + float(cz) * h, y0 = loy + float(cy) * h;
            const float dz = fmaxf(0.f, fmaxf(z0 - bz_hi, bz_lo - (z0 + h)));
            const float dy = fmaxf(0.f, fmaxf(y0 - by_hi, by_lo - (y0 + h)));
            const float rem = reach2 - dy * dy - dz * dz;
            if (rem > 0.f) {
                const float wdt = chord_sqrt(rem);
                const int cx0 = clampi((int)floorf((bx_lo - lox - wdt) * inv_h), 0, ncx - 1);
                const int cx1 = clampi((int)floorf((bx_hi - lox + wdt) * inv_h), 0, ncx - 1);
                const int ca = max(cx0, bx * kBrick), cb = min(cx1, bx * kBrick + kBrick - 1);
                if (ca <= cb) {
                    const int r0 = (int)P.cell0 + cell_rank32(P, ca, cy, cz);
                    const int e = cstart[r0 + (cb - ca) + 1];
                    jb = max(cstart[r0], gend);
                    len = max(0, e - jb);
                }
            }
        }
        const int incl = wave_incl_scan(len);
        const int start = incl - len;
        pre[lane] = start;
        fst[lane] = jb;
        const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
        if (lane == 0) pre[kWave] = total;
        for (int t = 0; t < len && start + t < kClMap; ++t) map[start + t] = jb + t;
        __builtin_amdgcn_wave_barrier();
        auto atom_at = [&](int pos) -> int {
            if (pos < kClMap) return map[pos];
            int lo_ = 0, hi_ = kWave;   // pre[lo_] <= pos < pre[hi_]
            while (hi_ - lo_ > 1) {
                const int mid = (lo_ + hi_) >> 1;
                if (pre[mid] <= pos) lo_ = mid; else hi_ = mid;
            }
            return fst[lo_] + (pos - pre[lo_]);
        };
        int pj = -1;
        float4 pa;
        if (lane < total) {
            pj = atom_at(lane);
            pa = sx[pj];
        }
        for (int c0 = 0; c0 < total; c0 += kWave) {
            const bool have = c0 + lane < total;
            const float4 ca = pa;
            const int cj = pj;
            const int nxt = c0 + kWave + lane;   // the next chunk, in flight while this one is used
            if (nxt < total) {
                pj = atom_at(nxt);
                pa = sx[pj];
            }
            const float ddx = fmaxf(0.f, fmaxf(bx_lo - ca.x, ca.x - bx_hi));
            const float ddy = fmaxf(0.f, fmaxf(by_lo - ca.y, ca.y - by_hi));
            const float ddz = fmaxf(0.f, fmaxf(bz_lo - ca.z, ca.z - bz_hi));
            const bool keep = have && ddx * ddx + ddy * ddy + ddz * ddz < reach2;
            const uint64_t m = __ballot(keep);
            if (keep) {
                const int e = (tail + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))) &
                              (kClRing - 1);
                ring[e] = ca;
                ridx[e] = cj;
            }
            tail += __popcll(m);
            __builtin_amdgcn_wave_barrier();
            if (tail - head >= kWave) eval_block();
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (tail > head) {   // the last partial block, padded with far-away atoms of no index
        if (lane >= tail - head) {
            const int e = (head + lane) & (kClRing - 1);
            float4 far;
            far.x = far.y = far.z = 1e18f;
            far.w = 0.f;
            ring[e] = far;
            ridx[e] = -1;
        }
        __builtin_amdgcn_wave_barrier();
        eval_block();
    }

    // the cluster's sums across the 64 lanes: each exchange halves the values a
    // lane holds (the upper lane of a pair keeps the upper half), then the two
    // lanes left for each value add; lane 2v holds value v = 4 ia + component
    float v[4 * CA];
#pragma unroll
    for (int ia = 0; ia < CA; ++ia) {
        v[4 * ia] = fx[ia];
        v[4 * ia + 1] = fy[ia];
        v[4 * ia + 2] = fz[ia];
        v[4 * ia + 3] = u[ia];
    }
    halve<16, 32>(v, lane);
    halve<8, 16>(v, lane);
    halve<4, 8>(v, lane);
    halve<2, 4>(v, lane);
    halve<1, 2>(v, lane);
    v[0] += __shfl_xor(v[0], 1, kWave);
    const int vi = lane >> 1, ia = vi >> 2, comp = vi & 3;
    const int iat = __shfl(mi, ia, kWave);
    if ((lane & 1) == 0 && iat >= 0) reinterpret_cast<float *>(out)[4 * (int64_t)iat + comp] = v[0];
}

// Adds each atom's fixed-point accumulators to the stored sums and clears them.
__global__ __launch_bounds__(256) void k_n3_combine(int64_t n, float4 *__restrict__ out,
                                                    unsigned long long *__restrict__ acc, int64_t stride, int pot)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 o = out[i];
    const long long ax = (long long)acc[i], ay = (long long)acc[stride + i], az = (long long)acc[2 * stride + i];
    o.x = (float)((double)o.x + (double)ax * kFixUnit);
    o.y = (float)((double)o.y + (double)ay * kFixUnit);
    o.z = (float)((double)o.z + (double)az * kFixUnit);
    acc[i] = 0;
    acc[stride + i] = 0;
    acc[2 * stride + i] = 0;
    if (pot) {
        const long long au = (long long)acc[3 * stride + i];
        o.w = (float)((double)o.w + (double)au * kFixUnit);
        acc[3 * stride + i] = 0;
    }
    out[i] = o;
}

// k_pair_grp: the 8-atom clusters of one 64-atom group (GW = 8 waves in one
// workgroup) or of half a group (GW = 4) share one candidate stream: the
// cell-row pieces that reach the box around all of them. The waves build the
// piece table together (64 pieces each per batch), load the stream together
// (64 candidates each per round, the next round in flight while the current
// one is used) into a double buffer in LDS, and then each wave keeps, from
// every candidate of the round, those within the cutoff of its own cluster's
// box and evaluates them as k_pair_cl does with 8-atom clusters. The pieces
// are clipped to the common box, so each of them holds the pieces of the
// single-cluster stream as sub-runs, in the same order: every cluster keeps
// the same candidates in the same order as in k_pair_cl, and the results are
// the same bits. Building and loading the stream is paid once per workgroup
// instead of once per cluster.
template <int GW> constexpr int grp_map() { return GW * 256; }   // positions with a table entry

template <typename T, bool MD, int GW> struct GrpLds {
    vec4_t<T> cand[2][GW * kWave];   // one round of the stream, double buffered
    vec4_t<T> caux[MD ? 2 : 1][MD ? GW * kWave : 1];
    vec4_t<T> ring[GW][kClRing];
    vec4_t<T> raux[MD ? GW : 1][MD ? kClRing : 1];
    int map[grp_map<GW>()];          // stream position -> sorted atom
    int pre[GW * kWave + 1];         // piece stream offsets of the batch
    int first[GW * kWave];           // first atom of each piece
    int wtot[GW];                    // stream length of each wave's pieces
    T box[GW][6];                    // cluster boxes; an absent cluster's is empty (lo > hi)
};

template <typename T, bool MD, bool POT, int KIND, int GW>
__global__ __launch_bounds__(GW * kWave) void k_pair_grp(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                          const int *__restrict__ cstart,
                                                          const int *__restrict__ cluster,
                                                          vec4_t<T> *__restrict__ out, PairK<T> k,
                                                          const vec4_t<T> *__restrict__ saux)
{
    constexpr int CA = 8, kSlots = kWave / CA, kU = cl_unroll<MD>(), kBlock = kSlots * kU, NR = GW * kWave;
    constexpr int kMap = grp_map<GW>();
    __shared__ GrpLds<T, MD, GW> L;
    __shared__ WolfLds<T, KIND> wl;
    if (eval_failed(p)) return;   // the same for every workgroup
    wl.load(k);
    const float4 *wtab = wl.ptr();
    const int lane = threadIdx.x % kWave;
    const int wv = uni((int)(threadIdx.x / kWave));
    const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * GW + wv;   // this wave's cluster
    const int64_t g = c / (kWave / CA);
    const int s = find_segment(p.group_prefix, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int me = lane % CA, slot = lane / CA;
    const int cfirst = uni(cluster[c * CA]);
    const bool on = cfirst >= 0;   // uniform
    const int mi = cluster[c * CA + me];
    const bool valid = mi >= 0;
    // lanes of absent atoms evaluate a stand-in (a real atom) and write nothing
    const int64_t i = valid ? (int64_t)mi : (on ? (int64_t)cfirst : P.atom0 + (g - p.group_prefix[s]) * kWave);
    const vec4_t<T> ai = sx[i];
    vec4_t<T> xi;
    if (MD) xi = saux[i];
    const T bx_lo = uni(seg_min(ai.x, CA)), bx_hi = uni(seg_max(ai.x, CA));
    const T by_lo = uni(seg_min(ai.y, CA)), by_hi = uni(seg_max(ai.y, CA));
    const T bz_lo = uni(seg_min(ai.z, CA)), bz_hi = uni(seg_max(ai.z, CA));
    if (lane == 0) {
        const T inf = T(1e30);
        L.box[wv][0] = on ? bx_lo : inf;
        L.box[wv][1] = on ? by_lo : inf;
        L.box[wv][2] = on ? bz_lo : inf;
        L.box[wv][3] = on ? bx_hi : -inf;
        L.box[wv][4] = on ? by_hi : -inf;
        L.box[wv][5] = on ? bz_hi : -inf;
    }
    __syncthreads();
    // the box around the workgroup's clusters (the same in every wave)
    T bminx = L.box[0][0], bminy = L.box[0][1], bminz = L.box[0][2];
    T bmaxx = L.box[0][3], bmaxy = L.box[0][4], bmaxz = L.box[0][5];
#pragma unroll
    for (int w = 1; w < GW; ++w) {
        bminx = fmin(bminx, L.box[w][0]), bminy = fmin(bminy, L.box[w][1]), bminz = fmin(bminz, L.box[w][2]);
        bmaxx = fmax(bmaxx, L.box[w][3]), bmaxy = fmax(bmaxy, L.box[w][4]), bmaxz = fmax(bmaxz, L.box[w][5]);
    }
    if (!(bminx <= bmaxx)) return;   // no cluster here: the whole workgroup leaves
    const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]);
    const T inv_h = T(P.inv_h), h = T(1.0 / P.inv_h);
    const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
    const T reach = k.reach, reach2 = k.reach * k.reach;
    const int cy0 = clampi((int)floor((bminy - loy - reach) * inv_h), 0, ncy - 1);
    const int cy1 = clampi((int)floor((bmaxy - loy + reach) * inv_h), 0, ncy - 1);
    const int cz0 = clampi((int)floor((bminz - loz - reach) * inv_h), 0, ncz - 1);
    const int cz1 = clampi((int)floor((bmaxz - loz + reach) * inv_h), 0, ncz - 1);
    const int bx0 = clampi((int)floor((bminx - lox - reach) * inv_h), 0, ncx - 1) / kBrick;
    const int bx1 = clampi((int)floor((bmaxx - lox + reach) * inv_h), 0, ncx - 1) / kBrick;
    const int nbx = bx1 - bx0 + 1, ny = cy1 - cy0 + 1;
    const int nitems = nbx * ny * (cz1 - cz0 + 1);

    if (KIND == kPolyHigh)
        asm volatile("" : "+v"(k.c2), "+v"(k.d1));
    else if (KIND == kPoly)
        asm volatile("" : "+v"(k.c1), "+v"(k.d0));
    T fx = 0, fy = 0, fz = 0, u = 0;
    int head = 0, tail = 0;   // ring positions (uniform; taken modulo the capacity)
    vec4_t<T> *ring = L.ring[wv];
    vec4_t<T> *raux = L.raux[MD ? wv : 0];
    auto eval_block = [&]() {
        // a block starts at a multiple of its size, so it does not wrap
        const int e0 = (head & (kClRing - 1)) + slot;
        vec4_t<T> aj[kU], xj[kU];
#pragma unroll
        for (int v = 0; v < kU; ++v) {
            aj[v] = ring[e0 + kSlots * v];
            xj[v] = MD ? aux3<T>(raux[MD ? e0 + kSlots * v : 0]) : aj[v];
        }
#pragma unroll
        for (int v = 0; v < kU; ++v)
            pair_term<T, MD, POT, KIND>(ai, xi, aj[v], xj[v], k, fx, fy, fz, u, wtab);
        head += kBlock;
    };
    int *map = L.map, *pre = L.pre, *fst = L.first;
    for (int ib = 0; ib < nitems; ib += NR) {
        // this wave's 64 pieces of the batch
        const int q = ib + wv * kWave + lane;
        int len = 0, jb = 0;
        if (q < nitems) {
            const int bx = bx0 + q % nbx, row = q / nbx;
            const int cy = cy0 + row % ny, cz = cz0 + row / ny;
            const T z0 = loz + T(cz) * h, y0 = loy + T(cy) * h;
            const T dz = fmax(T(0), fmax(z0 - bmaxz, bminz - (z0 + h)));
            const T dy = fmax(T(0), fmax(y0 - bmaxy, bminy - (y0 + h)));
            const T rem = reach2 - dy * dy - dz * dz;
            if (rem > T(0)) {
                const T wdt = chord_sqrt(rem);
                const int cx0 = clampi((int)floor((bminx - lox - wdt) * inv_h), 0, ncx - 1);
                const int cx1 = clampi((int)floor((bmaxx - lox + wdt) * inv_h), 0, ncx - 1);
                const int ca = max(cx0, bx * kBrick), cb = min(cx1, bx * kBrick + kBrick - 1);
                if (ca <= cb) {
                    const int r0 = (int)P.cell0 + cell_rank32(P, ca, cy, cz);
                    jb = cstart[r0];
                    len = cstart[r0 + (cb - ca) + 1] - jb;
                }
            }
        }
        const int incl = wave_incl_scan(len);
        if (lane == kWave - 1) L.wtot[wv] = incl;
        __syncthreads();   // the previous batch's tables are no longer read
        int base = 0, total = 0;
#pragma unroll
        for (int w = 0; w < GW; ++w) {
            const int t = L.wtot[w];
            base += w < wv ? t : 0;
            total += t;
        }
        const int start = base + incl - len;
        pre[wv * kWave + lane] = start;
        fst[wv * kWave + lane] = jb;
        if (wv == GW - 1 && lane == kWave - 1) pre[NR] = total;
        for (int t = 0; t < len && start + t < kMap; ++t) map[start + t] = jb + t;
        __syncthreads();   // the batch's tables are complete
        auto atom_at = [&](int pos) -> int {
            if (pos < kMap) return map[pos];
            int lo_ = 0, hi_ = NR;   // pre[lo_] <= pos < pre[hi_]
            while (hi_ - lo_ > 1) {
                const int mid = (lo_ + hi_) >> 1;
                if (pre[mid] <= pos) lo_ = mid; else hi_ = mid;
            }
            return fst[lo_] + (pos - pre[lo_]);
        };
        // the first round
        const int own = wv * kWave + lane;   // this thread's place in a round
        if (own < total) {
            const int j = atom_at(own);
            L.cand[0][own] = sx[j];
            if (MD) L.caux[0][MD ? own : 0] = saux[j];
        }
        __syncthreads();
        int buf = 0;
        for (int r0 = 0; r0 < total; r0 += NR) {
            // the next round, in flight while this one is used
            const int nx = r0 + NR + own;
            vec4_t<T> pa, px;
            if (nx < total) {
                const int j = atom_at(nx);
                pa = sx[j];
                if (MD) px = saux[j];
            }
            if (on) {
#pragma unroll 1
                for (int kk = 0; kk < GW; ++kk) {
                    const int c0 = r0 + kk * kWave;
                    if (c0 >= total) break;   // uniform
                    const bool have = c0 + lane < total;
                    const vec4_t<T> ca = L.cand[buf][kk * kWave + lane];
                    const T ddx = fmax(T(0), fmax(bx_lo - ca.x, ca.x - bx_hi));
                    const T ddy = fmax(T(0), fmax(by_lo - ca.y, ca.y - by_hi));
                    const T ddz = fmax(T(0), fmax(bz_lo - ca.z, ca.z - bz_hi));
                    const bool keep = have && ddx * ddx + ddy * ddy + ddz * ddz < reach2;
                    const uint64_t m = __ballot(keep);
                    if (keep) {
                        const int e = (tail + (int)__builtin_amdgcn_mbcnt_hi(
                                                  (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))) &
                                      (kClRing - 1);
                        ring[e] = ca;
                        if (MD) raux[MD ? e : 0] = L.caux[MD ? buf : 0][MD ? kk * kWave + lane : 0];
                    }
                    tail += __popcll(m);
                    __builtin_amdgcn_wave_barrier();
                    while (tail - head >= kBlock) eval_block();
                    __builtin_amdgcn_wave_barrier();
                }
            }
            if (nx < total) {
                L.cand[buf ^ 1][own] = pa;
                if (MD) L.caux[MD ? buf ^ 1 : 0][MD ? own : 0] = px;
            }
            __syncthreads();   // the next round is in place; this one is no longer read
            buf ^= 1;
        }
    }
    if (!on) return;
    if (tail > head) {   // the last partial block, padded with a far-away atom
        if (lane < head + kBlock - tail) {
            vec4_t<T> far;
            far.x = far.y = far.z = T(1e18);
            far.w = T(0);
            ring[(tail + lane) & (kClRing - 1)] = far;
            if (MD) raux[MD ? (tail + lane) & (kClRing - 1) : 0] = far;
        }
        __builtin_amdgcn_wave_barrier();
        eval_block();
    }
    fx = sum_slots<CA>(fx);
    fy = sum_slots<CA>(fy);
    fz = sum_slots<CA>(fz);
    if (POT) u = sum_slots<CA>(u);
    if (slot == 0 && valid) {
        vec4_t<T> o;
        o.x = fx;
        o.y = fy;
        o.z = fz;
        o.w = u;
        out[i] = o;
    }
}

// ---------------------------------------------------------------------------
// The dynamics model (Section 2). The pair kernels sum the method's pair term
// for every pair inside the cutoff, the pairs inside one molecule included.
// Such a pair must leave only -gamma(r/a)/a in MSM (the negative of the smooth
// part the grids carry for it) and nothing in the simple cutoff method and
// Wolf summation, which have no grids: k_exclude takes away, for each partner
// within the cutoff, 1/r (MSM and the simple cutoff) or the Wolf pair term,
// with its force bracket. One thread per sorted atom, partners in a fixed
// order (the model's list, built from the molecule ids when it is bound).
template <typename T, int KIND, bool POT>
__global__ __launch_bounds__(256) void k_exclude(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                 const int *__restrict__ order, const vec4_t<T> *__restrict__ xin,
                                                 const int *__restrict__ xstart, const int *__restrict__ xidx,
                                                 int64_t period, vec4_t<T> *__restrict__ out, PairK<T> k)
{
    if (eval_failed(p)) return;
    const int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos >= p.natoms) return;
    const int64_t o = order[pos];
    const int64_t mdl = o % period, base = o - mdl;
    const int e0 = xstart[mdl], e1 = xstart[mdl + 1];
    if (e0 == e1) return;
    const vec4_t<T> ai = sx[pos];
    T fx = 0, fy = 0, fz = 0, u = 0;
    for (int e = e0; e < e1; ++e) {
        const int64_t j = base + xidx[e];
        if (j >= p.natoms) continue;   // a model that does not fit the batch
        const vec4_t<T> aj = xin[j];
        const T dx = ai.x - aj.x, dy = ai.y - aj.y, dz = ai.z - aj.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < k.a2 && r2 > T(0)) {
            const T rinv = rsqrt_t(r2);
            T br, pu;
            if (KIND == kWolf && sizeof(T) == 4) {
                const T r = r2 * rinv;
                float E, D;
                wolf_lookup(k.wtab, float(r), k.wscale, E, D);
                br = T(D) * rinv * rinv * rinv;
                pu = T(E) * rinv - k.wshift;
            } else if (KIND == kWolf) {
                const T r = r2 * rinv;
                const T er = erfc(k.alpha * r);
                br = (er * rinv + k.wexp * exp(-k.alpha2 * r2)) * rinv * rinv;
                pu = er * rinv - k.wshift;
            } else {
                br = rinv * rinv * rinv;
                pu = rinv;
            }
            const T t = aj.w * br;
            fx += t * dx;
            fy += t * dy;
            fz += t * dz;
            if (POT) u += aj.w * pu;
        }
    }
    vec4_t<T> v = out[pos];
    v.x -= fx;
    v.y -= fy;
    v.z -= fz;
    if (POT) v.w -= u;
    out[pos] = v;
}

template <typename T, int KIND, int GW>
static void pair_launch_grp(hipStream_t s, const DevPlan &p, const Work<T> &w, const PairK<T> &k, bool pot)
{
    hipLaunchKernelGGL((k_clusters<T, 8>), dim3((unsigned)p.ngroups), dim3(kWave), 0, s, p, w.sxyzq, w.cluster);
    const dim3 grid((unsigned)(p.ngroups * (8 / GW))), block(GW * kWave);
    const vec4_t<T> *none = nullptr;
    if (pot)
        hipLaunchKernelGGL((k_pair_grp<T, false, true, KIND, GW>), grid, block, 0, s, p, w.sxyzq, w.cell_start,
                           w.cluster, w.shrt, k, none);
    else
        hipLaunchKernelGGL((k_pair_grp<T, false, false, KIND, GW>), grid, block, 0, s, p, w.sxyzq, w.cell_start,
                           w.cluster, w.shrt, k, none);
}

template <typename T, int KIND, int NSUB, int CA>
static void pair_launch_cl(hipStream_t s, const DevPlan &p, const Work<T> &w, const PairK<T> &k, bool pot)
{
    hipLaunchKernelGGL((k_clusters<T, CA>), dim3((unsigned)p.ngroups), dim3(kWave), 0, s, p, w.sxyzq, w.cluster);
    const int64_t nclusters = p.ngroups * (kWave / CA);
    const int64_t per_wg = (int64_t)kClWgWaves * NSUB;
    const dim3 grid((unsigned)((nclusters + per_wg - 1) / per_wg)), block(kClWgWaves * kWave);
    const vec4_t<T> *none = nullptr;
    if (pot)
        hipLaunchKernelGGL((k_pair_cl<T, false, true, KIND, NSUB, CA>), grid, block, 0, s, p, w.sxyzq, w.cell_start,
                           w.cluster, w.shrt, k, none);
    else
        hipLaunchKernelGGL((k_pair_cl<T, false, false, KIND, NSUB, CA>), grid, block, 0, s, p, w.sxyzq, w.cell_start,
                           w.cluster, w.shrt, k, none);
}

// Newton's third law form: clusters, the pair kernel, then the accumulators
// added to the sums (single precision only; the caller checks)
template <int KIND>
static void pair_launch_n3(hipStream_t s, const DevPlan &p, const Work<float> &w, const PairK<float> &k, bool pot)
{
    hipLaunchKernelGGL((k_clusters<float, kN3Cl>), dim3((unsigned)p.ngroups), dim3(kWave), 0, s, p, w.sxyzq,
                       w.cluster);
    const int64_t nclusters = p.ngroups * (kWave / kN3Cl);
    const dim3 grid((unsigned)((nclusters + kClWgWaves - 1) / kClWgWaves)), block(kClWgWaves * kWave);
    if (pot)
        hipLaunchKernelGGL((k_pair_n3<true, KIND>), grid, block, 0, s, p, w.sxyzq, w.cell_start, w.cluster, w.shrt,
                           w.nacc, w.nacc_stride, k);
    else
        hipLaunchKernelGGL((k_pair_n3<false, KIND>), grid, block, 0, s, p, w.sxyzq, w.cell_start, w.cluster, w.shrt,
                           w.nacc, w.nacc_stride, k);
    hipLaunchKernelGGL(k_n3_combine, dim3((unsigned)((p.natoms + 255) / 256)), dim3(256), 0, s, p.natoms, w.shrt,
                       w.nacc, w.nacc_stride, pot ? 1 : 0);
}

template <typename T, int KIND>
static void pair_launch_sub(hipStream_t s, const DevPlan &p, const Work<T> &w, const PairK<T> &k, bool pot)
{
    const dim3 grid((unsigned)p.ngroups), block(kSubLanes * kWave);
    const vec4_t<T> *none = nullptr;
    if (pot)
        hipLaunchKernelGGL((k_pair_sub<T, false, true, KIND>), grid, block, 0, s, p, w.sxyzq, w.cell_start, w.shrt,
                           k, none);
    else
        hipLaunchKernelGGL((k_pair_sub<T, false, false, KIND>), grid, block, 0, s, p, w.sxyzq, w.cell_start, w.shrt,
                           k, none);
}

template <typename T, int KIND, int NW>
static void pair_launch(hipStream_t s, const DevPlan &p, const Work<T> &w, const PairK<T> &k, bool pot)
{
    const dim3 grid((unsigned)p.ngroups), block(NW * kWave);
    const vec4_t<T> *none = nullptr;
    if (pot)
        hipLaunchKernelGGL((k_pair<T, false, true, KIND, NW>), grid, block, 0, s, p, w.sxyzq, w.cell_start, w.shrt, k,
                           none);
    else
        hipLaunchKernelGGL((k_pair<T, false, false, KIND, NW>), grid, block, 0, s, p, w.sxyzq, w.cell_start, w.shrt,
                           k, none);
}

template <typename T, int NW>
static void pair_launch_m(hipStream_t s, const DevPlan &p, const Work<T> &w, const PairK<T> &k, bool pot, int kind)
{
    if constexpr (NW == 7 || NW == 9) {
        // 8-atom clusters sharing one stream per group (7) or half group (9)
        constexpr int GW = NW == 7 ? 8 : 4;
        if (kind == kWolf) pair_launch_grp<T, kWolf, GW>(s, p, w, k, pot);
        else if (kind == kPolyHigh) pair_launch_grp<T, kPolyHigh, GW>(s, p, w, k, pot);
        else pair_launch_grp<T, kPoly, GW>(s, p, w, k, pot);
    } else if constexpr (NW == 2 || NW == 3 || NW == 5 || NW == 6) {
        // cluster form: one 8-atom cluster per wave, or two sharing a stream;
        // one 16-atom or one 32-atom cluster per wave
        constexpr int NS = NW == 3 ? 2 : 1;
        constexpr int CA = NW == 5 ? 16 : (NW == 6 ? 32 : 8);
        if (kind == kWolf) pair_launch_cl<T, kWolf, NS, CA>(s, p, w, k, pot);
        else if (kind == kPolyHigh) pair_launch_cl<T, kPolyHigh, NS, CA>(s, p, w, k, pot);
        else pair_launch_cl<T, kPoly, NS, CA>(s, p, w, k, pot);
    } else if constexpr (NW == 1) {   // sub-group form
        if (kind == kWolf) pair_launch_sub<T, kWolf>(s, p, w, k, pot);
        else if (kind == kPolyHigh) pair_launch_sub<T, kPolyHigh>(s, p, w, k, pot);
        else pair_launch_sub<T, kPoly>(s, p, w, k, pot);
    } else {
        if (kind == kWolf) pair_launch<T, kWolf, NW>(s, p, w, k, pot);
        else if (kind == kPolyHigh) pair_launch<T, kPolyHigh, NW>(s, p, w, k, pot);
        else pair_launch<T, kPoly, NW>(s, p, w, k, pot);
    }
}

}  // namespace

void wolf_table(double a, double alpha, float *out)
{
    const double c = 2.0 * alpha / std::sqrt(std::acos(-1.0)), dr = a / kWolfPieces;
    auto E = [&](double r) { return std::erfc(alpha * r); };
    auto dE = [&](double r) { return -c * std::exp(-alpha * alpha * r * r); };
    auto D = [&](double r) { return std::erfc(alpha * r) + c * r * std::exp(-alpha * alpha * r * r); };
    auto dD = [&](double r) { return -2.0 * alpha * alpha * c * r * r * std::exp(-alpha * alpha * r * r); };
    auto piece = [&](double f0, double f1, double m0, double m1, float *o) {
        o[0] = float(f0);
        o[1] = float(m0);
        o[2] = float(3.0 * (f1 - f0) - 2.0 * m0 - m1);
        o[3] = float(2.0 * (f0 - f1) + m0 + m1);
    };
    for (int k = 0; k < kWolfPieces; k++) {
        const double r0 = k * dr, r1 = (k + 1) * dr;
        piece(E(r0), E(r1), dE(r0) * dr, dE(r1) * dr, out + 8 * k);
        piece(D(r0), D(r1), dD(r0) * dr, dD(r1) * dr, out + 8 * k + 4);
    }
}

// The pair constants of the method (all kernels of this file use them).
template <typename T> static PairK<T> pair_constants(const MethodConst &m)
{
    PairK<T> k{};
    const double a = m.a;
    k.a2 = T(a * a);
    k.reach = T(a * (1.0 + 1e-5));
    k.inv_a2 = T(1.0 / (a * a));
    // gamma(r/a)/a = sum_j g_j r^(2j) / a^(2j+1) and
    // -(d/dr)(gamma(r/a)/a) / r = -sum_{j>=1} 2 j g_j r^(2j-2) / a^(2j+1)
    // (m = 2: 15/8 a^-1 - 5/4 a^-3 r^2 + 3/8 a^-5 r^4 and 5/2 a^-3 - 3/2 a^-5 r^2);
    // the simple cutoff method and Wolf summation (Section 5) have no
    // smoothing: all zero
    double cp[kMaxSmooth + 1] = {}, dp[kMaxSmooth] = {};
    if (m.method == MSM_METHOD_MSM)
        for (int j = 0; j <= m.g.m; j++) {
            const double aj = std::pow(a, 2 * j + 1);
            cp[j] = m.g.c[j] / aj;
            if (j >= 1) dp[j - 1] = -2.0 * j * m.g.c[j] / aj;
        }
    k.c0 = T(cp[0]);
    k.c1 = T(cp[1]);
    k.c2 = T(cp[2]);
    k.c3 = T(cp[3]);
    k.d0 = T(dp[0]);
    k.d1 = T(dp[1]);
    k.d2 = T(dp[2]);
    k.alpha = T(m.alpha);
    k.alpha2 = T(m.alpha * m.alpha);
    k.wshift = T(std::erfc(m.alpha * a) / a);
    k.wexp = T(2.0 * m.alpha / std::sqrt(std::acos(-1.0)));
    k.wtab = m.wolf_tab;
    k.wscale = float(kWolfPieces / a);
    return k;
}

static int pair_kind(const MethodConst &m)
{
    return m.method == MSM_METHOD_WOLF ? kWolf : (m.method == MSM_METHOD_MSM && m.g.m == 3 ? kPolyHigh : kPoly);
}

// The pair sums from the pair search's own cells, in the batch's sorted order.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_permute(int64_t n, const int *__restrict__ order,
                                                      const int *__restrict__ pos_of, const vec4_t<T> *__restrict__ in,
                                                      vec4_t<T> *__restrict__ out)
{
    const int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos < n) out[pos] = in[pos_of[order[pos]]];
}

template <typename T>
hipError_t Launch<T>::pair(hipStream_t s, const DevPlan &p, const DevPlan *pp, const Work<T> &w0,
                           const vec4_t<T> *xyzq, const MethodConst &m, bool pot)
{
    if (p.ngroups == 0) return hipSuccess;
    const PairK<T> k = pair_constants<T>(m);
    if (m.method == MSM_METHOD_WOLF && sizeof(T) == 4 && !k.wtab) return hipErrorInvalidValue;
    const int kind = pair_kind(m);
    // with cells of its own, the search runs over a second binning of the
    // atoms (same systems and 64-atom groups, other cells) and its sums are
    // permuted back into the batch order afterwards
    Work<T> w = w0;
    if (pp) {
        if (!w0.pc.x) return hipErrorInvalidValue;
        hipError_t e = bin_sub<T>(s, p, *pp, w0.pc, xyzq, nullptr, 1);
        if (e != hipSuccess) return e;
        w.sxyzq = w0.pc.x;
        w.cell_start = w0.pc.start;
        w.shrt = w0.pc_out;
    }
    const DevPlan &q = pp ? *pp : p;
    switch (m.pair_waves) {
    case 1: pair_launch_m<T, 1>(s, q, w, k, pot, kind); break;
    case 2: pair_launch_m<T, 2>(s, q, w, k, pot, kind); break;
    case 3: pair_launch_m<T, 3>(s, q, w, k, pot, kind); break;
    case 4: pair_launch_m<T, 4>(s, q, w, k, pot, kind); break;
    case 5: pair_launch_m<T, 5>(s, q, w, k, pot, kind); break;
    case 6: pair_launch_m<T, 6>(s, q, w, k, pot, kind); break;
    case 7: pair_launch_m<T, 7>(s, q, w, k, pot, kind); break;
    case 9: pair_launch_m<T, 9>(s, q, w, k, pot, kind); break;
    case 8: pair_launch_m<T, 8>(s, q, w, k, pot, kind); break;
    case 16: pair_launch_m<T, 16>(s, q, w, k, pot, kind); break;
    case 10:
        if constexpr (sizeof(T) == 4) {
            if (!w.nacc || q.natoms > w.nacc_stride) return hipErrorInvalidValue;
            if (kind == kWolf) pair_launch_n3<kWolf>(s, q, w, k, pot);
            else if (kind == kPolyHigh) pair_launch_n3<kPolyHigh>(s, q, w, k, pot);
            else pair_launch_n3<kPoly>(s, q, w, k, pot);
            break;
        } else {
            return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
    if (pp)
        hipLaunchKernelGGL(k_pair_permute<T>, dim3((unsigned)((p.natoms + 255) / 256)), dim3(256), 0, s, p.natoms,
                           w0.order, w0.pc.pos_of, w0.pc_out, w0.shrt);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::exclusions(hipStream_t s, const DevPlan &p, const Work<T> &w, const vec4_t<T> *xyzq,
                                 const MethodConst &m, bool pot)
{
    if (p.natoms == 0 || !w.xstart) return hipSuccess;
    const PairK<T> k = pair_constants<T>(m);
    const dim3 grid((unsigned)((p.natoms + 255) / 256)), block(256);
#define MSMX_EXCL(KIND, POT)                                                                                         \
    hipLaunchKernelGGL((k_exclude<T, KIND, POT>), grid, block, 0, s, p, w.sxyzq, w.order, xyzq, w.xstart, w.xidx, \
                       w.period, w.shrt, k)
    if (m.method == MSM_METHOD_WOLF) {
        if (pot) MSMX_EXCL(kWolf, true);
        else MSMX_EXCL(kWolf, false);
    } else {
        if (pot) MSMX_EXCL(kPoly, true);
        else MSMX_EXCL(kPoly, false);
    }
#undef MSMX_EXCL
    return hipGetLastError();
}

// cluster size of the Lennard-Jones subset's pair kernel
#ifndef MSMX_LJ_CLUSTER
#define MSMX_LJ_CLUSTER 8
#endif
constexpr int kLjCluster = MSMX_LJ_CLUSTER;

template <typename T>
hipError_t Launch<T>::lj(hipStream_t s, const DevPlan &p, const DevPlan &sub, const Work<T> &w, const vec4_t<T> *xyzq,
                         const MethodConst &m, bool pot)
{
    if (!w.lj.x || p.natoms == 0) return hipSuccess;
    // the one-type kernel reads no model records: they are not gathered
    SubBins<T> lb = w.lj;
    if (w.lj_one) lb.aux = nullptr;
    hipError_t e = bin_sub<T>(s, p, sub, lb, xyzq, (const vec4_t<T> *)w.maux, w.period);
    if (e != hipSuccess || sub.ngroups == 0) return e;
    PairK<T> k = pair_constants<T>(m);
    constexpr int CA = kLjCluster;
    hipLaunchKernelGGL((k_clusters<T, CA>), dim3((unsigned)sub.ngroups), dim3(kWave), 0, s, sub, w.lj.x, w.lj_cluster);
    const int64_t nclusters = sub.ngroups * (kWave / CA);
    const dim3 grid((unsigned)((nclusters + kClWgWaves - 1) / kClWgWaves)), pblock(kClWgWaves * kWave);
    const vec4_t<T> *aux = w.lj.aux;
    if (w.lj_one) {
        const double s2 = w.lj_sigma * w.lj_sigma, e = w.lj_eps, c6 = std::pow(s2 / m.a / m.a, 3);
        k.lj_s2 = T(s2);
        k.lj_e4 = T(4 * e);
        k.lj_e24 = T(24 * e);
        k.lj_e48 = T(48 * e);
        k.lj_shift = T(4 * e * (c6 * c6 - c6));
        if (pot)
            hipLaunchKernelGGL((k_pair_cl<T, false, true, kLJ1, 1, CA>), grid, pblock, 0, s, sub, w.lj.x, w.lj.start,
                               w.lj_cluster, w.lj_out, k, nullptr);
        else
            hipLaunchKernelGGL((k_pair_cl<T, false, false, kLJ1, 1, CA>), grid, pblock, 0, s, sub, w.lj.x,
                               w.lj.start, w.lj_cluster, w.lj_out, k, nullptr);
    } else if (pot)
        hipLaunchKernelGGL((k_pair_cl<T, true, true, kLJ, 1, CA>), grid, pblock, 0, s, sub, w.lj.x, w.lj.start,
                           w.lj_cluster, w.lj_out, k, aux);
    else
        hipLaunchKernelGGL((k_pair_cl<T, true, false, kLJ, 1, CA>), grid, pblock, 0, s, sub, w.lj.x, w.lj.start,
                           w.lj_cluster, w.lj_out, k, aux);
    return hipGetLastError();
}

#define MSMX_PAIR_INST(T)                                                                                            \
    template hipError_t Launch<T>::pair(hipStream_t, const DevPlan &, const DevPlan *, const Work<T> &,              \
                                        const vec4_t<T> *, const MethodConst &, bool);                               \
    template hipError_t Launch<T>::exclusions(hipStream_t, const DevPlan &, const Work<T> &, const vec4_t<T> *,      \
                                              const MethodConst &, bool);                                            \
    template hipError_t Launch<T>::lj(hipStream_t, const DevPlan &, const DevPlan &, const Work<T> &,                \
                                      const vec4_t<T> *, const MethodConst &, bool);
MSMX_PAIR_INST(float)
MSMX_PAIR_INST(double)
#undef MSMX_PAIR_INST

}  // namespace msmx
