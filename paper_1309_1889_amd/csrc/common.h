// Shared definitions of the HIP library: per-system plan, workspace layout,
// device helpers for the smoothing function and nodal basis.
//
// Grid geometry (a reading of Section 3, which leaves it open): every level of
// a system shares the domain's lower corner as origin; level-k node (i, j, l)
// sits at lo + 2^k h (i, j, l). Atoms are binned into cells of edge h, cell c
// holding t = (x - lo)/h in [c, c+1), so an atom in cell c touches level-0
// nodes c-1 .. c+2. Level 0 spans node indices [-1, nc+1] with nc =
// floor(L/h) + 1 cells; level k+1 spans [ceil((i0-3)/2), floor((i1+3)/2)] of
// level k's [i0, i1], the nodes that restriction can reach. With these ranges
// no term of the nested sums is dropped.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msmx {

constexpr int kMaxLevels = 16;
constexpr int kBrick = 4;            // cells per brick edge; atoms are sorted brick-major
constexpr int kBrickCells = kBrick * kBrick * kBrick;
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kMaxReach = 12;        // stencil reach R (largest integer below 2a/h) is at most 11
constexpr int kGridPad = kMaxReach;  // zero halo below every charge grid (and above, plus a tile)
constexpr int kStencilTile = 8;      // stencil output tile edge (nodes per axis)

enum StatusBits : int { kStatusDomain = 1, kStatusNonFinite = 2, kStatusConstraint = 4 };

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec4_t = typename Vec4<T>::type;

// One system of a batch, as the kernels see it.
struct SysPlan {
    int64_t atom0;           // first atom in the batch arrays
    int64_t natoms;
    double lo[3];            // domain lower corner (grid origin)
    double inv_h;            // 1/h
    double tmax[3];          // (hi - lo)/h: largest valid t per axis
    int nc[3];               // cells per axis (floor(L/h) + 1)
    int nb[3];               // bricks per axis (nc rounded up to kBrick)
    int64_t cell0;           // first cell (brick-major) in the batch cell arrays
    int64_t ncells;          // nb[0]*nb[1]*nb[2]*kBrickCells
    int nlev;                // number of grids l
    int gorg[kMaxLevels][3]; // first node index per level
    int gdim[kMaxLevels][3]; // node count per level
    int64_t qoff[kMaxLevels];// offset of the padded charge grid: kGridPad zero nodes below
                             // and kGridPad + kStencilTile above the node range on each axis
    int64_t uoff[kMaxLevels];// offset of the unpadded potential grids
    int64_t toff[kMaxLevels];// composite restriction scratch of level k (>= 1)
    int64_t woff[kMaxLevels];// composite prolongation scratch of level k (>= 1)
    int64_t group0;          // first 64-atom pair group
    int64_t ngroups;
};

__host__ __device__ inline int padded_x(int d) { return d + 2 * kGridPad + kStencilTile; }
__host__ __device__ inline int padded_z(int d) { return d + 2 * kGridPad + kStencilTile; }

// Brick rows (the bricks of one (by, bz) pair, along x) are taken in strips
// of kRowStrip rows along y: all rows of a strip, z after y, before the next
// strip. The pair sum reads every atom within the cutoff of the atoms it is
// working on, about two bricks in each direction; with rows ordered z after y
// over the whole domain, the rows one brick away in z are a whole plane of
// rows away in the order, and at 65 x 65 rows of bricks the band a pass over
// the order touches is larger than an XCD's L2. Inside a strip it is
// kRowStrip rows wide. Strips and the y runs inside them alternate
// direction, so consecutive rows share a face. A domain narrower than
// kRowStripMin bricks in y is one strip (rows z after y): its band fits the
// L2 anyway, and on such domains with empty rows around the atoms (a
// dynamics box with room to move) strips measured 1.5-2.5x slower pair
// kernels.
#ifndef MSMX_ROW_STRIP
#define MSMX_ROW_STRIP 8
#endif
constexpr int kRowStrip = MSMX_ROW_STRIP;
constexpr int kRowStripMin = 32;

__host__ __device__ inline int64_t brick_row(const SysPlan &p, int by, int bz)
{
    const int nb1 = p.nb[1], nb2 = p.nb[2];
    if (nb1 < kRowStripMin) return (int64_t)bz * nb1 + ((bz & 1) ? nb1 - 1 - by : by);
    const int s = by / kRowStrip, yl = by - s * kRowStrip;
    const int ws = nb1 - s * kRowStrip < kRowStrip ? nb1 - s * kRowStrip : kRowStrip;
    const int zz = (s & 1) ? nb2 - 1 - bz : bz;
    const int yy = (zz & 1) ? ws - 1 - yl : yl;
    return (int64_t)s * kRowStrip * nb2 + (int64_t)zz * ws + yy;
}

// Rank of cell (cx, cy, cz) within its system. Bricks of 4x4x4 cells are
// visited row by row (brick_row), x alternating direction from row to row,
// so consecutive bricks always share a face and any run of consecutive
// sorted atoms stays spatially compact; cells inside a brick are x-fastest,
// so a brick row of up to 4 cells along x is one contiguous range.
__host__ __device__ inline int64_t cell_rank(const SysPlan &p, int cx, int cy, int cz)
{
    int bx = cx / kBrick, by = cy / kBrick, bz = cz / kBrick;
    int ix = cx % kBrick, iy = cy % kBrick, iz = cz % kBrick;
    int64_t row = brick_row(p, by, bz);
    int xb = (row & 1) ? p.nb[0] - 1 - bx : bx;
    int64_t brick = row * p.nb[0] + xb;
    return brick * kBrickCells + (iz * kBrick + iy) * kBrick + ix;
}

// Inverse of cell_rank: the cell coordinates of rank r within its system.
__host__ __device__ inline void cell_coords(const SysPlan &p, int64_t r, int c[3])
{
    const int64_t brick = r / kBrickCells;
    const int in = (int)(r % kBrickCells);
    const int64_t row = brick / p.nb[0];
    const int xb = (int)(brick % p.nb[0]);
    const int bx = (row & 1) ? p.nb[0] - 1 - xb : xb;
    const int nb1 = p.nb[1], nb2 = p.nb[2];
    if (nb1 < kRowStripMin) {
        const int bz = (int)(row / nb1), yr = (int)(row % nb1);
        c[0] = bx * kBrick + in % kBrick;
        c[1] = ((bz & 1) ? nb1 - 1 - yr : yr) * kBrick + (in / kBrick) % kBrick;
        c[2] = bz * kBrick + in / (kBrick * kBrick);
        return;
    }
    const int s = (int)(row / ((int64_t)kRowStrip * nb2));
    const int rem = (int)(row - (int64_t)s * kRowStrip * nb2);
    const int ws = nb1 - s * kRowStrip < kRowStrip ? nb1 - s * kRowStrip : kRowStrip;
    const int zz = rem / ws, yy = rem % ws;
    const int bz = (s & 1) ? nb2 - 1 - zz : zz;
    const int by = s * kRowStrip + ((zz & 1) ? ws - 1 - yy : yy);
    c[0] = bx * kBrick + in % kBrick;
    c[1] = by * kBrick + (in / kBrick) % kBrick;
    c[2] = bz * kBrick + in / (kBrick * kBrick);
}

// cell_rank in 32-bit arithmetic (a batch holds fewer than 2^31 cells), for
// the pair search's inner loops
static_assert(kBrick == 4 && kBrickCells == 64, "cell_rank32 assumes 4x4x4 bricks");
__host__ __device__ inline int cell_rank32(const SysPlan &p, int cx, int cy, int cz)
{
    static_assert((kRowStrip & (kRowStrip - 1)) == 0, "the strip width is a power of two");
    const int bx = cx >> 2, by = cy >> 2, bz = cz >> 2;
    const int nb0 = p.nb[0], nb1 = p.nb[1], nb2 = p.nb[2];
    int row;
    if (nb1 < kRowStripMin) {
        row = bz * nb1 + ((bz & 1) ? nb1 - 1 - by : by);
    } else {
        const int s = by / kRowStrip, yl = by & (kRowStrip - 1);
        const int ws = nb1 - s * kRowStrip < kRowStrip ? nb1 - s * kRowStrip : kRowStrip;
        const int zz = (s & 1) ? nb2 - 1 - bz : bz;
        row = s * kRowStrip * nb2 + zz * ws + ((zz & 1) ? ws - 1 - yl : yl);
    }
    const int xb = (row & 1) ? nb0 - 1 - bx : bx;
    return ((row * nb0 + xb) << 6) + ((cz & 3) << 4) + ((cy & 3) << 2) + (cx & 3);
}

// Find s with prefix[s] <= g < prefix[s+1]; prefix has n+1 increasing entries.
__device__ inline int find_segment(const int64_t *prefix, int n, int64_t g)
{
    int lo = 0, hi = n;   // invariant: prefix[lo] <= g < prefix[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// ---- Section 3: smoothing function gamma of order m (degree 2m). For rho < 1
// it is the Taylor polynomial of (rho^2)^(-1/2) about rho^2 = 1 up to the
// (rho^2 - 1)^m term, held here expanded in powers of rho^2:
// gamma(rho) = c[0] + c[1] rho^2 + ... + c[m] rho^(2m); 1/rho beyond. m = 2
// (15/8 - 5/4 rho^2 + 3/8 rho^4) is the paper's choice. ----
constexpr int kMaxSmooth = 3;
struct Smooth {
    double c[kMaxSmooth + 1];
    int m;
};

// Coefficients of gamma_m: with b_k = (-1/2 choose k),
// sum_k b_k (rho^2 - 1)^k = sum_j rho^(2j) sum_{k >= j} b_k (k choose j) (-1)^(k-j).
inline Smooth make_smooth(int m)
{
    Smooth g{};
    g.m = m;
    double b = 1.0;   // b_k
    for (int k = 0; k <= m; k++) {
        double kj = 1.0;   // (k choose j)
        for (int j = 0; j <= k; j++) {
            g.c[j] += b * kj * (((k - j) & 1) ? -1.0 : 1.0);
            kj = kj * (k - j) / (j + 1);
        }
        b *= (-0.5 - k) / (k + 1);
    }
    return g;
}

template <typename T> __host__ __device__ inline T gamma_s(T rho, const Smooth &g)
{
    if (rho >= T(1)) return T(1) / rho;
    const T r2 = rho * rho;
    T acc = T(g.c[g.m]);
    for (int k = g.m - 1; k >= 0; --k) acc = acc * r2 + T(g.c[k]);
    return acc;
}

// ---- Section 3: nodal basis Phi, the C1 cubic numerical Hermite interpolant
// (p = 3): 1 - 5/2 s^2 + 3/2 s^3 on |t| <= 1, -1/2 (s-1)(2-s)^2 on 1 < |t| < 2.
template <typename T> __host__ __device__ inline T basis(T t)
{
    T s = fabs(t);
    T inner = T(1) + s * s * (T(-2.5) + T(1.5) * s);
    T u = T(2) - s;
    T outer = T(-0.5) * (s - T(1)) * u * u;
    return s <= T(1) ? inner : (s < T(2) ? outer : T(0));
}

template <typename T> __device__ inline T dbasis(T t)
{
    T s = fabs(t);
    T inner = s * (T(-5) + T(4.5) * s);
    T u = T(2) - s;
    T outer = T(-0.5) * u * (T(4) - T(3) * s);
    T v = s <= T(1) ? inner : (s < T(2) ? outer : T(0));
    return t < T(0) ? -v : v;
}

// ---- Section 3: nodal basis of degree 5 (support |t| < 3), the quintic
// Hermite interpolant of the cardinal data whose node first and second
// derivatives are the five-point central differences; expanded here in
// x = |t| piece by piece:
//   [0,1): 1 - 5/4 x^2 - 35/12 x^3 + 21/4 x^4 - 25/12 x^5
//   [1,2): -4 + 75/4 x - 245/8 x^2 + 545/24 x^3 - 63/8 x^4 + 25/24 x^5
//   [2,3): 18 - 153/4 x + 255/8 x^2 - 313/24 x^3 + 21/8 x^4 - 5/24 x^5
template <typename T> __host__ __device__ inline T basis5(T t)
{
    const T x = fabs(t);
    if (x < T(1)) return T(1) + x * x * (T(-1.25) + x * (T(-35.0 / 12) + x * (T(5.25) + x * T(-25.0 / 12))));
    if (x < T(2))
        return T(-4) + x * (T(18.75) + x * (T(-30.625) + x * (T(545.0 / 24) + x * (T(-7.875) + x * T(25.0 / 24)))));
    if (x < T(3))
        return T(18) + x * (T(-38.25) + x * (T(31.875) + x * (T(-313.0 / 24) + x * (T(2.625) + x * T(-5.0 / 24)))));
    return T(0);
}

template <typename T> __device__ inline T dbasis5(T t)
{
    const T x = fabs(t);
    T v = T(0);
    if (x < T(1))
        v = x * (T(-2.5) + x * (T(-8.75) + x * (T(21) + x * T(-125.0 / 12))));
    else if (x < T(2))
        v = T(18.75) + x * (T(-61.25) + x * (T(545.0 / 8) + x * (T(-31.5) + x * T(125.0 / 24))));
    else if (x < T(3))
        v = T(-38.25) + x * (T(63.75) + x * (T(-313.0 / 8) + x * (T(10.5) + x * T(-25.0 / 24))));
    return t < T(0) ? -v : v;
}

// Phi of degree P on its piece j <= |t| <= j+1 (pieces meet with equal values
// at the knots, so a piece may be evaluated on its closed interval; 0 beyond
// the support, for an atom binned into an edge cell it lies outside of), and
// Phi anywhere inside |t| <= S by selecting the piece without a branch.
template <int P, typename T> __device__ inline T phi_piece(T t, int j)
{
    const T x = fabs(t);
    T v;
    if (P == 3) {
        const T u = T(2) - x;
        v = j == 0 ? T(1) + x * x * (T(-2.5) + T(1.5) * x) : T(-0.5) * (x - T(1)) * u * u;
        return x < T(2) ? v : T(0);
    }
    if (j == 0)
        v = T(1) + x * x * (T(-1.25) + x * (T(-35.0 / 12) + x * (T(5.25) + x * T(-25.0 / 12))));
    else if (j == 1)
        v = T(-4) + x * (T(18.75) + x * (T(-30.625) + x * (T(545.0 / 24) + x * (T(-7.875) + x * T(25.0 / 24)))));
    else
        v = T(18) + x * (T(-38.25) + x * (T(31.875) + x * (T(-313.0 / 24) + x * (T(2.625) + x * T(-5.0 / 24)))));
    return x < T(3) ? v : T(0);
}

template <int P, typename T> __device__ inline T phi_inside(T t)
{
    const T x = fabs(t);
    if (P == 3) {
        // both pieces, then a select (the same expressions as phi_piece)
        const T u = T(2) - x;
        const T inner = T(1) + x * x * (T(-2.5) + T(1.5) * x);
        const T outer = T(-0.5) * (x - T(1)) * u * u;
        const T v = x <= T(1) ? inner : outer;
        return x < T(2) ? v : T(0);
    }
    return x < T(1) ? phi_piece<5>(t, 0) : (x < T(2) ? phi_piece<5>(t, 1) : phi_piece<5>(t, 2));
}

// Basis of degree P (3 or 5) and its support half-width S: Phi(t) = 0 for |t| >= S.
template <int P> struct Basis {
    static constexpr int S = (P + 1) / 2;
    template <typename T> __device__ static T phi(T t) { return P == 5 ? basis5(t) : basis(t); }
    template <typename T> __device__ static T dphi(T t) { return P == 5 ? dbasis5(t) : dbasis(t); }
};

// Reciprocal: the hardware estimate for float (1 ulp), a division for double.
__device__ inline float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_t(double x) { return 1.0 / x; }

// Reciprocal square root: the hardware estimate for float; for double the
// estimate refined by two Newton-Raphson steps y <- y (3 - x y^2) / 2.
__device__ inline float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsqrt_t(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double hx = 0.5 * x;
    y = fma(y, fma(-hx * y, y, 0.5), y);
    y = fma(y, fma(-hx * y, y, 0.5), y);
    return y;
}

}  // namespace msmx
