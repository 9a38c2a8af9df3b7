// HIP kernels of one multilevel summation evaluation (Section 3), templated
// on the arithmetic type T (float or double). Every kernel works on all
// systems of a batch in one launch; a thread or wave finds its system by a
// binary search of a prefix table.
#include <cmath>

#include <type_traits>

#include "device_util.h"
#include "launch.h"
#include "md.h"

namespace msmx {

namespace {

// ---------------------------------------------------------------------------
// Anterpolation (Section 3): q^0_mu = sum_j phi^0_mu(r_j) q_j, as a gather
// (no atomics, fixed order) in one of two forms chosen per batch plan. With a
// basis of support half-width S (2 for the cubic, 3 for the quintic) an atom
// in cell c reaches nodes c-(S-1) .. c+S, so node mu gathers from cells
// mu-S .. mu+S-1.
//
// Tiled, for up to a few atoms per cell: a workgroup owns an 8x8x4 tile of
// nodes. It stages the atoms of the (8+2S-1)x(8+2S-1)x(4+2S-1) cells the
// tile can reach in LDS, as grid coordinates (t = (r - lo)/h, q), row by row
// in x order with a table of where each cell's atoms start; each thread then
// sums its node over the atoms of its (2S)^3 cells. A tile whose region holds
// more atoms than the LDS buffer gathers from global memory.
//
// Two passes, for crowded cells (coarse h), whose cost does not depend on the
// atoms per cell:
//  1. k_anterp_cells: one workgroup per cell; thread m sums the weights of the
//     cell's atoms (sorted order) on node c-(S-1)+m of the cell's (2S)^3
//     support, giving (2S)^3 partial charges per cell (zero when empty).
//  2. k_anterp_nodes: one thread per level-0 node adds the partials of the
//     (2S)^3 cells whose support covers it, in a fixed order.
// ---------------------------------------------------------------------------
// tiles of kAntX x kAntY x AZ nodes: AZ = 4, or 8 for the single precision
// cubic on grids with enough tiles to fill the chip (kAntDeep)
constexpr int kAntX = 8, kAntY = 8;
constexpr int kAntLoads = 4;   // atoms of a cell a staging thread loads at once
// atoms a tile stages in LDS: the cubic's 11x11x7-cell region holds about
// 1,300 water atoms (11x11x11 for AZ = 8: about 2,000), the quintic's 13x13x9
// about 2,400 (FP64: 3,072 x 32 bytes)
template <typename T, int PD, int AZ> constexpr int ant_atoms()
{
    return Basis<PD>::S == 2 ? (AZ == 8 ? 4096 : 2048) : (sizeof(T) == 4 ? 4096 : 3072);
}

// A fixed piece of the cubic along y or z in the tiled gather: the atom's
// row lies within the support (|t| <= 2, up to the rounding of an atom
// clamped into an edge cell), so unlike phi_piece no range test follows.
template <typename T> __device__ inline T cubic_row_piece(T t, int j)
{
    const T x = fabs(t);
    if (j == 0) return T(1) + x * x * (T(-2.5) + T(1.5) * x);
    const T u = T(2) - x;
    return T(-0.5) * (x - T(1)) * u * u;
}

// The cubic along x in the tiled gather: the run of a node's cells holds
// only atoms within the support, so the piece is chosen without a range test.
template <typename T> __device__ inline T cubic_run(T t)
{
    const T x = fabs(t);
    const T u = T(2) - x;
    const T inner = T(1) + x * x * (T(-2.5) + T(1.5) * x);
    const T outer = T(-0.5) * (x - T(1)) * u * u;
    return x <= T(1) ? inner : outer;
}

template <int S, int AZ> struct AntTile {
    static constexpr int CX = kAntX + 2 * S - 1, CY = kAntY + 2 * S - 1, CZ = AZ + 2 * S - 1;   // cells reached
    static constexpr int Rows = CY * CZ;
    static constexpr int Cells = Rows * CX;
};

template <typename T, int PD>
__device__ inline T gather_global(const SysPlan &P, const vec4_t<T> *__restrict__ sx, const int *__restrict__ cstart,
                                  int ix, int iy, int iz)
{
    using B = Basis<PD>;
    constexpr int S = B::S;
    const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]), inv_h = T(P.inv_h);
    const int cx0 = max(ix - S, 0), cx1 = min(ix + S - 1, P.nc[0] - 1);
    T acc = 0;
    for (int cz = max(iz - S, 0); cz <= min(iz + S - 1, P.nc[2] - 1); ++cz)
        for (int cy = max(iy - S, 0); cy <= min(iy + S - 1, P.nc[1] - 1); ++cy)
            for (int bx = cx0 / kBrick; cx0 <= cx1 && bx <= cx1 / kBrick; ++bx) {
                const int ca = max(cx0, bx * kBrick), cb = min(cx1, bx * kBrick + kBrick - 1);
                const int64_t r0 = P.cell0 + cell_rank(P, ca, cy, cz);
                const int jb = cstart[r0], je = cstart[r0 + (cb - ca) + 1];
                for (int j = jb; j < je; ++j) {
                    const vec4_t<T> a = sx[j];
                    const T tx = (a.x - lox) * inv_h, ty = (a.y - loy) * inv_h, tz = (a.z - loz) * inv_h;
                    acc += B::phi(tx - T(ix)) * B::phi(ty - T(iy)) * B::phi(tz - T(iz)) * a.w;
                }
            }
    return acc;
}

// cell layers along z per thread in the tiled form: one (a thread per layer),
// or two where one per layer would need more than 1024 threads (the quintic's
// six layers, the cubic's four with AZ = 8)
template <int PD, int AZ> constexpr int ant_layers_per_thread() { return Basis<PD>::S == 2 && AZ == 4 ? 1 : 2; }
template <int PD, int AZ> constexpr int ant_threads()
{
    return kAntX * kAntY * AZ * (2 * Basis<PD>::S / ant_layers_per_thread<PD, AZ>());
}

template <typename T, int PD, int AZ>
__global__ __launch_bounds__((ant_threads<PD, AZ>())) void k_anterp(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                                  const int *__restrict__ cstart, T *__restrict__ qgrid)
{
    using B = Basis<PD>;
    constexpr int S = B::S;
    using A = AntTile<S, AZ>;
    constexpr int NT = ant_threads<PD, AZ>(), NODES = kAntX * kAntY * AZ, CPT = ant_layers_per_thread<PD, AZ>();
    static_assert(NODES * 2 * S * sizeof(T) <= ant_atoms<T, PD, AZ>() * sizeof(vec4_t<T>), "layer sums fit the atom buffer");
    __shared__ vec4_t<T> atoms[ant_atoms<T, PD, AZ>()];
    __shared__ int start[A::Cells + 1];   // staged position of each region cell's first atom
    __shared__ int wsum[NT / kWave];
    if (eval_failed(p)) return;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int s = find_segment(p.ant_prefix, p.nsys, blk);
    const SysPlan &P = p.sys[s];
    const int dx = P.gdim[0][0], dy = P.gdim[0][1], dz = P.gdim[0][2];
    const int ntx = (dx + kAntX - 1) / kAntX, nty = (dy + kAntY - 1) / kAntY;
    const int64_t t = blk - p.ant_prefix[s];
    // tile origin in absolute node indices
    const int x0 = (int)(t % ntx) * kAntX + P.gorg[0][0];
    const int y0 = (int)((t / ntx) % nty) * kAntY + P.gorg[0][1];
    const int z0 = (int)(t / ((int64_t)ntx * nty)) * AZ + P.gorg[0][2];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;

    // cells of the reachable region (cells x0-S .. x0+kAntX+S-2, ...), 0 atoms
    // outside the grid: each thread counts a contiguous run of cells, a
    // workgroup scan places the runs
    constexpr int per = (A::Cells + NT - 1) / NT;
    int cnt[per], fst[per], sst[per];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        const int c = tid * per + j;
        int n = 0, f = 0;
        if (c < A::Cells) {
            const int ex = c % A::CX, row = c / A::CX;
            const int cx = x0 - S + ex, cy = y0 - S + row % A::CY, cz = z0 - S + row / A::CY;
            if (cx >= 0 && cy >= 0 && cz >= 0 && cx < P.nc[0] && cy < P.nc[1] && cz < P.nc[2]) {
                const int64_t r = P.cell0 + cell_rank(P, cx, cy, cz);
                f = cstart[r];
                n = cstart[r + 1] - f;
            }
        }
        cnt[j] = n;
        fst[j] = f;
        sum += n;
    }
    const int incl = wave_incl_scan(sum);
    if (lane == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    int run = incl - sum;
    for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
    for (int j = 0; j < per; ++j) {
        const int c = tid * per + j;
        if (c < A::Cells) start[c] = run;
        sst[j] = run;
        run += cnt[j];
    }
    if (tid == NT - 1) start[A::Cells] = run;
    __syncthreads();
    const int total = start[A::Cells];
    const bool staged = total <= ant_atoms<T, PD, AZ>();
    if (staged) {
        // each thread stages the atoms of the cells it counted, the first
        // kAntLoads of a cell loaded together
        const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]), inv_h = T(P.inv_h);
        auto put = [&](int pos, const vec4_t<T> &a) {
            vec4_t<T> o;
            o.x = (a.x - lox) * inv_h;
            o.y = (a.y - loy) * inv_h;
            o.z = (a.z - loz) * inv_h;
            o.w = a.w;
            atoms[pos] = o;
        };
#pragma unroll
        for (int j = 0; j < per; ++j) {
            const int n = cnt[j], f = fst[j], s0 = sst[j];
            vec4_t<T> v[kAntLoads];
#pragma unroll
            for (int k = 0; k < kAntLoads; ++k)
                if (k < n) v[k] = sx[f + k];
#pragma unroll
            for (int k = 0; k < kAntLoads; ++k)
                if (k < n) put(s0 + k, v[k]);
            for (int k = kAntLoads; k < n; ++k) put(s0 + k, sx[f + k]);
        }
    }
    __syncthreads();
    // node of this thread, and its share of the node's cell layers along z
    const int node = tid % NODES, q = uni(tid / NODES);
    const int lx = node % kAntX, ly = (node / kAntX) % kAntY, lz = node / (kAntX * kAntY);
    const int ix = x0 + lx, iy = y0 + ly, iz = z0 + lz;
    const int rx = ix - P.gorg[0][0], ry = iy - P.gorg[0][1], rz = iz - P.gorg[0][2];
    const bool inside = rx < dx && ry < dy && rz < dz;
    T acc[CPT];   // one sum per cell layer, so the order of the additions does not depend on CPT
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) acc[cc] = 0;
    if (inside && staged) {
        const T fx = T(ix), fy = T(iy), fz = T(iz);
        // the node's cells ix-S .. ix+S-1 are region columns lx .. lx+2S-1;
        // an atom in the node's cell row c (0 .. 2S-1) along an axis lies at
        // |t - node| in [|c - S|, |c - S| + 1] or [S - 1 - c, S - c], so the
        // piece of Phi along y and z is known for each row
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            const int c = q * CPT + cc;
            const int pz = c < S ? S - 1 - c : c - S;
#pragma unroll
            for (int b = 0; b < 2 * S; ++b) {
                const int py = b < S ? S - 1 - b : b - S;
                const int row = (lz + c) * A::CY + (ly + b);
                const int jb = start[row * A::CX + lx], je = start[row * A::CX + lx + 2 * S];
                for (int j = jb; j < je; ++j) {
                    const vec4_t<T> a = atoms[j];
                    if constexpr (PD == 3)
                        acc[cc] += cubic_run(a.x - fx) * cubic_row_piece(a.y - fy, py) * cubic_row_piece(a.z - fz, pz) * a.w;
                    else
                        acc[cc] += phi_inside<PD>(a.x - fx) * phi_piece<PD>(a.y - fy, py) * phi_piece<PD>(a.z - fz, pz) *
                                   a.w;
                }
            }
        }
    } else if (inside && q == 0) {
        acc[0] = gather_global<T, PD>(P, sx, cstart, ix, iy, iz);
    }
    // the layers' partial sums, added in layer order
    __syncthreads();
    T *part = reinterpret_cast<T *>(atoms);
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) part[(q * CPT + cc) * NODES + node] = acc[cc];
    __syncthreads();
    if (q != 0 || !inside) return;
    T v = part[node];
    for (int c = 1; c < 2 * S; ++c) v += part[c * NODES + node];
    const int PX = padded_x(dx), PY = padded_x(dy);
    qgrid[P.qoff[0] + ((int64_t)(rz + kGridPad) * PY + (ry + kGridPad)) * PX + (rx + kGridPad)] = v;
}

// pass 1: 256 / (2S)^3 cells per workgroup of 256 threads (4 for the cubic,
// one wave each; 1 for the quintic), one thread per support node
template <int PD> constexpr int ant_cells_per_block()
{
    return 256 / ((2 * Basis<PD>::S) * (2 * Basis<PD>::S) * (2 * Basis<PD>::S));
}

template <typename T, int PD>
__global__ __launch_bounds__(256) void k_anterp_cells(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                      const int *__restrict__ cstart, T *__restrict__ part)
{
    using B = Basis<PD>;
    constexpr int S = B::S, W = 2 * S, NP = W * W * W;   // partials per cell
    constexpr int CPB = ant_cells_per_block<PD>();
    if ((int)threadIdx.x >= CPB * NP || eval_failed(p)) return;
    // the cell index is uniform over each wave (NP is a multiple of 64 or CPB is 1)
    const int64_t c = (int64_t)blockIdx.x * CPB + uni((int)(threadIdx.x / NP));   // batch cell
    if (c >= p.ncells) return;
    const int m = threadIdx.x % NP;
    const int jb = uni(cstart[c]), je = uni(cstart[c + 1]);
    T acc = 0;
    if (je > jb) {
        const int s = find_segment(p.cell_prefix, p.nsys, c);
        const SysPlan &P = p.sys[s];
        int cc[3];
        cell_coords(P, c - P.cell0, cc);
        const T lox = T(P.lo[0]), loy = T(P.lo[1]), loz = T(P.lo[2]), inv_h = T(P.inv_h);
        const T nx = T(cc[0] - (S - 1) + m % W), ny = T(cc[1] - (S - 1) + (m / W) % W),
                nz = T(cc[2] - (S - 1) + m / (W * W));
        for (int j = jb; j < je; ++j) {
            const vec4_t<T> a = sx[j];
            acc += B::phi((a.x - lox) * inv_h - nx) * B::phi((a.y - loy) * inv_h - ny) *
                   B::phi((a.z - loz) * inv_h - nz) * a.w;
        }
    }
    part[c * NP + m] = acc;
}

// pass 2
template <typename T, int PD>
__global__ __launch_bounds__(256) void k_anterp_nodes(DevPlan p, const T *__restrict__ part, T *__restrict__ qgrid)
{
    constexpr int S = Basis<PD>::S, W = 2 * S, NP = W * W * W;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= p.nnodes[0]) return;
    const int64_t *pref = p.node_prefix;   // level 0
    const int s = find_segment(pref, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int dx = P.gdim[0][0], dy = P.gdim[0][1];
    const int loc = (int)(g - pref[s]);
    const int rx = loc % dx, ry = (loc / dx) % dy, rz = loc / (dx * dy);
    const int mx = rx + P.gorg[0][0], my = ry + P.gorg[0][1], mz = rz + P.gorg[0][2];   // absolute node
    T acc = 0;
    for (int cz = max(mz - S, 0); cz <= min(mz + S - 1, P.nc[2] - 1); ++cz)
        for (int cy = max(my - S, 0); cy <= min(my + S - 1, P.nc[1] - 1); ++cy)
            for (int cx = max(mx - S, 0); cx <= min(mx + S - 1, P.nc[0] - 1); ++cx) {
                const int64_t r = P.cell0 + cell_rank(P, cx, cy, cz);
                // node mu is entry mu - (c - (S-1)) of cell c's support
                const int e = (mx - cx + S - 1) + W * (my - cy + S - 1) + W * W * (mz - cz + S - 1);
                acc += part[r * NP + e];
            }
    const int PX = padded_x(dx), PY = padded_x(dy);
    qgrid[P.qoff[0] + ((int64_t)(rz + kGridPad) * PY + (ry + kGridPad)) * PX + (rx + kGridPad)] = acc;
}

// ---------------------------------------------------------------------------
// Restriction (Section 3): q^{k+1}_mu = sum_nu phi^{k+1}_mu(r^k_nu) q^k_nu.
// Level-k node nu sits at coarse coordinate nu/2, so the weight is
// prod_d Phi((nu_d - 2 mu_d)/2), non-zero at the offsets nu_d - 2 mu_d = 0
// and odd |d| < 2S: for the cubic 1, 9/16, -1/16 at 0, +-1, +-3; for the
// quintic 1, 150/256, -25/256, 3/256 at 0, +-1, +-3, +-5. The zero halo of
// the fine grid stands in for nodes outside its range.
// ---------------------------------------------------------------------------
template <typename T, int PD>
__device__ inline void restrict_node(const SysPlan &P, T *__restrict__ qgrid, int k, int64_t loc)
{
    using B = Basis<PD>;
    constexpr int S = B::S, NT = 2 * S + 1;   // taps per axis
    const int cdx = P.gdim[k + 1][0], cdy = P.gdim[k + 1][1];
    const int l = (int)loc;   // nodes of one grid fit in int
    const int rx = l % cdx, ry = (l / cdx) % cdy, rz = l / (cdx * cdy);
    // fine-grid relative index of the coincident node 2 mu
    const int fx = 2 * (rx + P.gorg[k + 1][0]) - P.gorg[k][0];
    const int fy = 2 * (ry + P.gorg[k + 1][1]) - P.gorg[k][1];
    const int fz = 2 * (rz + P.gorg[k + 1][2]) - P.gorg[k][2];
    const int FX = padded_x(P.gdim[k][0]), FY = padded_x(P.gdim[k][1]);
    const T *qf = qgrid + P.qoff[k];
    int off[NT];
    T wt[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {   // offsets -(2S-1), .., -1, 0, 1, .., 2S-1 (odd, and 0)
        const int o = i < S ? -(2 * (S - i) - 1) : (i == S ? 0 : 2 * (i - S) - 1);
        off[i] = o;
        wt[i] = o == 0 ? T(1) : B::phi(T(0.5 * o));
    }
    T acc = 0;
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const int64_t zrow = (int64_t)(fz + off[c] + kGridPad) * FY;
        T accy = 0;
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            const T *row = qf + (zrow + (fy + off[b] + kGridPad)) * FX + (fx + kGridPad);
            T accx = 0;
#pragma unroll
            for (int a = 0; a < NT; ++a) accx += wt[a] * row[off[a]];
            accy += wt[b] * accx;
        }
        acc += wt[c] * accy;
    }
    const int CX = padded_x(cdx), CY = padded_x(cdy);
    qgrid[P.qoff[k + 1] + ((int64_t)(rz + kGridPad) * CY + (ry + kGridPad)) * CX + (rx + kGridPad)] = acc;
}

// one level for every system that has a level k+1
template <typename T, int PD>
__global__ __launch_bounds__(256) void k_restrict(DevPlan p, T *__restrict__ qgrid, int k)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= p.nnodes[k + 1]) return;
    const int64_t *pref = p.node_prefix + (int64_t)(k + 1) * (p.nsys + 1);
    const int s = find_segment(pref, p.nsys, g);
    const SysPlan &P = p.sys[s];
    if (k + 1 >= P.nlev) return;
    restrict_node<T, PD>(P, qgrid, k, g - pref[s]);
}

// ---------------------------------------------------------------------------
// Top level (Section 3): u^{l-1}_mu = sum_nu g^{l-1}(r_mu, r_nu) q^{l-1}_nu over
// all node pairs, g^{l-1}(r) = gamma(r / (2^{l-1} a)) / (2^{l-1} a). The grid
// is at most a few hundred nodes; 8 threads share each output node (the
// source z-planes dealt round-robin). The blocks run in the lattice-cutoff
// launch, in LDS the tiles do not use at that point, or alone when a batch
// has no lattice-cutoff tiles.
// ---------------------------------------------------------------------------
constexpr int kTopTable = 4096;   // weights by squared index distance held in LDS (at most)
constexpr int kTopStage = 4096;   // top-grid charges held in LDS (at most)
constexpr int kTopNodes = 32;     // output nodes per block
constexpr int kTopShares = 8;     // threads per output node
constexpr int kTopThreads = kTopNodes * kTopShares;

// top block blk on threads 0..255; lds holds at least kTopThreads + 2 elements
template <typename T>
__device__ inline void top_block(const DevPlan &p, int64_t blk, const T *__restrict__ qgrid, T *__restrict__ ucut,
                                 T *__restrict__ ugrid, double h, double a, int ntab, const Smooth &g, T *lds,
                                 int ldsn)
{
    // weights by squared integer distance d2: gamma(h sqrt(d2) / a) / a; the
    // level's factor 2^-(l-1) is applied to the sum
    T *part = lds;                                   // [kTopShares][kTopNodes]
    const int avail = (ldsn - kTopThreads) / 2;
    const int tabcap = min(kTopTable, avail), qcap = min(kTopStage, avail);
    T *tab = lds + kTopThreads;
    T *qs = tab + tabcap;
    const int s = find_segment(p.top_prefix, p.nsys, blk);
    const SysPlan &P = p.sys[s];
    const int k = P.nlev - 1;
    const int dx = P.gdim[k][0], dy = P.gdim[k][1], dz = P.gdim[k][2];
    const int M = dx * dy * dz;
    const int PX = padded_x(dx), PY = padded_x(dy);
    const T *q = qgrid + P.qoff[k];
    const int tid = threadIdx.x;
    const bool on = tid < kTopThreads;
    for (int d2 = tid; on && d2 < ntab && d2 < tabcap; d2 += kTopThreads)
        tab[d2] = gamma_s(T(h / a) * sqrt(T(d2)), g) * T(1.0 / a);
    for (int e = tid; on && e < M && e < qcap; e += kTopThreads) {
        const int x = e % dx, y = (e / dx) % dy, z = e / (dx * dy);
        qs[e] = q[((int64_t)(z + kGridPad) * PY + (y + kGridPad)) * PX + (x + kGridPad)];
    }
    __syncthreads();
    const int lane = tid % kTopNodes, share = tid / kTopNodes;
    const int node = (int)(blk - p.top_prefix[s]) * kTopNodes + lane;
    T acc = 0;
    if (on && node < M) {
        const int x = node % dx, y = (node / dx) % dy, z = node / (dx * dy);
        for (int nz = share; nz < dz; nz += kTopShares)
            for (int ny = 0; ny < dy; ++ny) {
                const int eyz = (nz - z) * (nz - z) + (ny - y) * (ny - y);
                const int e0 = (nz * dy + ny) * dx;
                for (int nx = 0; nx < dx; ++nx) {
                    const int d2 = eyz + (nx - x) * (nx - x);
                    const T w = d2 < tabcap ? tab[d2] : gamma_s(T(h / a) * sqrt(T(d2)), g) * T(1.0 / a);
                    const int e = e0 + nx;
                    const T qv = e < qcap
                                     ? qs[e]
                                     : q[((int64_t)(nz + kGridPad) * PY + (ny + kGridPad)) * PX + (nx + kGridPad)];
                    acc += w * qv;
                }
            }
    }
    if (on) part[share * kTopNodes + lane] = acc;
    __syncthreads();
    if (on && share == 0 && node < M) {
        T sum = part[lane];
        for (int sh = 1; sh < kTopShares; ++sh) sum += part[sh * kTopNodes + lane];   // fixed order
        sum *= T(ldexp(1.0, -k));
        const int64_t o = P.uoff[k] + node;
        ucut[o] = sum;
        ugrid[o] = sum;
    }
}

template <typename T>
__global__ __launch_bounds__(kTopThreads) void k_top(DevPlan p, const T *__restrict__ qgrid, T *__restrict__ ucut,
                                                     T *__restrict__ ugrid, double h, double a, int ntab, Smooth g)
{
    __shared__ T lds[kTopThreads + kTopTable + kTopStage];
    top_block<T>(p, blockIdx.x, qgrid, ucut, ugrid, h, a, ntab, g, lds, kTopThreads + kTopTable + kTopStage);
}

// Top-level parameters for the lattice-cutoff launch.
struct TopArgs {
    double h, a;
    int ntab;
    int64_t nblocks;     // top blocks run first in the launch (0: none)
    Smooth g;
};

// ---------------------------------------------------------------------------
// Lattice cutoff on level k < l-1 (Section 3): u^{k,cutoff}_mu =
// sum_nu g^k(r^k_mu, r^k_nu) q^k_nu. On level k the node distance is 2^k h |o|,
// and g^k(2^k h |o|) = 2^{-k} g^0(h |o|), so one set of weights g^0(h |o|),
// zero for |o| >= 2a/h, serves every level with an exact power-of-two scale.
//
// A workgroup owns a TXY x TXY x TZ tile of outputs and stages the charges of
// the tile grown by the reach R in LDS. Each thread owns one (x, y) output
// column of TZ nodes and one share of the stencil's columns (ox, oy). The
// weights depend on |o| only, so the (up to) four mirrored columns
// (+-ox, +-oy) are added first and share one pass of the 2R+1 weights along z,
// in which the charges at +-oz are paired too: the quarter-disc of columns
// and half of each carry the whole sphere. The shares are summed in a fixed
// order at the end.
// ---------------------------------------------------------------------------
template <typename T, int R, int NT> struct StencilGeom {
    static constexpr int TZ = (sizeof(T) == 8 && R >= 10) ? 4 : kStencilTile;
    static constexpr int TXY = (sizeof(T) == 8 && R >= 10) ? 4 : kStencilTile;
    static constexpr int EX = TXY + 2 * R;
    static constexpr int EZ = TZ + 2 * R;
    static constexpr int THREADS = NT;
    static constexpr int COLS = TXY * TXY;            // output columns per tile
    static constexpr int SHARES = THREADS / COLS;     // threads per output column
    // LDS holds each (x, y) column's EZ charges contiguously, padded to EZP so
    // that a column is a whole number of 16-byte vectors and the stride
    // between neighbouring columns is an odd number of them: 8 lanes reading
    // 8 neighbouring columns with 16-byte reads then touch all 32 banks once
    static constexpr int VW = 16 / (int)sizeof(T);
    static constexpr int EZV = (EZ + VW - 1) / VW;    // vectors per column
    static constexpr int EZP = (EZV % 2 ? EZV : EZV + 1) * VW;
    static constexpr int IN = EZP * EX * EX;          // staged charges
    static constexpr int LDS = IN > THREADS * TZ ? IN : THREADS * TZ;   // also holds the share sums
};

template <typename T, int R, int NT>
__global__ __launch_bounds__(NT) void k_stencil(DevPlan p, const T *__restrict__ qgrid, T *__restrict__ ucut,
                                                 const int2 *__restrict__ qcols, const T *__restrict__ qw, int ncols,
                                                 T *__restrict__ ugrid, TopArgs top)
{
    using G = StencilGeom<T, R, NT>;
    constexpr int D = 2 * R + 1;
    constexpr int L = G::TZ + 2 * R;
    constexpr int NL = G::LDS > kTopThreads + 2 ? G::LDS : kTopThreads + 2;
    __shared__ __align__(16) T tile[NL];
    if ((int64_t)blockIdx.x < top.nblocks) {
        top_block<T>(p, blockIdx.x, qgrid, ucut, ugrid, top.h, top.a, top.ntab, top.g, tile, NL);
        return;
    }
    const int64_t blk = xcd_remap(blockIdx.x - top.nblocks, gridDim.x - top.nblocks);
    const int seg = find_segment(p.tile_prefix, p.ntile_seg, blk);
    const int k = seg / p.nsys, s = seg % p.nsys;
    const SysPlan &P = p.sys[s];
    const int dx = P.gdim[k][0], dy = P.gdim[k][1], dz = P.gdim[k][2];
    const int ntx = (dx + G::TXY - 1) / G::TXY, nty = (dy + G::TXY - 1) / G::TXY;
    const int64_t t = blk - p.tile_prefix[seg];
    const int x0 = (int)(t % ntx) * G::TXY, y0 = (int)((t / ntx) % nty) * G::TXY;
    const int z0 = (int)(t / ((int64_t)ntx * nty)) * G::TZ;
    const int PX = padded_x(dx), PY = padded_x(dy);
    const T *q = qgrid + P.qoff[k];

    // stage the charges of the grown tile (the grid's zero halo covers the
    // overhang), read along x, stored column by column
    for (int e = threadIdx.x; e < G::EZ * G::EX * G::EX; e += G::THREADS) {
        const int ex = e % G::EX, ey = (e / G::EX) % G::EX, ez = e / (G::EX * G::EX);
        tile[(ey * G::EX + ex) * G::EZP + ez] =
            q[((int64_t)(z0 + kGridPad - R + ez) * PY + (y0 + kGridPad - R + ey)) * PX + (x0 + kGridPad - R + ex)];
    }
    __syncthreads();
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int NV = (L + G::VW - 1) / G::VW;   // vectors read per column
    auto column = [&](int x, int y, T *S) {
        const V *cp = reinterpret_cast<const V *>(tile + (y * G::EX + x) * G::EZP);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const V d = cp[v];
            const T *dv = reinterpret_cast<const T *>(&d);
#pragma unroll
            for (int i = 0; i < G::VW; ++i)
                if (v * G::VW + i < L) S[v * G::VW + i] += dv[i];
        }
    };

    const int col = threadIdx.x % G::COLS;
    const int share = threadIdx.x / G::COLS;
    const int cx = col % G::TXY + R, cy = col / G::TXY + R;
    T acc[G::TZ];
#pragma unroll
    for (int z = 0; z < G::TZ; ++z) acc[z] = T(0);
    for (int c = share; c < ncols; c += G::SHARES) {
        const int2 o = qcols[c];
        T S[L];
#pragma unroll
        for (int z = 0; z < L; ++z) S[z] = T(0);
        column(cx + o.x, cy + o.y, S);
        if (o.x) column(cx - o.x, cy + o.y, S);
        if (o.y) {
            column(cx + o.x, cy - o.y, S);
            if (o.x) column(cx - o.x, cy - o.y, S);
        }
        // the weights along z are even in oz as well: the pair of charges at
        // +-oz is added first and shares one multiply
        const T *w = qw + (int64_t)c * D;
        {
            const T wv = w[R];
#pragma unroll
            for (int z = 0; z < G::TZ; ++z) acc[z] += wv * S[z + R];
        }
        // beyond the sphere (|o| >= 2a/h) the weights of a column are zero
        // from some d on: the column's remaining pairs are skipped (the
        // weights are the same for the whole wave)
#pragma unroll
        for (int d = 1; d <= R; ++d) {
            const T wv = w[R + d];
            if (wv == T(0)) break;
#pragma unroll
            for (int z = 0; z < G::TZ; ++z) acc[z] += wv * (S[z + R + d] + S[z + R - d]);
        }
    }
    __syncthreads();
    // sum the shares in a fixed order; the tile storage is reused
    T *part = tile;
#pragma unroll
    for (int z = 0; z < G::TZ; ++z) part[(share * G::COLS + col) * G::TZ + z] = acc[z];
    __syncthreads();
    const T scale = T(ldexp(1.0, -k));
    T *u = ucut + P.uoff[k];
    for (int e = threadIdx.x; e < G::COLS * G::TZ; e += G::THREADS) {
        const int c = e / G::TZ, z = e % G::TZ;
        T v = part[c * G::TZ + z];
        for (int sh = 1; sh < G::SHARES; ++sh) v += part[(sh * G::COLS + c) * G::TZ + z];
        const int gx = x0 + c % G::TXY, gy = y0 + c / G::TXY, gz = z0 + z;
        if (gx < dx && gy < dy && gz < dz) u[((int64_t)gz * dy + gy) * dx + gx] = v * scale;
    }
}

// ---------------------------------------------------------------------------
// Prolongation (Section 3): u^k_mu = u^{k,cutoff}_mu + sum_nu phi^{k+1}_nu(r^k_mu) u^{k+1}_nu,
// the transpose of restriction. Per axis, fine index m sits at coarse
// coordinate m/2; with n = floor(m/2) the coarse nodes n-(S-1) .. n+S carry
// the weights Phi((m - 2 nu)/2). For odd m these are the 2S nodes of the
// support (cubic: -1/16, 9/16, 9/16, -1/16); for even m Phi of an integer is
// 1 at nu = n and 0 elsewhere (set exactly), so the same 2S taps serve both
// parities. The taps are fully unrolled, so the loads of a node do not wait
// for one another. An even m at the top of the range can name a coarse node
// one past the coarse grid; its weight is 0 and its index is clamped into the
// grid.
// ---------------------------------------------------------------------------
template <typename T, int PD>
__device__ inline void prolong_node(const SysPlan &P, const T *__restrict__ ucut, T *__restrict__ ugrid, int k,
                                    int64_t loc)
{
    using B = Basis<PD>;
    constexpr int S = B::S, W = 2 * S;
    const int dx = P.gdim[k][0], dy = P.gdim[k][1];
    const int l = (int)loc;   // nodes of one grid fit in int
    const int r[3] = {l % dx, (l / dx) % dy, l / (dx * dy)};
    int cn[3][W];
    T cw[3][W];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int m = r[d] + P.gorg[k][d];          // absolute fine index
        const int c0 = P.gorg[k + 1][d], cd = P.gdim[k + 1][d];
        const int n = m >> 1;                       // floor(m/2), m may be negative
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int nu = n - (S - 1) + j;
            cn[d][j] = min(max(nu - c0, 0), cd - 1);
            // even m: exactly the cardinal weights (1 at nu = n)
            cw[d][j] = (m & 1) ? B::phi(T(0.5 * (m - 2 * nu))) : T(j == S - 1 ? 1 : 0);
        }
    }
    const int cdx = P.gdim[k + 1][0], cdy = P.gdim[k + 1][1];
    const T *uc = ugrid + P.uoff[k + 1];
    // an even fine index along y or z takes one coarse row or plane (the
    // others weigh exactly 0); the lanes of a wave share their y and z, so
    // the skipped rows cost nothing
    const bool ey = !((r[1] + P.gorg[k][1]) & 1), ez = !((r[2] + P.gorg[k][2]) & 1);
    T acc = 0;
#pragma unroll
    for (int c = 0; c < W; ++c) {
        if (ez && c != S - 1) continue;
        T accy = 0;
#pragma unroll
        for (int b = 0; b < W; ++b) {
            if (ey && b != S - 1) continue;
            const T *row = uc + ((int64_t)cn[2][c] * cdy + cn[1][b]) * cdx;
            T accx = 0;
#pragma unroll
            for (int a = 0; a < W; ++a) accx += cw[0][a] * row[cn[0][a]];
            accy += cw[1][b] * accx;
        }
        acc += cw[2][c] * accy;
    }
    const int64_t o = P.uoff[k] + loc;
    ugrid[o] = ucut[o] + acc;
}

// one level for every system that has a level k+1 above level k
template <typename T, int PD>
__global__ __launch_bounds__(256) void k_prolong(DevPlan p, const T *__restrict__ ucut, T *__restrict__ ugrid,
                                                 int k)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= p.nnodes[k]) return;
    const int64_t *pref = p.node_prefix + (int64_t)k * (p.nsys + 1);
    const int s = find_segment(pref, p.nsys, g);
    const SysPlan &P = p.sys[s];
    if (k >= P.nlev - 1) return;
    prolong_node<T, PD>(P, ucut, ugrid, k, g - pref[s]);
}

// ---------------------------------------------------------------------------
// Composite transfers. Restriction from level k to k+1 and prolongation back
// are, axis by axis, the filter phi_1(m) = Phi(m/2) between level-k node F
// and level-(k+1) node C (absolute indices) at m = F - 2C (Section 3: the
// level-(k+1) basis function at a level-k node), so the restriction from
// level 0 straight to level k is the product of three one-axis filters
// phi_k(F - 2^k C) with phi_{k+1}(m) = sum_j phi_1(j) phi_k(m - 2^k j), and
// the prolongation from level k straight to level 0 is its transpose. The
// level ranges keep every non-zero term, so q^k = R_k q^0 and
// u^0 = u^{0,cutoff} + sum_k P_k u^{k,cutoff} (u^{l-1,cutoff} being the top
// level's u) equal the level-by-level results up to rounding. Each takes two
// launches for all levels and systems: one workgroup per plane does two axes
// in LDS, then one thread per output node does the third.
// ---------------------------------------------------------------------------
constexpr int kZBatch = 16;   // z terms of the composite transfers loaded together
// threads of a plane workgroup: the planes are few (one per level-0 z-plane and
// level, or per level-k z-plane), so each gets a full CU's worth of waves
constexpr int kXYThreads = 1024;
// threads of a z workgroup (one thread per output node): small workgroups
// spread the few nodes over more CUs
constexpr int kZThreads = 64;

constexpr int kPhiCap = 1024;   // composite filter entries staged in LDS (all levels)

// stage the composite filters in LDS in the working precision; returns false
// when they do not fit (the caller then reads the table in global memory)
template <typename T> __device__ inline int stage_phi(const DevPlan &p, T *lphi)
{
    const int k = p.maxlev - 1;
    const int n = k >= 1 ? p.phi_off[k] + 2 * p.phi_s[k] + 1 : 0;
    for (int e = threadIdx.x; e < n && e < kPhiCap; e += blockDim.x) lphi[e] = T(p.phi[e]);
    __syncthreads();
    return n;
}

// restriction, x and y: block = (system, level-0 z-plane fz, level k >= 1):
// tscr_k[fz][cy][cx] = sum_{y,x} phi_k(y - 2^k cy) phi_k(x - 2^k cx) q^0[fz][y][x]
template <typename T>
__global__ __launch_bounds__(kXYThreads) void k_restrict_xy(DevPlan p, const T *__restrict__ qgrid, T *__restrict__ tscr)
{
    __shared__ T plane[kPlaneCap];
    __shared__ T tmp[kTmpCap];
    __shared__ T lphi[kPhiCap];
    const int64_t blk = blockIdx.x;
    const int s = find_segment(p.rxy_prefix, p.nsys, blk);
    const SysPlan &P = p.sys[s];
    const int r = (int)(blk - p.rxy_prefix[s]);
    const int fz = r / (P.nlev - 1), k = 1 + r % (P.nlev - 1);
    const int fx_n = P.gdim[0][0], fy_n = P.gdim[0][1];
    const int gx0 = P.gorg[0][0], gy0 = P.gorg[0][1];
    const int PX = padded_x(fx_n), PY = padded_x(fy_n);
    const T *q0 = qgrid + P.qoff[0] + ((int64_t)(fz + kGridPad) * PY + kGridPad) * PX + kGridPad;
    const int tid = threadIdx.x;
    for (int e = tid; e < fx_n * fy_n; e += kXYThreads) {
        const int y = e / fx_n, x = e - y * fx_n;
        plane[e] = q0[(int64_t)y * PX + x];
    }
    const bool lds_phi = stage_phi<T>(p, lphi) <= kPhiCap;   // (synchronizes)
    const int cx_n = P.gdim[k][0], cy_n = P.gdim[k][1];
    const int st = 1 << k, sk = p.phi_s[k];
    const T *lph = lphi + p.phi_off[k] + sk;                 // lph[m], |m| <= sk
    const double *gph = p.phi + p.phi_off[k] + sk;
    auto w = [&](int m) { return lds_phi ? lph[m] : T(gph[m]); };
    // x: tmp[y][cx]
    for (int e = tid; e < fy_n * cx_n; e += kXYThreads) {
        const int y = e / cx_n, cx = e - y * cx_n;
        const int c = st * (cx + P.gorg[k][0]);                 // 2^k C in absolute level-0 index
        const int x0 = max(c - sk - gx0, 0), x1 = min(c + sk - gx0, fx_n - 1);
        T acc = 0;
#pragma unroll 4
        for (int x = x0; x <= x1; ++x) acc += w(x + gx0 - c) * plane[y * fx_n + x];
        tmp[e] = acc;
    }
    __syncthreads();
    // y: into the scratch
    T *out = tscr + P.toff[k] + (int64_t)fz * cy_n * cx_n;
    for (int e = tid; e < cy_n * cx_n; e += kXYThreads) {
        const int cy = e / cx_n, cx = e - cy * cx_n;
        const int c = st * (cy + P.gorg[k][1]);
        const int y0 = max(c - sk - gy0, 0), y1 = min(c + sk - gy0, fy_n - 1);
        T acc = 0;
#pragma unroll 4
        for (int y = y0; y <= y1; ++y) acc += w(y + gy0 - c) * tmp[y * cx_n + cx];
        out[e] = acc;
    }
}

// level of a node of the flat range over levels >= 1, and its index in that level
__device__ inline int level_of(const DevPlan &p, int64_t &g)
{
    int k = 1;
    while (k + 1 < kMaxLevels && g >= p.nnodes[k]) {
        g -= p.nnodes[k];
        ++k;
    }
    return k;
}

// restriction, z: one thread per node of every level >= 1
template <typename T>
__global__ __launch_bounds__(kZThreads) void k_restrict_z(DevPlan p, const T *__restrict__ tscr, T *__restrict__ qgrid)
{
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= p.nrz) return;
    const int k = level_of(p, g);
    const int64_t *pref = p.node_prefix + (int64_t)k * (p.nsys + 1);
    const int s = find_segment(pref, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int loc = (int)(g - pref[s]);
    const int cx_n = P.gdim[k][0], cy_n = P.gdim[k][1];
    const int cx = loc % cx_n, cy = (loc / cx_n) % cy_n, cz = loc / (cx_n * cy_n);
    const int st = 1 << k, sk = p.phi_s[k];
    const double *gph = p.phi + p.phi_off[k] + sk;
    const int gz0 = P.gorg[0][2], fz_n = P.gdim[0][2];
    const int c = st * (cz + P.gorg[k][2]);
    const int z0 = max(c - sk - gz0, 0), z1 = min(c + sk - gz0, fz_n - 1);
    const T *src = tscr + P.toff[k] + (int64_t)cy * cx_n + cx;
    const int64_t plane = (int64_t)cy_n * cx_n;
    // the terms in z order; each batch's weights and values are loaded together
    T acc = 0;
    for (int zb = z0; zb <= z1; zb += kZBatch) {
        // indices past the range repeat the last term's (valid addresses, no
        // branches between the loads); those terms are not added
        T v[kZBatch];
        double wt[kZBatch];
#pragma unroll
        for (int j = 0; j < kZBatch; ++j) {
            const int z = min(zb + j, z1);
            v[j] = src[z * plane];
            wt[j] = gph[z + gz0 - c];
        }
#pragma unroll
        for (int j = 0; j < kZBatch; ++j)
            if (zb + j <= z1) acc += T(wt[j]) * v[j];
    }
    const int CX = padded_x(cx_n), CY = padded_x(cy_n);
    qgrid[P.qoff[k] + ((int64_t)(cz + kGridPad) * CY + (cy + kGridPad)) * CX + (cx + kGridPad)] = acc;
}

// prolongation, x and y: block = (system, level k >= 1, level-k z-plane cz):
// wscr_k[cz][fy][fx] = sum_{cy,cx} phi_k(fy - 2^k cy) phi_k(fx - 2^k cx) u^{k,cutoff}[cz][cy][cx]
template <typename T>
__global__ __launch_bounds__(kXYThreads) void k_prolong_xy(DevPlan p, const T *__restrict__ ucut, T *__restrict__ wscr)
{
    __shared__ T plane[kPlaneCap];
    __shared__ T tmp[kTmpCap];
    __shared__ T lphi[kPhiCap];
    const bool lds_phi = stage_phi<T>(p, lphi) <= kPhiCap;
    const int64_t blk = blockIdx.x;
    const int s = find_segment(p.pxy_prefix, p.nsys, blk);
    const SysPlan &P = p.sys[s];
    int r = (int)(blk - p.pxy_prefix[s]);
    int k = 1;
    while (r >= P.gdim[k][2]) {
        r -= P.gdim[k][2];
        ++k;
    }
    const int cz = r;
    const int cx_n = P.gdim[k][0], cy_n = P.gdim[k][1];
    const int fx_n = P.gdim[0][0], fy_n = P.gdim[0][1];
    const int st = 1 << k, sk = p.phi_s[k];
    const T *lph = lphi + p.phi_off[k] + sk;
    const double *gph = p.phi + p.phi_off[k] + sk;
    auto w = [&](int m) { return lds_phi ? lph[m] : T(gph[m]); };
    const T *src = ucut + P.uoff[k] + (int64_t)cz * cy_n * cx_n;
    const int tid = threadIdx.x;
    for (int e = tid; e < cy_n * cx_n; e += kXYThreads) plane[e] = src[e];
    __syncthreads();
    // x: tmp[cy][fx]
    for (int e = tid; e < cy_n * fx_n; e += kXYThreads) {
        const int cy = e / fx_n, fx = e - cy * fx_n;
        const int f = fx + P.gorg[0][0];                            // absolute level-0 index
        const int c0 = max((f - sk + st - 1) >> k, P.gorg[k][0]);   // floor division by 2^k
        const int c1 = min((f + sk) >> k, P.gorg[k][0] + cx_n - 1);
        T acc = 0;
#pragma unroll 4
        for (int c = c0; c <= c1; ++c) acc += w(f - st * c) * plane[cy * cx_n + (c - P.gorg[k][0])];
        tmp[e] = acc;
    }
    __syncthreads();
    // y: into the scratch
    T *out = wscr + P.woff[k] + (int64_t)cz * fy_n * fx_n;
    for (int e = tid; e < fy_n * fx_n; e += kXYThreads) {
        const int fy = e / fx_n, fx = e - fy * fx_n;
        const int f = fy + P.gorg[0][1];
        const int c0 = max((f - sk + st - 1) >> k, P.gorg[k][1]);
        const int c1 = min((f + sk) >> k, P.gorg[k][1] + cy_n - 1);
        T acc = 0;
#pragma unroll 4
        for (int c = c0; c <= c1; ++c) acc += w(f - st * c) * tmp[(c - P.gorg[k][1]) * fx_n + fx];
        out[e] = acc;
    }
}

// prolongation, z, and the sum over levels: one thread per level-0 node
template <typename T>
__global__ __launch_bounds__(kZThreads) void k_prolong_z(DevPlan p, const T *__restrict__ ucut, const T *__restrict__ wscr,
                                                   T *__restrict__ ugrid)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= p.nnodes[0]) return;
    const int64_t *pref = p.node_prefix;   // level 0
    const int s = find_segment(pref, p.nsys, g);
    const SysPlan &P = p.sys[s];
    const int loc = (int)(g - pref[s]);
    const int fx_n = P.gdim[0][0], fy_n = P.gdim[0][1];
    const int fx = loc % fx_n, fy = (loc / fx_n) % fy_n, fz = loc / (fx_n * fy_n);
    const int f = fz + P.gorg[0][2];
    const int64_t plane = (int64_t)fy_n * fx_n;
    T acc = 0;
    for (int k = 1; k < P.nlev; ++k) {
        const int st = 1 << k, sk = p.phi_s[k];
        const double *gph = p.phi + p.phi_off[k] + sk;
        // level-k planes c with |f - 2^k c| <= s_k (arithmetic shifts: floor division by 2^k)
        const int c0 = max((f - sk + st - 1) >> k, P.gorg[k][2]);
        const int c1 = min((f + sk) >> k, P.gorg[k][2] + P.gdim[k][2] - 1);
        const T *src = wscr + P.woff[k] + (int64_t)fy * fx_n + fx;
        // the terms in plane order; each batch's weights and values are loaded together
        for (int cb = c0; cb <= c1; cb += kZBatch) {
            T v[kZBatch];
            double wt[kZBatch];
#pragma unroll
            for (int j = 0; j < kZBatch; ++j) {
                const int c = min(cb + j, c1);   // as in the restriction: valid, not added
                v[j] = src[(c - P.gorg[k][2]) * plane];
                wt[j] = gph[f - st * c];
            }
#pragma unroll
            for (int j = 0; j < kZBatch; ++j)
                if (cb + j <= c1) acc += T(wt[j]) * v[j];
        }
    }
    const int64_t o = P.uoff[0] + loc;
    ugrid[o] = ucut[o] + acc;
}

// ---------------------------------------------------------------------------
// Interpolation (Section 3): u_i^long = sum_mu phi^0_mu(r_i) u^0_mu, with the
// analytic gradient, and the combination into the outputs:
// phi_i = k (u_i^short + u_i^long - q_i gamma(0)/a), F_i = k q_i (b_i - grad u_i^long),
// written in the caller's atom order; each block also adds up q_i phi_i in
// double for the energy, in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kInterpThreads = 256;

// GRID: add the grid part; SHORT: add the short-range pair part that the
// pair kernel left in shrt, and, with a molecular model bound, the
// Lennard-Jones force and energy of the atoms that carry it (ljof: input
// atom -> index into ljout, or -1; null without a model).
// least waves per SIMD the compiler fits the interpolation kernel to: the
// single precision cubic form in 128 registers (4 waves instead of 3, its 16
// row loads still issued together); the others as they come (fewer registers
// would spill)
template <typename T, int PD> constexpr int interp_waves() { return sizeof(T) == 4 && PD == 3 ? 4 : 1; }

template <typename T, bool GRID, bool SHORT, int PD>
__global__ __launch_bounds__(kInterpThreads) __attribute__((amdgpu_waves_per_eu(interp_waves<T, PD>()))) void k_interp(DevPlan p, const vec4_t<T> *__restrict__ sx,
                                                           const vec4_t<T> *__restrict__ shrt,
                                                           const int *__restrict__ order,
                                                           const T *__restrict__ ugrid, T *__restrict__ forces,
                                                           T *__restrict__ potentials, double *__restrict__ eparts,
                                                           T ke, T self, const int *__restrict__ ljof,
                                                           const vec4_t<T> *__restrict__ ljout)
{
    __shared__ double wpart[kInterpThreads / kWave];
    const int64_t blk = blockIdx.x;
    // every stage that reads the failure flag has run (the pair sum joins
    // before interpolation): clear it for the next evaluation
    if (blk == 0 && threadIdx.x == 0 && p.evflag) *p.evflag = 0;
    const int s = find_segment(p.iblk_prefix, p.nsys, blk);
    const SysPlan &P = p.sys[s];
    const int64_t pos = P.atom0 + (blk - p.iblk_prefix[s]) * kInterpThreads + threadIdx.x;
    double e = 0;
    if (pos < P.atom0 + P.natoms) {
        const vec4_t<T> a = sx[pos];
        T ul = 0, gx = 0, gy = 0, gz = 0;
        if (GRID) {
            // the nodes base-(S-1) .. base+S of each axis
            using B = Basis<PD>;
            constexpr int S = B::S, W = 2 * S;
            const T inv_h = T(P.inv_h);
            const T t[3] = {(a.x - T(P.lo[0])) * inv_h, (a.y - T(P.lo[1])) * inv_h, (a.z - T(P.lo[2])) * inv_h};
            T w[3][W], dw[3][W];
            int base[3];
            for (int d = 0; d < 3; ++d) {
                base[d] = cell_floor(t[d], P.nc[d]) - (S - 1);
#pragma unroll
                for (int m = 0; m < W; ++m) {
                    const T o = t[d] - T(base[d] + m);
                    if constexpr (PD == 3) {
                        // node m of the four lies at |o| in [1, 2] (m = 0, 3) or
                        // [0, 1] (m = 1, 2) from the atom, o < 0 for m = 2, 3:
                        // a fixed piece of the cubic and of its derivative
                        const T x = m < 2 ? o : -o;
                        T v, dv;
                        if (m == 1 || m == 2) {
                            v = T(1) + x * x * (T(-2.5) + T(1.5) * x);
                            dv = x * (T(-5) + T(4.5) * x);
                        } else {
                            const T u = T(2) - x;
                            v = T(-0.5) * (x - T(1)) * u * u;
                            dv = T(-0.5) * u * (T(4) - T(3) * x);
                        }
                        w[d][m] = v;
                        dw[d][m] = (m < 2 ? dv : -dv) * inv_h;
                    } else {
                        w[d][m] = B::phi(o);
                        dw[d][m] = B::dphi(o) * inv_h;
                    }
                }
            }
            const int dx = P.gdim[0][0], dy = P.gdim[0][1];
            const T *u0 = ugrid + P.uoff[0];
            for (int mz = 0; mz < W; ++mz) {
                for (int my = 0; my < W; ++my) {
                    const T *row = u0 + ((int64_t)(base[2] + mz - P.gorg[0][2]) * dy + (base[1] + my - P.gorg[0][1])) * dx +
                                   (base[0] - P.gorg[0][0]);
                    T sx0 = 0, sdx = 0;
#pragma unroll
                    for (int mx = 0; mx < W; ++mx) {
                        const T v = row[mx];
                        sx0 += w[0][mx] * v;
                        sdx += dw[0][mx] * v;
                    }
                    const T wyz = w[1][my] * w[2][mz];
                    ul += wyz * sx0;
                    gx += wyz * sdx;
                    gy += dw[1][my] * w[2][mz] * sx0;
                    gz += w[1][my] * dw[2][mz] * sx0;
                }
            }
        }
        vec4_t<T> sr;
        sr.x = sr.y = sr.z = sr.w = T(0);
        if (SHORT) sr = shrt[pos];
        const T phi = ke * (sr.w + ul - a.w * self);
        const int64_t o = order[pos];
        if (potentials) potentials[o] = phi;
        vec4_t<T> lj;
        lj.x = lj.y = lj.z = lj.w = T(0);
        if (SHORT && ljof && !eval_failed(p)) {
            const int li = ljof[o];
            if (li >= 0) lj = ljout[li];
        }
        if (forces) {
            const T kq = ke * a.w;
            forces[3 * o + 0] = kq * (sr.x - gx) + lj.x;
            forces[3 * o + 1] = kq * (sr.y - gy) + lj.y;
            forces[3 * o + 2] = kq * (sr.z - gz) + lj.z;
        }
        e = (double)a.w * (double)phi + (double)lj.w;
    }
    e = block_sum<kInterpThreads>(e, wpart);
    if (threadIdx.x == 0) eparts[blk] = e;
}

// Per-system sum of block partials times `scale` (the energy U = 1/2 sum_i
// q_i phi_i uses 1/2): one workgroup per system, each thread a fixed stride of
// partials, then a fixed order across lanes and waves, so the result does not
// depend on timing.
__global__ __launch_bounds__(256) void k_energy(DevPlan p, const double *__restrict__ eparts,
                                                double *__restrict__ energy, double scale)
{
    __shared__ double wpart[256 / kWave];
    const int s = blockIdx.x;
    double acc = 0;
    for (int64_t b = p.iblk_prefix[s] + threadIdx.x; b < p.iblk_prefix[s + 1]; b += 256) acc += eparts[b];
    acc = block_sum<256>(acc, wpart);
    if (threadIdx.x == 0) energy[s] = scale * acc;
}

template <typename T>
__global__ void k_stage_atoms(const SysPlan *sys, int s, const vec4_t<T> *__restrict__ shrt,
                              const int *__restrict__ order, double *u_short, double *f_short)
{
    const SysPlan &P = sys[s];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= P.natoms) return;
    const int64_t pos = P.atom0 + i;
    const int64_t o = order[pos] - P.atom0;
    const vec4_t<T> v = shrt[pos];
    if (u_short) u_short[o] = (double)v.w;
    if (f_short) {
        f_short[3 * o] = (double)v.x;
        f_short[3 * o + 1] = (double)v.y;
        f_short[3 * o + 2] = (double)v.z;
    }
}

template <typename T>
__global__ void k_stage_grid(const SysPlan *sys, int s, int k, const T *__restrict__ src, int padded,
                             double *__restrict__ dst)
{
    const SysPlan &P = sys[s];
    const int dx = P.gdim[k][0], dy = P.gdim[k][1], dz = P.gdim[k][2];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)dx * dy * dz) return;
    const int x = (int)(i % dx), y = (int)((i / dx) % dy), z = (int)(i / ((int64_t)dx * dy));
    if (padded) {
        const int PX = padded_x(dx), PY = padded_x(dy);
        dst[i] = (double)src[P.qoff[k] + ((int64_t)(z + kGridPad) * PY + (y + kGridPad)) * PX + (x + kGridPad)];
    } else {
        dst[i] = (double)src[P.uoff[k] + i];
    }
}

}  // namespace

int anterp_tiles(int dx, int dy, int dz, int depth)
{
    return ((dx + kAntX - 1) / kAntX) * ((dy + kAntY - 1) / kAntY) * ((dz + depth - 1) / depth);
}

// The tiles stage at least twice as many atoms as their region has cells
// (2,048 for the cubic's 847 cells, 3,072 or 4,096 for the quintic's 1,521):
// above about 2 atoms per cell on average, many would overflow to the global
// gather.
bool anterp_two_pass(const DevPlan &p) { return p.natoms > 2 * p.ncells; }

template <typename T, int PD> static hipError_t anterp_p(hipStream_t s, const DevPlan &p, const Work<T> &w)
{
    if (!anterp_two_pass(p)) {
        if constexpr (sizeof(T) == 4 && PD == 3) {
            if (p.ant_depth == 8) {
                hipLaunchKernelGGL((k_anterp<T, PD, 8>), dim3((unsigned)p.nant), dim3(ant_threads<PD, 8>()), 0, s, p,
                                   w.sxyzq, w.cell_start, w.qgrid);
                return hipGetLastError();
            }
        }
        if (p.ant_depth == 4)
            hipLaunchKernelGGL((k_anterp<T, PD, 4>), dim3((unsigned)p.nant), dim3(ant_threads<PD, 4>()), 0, s, p,
                               w.sxyzq, w.cell_start, w.qgrid);
        else
            return hipErrorInvalidValue;   // a plan whose tiles no kernel form has
        return hipGetLastError();
    }
    constexpr int cpb = ant_cells_per_block<PD>();
    if (p.ncells > 0)
        hipLaunchKernelGGL((k_anterp_cells<T, PD>), dim3((unsigned)((p.ncells + cpb - 1) / cpb)), dim3(256), 0, s, p,
                           w.sxyzq, w.cell_start, w.apart);
    hipLaunchKernelGGL((k_anterp_nodes<T, PD>), dim3(nblocks(p.nnodes[0], 256)), dim3(256), 0, s, p, w.apart,
                       w.qgrid);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::anterp(hipStream_t s, const DevPlan &p, const Work<T> &w, const MethodConst &m)
{
    if (p.nnodes[0] == 0) return hipSuccess;   // no grids (simple cutoff method)
    return m.p == 5 ? anterp_p<T, 5>(s, p, w) : anterp_p<T, 3>(s, p, w);
}

template <typename T>
hipError_t Launch<T>::restrict_level(hipStream_t s, const DevPlan &p, const Work<T> &w, int k, const MethodConst &m)
{
    if (p.nnodes[k + 1] == 0) return hipSuccess;
    if (m.p == 5)
        hipLaunchKernelGGL((k_restrict<T, 5>), dim3(nblocks(p.nnodes[k + 1], 256)), dim3(256), 0, s, p, w.qgrid, k);
    else
        hipLaunchKernelGGL((k_restrict<T, 3>), dim3(nblocks(p.nnodes[k + 1], 256)), dim3(256), 0, s, p, w.qgrid, k);
    return hipGetLastError();
}

template <typename T, int R>
static hipError_t stencil_r(hipStream_t s, const DevPlan &p, const Work<T> &w, const StencilTables<T> &tb,
                            const TopArgs &top)
{
    const dim3 grid((unsigned)(p.ntiles + top.nblocks));
    if (tb.threads == 256) {
        hipLaunchKernelGGL((k_stencil<T, R, 256>), grid, dim3(256), 0, s, p, w.qgrid, w.ucut, tb.cols, tb.w,
                           tb.ncols, w.ugrid, top);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_stencil<T, R, 1024>), grid, dim3(1024), 0, s, p, w.qgrid, w.ucut, tb.cols, tb.w, tb.ncols,
                       w.ugrid, top);
    return hipGetLastError();
}

// The lattice cutoff of every level below the top, with the top level's
// blocks in the same launch; the top alone when there are no tiles.
template <typename T>
hipError_t Launch<T>::stencil(hipStream_t s, const DevPlan &p, const Work<T> &w, const StencilTables<T> &tb,
                              const MethodConst &m)
{
    TopArgs top{m.h, m.a, p.top_d2 + 1, p.ntop, m.g};
    if (p.ntiles == 0) {
        if (p.ntop == 0) return hipSuccess;
        hipLaunchKernelGGL(k_top<T>, dim3((unsigned)p.ntop), dim3(kTopThreads), 0, s, p, w.qgrid, w.ucut, w.ugrid,
                           m.h, m.a, p.top_d2 + 1, m.g);
        return hipGetLastError();
    }
    switch (tb.reach) {
    case 1: return stencil_r<T, 1>(s, p, w, tb, top);
    case 2: return stencil_r<T, 2>(s, p, w, tb, top);
    case 3: return stencil_r<T, 3>(s, p, w, tb, top);
    case 4: return stencil_r<T, 4>(s, p, w, tb, top);
    case 5: return stencil_r<T, 5>(s, p, w, tb, top);
    case 6: return stencil_r<T, 6>(s, p, w, tb, top);
    case 7: return stencil_r<T, 7>(s, p, w, tb, top);
    case 8: return stencil_r<T, 8>(s, p, w, tb, top);
    case 9: return stencil_r<T, 9>(s, p, w, tb, top);
    case 10: return stencil_r<T, 10>(s, p, w, tb, top);
    case 11: return stencil_r<T, 11>(s, p, w, tb, top);
    default: return hipErrorInvalidValue;
    }
}

int top_blocks(int nodes) { return (nodes + kTopNodes - 1) / kTopNodes; }

int stencil_tile_xy(int elem_bytes, int reach) { return (elem_bytes == 8 && reach >= 10) ? 4 : kStencilTile; }
int stencil_tile_z(int elem_bytes, int reach) { return (elem_bytes == 8 && reach >= 10) ? 4 : kStencilTile; }

template <typename T>
hipError_t Launch<T>::prolong_level(hipStream_t s, const DevPlan &p, const Work<T> &w, int k, const MethodConst &m)
{
    if (p.nnodes[k] == 0) return hipSuccess;
    if (m.p == 5)
        hipLaunchKernelGGL((k_prolong<T, 5>), dim3(nblocks(p.nnodes[k], 256)), dim3(256), 0, s, p, w.ucut, w.ugrid, k);
    else
        hipLaunchKernelGGL((k_prolong<T, 3>), dim3(nblocks(p.nnodes[k], 256)), dim3(256), 0, s, p, w.ucut, w.ugrid, k);
    return hipGetLastError();
}

template <typename T> hipError_t Launch<T>::restrict_all(hipStream_t s, const DevPlan &p, const Work<T> &w)
{
    if (p.nrxy == 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict_xy<T>, dim3((unsigned)p.nrxy), dim3(kXYThreads), 0, s, p, w.qgrid, w.tscr);
    hipLaunchKernelGGL(k_restrict_z<T>, dim3(nblocks(p.nrz, kZThreads)), dim3(kZThreads), 0, s, p, w.tscr, w.qgrid);
    return hipGetLastError();
}

template <typename T> hipError_t Launch<T>::prolong_all(hipStream_t s, const DevPlan &p, const Work<T> &w)
{
    if (p.npxy == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prolong_xy<T>, dim3((unsigned)p.npxy), dim3(kXYThreads), 0, s, p, w.ucut, w.wscr);
    hipLaunchKernelGGL(k_prolong_z<T>, dim3(nblocks(p.nnodes[0], kZThreads)), dim3(kZThreads), 0, s, p, w.ucut, w.wscr,
                       w.ugrid);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::interp(hipStream_t s, const DevPlan &p, const Work<T> &w, const MethodConst &m, T *forces,
                             T *potentials, int part)
{
    if (p.niblk == 0) return hipSuccess;
    const int *ljof = w.lj.x ? w.lj.pos_of : nullptr;
    const vec4_t<T> *ljout = w.lj_out;
    const dim3 grid((unsigned)p.niblk), block(kInterpThreads);
    if (m.cutoff) {
        // no grid potential; the simple cutoff has no self term, Wolf's is
        // 2 C q_i in phi_i with C = erfc(alpha a)/(2a) + alpha/sqrt(pi)
        const double c_wolf = std::erfc(m.alpha * m.a) / (2.0 * m.a) + m.alpha / std::sqrt(std::acos(-1.0));
        const T self_nogrid = m.method == MSM_METHOD_WOLF ? T(2.0 * c_wolf) : T(0);
        hipLaunchKernelGGL((k_interp<T, false, true, 3>), grid, block, 0, s, p, w.sxyzq, w.shrt, w.order,
                           (const T *)nullptr, forces, potentials, w.eparts, T(m.ke), self_nogrid, ljof, ljout);
        return hipGetLastError();
    }
    // the smooth self term gamma(0)/a goes with the grid part
    const T self = part == 1 ? T(0) : T(m.g.c[0] / m.a);
    const T *ug = w.ugrid;
    const T ke = T(m.ke);
#define MSMX_INTERP(G, S, P)                                                                                        \
    hipLaunchKernelGGL((k_interp<T, G, S, P>), grid, block, 0, s, p, w.sxyzq, w.shrt, w.order, ug, forces,          \
                       potentials, w.eparts, ke, self, ljof, ljout)
    if (part == 1)
        MSMX_INTERP(false, true, 3);
    else if (part == 2 && m.p == 5)
        MSMX_INTERP(true, false, 5);
    else if (part == 2)
        MSMX_INTERP(true, false, 3);
    else if (m.p == 5)
        MSMX_INTERP(true, true, 5);
    else
        MSMX_INTERP(true, true, 3);
#undef MSMX_INTERP
    return hipGetLastError();
}

hipError_t reduce_blocks(hipStream_t s, const DevPlan &p, const double *parts, double *out, double scale)
{
    if (!out) return hipSuccess;
    hipLaunchKernelGGL(k_energy, dim3((unsigned)p.nsys), dim3(256), 0, s, p, parts, out, scale);
    return hipGetLastError();
}

template <typename T> hipError_t Launch<T>::energy(hipStream_t s, const DevPlan &p, const Work<T> &w, double *energy)
{
    return reduce_blocks(s, p, w.eparts, energy, 0.5);
}

template <typename T>
hipError_t Launch<T>::stage_copy(hipStream_t s, const DevPlan &p, const Work<T> &w, int sys, double *u_short,
                                 double *f_short, double *const *qg, double *const *ucut, double *const *ug)
{
    // host copy of the plan of this system, for the launch sizes
    SysPlan P;
    hipError_t e = hipMemcpyAsync(&P, p.sys + sys, sizeof(SysPlan), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if ((u_short || f_short) && P.natoms > 0)
        hipLaunchKernelGGL(k_stage_atoms<T>, dim3(nblocks(P.natoms, 256)), dim3(256), 0, s, p.sys, sys, w.shrt,
                           w.order, u_short, f_short);
    for (int k = 0; k < P.nlev; ++k) {
        const int64_t n = (int64_t)P.gdim[k][0] * P.gdim[k][1] * P.gdim[k][2];
        if (qg && qg[k])
            hipLaunchKernelGGL(k_stage_grid<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, p.sys, sys, k, w.qgrid, 1, qg[k]);
        if (ucut && ucut[k])
            hipLaunchKernelGGL(k_stage_grid<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, p.sys, sys, k, w.ucut, 0, ucut[k]);
        if (ug && ug[k])
            hipLaunchKernelGGL(k_stage_grid<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, p.sys, sys, k, w.ugrid, 0, ug[k]);
    }
    return hipGetLastError();
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace msmx
