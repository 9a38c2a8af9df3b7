// Host-side launchers of the HIP kernels (one translation unit per kernel
// family); every launcher enqueues on the given stream and returns the launch
// status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "../../include/msm.h"

namespace msmx {

// Read-only tables of one evaluation, resident in device memory.
struct DevPlan {
    const SysPlan *sys;          // nsys plans
    int nsys;
    const int64_t *atom_prefix;  // nsys+1: atom offsets
    const int64_t *group_prefix; // nsys+1: 64-atom pair groups
    const int64_t *cell_prefix;  // nsys+1: brick-major cells
    const int64_t *node_prefix;  // kMaxLevels x (nsys+1): level-k nodes per system
    const int64_t *iblk_prefix;  // nsys+1: interpolation blocks per system
    const int64_t *tile_prefix;  // ntile_seg+1: stencil tiles of segment k*nsys + s (levels below the top)
    const int64_t *top_prefix;   // nsys+1: top-level workgroups per system
    const int64_t *ant_prefix;   // nsys+1: anterpolation tiles per system
    int ant_depth;               // node layers along z per anterpolation tile: 4 or 8
    int ntile_seg;               // (maxlev - 1) * nsys
    int top_d2;                  // largest squared index distance on any top grid
    int64_t natoms, ngroups, ncells, niblk, ntop, ntiles, nant;
    int64_t nnodes[kMaxLevels];  // level-k nodes over the batch
    int maxlev;                  // largest level count in the batch
    // composite transfers (all levels at once; composite = 0: one launch per level)
    int composite;
    const double *phi;           // composite filters: phi_k(m) at phi[phi_off[k] + m + phi_s[k]], |m| <= phi_s[k]
    int phi_off[kMaxLevels], phi_s[kMaxLevels];
    const int64_t *rxy_prefix;   // nsys+1: level-0 z-planes x levels >= 1 (restriction xy blocks)
    const int64_t *pxy_prefix;   // nsys+1: z-planes of levels >= 1 (prolongation xy blocks)
    int64_t nrxy, npxy, nrz;     // those block counts, and the nodes of levels >= 1
    // set by binning when this evaluation has an atom outside its domain or a
    // non-finite value (its results are undefined), cleared by interpolation
    int *evflag;
};

// The evaluation's results are undefined (see DevPlan::evflag): the stages
// whose cost grows with the atoms piled into one cell skip their work, so a
// diverging trajectory fails at the cost of an ordinary step.
__device__ inline bool eval_failed(const DevPlan &p) { return p.evflag && *p.evflag; }

// A second binning of the atoms of the batch plan p into the cells of plan pl:
// every atom (maux null) or those whose model record carries Lennard-Jones.
template <typename T> struct SubBins {
    int *cell_of;     // per input atom: its cell, or -1
    int *slot_of;     // per input atom: arrival slot within that cell
    int *cnt;         // cells + 1: histogram, zero between evaluations
    int *start;       // cells + 1: cell starts
    int *blocks;      // block sums of that scan
    int *order;       // sorted position -> input atom
    int *pos_of;      // input atom -> sorted position, or -1
    vec4_t<T> *x;     // sorted positions and charges
    vec4_t<T> *aux;   // sorted model records (null: not gathered)
};

// Scratch arrays owned by the context.
template <typename T> struct Work {
    int *cell_of;        // per input atom: brick-major cell (batch-global)
    int *slot_of;        // per input atom: arrival slot within its cell
    int *cell_start;     // ncells + 1: exclusive scan of cell counts
    int *counts;         // ncells + 1: cell histogram, zero between evaluations
    int *scan_blocks;    // block sums of the scan
    int *order;          // sorted position -> input atom
    vec4_t<T> *sxyzq;    // atoms in sorted order
    vec4_t<T> *shrt;     // sorted order: (bracket of F^short, u^short)
    int *cluster;        // per 64-atom pair group: its atoms in k-d cluster order (sorted index, -1 absent)
    T *apart;            // ncells x 64: each cell's partial charges on its 4x4x4 support nodes
    T *qgrid;            // padded charge grids, all levels and systems
    T *ucut;             // lattice-cutoff potentials (top level: u^{l-1})
    T *ugrid;            // prolongated potentials u^k
    T *tscr;             // composite restriction: per level, level-0 z-planes x level-k (y, x)
    T *wscr;             // composite prolongation: per level, level-k z-planes x level-0 (y, x)
    double *eparts;      // per interpolation block: sum q_i phi_i
    int *status;         // device status word; status[1]: the current evaluation's failure flag
    // dynamics model (null when no model is bound)
    vec4_t<T> *maux;     // per model atom: (molecule id bits, sigma/2, sqrt(eps), 0)
    vec4_t<T> *saux;     // sorted copy of maux
    int64_t period;      // batch atom i uses model entry i % period
    int *xstart, *xidx;  // excluded partners of model atom m: xidx[xstart[m] .. xstart[m+1]) (model
                         // indices, ascending); null without molecule ids
    // the atoms that carry Lennard-Jones, binned into cells of their own (the
    // subset plan's); lj.x null when no atom carries it
    SubBins<T> lj;
    int lj_one;          // one Lennard-Jones type (lj_sigma, lj_eps) and at most one such atom per molecule
    double lj_sigma, lj_eps;
    int *lj_cluster;     // the subset's k-d clusters
    vec4_t<T> *lj_out;   // subset: Lennard-Jones force and energy (counted from both sides)
    // pair search in cells finer than h (null unless tuned so): every atom binned
    // a second time, the pair sums in that order, then permuted into shrt
    SubBins<T> pc;
    vec4_t<T> *pc_out;
    // the Newton's third law pair form (single precision): per sorted atom the
    // fixed-point sums (unit 2^-32) of the contributions it received as a
    // candidate, components x, y, z, u at nacc[c * nacc_stride + atom]; zero
    // between evaluations (null until that form is chosen)
    unsigned long long *nacc;
    int64_t nacc_stride;
};

// Quarter-disc stencil columns (ox >= 0, oy >= 0 inside the sphere) and their
// 2R+1 weights g^0(h |o|) along z.
template <typename T> struct StencilTables {
    const int2 *cols;
    const T *w;
    int ncols;
    int reach;
    int threads;         // threads per tile: 256 or 1024
};

int stencil_tile_xy(int elem_bytes, int reach);
int top_blocks(int nodes);
int stencil_tile_z(int elem_bytes, int reach);

struct MethodConst {
    double a, h, ke;
    int method;                // MSM_METHOD_MSM, _CUTOFF or _WOLF
    int cutoff;                // 1: no grids (the simple cutoff method or Wolf summation)
    double alpha;              // Wolf damping (1/nm)
    Smooth g;                  // smoothing function gamma of order g.m
    int p;                     // degree of the nodal basis Phi: 3 or 5
    int reach;                 // stencil reach R: largest integer with R < 2a/h
    // Wolf summation in single precision: kWolfPieces cubic pieces on [0, a)
    // of E(r) = erfc(alpha r) and D(r) = E(r) + (2 alpha r / sqrt(pi)) exp(-alpha^2 r^2),
    // two float4 per piece (E, then D), in device memory
    const float4 *wolf_tab;
    int pair_waves;            // waves per 64-atom group in the pair kernel: 4, 8 or 16; 1: 16-atom sub-groups;
                               // 2: 8-atom clusters with bounding-box candidate filtering;
                               // 3: two such clusters per wave sharing one candidate stream;
                               // 5, 6: one 16-atom (5) or 32-atom (6) cluster per wave;
                               // 7, 9: as 2, the clusters of a group (7) or half group (9)
                               // sharing one stream built and loaded by the workgroup;
                               // 10: as 2, each pair evaluated once (Newton's third law), single precision
    int stencil_threads;       // threads per stencil tile: 256 or 1024
    int pair_cell;             // the pair search's cells: edge h / pair_cell (1: the grid cells)
};

// Pieces of the single-precision Wolf pair table (see MethodConst::wolf_tab).
constexpr int kWolfPieces = 128;
// Coefficients c0..c3 of each piece in its local coordinate u in [0, 1):
// f(r_k + u a / kWolfPieces) = c0 + u (c1 + u (c2 + u c3)), from the values
// and derivatives of f at the piece ends (cubic Hermite); out holds
// 8 * kWolfPieces floats.
void wolf_table(double a, double alpha, float *out);

// anterpolation tiles of a level-0 grid, 8 x 8 x depth nodes each (depth 4,
// or 8 for the single precision cubic basis on grids of at least kAntDeep
// tiles of that depth over the batch)
int anterp_tiles(int dx, int dy, int dz, int depth);
constexpr int64_t kAntDeep = 1024;
// composite transfers: LDS capacity (elements) of a level-0 xy plane and of
// the one-axis partial sums
constexpr int kPlaneCap = 6144;
constexpr int kTmpCap = 4096;
bool anterp_two_pass(const DevPlan &p);   // anterpolation by cell partials (crowded cells) rather than tiles

// exclusive scan of the cell counts: threads per block, and the largest block
// count of the four-counts-per-thread form (block sums needed: at most
// max(kScanFewBlocks, (n + 4095) / 4096))
constexpr int kScanThreads = 256;
constexpr int kScanFewBlocks = 256;
int scan_cells(hipStream_t s, int *counts, int *start, int64_t n, int *block_sums);

template <typename T> struct Launch {
    static hipError_t bin(hipStream_t s, const DevPlan &p, const Work<T> &w, const vec4_t<T> *xyzq);
    // pot = false: forces only, the short-range potentials are left at zero;
    // pp: the plan of the pair search's own cells (null: the batch cells)
    static hipError_t pair(hipStream_t s, const DevPlan &p, const DevPlan *pp, const Work<T> &w,
                           const vec4_t<T> *xyzq, const MethodConst &m, bool pot);
    // after pair, with a molecular model bound: take the excluded pairs of each
    // molecule out of the short-range sums (xyzq: the evaluation's input), and
    // the Lennard-Jones forces and energies of the atoms that carry them,
    // binned into the cells of their own plan sub
    static hipError_t exclusions(hipStream_t s, const DevPlan &p, const Work<T> &w, const vec4_t<T> *xyzq,
                                 const MethodConst &m, bool pot);
    static hipError_t lj(hipStream_t s, const DevPlan &p, const DevPlan &sub, const Work<T> &w,
                         const vec4_t<T> *xyzq, const MethodConst &m, bool pot);
    static hipError_t anterp(hipStream_t s, const DevPlan &p, const Work<T> &w, const MethodConst &m);
    static hipError_t restrict_level(hipStream_t s, const DevPlan &p, const Work<T> &w, int k, const MethodConst &m);
    // the lattice cutoff of every level below the top and the top level
    static hipError_t stencil(hipStream_t s, const DevPlan &p, const Work<T> &w, const StencilTables<T> &tb,
                              const MethodConst &m);
    static hipError_t prolong_level(hipStream_t s, const DevPlan &p, const Work<T> &w, int k, const MethodConst &m);
    // every level >= 1 from level 0 / u^0 from every level, by composite filters
    static hipError_t restrict_all(hipStream_t s, const DevPlan &p, const Work<T> &w);
    static hipError_t prolong_all(hipStream_t s, const DevPlan &p, const Work<T> &w);
    // part: 0 everything, 1 the short-range pairs only, 2 the grid part only
    static hipError_t interp(hipStream_t s, const DevPlan &p, const Work<T> &w, const MethodConst &m,
                             T *forces, T *potentials, int part);
    static hipError_t energy(hipStream_t s, const DevPlan &p, const Work<T> &w, double *energy);
    static hipError_t stage_copy(hipStream_t s, const DevPlan &p, const Work<T> &w, int sys,
                                 double *u_short, double *f_short, double *const *qg,
                                 double *const *ucut, double *const *ug);
};

hipError_t fill_i32(hipStream_t s, int *p, int64_t n, int v);
// Lennard-Jones subset cells: an edge that holds about this many of its atoms
// at their mean density (clamped to [h, a])
#ifndef MSMX_LJ_CELL_ATOMS
#define MSMX_LJ_CELL_ATOMS 2.0
#endif
constexpr double kLjCellAtoms = MSMX_LJ_CELL_ATOMS;
template <typename T>
hipError_t bin_sub(hipStream_t s, const DevPlan &p, const DevPlan &pl, const SubBins<T> &b, const vec4_t<T> *xyzq,
                   const vec4_t<T> *maux, int64_t period);
// Copy bytes of host memory to device memory through kernel arguments
// (2 KiB per launch), so that the copy allocates nothing and the source may
// be reused as soon as the call returns. dst and bytes: multiples of 4.
hipError_t put_bytes(hipStream_t s, void *dst, const void *src_host, size_t bytes);
template <typename T> hipError_t fill_t(hipStream_t s, T *p, int64_t n, T v);

}  // namespace msmx
