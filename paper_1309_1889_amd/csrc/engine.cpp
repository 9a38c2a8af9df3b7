// Host side of libmsmx: context, per-call plan of a batch of systems,
// workspace carving, and the launch sequence of one multilevel summation
// evaluation. Implements the msm_* entry points of include/msm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

using namespace msmx;

namespace {

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int64_t floordiv2(int64_t v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }
int64_t ceildiv2(int64_t v) { return -floordiv2(-v); }

// Number of grids (a reading of Section 3): the smallest l for which the
// coarsest spacing 2^(l-1) h spans the domain in at most 4 steps on every axis.
int auto_levels(double h, const double *len)
{
    for (int l = 1; l <= kMaxLevels; l++) {
        bool ok = true;
        for (int d = 0; d < 3; d++)
            if (std::ceil(len[d] / std::ldexp(h, l - 1)) > 4.0) ok = false;
        if (ok) return l;
    }
    return kMaxLevels;
}

int basis_degree(const msm_params &prm) { return prm.basis ? prm.basis : 3; }

int geometry(const msm_params &prm, const double *lo, const double *hi, Geometry &g)
{
    double len[3];
    for (int d = 0; d < 3; d++) {
        len[d] = hi[d] - lo[d];
        if (!(len[d] > 0) || !std::isfinite(len[d])) return MSM_ERR_ARG;
        double ncd = std::floor(len[d] / prm.h) + 1.0;
        if (ncd > 1 << 20) return MSM_ERR_CAPACITY;
        g.nc[d] = (int)ncd;
    }
    if (prm.method != MSM_METHOD_MSM) {   // no grids: cells for the pair search only
        g.nlev = 0;
        return MSM_OK;
    }
    g.nlev = prm.levels > 0 ? prm.levels : auto_levels(prm.h, len);
    if (g.nlev < 1 || g.nlev > kMaxLevels) return MSM_ERR_UNSUPPORTED;
    // level 0: the nodes base-(S-1) .. base+S of every cell; level k+1: the
    // nodes whose restriction window 2 mu -+ (2S-1) meets level k
    const int S = (basis_degree(prm) + 1) / 2, W = 2 * S - 1;
    for (int d = 0; d < 3; d++) {
        int64_t i0 = -(S - 1), i1 = (g.nc[d] - 1) + S;
        for (int k = 0; k < g.nlev; k++) {
            g.gorg[k][d] = (int)i0;
            g.gdim[k][d] = (int)(i1 - i0 + 1);
            i0 = ceildiv2(i0 - W);
            i1 = floordiv2(i1 + W);
        }
    }
    return MSM_OK;
}

struct Sizes {
    int64_t cells, q, u, t, w;
};

// composite-transfer scratch of one system's geometry (elements)
int64_t comp_t(const int gdim[][3], int nlev, int k)
{
    return round_up((int64_t)gdim[0][2] * gdim[k][1] * gdim[k][0], 64);
}
int64_t comp_w(const int gdim[][3], int nlev, int k)
{
    return round_up((int64_t)gdim[k][2] * gdim[0][1] * gdim[0][0], 64);
}

// a system's grids fit the composite transfers' LDS planes
bool comp_fits(const int gdim[][3], int nlev)
{
    if (nlev < 2 || (int64_t)gdim[0][0] * gdim[0][1] > kPlaneCap) return false;
    for (int k = 1; k < nlev; k++) {
        if ((int64_t)gdim[0][1] * gdim[k][0] > kTmpCap || (int64_t)gdim[k][1] * gdim[0][0] > kTmpCap) return false;
        if ((int64_t)gdim[k][1] * gdim[k][0] > kPlaneCap) return false;
    }
    return true;
}

Sizes sizes_of(const Geometry &g)
{
    Sizes s{};
    int64_t nb = 1;
    for (int d = 0; d < 3; d++) nb *= (g.nc[d] + kBrick - 1) / kBrick;
    s.cells = nb * kBrickCells;
    for (int k = 0; k < g.nlev; k++) {
        s.q += round_up((int64_t)padded_x(g.gdim[k][0]) * padded_x(g.gdim[k][1]) * padded_z(g.gdim[k][2]), 64);
        s.u += round_up((int64_t)g.gdim[k][0] * g.gdim[k][1] * g.gdim[k][2], 64);
    }
    if (comp_fits(g.gdim, g.nlev))
        for (int k = 1; k < g.nlev; k++) {
            s.t += comp_t(g.gdim, g.nlev, k);
            s.w += comp_w(g.gdim, g.nlev, k);
        }
    return s;
}

template <typename T> size_t vec_bytes() { return sizeof(vec4_t<T>); }

}  // namespace

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? MSM_OK : MSM_ERR_HIP; }

template <typename T> void carve(msm_ctx *c, Work<T> &w, char *base, size_t *used, bool commit)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    const int64_t na = std::max<int64_t>(c->prm.max_atoms, 1);
    w.cell_of = (int *)take(sizeof(int) * na);
    w.slot_of = (int *)take(sizeof(int) * na);
    w.cell_start = (int *)take(sizeof(int) * (c->cap_cells + 1));
    w.counts = (int *)take(sizeof(int) * (c->cap_cells + 1));
    w.scan_blocks = (int *)take(sizeof(int) * std::max<int64_t>(kScanFewBlocks, (c->cap_cells + 1) / 4096 + 2));
    w.order = (int *)take(sizeof(int) * na);
    w.sxyzq = (vec4_t<T> *)take(vec_bytes<T>() * (na + 64));   // spare tail for the pair prefetch
    w.shrt = (vec4_t<T> *)take(vec_bytes<T>() * na);
    w.cluster = (int *)take(sizeof(int) * (na + (int64_t)kWave * c->prm.max_systems));
    // partial charges per cell for the two-pass anterpolation, which a plan
    // uses only with more than 2 atoms per cell (so fewer cells than
    // max_atoms / 2); none without grids
    const int64_t part_cells = std::min<int64_t>(c->cap_cells, na / 2 + 1);
    const int64_t support = 2 * ((basis_degree(c->prm) + 1) / 2);   // nodes per axis an atom reaches
    w.apart = (T *)take(c->prm.method != MSM_METHOD_MSM ? 0
                                                         : sizeof(T) * support * support * support * part_cells);
    w.qgrid = (T *)take(sizeof(T) * c->cap_q);
    w.ucut = (T *)take(sizeof(T) * c->cap_u);
    w.ugrid = (T *)take(sizeof(T) * c->cap_u);
    w.tscr = (T *)take(sizeof(T) * c->cap_t);
    w.wscr = (T *)take(sizeof(T) * c->cap_w);
    w.eparts = (double *)take(sizeof(double) * c->cap_iblk);
    w.status = (int *)take(sizeof(int) * 64);
    *used = off;
    (void)commit;
}

}  // namespace

// Build the device tables of a batch; returns MSM_OK or an error.
int msmx::build_plan(msm_ctx *c, int nsys, const int64_t *offsets, const double *domains)
{
    if (c->plan_valid && (int)c->last_offsets.size() == nsys + 1 &&
        std::equal(offsets, offsets + nsys + 1, c->last_offsets.begin())) {
        bool same = domains ? (c->last_domains.size() == (size_t)nsys * 6 &&
                               std::equal(domains, domains + nsys * 6, c->last_domains.begin()))
                            : c->last_domains.empty();
        if (same) return MSM_OK;
    }
    if (offsets[0] != 0) return MSM_ERR_ARG;
    for (int s = 0; s < nsys; s++)
        if (offsets[s + 1] < offsets[s]) return MSM_ERR_ARG;
    if (offsets[nsys] > c->prm.max_atoms) return MSM_ERR_CAPACITY;

    // host tables in the context's own vectors: their capacity persists, so
    // a batch shape seen before allocates no host memory
    PlanScratch &ps = c->ps;
    std::vector<SysPlan> &sys = ps.sys;
    sys.resize(nsys);
    const int W = nsys + 1;
    std::vector<int64_t> &atom_p = ps.atom_p, &group_p = ps.group_p, &cell_p = ps.cell_p, &iblk_p = ps.iblk_p,
                         &top_p = ps.top_p, &ant_p = ps.ant_p, &ant_p8 = ps.ant_p8, &node_p = ps.node_p, &rxy_p = ps.rxy_p,
                         &pxy_p = ps.pxy_p, &tile_p = ps.tile_p;
    for (auto *v : {&atom_p, &group_p, &cell_p, &iblk_p, &top_p, &ant_p, &ant_p8, &rxy_p, &pxy_p}) v->assign(W, 0);
    node_p.assign((size_t)kMaxLevels * W, 0);
    int64_t cells = 0, q = 0, u = 0, groups = 0, iblk = 0, top = 0, ant = 0, ant8 = 0;
    int64_t tsz = 0, wsz = 0, rxy = 0, pxy = 0;
    bool composite = true;
    int64_t nodes[kMaxLevels] = {0};
    int maxlev = 1, top_d2 = 0;
    for (int s = 0; s < nsys; s++) {
        const double *lo = domains ? domains + 6 * s : c->prm.lo;
        const double *hi = domains ? domains + 6 * s + 3 : c->prm.hi;
        for (int d = 0; d < 3; d++)
            if (!(hi[d] - lo[d] <= c->prm.hi[d] - c->prm.lo[d] + 1e-12 * std::fabs(c->prm.hi[d] - c->prm.lo[d])))
                return MSM_ERR_CAPACITY;
        Geometry g;
        int rc = geometry(c->prm, lo, hi, g);
        if (rc) return rc;
        SysPlan &P = sys[s];
        std::memset(&P, 0, sizeof(P));
        P.atom0 = offsets[s];
        P.natoms = offsets[s + 1] - offsets[s];
        P.inv_h = 1.0 / c->prm.h;
        for (int d = 0; d < 3; d++) {
            P.lo[d] = lo[d];
            P.tmax[d] = (hi[d] - lo[d]) / c->prm.h;
            P.nc[d] = g.nc[d];
            P.nb[d] = (g.nc[d] + kBrick - 1) / kBrick;
        }
        P.nlev = g.nlev;
        maxlev = std::max(maxlev, g.nlev);
        std::memcpy(P.gorg, g.gorg, sizeof(P.gorg));
        std::memcpy(P.gdim, g.gdim, sizeof(P.gdim));
        P.cell0 = cells;
        P.ncells = (int64_t)P.nb[0] * P.nb[1] * P.nb[2] * kBrickCells;
        P.group0 = groups;
        P.ngroups = (P.natoms + kWave - 1) / kWave;
        atom_p[s] = P.atom0;
        group_p[s] = groups;
        cell_p[s] = cells;
        iblk_p[s] = iblk;
        top_p[s] = top;
        ant_p[s] = ant;
        ant_p8[s] = ant8;
        if (g.nlev > 0) {
            ant += anterp_tiles(g.gdim[0][0], g.gdim[0][1], g.gdim[0][2], 4);
            ant8 += anterp_tiles(g.gdim[0][0], g.gdim[0][1], g.gdim[0][2], 8);
        }
        for (int k = 0; k < kMaxLevels; k++) node_p[(size_t)k * W + s] = nodes[k];
        for (int k = 0; k < g.nlev; k++) {
            P.qoff[k] = q;
            P.uoff[k] = u;
            const int64_t n = (int64_t)g.gdim[k][0] * g.gdim[k][1] * g.gdim[k][2];
            q += round_up((int64_t)padded_x(g.gdim[k][0]) * padded_x(g.gdim[k][1]) * padded_z(g.gdim[k][2]), 64);
            u += round_up(n, 64);
            nodes[k] += n;
        }
        rxy_p[s] = rxy;
        pxy_p[s] = pxy;
        if (g.nlev >= 2) {
            if (!comp_fits(g.gdim, g.nlev)) composite = false;
            rxy += (int64_t)g.gdim[0][2] * (g.nlev - 1);
            for (int k = 1; k < g.nlev; k++) {
                P.toff[k] = tsz;
                P.woff[k] = wsz;
                tsz += comp_t(g.gdim, g.nlev, k);
                wsz += comp_w(g.gdim, g.nlev, k);
                pxy += g.gdim[k][2];
            }
        }
        cells += P.ncells;
        groups += P.ngroups;
        iblk += (P.natoms + 255) / 256;
        if (g.nlev == 0) continue;   // simple cutoff method: no grids
        const int kt = g.nlev - 1;
        top += top_blocks(g.gdim[kt][0] * g.gdim[kt][1] * g.gdim[kt][2]);
        int d2 = 0;
        for (int d = 0; d < 3; d++) d2 += (g.gdim[kt][d] - 1) * (g.gdim[kt][d] - 1);
        top_d2 = std::max(top_d2, d2);
    }
    rxy_p[nsys] = rxy;
    pxy_p[nsys] = pxy;
    if (tsz > c->cap_t || wsz > c->cap_w || maxlev < 2) composite = false;
    // composite filters of the transfers between level 0 and level k:
    // phi_1(m) = Phi(m/2) and phi_{k+1}(m) = sum_j phi_1(j) phi_k(m - 2^k j),
    // |m| <= s_k with s_1 = 2S-1 and s_{k+1} = s_k + 2^k s_1 (exact dyadic
    // rationals: products and sums of the half-integer basis values)
    const int S = (basis_degree(c->prm) + 1) / 2, s1 = 2 * S - 1;
    std::vector<double> &phi_tab = ps.phi_tab;
    phi_tab.clear();
    int phi_off[kMaxLevels] = {0}, phi_s[kMaxLevels] = {0};
    if (composite) {   // only the composite transfers read the filters
        std::vector<double> &p1 = ps.p1, &cur = ps.cur, &nxt = ps.nxt;
        p1.assign(2 * s1 + 1, 0.0);
        for (int m = -s1; m <= s1; m++)
            p1[m + s1] = m == 0 ? 1.0 : ((m & 1) ? (S == 3 ? basis5(0.5 * m) : basis(0.5 * m)) : 0.0);
        cur = p1;
        int sk = s1;
        for (int k = 1; k < maxlev && k < kMaxLevels; k++) {
            phi_off[k] = (int)phi_tab.size();
            phi_s[k] = sk;
            phi_tab.insert(phi_tab.end(), cur.begin(), cur.end());
            const int sn = sk + (1 << k) * s1;
            nxt.assign(2 * sn + 1, 0.0);
            for (int m = -sn; m <= sn; m++) {
                double acc = 0;
                for (int j = -s1; j <= s1; j++) {
                    const int mm = m - (1 << k) * j;
                    if (mm >= -sk && mm <= sk) acc += p1[j + s1] * cur[mm + sk];
                }
                nxt[m + sn] = acc;
            }
            cur.swap(nxt);
            sk = sn;
        }
    }
    atom_p[nsys] = offsets[nsys];
    group_p[nsys] = groups;
    cell_p[nsys] = cells;
    iblk_p[nsys] = iblk;
    top_p[nsys] = top;
    ant_p[nsys] = ant;
    ant_p8[nsys] = ant8;
    // deeper anterpolation tiles (single precision, cubic basis) where there
    // are enough of them to fill the chip: fewer staged halo atoms per node
    int ant_depth = 4;
    if (c->prm.precision == MSM_FP32 && basis_degree(c->prm) == 3 && ant8 >= kAntDeep) {
        ant_depth = 8;
        ant = ant8;
        ant_p.swap(ant_p8);
    }
    for (int k = 0; k < kMaxLevels; k++) node_p[(size_t)k * W + nsys] = nodes[k];
    // stencil tiles of every level below each system's top, segment k*nsys + s
    const int esz = c->prm.precision == MSM_FP32 ? 4 : 8;
    const int txy = stencil_tile_xy(esz, c->mc.reach), tz = stencil_tile_z(esz, c->mc.reach);
    const int nseg = (maxlev - 1) * nsys;
    tile_p.assign((size_t)nseg + 1, 0);
    int64_t tiles = 0;
    for (int k = 0; k + 1 < maxlev; k++)
        for (int s = 0; s < nsys; s++) {
            tile_p[(size_t)k * nsys + s] = tiles;
            const SysPlan &P = sys[s];
            if (k < P.nlev - 1)
                tiles += (int64_t)((P.gdim[k][0] + txy - 1) / txy) * ((P.gdim[k][1] + txy - 1) / txy) *
                         ((P.gdim[k][2] + tz - 1) / tz);
        }
    tile_p[nseg] = tiles;
    if (cells > c->cap_cells || q > c->cap_q || u > c->cap_u || iblk > c->cap_iblk) return MSM_ERR_CAPACITY;
    if (cells >= (int64_t)1 << 31) return MSM_ERR_CAPACITY;
    // the atoms that carry Lennard-Jones (a bound model): per system their
    // count from the model's prefix (batch atom i is model atom i % period),
    // the same systems and cells, their own 64-atom groups
    const bool lj = c->md_bound && !c->lj_prefix.empty();
    std::vector<SysPlan> &lj_sys = ps.lj_sys;
    std::vector<int64_t> &lj_group_p = ps.lj_group_p;
    int64_t lj_atoms = 0, lj_groups = 0;
    // the pair search's own cells: edge h / pair_cell, the same atoms and groups
    const int pcm = c->mc.pair_cell;
    std::vector<SysPlan> &pc_sys = ps.pc_sys;
    int64_t pc_cells = 0;
    if (pcm > 1) {
        pc_sys = sys;
        for (int s = 0; s < nsys; s++) {
            SysPlan &P = pc_sys[s];
            P.inv_h = pcm / c->prm.h;
            for (int d = 0; d < 3; d++) {
                P.tmax[d] = sys[s].tmax[d] * pcm;
                P.nc[d] = (int)std::floor(P.tmax[d]) + 1;
                P.nb[d] = (P.nc[d] + kBrick - 1) / kBrick;
            }
            P.cell0 = pc_cells;
            P.ncells = (int64_t)P.nb[0] * P.nb[1] * P.nb[2] * kBrickCells;
            pc_cells += P.ncells;
        }
        if (pc_cells > c->pc_cap) return MSM_ERR_CAPACITY;
    }
    int64_t lj_cells = 0;
    if (lj) {
        const int64_t period = (int64_t)c->lj_prefix.size() - 1, per = c->lj_prefix[period];
        auto before = [&](int64_t i) { return (i / period) * per + c->lj_prefix[i % period]; };
        lj_sys = sys;
        lj_group_p.assign(W, 0);
        for (int s = 0; s < nsys; s++) {
            SysPlan &P = lj_sys[s];
            const int64_t n = before(offsets[s + 1]) - before(offsets[s]);
            // cells of their own: an edge that holds about kLjCellAtoms of them
            // at their mean density, no finer than h (the cell capacity) and
            // no coarser than a
            double vol = 1.0;
            for (int d = 0; d < 3; d++) vol *= std::max(sys[s].tmax[d] * c->prm.h, c->prm.h);
            const double edge = std::min(c->prm.a, std::max(c->prm.h, std::cbrt(kLjCellAtoms * vol / std::max<int64_t>(n, 1))));
            P.inv_h = 1.0 / edge;
            for (int d = 0; d < 3; d++) {
                P.tmax[d] = sys[s].tmax[d] * c->prm.h / edge;
                P.nc[d] = (int)std::floor(P.tmax[d]) + 1;
                P.nb[d] = (P.nc[d] + kBrick - 1) / kBrick;
            }
            P.cell0 = lj_cells;
            P.ncells = (int64_t)P.nb[0] * P.nb[1] * P.nb[2] * kBrickCells;
            lj_cells += P.ncells;
            P.atom0 = lj_atoms;
            P.natoms = n;
            P.group0 = lj_groups;
            P.ngroups = (n + kWave - 1) / kWave;
            lj_group_p[s] = lj_groups;
            lj_atoms += n;
            lj_groups += P.ngroups;
        }
        lj_group_p[nsys] = lj_groups;
        if (lj_cells > c->cap_cells) return MSM_ERR_CAPACITY;
    }

    // pack the tables into one blob
    size_t off = 0;
    auto place = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_sys = place(sizeof(SysPlan) * nsys);
    const size_t o_atom = place(sizeof(int64_t) * W), o_group = place(sizeof(int64_t) * W);
    const size_t o_cell = place(sizeof(int64_t) * W), o_iblk = place(sizeof(int64_t) * W);
    const size_t o_top = place(sizeof(int64_t) * W), o_ant = place(sizeof(int64_t) * W);
    const size_t o_node = place(sizeof(int64_t) * kMaxLevels * W), o_tile = place(sizeof(int64_t) * (nseg + 1));
    const size_t o_rxy = place(sizeof(int64_t) * W), o_pxy = place(sizeof(int64_t) * W);
    const size_t o_phi = place(sizeof(double) * std::max<size_t>(phi_tab.size(), 1));
    const size_t o_ljsys = lj ? place(sizeof(SysPlan) * nsys) : 0, o_ljgroup = lj ? place(sizeof(int64_t) * W) : 0;
    const size_t o_pcsys = pcm > 1 ? place(sizeof(SysPlan) * nsys) : 0;
    char *h = nullptr;
    int slot = -1;
    if (c->fixed_plan) {
        // allocation-free contexts: the tables go to a fixed device region
        // through kernel arguments, from the context's host image
        if (off > c->fixed_plan_cap) return MSM_ERR_CAPACITY;
        if (ps.blob.size() < off) ps.blob.resize(off);
        h = ps.blob.data();
    } else if (off > c->plan_cap) {
        // the current tables may still be read by queued work
        if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
        if (c->plan_dev) (void)hipFree(c->plan_dev);
        if (c->plan_host) (void)hipHostFree(c->plan_host);
        c->plan_dev = nullptr;
        c->plan_host = nullptr;
        c->plan_cap = 0;
        if (hipMalloc((void **)&c->plan_dev, off) != hipSuccess) return MSM_ERR_HIP;
        if (hipHostMalloc((void **)&c->plan_host, off * msm_ctx::kPlanStage, hipHostMallocDefault) != hipSuccess)
            return MSM_ERR_HIP;
        c->plan_cap = off;
        for (bool &l : c->plan_ev_live) l = false;
    }
    if (!c->fixed_plan) {
        slot = c->plan_slot;
        c->plan_slot = (slot + 1) % msm_ctx::kPlanStage;
        if (!c->plan_ev[slot] && hipEventCreateWithFlags(&c->plan_ev[slot], hipEventDisableTiming) != hipSuccess)
            return MSM_ERR_HIP;
        // the slot's previous copy must have run before it is overwritten
        if (c->plan_ev_live[slot] && hipEventSynchronize(c->plan_ev[slot]) != hipSuccess) return MSM_ERR_HIP;
        h = c->plan_host + (size_t)slot * c->plan_cap;
    }
    std::memcpy(h + o_sys, sys.data(), sizeof(SysPlan) * nsys);
    std::memcpy(h + o_atom, atom_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_group, group_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_cell, cell_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_iblk, iblk_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_top, top_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_ant, ant_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_node, node_p.data(), sizeof(int64_t) * kMaxLevels * W);
    std::memcpy(h + o_tile, tile_p.data(), sizeof(int64_t) * (nseg + 1));
    std::memcpy(h + o_rxy, rxy_p.data(), sizeof(int64_t) * W);
    std::memcpy(h + o_pxy, pxy_p.data(), sizeof(int64_t) * W);
    if (!phi_tab.empty()) std::memcpy(h + o_phi, phi_tab.data(), sizeof(double) * phi_tab.size());
    if (pcm > 1) std::memcpy(h + o_pcsys, pc_sys.data(), sizeof(SysPlan) * nsys);
    if (lj) {
        std::memcpy(h + o_ljsys, lj_sys.data(), sizeof(SysPlan) * nsys);
        std::memcpy(h + o_ljgroup, lj_group_p.data(), sizeof(int64_t) * W);
    }
    if (c->fixed_plan) {
        if (put_bytes(c->stream, c->fixed_plan, h, off) != hipSuccess) return MSM_ERR_HIP;
    } else {
        if (hipMemcpyAsync(c->plan_dev, h, off, hipMemcpyHostToDevice, c->stream) != hipSuccess) return MSM_ERR_HIP;
        if (hipEventRecord(c->plan_ev[slot], c->stream) != hipSuccess) return MSM_ERR_HIP;
        c->plan_ev_live[slot] = true;
    }

    DevPlan &dp = c->dp;
    char *d = c->fixed_plan ? c->fixed_plan : c->plan_dev;
    dp.sys = (const SysPlan *)(d + o_sys);
    dp.nsys = nsys;
    dp.atom_prefix = (const int64_t *)(d + o_atom);
    dp.group_prefix = (const int64_t *)(d + o_group);
    dp.cell_prefix = (const int64_t *)(d + o_cell);
    dp.iblk_prefix = (const int64_t *)(d + o_iblk);
    dp.top_prefix = (const int64_t *)(d + o_top);
    dp.ant_prefix = (const int64_t *)(d + o_ant);
    dp.node_prefix = (const int64_t *)(d + o_node);
    dp.tile_prefix = (const int64_t *)(d + o_tile);
    dp.ntile_seg = nseg;
    dp.ntiles = tiles;
    dp.top_d2 = top_d2;
    dp.natoms = offsets[nsys];
    dp.ngroups = groups;
    dp.ncells = cells;
    dp.niblk = iblk;
    dp.ntop = top;
    dp.nant = ant;
    dp.ant_depth = ant_depth;
    for (int k = 0; k < kMaxLevels; k++) dp.nnodes[k] = nodes[k];
    dp.maxlev = maxlev;
    dp.composite = composite ? 1 : 0;
    dp.phi = (const double *)(d + o_phi);
    std::memcpy(dp.phi_off, phi_off, sizeof(phi_off));
    std::memcpy(dp.phi_s, phi_s, sizeof(phi_s));
    dp.rxy_prefix = (const int64_t *)(d + o_rxy);
    dp.pxy_prefix = (const int64_t *)(d + o_pxy);
    dp.nrxy = rxy;
    dp.npxy = pxy;
    dp.nrz = 0;
    for (int k = 1; k < kMaxLevels; k++) dp.nrz += nodes[k];
    dp.evflag = (c->prm.precision == MSM_FP32 ? c->wf.status : c->wd.status) + 1;
    // the pair search's own cells
    c->dpp = dp;
    if (pcm > 1) {
        c->dpp.sys = (const SysPlan *)(d + o_pcsys);
        c->dpp.ncells = pc_cells;
    }
    // the subset plan: its own cells, atoms and groups
    c->dps = dp;
    if (lj) {
        c->dps.sys = (const SysPlan *)(d + o_ljsys);
        c->dps.group_prefix = (const int64_t *)(d + o_ljgroup);
        c->dps.natoms = lj_atoms;
        c->dps.ngroups = lj_groups;
        c->dps.ncells = lj_cells;
    } else {
        c->dps.natoms = 0;
        c->dps.ngroups = 0;
        c->dps.ncells = 0;
    }
    c->host_sys = sys;
    c->last_offsets.assign(offsets, offsets + nsys + 1);
    if (domains) c->last_domains.assign(domains, domains + nsys * 6);
    else c->last_domains.clear();
    c->plan_valid = true;
    c->plan_version++;
    return MSM_OK;
}

namespace {

template <typename T> Work<T> &work(msm_ctx *c);
template <> Work<float> &work<float>(msm_ctx *c) { return c->wf; }
template <> Work<double> &work<double>(msm_ctx *c) { return c->wd; }

template <typename T>
int evaluate(msm_ctx *c, const void *xyzq, double *energy, void *forces, void *pots, int part)
{
    using L = Launch<T>;
    const DevPlan &p = c->dp;
    Work<T> &w = work<T>(c);
    hipStream_t s = c->stream;
    hipError_t e;
    auto mark = [&](int stage) {
        if (c->timing) (void)hipEventRecord(c->ev[stage], s);
    };
    mark(MSM_STAGE_BIN);
    if ((e = L::bin(s, p, w, (const vec4_t<T> *)xyzq)) != hipSuccess) return MSM_ERR_HIP;
    mark(MSM_STAGE_SHORT);
    // the short-range potentials are needed only for the energy and the potentials
    const bool pot = energy || pots || c->tuning_pass;
    const bool do_short = part != kEvalLong, do_long = part != kEvalShort;
    // the pair sum and the grid stages share only the binned atoms: with
    // concurrency on, the pair kernel runs on the side stream from here until
    // the join before interpolation
    const bool fork = do_short && do_long && c->concurrent && !c->timing && p.nnodes[0] > 0;
    // mode 2: anterpolation first, alone (its large LDS tiles are starved by
    // long-lived pair workgroups when both start together), then the fork
    const bool ant_first = fork && c->concurrent == 2;
    if (ant_first) {
        mark(MSM_STAGE_ANTERP);
        if ((e = L::anterp(s, p, w, c->mc)) != hipSuccess) return MSM_ERR_HIP;
    }
    hipStream_t ps = s;
    if (fork) {
        if (!c->side_stream && hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess)
            return MSM_ERR_HIP;
        if (!c->ev_fork && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess)
            return MSM_ERR_HIP;
        if (!c->ev_join && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
            return MSM_ERR_HIP;
        if (hipEventRecord(c->ev_fork, s) != hipSuccess || hipStreamWaitEvent(c->side_stream, c->ev_fork, 0) != hipSuccess)
            return MSM_ERR_HIP;
        ps = c->side_stream;
    }
    const DevPlan *pp = c->mc.pair_cell > 1 ? &c->dpp : nullptr;
    if (do_short && (e = L::pair(ps, p, pp, w, (const vec4_t<T> *)xyzq, c->mc, pot)) != hipSuccess) return MSM_ERR_HIP;
    // Lennard-Jones needs only the input positions: with the fork it runs on
    // the first stream ahead of the grid stages, beside the pair kernel, which
    // a small system does not fill (after the grid stages it measured slower:
    // the join then waits for it)
    const bool lj_beside = fork;
    if (do_short && c->md_bound) {
        if ((e = L::exclusions(ps, p, w, (const vec4_t<T> *)xyzq, c->mc, pot)) != hipSuccess) return MSM_ERR_HIP;
        if (!lj_beside && (e = L::lj(ps, p, c->dps, w, (const vec4_t<T> *)xyzq, c->mc, pot)) != hipSuccess)
            return MSM_ERR_HIP;
    }
    if (lj_beside && c->md_bound && (e = L::lj(s, p, c->dps, w, (const vec4_t<T> *)xyzq, c->mc, pot)) != hipSuccess)
        return MSM_ERR_HIP;
    if (!ant_first) {
        mark(MSM_STAGE_ANTERP);
        if (do_long && (e = L::anterp(s, p, w, c->mc)) != hipSuccess) return MSM_ERR_HIP;
    }
    mark(MSM_STAGE_RESTRICT);
    // every level from level 0 by composite filters (two launches), or one
    // launch per level; each launch serves all systems of the batch
    if (do_long && p.composite) {
        if ((e = L::restrict_all(s, p, w)) != hipSuccess) return MSM_ERR_HIP;
    } else {
        for (int k = 0; do_long && k + 1 < p.maxlev; k++)
            if ((e = L::restrict_level(s, p, w, k, c->mc)) != hipSuccess) return MSM_ERR_HIP;
    }
    mark(MSM_STAGE_CUTOFF);
    if (do_long) {
        StencilTables<T> tb{c->wcols, (const T *)c->weights, c->ncols, c->mc.reach, c->mc.stencil_threads};
        if ((e = L::stencil(s, p, w, tb, c->mc)) != hipSuccess) return MSM_ERR_HIP;
    }
    mark(MSM_STAGE_TOP);   // the top level runs in the lattice-cutoff launch
    mark(MSM_STAGE_PROLONG);
    if (do_long && p.composite) {   // u^0 from every level at once; u^k (k >= 1) is not formed
        if ((e = L::prolong_all(s, p, w)) != hipSuccess) return MSM_ERR_HIP;
    } else {
        for (int k = p.maxlev - 2; do_long && k >= 0; k--)
            if ((e = L::prolong_level(s, p, w, k, c->mc)) != hipSuccess) return MSM_ERR_HIP;
    }
    if (fork && (hipEventRecord(c->ev_join, ps) != hipSuccess || hipStreamWaitEvent(s, c->ev_join, 0) != hipSuccess))
        return MSM_ERR_HIP;
    mark(MSM_STAGE_INTERP);
    if ((e = L::interp(s, p, w, c->mc, (T *)forces, (T *)pots, part)) != hipSuccess) return MSM_ERR_HIP;
    if ((e = L::energy(s, p, w, energy)) != hipSuccess) return MSM_ERR_HIP;
    if (c->timing) {
        mark(MSM_NSTAGES);
        if (hipEventSynchronize(c->ev[MSM_NSTAGES]) != hipSuccess) return MSM_ERR_HIP;
        for (int st = 0; st < MSM_NSTAGES; st++) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, c->ev[st], c->ev[st + 1]) != hipSuccess) return MSM_ERR_HIP;
            c->stage_ms[st] += ms;
        }
        c->timed_evals++;
    }
    return MSM_OK;
}

}  // namespace

static int evaluate_eager(msm_ctx *c, const void *xyzq, double *energy, void *forces, void *pots, int part)
{
    if (c->prm.precision == MSM_FP32) return evaluate<float>(c, xyzq, energy, forces, pots, part);
    return evaluate<double>(c, xyzq, energy, forces, pots, part);
}

static void drop_graph(msm_ctx::GraphEntry &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = msm_ctx::GraphEntry{};
}

// With graphs enabled, an evaluation is captured once per batch plan and set
// of buffers (on an internal stream) and replayed on the context stream; the
// launch sequence is the same as the eager one, so results are identical.
int msmx::evaluate_any(msm_ctx *c, const void *xyzq, double *energy, void *forces, void *pots, int part)
{
    if (!c->use_graphs || c->timing) return evaluate_eager(c, xyzq, energy, forces, pots, part);
    msm_ctx::GraphEntry *hit = nullptr, *victim = &c->graphs[0];
    for (auto &g : c->graphs) {
        if (g.valid && g.plan_version == c->plan_version && g.xyzq == xyzq && g.energy == energy &&
            g.forces == forces && g.pots == pots && g.part == part)
            hit = &g;
        if (!g.valid || g.last_use < victim->last_use) victim = &g;
    }
    if (!hit) {
        if (!c->capture_stream && hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return MSM_ERR_HIP;
        drop_graph(*victim);
        hipStream_t saved = c->stream;
        c->stream = c->capture_stream;
        if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            c->stream = saved;
            return MSM_ERR_HIP;
        }
        int rc = evaluate_eager(c, xyzq, energy, forces, pots, part);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
        c->stream = saved;
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return MSM_ERR_HIP;
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return MSM_ERR_HIP;
        }
        victim->valid = true;
        victim->plan_version = c->plan_version;
        victim->xyzq = xyzq;
        victim->energy = energy;
        victim->forces = forces;
        victim->pots = pots;
        victim->part = part;
        victim->graph = graph;
        victim->exec = exec;
        hit = victim;
    }
    hit->last_use = ++c->graph_clock;
    return hipGraphLaunch(hit->exec, c->stream) == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

namespace {

// Quarter-disc columns (ox, oy >= 0, ox^2 + oy^2 <= d2max) and, per column,
// the weights g^0(h |o|) = gamma(h|o|/a)/a - gamma(h|o|/(2a))/(2a) for
// oz = -R .. R (zero where |o|^2 > d2max: g^0 vanishes for r >= 2a).
template <typename T>
void stencil_tables(double a, double h, int R, int d2max, const Smooth &g, std::vector<int2> &cols,
                    std::vector<T> &w)
{
    cols.clear();
    w.clear();
    for (int oy = 0; oy <= R; oy++)
        for (int ox = 0; ox <= R; ox++) {
            if (ox * ox + oy * oy > d2max) continue;
            cols.push_back(make_int2(ox, oy));
            for (int oz = -R; oz <= R; oz++) {
                const int d2 = ox * ox + oy * oy + oz * oz;
                double g0 = 0.0;
                if (d2 <= d2max) {
                    const double r = h * std::sqrt((double)d2);
                    g0 = gamma_s(r / a, g) / a - gamma_s(r / (2 * a), g) / (2 * a);
                }
                w.push_back(T(g0));
            }
        }
}

template <typename T> std::vector<T> &weights_image(msm_ctx *c);
template <> std::vector<float> &weights_image<float>(msm_ctx *c) { return c->ps.wf; }
template <> std::vector<double> &weights_image<double>(msm_ctx *c) { return c->ps.wd; }

// The context's constant device table: the lattice-cutoff columns and
// weights (MSM), or the single-precision Wolf pair table (Wolf summation in
// FP32, in the weights slot); nothing otherwise.
template <typename T> void stencil_image_t(msm_ctx *c, size_t *col_bytes, size_t *w_bytes)
{
    std::vector<T> &w = weights_image<T>(c);
    c->ps.cols.clear();
    w.clear();
    if (c->mc.method == MSM_METHOD_MSM) {
        stencil_tables<T>(c->prm.a, c->prm.h, c->mc.reach, c->d2max, c->mc.g, c->ps.cols, w);
    } else if (c->mc.method == MSM_METHOD_WOLF && sizeof(T) == 4) {
        w.resize(8 * kWolfPieces);
        wolf_table(c->prm.a, c->mc.alpha, (float *)w.data());
    }
    c->ncols = (int)c->ps.cols.size();
    *col_bytes = c->ps.cols.size() * sizeof(int2);
    *w_bytes = w.size() * sizeof(T);
}

bool has_table(const msm_ctx *c)
{
    return c->mc.method == MSM_METHOD_MSM || (c->mc.method == MSM_METHOD_WOLF && c->prm.precision == MSM_FP32);
}

// after the table is in device memory
void bind_table(msm_ctx *c)
{
    c->mc.wolf_tab = c->mc.method == MSM_METHOD_WOLF ? (const float4 *)c->weights : nullptr;
}

template <typename T> int upload_stencil(msm_ctx *c)
{
    size_t cb = 0, wb = 0;
    stencil_image_t<T>(c, &cb, &wb);
    if (wb && hipMalloc(&c->weights, wb) != hipSuccess) return MSM_ERR_HIP;
    if (cb && hipMalloc((void **)&c->wcols, cb) != hipSuccess) return MSM_ERR_HIP;
    if (wb && hipMemcpy(c->weights, weights_image<T>(c).data(), wb, hipMemcpyHostToDevice) != hipSuccess)
        return MSM_ERR_HIP;
    if (cb && hipMemcpy(c->wcols, c->ps.cols.data(), cb, hipMemcpyHostToDevice) != hipSuccess) return MSM_ERR_HIP;
    bind_table(c);
    return MSM_OK;
}

}  // namespace

int msmx::init_context(msm_ctx *c, const msm_params *prm)
{
    if (!prm) return MSM_ERR_ARG;
    if (!(prm->a > 0) || !(prm->h > 0) || !std::isfinite(prm->a) || !std::isfinite(prm->h)) return MSM_ERR_ARG;
    if (prm->precision != MSM_FP32 && prm->precision != MSM_FP64) return MSM_ERR_ARG;
    if (prm->max_atoms < 0 || prm->max_atoms >= ((int64_t)1 << 31) || prm->max_systems < 1) return MSM_ERR_ARG;
    if (prm->levels < 0 || prm->levels > kMaxLevels) return MSM_ERR_ARG;
    if (!std::isfinite(prm->coulomb_k)) return MSM_ERR_ARG;
    if (prm->method != MSM_METHOD_MSM && prm->method != MSM_METHOD_CUTOFF && prm->method != MSM_METHOD_WOLF)
        return MSM_ERR_ARG;
    if (prm->method == MSM_METHOD_WOLF && !(prm->alpha >= 0 && std::isfinite(prm->alpha))) return MSM_ERR_ARG;
    const int smoothing = prm->smoothing ? prm->smoothing : 2;
    if (smoothing < 1 || smoothing > kMaxSmooth) return MSM_ERR_UNSUPPORTED;
    if (prm->basis != 0 && prm->basis != 3 && prm->basis != 5) return MSM_ERR_UNSUPPORTED;
    const bool cutoff = prm->method != MSM_METHOD_MSM;   // no grids
    const double ratio = 2.0 * prm->a / prm->h;
    const int reach = (int)std::ceil(ratio) - 1;       // largest integer below 2a/h
    if (!cutoff && (reach < 1 || reach > kMaxReach - 1)) return MSM_ERR_UNSUPPORTED;

    c->prm = *prm;
    c->mc = MethodConst{};
    c->mc.a = prm->a;
    c->mc.h = prm->h;
    c->mc.ke = prm->coulomb_k;
    c->mc.method = prm->method;
    c->mc.cutoff = cutoff ? 1 : 0;
    c->mc.alpha = prm->method == MSM_METHOD_WOLF ? prm->alpha : 0.0;
    c->mc.g = make_smooth(smoothing);
    c->mc.p = basis_degree(*prm);
    c->mc.reach = cutoff ? 0 : reach;
    c->mc.pair_waves = 2;
    c->mc.stencil_threads = 1024;
    c->mc.pair_cell = 1;
    c->d2max = (int)std::ceil(ratio * ratio) - 1;      // largest integer below (2a/h)^2
    int rc = geometry(*prm, prm->lo, prm->hi, c->ctx_geom);
    if (rc) return rc;
    const Sizes sz = sizes_of(c->ctx_geom);
    const int64_t ns = prm->max_systems;
    c->cap_cells = sz.cells * ns;
    c->cap_q = sz.q * ns;
    c->cap_u = sz.u * ns;
    c->cap_t = sz.t * ns;
    c->cap_w = sz.w * ns;
    c->cap_iblk = (prm->max_atoms + 255) / 256 + ns;
    if (c->cap_cells >= ((int64_t)1 << 31)) return MSM_ERR_CAPACITY;
    return MSM_OK;
}

size_t msmx::workspace_bytes(msm_ctx *c)
{
    size_t bytes = 0;
    if (c->prm.precision == MSM_FP32) carve<float>(c, c->wf, nullptr, &bytes, false);
    else carve<double>(c, c->wd, nullptr, &bytes, false);
    return bytes;
}

void msmx::carve_workspace(msm_ctx *c, char *base)
{
    size_t bytes = 0;
    if (c->prm.precision == MSM_FP32) carve<float>(c, c->wf, base, &bytes, true);
    else carve<double>(c, c->wd, base, &bytes, true);
}

void msmx::stencil_image(msm_ctx *c, size_t *col_bytes, size_t *w_bytes)
{
    *col_bytes = *w_bytes = 0;
    if (!has_table(c)) return;
    if (c->prm.precision == MSM_FP32) stencil_image_t<float>(c, col_bytes, w_bytes);
    else stencil_image_t<double>(c, col_bytes, w_bytes);
}

int msmx::put_stencil(msm_ctx *c, void *cols_dev, void *w_dev)
{
    const void *w = c->prm.precision == MSM_FP32 ? (const void *)c->ps.wf.data() : (const void *)c->ps.wd.data();
    const size_t wb = c->prm.precision == MSM_FP32 ? c->ps.wf.size() * 4 : c->ps.wd.size() * 8;
    if (put_bytes(c->stream, cols_dev, c->ps.cols.data(), c->ps.cols.size() * sizeof(int2)) != hipSuccess ||
        put_bytes(c->stream, w_dev, w, wb) != hipSuccess)
        return MSM_ERR_HIP;
    c->wcols = (int2 *)cols_dev;
    c->weights = w_dev;
    bind_table(c);
    return MSM_OK;
}


extern "C" {

const char *msm_status_string(int code)
{
    switch (code) {
    case MSM_OK: return "ok";
    case MSM_NOT_CONVERGED: return "parareal did not converge within kmax iterations";
    case MSM_ERR_ARG: return "invalid argument";
    case MSM_ERR_DOMAIN: return "an atom lies outside its domain";
    case MSM_ERR_NONFINITE: return "non-finite position or charge";
    case MSM_ERR_CAPACITY: return "capacity of the context exceeded";
    case MSM_ERR_HIP: return "HIP runtime error";
    case MSM_ERR_UNSUPPORTED: return "parameters outside the supported range";
    case MSM_ERR_CONSTRAINT: return "a rigid molecule's constraint iteration did not converge";
    default: return "unknown status";
    }
}

int msm_setup(const msm_params *prm, void *stream, msm_ctx **out)
{
    if (!prm || !out) return MSM_ERR_ARG;
    *out = nullptr;
    msm_ctx *c = new (std::nothrow) msm_ctx();
    if (!c) return MSM_ERR_ARG;
    int rc = init_context(c, prm);
    if (rc) {
        delete c;
        return rc;
    }
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MSM_ERR_HIP;
    }
    size_t bytes = workspace_bytes(c);
    if (hipMalloc((void **)&c->wbuf, bytes) != hipSuccess) {
        delete c;
        return MSM_ERR_HIP;
    }
    c->wbytes = bytes;
    carve_workspace(c, c->wbuf);

    // zero everything once: the halos of the charge grids are never written
    if (hipMemsetAsync(c->wbuf, 0, c->wbytes, c->stream) != hipSuccess) {
        msm_destroy(c);
        return MSM_ERR_HIP;
    }
    if (has_table(c)) rc = prm->precision == MSM_FP32 ? upload_stencil<float>(c) : upload_stencil<double>(c);
    if (rc) {
        msm_destroy(c);
        return rc;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        msm_destroy(c);
        return MSM_ERR_HIP;
    }
    *out = c;
    return MSM_OK;
}

void msm_destroy(msm_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->plan_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (auto &g : c->graphs) drop_graph(g);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->wbuf) (void)hipFree(c->wbuf);
    if (c->weights) (void)hipFree(c->weights);
    if (c->wcols) (void)hipFree(c->wcols);
    if (c->plan_dev) (void)hipFree(c->plan_dev);
    if (c->plan_host) (void)hipHostFree(c->plan_host);
    if (c->mdbuf) (void)hipFree(c->mdbuf);
    if (c->pcbuf) (void)hipFree(c->pcbuf);
    if (c->n3buf) (void)hipFree(c->n3buf);
    delete c;
}

int msm_set_stream(msm_ctx *c, void *stream)
{
    if (!c) return MSM_ERR_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    c->stream = (hipStream_t)stream;
    return MSM_OK;
}

int msm_energy_forces(msm_ctx *c, int nsys, const int64_t *offsets, const double *domains, const void *xyzq,
                      double *energy, void *forces, void *pots)
{
    if (!c || nsys < 1 || !offsets) return MSM_ERR_ARG;
    if (nsys > c->prm.max_systems) return MSM_ERR_CAPACITY;
    if (offsets[nsys] > 0 && !xyzq) return MSM_ERR_ARG;
    int rc = build_plan(c, nsys, offsets, domains);
    if (rc) return rc;
    return evaluate_any(c, xyzq, energy, forces, pots);
}

int msm_get_tuning(const msm_ctx *c, msm_tuning *t)
{
    if (!c || !t) return MSM_ERR_ARG;
    t->pair_waves = c->mc.pair_waves;
    t->stencil_threads = c->mc.stencil_threads;
    t->concurrent = c->concurrent;
    t->pair_cell = c->mc.pair_cell;
    return MSM_OK;
}

// Arrays of the pair search's own cells for edge h / m (grown, never shrunk).
static int ensure_pair_cells(msm_ctx *c, int m)
{
    if (m <= 1) return MSM_OK;
    Geometry g{};
    msm_params fine = c->prm;
    fine.h = c->prm.h / m;
    fine.method = MSM_METHOD_CUTOFF;   // cells only
    int rc = geometry(fine, c->prm.lo, c->prm.hi, g);
    if (rc) return rc;
    int64_t nb = 1;
    for (int d = 0; d < 3; d++) nb *= (g.nc[d] + kBrick - 1) / kBrick;
    const int64_t cells = nb * kBrickCells * c->prm.max_systems;
    if (cells >= ((int64_t)1 << 31)) return MSM_ERR_CAPACITY;
    if (c->pcbuf && cells <= c->pc_cap) return MSM_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    if (c->pcbuf) (void)hipFree(c->pcbuf);
    c->pcbuf = nullptr;
    c->pc_cap = 0;
    const int64_t na = std::max<int64_t>(c->prm.max_atoms, 1);
    const size_t vb = c->prm.precision == MSM_FP32 ? sizeof(float4) : sizeof(double4);
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += (b + 255) / 256 * 256;
        return o;
    };
    const size_t o_cell = take(4 * na), o_slot = take(4 * na), o_cnt = take(4 * (cells + 1)),
                 o_start = take(4 * (cells + 1)), o_blk = take(4 * std::max<int64_t>(kScanFewBlocks, (cells + 1) / 4096 + 2)),
                 o_ord = take(4 * na), o_pos = take(4 * na), o_x = take(vb * (na + 64)), o_out = take(vb * na);
    if (hipMalloc((void **)&c->pcbuf, off) != hipSuccess) return MSM_ERR_HIP;
    if (hipMemsetAsync(c->pcbuf, 0, off, c->stream) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        return MSM_ERR_HIP;
    char *b = c->pcbuf;
    auto fill = [&](auto &w) {
        using V = std::remove_pointer_t<decltype(w.pc.x)>;
        w.pc.cell_of = (int *)(b + o_cell);
        w.pc.slot_of = (int *)(b + o_slot);
        w.pc.cnt = (int *)(b + o_cnt);
        w.pc.start = (int *)(b + o_start);
        w.pc.blocks = (int *)(b + o_blk);
        w.pc.order = (int *)(b + o_ord);
        w.pc.pos_of = (int *)(b + o_pos);
        w.pc.x = (V *)(b + o_x);
        w.pc.aux = nullptr;
        w.pc_out = (V *)(b + o_out);
    };
    if (c->prm.precision == MSM_FP32) fill(c->wf);
    else fill(c->wd);
    c->pc_cap = cells;
    return MSM_OK;
}

// The accumulators of the Newton's third law pair form, zero (single
// precision contexts that own their memory only).
static int ensure_newton(msm_ctx *c)
{
    if (c->prm.precision != MSM_FP32 || c->fixed_plan) return MSM_ERR_UNSUPPORTED;
    const int64_t na = std::max<int64_t>(c->prm.max_atoms, 1);
    if (c->n3buf && na <= c->n3_cap) return MSM_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    if (c->n3buf) (void)hipFree(c->n3buf);
    c->n3buf = nullptr;
    c->n3_cap = 0;
    c->wf.nacc = nullptr;
    c->wf.nacc_stride = 0;
    const size_t bytes = sizeof(unsigned long long) * 4 * (size_t)na;
    if (hipMalloc(&c->n3buf, bytes) != hipSuccess) return MSM_ERR_HIP;
    if (hipMemsetAsync(c->n3buf, 0, bytes, c->stream) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        return MSM_ERR_HIP;
    c->n3_cap = na;
    c->wf.nacc = (unsigned long long *)c->n3buf;
    c->wf.nacc_stride = na;
    return MSM_OK;
}

int msm_set_tuning(msm_ctx *c, const msm_tuning *t)
{
    if (!c || !t) return MSM_ERR_ARG;
    if (t->pair_waves != 1 && t->pair_waves != 2 && t->pair_waves != 3 && t->pair_waves != 4 && t->pair_waves != 5 &&
        t->pair_waves != 6 && t->pair_waves != 7 && t->pair_waves != 8 && t->pair_waves != 9 && t->pair_waves != 10 &&
        t->pair_waves != 16)
        return MSM_ERR_ARG;
    if (t->stencil_threads != 256 && t->stencil_threads != 1024) return MSM_ERR_ARG;
    if (t->concurrent < 0 || t->concurrent > 2) return MSM_ERR_ARG;
    if (t->pair_cell < 1 || t->pair_cell > 3) return MSM_ERR_ARG;
    if (c->fixed_plan && t->pair_cell != 1) return MSM_ERR_UNSUPPORTED;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    int rc = ensure_pair_cells(c, t->pair_cell);
    if (rc) return rc;
    if (t->pair_waves == 10 && (rc = ensure_newton(c))) return rc;
    for (auto &g : c->graphs) drop_graph(g);     // captured launches use the old kernels
    if (t->pair_cell != c->mc.pair_cell) c->plan_valid = false;   // the plan holds the cells
    c->mc.pair_waves = t->pair_waves;
    c->mc.stencil_threads = t->stencil_threads;
    c->concurrent = t->concurrent;
    c->mc.pair_cell = t->pair_cell;
    return MSM_OK;
}

int msm_autotune(msm_ctx *c, int nsys, const int64_t *offsets, const double *domains, const void *xyzq, int reps,
                 msm_tuning *chosen)
{
    if (!c || nsys < 1 || !offsets || reps < 1) return MSM_ERR_ARG;
    if (nsys > c->prm.max_systems) return MSM_ERR_CAPACITY;
    const msm_tuning start{c->mc.pair_waves, c->mc.stencil_threads, c->concurrent, c->mc.pair_cell};
    // first the kernels with the grid cells, then the pair search's own cells
    if (c->mc.pair_cell != 1) c->plan_valid = false;
    c->mc.pair_cell = 1;
    int rc = build_plan(c, nsys, offsets, domains);
    if (rc) {
        c->mc.pair_cell = start.pair_cell;
        return rc;
    }
    // whole evaluations, launched eagerly with the context's stream use: with
    // concurrent stages the pair kernel that fits best beside the grid stages
    // is not the fastest one alone
    const bool was_timing = c->timing, had_graphs = c->use_graphs;
    c->timing = false;
    c->use_graphs = false;
    c->tuning_pass = true;   // time the pair kernel that also sums the potentials
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = MSM_ERR_HIP;
    auto eval_time = [&](double *ms) {
        int r = evaluate_any(c, xyzq, nullptr, nullptr, nullptr);   // warm-up
        if (r) return r;
        if (hipEventRecord(e0, c->stream) != hipSuccess) return (int)MSM_ERR_HIP;
        for (int i = 0; i < reps && !r; i++) r = evaluate_any(c, xyzq, nullptr, nullptr, nullptr);
        if (r) return r;
        float t = 0;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return (int)MSM_ERR_HIP;
        *ms = t / reps;
        return (int)MSM_OK;
    };
    msm_tuning best = start;
    double best_ms = 1e300;
    // with concurrent stages, both fork points: after binning, or after anterpolation
    const int modes[2] = {1, 2};
    const int nmodes = start.concurrent ? 2 : 1;
    for (int mi = 0; mi < nmodes; mi++)
        for (int pw : {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 16})
            for (int st : {256, 1024}) {
                if (rc) break;
                if (pw == 10 && ensure_newton(c) != MSM_OK) continue;   // single precision only
                c->mc.pair_waves = pw;
                c->mc.stencil_threads = st;
                c->concurrent = start.concurrent ? modes[mi] : 0;
                double ms = 0;
                if ((rc = eval_time(&ms))) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best.pair_waves = pw;
                    best.stencil_threads = st;
                    best.concurrent = c->concurrent;
                    best.pair_cell = 1;
                }
            }
    // cells of edge h/2 and h/3 for the pair search, with the chosen kernels
    // (skipped where their arrays would not fit)
    for (int m = 2; m <= 3 && !rc && !c->fixed_plan; m++) {
        if (ensure_pair_cells(c, m) != MSM_OK) break;
        c->mc.pair_waves = best.pair_waves;
        c->mc.stencil_threads = best.stencil_threads;
        c->concurrent = best.concurrent;
        c->mc.pair_cell = m;
        c->plan_valid = false;
        if ((rc = build_plan(c, nsys, offsets, domains))) break;
        double ms = 0;
        if ((rc = eval_time(&ms))) break;
        if (ms < best_ms) {
            best_ms = ms;
            best.pair_cell = m;
        }
    }
    if (c->mc.pair_cell != start.pair_cell) c->plan_valid = false;
    c->mc.pair_cell = start.pair_cell;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->timing = was_timing;
    c->use_graphs = had_graphs;
    c->tuning_pass = false;
    c->mc.pair_waves = start.pair_waves;
    c->mc.stencil_threads = start.stencil_threads;
    c->concurrent = start.concurrent;
    if (rc) return rc;
    int r2 = msm_set_tuning(c, &best);
    if (r2) return r2;
    if (chosen) *chosen = best;
    return MSM_OK;
}

int msm_set_graphs(msm_ctx *c, int enable)
{
    if (!c) return MSM_ERR_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    c->use_graphs = enable != 0;
    if (!c->use_graphs)
        for (auto &g : c->graphs) drop_graph(g);
    return MSM_OK;
}

int msm_get_status(msm_ctx *c)
{
    if (!c) return MSM_ERR_ARG;
    int *st = c->prm.precision == MSM_FP32 ? c->wf.status : c->wd.status;
    int v = 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    if (hipMemcpy(&v, st, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return MSM_ERR_HIP;
    if (v) {
        if (fill_i32(c->stream, st, 1, 0) != hipSuccess) return MSM_ERR_HIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    }
    // an atom that left its domain is the first cause of what follows from
    // it (forces and constraint iterations that turn non-finite)
    if (v & kStatusDomain) return MSM_ERR_DOMAIN;
    if (v & kStatusNonFinite) return MSM_ERR_NONFINITE;
    if (v & kStatusConstraint) return MSM_ERR_CONSTRAINT;
    return MSM_OK;
}

int msm_grid_shape(const msm_ctx *c, const double *domain, int *org, int *dim)
{
    if (!c || !org || !dim) return MSM_ERR_ARG;
    Geometry g;
    int rc = geometry(c->prm, domain ? domain : c->prm.lo, domain ? domain + 3 : c->prm.hi, g);
    if (rc) return rc;
    for (int k = 0; k < g.nlev; k++)
        for (int d = 0; d < 3; d++) {
            org[3 * k + d] = g.gorg[k][d];
            dim[3 * k + d] = g.gdim[k][d];
        }
    return g.nlev;
}

int msm_debug_stages(msm_ctx *c, int sys, double *u_short, double *f_short, double *const *qg,
                     double *const *ucut, double *const *ug)
{
    if (!c || !c->plan_valid || sys < 0 || sys >= c->dp.nsys) return MSM_ERR_ARG;
    // the composite prolongation forms u^0 only: form every level's u^k one
    // level at a time from the lattice-cutoff potentials the evaluation left
    for (int k = c->dp.maxlev - 2; c->dp.composite && k >= 0; k--) {
        const hipError_t pe = c->prm.precision == MSM_FP32
                                  ? Launch<float>::prolong_level(c->stream, c->dp, c->wf, k, c->mc)
                                  : Launch<double>::prolong_level(c->stream, c->dp, c->wd, k, c->mc);
        if (pe != hipSuccess) return MSM_ERR_HIP;
    }
    hipError_t e = c->prm.precision == MSM_FP32
                       ? Launch<float>::stage_copy(c->stream, c->dp, c->wf, sys, u_short, f_short, qg, ucut, ug)
                       : Launch<double>::stage_copy(c->stream, c->dp, c->wd, sys, u_short, f_short, qg, ucut, ug);
    return hip_status(e);
}

int msm_enable_stage_timing(msm_ctx *c, int enable)
{
    if (!c) return MSM_ERR_ARG;
    if (enable && !c->ev[0])
        for (auto &e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) return MSM_ERR_HIP;
    c->timing = enable != 0;
    return MSM_OK;
}

int msm_stage_timing(msm_ctx *c, double *ms_out, int64_t *evaluations, int reset)
{
    if (!c) return MSM_ERR_ARG;
    if (ms_out)
        for (int st = 0; st < MSM_NSTAGES; st++) ms_out[st] = c->stage_ms[st];
    if (evaluations) *evaluations = c->timed_evals;
    if (reset) {
        for (double &v : c->stage_ms) v = 0;
        c->timed_evals = 0;
    }
    return MSM_OK;
}

}  // extern "C"
