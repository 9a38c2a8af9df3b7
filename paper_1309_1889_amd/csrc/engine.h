// Internal interface of the engine: the context and the plan/evaluation
// entry points shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/msm.h"
#include "launch.h"
#include "md.h"

namespace msmx {

struct Geometry {
    int nlev;
    int nc[3];
    int gorg[kMaxLevels][3];
    int gdim[kMaxLevels][3];
};

// Host vectors of a plan build, kept by the context so that their capacity
// is reused from one build to the next.
struct PlanScratch {
    std::vector<SysPlan> sys;
    std::vector<int64_t> atom_p, group_p, cell_p, iblk_p, top_p, ant_p, ant_p8, node_p, rxy_p, pxy_p, tile_p;
    std::vector<SysPlan> lj_sys;      // the Lennard-Jones subset's system plans
    std::vector<int64_t> lj_group_p;  // and its 64-atom groups
    std::vector<SysPlan> pc_sys;      // the system plans of the pair search's own cells
    std::vector<double> phi_tab, p1, cur, nxt;
    std::vector<char> blob;            // image of the tables for a fixed device region
    std::vector<int2> cols;            // stencil columns and weights before upload
    std::vector<float> wf;
    std::vector<double> wd;
};

}  // namespace msmx

struct msm_ctx {
    msm_params prm;
    hipStream_t stream = nullptr;
    int device = 0;
    msmx::MethodConst mc{};
    int d2max = 0;
    msmx::Geometry ctx_geom{};
    // capacities
    int64_t cap_cells = 0, cap_q = 0, cap_u = 0, cap_iblk = 0, cap_t = 0, cap_w = 0;
    // device memory
    char *wbuf = nullptr;
    size_t wbytes = 0;
    void *weights = nullptr;     // stencil weights along z per quarter-disc column, precision T
    int2 *wcols = nullptr;       // quarter-disc columns (ox, oy)
    int ncols = 0;
    char *plan_dev = nullptr;    // tables of the current batch
    // pinned staging copies of the tables: a ring of kPlanStage slots of
    // plan_cap bytes, each reused only after the copy it fed has run, so a new
    // plan never waits for the work queued on the stream
    static constexpr int kPlanStage = 4;
    char *plan_host = nullptr;
    size_t plan_cap = 0;
    hipEvent_t plan_ev[kPlanStage] = {};
    bool plan_ev_live[kPlanStage] = {};
    int plan_slot = 0;
    msmx::DevPlan dp{};
    msmx::DevPlan dps{};         // the plan of the atoms that carry Lennard-Jones (dynamics model)
    // allocation-free contexts: the tables are written to this fixed device
    // region (at most fixed_plan_cap bytes) instead of plan_dev
    char *fixed_plan = nullptr;
    size_t fixed_plan_cap = 0;
    msmx::PlanScratch ps;
    bool plan_valid = false;
    std::vector<int64_t> last_offsets;
    std::vector<double> last_domains;
    std::vector<msmx::SysPlan> host_sys;
    msmx::Work<float> wf{};
    msmx::Work<double> wd{};
    // stage timing (benchmarks)
    bool timing = false;
    bool tuning_pass = false;                   // msm_autotune: evaluate as if potentials were asked for
    hipEvent_t ev[MSM_NSTAGES + 1] = {};
    double stage_ms[MSM_NSTAGES] = {};
    int64_t timed_evals = 0;
    // concurrent stages: the short-range sum on side_stream between the two
    // events; 1: forked after binning, 2: forked after anterpolation (which
    // then runs alone on the whole chip), 0: every stage in turn
    int concurrent = 1;
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // captured evaluations (msm_set_graphs)
    bool use_graphs = false;
    hipStream_t capture_stream = nullptr;
    uint64_t plan_version = 0;
    struct GraphEntry {
        bool valid = false;
        uint64_t plan_version = 0;
        const void *xyzq = nullptr;
        double *energy = nullptr;
        void *forces = nullptr, *pots = nullptr;
        int part = 0;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint64_t last_use = 0;
    } graphs[8];
    uint64_t graph_clock = 0;
    // dynamics (msm_md_bind)
    bool md_bound = false;
    // model atoms that carry Lennard-Jones: lj_prefix[m] counts those before
    // model atom m (period + 1 entries); empty when none does
    std::vector<int64_t> lj_prefix;
    bool rigid = false;
    msmx::TriModel tri{};
    char *mdbuf = nullptr;       // model, forces and parareal scratch
    // the pair search's own cells (tuning pair_cell > 1): their arrays, sized
    // for pc_cap cells and max_atoms atoms, and the plan of those cells
    char *pcbuf = nullptr;
    int64_t pc_cap = 0;
    // accumulators of the Newton's third law pair form (tuning pair_waves 10),
    // 4 x n3_cap 64-bit words
    void *n3buf = nullptr;
    int64_t n3_cap = 0;
    msmx::DevPlan dpp{};
    void *md_forces = nullptr;                  // max_atoms x 3, precision T
    void *md_forces_slow = nullptr;             // multiple time steps: the grid part, max_atoms x 3
    double *md_parts = nullptr;  // per-block partial sums (kinetic energy)
    double *md_scalar = nullptr; // scratch words: the changes of a parareal iteration, 64 + max_systems
    void *px = nullptr, *pv = nullptr;          // propagator state, max_atoms x 4 doubles each
    void *pe = nullptr;                         // FP32 contexts: positions for the evaluation, max_atoms x 4
    double *fout = nullptr, *gold = nullptr;    // parareal: fine results and coarse values, max_atoms x 6
    double *gnew = nullptr;                     // parareal: coarse result of one slice, max_atoms x 6
};


namespace msmx {

// Validate the parameters and fill the context's method constants, geometry
// and capacities (everything msm_setup does before allocating).
int init_context(msm_ctx *c, const msm_params *prm);
// Bytes of the workspace the context's capacities need.
size_t workspace_bytes(msm_ctx *c);
// Point the context's workspace arrays into base (workspace_bytes long).
void carve_workspace(msm_ctx *c, char *base);
// Host image of the stencil columns and weights of the context (in c->ps),
// their byte sizes, and the upload of that image to device memory at cols_dev
// and w_dev through kernel arguments.
void stencil_image(msm_ctx *c, size_t *col_bytes, size_t *w_bytes);
int put_stencil(msm_ctx *c, void *cols_dev, void *w_dev);

// Build (or reuse) the device tables of a batch.
int build_plan(msm_ctx *c, int nsys, const int64_t *offsets, const double *domains);
// One evaluation of the current plan on xyzq (precision of the context).
// Which part of the MSM interaction an evaluation computes: everything, only
// the short-range pairs (with the model's Lennard-Jones), or only the grid
// (long-range) part with the smooth self term, for multiple time steps.
enum EvalPart { kEvalAll = 0, kEvalShort = 1, kEvalLong = 2 };
int evaluate_any(msm_ctx *c, const void *xyzq, double *energy, void *forces, void *pots, int part = kEvalAll);

}  // namespace msmx
