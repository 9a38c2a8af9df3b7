// msm_energy_forces_noalloc: one multilevel summation evaluation of one
// system with every work array in a static device array, for callers that
// cannot allocate device memory. The kernels and the launch sequence are
// those of msm_energy_forces on a context with the default launch
// configuration, run on one stream (no side stream, no graphs).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>

#include "engine.h"

using namespace msmx;

static constexpr size_t kScratchBytes = (size_t)MSM_NOALLOC_SCRATCH_MIB << 20;

// The work arrays of every call on a device. Host code never uses this name
// as an address: each device's copy is found once with hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kPlanBytes = 64 << 10;   // the plan tables of one system fit easily

struct DeviceSlot {
    std::mutex lock;     // serialises the host side of calls on one device
    bool ready = false;
    char *ptr = nullptr; // this device's copy of scratch
    msm_ctx *ctx = nullptr;
};
DeviceSlot g_slots[kMaxDevices];

__global__ void k_status_code(const int *__restrict__ st, int *__restrict__ out)
{
    const int v = *st;
    *out = (v & kStatusNonFinite) ? MSM_ERR_NONFINITE : ((v & kStatusDomain) ? MSM_ERR_DOMAIN : MSM_OK);
}

// Set-up of a device (first call there): the address of its scratch copy
// and a context object whose host vectors are reserved for one system.
int setup_slot(DeviceSlot &d)
{
    if (d.ready) return MSM_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MSM_ERR_HIP;
    msm_ctx *c = new (std::nothrow) msm_ctx();
    if (!c) return MSM_ERR_HIP;
    PlanScratch &ps = c->ps;
    ps.sys.reserve(1);
    for (auto *v : {&ps.atom_p, &ps.group_p, &ps.cell_p, &ps.iblk_p, &ps.top_p, &ps.ant_p, &ps.ant_p8, &ps.rxy_p, &ps.pxy_p})
        v->reserve(2);
    ps.node_p.reserve((size_t)kMaxLevels * 2);
    ps.tile_p.reserve(kMaxLevels + 1);
    // composite filters of at most MSM_NOALLOC_MAX_LEVELS grids of the
    // quintic basis: level k's filter has 2 s_k + 1 taps, s_1 = 5 and
    // s_{k+1} = s_k + 2^k s_1; the recurrence also forms level maxlev's
    size_t phi = 0, last = 0;
    for (int k = 1, sk = 5; k <= MSM_NOALLOC_MAX_LEVELS; k++, sk += (1 << (k - 1)) * 5) {
        last = 2 * (size_t)sk + 1;
        if (k < MSM_NOALLOC_MAX_LEVELS) phi += last;
    }
    ps.phi_tab.reserve(phi);
    ps.p1.reserve(16);
    ps.cur.reserve(last);
    ps.nxt.reserve(last);
    ps.blob.reserve(kPlanBytes);
    ps.cols.reserve((kMaxReach + 1) * (kMaxReach + 1));
    ps.wf.reserve((size_t)(kMaxReach + 1) * (kMaxReach + 1) * (2 * kMaxReach + 1));
    ps.wd.reserve((size_t)(kMaxReach + 1) * (kMaxReach + 1) * (2 * kMaxReach + 1));
    c->host_sys.reserve(1);
    c->last_offsets.reserve(2);
    d.ptr = (char *)p;
    d.ctx = c;
    d.ready = true;
    return MSM_OK;
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

extern "C" int msm_energy_forces_noalloc(const msm_params *params, void *stream, int64_t natoms,
                                         const void *xyzq, double *energy, void *forces, void *pots,
                                         int32_t *status)
{
    if (!params || natoms < 0 || (natoms > 0 && !xyzq)) return MSM_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MSM_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return MSM_ERR_UNSUPPORTED;
    DeviceSlot &d = g_slots[dev];
    std::lock_guard<std::mutex> guard(d.lock);
    int rc = setup_slot(d);
    if (rc) return rc;
    msm_ctx *c = d.ctx;

    // a context for exactly this system: capacity natoms, one system
    msm_params prm = *params;
    prm.max_atoms = natoms;
    prm.max_systems = 1;
    rc = init_context(c, &prm);
    if (rc) return rc;
    if (c->ctx_geom.nlev > MSM_NOALLOC_MAX_LEVELS) return MSM_ERR_CAPACITY;
    c->stream = (hipStream_t)stream;
    c->device = dev;
    c->concurrent = 0;
    c->use_graphs = false;
    c->timing = false;
    c->tuning_pass = false;
    c->plan_valid = false;   // the tables in scratch may be another call's

    // scratch layout: work arrays | stencil columns | stencil weights | plan tables
    const size_t wbytes = up256(workspace_bytes(c));
    size_t cb = 0, wb = 0;
    stencil_image(c, &cb, &wb);   // the lattice-cutoff or Wolf table, if the method has one
    const size_t o_cols = wbytes, o_w = o_cols + up256(cb), o_plan = o_w + up256(wb);
    if (o_plan + kPlanBytes > kScratchBytes) return MSM_ERR_CAPACITY;
    carve_workspace(c, d.ptr);
    c->wbuf = nullptr;   // the context owns no memory
    c->wbytes = 0;
    c->fixed_plan = d.ptr + o_plan;
    c->fixed_plan_cap = kPlanBytes;

    // the work arrays keep the last call's contents: clear them (the charge
    // grid halos, the cell histogram and the status word must start at zero)
    if (fill_i32(c->stream, (int *)d.ptr, (int64_t)(wbytes / 4), 0) != hipSuccess) return MSM_ERR_HIP;
    if ((rc = put_stencil(c, d.ptr + o_cols, d.ptr + o_w))) return rc;
    const int64_t offsets[2] = {0, natoms};
    if ((rc = build_plan(c, 1, offsets, nullptr))) return rc;
    if ((rc = evaluate_any(c, xyzq, energy, forces, pots))) return rc;
    if (status) {
        const int *st = c->prm.precision == MSM_FP32 ? c->wf.status : c->wd.status;
        hipLaunchKernelGGL(k_status_code, dim3(1), dim3(1), 0, c->stream, st, (int *)status);
        if (hipGetLastError() != hipSuccess) return MSM_ERR_HIP;
    }
    return MSM_OK;
}
