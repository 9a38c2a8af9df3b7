// Host side of the dynamics entry points: model binding, velocity Verlet on a
// batch of systems, and the parareal iteration (Section 4) with a batched
// fine propagator and a serial coarse sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

using namespace msmx;

namespace {

template <typename T> Work<T> &work_of(msm_ctx *c);
template <> Work<float> &work_of<float>(msm_ctx *c) { return c->wf; }
template <> Work<double> &work_of<double>(msm_ctx *c) { return c->wd; }

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

template <typename T> int bind(msm_ctx *c, const msm_md_model *m)
{
    const int64_t na = std::max<int64_t>(c->prm.max_atoms, 1);
    const int64_t period = m->period;
    if (period < 1) return MSM_ERR_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    if (c->mdbuf) {
        (void)hipFree(c->mdbuf);
        c->mdbuf = nullptr;
    }
    c->md_bound = false;
    c->lj_prefix.clear();
    c->plan_valid = false;   // the plan of the Lennard-Jones atoms depends on the model
    const bool aux = m->molid_dev || m->lj_dev;
    // the model on the host: molecule ids (every atom its own molecule
    // without them) and (sigma, epsilon)
    std::vector<int32_t> mol(aux ? period : 0, -1);
    std::vector<double> lj(aux ? 2 * period : 0, 0.0);
    if (m->molid_dev &&
        hipMemcpy(mol.data(), m->molid_dev, sizeof(int32_t) * period, hipMemcpyDeviceToHost) != hipSuccess)
        return MSM_ERR_HIP;
    if (aux && !m->molid_dev)
        for (int64_t i = 0; i < period; i++) mol[i] = -1 - (int32_t)i;
    if (m->lj_dev && hipMemcpy(lj.data(), m->lj_dev, sizeof(double) * 2 * period, hipMemcpyDeviceToHost) != hipSuccess)
        return MSM_ERR_HIP;
    for (int64_t i = 0; aux && i < period; i++)
        if (lj[2 * i] < 0 || lj[2 * i + 1] < 0 || !std::isfinite(lj[2 * i]) || !std::isfinite(lj[2 * i + 1]))
            return MSM_ERR_ARG;
    // excluded partners: the other atoms of each molecule, ascending
    std::vector<int32_t> xstart, xidx;
    if (m->molid_dev) {
        std::vector<std::pair<int32_t, int32_t>> by(period);
        for (int64_t i = 0; i < period; i++) by[i] = {mol[i], (int32_t)i};
        std::sort(by.begin(), by.end());
        std::vector<int32_t> cnt(period, 0);
        for (int64_t b = 0; b < period;) {
            int64_t e = b;
            while (e < period && by[e].first == by[b].first) e++;
            if (e - b > kMaxMoleculeAtoms) return MSM_ERR_ARG;
            for (int64_t k = b; k < e; k++) cnt[by[k].second] = (int32_t)(e - b - 1);
            b = e;
        }
        xstart.assign(period + 1, 0);
        for (int64_t i = 0; i < period; i++) xstart[i + 1] = xstart[i] + cnt[i];
        xidx.assign(std::max<int32_t>(xstart[period], 1), 0);
        std::vector<int32_t> fill(xstart.begin(), xstart.end() - 1);
        for (int64_t b = 0; b < period;) {
            int64_t e = b;
            while (e < period && by[e].first == by[b].first) e++;
            for (int64_t k = b; k < e; k++)
                for (int64_t q = b; q < e; q++)
                    if (q != k) xidx[fill[by[k].second]++] = by[q].second;
            b = e;
        }
        if (xstart[period] == 0) xstart.clear();   // no molecule of two atoms or more
    }
    // the atoms that carry Lennard-Jones, as the kernels see them (a nonzero
    // sqrt(epsilon) in the context's precision)
    int64_t nlj = 0;
    if (aux) {
        c->lj_prefix.assign(period + 1, 0);
        for (int64_t i = 0; i < period; i++) {
            c->lj_prefix[i + 1] = c->lj_prefix[i] + (T(std::sqrt(lj[2 * i + 1])) != T(0) ? 1 : 0);
        }
        nlj = c->lj_prefix[period];
        if (nlj == 0) c->lj_prefix.clear();
    }
    // one Lennard-Jones type and at most one such atom per molecule: the
    // pair kernel then takes the parameters as constants and reads no records
    bool lj_one = nlj > 0;
    double lj_sigma = 0, lj_eps = 0;
    if (lj_one) {
        std::vector<int32_t> ljmol;
        for (int64_t i = 0; i < period; i++) {
            if (T(std::sqrt(lj[2 * i + 1])) == T(0)) continue;
            if (ljmol.empty()) {
                lj_sigma = lj[2 * i];
                lj_eps = lj[2 * i + 1];
            } else if (lj[2 * i] != lj_sigma || lj[2 * i + 1] != lj_eps) {
                lj_one = false;
            }
            ljmol.push_back(mol[i]);
        }
        std::sort(ljmol.begin(), ljmol.end());
        if (std::adjacent_find(ljmol.begin(), ljmol.end()) != ljmol.end()) lj_one = false;
    }
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += up256(b);
        return o;
    };
    const bool excl = !xstart.empty(), ljs = nlj > 0;
    const int64_t cells1 = c->cap_cells + 1;
    const size_t o_maux = aux ? take(sizeof(vec4_t<T>) * period) : 0;
    const size_t o_saux = aux ? take(sizeof(vec4_t<T>) * (na + 64)) : 0;
    const size_t o_xs = excl ? take(sizeof(int32_t) * xstart.size()) : 0;
    const size_t o_xi = excl ? take(sizeof(int32_t) * xidx.size()) : 0;
    const size_t o_lcnt = ljs ? take(sizeof(int) * cells1) : 0, o_lstart = ljs ? take(sizeof(int) * cells1) : 0;
    const size_t o_lblk = ljs ? take(sizeof(int) * std::max<int64_t>(kScanFewBlocks, cells1 / 4096 + 2)) : 0;
    const size_t o_lof = ljs ? take(sizeof(int) * na) : 0, o_lord = ljs ? take(sizeof(int) * na) : 0;
    const size_t o_lcell = ljs ? take(sizeof(int) * na) : 0, o_lslot = ljs ? take(sizeof(int) * na) : 0;
    const size_t o_lcl = ljs ? take(sizeof(int) * (na + (int64_t)kWave * c->prm.max_systems)) : 0;
    const size_t o_lx = ljs ? take(sizeof(vec4_t<T>) * (na + 64)) : 0, o_laux = ljs ? take(sizeof(vec4_t<T>) * (na + 64)) : 0;
    const size_t o_lout = ljs ? take(sizeof(vec4_t<T>) * na) : 0;
    const size_t o_f = take(sizeof(T) * 3 * na), o_fs = take(sizeof(T) * 3 * na);
    const size_t o_parts = take(sizeof(double) * c->cap_iblk);
    const size_t o_scal = take(sizeof(double) * (64 + std::max(c->prm.max_systems, 1)));
    const size_t o_px = take(sizeof(double4) * na), o_pv = take(sizeof(double4) * na);
    const size_t o_pe = sizeof(T) == 4 ? take(sizeof(vec4_t<T>) * na) : 0;
    const size_t o_fout = take(sizeof(double) * 6 * na), o_gold = take(sizeof(double) * 6 * na);
    const size_t o_gnew = take(sizeof(double) * 6 * na);
    if (hipMalloc((void **)&c->mdbuf, off) != hipSuccess) return MSM_ERR_HIP;
    if (hipMemsetAsync(c->mdbuf, 0, off, c->stream) != hipSuccess) return MSM_ERR_HIP;
    char *b = c->mdbuf;
    Work<T> &w = work_of<T>(c);
    w.maux = aux ? (vec4_t<T> *)(b + o_maux) : nullptr;
    w.saux = aux ? (vec4_t<T> *)(b + o_saux) : nullptr;
    w.period = period;
    w.xstart = excl ? (int *)(b + o_xs) : nullptr;
    w.xidx = excl ? (int *)(b + o_xi) : nullptr;
    w.lj = SubBins<T>{};
    w.lj_one = ljs && lj_one;
    w.lj_sigma = lj_sigma;
    w.lj_eps = lj_eps;
    if (ljs) {
        w.lj.cell_of = (int *)(b + o_lcell);
        w.lj.slot_of = (int *)(b + o_lslot);
        w.lj.cnt = (int *)(b + o_lcnt);
        w.lj.start = (int *)(b + o_lstart);
        w.lj.blocks = (int *)(b + o_lblk);
        w.lj.order = (int *)(b + o_lord);
        w.lj.pos_of = (int *)(b + o_lof);
        w.lj.x = (vec4_t<T> *)(b + o_lx);
        w.lj.aux = (vec4_t<T> *)(b + o_laux);
    }
    w.lj_cluster = ljs ? (int *)(b + o_lcl) : nullptr;
    w.lj_out = ljs ? (vec4_t<T> *)(b + o_lout) : nullptr;
    c->md_forces = b + o_f;
    c->md_forces_slow = b + o_fs;
    c->md_parts = (double *)(b + o_parts);
    c->md_scalar = (double *)(b + o_scal);
    c->px = b + o_px;
    c->pv = b + o_pv;
    c->pe = sizeof(T) == 4 ? b + o_pe : nullptr;
    c->fout = (double *)(b + o_fout);
    c->gold = (double *)(b + o_gold);
    c->gnew = (double *)(b + o_gnew);
    if (aux) {
        // per model atom: (molecule id bits, sigma/2, sqrt(epsilon), 0)
        std::vector<vec4_t<T>> h(period);
        for (int64_t i = 0; i < period; i++) {
            vec4_t<T> r;
            if (sizeof(T) == 4) {
                int32_t bits = mol[i];
                std::memcpy(&r.x, &bits, 4);
            } else {
                int64_t bits = mol[i];
                std::memcpy(&r.x, &bits, 8);
            }
            r.y = T(0.5 * lj[2 * i]);
            r.z = T(std::sqrt(lj[2 * i + 1]));
            r.w = T(0);
            h[i] = r;
        }
        if (hipMemcpyAsync(w.maux, h.data(), sizeof(vec4_t<T>) * period, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess)
            return MSM_ERR_HIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    }
    if (excl) {
        if (hipMemcpyAsync(w.xstart, xstart.data(), sizeof(int32_t) * xstart.size(), hipMemcpyHostToDevice,
                           c->stream) != hipSuccess ||
            hipMemcpyAsync(w.xidx, xidx.data(), sizeof(int32_t) * xidx.size(), hipMemcpyHostToDevice, c->stream) !=
                hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return MSM_ERR_HIP;
    }
    c->rigid = m->rigid_triples != 0;
    for (int d = 0; d < 3; d++) c->tri.len[d] = m->tri_len[d];
    c->tri.tol = m->constraint_tol > 0 ? m->constraint_tol : 1e-10;   // the state is FP64 either way
    c->tri.max_iter = 500;
    c->tri.status = c->prm.precision == MSM_FP32 ? c->wf.status : c->wd.status;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MSM_ERR_HIP;
    c->md_bound = true;
    return MSM_OK;
}

// Velocity Verlet on the current plan (built by the caller), FP64 state,
// forces in the context's precision T.
template <typename T> int vv(msm_ctx *c, void *xyzq, void *vel, int nsteps, double dt, double *epot, double *ekin)
{
    using M = MdLaunch<T>;
    hipStream_t s = c->stream;
    const int64_t n = c->dp.natoms;
    double4 *x = (double4 *)xyzq, *v = (double4 *)vel;
    // the evaluation reads T positions: the state itself for FP64, a copy for FP32
    vec4_t<T> *xe = sizeof(T) == 8 ? (vec4_t<T> *)x : (vec4_t<T> *)c->pe;
    vec4_t<T> *xe_out = sizeof(T) == 8 ? nullptr : xe;
    T *f = (T *)c->md_forces;
    const TriModel *tm = c->rigid ? &c->tri : nullptr;
    if (xe_out && M::to_eval(s, n, x, xe_out) != hipSuccess) return MSM_ERR_HIP;
    int rc = evaluate_any(c, xe, nsteps == 0 ? epot : nullptr, f, nullptr);
    if (rc) return rc;
    for (int st = 0; st < nsteps; st++) {
        if (M::kick_drift(s, n, x, v, f, dt, tm, xe_out) != hipSuccess) return MSM_ERR_HIP;
        rc = evaluate_any(c, xe, st == nsteps - 1 ? epot : nullptr, f, nullptr);
        if (rc) return rc;
        if (M::kick(s, n, x, v, f, dt, tm) != hipSuccess) return MSM_ERR_HIP;
    }
    if (ekin && md_kinetic(s, c->dp, v, c->md_parts, ekin) != hipSuccess) return MSM_ERR_HIP;
    return MSM_OK;
}

// Impulse multiple-time-step velocity Verlet (r-RESPA): each outer step of dt
// is a half kick with the grid (slow) force, ninner velocity-Verlet steps of
// dt/ninner with the short-range (fast) force, the slow force at the new
// positions and a second slow half kick; the kicks of rigid triples end with
// RATTLE's velocity stage. The energy is a full evaluation at the end.
template <typename T>
int vv_mts(msm_ctx *c, void *xyzq, void *vel, int nouter, int ninner, double dt, double *epot, double *ekin)
{
    using M = MdLaunch<T>;
    hipStream_t s = c->stream;
    const int64_t n = c->dp.natoms;
    double4 *x = (double4 *)xyzq, *v = (double4 *)vel;
    vec4_t<T> *xe = sizeof(T) == 8 ? (vec4_t<T> *)x : (vec4_t<T> *)c->pe;
    vec4_t<T> *xe_out = sizeof(T) == 8 ? nullptr : xe;
    T *ff = (T *)c->md_forces, *fs = (T *)c->md_forces_slow;
    const TriModel *tm = c->rigid ? &c->tri : nullptr;
    const double di = dt / ninner;
    if (xe_out && M::to_eval(s, n, x, xe_out) != hipSuccess) return MSM_ERR_HIP;
    int rc = evaluate_any(c, xe, nullptr, fs, nullptr, kEvalLong);
    if (!rc) rc = evaluate_any(c, xe, nullptr, ff, nullptr, kEvalShort);
    for (int o = 0; o < nouter && !rc; o++) {
        if (M::kick(s, n, x, v, fs, dt, tm) != hipSuccess) return MSM_ERR_HIP;
        for (int i = 0; i < ninner && !rc; i++) {
            if (M::kick_drift(s, n, x, v, ff, di, tm, xe_out) != hipSuccess) return MSM_ERR_HIP;
            rc = evaluate_any(c, xe, nullptr, ff, nullptr, kEvalShort);
            if (!rc && M::kick(s, n, x, v, ff, di, tm) != hipSuccess) return MSM_ERR_HIP;
        }
        if (!rc) rc = evaluate_any(c, xe, nullptr, fs, nullptr, kEvalLong);
        if (!rc && M::kick(s, n, x, v, fs, dt, tm) != hipSuccess) return MSM_ERR_HIP;
    }
    if (rc) return rc;
    if (epot && (rc = evaluate_any(c, xe, epot, nullptr, nullptr, kEvalAll))) return rc;
    if (ekin && md_kinetic(s, c->dp, v, c->md_parts, ekin) != hipSuccess) return MSM_ERR_HIP;
    return MSM_OK;
}

int vv_any(msm_ctx *c, void *xyzq, void *vel, int nsteps, double dt, double *epot, double *ekin)
{
    if (c->prm.precision == MSM_FP32) return vv<float>(c, xyzq, vel, nsteps, dt, epot, ekin);
    return vv<double>(c, xyzq, vel, nsteps, dt, epot, ekin);
}

int check_rigid_offsets(const msm_ctx *c, int nsys, const int64_t *offsets)
{
    if (!c->rigid) return MSM_OK;
    for (int s = 0; s <= nsys; s++)
        if (offsets[s] % 3) return MSM_ERR_ARG;
    return MSM_OK;
}

// Propagate `count` consecutive slices of one system of n atoms stored in
// lam_in (FP64, n x 6 each) and write the results to lam_out.
int propagate(msm_ctx *c, int64_t n, int count, const double *q, const double *invm, const double *lam_in,
              double *lam_out, int steps, double dt)
{
    std::vector<int64_t> offs(count + 1);
    for (int i = 0; i <= count; i++) offs[i] = n * i;
    int rc = build_plan(c, count, offs.data(), nullptr);
    if (rc) return rc;
    const int64_t tot = n * count;
    hipStream_t s = c->stream;
    if (md_state_in(s, n, tot, lam_in, q, invm, (double4 *)c->px, (double4 *)c->pv) != hipSuccess) return MSM_ERR_HIP;
    rc = vv_any(c, c->px, c->pv, steps, dt, nullptr, nullptr);
    if (rc) return rc;
    return md_state_out(s, tot, (double4 *)c->px, (double4 *)c->pv, lam_out) == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

// Sliding-window parareal (Section 4). The coarse context's stream runs the
// serial coarse work (predictions, sweeps), the fine context's stream the
// batched fine runs; events order the two. Slice s keeps G(lambda_s) in slot
// s % width of the coarse ring. The plain mode runs the window's fine batch at
// the start of each iteration into one buffer, slice s at slot s - start. The
// pipelined mode uses two buffers alternately, slice s at slot s % width: the
// sweep of one iteration reads one while the fine runs for the next iteration
// fill the other.
class WindowRun {
  public:
    WindowRun(msm_ctx *fine, msm_ctx *coarse, const parareal_window_params *pp, int64_t n, const double *q,
              const double *invm, double *lambda, double *ring, parareal_window_state *st, bool rigid)
        : f_(fine), g_(coarse), p_(*pp), n_(n), q_(q), invm_(invm), lam_(lambda), ring_(ring), st_(st),
          rigid_(rigid), W_(pp->width), N6_(6 * n), fev_(2 * pp->width, nullptr), frec_(2 * pp->width, 0)
    {
        fbuf_[0] = fine->fout;
        fbuf_[1] = fine->gold;
        pipe_ = p_.pipeline != 0;
        chunk_ = pipe_ ? (p_.chunk > 0 ? std::min(p_.chunk, W_) : (W_ + 3) / 4) : W_;
    }
    ~WindowRun()
    {
        // the caller waits for both streams before the events go
        (void)hipStreamSynchronize(f_->stream);
        (void)hipStreamSynchronize(g_->stream);
        for (hipEvent_t e : fev_)
            if (e) (void)hipEventDestroy(e);
        if (eva_) (void)hipEventDestroy(eva_);
    }

    int run()
    {
        for (hipEvent_t &e : fev_)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MSM_ERR_HIP;
        if (hipEventCreateWithFlags(&eva_, hipEventDisableTiming) != hipSuccess) return MSM_ERR_HIP;
        const int T = p_.nslices;
        int b = st_->start;
        if (b == T) return MSM_OK;
        int end = b + std::min(W_, T - b);
        int cur = 0, rc = MSM_OK;
        const bool pipe = pipe_;
        base_ = b;
        // fine runs of the first iteration: from the window's states as they are ready
        if (!st_->window_valid) {
            if ((rc = produced(cur, b, end))) return rc;
            for (int s = b; s < end; s++) {
                if ((rc = predict(s))) return rc;
                if (pipe && (rc = produced(cur, s + 1, end))) return rc;
            }
            st_->window_valid = 1;
            for (int s = b + 1; !pipe && s < end; s++)   // one batch after the prediction
                if ((rc = produced(cur, s, end))) return rc;
        } else {
            for (int s = b; s < end; s++)
                if ((rc = produced(cur, s, end))) return rc;
        }
        if ((rc = flush())) return rc;
        std::vector<unsigned long long> bits(W_);
        for (int it = 0; b < T && (p_.max_iters == 0 || it < p_.max_iters); it++) {
            const int we = end - b;
            const int nxt = pipe ? 1 - cur : cur;
            const bool ahead = pipe && !(p_.max_iters > 0 && it + 1 == p_.max_iters);
            if (!pipe && it > 0) {
                base_ = b;
                if ((rc = launch_f(cur, b, end))) return rc;
            }
            if (zero_u64(g_->stream, change(), we) != hipSuccess) return MSM_ERR_HIP;
            for (int s = b; s < end; s++) {
                if ((rc = sweep_step(cur, s, end, s - b))) return rc;
                if (ahead && (rc = produced(nxt, s + 1, T))) return rc;
            }
            if ((rc = flush())) return rc;
            st_->coarse_slices += we;
            if (hipMemcpyAsync(bits.data(), change(), sizeof(unsigned long long) * we, hipMemcpyDeviceToHost,
                               g_->stream) != hipSuccess ||
                hipStreamSynchronize(g_->stream) != hipSuccess)
                return MSM_ERR_HIP;
            std::vector<double> chg(we);
            std::memcpy(chg.data(), bits.data(), sizeof(double) * we);
            // the first open state is exact; then accept the leading states that moved less than tol
            int acc = 1;
            while (acc < we && chg[acc] < p_.tol) acc++;
            st_->last_accepted = acc;
            st_->last_change = *std::max_element(chg.begin(), chg.end());
            st_->iterations++;
            b += acc;
            st_->start = b;
            const int new_end = b + std::min(W_, T - b);
            for (int s = end; s < new_end; s++) {
                if ((rc = predict(s))) return rc;
                if (ahead && (rc = produced(nxt, s + 1, new_end))) return rc;
            }
            if ((rc = flush())) return rc;
            end = new_end;
            cur = nxt;
        }
        return MSM_OK;
    }

  private:
    double *lam(int s) const { return lam_ + (int64_t)s * N6_; }
    double *rslot(int s) const { return ring_ + (int64_t)(s % W_) * N6_; }
    int slot(int s) const { return pipe_ ? s % W_ : s - base_; }
    double *fslot(int par, int s) const { return fbuf_[par] + (int64_t)slot(s) * N6_; }
    unsigned long long *change() const { return (unsigned long long *)f_->md_scalar; }

    // lambda_{s+1} = G(lambda_s), kept in the ring as the old coarse value
    int predict(int s)
    {
        int rc = propagate(g_, n_, 1, q_, invm_, lam(s), lam(s + 1), p_.steps_g, p_.dt_g);
        if (rc) return rc;
        st_->coarse_slices++;
        return copy_f64(g_->stream, lam(s + 1), rslot(s), N6_) == hipSuccess ? MSM_OK : MSM_ERR_HIP;
    }

    // Fine runs of slices [s0, s1) into buffer par, as batches whose slots do not wrap.
    int launch_f(int par, int s0, int s1)
    {
        while (s0 < s1) {
            const int e = std::min(s1, s0 + (W_ - slot(s0)));
            if (hipEventRecord(eva_, g_->stream) != hipSuccess || hipStreamWaitEvent(f_->stream, eva_, 0) != hipSuccess)
                return MSM_ERR_HIP;
            int rc = propagate(f_, n_, e - s0, q_, invm_, lam(s0), fslot(par, s0), p_.steps_f, p_.dt_f);
            if (rc) return rc;
            for (int s = s0; s < e; s++) {
                const int k = par * W_ + slot(s);
                if (hipEventRecord(fev_[k], f_->stream) != hipSuccess) return MSM_ERR_HIP;
                frec_[k] = 1;
            }
            st_->fine_slices += e - s0;
            s0 = e;
        }
        return MSM_OK;
    }

    // lambda_s is set for the coming sweep and needs a fine run (s < limit):
    // queue it, and start the queued batch once it holds chunk slices.
    int produced(int par, int s, int limit)
    {
        if (s >= limit) return MSM_OK;
        if (pend0_ < 0) {
            pend0_ = s;
            ppar_ = par;
        }
        pend1_ = s + 1;
        return pend1_ - pend0_ >= chunk_ ? flush() : MSM_OK;
    }
    int flush()
    {
        if (pend0_ < 0) return MSM_OK;
        const int a = pend0_, e = pend1_;
        pend0_ = -1;
        return launch_f(ppar_, a, e);
    }

    int wait_f(int par, int s)
    {
        const int k = par * W_ + slot(s);
        if (frec_[k] && hipStreamWaitEvent(g_->stream, fev_[k], 0) != hipSuccess) return MSM_ERR_HIP;
        return MSM_OK;
    }

    // One step of the coarse sweep: lambda_{s+1} = F(lambda_s) + (G(lambda_s) - G_old(lambda_s)).
    int sweep_step(int cur, int s, int end, int j)
    {
        // F(lambda_s) must be done, and the run that reads lambda_{s+1} before it is overwritten
        int rc = wait_f(cur, s);
        if (!rc && s + 1 < end) rc = wait_f(cur, s + 1);
        if (rc) return rc;
        double *gnew = g_->gnew;
        if ((rc = propagate(g_, n_, 1, q_, invm_, lam(s), gnew, p_.steps_g, p_.dt_g))) return rc;
        const hipError_t e =
            rigid_ ? parareal_correct_rigid(g_->stream, n_, lam(s + 1), fslot(cur, s), gnew, rslot(s), invm_, f_->tri,
                                            change() + j)
                   : parareal_correct(g_->stream, N6_, lam(s + 1), fslot(cur, s), gnew, rslot(s), change() + j);
        return e == hipSuccess ? MSM_OK : MSM_ERR_HIP;
    }

    msm_ctx *f_, *g_;
    parareal_window_params p_;
    int64_t n_;
    const double *q_, *invm_;
    double *lam_, *ring_;
    parareal_window_state *st_;
    bool rigid_;
    int W_;
    int64_t N6_;
    bool pipe_ = false;
    int chunk_ = 1;
    int base_ = 0;   // plain mode: the window's first slice
    double *fbuf_[2] = {};
    std::vector<hipEvent_t> fev_;
    std::vector<char> frec_;
    hipEvent_t eva_ = nullptr;
    int pend0_ = -1, pend1_ = -1, ppar_ = 0;
};

}  // namespace

extern "C" {

int msm_md_bind(msm_ctx *c, const msm_md_model *m)
{
    if (!c || !m) return MSM_ERR_ARG;
    if (m->rigid_triples) {
        for (int d = 0; d < 3; d++)
            if (!(m->tri_len[d] > 0)) return MSM_ERR_ARG;
        if (m->period % 3) return MSM_ERR_ARG;
    }
    return c->prm.precision == MSM_FP32 ? bind<float>(c, m) : bind<double>(c, m);
}

int msm_vv_run(msm_ctx *c, int nsys, const int64_t *offsets, const double *domains, void *xyzq, void *vel, int nsteps,
               double dt, double *epot, double *ekin)
{
    if (!c || nsys < 1 || !offsets || nsteps < 0 || !(dt > 0)) return MSM_ERR_ARG;
    if (!c->md_bound) return MSM_ERR_ARG;
    if (nsys > c->prm.max_systems) return MSM_ERR_CAPACITY;
    if (offsets[nsys] > 0 && (!xyzq || !vel)) return MSM_ERR_ARG;
    int rc = check_rigid_offsets(c, nsys, offsets);
    if (rc) return rc;
    rc = build_plan(c, nsys, offsets, domains);
    if (rc) return rc;
    return vv_any(c, xyzq, vel, nsteps, dt, epot, ekin);
}

int msm_vv_mts_run(msm_ctx *c, int nsys, const int64_t *offsets, const double *domains, void *xyzq, void *vel,
                   int nouter, int ninner, double dt, double *epot, double *ekin)
{
    if (!c || nsys < 1 || !offsets || nouter < 0 || ninner < 1 || !(dt > 0)) return MSM_ERR_ARG;
    if (!c->md_bound) return MSM_ERR_ARG;
    if (c->prm.method != MSM_METHOD_MSM) return MSM_ERR_UNSUPPORTED;   // no grid part to split off
    if (nsys > c->prm.max_systems) return MSM_ERR_CAPACITY;
    if (offsets[nsys] > 0 && (!xyzq || !vel)) return MSM_ERR_ARG;
    int rc = check_rigid_offsets(c, nsys, offsets);
    if (rc) return rc;
    rc = build_plan(c, nsys, offsets, domains);
    if (rc) return rc;
    if (c->prm.precision == MSM_FP32) return vv_mts<float>(c, xyzq, vel, nouter, ninner, dt, epot, ekin);
    return vv_mts<double>(c, xyzq, vel, nouter, ninner, dt, epot, ekin);
}

int parareal_run(msm_ctx *fine, msm_ctx *coarse, const parareal_params *pp, int64_t n, const double *q,
                 const double *invm, const double *state0, double *lambda, parareal_report *rep)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!fine || !coarse || !pp || !q || !invm || !state0 || !lambda || !rep || n < 1) return MSM_ERR_ARG;
    const int S = pp->nslices;
    if (S < 1 || pp->kmax < 0 || pp->steps_f < 0 || pp->steps_g < 0 || !(pp->dt_f > 0) || !(pp->dt_g > 0))
        return MSM_ERR_ARG;
    if (!fine->md_bound || !coarse->md_bound || fine->stream != coarse->stream) return MSM_ERR_ARG;
    if ((fine->rigid || coarse->rigid) && n % 3) return MSM_ERR_ARG;
    // rigid triples: the corrected states are projected back onto the constraints
    const bool rigid = fine->rigid && coarse->rigid;
    if (fine->prm.max_atoms < (int64_t)S * n || fine->prm.max_systems < S || coarse->prm.max_atoms < n)
        return MSM_ERR_CAPACITY;
    std::memset(rep, 0, sizeof(*rep));
    hipStream_t s = fine->stream;
    const int64_t N6 = 6 * n;
    auto slot = [&](double *base, int i) { return base + (int64_t)i * N6; };
    int rc = MSM_OK;
    int converged = 0;
    auto status = [&]() {
        int a = msm_get_status(fine), b = msm_get_status(coarse);
        return a ? a : b;
    };

    if (copy_f64(s, state0, lambda, N6) != hipSuccess) return MSM_ERR_HIP;
    // initial coarse sweep: lambda^0_{n+1} = G(lambda^0_n); keep G(lambda^0_n) as the old coarse value
    for (int i = 0; i < S && !rc; i++) {
        rc = propagate(coarse, n, 1, q, invm, slot(lambda, i), slot(lambda, i + 1), pp->steps_g, pp->dt_g);
        if (!rc && copy_f64(s, slot(lambda, i + 1), slot(fine->gold, i), N6) != hipSuccess) rc = MSM_ERR_HIP;
    }
    if (!rc) rc = status();
    unsigned long long *change = (unsigned long long *)fine->md_scalar;
    for (int k = 0; k < pp->kmax && !rc && !converged; k++) {
        // fine propagator on slices k .. S-1 (slices < k are already exact), one batch
        rc = propagate(fine, n, S - k, q, invm, slot(lambda, k), slot(fine->fout, k), pp->steps_f, pp->dt_f);
        if (rc) break;
        if (zero_u64(s, change) != hipSuccess) {
            rc = MSM_ERR_HIP;
            break;
        }
        // serial coarse sweep with the correction
        for (int i = k; i < S && !rc; i++) {
            rc = propagate(coarse, n, 1, q, invm, slot(lambda, i), fine->gnew, pp->steps_g, pp->dt_g);
            if (rc) break;
            const hipError_t e =
                rigid ? parareal_correct_rigid(s, n, slot(lambda, i + 1), slot(fine->fout, i), fine->gnew,
                                               slot(fine->gold, i), invm, fine->tri, change)
                      : parareal_correct(s, N6, slot(lambda, i + 1), slot(fine->fout, i), fine->gnew,
                                         slot(fine->gold, i), change);
            if (e != hipSuccess) rc = MSM_ERR_HIP;
        }
        if (rc) break;
        unsigned long long bits = 0;
        if (hipMemcpyAsync(&bits, change, sizeof(bits), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = MSM_ERR_HIP;
            break;
        }
        double ch;
        std::memcpy(&ch, &bits, sizeof(ch));
        rc = status();
        if (rc) break;
        if (k < 64) rep->residual[k] = ch;
        rep->iterations = k + 1;
        if (ch < pp->tol || k + 1 >= S) converged = 1;
    }
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = MSM_ERR_HIP;
    if (!rc) rc = status();
    rep->converged = converged;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc) return rc;
    return converged ? MSM_OK : MSM_NOT_CONVERGED;
}

int parareal_window_run(msm_ctx *fine, msm_ctx *coarse, const parareal_window_params *pp, int64_t n,
                        const double *q, const double *invm, double *lambda, double *ring,
                        parareal_window_state *st)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!fine || !coarse || !pp || !q || !invm || !lambda || !ring || !st || n < 1) return MSM_ERR_ARG;
    const int T = pp->nslices, W = pp->width;
    if (T < 1 || W < 1 || pp->max_iters < 0 || pp->chunk < 0 || pp->steps_f < 0 || pp->steps_g < 0 ||
        !(pp->dt_f > 0) || !(pp->dt_g > 0) || !(pp->tol >= 0))
        return MSM_ERR_ARG;
    if (st->start < 0 || st->start > T) return MSM_ERR_ARG;
    if (!fine->md_bound || !coarse->md_bound || fine->device != coarse->device) return MSM_ERR_ARG;
    if ((fine->rigid || coarse->rigid) && n % 3) return MSM_ERR_ARG;
    const bool rigid = fine->rigid && coarse->rigid;
    if (fine->prm.max_atoms < (int64_t)W * n || fine->prm.max_systems < W || coarse->prm.max_atoms < n)
        return MSM_ERR_CAPACITY;
    WindowRun r(fine, coarse, pp, n, q, invm, lambda, ring, st, rigid);
    int rc = r.run();
    const int sa = msm_get_status(coarse), sb = msm_get_status(fine);   // both streams idle after these
    if (!rc) rc = sa ? sa : sb;
    st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc) return rc;
    return st->start == T ? MSM_OK : MSM_NOT_CONVERGED;
}

}  // extern "C"
