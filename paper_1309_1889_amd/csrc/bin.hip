// Binning of atoms into cells of edge h (the cells that the short-range pair
// search and the gather forms of anterpolation and interpolation walk), as a
// counting sort: histogram, exclusive scan (block sums, then each block adds
// the sums before it), scatter. The histogram lives in a counts array that is
// zero between evaluations (the scan clears it), so no launch clears it.
// Cells are ranked brick-major (4x4x4 cells per brick) so that 64 consecutive
// sorted atoms form a compact group, while the cells of one brick row along x
// stay contiguous.
// A final per-cell sort by input index makes the order independent of the
// arrival order of the histogram atomics, so every evaluation is bitwise
// reproducible.
#include <algorithm>
#include <cstring>

#include "device_util.h"
#include "launch.h"

namespace msmx {

namespace {


__global__ void k_fill_i32(int *p, int64_t n, int v)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// put_bytes: one launch writes up to kPutWords words carried in its arguments
constexpr int kPutWords = 512;
struct PutChunk {
    uint32_t w[kPutWords];
};
__global__ __launch_bounds__(kPutWords) void k_put(uint32_t *__restrict__ dst, PutChunk c, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = c.w[threadIdx.x];
}

template <typename T> __global__ void k_fill_t(T *p, int64_t n, T v)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__global__ void k_bin_count(DevPlan p, const vec4_t<T> *__restrict__ xyzq, int *__restrict__ cell_of,
                            int *__restrict__ slot_of, int *__restrict__ counts, int *__restrict__ status)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= p.natoms) return;
    const int s = find_segment(p.atom_prefix, p.nsys, i);
    const SysPlan &P = p.sys[s];
    const vec4_t<T> a = xyzq[i];
    const T pos[3] = {a.x, a.y, a.z};
    int c[3];
    int bad = 0;
    for (int d = 0; d < 3; d++) {
        const T t = (pos[d] - T(P.lo[d])) * T(P.inv_h);
        // an atom may sit on the boundary; a rounding overshoot of a fraction
        // of a cell is tolerated and binned into the edge cell
        if (!(t >= T(-1e-4) && t <= T(P.tmax[d] + 1e-4))) bad |= isfinite(t) ? kStatusDomain : kStatusNonFinite;
        int ci = (t >= T(0)) ? (int)floor(t) : 0;
        if (!(t >= T(0))) ci = 0;
        if (ci > P.nc[d] - 1) ci = P.nc[d] - 1;
        c[d] = ci;
    }
    if (!isfinite(a.w)) bad |= kStatusNonFinite;
    if (bad) {
        atomicOr(status, bad);
        atomicOr(status + 1, 1);   // this evaluation's failure flag
    }
    const int cell = (int)(P.cell0 + cell_rank(P, c[0], c[1], c[2]));
    cell_of[i] = cell;
    slot_of[i] = atomicAdd(&counts[cell], 1);
}

// A second binning of the batch's atoms into cells of another edge (cell
// layout from the subset plan pl, one system plan per system of the batch
// plan p): all atoms (maux null: the pair search in cells finer than h), or
// the atoms that carry Lennard-Jones (a nonzero sqrt(eps) in their model
// record; the others get cell -1). The histogram of k_bin_count; positions
// were checked by the batch's own binning, here they are only clamped.
template <typename T>
__global__ void k_sub_bin_count(DevPlan p, const SysPlan *__restrict__ lsys, const vec4_t<T> *__restrict__ xyzq,
                                const vec4_t<T> *__restrict__ maux, int64_t period, int *__restrict__ cell_of,
                                int *__restrict__ slot_of, int *__restrict__ counts)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= p.natoms) return;
    if (maux && maux[i % period].z == T(0)) {
        cell_of[i] = -1;
        return;
    }
    const SysPlan &P = lsys[find_segment(p.atom_prefix, p.nsys, i)];
    const vec4_t<T> a = xyzq[i];
    const T pos[3] = {a.x, a.y, a.z};
    int c[3];
    for (int d = 0; d < 3; d++) {
        const T t = (pos[d] - T(P.lo[d])) * T(P.inv_h);
        int ci = (t >= T(0)) ? (int)floor(t) : 0;   // also 0 for a non-finite t
        if (ci > P.nc[d] - 1) ci = P.nc[d] - 1;
        c[d] = ci;
    }
    const int cell = (int)(P.cell0 + cell_rank(P, c[0], c[1], c[2]));
    cell_of[i] = cell;
    slot_of[i] = atomicAdd(&counts[cell], 1);
}

__global__ void k_sub_scatter(int64_t n, const int *__restrict__ cell_of, const int *__restrict__ slot_of,
                             const int *__restrict__ start, int *__restrict__ order, int *__restrict__ pos_of)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cell = cell_of[i];
    if (cell < 0) pos_of[i] = -1;
    else order[start[cell] + slot_of[i]] = (int)i;
}

// Exclusive scan of int counts: per-block sums, then each block adds the
// sums of the blocks before it to its own scan. A thread takes IPT
// consecutive counts (16-byte loads), waves scan with lane shuffles, and one
// barrier joins the waves of a block.
template <int IPT> __device__ inline void load_counts(const int *__restrict__ in, int64_t n, int64_t idx, int (&v)[IPT])
{
    if (idx + IPT <= n) {
#pragma unroll
        for (int q = 0; q < IPT / 4; q++) {
            const int4 t = *(const int4 *)(in + idx + 4 * q);
            v[4 * q] = t.x, v[4 * q + 1] = t.y, v[4 * q + 2] = t.z, v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; j++) v[j] = idx + j < n ? in[idx + j] : 0;
    }
}

__device__ inline int wave_sum_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int IPT>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int *__restrict__ in, int64_t n,
                                                               int *__restrict__ bsum)
{
    __shared__ int red[kScanThreads / kWave];
    const int64_t idx = blockIdx.x * (int64_t)(kScanThreads * IPT) + (int64_t)threadIdx.x * IPT;
    int v[IPT];
    load_counts<IPT>(in, n, idx, v);
    int acc = 0;
#pragma unroll
    for (int j = 0; j < IPT; j++) acc += v[j];
    acc = wave_sum_i(acc);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kScanThreads / kWave; w++) t += red[w];
        bsum[blockIdx.x] = t;
    }
}

// start[idx] = exclusive prefix of counts for idx < n (the caller passes n =
// cells + 1 with a zero count at the end), clearing counts
template <int IPT>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int *__restrict__ counts, int *__restrict__ start,
                                                              int64_t n, const int *__restrict__ bsum)
{
    __shared__ int wsum[kScanThreads / kWave], wbefore[kScanThreads / kWave];
    const int64_t idx = blockIdx.x * (int64_t)(kScanThreads * IPT) + (int64_t)threadIdx.x * IPT;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    int v[IPT];
    load_counts<IPT>(counts, n, idx, v);
    int acc = 0;
#pragma unroll
    for (int j = 0; j < IPT; j++) acc += v[j];
    // this block's offset: the sum of the earlier blocks' sums
    int before = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanThreads) before += bsum[b];
    before = wave_sum_i(before);
    const int incl = wave_incl_scan(acc);   // inclusive scan over the wave's threads
    if (lane == kWave - 1) wsum[wv] = incl;
    if (lane == 0) wbefore[wv] = before;
    __syncthreads();
    int ex = incl - acc;
    for (int w = 0; w < kScanThreads / kWave; w++) {
        ex += w < wv ? wsum[w] : 0;
        ex += wbefore[w];
    }
    int o[IPT];
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        o[j] = ex;
        ex += v[j];
    }
    if (idx + IPT <= n) {
#pragma unroll
        for (int q = 0; q < IPT / 4; q++) {
            *(int4 *)(start + idx + 4 * q) = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
            *(int4 *)(counts + idx + 4 * q) = make_int4(0, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; j++)
            if (idx + j < n) {
                start[idx + j] = o[j];
                counts[idx + j] = 0;
            }
    }
}

__global__ void k_scatter(int64_t n, const int *__restrict__ cell_of, const int *__restrict__ slot_of,
                          const int *__restrict__ start, int *__restrict__ order)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    order[start[cell_of[i]] + slot_of[i]] = (int)i;
}

// Sort a[0..n) ascending in one thread: insertion sort for a handful of
// atoms, heapsort (O(n log n)) for crowded cells, which arise when
// out-of-domain or non-finite atoms are clamped into one cell.
__device__ inline void sort_range(int *a, int n)
{
    if (n <= 32) {
        for (int i = 1; i < n; i++) {
            int v = a[i], j = i - 1;
            while (j >= 0 && a[j] > v) {
                a[j + 1] = a[j];
                j--;
            }
            a[j + 1] = v;
        }
        return;
    }
    auto sift = [&](int root, int end) {
        while (2 * root + 1 < end) {
            int child = 2 * root + 1;
            if (child + 1 < end && a[child] < a[child + 1]) child++;
            if (a[root] >= a[child]) return;
            int t = a[root];
            a[root] = a[child];
            a[child] = t;
            root = child;
        }
    };
    for (int i = n / 2 - 1; i >= 0; i--) sift(i, n);
    for (int end = n - 1; end > 0; end--) {
        int t = a[0];
        a[0] = a[end];
        a[end] = t;
        sift(0, end);
    }
}

// Order each cell's atoms by input index and gather them (and their model
// records) into cell order, in one of two forms chosen per batch plan (the
// order they produce is the same).
//
// One thread per cell, for up to a few atoms per cell on average.
template <typename T>
__global__ void k_cell_sort_thread(int64_t ncells, const int *__restrict__ start, int *__restrict__ order,
                                   const vec4_t<T> *__restrict__ xyzq, vec4_t<T> *__restrict__ sxyzq,
                                   const vec4_t<T> *__restrict__ maux, vec4_t<T> *__restrict__ saux, int64_t period,
                                   const int *__restrict__ evflag, int *__restrict__ pos_of)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int b = start[c], e = start[c + 1];
    if (e - b > 64 && *evflag) return;   // a cell of clamped atoms of a failed evaluation
    sort_range(order + b, e - b);
    for (int i = b; i < e; i++) sxyzq[i] = xyzq[order[i]];
    if (maux)
        for (int i = b; i < e; i++) saux[i] = maux[order[i] % period];
    if (pos_of)
        for (int i = b; i < e; i++) pos_of[order[i]] = i;
}

// One wave per cell, for crowded cells (coarse h): lane l holds the cell's l-th
// index as the scatter left it, counts the smaller indices of its cell (the
// indices are distinct, so the counts are a permutation) and writes its atom
// to that rank. A cell of more than 64 atoms (non-finite positions are all
// clamped into one) is sorted by its first lane.
template <typename T>
__global__ __launch_bounds__(256) void k_cell_sort(int64_t ncells, const int *__restrict__ start,
                                                   int *__restrict__ order, const vec4_t<T> *__restrict__ xyzq,
                                                   vec4_t<T> *__restrict__ sxyzq, const vec4_t<T> *__restrict__ maux,
                                                   vec4_t<T> *__restrict__ saux, int64_t period,
                                                   const int *__restrict__ evflag, int *__restrict__ pos_of)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    if (c >= ncells) return;
    const int lane = threadIdx.x % 64;
    const int b = __builtin_amdgcn_readfirstlane(start[c]);
    const int n = __builtin_amdgcn_readfirstlane(start[c + 1]) - b;
    if (n == 0) return;
    if (n > 64) {
        if (lane == 0 && !*evflag) {   // a cell of clamped atoms of a failed evaluation is left
            sort_range(order + b, n);
            for (int i = b; i < b + n; i++) sxyzq[i] = xyzq[order[i]];
            if (maux)
                for (int i = b; i < b + n; i++) saux[i] = maux[order[i] % period];
            if (pos_of)
                for (int i = b; i < b + n; i++) pos_of[order[i]] = i;
        }
        return;
    }
    const int v = lane < n ? order[b + lane] : 0x7fffffff;
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += __shfl(v, k, 64) < v ? 1 : 0;
    if (lane < n) {
        order[b + rank] = v;
        sxyzq[b + rank] = xyzq[v];
        if (maux) saux[b + rank] = maux[v % period];
        if (pos_of) pos_of[v] = b + rank;
    }
}

}  // namespace

hipError_t fill_i32(hipStream_t s, int *p, int64_t n, int v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t put_bytes(hipStream_t s, void *dst, const void *src_host, size_t bytes)
{
    const uint32_t *src = (const uint32_t *)src_host;
    const size_t nw = bytes / 4;
    for (size_t o = 0; o < nw; o += kPutWords) {
        PutChunk c;
        const int n = (int)std::min<size_t>(kPutWords, nw - o);
        std::memcpy(c.w, src + o, sizeof(uint32_t) * n);
        hipLaunchKernelGGL(k_put, dim3(1), dim3(kPutWords), 0, s, (uint32_t *)dst + o, c, n);
    }
    return hipGetLastError();
}

template <typename T> hipError_t fill_t(hipStream_t s, T *p, int64_t n, T v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_t<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
template hipError_t fill_t<float>(hipStream_t, float *, int64_t, float);
template hipError_t fill_t<double>(hipStream_t, double *, int64_t, double);

// Exclusive scan of n counts into start, clearing the counts (the caller
// passes n = cells + 1 with a zero count at the end: start[cells] then holds
// the total).
int scan_cells(hipStream_t s, int *counts, int *start, int64_t n, int *block_sums)
{
    // four counts per thread while that takes at most kScanFewBlocks blocks
    // (more blocks in flight), sixteen beyond (fewer block sums to add up)
    const int64_t nb4 = (n + kScanThreads * 4 - 1) / (kScanThreads * 4);
    if (nb4 <= kScanFewBlocks) {
        const unsigned nb = (unsigned)std::max<int64_t>(nb4, 1);
        hipLaunchKernelGGL(k_scan_reduce<4>, dim3(nb), dim3(kScanThreads), 0, s, counts, n, block_sums);
        hipLaunchKernelGGL(k_scan_apply<4>, dim3(nb), dim3(kScanThreads), 0, s, counts, start, n, block_sums);
    } else {
        const unsigned nb = (unsigned)((n + kScanThreads * 16 - 1) / (kScanThreads * 16));
        hipLaunchKernelGGL(k_scan_reduce<16>, dim3(nb), dim3(kScanThreads), 0, s, counts, n, block_sums);
        hipLaunchKernelGGL(k_scan_apply<16>, dim3(nb), dim3(kScanThreads), 0, s, counts, start, n, block_sums);
    }
    return (int)hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::bin(hipStream_t s, const DevPlan &p, const Work<T> &w, const vec4_t<T> *xyzq)
{
    if (p.natoms > 0)
        hipLaunchKernelGGL(k_bin_count<T>, dim3(nblocks(p.natoms, 256)), dim3(256), 0, s, p, xyzq, w.cell_of,
                           w.slot_of, w.counts, w.status);
    scan_cells(s, w.counts, w.cell_start, p.ncells + 1, w.scan_blocks);
    if (p.natoms > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(nblocks(p.natoms, 256)), dim3(256), 0, s, p.natoms, w.cell_of,
                           w.slot_of, w.cell_start, w.order);
        if (p.natoms > 2 * p.ncells)
            hipLaunchKernelGGL(k_cell_sort<T>, dim3(nblocks(p.ncells, 4)), dim3(256), 0, s, p.ncells,
                               w.cell_start, w.order, xyzq, w.sxyzq, (const vec4_t<T> *)w.maux, w.saux, w.period,
                               (const int *)p.evflag, (int *)nullptr);
        else
            hipLaunchKernelGGL(k_cell_sort_thread<T>, dim3(nblocks(p.ncells, 256)), dim3(256), 0, s, p.ncells,
                               w.cell_start, w.order, xyzq, w.sxyzq, (const vec4_t<T> *)w.maux, w.saux, w.period,
                               (const int *)p.evflag, (int *)nullptr);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t bin_sub(hipStream_t s, const DevPlan &p, const DevPlan &pl, const SubBins<T> &b, const vec4_t<T> *xyzq,
                   const vec4_t<T> *maux, int64_t period)
{
    if (p.natoms == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub_bin_count<T>, dim3(nblocks(p.natoms, 256)), dim3(256), 0, s, p, pl.sys, xyzq, maux,
                       period, b.cell_of, b.slot_of, b.cnt);
    scan_cells(s, b.cnt, b.start, pl.ncells + 1, b.blocks);
    hipLaunchKernelGGL(k_sub_scatter, dim3(nblocks(p.natoms, 256)), dim3(256), 0, s, p.natoms, b.cell_of, b.slot_of,
                       b.start, b.order, b.pos_of);
    // per-cell order by input index, the atoms (and their model records, for
    // the Lennard-Jones subset) gathered, and each atom's place recorded
    const vec4_t<T> *ma = b.aux ? maux : nullptr;
    if (pl.natoms > 2 * pl.ncells)
        hipLaunchKernelGGL(k_cell_sort<T>, dim3(nblocks(pl.ncells, 4)), dim3(256), 0, s, pl.ncells, b.start, b.order,
                           xyzq, b.x, ma, b.aux, period, (const int *)p.evflag, b.pos_of);
    else
        hipLaunchKernelGGL(k_cell_sort_thread<T>, dim3(nblocks(pl.ncells, 256)), dim3(256), 0, s, pl.ncells, b.start,
                           b.order, xyzq, b.x, ma, b.aux, period, (const int *)p.evflag, b.pos_of);
    return hipGetLastError();
}
template hipError_t bin_sub<float>(hipStream_t, const DevPlan &, const DevPlan &, const SubBins<float> &,
                                   const vec4_t<float> *, const vec4_t<float> *, int64_t);
template hipError_t bin_sub<double>(hipStream_t, const DevPlan &, const DevPlan &, const SubBins<double> &,
                                    const vec4_t<double> *, const vec4_t<double> *, int64_t);

template hipError_t Launch<float>::bin(hipStream_t, const DevPlan &, const Work<float> &, const vec4_t<float> *);
template hipError_t Launch<double>::bin(hipStream_t, const DevPlan &, const Work<double> &, const vec4_t<double> *);

}  // namespace msmx
