// Small device helpers shared by the kernel files: launch sizes, wave-level
// broadcasts and reductions, workgroup reductions, and the clamped cell index of a grid coordinate.
#pragma once

#include "launch.h"

namespace msmx {
namespace {

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Broadcast lane 0's value to the whole wave as a scalar (the value must
// already be uniform); lets the compiler keep loop bounds and the j-atom
// loads of the pair kernel in scalar registers.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline double uni(double v)
{
    int64_t b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Lane l receives v from lane l ^ m, m a power of two below 64: the values
// of __shfl_xor(v, m, 64), moved by a DPP quad permutation (m = 1, 2) or a
// row rotation (m = 8) inside the VALU, by a swizzle within each half wave
// (m = 4, 16), and by a permute for m = 32.
__device__ inline int xor_lane(int v, int m)
{
    switch (m) {
    case 1: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    case 2: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    case 8: return __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    case 4: return __builtin_amdgcn_ds_swizzle(v, 0x1F | (4 << 10));
    case 16: return __builtin_amdgcn_ds_swizzle(v, 0x1F | (16 << 10));
    default: return __shfl_xor(v, m, 64);
    }
}
__device__ inline float xor_lane(float v, int m) { return __int_as_float(xor_lane(__float_as_int(v), m)); }
__device__ inline double xor_lane(double v, int m)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = xor_lane((int)(b & 0xffffffff), m), hi = xor_lane((int)(b >> 32), m);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Inclusive prefix sum over the 64 lanes of a wave, by DPP: shifts within
// each row of 16 lanes, then each row's total carried into the rows after it
// by the row broadcasts (lanes 15 and 31). Integer sums, so the values of the
// shuffle-based scan.
__device__ inline int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);    // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);    // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);    // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);    // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);   // row_bcast:15 into rows 1 and 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);   // row_bcast:31 into rows 2 and 3
    return x;
}

template <typename T> __device__ inline T wave_min(T v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
template <typename T> __device__ inline T wave_max(T v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum (max) over a workgroup of NT threads in a fixed order: a butterfly
// across the lanes of each wave, then the waves in turn; one barrier. The
// result is valid in thread 0; wpart holds NT / 64 values.
template <int NT> __device__ inline double block_sum(double v, double *wpart)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x % 64 == 0) wpart[threadIdx.x / 64] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) t += wpart[w];
    return t;
}
template <int NT> __device__ inline double block_max(double v, double *wpart)
{
    v = wave_max(v);
    if (threadIdx.x % 64 == 0) wpart[threadIdx.x / 64] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) t = fmax(t, wpart[w]);
    return t;
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Workgroups are handed to the 8 XCDs (each with its own L2) round-robin by
// launch index. Remap the index so that XCD x works on one contiguous range
// of tiles: neighbouring tiles share their halo data in that XCD's L2.
__device__ inline int64_t xcd_remap(int64_t b, int64_t n)
{
    constexpr int kXcd = 8;
    const int64_t base = n / kXcd, rem = n % kXcd;
    const int64_t x = b % kXcd, i = b / kXcd;
    return x * base + (x < rem ? x : rem) + i;
}

template <typename T> __device__ inline int cell_floor(T t, int nc)
{
    // floor, clamped to the cell range; NaN maps to 0
    if (!(t >= T(0))) return 0;
    int c = (int)floor(t);
    return c > nc - 1 ? nc - 1 : c;
}

}  // namespace
}  // namespace msmx
