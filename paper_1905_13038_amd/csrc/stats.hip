// Global statistics of an image (Table 1's L, M and S): the minimum, maximum,
// sum and sum of squares of all gray levels as exact integers, then the mean
// M = T1 / N and population standard deviation S = sqrt(VN / (N N)) with
// VN = N T2 - T1^2 formed exactly in 128 bits and rounded to binary64 once.
//
// Three launches, all graph-capturable (no memset): a one-lane reset of the
// record, a grid of workgroups that each reduce a set of rows in registers
// and fold their totals into the record with integer atomics (order-free, so
// the result is deterministic), and a one-lane finish.
#include "internal.hpp"

#include <math.h>

namespace bz {
namespace {

constexpr int STATS_THREADS = 256;
constexpr int STATS_MAX_BLOCKS = 1024;

__global__ void k_gstats_reset(GlobalStats *g)
{
    g->n = 0;
    g->sum = 0;
    g->sumsq = 0;
    g->min = 255u;
    g->max = 0u;
    g->mean = 0.0;
    g->stdev = 0.0;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int d = 32; d >= 1; d >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, d, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int d = 32; d >= 1; d >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
    return v;
}

// Workgroup b takes rows b, b + gridDim.x, ...; its lanes stride the columns.
// Per-lane sums stay below 2^64 (at most 2^46 pixels of at most 255^2).
__global__ __launch_bounds__(STATS_THREADS) void k_gstats_acc(const uint8_t *I, int H, int W, int64_t ld,
                                                             GlobalStats *g)
{
    uint64_t s = 0, q = 0;
    uint32_t lo = 255u, hi = 0u;
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
        const uint8_t *row = I + (int64_t)y * ld;
        for (int x = threadIdx.x; x < W; x += STATS_THREADS) {
            const uint32_t v = row[x];
            s += v;
            q += v * v;
            lo = min(lo, v);
            hi = max(hi, v);
        }
    }
    s = wave_sum_u64(s);
    q = wave_sum_u64(q);
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long *)&g->sum, (unsigned long long)s);
        atomicAdd((unsigned long long *)&g->sumsq, (unsigned long long)q);
        atomicMin(&g->min, lo);
        atomicMax(&g->max, hi);
    }
}

__global__ void k_gstats_finish(GlobalStats *g, uint64_t N)
{
#pragma clang fp contract(off)
    const uint64_t T1 = g->sum, T2 = g->sumsq;
    const unsigned __int128 VN = (unsigned __int128)N * T2 - (unsigned __int128)T1 * T1;
    const double Nd = (double)N;
    g->n = N;
    g->mean = (double)T1 / Nd;
    g->stdev = sqrt((double)VN / (Nd * Nd));
}

}  // namespace

hipError_t launch_global_stats(const uint8_t *I, int H, int W, int64_t ld, GlobalStats *out,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(k_gstats_reset, dim3(1), dim3(1), 0, stream, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int blocks = H < STATS_MAX_BLOCKS ? H : STATS_MAX_BLOCKS;
    hipLaunchKernelGGL(k_gstats_acc, dim3(blocks), dim3(STATS_THREADS), 0, stream, I, H, W, ld, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gstats_finish, dim3(1), dim3(1), 0, stream, out, (uint64_t)H * (uint64_t)W);
    return hipGetLastError();
}

}  // namespace bz
