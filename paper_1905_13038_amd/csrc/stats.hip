// Global statistics of an image (Table 1's L, M and S): the minimum, maximum,
// sum and sum of squares of all gray levels as exact integers, then the mean
// M = T1 / N and population standard deviation S = sqrt(VN / (N N)) with
// VN = N T2 - T1^2 formed exactly in 128 bits and rounded to binary64 once.
//
// Two launches, both graph-capturable (no memset): a one-lane reset of the
// record, then a grid of workgroups that each reduce a set of rows in
// registers and LDS and fold their totals into the record with one integer
// atomic per statistic (order-free, so the result is deterministic).  The
// record's count n serves as the tally of finished workgroups meanwhile; the
// last workgroup to finish forms the mean and the standard deviation and
// sets n.
#include "internal.hpp"

#include <math.h>
#include <stdlib.h>

namespace bz {
namespace {

constexpr int STATS_THREADS = 256;
// Workgroups of the accumulation: every one adds five atomics to the one
// cache line of the record, which serialise, so fewer workgroups with more
// rows in flight each are faster.  Measured on a 4096 x 3072 page (the whole
// call, back to back): 128 workgroups 19.6-20.3 us, 96 20.0, 192 21.1, 256
// 24.2, 64 23.5 (eight rows in flight); with four rows in flight 128
// workgroups took 20.7-20.9 us.  The three-launch form (separate finish, 256
// workgroups, four rows in flight) took 22.1 us.
constexpr int STATS_MAX_BLOCKS = 128;

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

// Workgroup b takes rows b, b + gridDim.x, ...; its lanes stride the columns,
// four gray levels per dword load when rows allow it (AL), else one byte.
// Per-lane sums stay below 2^64 (at most 2^46 pixels of at most 255^2).  The
// four waves of a workgroup combine through LDS, so each workgroup issues one
// atomic per statistic.
__device__ __forceinline__ void add_word(uint32_t d, uint64_t &s, uint64_t &q, uint32_t &lo, uint32_t &hi)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t v = (d >> (8 * b)) & 0xffu;
        s += v;
        q += v * v;
        lo = min(lo, v);
        hi = max(hi, v);
    }
}

// mean = T1 / N and S = sqrt(VN / N^2), VN = N T2 - T1^2 exact in 128 bits and
// rounded to binary64 once; each operation rounded once (no contraction)
__device__ __forceinline__ void gstats_finish(GlobalStats *g, uint64_t N, uint64_t T1, uint64_t T2)
{
#pragma clang fp contract(off)
    const unsigned __int128 VN = (unsigned __int128)N * T2 - (unsigned __int128)T1 * T1;
    const double Nd = (double)N;
    g->mean = (double)T1 / Nd;
    g->stdev = sqrt((double)VN / (Nd * Nd));
    g->n = N;
}

// AL: 0 bytes, 1 dwords (rows 4-byte aligned, W % 4 == 0), 2 16-byte vectors
// (rows 16-byte aligned, W % 16 == 0) with the loads of eight rows in flight.
template <int AL>
__global__ __launch_bounds__(STATS_THREADS) void k_gstats_acc(const uint8_t *I, int H, int W, int64_t ld,
                                                             GlobalStats *g, uint64_t N)
{
    __shared__ uint64_t ws[2][STATS_THREADS / 64];
    __shared__ uint32_t wm[2][STATS_THREADS / 64];
    uint64_t s = 0, q = 0;
    uint32_t lo = 255u, hi = 0u;
    int y = blockIdx.x;
    if (AL == 2) {
        constexpr int U = 8;
        for (; y + (U - 1) * (int)gridDim.x < H; y += U * gridDim.x) {
            for (int x = threadIdx.x; 16 * x < W; x += STATS_THREADS) {
                uint4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    v[u] = ((const uint4 *)(I + (int64_t)(y + u * gridDim.x) * ld))[x];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    add_word(v[u].x, s, q, lo, hi);
                    add_word(v[u].y, s, q, lo, hi);
                    add_word(v[u].z, s, q, lo, hi);
                    add_word(v[u].w, s, q, lo, hi);
                }
            }
        }
        for (; y < H; y += gridDim.x) {
            const uint4 *r16 = (const uint4 *)(I + (int64_t)y * ld);
            for (int x = threadIdx.x; 16 * x < W; x += STATS_THREADS) {
                const uint4 v = r16[x];
                add_word(v.x, s, q, lo, hi);
                add_word(v.y, s, q, lo, hi);
                add_word(v.z, s, q, lo, hi);
                add_word(v.w, s, q, lo, hi);
            }
        }
    }
    for (; AL != 2 && y < H; y += gridDim.x) {
        const uint8_t *row = I + (int64_t)y * ld;
        if (AL == 1) {
            const uint32_t *r4 = (const uint32_t *)row;
            for (int x = threadIdx.x; 4 * x < W; x += STATS_THREADS) {
                const uint32_t d = r4[x];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t v = (d >> (8 * b)) & 0xffu;
                    s += v;
                    q += v * v;
                    lo = min(lo, v);
                    hi = max(hi, v);
                }
            }
        } else {
            for (int x = threadIdx.x; x < W; x += STATS_THREADS) {
                const uint32_t v = row[x];
                s += v;
                q += v * v;
                lo = min(lo, v);
                hi = max(hi, v);
            }
        }
    }
    s = wave_sum_u64(s);
    q = wave_sum_u64(q);
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ws[0][wave] = s;
        ws[1][wave] = q;
        wm[0][wave] = lo;
        wm[1][wave] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < STATS_THREADS / 64; ++i) {
            s += ws[0][i];
            q += ws[1][i];
            lo = min(lo, wm[0][i]);
            hi = max(hi, wm[1][i]);
        }
        atomicAdd((unsigned long long *)&g->sum, (unsigned long long)s);
        atomicAdd((unsigned long long *)&g->sumsq, (unsigned long long)q);
        atomicMin(&g->min, lo);
        atomicMax(&g->max, hi);
        // the last workgroup to finish (every other one's atomics are then
        // done) forms the mean and the standard deviation, reading the sums
        // back through atomics so that no stale cached copy is seen
        __threadfence();
        const unsigned long long done = atomicAdd((unsigned long long *)&g->n, 1ull);
        if (done == (unsigned long long)gridDim.x - 1ull) {
            __threadfence();
            const uint64_t T1 = atomicAdd((unsigned long long *)&g->sum, 0ull);
            const uint64_t T2 = atomicAdd((unsigned long long *)&g->sumsq, 0ull);
            gstats_finish(g, N, T1, T2);
        }
    }
}

}  // namespace

hipError_t launch_global_stats(const uint8_t *I, int H, int W, int64_t ld, GlobalStats *out,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(k_gstats_reset, dim3(1), dim3(1), 0, stream, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nb = STATS_MAX_BLOCKS;
    const char *env = getenv("BZ_GSTATS_BLOCKS");  // tuning override
    if (env && atoi(env) > 0) nb = atoi(env);
    const int blocks = H < nb ? H : nb;
    const uint64_t N = (uint64_t)H * (uint64_t)W;
    const bool al4 = ((uintptr_t)I % 4 == 0) && (ld % 4 == 0) && (W % 4 == 0);
    const bool al16 = ((uintptr_t)I % 16 == 0) && (ld % 16 == 0) && (W % 16 == 0);
    if (al16)
        hipLaunchKernelGGL(k_gstats_acc<2>, dim3(blocks), dim3(STATS_THREADS), 0, stream, I, H, W, ld, out, N);
    else if (al4)
        hipLaunchKernelGGL(k_gstats_acc<1>, dim3(blocks), dim3(STATS_THREADS), 0, stream, I, H, W, ld, out, N);
    else
        hipLaunchKernelGGL(k_gstats_acc<0>, dim3(blocks), dim3(STATS_THREADS), 0, stream, I, H, W, ld, out, N);
    return hipGetLastError();
}

}  // namespace bz
