// Windowed quantiles from sliding 256-bin gray-level histograms (Section 3.4).
//
// A workgroup is one wavefront; lane t owns column x0 + t and slides its
// window histogram DOWN a strip of rows: per row it adds the w gray levels of
// the entering row and removes those of the leaving row (the Theta(max{h,w})
// per-pixel cost the paper states).  Histograms are private per lane and live
// in LDS with the bin index as the major dimension (bin b of lane t at word
// b * 64 + t), so each lane always hits its own bank.  Bin updates are
// fire-and-forget LDS atomics.  The quantile is tracked incrementally: the
// lane keeps its current answer Q and lt = #{window values < Q}, adjusts lt
// as values enter and leave, then walks Q up or down until
// lt < rho <= lt + hist[Q].
#include "internal.hpp"

#include <math.h>

namespace bz {
namespace {

constexpr int QLANES = 64;

__device__ __forceinline__ int xcd_remap_q(int b, int n)
{
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, i = b >> 3;
    return (x < rem) ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

__global__ __launch_bounds__(QLANES) void k_quantile(QuantJob a, int seg, int nsy)
{
    extern __shared__ uint32_t hist[];  // [256][QLANES]
    const int lane = threadIdx.x;
    const int L = xcd_remap_q(blockIdx.x, gridDim.x);
    const int tx = L / nsy;
    const int sy = L - tx * nsy;
    const int j = tx * QLANES + lane;
    const bool active = j < a.W;
    const int y0 = sy * seg;
    const int y1 = min(y0 + seg, a.H);
    const int H = a.H, W = a.W;

    uint32_t *hb = hist + lane;
#pragma unroll 8
    for (int b = 0; b < 256; ++b) hb[b * QLANES] = 0u;

    // clipped window columns of this lane
    const int c0 = max(j - a.l + 1, 0);
    const int c1 = active ? min(j + a.r, W - 1) : c0 - 1;
    const int nc = c1 - c0 + 1;

    // histogram of the window of row y0
    {
        const int r0 = max(y0 - a.o + 1, 0), r1 = min(y0 + a.u, H - 1);
        for (int row = r0; row <= r1; ++row) {
            const uint8_t *p = a.I + (int64_t)row * a.ldI;
#pragma unroll 4
            for (int c = c0; c <= c1; ++c) atomicAdd(&hb[(uint32_t)p[c] * QLANES], 1u);
        }
    }

    int Q = 0;   // current answer
    int lt = 0;  // number of window values below Q
    for (int y = y0; y < y1; ++y) {
        if (y > y0) {
            const int ra = y + a.u, rb = y - a.o;
            if (ra < H) {
                const uint8_t *p = a.I + (int64_t)ra * a.ldI;
#pragma unroll 4
                for (int c = c0; c <= c1; ++c) {
                    const uint32_t v = p[c];
                    atomicAdd(&hb[v * QLANES], 1u);
                    lt += (int)(v < (uint32_t)Q);
                }
            }
            if (rb >= 0) {
                const uint8_t *p = a.I + (int64_t)rb * a.ldI;
#pragma unroll 4
                for (int c = c0; c <= c1; ++c) {
                    const uint32_t v = p[c];
                    atomicSub(&hb[v * QLANES], 1u);
                    lt -= (int)(v < (uint32_t)Q);
                }
            }
        }
        if (!active) continue;
        const int nr = min(y + a.u, H - 1) - max(y - a.o, -1);
        const int64_t n = (int64_t)nr * nc;
        int64_t rho = (int64_t)ceil(a.q * (double)n);
        if (rho < 1) rho = 1;
        // walk down while too many values lie below Q
        // (the bounds on Q keep both walks finite whatever the counts hold)
        while (lt >= rho && Q > 0) {
            --Q;
            lt -= (int)hb[Q * QLANES];
        }
        // walk up while the values up to Q are still fewer than rho
        while (Q < 255) {
            const int hq = (int)hb[Q * QLANES];
            if (lt + hq >= rho) break;
            lt += hq;
            ++Q;
        }
        const uint8_t iv = a.I[(int64_t)y * a.ldI + j];
        a.Q[(int64_t)y * a.ldQ + j] = (uint8_t)Q;
        if (a.mask) a.mask[(int64_t)y * a.ldM + j] = (iv < (uint8_t)Q) ? 1 : 0;
    }
}

}  // namespace

hipError_t launch_quantile(const QuantJob &a, hipStream_t stream)
{
    const int ntx = (a.W + QLANES - 1) / QLANES;
    // strips long enough that building the first window (h*w updates) stays
    // small next to the 2w updates per row of the slide
    int seg = (int)(((long)a.H * ntx + 511) / 512);
    if (seg < 2 * a.h) seg = 2 * a.h;
    if (seg < 8) seg = 8;
    if (seg > a.H) seg = a.H;
    const int nsy = (a.H + seg - 1) / seg;
    const size_t lds = 256 * QLANES * sizeof(uint32_t);
    hipLaunchKernelGGL(k_quantile, dim3(ntx * nsy), dim3(QLANES), lds, stream, a, seg, nsy);
    return hipGetLastError();
}

}  // namespace bz
