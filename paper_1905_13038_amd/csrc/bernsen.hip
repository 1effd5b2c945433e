// Bernsen's rule on the window extremes: mask = 1 where the window's range
// mx - mn reaches the contrast threshold and the pixel lies below the
// midrange, 2 I < mn + mx (exact in integers); windows of lower contrast are
// background.  The extremes come from the windowed-quantile kernel with
// q = 0 and q = 1; this kernel is the elementwise decision over I, mn, mx.
#include "internal.hpp"

namespace bz {
namespace {

constexpr int BERNSEN_THREADS = 256;

// One thread per four adjacent pixels of a row (byte loads: rows of any
// alignment); grid.y walks rows.
__global__ __launch_bounds__(BERNSEN_THREADS) void k_bernsen(const uint8_t *I, int64_t ldI, const uint8_t *mn,
                                                             const uint8_t *mx, int64_t ldE, int H, int W,
                                                             int cmin, uint8_t *mask, int64_t ldM)
{
    const int x0 = 4 * (blockIdx.x * BERNSEN_THREADS + threadIdx.x);
    for (int y = blockIdx.y; y < H; y += gridDim.y) {
        const uint8_t *ri = I + (int64_t)y * ldI;
        const uint8_t *rl = mn + (int64_t)y * ldE;
        const uint8_t *rh = mx + (int64_t)y * ldE;
        uint8_t *rm = mask + (int64_t)y * ldM;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + k;
            if (x < W) {
                const int v = ri[x], lo = rl[x], hi = rh[x];
                rm[x] = (hi - lo >= cmin && 2 * v < lo + hi) ? 1 : 0;
            }
        }
    }
}

}  // namespace

hipError_t launch_bernsen(const uint8_t *I, int64_t ldI, const uint8_t *mn, const uint8_t *mx, int64_t ldE,
                          int H, int W, int cmin, uint8_t *mask, int64_t ldM, hipStream_t stream)
{
    const int bx = (W + 4 * BERNSEN_THREADS - 1) / (4 * BERNSEN_THREADS);
    const int by = H < 4096 ? H : 4096;
    hipLaunchKernelGGL(k_bernsen, dim3(bx, by), dim3(BERNSEN_THREADS), 0, stream, I, ldI, mn, mx, ldE, H, W,
                       cmin, mask, ldM);
    return hipGetLastError();
}

}  // namespace bz
