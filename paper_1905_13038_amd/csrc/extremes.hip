// Window minimum and maximum over clipped windows, separably: a vertical pass
// into a 16-bit field (low byte max, high byte min), then a horizontal pass
// into the outputs (and, for Bernsen's rule, the mask).
//
// Each pass splits its axis into strips of h (or w) outputs.  All windows of
// a strip contain one pivot element c (for rows: c = y0 + u, since the
// window of y0 ends at y0 + u and that of y0 + h - 1 starts there), so
// a window's extremes are those of the suffix from its first element up to c
// and of the prefix from c to its last element: suffix extremes are built
// backwards from c and kept in LDS, prefix extremes forwards, about three
// comparisons per output (the van Herk / Gil-Werman scheme).  Elements
// outside the image take the identity (0 for max, 255 for min); every
// window holds its own centre, so none is empty.
#include "internal.hpp"

namespace bz {
namespace {

constexpr int EXT_LANES = 64;  // one wavefront per workgroup

__device__ __forceinline__ uint32_t ext_pack(uint32_t v) { return v | (v << 8); }  // max | min << 8
__device__ __forceinline__ uint32_t ext_join(uint32_t a, uint32_t b)
{
    return max(a & 0xffu, b & 0xffu) | (min(a >> 8, b >> 8) << 8);
}
constexpr uint32_t EXT_NONE = 0xff00u;  // max 0, min 255

// Loads are issued EXT_BATCH at a time, so that a lane has several in flight
// (one at a time left each lane waiting on the latency of every element).
constexpr int EXT_BATCH = 8;

// Vertical pass.  Workgroup (bx, sy): columns bx*64 .. +63 (one per lane),
// output rows y0 = sy*h .. y0+h-1; writes V[y][x] (16 bits) for them.
__global__ __launch_bounds__(EXT_LANES) void k_ext_v(const uint8_t *I, int64_t ld, int H, int W, int h, int o,
                                                     int u, uint16_t *V)
{
    extern __shared__ uint16_t suf[];  // [h][64]
    const int x = blockIdx.x * EXT_LANES + threadIdx.x;
    const int y0 = blockIdx.y * h;
    const int c = y0 + u;  // pivot row
    const bool col = x < W;
    // suffix extremes of rows y0-o+1+j .. c, j = h-1 down to 0
    uint32_t acc = EXT_NONE;
    for (int jb = h - 1; jb >= 0; jb -= EXT_BATCH) {
        uint32_t v[EXT_BATCH];
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int r = y0 - o + 1 + jb - q;
            v[q] = (col && jb - q >= 0 && r >= 0 && r < H) ? ext_pack(I[(int64_t)r * ld + x]) : EXT_NONE;
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            if (jb - q < 0) break;
            acc = ext_join(acc, v[q]);
            suf[(jb - q) * EXT_LANES + threadIdx.x] = (uint16_t)acc;
        }
    }
    // prefix extremes of rows c .. c+t; output row y0+t
    acc = EXT_NONE;
    for (int tb = 0; tb < h; tb += EXT_BATCH) {
        uint32_t v[EXT_BATCH];
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int r = c + tb + q;
            v[q] = (col && tb + q < h && r < H) ? ext_pack(I[(int64_t)r * ld + x]) : EXT_NONE;
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int t = tb + q, y = y0 + t;
            if (t >= h || y >= H) break;
            acc = ext_join(acc, v[q]);
            if (col) V[(int64_t)y * W + x] = (uint16_t)ext_join(acc, suf[t * EXT_LANES + threadIdx.x]);
        }
    }
}

// Horizontal pass.  Workgroup (sx, by): rows by*64 .. +63 (one per lane),
// output columns x0 = sx*w .. x0+w-1.  Writes mn, mx and, when mask is not
// null, Bernsen's decision from I.
__global__ __launch_bounds__(EXT_LANES) void k_ext_h(const uint16_t *V, int H, int W, int w, int l, int r,
                                                     uint8_t *mn, uint8_t *mx, int64_t ldE, const uint8_t *I,
                                                     int64_t ldI, int cmin, uint8_t *mask, int64_t ldM)
{
    extern __shared__ uint16_t suf[];  // [w][64]
    const int y = blockIdx.y * EXT_LANES + threadIdx.x;
    const int x0 = blockIdx.x * w;
    const int c = x0 + r;  // pivot column
    if (y >= H) return;    // no barriers below: lanes are independent
    const uint16_t *row = V + (int64_t)y * W;
    uint32_t acc = EXT_NONE;
    for (int jb = w - 1; jb >= 0; jb -= EXT_BATCH) {
        uint32_t v[EXT_BATCH];
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int x = x0 - l + 1 + jb - q;
            v[q] = (jb - q >= 0 && x >= 0 && x < W) ? (uint32_t)row[x] : EXT_NONE;
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            if (jb - q < 0) break;
            acc = ext_join(acc, v[q]);
            suf[(jb - q) * EXT_LANES + threadIdx.x] = (uint16_t)acc;
        }
    }
    acc = EXT_NONE;
    for (int tb = 0; tb < w; tb += EXT_BATCH) {
        uint32_t v[EXT_BATCH], iv[EXT_BATCH];
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int x = c + tb + q, xo = x0 + tb + q;
            v[q] = (tb + q < w && x < W) ? (uint32_t)row[x] : EXT_NONE;
            iv[q] = (mask && tb + q < w && xo < W) ? (uint32_t)I[(int64_t)y * ldI + xo] : 0u;
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int t = tb + q, xo = x0 + t;
            if (t >= w || xo >= W) break;
            acc = ext_join(acc, v[q]);
            const uint32_t e = ext_join(acc, suf[t * EXT_LANES + threadIdx.x]);
            const uint32_t hi = e & 0xffu, lo = e >> 8;
            mx[(int64_t)y * ldE + xo] = (uint8_t)hi;
            mn[(int64_t)y * ldE + xo] = (uint8_t)lo;
            if (mask) mask[(int64_t)y * ldM + xo] = ((int)(hi - lo) >= cmin && 2 * iv[q] < lo + hi) ? 1 : 0;
        }
    }
}

}  // namespace

size_t extremes_workspace_bytes(int H, int W) { return (size_t)H * (size_t)W * sizeof(uint16_t); }

hipError_t launch_extremes(const uint8_t *I, int64_t ldI, int H, int W, int h, int w, uint16_t *V, uint8_t *mn,
                           uint8_t *mx, int64_t ldE, int cmin, uint8_t *mask, int64_t ldM, hipStream_t stream)
{
    const int o = (h + 1) / 2, u = h / 2, l = (w + 1) / 2, r = w / 2;
    const dim3 gv((W + EXT_LANES - 1) / EXT_LANES, (H + h - 1) / h);
    hipLaunchKernelGGL(k_ext_v, gv, dim3(EXT_LANES), (size_t)h * EXT_LANES * sizeof(uint16_t), stream, I, ldI,
                       H, W, h, o, u, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gh((W + w - 1) / w, (H + EXT_LANES - 1) / EXT_LANES);
    hipLaunchKernelGGL(k_ext_h, gh, dim3(EXT_LANES), (size_t)w * EXT_LANES * sizeof(uint16_t), stream, V, H, W,
                       w, l, r, mn, mx, ldE, I, ldI, cmin, mask, ldM);
    return hipGetLastError();
}

}  // namespace bz
