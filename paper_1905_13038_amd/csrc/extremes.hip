// Window minimum and maximum over clipped windows, separably: a vertical pass
// into a 16-bit field (low byte max, high byte min) stored transposed, then a
// horizontal pass into the outputs (and, for Bernsen's rule, the mask).
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

#include <algorithm>

namespace bz {
namespace {

constexpr int EXT_LANES = 64;         // lanes of a wavefront: one line each
constexpr int EXT_MAX_STRIPS = 16;    // wavefronts (strips) per workgroup
constexpr int EXT_MAX_THREADS = EXT_LANES * EXT_MAX_STRIPS;

__device__ __forceinline__ uint32_t ext_pack(uint32_t v) { return v | (v << 8); }  // max | min << 8
__device__ __forceinline__ uint32_t ext_join(uint32_t a, uint32_t b)
{
    return max(a & 0xffu, b & 0xffu) | (min(a >> 8, b >> 8) << 8);
}
constexpr uint32_t EXT_NONE = 0xff00u;  // max 0, min 255

// Loads are issued EXT_BATCH at a time per chain, so that a lane has several
// in flight (one at a time left each lane waiting on the latency of every
// element).
constexpr int EXT_BATCH = 8;

// LDS rows of 66 16-bit entries (33 dwords, an odd count): a wavefront that
// reads entry (t, k) with t across its lanes then hits distinct banks.
constexpr int EXT_PITCH = EXT_LANES + 2;

// One lane's strip along its line of len elements (fetched by at(i); the
// identity outside [0, len)): the window extremes of the n outputs a0 ..
// a0+n-1, where the window of output a covers a-f+1 .. a+pv and n = f + pv,
// so that every window of the strip holds the pivot a0 + pv.  The result for
// output t goes to s[t * EXT_PITCH].
//
// The suffix extremes of elements a0-f+1+j .. a0+pv (j from n-1 down to 0)
// and the prefix extremes of elements a0+pv .. a0+pv+t (t from 0 up) are two
// independent chains; they advance together, EXT_BATCH elements of each per
// step, so that the loads of both are in flight at once.  Entry e of s takes
// whichever chain reaches it first as is and joins the other: the suffix
// chain has covered j >= n - (b + EXT_BATCH) after its part of step b, the
// prefix chain t < b before its part.
template <typename F>
__device__ __forceinline__ void ext_strip(F at, int len, int a0, int n, int f, int pv, uint16_t *s)
{
    uint32_t as = EXT_NONE, ap = EXT_NONE;
    for (int b = 0; b < n; b += EXT_BATCH) {
        uint32_t vs[EXT_BATCH], vp[EXT_BATCH];
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int j = n - 1 - (b + q), is = a0 - f + 1 + j;
            vs[q] = (j >= 0 && is >= 0 && is < len) ? at(is) : EXT_NONE;
            const int tq = b + q, ip = a0 + pv + tq;
            vp[q] = (tq < n && ip < len) ? at(ip) : EXT_NONE;
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int j = n - 1 - (b + q);
            if (j < 0) break;
            as = ext_join(as, vs[q]);
            uint16_t *e = &s[j * EXT_PITCH];
            *e = (uint16_t)(j < b ? ext_join(as, *e) : as);
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int tq = b + q;
            if (tq >= n) break;
            ap = ext_join(ap, vp[q]);
            uint16_t *e = &s[tq * EXT_PITCH];
            *e = (uint16_t)(tq >= n - (b + EXT_BATCH) ? ext_join(ap, *e) : ap);
        }
    }
}

// Vertical pass.  Workgroup (bx, by): S wavefronts, columns bx*64 .. +63
// (one per lane), wavefront sy on strip sy of the S strips of h rows from
// Y0 = by*S*h.  Writes the field transposed, VT[x][y] = VT[x*H + y] (16 bits),
// through LDS, so that a store instruction covers consecutive y of a column
// and each column's segment spans S*h rows.
__global__ __launch_bounds__(EXT_MAX_THREADS) void k_ext_v(const uint8_t *I, int64_t ld, int H, int W, int h,
                                                           int o, int u, int S, uint16_t *VT)
{
    extern __shared__ uint16_t suf[];  // [S*h][66]
    const int lane = threadIdx.x % EXT_LANES, sy = threadIdx.x / EXT_LANES;
    const int x0 = blockIdx.x * EXT_LANES;
    const int x = x0 + lane;
    const int Y0 = blockIdx.y * S * h;
    const int R = min(S * h, H - Y0);  // rows of this workgroup
    if (x < W && sy * h < R) {
        const uint8_t *col = I + x;
        auto at = [=](int i) { return ext_pack(col[(int64_t)i * ld]); };
        ext_strip(at, H, Y0 + sy * h, h, o, u, &suf[sy * h * EXT_PITCH + lane]);
    }
    __syncthreads();
    const int C = min(EXT_LANES, W - x0);
    uint16_t *base = VT + (int64_t)x0 * H + Y0;
    for (int i = threadIdx.x; i < R * C; i += blockDim.x) {
        const int k = i / R, t = i - k * R;
        base[(int64_t)k * H + t] = suf[t * EXT_PITCH + k];
    }
}

// Horizontal pass over VT.  Workgroup (bx, by): S wavefronts, rows
// by*64 .. +63 (one per lane), wavefront sx on strip sx of the S strips of w
// columns from X0 = bx*S*w; reads VT[x][y] with consecutive y across the
// lanes.  The results go through LDS, and rows are stored with the lanes
// across columns: mn, mx and, when mask is not null, Bernsen's decision
// from I.
__global__ __launch_bounds__(EXT_MAX_THREADS) void k_ext_h(const uint16_t *__restrict__ VT, int H, int W, int w,
                                                           int l, int r, int S, uint8_t *__restrict__ mn,
                                                           uint8_t *__restrict__ mx, int64_t ldE,
                                                           const uint8_t *__restrict__ I, int64_t ldI, int cmin,
                                                           uint8_t *__restrict__ mask, int64_t ldM)
{
    extern __shared__ uint16_t suf[];  // [S*w][66]
    const int lane = threadIdx.x % EXT_LANES, sx = threadIdx.x / EXT_LANES;
    const int y0 = blockIdx.y * EXT_LANES;
    const int y = y0 + lane;
    const int X0 = blockIdx.x * S * w;
    const int C = min(S * w, W - X0);  // columns of this workgroup
    if (y < H && sx * w < C) {
        const uint16_t *row = VT + y;
        auto at = [=](int i) { return (uint32_t)row[(int64_t)i * H]; };
        ext_strip(at, W, X0 + sx * w, w, l, r, &suf[sx * w * EXT_PITCH + lane]);
    }
    __syncthreads();
    // EXT_BATCH elements per thread at a time: their gray levels (for the
    // mask) are all loaded before any is used
    const int R = min(EXT_LANES, H - y0), RC = R * C;
    for (int i0 = threadIdx.x; i0 < RC; i0 += EXT_BATCH * blockDim.x) {
        int kq[EXT_BATCH], tq[EXT_BATCH];
        uint32_t iv[EXT_BATCH];
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            const int i = i0 + q * blockDim.x;
            kq[q] = i / C;
            tq[q] = i - kq[q] * C;
            iv[q] = (mask && i < RC) ? I[(int64_t)(y0 + kq[q]) * ldI + X0 + tq[q]] : 0u;
        }
#pragma unroll
        for (int q = 0; q < EXT_BATCH; ++q) {
            if (i0 + q * (int)blockDim.x >= RC) break;
            const uint32_t e = suf[tq[q] * EXT_PITCH + kq[q]];
            const uint32_t hi = e & 0xffu, lo = e >> 8;
            const int64_t yk = y0 + kq[q], xo = X0 + tq[q];
            mx[yk * ldE + xo] = (uint8_t)hi;
            mn[yk * ldE + xo] = (uint8_t)lo;
            if (mask) mask[yk * ldM + xo] = ((int)(hi - lo) >= cmin && 2 * iv[q] < lo + hi) ? 1 : 0;
        }
    }
}

}  // namespace

size_t extremes_workspace_bytes(int H, int W) { return (size_t)H * (size_t)W * sizeof(uint16_t); }

// Strips (wavefronts) per workgroup: enough that a column segment of the
// transposed field spans 64 rows (128 bytes) and a row segment of the outputs
// 64 columns, at most 16.
int ext_strips(int len) { return std::min((EXT_LANES + len - 1) / len, EXT_MAX_STRIPS); }

hipError_t launch_extremes(const uint8_t *I, int64_t ldI, int H, int W, int h, int w, uint16_t *V, uint8_t *mn,
                           uint8_t *mx, int64_t ldE, int cmin, uint8_t *mask, int64_t ldM, hipStream_t stream)
{
    const int o = (h + 1) / 2, u = h / 2, l = (w + 1) / 2, r = w / 2;
    const int Sv = ext_strips(h), Sh = ext_strips(w);
    const dim3 gv((W + EXT_LANES - 1) / EXT_LANES, (H + Sv * h - 1) / (Sv * h));
    hipLaunchKernelGGL(k_ext_v, gv, dim3(EXT_LANES * Sv), (size_t)Sv * h * EXT_PITCH * sizeof(uint16_t), stream, I,
                       ldI, H, W, h, o, u, Sv, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gh((W + Sh * w - 1) / (Sh * w), (H + EXT_LANES - 1) / EXT_LANES);
    hipLaunchKernelGGL(k_ext_h, gh, dim3(EXT_LANES * Sh), (size_t)Sh * w * EXT_PITCH * sizeof(uint16_t), stream, V, H,
                       W, w, l, r, Sh, mn, mx, ldE, I, ldI, cmin, mask, ldM);
    return hipGetLastError();
}

}  // namespace bz
