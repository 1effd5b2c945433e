// Window minimum and maximum over clipped windows.
//
// Windows of at most 64 x 64 (k_ext_fused): one launch, a workgroup per tile
// of 64 x 64 outputs that loads its input tile with the window's halo into
// LDS and runs both separable passes there (see k_ext_fused).
//
// Larger windows: a vertical pass into a 16-bit field (low byte max, high
// byte min) stored transposed, then a horizontal pass into the outputs (and,
// for Bernsen's rule, the mask).
//
// Both forms split each axis into pivot blocks of h (or w) outputs.  All
// windows of a block contain one pivot element c (for rows: c = y0 + u,
// since the window of y0 ends at y0 + u and that of y0 + h - 1 starts
// there), so a window's extremes are those of the suffix from its first
// element up to c and of the prefix from c to its last element: suffix
// extremes are built backwards from c, prefix extremes forwards, about three
// comparisons per output (the van Herk / Gil-Werman scheme).  Elements
// outside the image take the identity (0 for max, 255 for min); every
// window holds its own centre, so none is empty.
#include "device.hpp"
#include "internal.hpp"

#include <stdlib.h>

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

// Gray levels of the horizontal pass's epilogue are loaded EXT_BATCH at a
// time per thread, and ext_strip loads EXT_CHUNK elements of each chain
// together, so that a lane has many loads in flight (one at a time left each
// lane waiting on the latency of every element).
constexpr int EXT_BATCH = 8;
constexpr int EXT_CHUNK = 32;

// LDS rows of 66 16-bit entries (33 dwords, an odd count): a wavefront that
// reads entry (t, k) with t across its lanes then hits distinct banks.
constexpr int EXT_PITCH = EXT_LANES + 2;

// One lane's strip along its line of len elements (fetched by at(i); the
// identity outside [0, len)): the window extremes of the n outputs a0 ..
// a0+n-1, where the window of output a covers a-f+1 .. a+pv and n = f + pv,
// so that every window of the strip holds the pivot a0 + pv.  The result for
// output t goes to s[t * EXT_PITCH].
//
// Entry t is the join of the suffix extremes of elements a0-f+1+t .. a0+pv
// and the prefix extremes of elements a0+pv .. a0+pv+t.  Per chunk of
// EXT_CHUNK outputs the loads of both chains are issued together; the suffix
// chain (built backwards from the pivot, so its chunks go from the last
// outputs down) writes its entries, and the prefix chain, once every suffix
// entry is written, reads each entry back in one batch and writes the join.
// A lane only touches its own entries, so the two passes over s need no
// barrier.  Every load is issued unconditionally, at a position clamped into
// the line, and replaced by the identity where it lies outside: a
// conditional load would become a branch, and the compiler then waits for
// each load before the next.
template <typename F>
__device__ __forceinline__ void ext_strip(F at, int len, int a0, int n, int f, int pv, uint16_t *s)
{
    uint32_t as = EXT_NONE;
    for (int b = 0; b < n; b += EXT_CHUNK) {
        uint32_t vs[EXT_CHUNK];
#pragma unroll
        for (int q = 0; q < EXT_CHUNK; ++q) {
            const int j = n - 1 - (b + q), is = a0 - f + 1 + j;
            vs[q] = at(min(max(is, 0), len - 1));
            vs[q] = (j >= 0 && is >= 0 && is < len) ? vs[q] : EXT_NONE;
        }
#pragma unroll
        for (int q = 0; q < EXT_CHUNK; ++q) {
            const int j = n - 1 - (b + q);
            if (j < 0) break;
            as = ext_join(as, vs[q]);
            s[j * EXT_PITCH] = (uint16_t)as;
        }
    }
    uint32_t ap = EXT_NONE;
    for (int b = 0; b < n; b += EXT_CHUNK) {
        uint32_t vp[EXT_CHUNK], sv[EXT_CHUNK];
#pragma unroll
        for (int q = 0; q < EXT_CHUNK; ++q) {
            const int t = b + q, ip = a0 + pv + t;
            vp[q] = at(min(ip, len - 1));
            vp[q] = (t < n && ip < len) ? vp[q] : EXT_NONE;
        }
#pragma unroll
        for (int q = 0; q < EXT_CHUNK; ++q) sv[q] = b + q < n ? (uint32_t)s[(b + q) * EXT_PITCH] : EXT_NONE;
#pragma unroll
        for (int q = 0; q < EXT_CHUNK; ++q) {
            const int t = b + q;
            if (t >= n) break;
            ap = ext_join(ap, vp[q]);
            s[t * EXT_PITCH] = (uint16_t)ext_join(ap, sv[q]);
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
            // loaded unconditionally (a clamped position), so that the
            // loads of the batch stay in flight together
            const int ic = min(i, RC - 1), kc = ic / C, tc = ic - kc * C;
            iv[q] = mask ? I[(int64_t)(y0 + kc) * ldI + X0 + tc] : 0u;
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

// Fused form for windows of at most EXT_FMAX rows and columns: one
// workgroup per tile of EXT_T x EXT_T outputs, both passes in LDS, no field
// in memory and one launch.
//   1. The input tile (rows y0-o+1 .. y0+EXT_T-1+u, columns x0-l+1 ..
//      x0+EXT_T-1+r; the identity outside the image) into LDS, a thread per
//      column and every other row, EXT_FLOADS loads in flight.
//   2. Vertical extremes of every tile column for the EXT_T output rows, in
//      pivot blocks of h rows (a thread per column and block): the suffix
//      from the block's pivot row up, then the prefix down, each entry
//      joined with the other's.
//   3. The same along the rows of that result, in blocks of w columns (a
//      thread per row and block), into the space of the input tile.
//   4. The outputs (and Bernsen's decision, from the gray levels, loaded
//      unconditionally at clamped positions) stored with threads along
//      rows, four columns per thread.
// An LDS entry holds the maximum in its low byte and 255 minus the minimum
// in its high byte, so that a join is a bytewise maximum and the identity is
// 0; a running value keeps the two bytes in separate 16-bit halves, where the
// join is one packed 16-bit maximum.  LDS rows have an odd number of dwords,
// so that threads on consecutive rows hit distinct banks.
constexpr int EXT_T = 64;
constexpr int EXT_FMAX = 64;
constexpr int EXT_FT = 256;
constexpr int EXT_FLOADS = 16;

typedef unsigned short ext_u16x2 __attribute__((ext_vector_type(2)));

__host__ __device__ inline int ext_fpitch(int cols) { return 2 * (((cols + 1) >> 1) | 1); }

// entry -> running form (max in bits 0..7, 255 - min in bits 16..23) and back
__device__ __forceinline__ uint32_t ext_spread(uint32_t e) { return __builtin_amdgcn_perm(0u, e, 0x0c010c00u); }
__device__ __forceinline__ uint16_t ext_fold(uint32_t a) { return (uint16_t)__builtin_amdgcn_perm(0u, a, 0x0c0c0200u); }
__device__ __forceinline__ uint32_t ext_max2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(ext_u16x2, a),
                                                                  __builtin_bit_cast(ext_u16x2, b)));
}

// One pivot block along a line of LDS entries src[i * st]: outputs t0 ..
// t0+n-1, output t covering elements t .. t+f-1, all holding the pivot p =
// t0 + f - 1.  dst[t * st] = the join of the suffix t .. p (built from the
// pivot down) and the prefix p .. t+f-1.  src and dst are distinct arrays
// (restrict), so the compiler may issue the reads of src ahead of the writes
// to dst.
// The two halves of a pivot block in separate arrays (for the horizontal
// pass, where a thread takes each): suf[t * st] = the suffix t .. p, pre[t *
// st] = the prefix p .. t+f-1.
__device__ __forceinline__ void ext_suffix(const uint16_t *__restrict__ src, uint16_t *__restrict__ suf, int st, int t0,
                                           int n, int p)
{
    uint32_t a = 0;
    const uint16_t *s = src + p * st;
    for (int i = p; i >= t0 + n; --i, s -= st) a = ext_max2(a, ext_spread(*s));
    uint16_t *d = suf + (t0 + n - 1) * st;
#pragma unroll 8
    for (int i = t0 + n - 1; i >= t0; --i, s -= st, d -= st) {
        a = ext_max2(a, ext_spread(*s));
        *d = ext_fold(a);
    }
}

__device__ __forceinline__ void ext_prefix(const uint16_t *__restrict__ src, uint16_t *__restrict__ pre, int st, int t0,
                                           int n, int f)
{
    uint32_t a = 0;
    const uint16_t *s = src + (t0 + f - 1) * st;
    uint16_t *d = pre + t0 * st;
#pragma unroll 8
    for (int t = 0; t < n; ++t, s += st, d += st) {
        a = ext_max2(a, ext_spread(*s));
        *d = ext_fold(a);
    }
}

__device__ __forceinline__ void ext_pivot_block(const uint16_t *__restrict__ src, uint16_t *__restrict__ dst, int st,
                                                int t0, int n, int p, int f)
{
    uint32_t a = 0;
    const uint16_t *s = src + p * st;
    for (int i = p; i >= t0 + n; --i, s -= st) a = ext_max2(a, ext_spread(*s));
    uint16_t *d = dst + (t0 + n - 1) * st;
#pragma unroll 8
    for (int i = t0 + n - 1; i >= t0; --i, s -= st, d -= st) {
        a = ext_max2(a, ext_spread(*s));
        *d = ext_fold(a);
    }
    a = 0;
    s = src + (t0 + f - 1) * st;
    d = dst + t0 * st;
#pragma unroll 8
    for (int t = 0; t < n; ++t, s += st, d += st) {
        a = ext_max2(a, ext_spread(*s));
        *d = ext_fold(ext_max2(a, ext_spread(*d)));
    }
}

__global__ __launch_bounds__(EXT_FT) void k_ext_fused(const uint8_t *__restrict__ I, int64_t ldI, int H, int W, int h,
                                                      int w, int o, int l, int ntx, uint8_t *__restrict__ mn,
                                                      uint8_t *__restrict__ mx, int64_t ldE, int cmin,
                                                      uint8_t *__restrict__ mask, int64_t ldM, int flags)
{
    extern __shared__ uint16_t sh[];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int by = L / ntx, bx = L - by * ntx;
    const int y0 = by * EXT_T, x0 = bx * EXT_T;
    const int RH = EXT_T - 1 + h, CW = EXT_T - 1 + w;
    const int CP = ext_fpitch(CW);
    // tin: [max(RH, 2 EXT_T)][CP], row i = image row y0-o+1+i, column j =
    // x0-l+1+j; after the vertical pass its first 2 EXT_T rows hold the
    // horizontal suffixes and prefixes.  tv: [EXT_T][CP], the vertical
    // extremes of output row t, tile column j.
    uint16_t *tin = sh;
    uint16_t *tv = sh + max(RH, 2 * EXT_T) * CP;
    const int ty0 = y0 - o + 1, tx0 = x0 - l + 1;
    const int tid = threadIdx.x;

    const bool vout = flags & 1, vin = flags & 2;
    // one descriptor over the whole image (vin: 4-byte aligned base and
    // stride, and the image under 2^31 bytes), rounded up to the aligned
    // word holding its last byte
    const __amdgpu_buffer_rsrc_t dimg = rsrc(I, vin ? (uint32_t)((int64_t)(H - 1) * ldI + ((W + 3) & ~3)) : 0u);

    // The gray levels of the quads this thread decides in phase 4 (thread i
    // covers the four columns 4 (i mod 16) .. +3 of tile row i / 16 + 16 k),
    // loaded now so that their latency hides behind phases 1 to 3: one
    // aligned dword per quad where vin (past W: unused), else four bytes at
    // clamped positions; byte j is column x0 + xq + j
    constexpr int QPR = EXT_T / 4;                // quads per tile row
    constexpr int PER = EXT_T * QPR / EXT_FT;     // quads per thread
    const int xq = 4 * (tid % QPR), tr = tid / QPR;
    uint32_t ivw[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = tr + (EXT_FT / QPR) * k;
        const int yc = min(y0 + t, H - 1);
        if (!mask) {
            ivw[k] = 0u;
        } else if (vin) {
            ivw[k] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(dimg, (int)((int64_t)yc * ldI + x0 + xq), 0, 0);
        } else {
            const uint8_t *irow = I + (int64_t)yc * ldI;
            ivw[k] = 0u;
#pragma unroll
            for (int j = 0; j < 4; ++j) ivw[k] |= (uint32_t)irow[min(x0 + xq + j, W - 1)] << (8 * j);
        }
    }

    // 1. input tile.  vin: aligned dwords, one per thread and pass (the
    // columns from tx0 rounded down to a multiple of 4), each byte kept where
    // it lies in the tile and the image; otherwise thread (c, r0) takes
    // column c < CW (at most 127) of rows r0, r0 + 2, ..., one byte each
    if (vin) {
        const int m = tx0 & 3, xb = tx0 - m;
        const int ND = (CW + m + 3) >> 2, N = RH * ND;
        for (int i0 = tid; i0 < N; i0 += EXT_FLOADS * EXT_FT) {
            uint32_t v[EXT_FLOADS];
#pragma unroll
            for (int q = 0; q < EXT_FLOADS; ++q) {
                const int i = min(i0 + q * EXT_FT, N - 1), r = i / ND, d = i - r * ND;
                const int yy = min(max(ty0 + r, 0), H - 1), x = xb + 4 * d;
                const uint32_t off = x >= 0 ? (uint32_t)((int64_t)yy * ldI + x) : 0x80000000u;
                v[q] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(dimg, (int)off, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < EXT_FLOADS; ++q) {
                const int i = i0 + q * EXT_FT;
                if (i >= N) break;
                const int r = i / ND, d = i - r * ND, yy = ty0 + r;
                const bool rin = yy >= 0 && yy < H;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c = 4 * d - m + j, xx = tx0 + c;
                    if (c < 0 || c >= CW) continue;
                    const uint32_t e = (v[q] >> (8 * j)) & 0xffu;
                    tin[r * CP + c] = (uint16_t)((rin && xx >= 0 && xx < W) ? (e | ((255u - e) << 8)) : 0u);
                }
            }
        }
    } else {
        const int c = tid & 127, r0 = tid >> 7;
        const int xx = tx0 + c;
        const bool cin = c < CW && xx >= 0 && xx < W;
        const uint8_t *col = I + min(max(xx, 0), W - 1);
        for (int rb = r0; rb < RH; rb += 2 * EXT_FLOADS) {
            uint32_t v[EXT_FLOADS];
#pragma unroll
            for (int q = 0; q < EXT_FLOADS; ++q) {
                const int yy = min(max(ty0 + rb + 2 * q, 0), H - 1);
                v[q] = col[(int64_t)yy * ldI];
            }
            if (c < CW) {
#pragma unroll
                for (int q = 0; q < EXT_FLOADS; ++q) {
                    const int r = rb + 2 * q, yy = ty0 + r;
                    if (r >= RH) break;
                    const bool in = cin && yy >= 0 && yy < H;
                    tin[r * CP + c] = (uint16_t)(in ? (v[q] | ((255u - v[q]) << 8)) : 0u);
                }
            }
        }
    }
    __syncthreads();

    // 2. vertical: outputs t of block b cover tile rows t .. t+h-1, and all
    // hold the pivot row p = b h + h - 1
    const int nbv = (EXT_T + h - 1) / h;
    for (int task = tid; task < CW * nbv; task += EXT_FT) {
        const int b = task / CW, c = task - b * CW;
        const int t0 = b * h, n = min(h, EXT_T - t0);
        ext_pivot_block(tin + c, tv + c, CP, t0, n, t0 + h - 1, h);
    }
    __syncthreads();

    // 3. horizontal, into tin's space: outputs x of block b cover tile
    // columns x .. x+w-1, and all hold the pivot column b w + w - 1; one
    // thread builds a block's suffixes (into tsu) and another its prefixes
    // (into tpr), joined as they are stored
    uint16_t *tsu = tin, *tpr = tin + EXT_T * CP;  // [EXT_T][CP] each
    const int nbh = (EXT_T + w - 1) / w;
    for (int task = tid; task < 2 * EXT_T * nbh; task += EXT_FT) {
        const int half = task / (EXT_T * nbh), rest = task - half * EXT_T * nbh;
        const int b = rest / EXT_T, t = rest - b * EXT_T;
        const int c0 = b * w, n = min(w, EXT_T - c0);
        if (half == 0)
            ext_suffix(tv + t * CP, tsu + t * CP, 1, c0, n, c0 + w - 1);
        else
            ext_prefix(tv + t * CP, tpr + t * CP, 1, c0, n, w);
    }
    __syncthreads();

    // 4. outputs: thread i covers the four columns 4 (i mod 16) .. +3 of tile
    // row i / 16 + 16 k; as dwords where every row stride and base is a
    // multiple of 4 (vec) and the four columns lie in the image, else as
    // bytes (their gray levels were loaded before phase 1)
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = tr + (EXT_FT / QPR) * k;
        const int yy = y0 + t, xx = x0 + xq;
        if (yy >= H || xx >= W) continue;
        uint32_t hi[4], lo[4], mk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t e = ext_fold(ext_max2(ext_spread(tsu[t * CP + xq + j]), ext_spread(tpr[t * CP + xq + j])));
            hi[j] = e & 0xffu;
            lo[j] = 255u - (e >> 8);
            mk[j] = ((int)(hi[j] - lo[j]) >= cmin && 2 * ((ivw[k] >> (8 * j)) & 0xffu) < lo[j] + hi[j]) ? 1u : 0u;
        }
        uint8_t *pmx = mx + (int64_t)yy * ldE + xx, *pmn = mn + (int64_t)yy * ldE + xx;
        uint8_t *pmk = mask ? mask + (int64_t)yy * ldM + xx : nullptr;
        if (vout && xx + 3 < W) {
            *(uint32_t *)pmx = hi[0] | (hi[1] << 8) | (hi[2] << 16) | (hi[3] << 24);
            *(uint32_t *)pmn = lo[0] | (lo[1] << 8) | (lo[2] << 16) | (lo[3] << 24);
            if (mask) *(uint32_t *)pmk = mk[0] | (mk[1] << 8) | (mk[2] << 16) | (mk[3] << 24);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (xx + j >= W) break;
                pmx[j] = (uint8_t)hi[j];
                pmn[j] = (uint8_t)lo[j];
                if (mask) pmk[j] = (uint8_t)mk[j];
            }
        }
    }
}

size_t ext_fused_lds(int h, int w)
{
    return (size_t)(std::max(EXT_T - 1 + h, 2 * EXT_T) + EXT_T) * (size_t)ext_fpitch(EXT_T - 1 + w) *
           sizeof(uint16_t);
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
    const char *fe = getenv("BZ_EXT_FUSED");
    if (h <= EXT_FMAX && w <= EXT_FMAX && !(fe && atoi(fe) == 0)) {
        const int ntx = (W + EXT_T - 1) / EXT_T, nty = (H + EXT_T - 1) / EXT_T;
        const size_t lds = ext_fused_lds(h, w);
        if (lds > 64 * 1024) {
            const hipError_t ea = hipFuncSetAttribute((const void *)k_ext_fused,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (ea != hipSuccess) return ea;
        }
        const bool vout = ((uintptr_t)mn & 3u) == 0 && ((uintptr_t)mx & 3u) == 0 && (ldE & 3) == 0 &&
                          (mask == nullptr || (((uintptr_t)mask & 3u) == 0 && (ldM & 3) == 0));
        const bool vin = ((uintptr_t)I & 3u) == 0 && (ldI & 3) == 0 && (int64_t)(H - 1) * ldI + W + 3 < (1ll << 31);
        const char *fv = getenv("BZ_EXT_VEC");  // 0: byte loads and stores (tests)
        const int flags = (fv && atoi(fv) == 0) ? 0 : (vout ? 1 : 0) | (vin ? 2 : 0);
        hipLaunchKernelGGL(k_ext_fused, dim3(ntx * nty), dim3(EXT_FT), lds, stream, I, ldI, H, W, h, w, o, l, ntx, mn,
                           mx, ldE, cmin, mask, ldM, flags);
        return hipGetLastError();
    }
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
