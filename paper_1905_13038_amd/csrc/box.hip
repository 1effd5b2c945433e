// Sliding-window sums, moments and Sauvola/Niblack thresholds on gfx950.
//
// One workgroup owns a tile of output columns [x0, x1) and a strip of output
// rows [y0, y1).  Each lane owns four adjacent columns of the tile's halo'd
// column range and keeps their vertical window sums C (sum of I) and D (sum of
// I^2) in registers, updated row by row with the entering and leaving rows --
// the column recurrence of Section 3.1 / Algorithm 1.  The horizontal window
// sums are differences of a row prefix sum (S = P[j+r] - P[j-l]) built with a
// DPP wavefront scan plus a cross-wave combine through LDS; unsigned 32-bit
// wrap-around keeps the differences exact.  The threshold epilogue forms
// n*S2 - S1^2 exactly (binary64 FMA on exact integers), derives float32 m and
// s, and decides I < t in float32 with a proven error guard; pixels inside the
// guard are re-decided with the binary64 reference sequence.
#include "internal.hpp"

#include <math.h>

namespace bz {
namespace {

// Workgroup b is placed on XCD (b mod 8).  Give every XCD a contiguous range
// of logical tiles so that the halo rows shared by vertically adjacent strips
// stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, i = b >> 3;
    return (x < rem) ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v)
{
    // lanes without a DPP source (or in rows masked off) read 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes of a wavefront (Hillis-Steele within
// rows of 16 lanes, then the row_bcast steps that carry row totals forward).
__device__ __forceinline__ uint32_t wave_scan(uint32_t v)
{
    v += dpp_or_zero<0x111, 0xf>(v);  // row_shr:1
    v += dpp_or_zero<0x112, 0xf>(v);  // row_shr:2
    v += dpp_or_zero<0x114, 0xf>(v);  // row_shr:4
    v += dpp_or_zero<0x118, 0xf>(v);  // row_shr:8
    v += dpp_or_zero<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v += dpp_or_zero<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

// Inclusive prefix sum over the first 16 lanes (row 0).
__device__ __forceinline__ uint32_t row_scan16(uint32_t v)
{
    v += dpp_or_zero<0x111, 0xf>(v);
    v += dpp_or_zero<0x112, 0xf>(v);
    v += dpp_or_zero<0x114, 0xf>(v);
    v += dpp_or_zero<0x118, 0xf>(v);
    return v;
}

// Four pixels of one row starting at column c (c is a multiple of 4).
// Out-of-image columns read as zero (Section 3.2's convention).
template <bool AL>
__device__ __forceinline__ uint32_t load4(const uint8_t *row, int c, int W)
{
    if (c >= 0 && c + 4 <= W) {
        if (AL) return *(const uint32_t *)(row + c);
        return (uint32_t)row[c] | ((uint32_t)row[c + 1] << 8) | ((uint32_t)row[c + 2] << 16) |
               ((uint32_t)row[c + 3] << 24);
    }
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (c + q >= 0 && c + q < W) v |= (uint32_t)row[c + q] << (8 * q);
    return v;
}

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xffu; }

// The binary64 reference decision I < t (each operation rounded once).
__device__ __attribute__((noinline)) bool below_reference(uint32_t I, uint32_t S1, uint32_t S2,
                                                          int64_t n, int mode, double k64,
                                                          double R64)
{
#pragma clang fp contract(off)
    const int64_t Vn = n * (int64_t)S2 - (int64_t)S1 * (int64_t)S1;
    const double nd = (double)n;
    const double m = (double)S1 / nd;
    const double v = (double)Vn / (nd * nd);
    const double s = __builtin_sqrt(v);
    double t;
    if (mode == MODE_SAUVOLA) {
        double q = s / R64;
        q = q - 1.0;
        q = k64 * q;
        q = 1.0 + q;
        t = m * q;
    } else {
        const double q = k64 * s;
        t = m + q;
    }
    return (double)I < t;
}

// Guard of the float32 decision: |t32 - t64| <= 2^-18 * mag, where mag bounds
// the magnitudes of the terms of t (|m| (c1 s + |c0|) for Sauvola,
// m + |k| s for Niblack).  The rounding-error bound of the float32 sequence is
// below 20 units of 2^-24 relative to mag; 2^-18 leaves a factor 3 margin.
constexpr float GUARD = 3.814697265625e-06f;  // 2^-18

template <int MODE, bool AL>
__global__ __launch_bounds__(MAX_THREADS) void k_box(BoxJob a)
{
    extern __shared__ uint32_t smem[];
    const int NT = blockDim.x;
    const int NH = COLS_PER_LANE * NT;   // halo'd columns of the tile
    const int PS = NH + 4;               // prefix row: [0] = 0, [1..NH]
    uint32_t *Pc = smem;                 // [2][PS]
    uint32_t *Pd = smem + 2 * PS;        // [2][PS]
    uint32_t *Tc = smem + 4 * PS;        // [2][MAX_WAVES] wave totals
    uint32_t *Td = Tc + 2 * MAX_WAVES;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = NT >> 6;

    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = L / a.nsy;
    const int sy = L - tx * a.nsy;
    const int x0 = tx * a.tile_w;
    const int x1 = min(x0 + a.tile_w, a.W);
    const int y0 = sy * a.strip;
    const int y1 = min(y0 + a.strip, a.H);
    const int xh = (tx == 0) ? 0 : x0 - a.halo_l;
    const int cb = xh + COLS_PER_LANE * tid;  // first column of this lane

    const int H = a.H, W = a.W, o = a.o, u = a.u;

    if (tid == 0) {
        Pc[0] = 0; Pc[PS] = 0; Pd[0] = 0; Pd[PS] = 0;
    }

    // Per-column constants: prefix indices of the window's right end and of
    // the column just left of it (clamped: prefixes are flat outside the
    // image), the column count nc and its reciprocal.
    int ai[4], bi[4], nc[4];
    float rnc[4];
    bool valid[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = cb + k;
        valid[k] = (j >= x0) && (j < x1);
        const int ar = min(j + a.r, W - 1);
        const int bl = max(j - a.l, -1);
        ai[k] = valid[k] ? ar - xh + 1 : 0;
        bi[k] = valid[k] ? bl - xh + 1 : 0;
        nc[k] = ar - bl;
        rnc[k] = valid[k] ? 1.0f / (float)nc[k] : 0.0f;
    }

    // ---- priming: column sums over rows y0-o .. y0+u-1 ----
    uint32_t C[4] = {0, 0, 0, 0}, D[4] = {0, 0, 0, 0};
    {
        const int p0 = max(y0 - o, 0);
        const int p1 = min(y0 + u - 1, H - 1);
        int row = p0;
        // four rows at a time: transpose the 4x4 bytes so each dword holds one
        // column, then one SAD (sum) and one DOT4 (sum of squares) per column
        for (; row + 3 <= p1; row += 4) {
            const uint32_t r0 = load4<AL>(a.I + (int64_t)row * a.ldI, cb, W);
            const uint32_t r1 = load4<AL>(a.I + (int64_t)(row + 1) * a.ldI, cb, W);
            const uint32_t r2 = load4<AL>(a.I + (int64_t)(row + 2) * a.ldI, cb, W);
            const uint32_t r3 = load4<AL>(a.I + (int64_t)(row + 3) * a.ldI, cb, W);
            const uint32_t x0l = __builtin_amdgcn_perm(r1, r0, 0x05010400u);
            const uint32_t x1l = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
            const uint32_t y0l = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
            const uint32_t y1l = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
            const uint32_t t0 = __builtin_amdgcn_perm(y0l, x0l, 0x05040100u);
            const uint32_t t1 = __builtin_amdgcn_perm(y0l, x0l, 0x07060302u);
            const uint32_t t2 = __builtin_amdgcn_perm(y1l, x1l, 0x05040100u);
            const uint32_t t3 = __builtin_amdgcn_perm(y1l, x1l, 0x07060302u);
            C[0] = __builtin_amdgcn_sad_u8(t0, 0u, C[0]);
            C[1] = __builtin_amdgcn_sad_u8(t1, 0u, C[1]);
            C[2] = __builtin_amdgcn_sad_u8(t2, 0u, C[2]);
            C[3] = __builtin_amdgcn_sad_u8(t3, 0u, C[3]);
            D[0] = __builtin_amdgcn_udot4(t0, t0, D[0], false);
            D[1] = __builtin_amdgcn_udot4(t1, t1, D[1], false);
            D[2] = __builtin_amdgcn_udot4(t2, t2, D[2], false);
            D[3] = __builtin_amdgcn_udot4(t3, t3, D[3], false);
        }
        for (; row <= p1; ++row) {
            const uint32_t v = load4<AL>(a.I + (int64_t)row * a.ldI, cb, W);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t b = byte_of(v, k);
                C[k] += b;
                D[k] += b * b;
            }
        }
    }

    // ---- march down the strip ----
    const bool need_i = (MODE == MODE_SAUVOLA || MODE == MODE_NIBLACK);
    uint32_t na = 0, nb = 0, ni = 0;
    {
        const int ra = y0 + u, rb = y0 - o;
        if (ra < H) na = load4<AL>(a.I + (int64_t)ra * a.ldI, cb, W);
        if (rb >= 0) nb = load4<AL>(a.I + (int64_t)rb * a.ldI, cb, W);
        if (need_i) ni = load4<AL>(a.I + (int64_t)y0 * a.ldI, cb, W);
    }
    for (int y = y0; y < y1; ++y) {
        const int buf = (y - y0) & 1;
        const uint32_t va = na, vb = nb, vi = ni;
        if (y + 1 < y1) {  // prefetch the next row's three dwords
            const int ra = y + 1 + u, rb = y + 1 - o;
            na = (ra < H) ? load4<AL>(a.I + (int64_t)ra * a.ldI, cb, W) : 0u;
            nb = (rb >= 0) ? load4<AL>(a.I + (int64_t)rb * a.ldI, cb, W) : 0u;
            if (need_i) ni = load4<AL>(a.I + (int64_t)(y + 1) * a.ldI, cb, W);
        }
        // column recurrence: add the entering row, drop the leaving row
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ak = (int)byte_of(va, k), bk = (int)byte_of(vb, k);
            const int dk = ak - bk;
            C[k] += (uint32_t)dk;
            D[k] += (uint32_t)(dk * (ak + bk));
        }
        // row prefix sums of C and D over the tile (mod 2^32)
        const uint32_t pc0 = C[0], pc1 = pc0 + C[1], pc2 = pc1 + C[2], pc3 = pc2 + C[3];
        const uint32_t pd0 = D[0], pd1 = pd0 + D[1], pd2 = pd1 + D[2], pd3 = pd2 + D[3];
        const uint32_t sc = wave_scan(pc3);
        const uint32_t sd = wave_scan(pd3);
        if (lane == 63) {
            Tc[buf * MAX_WAVES + wave] = sc;
            Td[buf * MAX_WAVES + wave] = sd;
        }
        __syncthreads();
        uint32_t wc = (lane < nwaves) ? Tc[buf * MAX_WAVES + lane] : 0u;
        uint32_t wd = (lane < nwaves) ? Td[buf * MAX_WAVES + lane] : 0u;
        wc = row_scan16(wc);
        wd = row_scan16(wd);
        const uint32_t oc = (wave > 0) ? (uint32_t)__builtin_amdgcn_readlane((int)wc, wave - 1) : 0u;
        const uint32_t od = (wave > 0) ? (uint32_t)__builtin_amdgcn_readlane((int)wd, wave - 1) : 0u;
        const uint32_t ec = sc - pc3 + oc, ed = sd - pd3 + od;
        uint32_t *pc = Pc + buf * PS + 1 + COLS_PER_LANE * tid;
        uint32_t *pd = Pd + buf * PS + 1 + COLS_PER_LANE * tid;
        pc[0] = pc0 + ec; pc[1] = pc1 + ec; pc[2] = pc2 + ec; pc[3] = pc3 + ec;
        pd[0] = pd0 + ed; pd[1] = pd1 + ed; pd[2] = pd2 + ed; pd[3] = pd3 + ed;
        __syncthreads();

        const uint32_t *Pcb = Pc + buf * PS;
        const uint32_t *Pdb = Pd + buf * PS;
        uint32_t S1[4], S2[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            S1[k] = Pcb[ai[k]] - Pcb[bi[k]];
            S2[k] = Pdb[ai[k]] - Pdb[bi[k]];
        }
        const bool full = valid[0] && valid[3];

        if (MODE == MODE_SUMS) {
            uint32_t *o1 = a.S1 + (int64_t)y * a.ldS + cb;
            uint32_t *o2 = a.S2 + (int64_t)y * a.ldS + cb;
            if (AL && full) {
                *(uint4 *)o1 = make_uint4(S1[0], S1[1], S1[2], S1[3]);
                *(uint4 *)o2 = make_uint4(S2[0], S2[1], S2[2], S2[3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (valid[k]) { o1[k] = S1[k]; o2[k] = S2[k]; }
            }
            continue;
        }

        // moments
        const int nr = min(y + u, H - 1) - max(y - o, -1);
        const float rnr = (nr == a.h) ? a.rh : 1.0f / (float)nr;
        const double nrd = (double)nr;
        float m[4], s[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float rn = rnr * rnc[k];
            m[k] = (float)S1[k] * rn;
            const double s1d = (double)S1[k];
            // n*S2 - S1^2: every term is an integer below 2^53, so exact
            const double vn = __builtin_fma(nrd * (double)nc[k], (double)S2[k], -(s1d * s1d));
            s[k] = __builtin_amdgcn_sqrtf((float)vn) * rn;
        }
        if (a.mean != nullptr) {
            float *om = a.mean + (int64_t)y * a.ldMS + cb;
            float *os = a.stdv + (int64_t)y * a.ldMS + cb;
            if (AL && full) {
                *(float4 *)om = make_float4(m[0], m[1], m[2], m[3]);
                *(float4 *)os = make_float4(s[0], s[1], s[2], s[3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (valid[k]) { om[k] = m[k]; os[k] = s[k]; }
            }
        }
        if (MODE == MODE_MEANSTD) continue;

        // threshold and mask
        uint32_t word = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float t, mag;
            if (MODE == MODE_SAUVOLA) {
                t = m[k] * __builtin_fmaf(a.c1, s[k], a.c0);
                mag = m[k] * __builtin_fmaf(a.c1, s[k], __builtin_fabsf(a.c0));
            } else {
                t = __builtin_fmaf(a.c1, s[k], m[k]);
                mag = __builtin_fmaf(a.kabs, s[k], m[k]);
            }
            const uint32_t iv = byte_of(vi, k);
            const float d = (float)iv - t;
            uint32_t bit = (d < 0.0f) ? 1u : 0u;
            if (valid[k] && (a.force_ref || __builtin_fabsf(d) <= GUARD * mag)) {
                const int64_t n = (int64_t)nr * nc[k];
                bit = below_reference(iv, S1[k], S2[k], n, MODE, a.k64, a.R64) ? 1u : 0u;
            }
            word |= bit << (8 * k);
        }
        uint8_t *omk = a.mask + (int64_t)y * a.ldM + cb;
        if (AL && full) {
            *(uint32_t *)omk = word;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (valid[k]) omk[k] = (uint8_t)byte_of(word, k);
        }
    }
}

template <int MODE, bool AL>
hipError_t launch_mode(const BoxJob &a, hipStream_t stream)
{
    const int NT = a.threads;
    const size_t lds = (size_t)(4 * (COLS_PER_LANE * NT + 4) + 4 * MAX_WAVES) * sizeof(uint32_t);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_box<MODE, AL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = a.ntx * a.nsy;
    hipLaunchKernelGGL((k_box<MODE, AL>), dim3(blocks), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

}  // namespace

void plan_box(BoxJob &a, int strip_override, int threads_override)
{
    a.o = (a.h + 1) / 2;
    a.u = a.h / 2;
    a.l = (a.w + 1) / 2;
    a.r = a.w / 2;
    const int lanes_cols = 256;  // columns covered by one wave
    int NT;
    if (threads_override >= 64 && threads_override <= MAX_THREADS && threads_override % 64 == 0) {
        NT = threads_override;
    } else if (a.W <= MAX_THREADS * COLS_PER_LANE) {
        NT = 64 * ((a.W + lanes_cols - 1) / lanes_cols);
    } else {
        NT = MAX_THREADS;
    }
    const int NH = COLS_PER_LANE * NT;
    a.threads = NT;
    if (a.W <= NH) {
        a.tile_w = a.W;
        a.ntx = 1;
        a.halo_l = 0;
    } else {
        a.halo_l = ((a.l - 1) + 3) & ~3;
        a.tile_w = (NH - a.halo_l - a.r) & ~3;
        if (a.tile_w < 256) {  // too narrow for the window: use the widest block
            a.threads = NT = MAX_THREADS;
            a.tile_w = (COLS_PER_LANE * NT - a.halo_l - a.r) & ~3;
        }
        a.ntx = (a.W + a.tile_w - 1) / a.tile_w;
    }
    int strip;
    if (strip_override > 0) {
        strip = strip_override;
    } else {
        const int waves = NT / 64;
        int per_cu = 16 / waves;
        if (per_cu < 1) per_cu = 1;
        if (per_cu > 8) per_cu = 8;
        const long target = 256L * per_cu;
        strip = (int)(((long)a.H * a.ntx + target - 1) / target);
        if (strip < 4) strip = 4;
    }
    a.strip = strip;
    a.nsy = (a.H + strip - 1) / strip;
}

hipError_t launch_box(const BoxJob &a, hipStream_t stream)
{
    const bool al = a.aligned != 0;
    switch (a.mode) {
    case MODE_SUMS: return al ? launch_mode<MODE_SUMS, true>(a, stream) : launch_mode<MODE_SUMS, false>(a, stream);
    case MODE_MEANSTD: return al ? launch_mode<MODE_MEANSTD, true>(a, stream) : launch_mode<MODE_MEANSTD, false>(a, stream);
    case MODE_SAUVOLA: return al ? launch_mode<MODE_SAUVOLA, true>(a, stream) : launch_mode<MODE_SAUVOLA, false>(a, stream);
    case MODE_NIBLACK: return al ? launch_mode<MODE_NIBLACK, true>(a, stream) : launch_mode<MODE_NIBLACK, false>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bz
