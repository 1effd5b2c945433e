// Differentiable ("soft") Sauvola on float32 images with binary64 window sums.
//
// Forward:  y = sigmoid((I - t) / tau), t = m (1 + k_b (s / R - 1)), with m, s
//           from the window sums S1 = sum I, S2 = sum I^2 (Introduction).
// Backward: for L with dL/dy = gy, per pixel p
//           delta = gy y (1 - y),  e = -delta / tau  (= dL/dt),
//           dL/dk_b += e m (s/R - 1),  dL/dR += -e k_b m s / R^2,
//           G1 = dL/dS1 = e (1 + k(s/R-1)) / n - (e k m / R) m / (n s),
//           G2 = dL/dS2 = (e k m / R) / (2 n s)      (s-terms dropped if s = 0),
//           dL/dI_q = delta_q / tau + sum_{p : q in window(p)} (G1_p + 2 I_q G2_p).
//           The last sum is the adjoint of the window sum: a window sum over the
//           window reflected through q (rows q-u .. q+o-1, columns
//           q-r .. q+l-1), so it reuses the same sliding-sum machinery with the
//           extents swapped.
//
// Three phases of one tile kernel: FWD (sums -> y), BWD1 (sums -> G1, G2,
// delta/tau and per-workgroup partials of dL/dk, dL/dR) and ADJ (adjoint
// sums of G1, G2 -> dL/dI), then k_soft_reduce (fixed-order reduction of
// the partials, so the k and R gradients are deterministic).  Nothing is
// saved by the forward: the backward recomputes m and s from I.  A fourth
// phase, SUMS, writes the binary64 window sums themselves (the export that
// tests the running sums against a direct summation).
//
// Layout of a tile (as in the box kernels): lane t owns four adjacent columns
// for the vertical running sums, loaded as one 16-byte vector per row when
// rows allow it; the running sums and the row prefixes are binary64 (the
// inputs are real-valued, so float32 running sums would drift); the epilogue
// lane takes columns t, t+64, t+128, t+192 of its wave's 256, so prefix
// reads are conflict-free and each load or store instruction covers 64
// consecutive elements.  After the sums, the forward's per-pixel arithmetic
// is float32 except n S2 - S1^2 (binary64, against cancellation); the
// backward evaluates m, s, t and z in binary64 (z scales every gradient term,
// and the k and R gradients are sums with cancellation), then the sigmoid
// and the gradient fields in float32.
#include "../../include/binarize.h"
#include "device.hpp"
#include "internal.hpp"

#include <math.h>
#include <stdlib.h>
#include <string.h>

namespace bz {
namespace {

enum Phase { FWD = 0, BWD1 = 1, ADJ = 2, SUMS = 3 };

// Two tile shapes: a workgroup of 4 waves over 1024 halo'd columns (any
// window up to 257), and a single wave for rows of at most 256 columns (no
// workgroup barriers: the wave owns its prefix rows).  Single-wave tiles
// over wider rows would repeat their halo columns in every tile; measured
// on 1024-column rows at h = w = 32 that costs more than the barriers of
// the four-wave tile save.
template <int NT>
struct SoftTile {
    static constexpr int WAVES = NT / 64;
    static constexpr int SNH = 4 * NT;  // halo'd columns of a tile
    // Prefix row (binary64) of a tile: index i (0 = empty prefix) at LPAD + i;
    // the LPAD entries below hold zeros and the RPAD entries above repeat the
    // tile total, so windows reaching past either end need no clamp.  The
    // single-wave tile takes windows with max(l, r + 1) <= 65 and
    // max(r, l - 1) <= 64.
    static constexpr int LPAD = NT == 64 ? 67 : 131;
    static constexpr int RPAD = NT == 64 ? 64 : 256;
    static constexpr int PS = LPAD + 1 + SNH + RPAD;
};
constexpr int WIDE_THREADS = 256;
constexpr int WAVE_THREADS = 64;
constexpr uint32_t SOFF_OUT = 0x80000000u;

struct SoftArgs {
    const float *I;     // B images, image b at I + b*H*ld
    const float *gy;    // upstream gradient (BWD1), same layout as I
    float *y;           // FWD output, layout of I
    float *G1, *G2, *dd;  // BWD1 outputs / ADJ inputs: B*H*W, row stride W
    float *gI;          // ADJ output, layout of I
    double *S1, *S2;    // SUMS outputs: B images of H rows, row stride ldS
    int64_t ldS;
    double *part;       // BWD1: per-workgroup (dk, dR) partials
    const float *k;     // [B] device
    const float *R;     // [1] device
    int B, H, W;
    int64_t ld;
    int h, w;
    int o, u, l, r;     // forward window extents
    int eo, eu, el, er; // extents summed by this phase
    float tau;
    int tile_w, ntx, halo_l, strip, nsy;
    int nt;             // tile shape: 64 (one wave) or 256 threads
    int vec;            // rows allow 16-byte loads (ld and W multiples of 4)
};

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

// inclusive prefix over the 64 lanes, in a fixed order
__device__ __forceinline__ double wave_scan_f64(double v)
{
    v += dpp_f64<0x111, 0xf>(v);
    v += dpp_f64<0x112, 0xf>(v);
    v += dpp_f64<0x114, 0xf>(v);
    v += dpp_f64<0x118, 0xf>(v);
    v += dpp_f64<0x142, 0xa>(v);
    v += dpp_f64<0x143, 0xc>(v);
    return v;
}

__device__ __forceinline__ double lane_f64(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// 1/n for a count n >= 1: a float32 estimate refined by two binary64
// Newton steps (relative error below 2^-52).
__device__ __forceinline__ double recip64(int n)
{
    const double d = (double)n;
    double r = (double)__builtin_amdgcn_rcpf((float)n);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    return r;
}

// sqrt(v) for v > 0 (0 for v <= 0): a float32 square root refined by one
// binary64 Newton step, relative error about 2^-46 (both float32 estimates
// carry about 2^-23).  Values below the float32 normal range take the
// binary64 square root.
__device__ __forceinline__ double sqrt_pos(double v)
{
    const float vf = (float)v;
    if (!(vf >= 0x1p-100f)) return v > 0.0 ? __builtin_sqrt(v) : 0.0;
    const float sf = __builtin_amdgcn_sqrtf(vf);
    const double x = (double)sf;
    const double h = 0.5 * (double)__builtin_amdgcn_rcpf(sf);
    return __builtin_fma(__builtin_fma(-x, x, v), h, x);
}

// Four adjacent floats of one row (columns cb .. cb+3) through a descriptor
// over whole rows, the row chosen by the scalar byte offset so.  VEC: one
// 16-byte load (all four columns inside or outside the image together);
// otherwise four dword loads with per-column offsets.  Offsets of 2^31 (and
// descriptors of no bytes, for rows outside the image) read zero.
template <bool VEC>
struct QuadLoader {
    uint32_t off[4];
    __device__ __forceinline__ QuadLoader(int cb, int W)
    {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            off[q] = (cb + q >= 0 && cb + q < W) ? 4u * (uint32_t)(cb + q) : SOFF_OUT;
    }
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t d, uint32_t so, float v[4]) const
    {
        if (VEC) {
            typedef int v4i __attribute__((ext_vector_type(4)));
            const v4i x = __builtin_amdgcn_raw_buffer_load_b128(d, (int)off[0], (int)so, 0);
            v[0] = __int_as_float(x[0]);
            v[1] = __int_as_float(x[1]);
            v[2] = __int_as_float(x[2]);
            v[3] = __int_as_float(x[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[q] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(d, (int)off[q], (int)so, 0));
        }
    }
};

template <int PH, bool VEC, int NT>
__global__ __launch_bounds__(NT) void k_soft(SoftArgs a)
{
    using T = SoftTile<NT>;
    constexpr int SLPAD = T::LPAD, SRPAD = T::RPAD, SNH = T::SNH, SOFT_WAVES = T::WAVES;
    static_assert(NT == 64 || NT == 256, "tile shapes: one wave, or four");
    __shared__ double P[2][T::PS];               // prefix rows of S1 and S2
    __shared__ double Tl[2][NT == 64 ? 1 : NT];  // lane totals (4 columns each)
    __shared__ double El[2][NT + 4];             // exclusive lane offsets, then the row total
    __shared__ double Red[2][SOFT_WAVES];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int per_img = a.ntx * a.nsy;
    const int b = L / per_img;
    const int rem = L - b * per_img;
    const int tx = rem / a.nsy, sy = rem - tx * a.nsy;
    const int x0 = tx * a.tile_w, x1 = min(x0 + a.tile_w, a.W);
    const int y0 = sy * a.strip, y1 = min(y0 + a.strip, a.H);
    const int xh = (tx == 0) ? 0 : x0 - a.halo_l;
    const int cb = xh + 4 * tid;
    const int H = a.H, W = a.W;
    const int64_t ld = a.ld;

    for (int i = tid; i < 2 * (SLPAD + 1); i += NT) P[i / (SLPAD + 1)][i % (SLPAD + 1)] = 0.0;

    // rows read by the vertical pass: rlo .. rhi of image b
    const int rlo = max(y0 - a.eo, 0), rhi = min(y1 - 1 + a.eu, H - 1);
    const QuadLoader<VEC> ql(cb, W);
    const int64_t pitch = (PH == ADJ) ? (int64_t)W : ld;  // rows of the summed fields
    const uint32_t span = (uint32_t)(4 * ((int64_t)(rhi - rlo) * pitch + W));
    const float *src1 = (PH == ADJ) ? a.G1 : a.I;
    // raw values of a row: I, or (G1, G2); rows outside [rlo, rhi] read zero
    const float *base1 = src1 + ((int64_t)b * H + rlo) * pitch;
    const float *base2 = (PH == ADJ) ? a.G2 + ((int64_t)b * H + rlo) * pitch : nullptr;
    auto load_row = [&](int row, float v1[4], float v2[4]) {
        const bool in = row >= rlo && row <= rhi;
        const uint32_t so = in ? (uint32_t)(4 * (int64_t)(row - rlo) * pitch) : 0u;
        ql.load(rsrc(base1, in ? span : 0u), so, v1);
        if (PH == ADJ) ql.load(rsrc(base2, in ? span : 0u), so, v2);
    };
    // X1 += sign v1 and X2 += sign (v1^2 or v2), binary64 (squares exact)
    auto accumulate = [&](double X1[4], double X2[4], const float v1[4], const float v2[4], bool add) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double d1 = (double)v1[q];
            if (add) {
                X1[q] += d1;
                X2[q] = (PH == ADJ) ? X2[q] + (double)v2[q] : __builtin_fma(d1, d1, X2[q]);
            } else {
                X1[q] -= d1;
                X2[q] = (PH == ADJ) ? X2[q] - (double)v2[q] : __builtin_fma(-d1, d1, X2[q]);
            }
        }
    };

    // epilogue columns x0 + eo + 64 j (j = 0..3) and their element offsets
    const int eo = 256 * wave + lane;
    const int ec0 = x0 + eo;
    const int ai0 = SLPAD + ec0 + a.er - xh + 1;  // prefix index of j + er
    const int bi0 = SLPAD + ec0 - a.el - xh + 1;  // prefix index of j - el
    uint32_t oe[4];  // byte offset of the column in a row, 2^31 outside the tile
    double ncd[4], rnc[4];  // forward column counts and their reciprocals
    float rnf[4] = {0, 0, 0, 0};  // FWD: float32 1/n of the current row count
    int nr_prev = -1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = ec0 + 64 * j;
        oe[j] = (c < x1) ? 4u * (uint32_t)c : SOFF_OUT;
        ncd[j] = (double)max(min(c + a.r, W - 1) - max(c - a.l, -1), 1);
        rnc[j] = 1.0 / ncd[j];
    }
    // descriptors of the epilogue's per-pixel rows of image b (byte offset of
    // row y: 4 y pitch); the planner keeps image spans under 2^31 bytes
    const uint32_t img_bytes = (uint32_t)(4 * ((int64_t)(H - 1) * ld + W));
    const uint32_t fld_bytes = (uint32_t)(4 * (int64_t)H * W);
    const __amdgpu_buffer_rsrc_t dI = rsrc(a.I + (int64_t)b * H * ld, img_bytes);

    float kb = 0.0f, kR = 0.0f, rRf = 0.0f;
    double kb64 = 0.0, rR64 = 1.0, cR64 = 0.0;
    if (PH == FWD || PH == BWD1) {
        kb = a.k[b];
        kb64 = (double)kb;
        rR64 = 1.0 / (double)a.R[0];
        kR = (float)(kb64 * rR64);
        rRf = (float)rR64;
        cR64 = -kb64 * rR64 * rR64;  // dt/dR = -k m s / R^2
    }
    const float rtau = 1.0f / a.tau;

    // priming: rows y0-eo .. y0+eu-1, loaded PRIME rows at a time
    constexpr int PRIME = 8;
    double C[4] = {0, 0, 0, 0}, D[4] = {0, 0, 0, 0};
    for (int r0 = y0 - a.eo; r0 < y0 + a.eu; r0 += PRIME) {
        float v1[PRIME][4], v2[PRIME][4];
#pragma unroll
        for (int i = 0; i < PRIME; ++i) load_row(r0 + i < y0 + a.eu ? r0 + i : -1, v1[i], v2[i]);
#pragma unroll
        for (int i = 0; i < PRIME; ++i) accumulate(C, D, v1[i], v2[i], true);
    }

    // the vertical pass of row y reads rows y + eu (entering) and y - eo
    // (leaving); each row's are loaded one row ahead
    float ne1[4], ne2[4], nl1[4], nl2[4];
    load_row(y0 + a.eu, ne1, ne2);
    load_row(y0 - a.eo, nl1, nl2);
    double dk_acc = 0.0, dR_acc = 0.0;
    const __amdgpu_buffer_rsrc_t dX =  // second per-pixel input of the epilogue
        (PH == BWD1) ? rsrc(a.gy + (int64_t)b * H * ld, img_bytes)
                     : rsrc((PH == ADJ) ? a.dd + (int64_t)b * H * W : a.I, (PH == ADJ) ? fld_bytes : 0u);
    // the epilogue's per-pixel inputs of a row (I, and gy or dd), loaded one
    // row ahead; row H lies past the descriptors and reads zero
    auto load_epi = [&](int y, float Iv[4], float Xv[4]) {
        const uint32_t soI = (uint32_t)(4 * (int64_t)y * ld);
        const uint32_t soF = (uint32_t)(4 * (int64_t)y * W);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Iv[j] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(dI, (int)oe[j], (int)soI, 0));
            if (PH == BWD1 || PH == ADJ)
                Xv[j] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(dX, (int)oe[j],
                                                                            (int)(PH == ADJ ? soF : soI), 0));
        }
    };
    float nIv[4], nXv[4];
    load_epi(y0, nIv, nXv);
    for (int y = y0; y < y1; ++y) {
        const uint32_t soI = (uint32_t)(4 * (int64_t)y * ld);
        const uint32_t soF = (uint32_t)(4 * (int64_t)y * W);
        float Ivs[4], Xvs[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Ivs[j] = nIv[j];
            Xvs[j] = (PH == BWD1 || PH == ADJ) ? nXv[j] : 0.0f;
        }
        load_epi(y + 1, nIv, nXv);
        {
            float e1[4], e2[4], l1[4], l2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                e1[q] = ne1[q];
                e2[q] = ne2[q];
                l1[q] = nl1[q];
                l2[q] = nl2[q];
            }
            load_row(y + 1 < y1 ? y + 1 + a.eu : -1, ne1, ne2);
            load_row(y + 1 < y1 ? y + 1 - a.eo : -1, nl1, nl2);
            accumulate(C, D, e1, e2, true);
            accumulate(C, D, l1, l2, false);
        }
        // row prefix: lane-local prefix of its 4 columns, then the lane
        // offsets in a fixed order (four-wave tiles: wave 0 scans the S1 lane
        // totals and wave 1 those of S2)
        double pc[4], pd[4];
        pc[0] = C[0]; pc[1] = pc[0] + C[1]; pc[2] = pc[1] + C[2]; pc[3] = pc[2] + C[3];
        pd[0] = D[0]; pd[1] = pd[0] + D[1]; pd[2] = pd[1] + D[2]; pd[3] = pd[2] + D[3];
        double ec, ed, tc, td;
        if (NT == 64) {
            // one wave: its scan gives the offsets and the row total directly
            const double ic = wave_scan_f64(pc[3]), id = wave_scan_f64(pd[3]);
            ec = ic - pc[3];
            ed = id - pd[3];
            tc = lane_f64(ic, 63);
            td = lane_f64(id, 63);
        } else {
            Tl[0][tid] = pc[3];
            Tl[1][tid] = pd[3];
            __syncthreads();
            if (wave < 2) {
                const double *Tw = &Tl[wave][4 * lane];
                const double v0 = Tw[0], v1 = v0 + Tw[1], v2 = v1 + Tw[2], v3 = v2 + Tw[3];
                const double inc = wave_scan_f64(v3);
                const double ex = inc - v3;
                double *E = &El[wave][4 * lane];
                E[0] = ex;
                E[1] = ex + v0;
                E[2] = ex + v1;
                E[3] = ex + v2;
                if (lane == 63) El[wave][NT] = inc;
            }
            __syncthreads();
            ec = El[0][tid];
            ed = El[1][tid];
            tc = El[0][NT];
            td = El[1][NT];
        }
        if (NT == 64) __syncthreads();  // the previous row's epilogue read P
        {
            double *p1 = &P[0][SLPAD + 1 + 4 * tid];
            double *p2 = &P[1][SLPAD + 1 + 4 * tid];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                p1[q] = pc[q] + ec;
                p2[q] = pd[q] + ed;
            }
            if (wave == SOFT_WAVES - 1) {  // right pad: the tile totals
#pragma unroll
                for (int q = 0; q < SRPAD / 64; ++q) {
                    P[0][SLPAD + 1 + SNH + 64 * q + lane] = tc;
                    P[1][SLPAD + 1 + SNH + 64 * q + lane] = td;
                }
            }
        }
        __syncthreads();

        // the row's epilogue at raised wave priority: waves storing a row's
        // outputs issue ahead of waves still in the column pass (measured on
        // 32 pages of 1024 x 1024: backward 425 -> 418 us at h = 75, 361 ->
        // 358 us at h = 32; the forward unchanged)
        __builtin_amdgcn_s_setprio(3);
        float rowk = 0.0f, rowR = 0.0f;  // this row's dL/dk and dL/dR / (-k / R^2) terms
        const int nr = min(y + a.u, H - 1) - max(y - a.o, -1);
        const double rnr = recip64(nr);
        if (PH == FWD && nr != nr_prev) {  // row counts change only near the image's top and bottom
            nr_prev = nr;
#pragma unroll
            for (int j = 0; j < 4; ++j) rnf[j] = (float)(rnr * rnc[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double S1 = P[0][ai0 + 64 * j] - P[0][bi0 + 64 * j];
            const double S2 = P[1][ai0 + 64 * j] - P[1][bi0 + 64 * j];
            const float Iv = Ivs[j];
            if (PH == SUMS) {
                // binary64 sums: element offset 8 c of column c (2^31 outside the tile)
                const uint32_t o8 = oe[j] == SOFF_OUT ? SOFF_OUT : 2u * oe[j];
                const uint32_t so8 = (uint32_t)(8 * (int64_t)y * a.ldS);
                const uint32_t sbytes = (uint32_t)(8 * ((int64_t)(H - 1) * a.ldS + W));
                typedef int v2i __attribute__((ext_vector_type(2)));
                const v2i w1 = {__double2loint(S1), __double2hiint(S1)};
                const v2i w2 = {__double2loint(S2), __double2hiint(S2)};
                __builtin_amdgcn_raw_buffer_store_b64(w1, rsrc(a.S1 + (int64_t)b * H * a.ldS, sbytes), (int)o8,
                                                      (int)so8, 0);
                __builtin_amdgcn_raw_buffer_store_b64(w2, rsrc(a.S2 + (int64_t)b * H * a.ldS, sbytes), (int)o8,
                                                      (int)so8, 0);
                continue;
            }
            if (PH == ADJ) {
                const float g = Xvs[j] + (float)S1 + 2.0f * Iv * (float)S2;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(g), rsrc(a.gI + (int64_t)b * H * ld, img_bytes),
                                                      (int)oe[j], (int)soI, 2);
                continue;
            }
            if (PH == FWD) {
                // y needs t to about 1e-4: float32 from the binary64 sums on
                // (n S2 - S1^2 is formed in binary64 against cancellation)
                const float m = (float)S1 * rnf[j];
                const float vf = (float)__builtin_fma((double)nr * ncd[j], S2, -(S1 * S1));
                const float s = vf > 0.0f ? __builtin_amdgcn_sqrtf(vf) * rnf[j] : 0.0f;
                const float t = m * __builtin_fmaf(kb, __builtin_fmaf(s, rRf, -1.0f), 1.0f);
                const float z = (Iv - t) * rtau;
                const float ea = __expf(-fabsf(z));
                const float yv = (z >= 0.0f ? 1.0f : ea) * __builtin_amdgcn_rcpf(1.0f + ea);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(yv), rsrc(a.y + (int64_t)b * H * ld, img_bytes),
                                                      (int)oe[j], (int)soI, 2);
                continue;
            }
            // the gradients: the threshold and z in binary64 (z decides
            // delta, which every gradient scales), the sigmoid and what
            // follows in float32
            const double rn64 = rnr * rnc[j];
            const double n = (double)nr * ncd[j];
            const double m64 = S1 * rn64;
            const double vn = __builtin_fma(n, S2, -(S1 * S1));
            const double s64 = sqrt_pos(vn) * rn64;
            const double q64 = __builtin_fma(s64, rR64, -1.0);     // s/R - 1
            const double t64 = __builtin_fma(m64 * kb64, q64, m64);
            const float z = (float)((double)Iv - t64) * rtau;
            // sigmoid through e^-|z| <= 1: y and y (1 - y) = e / (1 + e)^2
            // keep their relative accuracy at both tails
            const float ea = __expf(-fabsf(z));
            const float rr = __builtin_amdgcn_rcpf(1.0f + ea);
            const float delta = Xvs[j] * (ea * rr * rr);
            const float e = -delta * rtau;
            const float m = (float)m64, s = (float)s64, q = (float)q64, rn = (float)rn64;
            // columns outside the tile read gy = 0, so e = 0 there
            const float em = e * m;
            rowk = __builtin_fmaf(em, q, rowk);
            rowR = __builtin_fmaf(em, s, rowR);
            const float aa = e * __builtin_fmaf(kb, q, 1.0f);
            const float beta = em * kR;
            // 1 / (n s), or 0 where s = 0: the s-terms drop out there
            const float rns = s > 0.0f ? rn * __builtin_amdgcn_rcpf(s) : 0.0f;
            const float g1 = __builtin_fmaf(-beta * m, rns, aa * rn);
            const float g2 = 0.5f * beta * rns;
            const __amdgpu_buffer_rsrc_t f1 = rsrc(a.G1 + (int64_t)b * H * W, fld_bytes);
            const __amdgpu_buffer_rsrc_t f2 = rsrc(a.G2 + (int64_t)b * H * W, fld_bytes);
            const __amdgpu_buffer_rsrc_t f3 = rsrc(a.dd + (int64_t)b * H * W, fld_bytes);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(g1), f1, (int)oe[j], (int)soF, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(g2), f2, (int)oe[j], (int)soF, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(delta * rtau), f3, (int)oe[j], (int)soF, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        if (PH == BWD1) {
            dk_acc += (double)rowk;
            dR_acc += (double)rowR * cR64;
        }
    }
    if (PH == BWD1) {
        const double wk = lane_f64(wave_scan_f64(dk_acc), 63), wr = lane_f64(wave_scan_f64(dR_acc), 63);
        if (lane == 0) {
            Red[0][wave] = wk;
            Red[1][wave] = wr;
        }
        __syncthreads();
        if (tid == 0) {
            double sk = 0.0, sr = 0.0;
            for (int w2 = 0; w2 < SOFT_WAVES; ++w2) {
                sk += Red[0][w2];
                sr += Red[1][w2];
            }
            a.part[2 * (int64_t)L] = sk;
            a.part[2 * (int64_t)L + 1] = sr;
        }
    }
}

// gk[b] = sum of image b's partials, gR = sum of all, each in a fixed order
// (lane-strided sums, then a fixed wave scan), so repeated runs agree.
constexpr int REDUCE_THREADS = 256;
__global__ __launch_bounds__(REDUCE_THREADS) void k_soft_reduce(const double *part, int B, int per_img,
                                                                float *gk, float *gR)
{
    __shared__ double wsum[REDUCE_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int b = wave; b < B; b += REDUCE_THREADS / 64) {
        double s = 0.0;
        for (int i = lane; i < per_img; i += 64) s += part[2 * ((int64_t)b * per_img + i)];
        s = lane_f64(wave_scan_f64(s), 63);
        if (lane == 0) gk[b] = (float)s;
    }
    double s = 0.0;
    const int64_t total = (int64_t)B * per_img;
    for (int64_t i = tid; i < total; i += REDUCE_THREADS) s += part[2 * i + 1];
    s = lane_f64(wave_scan_f64(s), 63);
    if (lane == 0) wsum[wave] = s;
    __syncthreads();
    if (tid == 0) {
        double r = 0.0;
        for (int w = 0; w < REDUCE_THREADS / 64; ++w) r += wsum[w];
        gR[0] = (float)r;
    }
}

// Strip height of a phase (or the whole image when shorter): the forward
// and the sums export take 8 rows, the backward's phases min(h, 32) rows and
// at least 8.  env (8 .. 32 rows) overrides it for tuning.
//
// Measured on 32 float32 pages of 1024 x 1024, forward: 8-row strips took
// 78-84 us at h = 9 .. 32 against 82-87 us for min(h, 32) rows, and 91 and
// 104 us at h = 51 and 75 against 110 and 125 us for 32 rows.  An XCD then
// holds the strips of one page at a time, all resident together, and the
// priming rows of adjacent strips are shared through its L2.  The backward
// measured slower with 8-row strips (BWD1 by 24 us at h = 32), so it keeps
// the taller ones.
void set_strip(SoftArgs &a, const char *env, bool forward)
{
    int strip = forward ? 8 : (a.h < 32 ? a.h : 32);
    const char *e = getenv(env);
    if (e && atoi(e) > 0) strip = atoi(e) > 32 ? 32 : atoi(e);
    if (strip < 8) strip = 8;
    if (strip > a.H) strip = a.H;
    a.strip = strip;
    a.nsy = (a.H + strip - 1) / strip;
}

// Tiling shared by the three phases: a single-wave tile when the row and
// the window fit one, else four-wave tiles: one column tile when W fits,
// else balanced tiles with a halo wide enough for either window orientation.
void plan_soft(SoftArgs &a)
{
    a.o = (a.h + 1) / 2;
    a.u = a.h / 2;
    a.l = (a.w + 1) / 2;
    a.r = a.w / 2;
    const int lmax = (a.l > a.r + 1) ? a.l : a.r + 1;   // forward l or adjoint r+1
    const int rmax = (a.r > a.l - 1) ? a.r : a.l - 1;   // forward r or adjoint l-1
    const int halo = ((lmax - 1) + 3) & ~3;
    constexpr int SN1 = SoftTile<WAVE_THREADS>::SNH, SN4 = SoftTile<WIDE_THREADS>::SNH;
    if (a.W <= SN1 && lmax <= SoftTile<WAVE_THREADS>::LPAD - 2 && rmax <= SoftTile<WAVE_THREADS>::RPAD) {
        a.nt = WAVE_THREADS;
        a.tile_w = a.W;
        a.ntx = 1;
        a.halo_l = 0;
    } else if (a.W <= SN4) {
        a.nt = WIDE_THREADS;
        a.tile_w = a.W;
        a.ntx = 1;
        a.halo_l = 0;
    } else {
        a.nt = WIDE_THREADS;
        a.halo_l = halo;
        const int tile4 = (SN4 - halo - rmax) & ~3;
        a.ntx = (a.W + tile4 - 1) / tile4;
        a.tile_w = ((a.W + a.ntx - 1) / a.ntx + 3) & ~3;
        a.ntx = (a.W + a.tile_w - 1) / a.tile_w;
    }
    // strips depend on the image geometry only, so an image gives the same
    // bits in any batch; the priming of a strip reads h rows beyond it
    set_strip(a, "BZ_SOFT_STRIP_BWD", false);
    a.vec = (a.ld % 4 == 0) && (a.W % 4 == 0);
}

size_t soft_fields_bytes(int B, int H, int W) { return (size_t)B * H * W * sizeof(float); }

template <int PH>
void launch_phase(const SoftArgs &a, int blocks, hipStream_t st)
{
    if (a.nt == WAVE_THREADS) {
        if (a.vec) hipLaunchKernelGGL((k_soft<PH, true, WAVE_THREADS>), dim3(blocks), dim3(WAVE_THREADS), 0, st, a);
        else hipLaunchKernelGGL((k_soft<PH, false, WAVE_THREADS>), dim3(blocks), dim3(WAVE_THREADS), 0, st, a);
    } else {
        if (a.vec) hipLaunchKernelGGL((k_soft<PH, true, WIDE_THREADS>), dim3(blocks), dim3(WIDE_THREADS), 0, st, a);
        else hipLaunchKernelGGL((k_soft<PH, false, WIDE_THREADS>), dim3(blocks), dim3(WIDE_THREADS), 0, st, a);
    }
}

}  // namespace

size_t soft_workspace_bytes(int B, int H, int W)
{
    // one partial pair per workgroup: column tiles are the whole row or at
    // least 1024 - 2 * 128 columns wide (windows up to 257), and strips at
    // least 8 rows tall (or the whole image)
    const size_t tiles = (size_t)B * ((W + 767) / 768) * (size_t)((H + 7) / 8);
    const size_t parts = tiles * 2 * sizeof(double);
    return 3 * ((soft_fields_bytes(B, H, W) + 255) & ~(size_t)255) + ((parts + 255) & ~(size_t)255);
}

hipError_t launch_soft_fwd(const float *I, int B, int H, int W, int64_t ld, int h, int w,
                           const float *k, const float *R, float tau, float *y, hipStream_t st)
{
    SoftArgs a;
    memset(&a, 0, sizeof(a));
    a.I = I;
    a.y = y;
    a.k = k;
    a.R = R;
    a.B = B;
    a.H = H;
    a.W = W;
    a.ld = ld;
    a.h = h;
    a.w = w;
    a.tau = tau;
    plan_soft(a);
    set_strip(a, "BZ_SOFT_STRIP", true);
    a.eo = a.o;
    a.eu = a.u;
    a.el = a.l;
    a.er = a.r;
    launch_phase<FWD>(a, B * a.ntx * a.nsy, st);
    return hipGetLastError();
}

hipError_t launch_soft_sums(const float *I, int B, int H, int W, int64_t ld, int h, int w, double *S1,
                            double *S2, int64_t ldS, hipStream_t st)
{
    SoftArgs a;
    memset(&a, 0, sizeof(a));
    a.I = I;
    a.S1 = S1;
    a.S2 = S2;
    a.ldS = ldS;
    a.B = B;
    a.H = H;
    a.W = W;
    a.ld = ld;
    a.h = h;
    a.w = w;
    a.tau = 1.0f;
    plan_soft(a);
    set_strip(a, "BZ_SOFT_STRIP", true);
    a.eo = a.o;
    a.eu = a.u;
    a.el = a.l;
    a.er = a.r;
    launch_phase<SUMS>(a, B * a.ntx * a.nsy, st);
    return hipGetLastError();
}

hipError_t launch_soft_bwd(const float *I, const float *gy, int B, int H, int W, int64_t ld, int h,
                           int w, const float *k, const float *R, float tau, float *gI, float *gk,
                           float *gR, void *ws, hipStream_t st)
{
    SoftArgs a;
    memset(&a, 0, sizeof(a));
    a.I = I;
    a.gy = gy;
    a.gI = gI;
    a.k = k;
    a.R = R;
    a.B = B;
    a.H = H;
    a.W = W;
    a.ld = ld;
    a.h = h;
    a.w = w;
    a.tau = tau;
    plan_soft(a);
    const size_t fb = (soft_fields_bytes(B, H, W) + 255) & ~(size_t)255;
    char *base = (char *)ws;
    a.G1 = (float *)base;
    a.G2 = (float *)(base + fb);
    a.dd = (float *)(base + 2 * fb);
    a.part = (double *)(base + 3 * fb);
    const int per_img = a.ntx * a.nsy;
    const int blocks = B * per_img;
    a.eo = a.o;
    a.eu = a.u;
    a.el = a.l;
    a.er = a.r;
    launch_phase<BWD1>(a, blocks, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the reflected window: rows q-u .. q+o-1, columns q-r .. q+l-1
    a.eo = a.u + 1;
    a.eu = a.o - 1;
    a.el = a.r + 1;
    a.er = a.l - 1;
    // the dense fields have row stride W: 16-byte loads need W % 4 == 0
    a.vec = (W % 4 == 0);
    set_strip(a, "BZ_SOFT_STRIP_ADJ", false);
    launch_phase<ADJ>(a, B * a.ntx * a.nsy, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_reduce, dim3(1), dim3(REDUCE_THREADS), 0, st, (const double *)a.part, B, per_img,
                       gk, gR);
    return hipGetLastError();
}

}  // namespace bz
