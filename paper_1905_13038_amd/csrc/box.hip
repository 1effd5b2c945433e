// Sliding-window sums, moments and Sauvola/Niblack thresholds on gfx950.
//
// One workgroup owns a tile of output columns [x0, x1) and a strip of output
// rows [y0, y1).  Each lane owns four adjacent columns of the tile's halo'd
// column range and keeps their vertical window sums C (sum of I) and D (sum of
// I^2) in registers, updated row by row with the entering and leaving rows --
// the column recurrence of Section 3.1 / Algorithm 1.  The horizontal window
// sums are differences of a row prefix sum (S = P[j+r] - P[j-l]) built with a
// DPP wavefront scan plus a cross-wave combine through LDS; unsigned 32-bit
// wrap-around keeps the differences exact.  Rows are handled in groups of R so
// that one pair of workgroup barriers serves R rows.
//
// The threshold epilogue forms n*S2 - S1^2 exactly (binary64 FMA on exact
// integers), derives float32 m and s, and decides I < t in float32 with an
// error guard; pixels inside the guard are re-decided with the binary64
// reference sequence.
//
// Two entry kernels share the tile body: k_box (one tile per workgroup, tiles
// mapped XCD-contiguously) and k_box_batched (a persistent grid that claims
// tiles of many images from an atomic counter, largest tiles first).
#include "device.hpp"
#include "internal.hpp"

#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include <vector>

namespace bz {
namespace {

#ifndef BZ_ROWS_PER_GROUP
#define BZ_ROWS_PER_GROUP 2
#endif
constexpr int ROWS_PER_GROUP = BZ_ROWS_PER_GROUP;

// Layout of one LDS prefix row for NT threads.  Prefix index i (i = 0 is the
// empty prefix, i = 1 .. 4 NT the tile's halo'd columns) lives at word
// PREFIX_LPAD + i.  The PREFIX_LPAD words below index 0 hold zeros and the
// PREFIX_RPAD words above index 4 NT repeat the last prefix, so a window that
// reaches past either end of the tile reads the right value without an index
// clamp (out-of-image columns contribute zero; the epilogue's columns run up
// to halo + 4 NT - 1, so the right pad covers halo + r <= 256 words).
// PREFIX_LPAD + 1 is a multiple of 4, so each lane's indices 4t+1 .. 4t+4
// form one aligned 16-byte group.
constexpr int PREFIX_LPAD = 131;
constexpr int PREFIX_RPAD = 256;
__host__ __device__ constexpr int prefix_row_words(int NT)
{
    return PREFIX_LPAD + 1 + COLS_PER_LANE * NT + PREFIX_RPAD + 4;
}
// LDS of a tile, for the R rows of a group: the prefix rows (S1 and S2 per
// row), the gray levels of the rows (one dword per lane), and the wave totals.
// Gray rows: two sets (alternating by group) of R rows of NT words plus 4
// words that absorb the writes of halo columns.
__host__ __device__ constexpr int gray_row_words(int NT) { return NT + 4; }
__host__ __device__ constexpr int box_buffer_words(int NT)
{
    return 2 * ROWS_PER_GROUP * prefix_row_words(NT) + 2 * ROWS_PER_GROUP * gray_row_words(NT) +
           2 * ROWS_PER_GROUP * MAX_WAVES;
}

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xffu; }

// Cache policy of the output stores: non-temporal.  Outputs are written once
// and not read back by the kernel; streaming them keeps the L2 for the input
// rows the strips share and raised the store rate of this access pattern by
// about 40% in measurements on MI355X.
constexpr int STORE_NT = 2;

// Reads the four pixels of a lane (columns cb .. cb+3, cb a multiple of 4) of
// one row through a descriptor d over whole rows from a first row r0, the row
// chosen by the scalar offset so = (row - r0) * ld.  Pixels outside the image
// read as zero (Section 3.2's convention): a lane's offset is its column,
// replaced by 2^31 where no column of the lane lies inside [0, W), and rows
// outside the image are read through a descriptor of no bytes.  The hardware
// range check compares the lane offset plus the scalar offset with the
// descriptor size: valid lanes stay below it and offsets of 2^31 exceed every
// size used here (spans are kept below 2^31 bytes).
//
// Aligned form (4-byte aligned rows, W a multiple of 4): one dword load.
// Otherwise the descriptor starts at the 4-byte boundary at or below the
// first row (delta bytes earlier); a row's bytes then start at a uniform
// misalignment mis, and a lane loads the two aligned dwords that hold its
// four bytes and extracts them with a byte funnel shift; bytes of columns
// at or past W are masked off.  The range check rejects a dword that does
// not fit in the descriptor, so the descriptor ends with the aligned word
// that holds the strip's last byte: reads past that byte stay within its
// aligned word (never in another page) and the following dword is rejected.
constexpr uint32_t OFF_OUT = 0x80000000u;

template <bool AL>
struct LaneRow {
    uint32_t off;   // lane's byte offset in a row (column cb), or 2^31
    uint32_t keep;  // bytes of the lane's columns inside [0, W)
    uint32_t delta; // misalignment of the descriptor base (unaligned form)

    __device__ __forceinline__ LaneRow(int cb, int W, uint32_t delta_)
        : off((cb >= 0 && cb < W) ? (uint32_t)cb : OFF_OUT),
          keep((cb + 4 <= W) ? 0xffffffffu : (cb < W ? (1u << (8 * (W - cb))) - 1u : 0u)),
          delta(delta_)
    {
    }

    __device__ __forceinline__ uint32_t load(__amdgpu_buffer_rsrc_t d, uint32_t so) const
    {
        if (AL) return __builtin_amdgcn_raw_buffer_load_b32(d, (int)off, (int)so, 0);
        const uint32_t sb = delta + so;    // the row's first byte in d
        const uint32_t mis = sb & 3u;
        const uint32_t sa = sb - mis;      // its aligned word
        const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b32(d, (int)off, (int)sa, 0);
        const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b32(d, (int)(off + 4u), (int)sa, 0);
        return __builtin_amdgcn_alignbyte(hi, lo, mis) & keep;
    }
};

__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Marks v as used here, so the wait for the load that produced it is placed
// at this point (and nowhere later).
__device__ __forceinline__ void settle(uint32_t v) { asm volatile("" : : "v"(v)); }

// Add four rows (one dword per row, four columns each) to the column sums:
// transpose the 4x4 bytes so each dword holds one column, then one SAD (sum)
// and one DOT4 (sum of squares) per column.
__device__ __forceinline__ void add4rows(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                         uint32_t C[4], uint32_t D[4])
{
    const uint32_t a0 = __builtin_amdgcn_perm(r1, r0, 0x05010400u);
    const uint32_t a1 = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
    const uint32_t b0 = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
    const uint32_t b1 = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
    const uint32_t t0 = __builtin_amdgcn_perm(b0, a0, 0x05040100u);
    const uint32_t t1 = __builtin_amdgcn_perm(b0, a0, 0x07060302u);
    const uint32_t t2 = __builtin_amdgcn_perm(b1, a1, 0x05040100u);
    const uint32_t t3 = __builtin_amdgcn_perm(b1, a1, 0x07060302u);
    C[0] = __builtin_amdgcn_sad_u8(t0, 0u, C[0]);
    C[1] = __builtin_amdgcn_sad_u8(t1, 0u, C[1]);
    C[2] = __builtin_amdgcn_sad_u8(t2, 0u, C[2]);
    C[3] = __builtin_amdgcn_sad_u8(t3, 0u, C[3]);
    D[0] = __builtin_amdgcn_udot4(t0, t0, D[0], false);
    D[1] = __builtin_amdgcn_udot4(t1, t1, D[1], false);
    D[2] = __builtin_amdgcn_udot4(t2, t2, D[2], false);
    D[3] = __builtin_amdgcn_udot4(t3, t3, D[3], false);
}

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

// The other rules of Table 1, decided in binary64 for every pixel: m, s as
// in below_reference, then the rule's threshold, each operation rounded once
// (RULE: the rule, a template argument so that each kernel carries only its
// own sequence; p: the rule's parameters; L, M, S: the image's minimum, mean
// and standard deviation).  Wolf t = m - k (m - L)(1 - s/R); Feng t = a1 m
// + k1 (s/R)^(1+g) (m - L) + k2 (s/R)^g L; Rais t = m + 0.3 (m s - M S) /
// max{m s, M S} s (the fraction is 0 where both products are 0); Khurshid
// (NICK) t = m + k sqrt(s^2 + m^2 (n-1)/n) with the clipped count n for h w;
// Phansalkar t = m (1 + p e^(-q m) + k (s/R - 1)).
template <int RULE>
__device__ __attribute__((noinline)) bool table1_below(uint32_t I, uint32_t S1, uint32_t S2,
                                                       int64_t n, double p0, double p1,
                                                       double p2, double p3, double p4, double L,
                                                       double M, double S)
{
#pragma clang fp contract(off)
    const int64_t Vn = n * (int64_t)S2 - (int64_t)S1 * (int64_t)S1;
    const double nd = (double)n;
    const double m = (double)S1 / nd;
    const double v = (double)Vn / (nd * nd);
    const double s = __builtin_sqrt(v);
    double t;
    if (RULE == T1_WOLF) {
        double a = s / p1;
        a = 1.0 - a;
        double b = m - L;
        b = p0 * b;
        b = b * a;
        t = m - b;
    } else if (RULE == T1_FENG) {
        const double x = s / p4;
        const double x1 = pow(x, 1.0 + p3);
        const double x0 = pow(x, p3);
        const double a = p0 * m;
        double b = p1 * x1;
        b = b * (m - L);
        double c = p2 * x0;
        c = c * L;
        t = a + b;
        t = t + c;
    } else if (RULE == T1_RAIS) {
        const double a = m * s, b = M * S;
        const double e = a > b ? a : b;
        double f = 0.0;
        if (e > 0.0) f = (a - b) / e;
        double g = 0.3 * f;
        g = g * s;
        t = m + g;
    } else if (RULE == T1_NICK) {
        const double a = s * s;
        double b = m * m;
        const double c = (nd - 1.0) / nd;
        b = b * c;
        const double r = __builtin_sqrt(a + b);
        const double q = p0 * r;
        t = m + q;
    } else {  // T1_PHANSALKAR
        double e = p1 * m;
        e = exp(-e);
        const double a = p0 * e;
        double b = s / p3;
        b = b - 1.0;
        b = p2 * b;
        double c = 1.0 + a;
        c = c + b;
        t = m * c;
    }
    return (double)I < t;
}

// Kernels of the Table 1 rules are specialised to the rule: their MODE
// template argument is MODE_T1_BASE + the rule (the job's mode stays
// MODE_TABLE1), so each keeps only its rule's constants and arithmetic.
constexpr int MODE_T1_BASE = 16;

// Float32 form of a Table 1 rule and its guard.  With m and s within 2 and 3
// units of 2^-24 (u) of their values, first-order error bounds of the float32
// threshold against the binary64 one, relative to the magnitude mag of its
// terms, are about: Wolf 12u, NICK 7.5u (the native square root, within
// 1 ulp), Rais 26u (the quotient as a product with the native reciprocal,
// within 1 ulp), Phansalkar (14 + 5|q m|)u of |m| C with
// C = 1 + |p| e^(-qm) + |k|(1 + s/R) (e^(-qm) as the native 2^(-qm log2 e):
// within 1.42u, plus |q m| u from the rounded argument), and Feng
// (11 + |g|(6.1 + 2.1 |log2 x|))u with x = s/R.  For Feng, x^g is
// 2^(g log2 x) from the native log2 and exp2, which, checked over every
// float32 input in the ranges used, are within 2u max(1, |log2 x|)
// (absolute) and 1.42u (relative); x is within 4u, so x^g is within
// (1.5 + |g|(6.1 + 2.1 |log2 x|))u.  The guard G mag takes 2^-18 (64u) for
// Wolf, 2^-18 for NICK, 2^-18 for Phansalkar (mag scaled by 1 + |q m|),
// 2^-17 for Rais and 2^-19 for Feng (mag scaled by 2 + |g|(1 + |log2 x|)):
// a factor of 4.5 or more over the bounds.  Where |I - t32| > G mag the float32 and
// binary64 decisions agree; other pixels, and any non-finite value, go to
// table1_below.
struct T1Fast {
    int rule;
    float p0, p1, p2, p3;
    float rR;   // 1/R
    float L;    // global minimum
    float MS;   // M S
    float G;    // guard factor
    float pow0; // Feng: 0^g (0 for g > 0, 1 for g = 0, infinity for g < 0)
};

__device__ __forceinline__ T1Fast t1_fast_params(int rule, const double *tp, double L, double M, double S)
{
    T1Fast f;
    f.rule = rule;
    f.p0 = (float)tp[0];
    f.p1 = (float)tp[1];
    f.p2 = (float)tp[2];
    f.p3 = (float)tp[3];
    const double R = rule == T1_WOLF ? tp[1] : rule == T1_FENG ? tp[4] : rule == T1_PHANSALKAR ? tp[3] : 1.0;
    f.rR = (float)(1.0 / R);
    f.L = (float)L;
    f.MS = (float)M * (float)S;
    f.pow0 = tp[3] > 0.0 ? 0.0f : tp[3] == 0.0 ? 1.0f : __builtin_inff();
    f.G = rule == T1_WOLF || rule == T1_NICK || rule == T1_PHANSALKAR ? 0x1p-18f
          : rule == T1_FENG                                           ? 0x1p-19f
                                                                      : 0x1p-17f;  // T1_RAIS
    return f;
}

// d = I - t32 and the guard g = G mag: the float32 decision is the sign of d,
// valid where |d| > g.
template <int RULE>
__device__ __forceinline__ void table1_fast(const T1Fast &f, float m, float s, float rn, float I,
                                            float &d, float &g)
{
    float t, mag;
    if constexpr (RULE == T1_WOLF) {
        const float a = 1.0f - s * f.rR;
        const float b = f.p0 * (m - f.L);
        t = m - b * a;
        mag = fabsf(m) + fabsf(f.p0) * (fabsf(m) + fabsf(f.L)) * (1.0f + s * f.rR);
    } else if constexpr (RULE == T1_NICK) {
        const float r = __builtin_amdgcn_sqrtf(fmaf(s, s, m * m * (1.0f - rn)));
        t = fmaf(f.p0, r, m);
        mag = fabsf(m) + fabsf(f.p0) * r;
    } else if constexpr (RULE == T1_RAIS) {
        const float a = m * s;
        const float e = fmaxf(a, f.MS);
        const float q = e > 0.0f ? (a - f.MS) * __builtin_amdgcn_rcpf(e) : 0.0f;
        t = fmaf(0.3f * s, q, m);
        mag = fabsf(m) + 0.3f * s;
    } else if constexpr (RULE == T1_PHANSALKAR) {
        const float qm = f.p1 * m;
        const float ex = __builtin_amdgcn_exp2f(-qm * 1.44269504088896340736f);  // e^(-qm)
        const float c = 1.0f + f.p0 * ex + f.p2 * (s * f.rR - 1.0f);
        t = m * c;
        mag = fabsf(m) * (1.0f + fabsf(f.p0) * ex + fabsf(f.p2) * (1.0f + s * f.rR)) * (1.0f + fabsf(qm));
    } else {  // T1_FENG
        // x^g = 2^(g log2 x) with the native log2 and exp2; x^(1+g) = x x^g.
        // A flat window (x = 0) takes pow's value (0, 1, or infinity for
        // g < 0, which sends it to the reference); an exponent beyond 120 in
        // magnitude (a result outside the normal range, or log2 of a
        // subnormal) gives NaN, which does too.
        const float x = s * f.rR;
        const float lg = __builtin_amdgcn_logf(x);
        const float e = f.p3 * lg;
        const float p = __builtin_amdgcn_exp2f(e);
        const float x0 = x == 0.0f ? f.pow0 : (fabsf(e) <= 120.0f ? p : __builtin_nanf(""));
        const float x1 = x * x0;
        const float al = x == 0.0f ? 0.0f : fabsf(lg);
        t = f.p0 * m + f.p1 * x1 * (m - f.L) + f.p2 * x0 * f.L;
        mag = (fabsf(f.p0 * m) + fabsf(f.p1) * x1 * (fabsf(m) + fabsf(f.L)) + fabsf(f.p2) * x0 * fabsf(f.L)) *
              (2.0f + fabsf(f.p3) * (1.0f + al));
    }
    d = I - t;
    g = f.G * mag;
}

// Guard of the float32 decision.  mag bounds the magnitudes of the terms of
// t: m (|c1| s + |c0|) for Sauvola, m + |k| s for Niblack.  With u = 2^-24:
// 1/n is correctly rounded, so m = S1 (1/n) is within 2u of S1/n; n*S2 -
// S1^2 is exact and its float32 conversion within u; the square root is
// within 1 ulp (2u) and the product with 1/n adds 2u, so s is within 4.5u;
// c1 = k/R and c0 = 1 - k are within u each; q = fma(c1, s, c0) and
// d = fma(-m, q, I) round once each.  Summed, t32 is within 8.5u mag of the
// exact t (Sauvola; 5.5u mag for Niblack), and the binary64 sequence within
// 2^-50 mag of it.  Where |d| >= 2^-19 mag = 32u mag (a margin of 3.7), the
// float32 sign is the binary64 one; other pixels are re-decided with the
// binary64 sequence.  A window of zeros (mag = 0, as for columns past the
// image) is decided exactly.
constexpr float GUARD = 1.9073486328125e-06f;  // 2^-19

// Input dwords of one row group: entering rows (y + u), leaving rows (y - o)
// and centre rows (y) of the group's R rows, for this lane's four columns.
template <int R>
struct GroupRows {
    uint32_t a[R], b[R], c[R];
};

// One tile: output columns [x0, x1) of the strip of rows [y0, y1).
//
// Rows are processed in groups of R.  Each group goes through three phases
// separated by workgroup barriers:
//   A  column recurrence for its rows, per-lane prefixes and wavefront scans
//      (wave totals to LDS),
//   B  cross-wave combine: the full row prefixes to LDS,
//   E  epilogue: window sums from the prefixes, moments, threshold, stores.
// Each phase is written without branches over its rows, so that the compiler
// can schedule the rows of a group together (the loads of one row under the
// arithmetic of the other).
//
// MS: also write the window mean and standard deviation (always true for
// MODE_MEANSTD, unused for MODE_SUMS).
template <int MODE, bool AL, bool MS>
__device__ __forceinline__ void box_tile(const BoxJob &a, int tx, int sy, uint32_t *smem)
{
    constexpr int R = ROWS_PER_GROUP;
    constexpr bool T1 = MODE >= MODE_T1_BASE;  // a Table 1 rule, MODE - MODE_T1_BASE
    constexpr bool need_i = (MODE == MODE_SAUVOLA || MODE == MODE_NIBLACK || T1);
    const int NT = blockDim.x;
    const int PS = prefix_row_words(NT);
    const int BW = box_buffer_words(NT);
    const int GS = gray_row_words(NT);
    // prefix row of statistic st (0: S1, 1: S2) for group row r; gray row r
    // of set g; wave totals of statistic st for row r
    auto prefix_row = [&](int b, int r, int st) { return smem + b * BW + (2 * r + st) * PS; };
    auto gray_row = [&](int g, int r) { return smem + 2 * R * PS + (g * R + r) * GS; };
    auto tot_row = [&](int b, int r, int st) {
        return smem + b * BW + 2 * R * PS + 2 * R * GS + (2 * r + st) * MAX_WAVES;
    };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = NT >> 6;

    const int x0 = tx * a.tile_w;
    const int x1 = min(x0 + a.tile_w, a.W);
    const int y0 = sy * a.strip;
    const int y1 = min(y0 + a.strip, a.H);
    const int xh = (tx == 0) ? 0 : x0 - a.halo_l;
    const int H = a.H, W = a.W, o = a.o, u = a.u;
    // vertical pass: lane owns the four columns cb .. cb+3
    const int cb = xh + COLS_PER_LANE * tid;
    // The strip reads input rows rlo .. rhi only (its priming rows, then the
    // entering, leaving and centre rows); one descriptor covers them (from
    // the 4-byte boundary at or below the first row in the unaligned form).
    // The planner keeps this span, and the output spans below, under 2^31
    // bytes.
    const int rlo = max(y0 - o, 0), rhi = min(y1 - 1 + u, H - 1);
    const uint32_t ld32 = (uint32_t)a.ldI;
    const uint8_t *rrow = a.I + (int64_t)rlo * a.ldI;
    const uint32_t delta = AL ? 0u : (uint32_t)((uintptr_t)rrow & 3u);
    const uint8_t *rbase = rrow - delta;
    // (unaligned form: rounded up to the end of the aligned word holding the
    // last byte, since a dword that crosses the descriptor end reads zero)
    const uint32_t rspan = AL ? (uint32_t)(rhi - rlo) * ld32 + (uint32_t)W
                              : (delta + (uint32_t)(rhi - rlo) * ld32 + (uint32_t)W + 3u) & ~3u;
    const LaneRow<AL> ld(cb, W, delta);
    // row `row` if rlo <= row <= rhi (in), else zeros
    auto row_load = [&](int row, bool in) -> uint32_t {
        return ld.load(rsrc(rbase, in ? rspan : 0u), in ? (uint32_t)(row - rlo) * ld32 : 0u);
    };

    // zero the left pads (and index 0) of every prefix row once
    for (int i = tid; i < 2 * R * (PREFIX_LPAD + 1); i += NT) {
        const int row = i / (PREFIX_LPAD + 1);  // 0 .. 2R-1
        smem[row * PS + (i - row * (PREFIX_LPAD + 1))] = 0u;
    }

    // Epilogue: wave w covers output columns x0 + 256 w .. x0 + 256 w + 255,
    // lane t taking columns t, t+64, t+128, t+192 of them, so that the prefix
    // reads of a wavefront hit consecutive LDS words (no bank conflicts) and
    // each store instruction writes 64 consecutive elements.  Lanes whose
    // columns lie past the tile compute as the others do; the range checks of
    // the output descriptors drop their stores.
    const int eo = 256 * wave + lane;  // column k is x0 + eo + 64 k
    const int ec0 = x0 + eo;
    const int ai0 = PREFIX_LPAD + ec0 + a.r - xh + 1;  // prefix word of j + r
    const int bi0 = PREFIX_LPAD + ec0 - a.l - xh + 1;  // prefix word of j - l
    const uint32_t ow = (uint32_t)(x1 - x0);  // output row width of the tile
    // Output descriptors cover the strip's rows of the tile (columns x0 ..
    // x1-1), the row chosen by scalar offset (the range check includes it);
    // a lane's element offsets are 2^31 for columns outside the tile, so
    // those stores fail the check.
    uint32_t o4[4], o1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = eo + 64 * k < (int)ow;
        o4[k] = in ? 4u * (uint32_t)(eo + 64 * k) : OFF_OUT;
        o1[k] = in ? (uint32_t)(eo + 64 * k) : OFF_OUT;
    }
    const uint32_t last = (uint32_t)(y1 - 1 - y0);  // strip rows - 1
    // descriptor of an output over the strip's rows; none for rows past it
    auto out_rsrc = [&](const void *p, int64_t ldo, int es, bool live) {
        return rsrc((const uint8_t *)p + ((int64_t)y0 * ldo + x0) * es,
                    live ? (uint32_t)es * (last * (uint32_t)ldo + ow) : 0u);
    };
    // The gray levels of a row, transposed for the epilogue: the dword of
    // epilogue lane t of wave w holds the levels of its four columns (byte
    // k: column x0 + 256 w + t + 64 k).  Vertical lane t writes its four
    // bytes (columns xh + 4t + q, q = 0..3, four consecutive epilogue lanes)
    // at gbyte + 4 q; halo columns left of x0 go to a spare word.
    int gbyte;
    {
        const int e = COLS_PER_LANE * tid - (x0 - xh);  // a multiple of 4
        gbyte = (e >= 0) ? 4 * (64 * (e >> 8) + (e & 63)) + ((e & 255) >> 6) : 4 * NT;
    }

    // Window sizes of the epilogue columns for rows whose window lies inside
    // the image vertically (nr = h), and their reciprocals.
    double ndh[4];
    float rnh[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = ec0 + 64 * k;
        const int nc = max(min(j + a.r, W - 1) - max(j - a.l, -1), 1);
        ndh[k] = (double)a.h * (double)nc;
        rnh[k] = 1.0f / (float)ndh[k];
    }
    // Guard of the float32 decision, near iff |d| < GUARD * mag'.  Sauvola:
    // s <= 127.5 for 8-bit data bounds mag by m (|c1| 127.5 + |c0|) = m MQ,
    // so near iff |d| + gA m < 0 with gA = -GUARD MQ.  Niblack: the exact
    // mag = m + |k| s.
    const float gA = (MODE == MODE_SAUVOLA)
                         ? -GUARD * __builtin_fmaf(__builtin_fabsf(a.c1), 127.5f, __builtin_fabsf(a.c0))
                         : -GUARD;
    // Table 1 rules: the image's global minimum, mean and standard deviation
    double gL = 0.0, gM = 0.0, gS = 0.0;
    if (T1 && a.gs != nullptr) {
        gL = (double)a.gs->min;
        gM = a.gs->mean;
        gS = a.gs->stdev;
    }
    const T1Fast t1f = t1_fast_params(a.rule, a.tp, gL, gM, gS);

    // ---- priming: column sums over rows y0-o .. y0+u-1 ----
    uint32_t C[4] = {0, 0, 0, 0}, D[4] = {0, 0, 0, 0};
    {
        const int p0 = max(y0 - o, 0);
        const int p1 = min(y0 + u - 1, H - 1);
        // batches of PB rows: all PB loads in flight, then PB/4 SAD/DOT4
        // groups (fewer rows per batch where each row takes four byte loads).
        // All strips prime at once when the kernel starts, so this phase is
        // bound by the L2 bandwidth; more loads in flight per wavefront were
        // measured to be slower.
        constexpr int PB = AL ? 32 : 16;
        const __amdgpu_buffer_rsrc_t rin = rsrc(rbase, rspan);
        int row = p0;  // p0 == rlo
        for (; row + PB - 1 <= p1; row += PB) {
            const uint32_t so = (uint32_t)(row - p0) * ld32;
            uint32_t v[PB];
#pragma unroll
            for (int q = 0; q < PB; ++q) v[q] = ld.load(rin, so + (uint32_t)q * ld32);
#pragma unroll
            for (int g = 0; g < PB / 4; ++g)
                add4rows(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3], C, D);
        }
        if (row <= p1) {  // fewer than PB rows left: rows past p1 read zero
            uint32_t v[PB];
#pragma unroll
            for (int q = 0; q < PB; ++q) v[q] = row_load(row + q, row + q <= p1);
#pragma unroll
            for (int g = 0; g < PB / 4; ++g)
                if (row + 4 * g <= p1) add4rows(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3], C, D);
        }
    }

    // ---- the row groups ----
    // The next group's rows are loaded during a group and waited for at its
    // end: one wait counter tracks loads and stores in issue order, so the
    // wait is placed after the group's stores rather than before them.
    GroupRows<R> X;
    auto load_group = [&](int yg, GroupRows<R> &g) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // rows past the strip load zeros: the recurrence leaves C, D as they are
            const int ra = yg + r + u, rb = yg + r - o;
            const bool on = yg + r < y1;
            g.a[r] = row_load(ra, on && ra <= rhi);
            g.b[r] = row_load(rb, on && rb >= rlo);
            if (need_i) g.c[r] = row_load(yg + r, yg + r <= rhi);
        }
    };
    auto settle_group = [&](GroupRows<R> &g) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            settle(g.a[r]);
            settle(g.b[r]);
            if (need_i) settle(g.c[r]);
        }
    };

    uint32_t pc[R][4], pd[R][4], sc[R], sd[R];
    // A: column recurrence, per-lane prefixes and wave scans of group rows
    // yg .. yg+R-1
    auto phase_A = [&](int gs, const GroupRows<R> &cur) {
        const int b = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // the centre row's gray levels, for the epilogue's column order
            // (read back by lanes of this same wavefront only)
            if (need_i) {
                uint8_t *gw = (uint8_t *)gray_row(gs, r) + gbyte;
#pragma unroll
                for (int q = 0; q < 4; ++q) gw[4 * q] = (uint8_t)byte_of(cur.c[r], q);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ak = (int)byte_of(cur.a[r], k), bk = (int)byte_of(cur.b[r], k);
                const int dk = ak - bk;
                C[k] += (uint32_t)dk;
                D[k] += (uint32_t)(dk * (ak + bk));
            }
            pc[r][0] = C[0];
            pc[r][1] = pc[r][0] + C[1];
            pc[r][2] = pc[r][1] + C[2];
            pc[r][3] = pc[r][2] + C[3];
            pd[r][0] = D[0];
            pd[r][1] = pd[r][0] + D[1];
            pd[r][2] = pd[r][1] + D[2];
            pd[r][3] = pd[r][2] + D[3];
            sc[r] = wave_scan(pc[r][3]);
            sd[r] = wave_scan(pd[r][3]);
            if (lane == 63) {
                tot_row(b, r, 0)[wave] = sc[r];
                tot_row(b, r, 1)[wave] = sd[r];
            }
        }
    };
    // B: offsets of the wave totals, full row prefixes into buffer b.  The
    // scan over the first 16 lanes gives wave w's offset at lane w-1 and the
    // tile totals (tc, td) at lane nwaves-1; lanes at or above nwaves never
    // feed those, so they read any total.  Branch-free, so that it can
    // interleave with the epilogue.
    uint32_t tc[R], td[R];
    auto phase_B = [&](int b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t wc = row_scan16(tot_row(b, r, 0)[lane & 15]);
            const uint32_t wd = row_scan16(tot_row(b, r, 1)[lane & 15]);
            const int wl = max(wave - 1, 0);
            uint32_t oc = (uint32_t)__builtin_amdgcn_readlane((int)wc, wl);
            uint32_t od = (uint32_t)__builtin_amdgcn_readlane((int)wd, wl);
            oc = (wave > 0) ? oc : 0u;
            od = (wave > 0) ? od : 0u;
            tc[r] = (uint32_t)__builtin_amdgcn_readlane((int)wc, nwaves - 1);
            td[r] = (uint32_t)__builtin_amdgcn_readlane((int)wd, nwaves - 1);
            const uint32_t ec_ = sc[r] - pc[r][3] + oc, ed_ = sd[r] - pd[r][3] + od;
            uint32_t *prc = prefix_row(b, r, 0) + PREFIX_LPAD + 1;  // index 1
            uint32_t *prd = prefix_row(b, r, 1) + PREFIX_LPAD + 1;
            *(uint4 *)(prc + COLS_PER_LANE * tid) =
                make_uint4(pc[r][0] + ec_, pc[r][1] + ec_, pc[r][2] + ec_, pc[r][3] + ec_);
            *(uint4 *)(prd + COLS_PER_LANE * tid) =
                make_uint4(pd[r][0] + ed_, pd[r][1] + ed_, pd[r][2] + ed_, pd[r][3] + ed_);
        }
    };
    // right pads of buffer b: repeat the tile totals (last wave)
    auto pads_B = [&](int b) {
        if (wave == nwaves - 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint32_t *prc = prefix_row(b, r, 0) + PREFIX_LPAD + 1 + COLS_PER_LANE * NT;
                uint32_t *prd = prefix_row(b, r, 1) + PREFIX_LPAD + 1 + COLS_PER_LANE * NT;
#pragma unroll
                for (int q = 0; q < PREFIX_RPAD / 64; ++q) {
                    prc[64 * q + lane] = tc[r];
                    prd[64 * q + lane] = td[r];
                }
            }
        }
    };

    // Statistics of epilogue column k of group row r from buffer b: window
    // sums, then n = nr * nc and the moments; n*S2 - S1^2 is formed exactly
    // in binary64 (every term is an integer below 2^53).
    struct ColStats {
        uint32_t S1, S2;
        double n;
        float m, s, rn;
    };
    auto col_stats = [&](int b, int r, int k, int y, bool interior) -> ColStats {
        ColStats c;
        const uint32_t *pa = prefix_row(b, r, 0) + ai0 + 64 * k;
        const uint32_t *pb = prefix_row(b, r, 0) + bi0 + 64 * k;
        c.S1 = pa[0] - pb[0];
        c.S2 = pa[PS] - pb[PS];
        float rn;
        if (interior) {
            c.n = (k == 0) ? ndh[0] : (k == 1) ? ndh[1] : (k == 2) ? ndh[2] : ndh[3];
            rn = (k == 0) ? rnh[0] : (k == 1) ? rnh[1] : (k == 2) ? rnh[2] : rnh[3];
        } else {
            const int nr = max(min(y + u, H - 1) - max(y - o, -1), 1);
            const int j = ec0 + 64 * k;
            const int nc = max(min(j + a.r, W - 1) - max(j - a.l, -1), 1);
            c.n = (double)nr * (double)nc;
            rn = 1.0f / (float)c.n;
        }
        c.rn = rn;
        c.m = (float)c.S1 * rn;
        const double s1d = (double)c.S1;
        const double vn = __builtin_fma(c.n, (double)c.S2, -(s1d * s1d));
        c.s = __builtin_amdgcn_sqrtf((float)vn) * rn;
        return c;
    };
    // float32 decision: d = I - t with the exact sign of I - t (the mask bit
    // is its sign bit; d is +0 when I equals t) and the guard metric nm
    // (the pixel is near the threshold when nm < 0)
    auto decide = [&](const ColStats &c, float gv, float &d, float &nm) {
        if (MODE == MODE_SAUVOLA) {
            const float q = __builtin_fmaf(a.c1, c.s, a.c0);  // 1 + k (s/R - 1)
            d = __builtin_fmaf(-c.m, q, gv);
            nm = __builtin_fmaf(gA, c.m, __builtin_fabsf(d));
        } else {
            d = gv - __builtin_fmaf(a.c1, c.s, c.m);
            nm = __builtin_fmaf(gA, __builtin_fmaf(a.kabs, c.s, c.m), __builtin_fabsf(d));
        }
    };

    // E: epilogue of the group whose rows start at yg, from buffer b and
    // gray set gs
    auto phase_E = [&](int yg, int b, int gs, auto interior_tag) {
        constexpr bool interior = decltype(interior_tag)::value;
        uint32_t bits[R][4];
        float nmv[R][4];  // guard metrics (near when < 0)
        float nmin = 1.0f;
        uint32_t t1near = 0;  // Table 1: pixels inside the float32 guard
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yg + r;
            const bool live = y < y1;  // rows past the strip store nothing
            const uint32_t dy = (uint32_t)(y - y0);
            ColStats c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = col_stats(b, r, k, y, interior);
            if (MODE == MODE_SUMS) {
                const uint32_t so = 4u * dy * (uint32_t)a.ldS;
                const __amdgpu_buffer_rsrc_t d1 = out_rsrc(a.S1, a.ldS, 4, live);
                const __amdgpu_buffer_rsrc_t d2 = out_rsrc(a.S2, a.ldS, 4, live);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    __builtin_amdgcn_raw_buffer_store_b32(c[k].S1, d1, (int)o4[k], (int)so, STORE_NT);
                    __builtin_amdgcn_raw_buffer_store_b32(c[k].S2, d2, (int)o4[k], (int)so, STORE_NT);
                }
                continue;
            }
            if (MS) {
                const uint32_t so = 4u * dy * (uint32_t)a.ldMS;
                const __amdgpu_buffer_rsrc_t dm = out_rsrc(a.mean, a.ldMS, 4, live);
                const __amdgpu_buffer_rsrc_t ds = out_rsrc(a.stdv, a.ldMS, 4, live);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(c[k].m), dm, (int)o4[k], (int)so, STORE_NT);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(c[k].s), ds, (int)o4[k], (int)so, STORE_NT);
                }
            }
            if (MODE == MODE_MEANSTD) continue;
            const uint32_t gw = gray_row(gs, r)[tid];  // byte k: column ec0 + 64 k (this lane's word)
            if constexpr (T1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    float d, g;
                    table1_fast<T1 ? MODE - MODE_T1_BASE : T1_FENG>(t1f, c[k].m, c[k].s, c[k].rn,
                                                                     (float)byte_of(gw, k), d, g);
                    bits[r][k] = d < 0.0f ? 1u : 0u;
                    if (a.force_ref || !(fabsf(d) > g)) t1near |= 1u << (4 * r + k);
                }
                continue;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float d;
                decide(c[k], (float)byte_of(gw, k), d, nmv[r][k]);
                bits[r][k] = __float_as_uint(d) >> 31;
                nmin = __builtin_fminf(nmin, nmv[r][k]);
            }
        }
        if (!need_i) return;
        // pixels within the guard: re-decided with the binary64 sequence
        // (rare; statistics recomputed from LDS, one call site)
        if constexpr (T1) {
            // pixels inside the guard: the binary64 sequence (statistics
            // recomputed from LDS)
            while (t1near != 0) {
                const int i = __builtin_ctz(t1near);
                t1near &= t1near - 1;
                const int r = i >> 2, k = i & 3;
                const ColStats c = col_stats(b, r, k, yg + r, false);
                const uint32_t gv = ((const uint8_t *)gray_row(gs, r))[4 * tid + k];
                const uint32_t bit =
                    table1_below<T1 ? MODE - MODE_T1_BASE : T1_FENG>(gv, c.S1, c.S2, (int64_t)c.n, a.tp[0], a.tp[1],
                                                                     a.tp[2], a.tp[3], a.tp[4], gL, gM, gS)
                        ? 1u
                        : 0u;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) bits[rr][kk] = (i == 4 * rr + kk) ? bit : bits[rr][kk];
            }
        } else if (a.force_ref || nmin < 0.0f) {
            uint32_t near = 0;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (a.force_ref || nmv[r][k] < 0.0f) near |= 1u << (4 * r + k);
            while (near != 0) {
                const int i = __builtin_ctz(near);
                near &= near - 1;
                const int r = i >> 2, k = i & 3;
                const ColStats c = col_stats(b, r, k, yg + r, false);
                const uint32_t gv = ((const uint8_t *)gray_row(gs, r))[4 * tid + k];
                const uint32_t bit =
                    below_reference(gv, c.S1, c.S2, (int64_t)c.n, MODE, a.k64, a.R64) ? 1u : 0u;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) bits[rr][kk] = (i == 4 * rr + kk) ? bit : bits[rr][kk];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yg + r;
            // (after the divergent branch above: scalar values restated as
            // uniform so the stores take them from scalar registers)
            const __amdgpu_buffer_rsrc_t dk = out_rsrc(a.mask, a.ldM, 1, y < y1);
            const uint32_t so = uniform((uint32_t)(y - y0) * (uint32_t)a.ldM);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)bits[r][k], dk, (int)o1[k], (int)so, STORE_NT);
        }
    };

    // ---- the groups of the strip ----
    load_group(y0, X);
    settle_group(X);
    int gs = 0;  // gray set of the group (alternates: a wave may still read
                 // the previous group's set while another writes the next)
    for (int yg = y0; yg < y1; yg += R, gs ^= 1) {
        const GroupRows<R> cur = X;
        if (yg + R < y1) load_group(yg + R, X);  // prefetch the next group
        phase_A(gs, cur);
        __syncthreads();
        phase_B(0);
        pads_B(0);
        __syncthreads();
        settle_group(X);  // the next group's rows, before this group's stores
        // rows whose windows lie vertically inside the image use the cached
        // window sizes
        const bool interior = (yg - o >= -1) && (yg + R - 1 + u <= H - 1);
        // the epilogue's waves take issue priority over those still in the
        // column pass, so its stores leave sooner (measured on the 4096 x 3072
        // page: mask only 27.8 -> 26.8 us at w = 75 and 31.8 -> 30.6 us at 151;
        // with mean and std within noise)
        __builtin_amdgcn_s_setprio(3);
        if (interior) phase_E(yg, 0, gs, std::true_type{});
        else phase_E(yg, 0, gs, std::false_type{});
        __builtin_amdgcn_s_setprio(0);
    }
}

// BIG: the instantiation launched with more than 64 KB of LDS.  It is a
// separate kernel so that raising its dynamic-LDS limit leaves the LDS
// reservation, and with it the occupancy, of smaller launches untouched.
template <int MODE, bool AL, bool MS, bool BIG>
__global__ __launch_bounds__(MAX_THREADS) void k_box(BoxJob a)
{
    extern __shared__ uint32_t smem[];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = L / a.nsy;
    box_tile<MODE, AL, MS>(a, tx, L - tx * a.nsy, smem);
}

template <int MODE, bool MS>
__device__ __forceinline__ void batched_tile(const BoxJob &a, int tx, int sy, uint32_t *smem)
{
    if (a.aligned) box_tile<MODE, true, MS>(a, tx, sy, smem);
    else box_tile<MODE, false, MS>(a, tx, sy, smem);
}

// A word of the batch workspace, the same for every lane.  The workspace is
// read with vector loads (the kernel also writes it: the tile counter), so
// without this the compiler keeps job fields in vector registers, and every
// buffer access through a resource built from them becomes a loop over the
// distinct values of the wavefront.
__device__ __forceinline__ int uniform_word(const int *p) { return (int)uniform((uint32_t)*p); }

// The job record at p, every field taken from the first lane.
__device__ __forceinline__ BoxJob uniform_job(const BoxJob *p)
{
    static_assert(sizeof(BoxJob) % 4 == 0, "a job record is a whole number of words");
    constexpr int N = (int)(sizeof(BoxJob) / 4);
    const int *src = (const int *)p;
    int w[N];
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = uniform_word(src + i);
    BoxJob j;
    __builtin_memcpy(&j, w, sizeof(BoxJob));
    return j;
}

// Persistent grid over the tiles of a ragged batch.  Tiles are numbered in the
// order of the job array (largest per-tile work first); prefix[i] is the first
// tile of job i and prefix[count] the total.  The last workgroup to finish
// resets the counters, so the next launch (or graph replay) starts from zero
// without a memset.  `tile(a, tx, sy)` processes one tile of job a.
template <typename TileFn>
__device__ __forceinline__ void batched_loop(BatchHeader *hdr, TileFn tile)
{
    __shared__ int s_tile;
    const int count = uniform_word(&hdr->count);
    const BoxJob *jobs = (const BoxJob *)(hdr + 1);
    const int *prefix = (const int *)(jobs + count);
    const int total = uniform_word(prefix + count);
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(&hdr->next_tile, 1u);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t >= total) break;
        int lo = 0, hi = count;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (uniform_word(prefix + mid) <= t) lo = mid;
            else hi = mid;
        }
        const BoxJob a = uniform_job(jobs + lo);
        const int local = t - uniform_word(prefix + lo);
        const int tx = local / a.nsy;
        tile(a, tx, local - tx * a.nsy);
        __syncthreads();  // the tile's LDS is free before the next claim
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(&hdr->done, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(&hdr->next_tile, 0u);
            atomicExch(&hdr->done, 0u);
        }
    }
}

// Any mix of Sauvola/Niblack, alignment and mean/std outputs.
__global__ __launch_bounds__(BATCH_THREADS) void k_box_batched(BatchHeader *hdr)
{
    extern __shared__ uint32_t smem[];
    batched_loop(hdr, [&](const BoxJob &a, int tx, int sy) {
        const bool ms = a.mean != nullptr;
        if (a.mode == MODE_SAUVOLA) {
            if (ms) batched_tile<MODE_SAUVOLA, true>(a, tx, sy, smem);
            else batched_tile<MODE_SAUVOLA, false>(a, tx, sy, smem);
        } else {
            if (ms) batched_tile<MODE_NIBLACK, true>(a, tx, sy, smem);
            else batched_tile<MODE_NIBLACK, false>(a, tx, sy, smem);
        }
    });
}

// Batches whose jobs all share one variant (mode, alignment, mean/std
// outputs): one tile body, and registers for four waves per SIMD.
template <int MODE, bool AL, bool MS>
__global__ __launch_bounds__(BATCH_THREADS, 4) void k_box_batched_v(BatchHeader *hdr)
{
    extern __shared__ uint32_t smem[];
    batched_loop(hdr, [&](const BoxJob &a, int tx, int sy) { box_tile<MODE, AL, MS>(a, tx, sy, smem); });
}

// Kernel of batch variant v (-1: mixed batch).
const void *batch_kernel(int v)
{
    switch (v) {
    case 0: return (const void *)k_box_batched_v<MODE_SAUVOLA, false, false>;
    case 1: return (const void *)k_box_batched_v<MODE_SAUVOLA, false, true>;
    case 2: return (const void *)k_box_batched_v<MODE_SAUVOLA, true, false>;
    case 3: return (const void *)k_box_batched_v<MODE_SAUVOLA, true, true>;
    case 4: return (const void *)k_box_batched_v<MODE_NIBLACK, false, false>;
    case 5: return (const void *)k_box_batched_v<MODE_NIBLACK, false, true>;
    case 6: return (const void *)k_box_batched_v<MODE_NIBLACK, true, false>;
    case 7: return (const void *)k_box_batched_v<MODE_NIBLACK, true, true>;
    default: return (const void *)k_box_batched;
    }
}

template <int MODE, bool AL, bool MS>
hipError_t launch_variant(const BoxJob &a, hipStream_t stream)
{
    const int NT = a.threads;
    const size_t lds = (size_t)box_lds_words(NT) * sizeof(uint32_t);
    const int blocks = a.ntx * a.nsy;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_box<MODE, AL, MS, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_box<MODE, AL, MS, true>), dim3(blocks), dim3(NT), lds, stream, a);
    } else {
        hipLaunchKernelGGL((k_box<MODE, AL, MS, false>), dim3(blocks), dim3(NT), lds, stream, a);
    }
    return hipGetLastError();
}

template <int MODE, bool MS>
hipError_t launch_mode(const BoxJob &a, hipStream_t stream)
{
    return a.aligned ? launch_variant<MODE, true, MS>(a, stream) : launch_variant<MODE, false, MS>(a, stream);
}

}  // namespace

int box_lds_words(int NT)
{
    return box_buffer_words(NT);
}

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
    a.threads = NT;
    if (a.W <= COLS_PER_LANE * NT) {
        a.tile_w = a.W;
        a.ntx = 1;
        a.halo_l = 0;
    } else {
        a.halo_l = ((a.l - 1) + 3) & ~3;
        a.tile_w = (COLS_PER_LANE * NT - a.halo_l - a.r) & ~3;
        if (a.tile_w < 4) {  // window wider than the block: use the widest block
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
        // one resident round of workgroups: at most `target` tiles (a tile
        // more would run in a second round and double the time)
        const long target = 256L * per_cu;
        strip = (int)(((long)a.H * a.ntx + target - 1) / target);
        if (strip < 4) strip = 4;
        while ((long)a.ntx * ((a.H + strip - 1) / strip) > target) ++strip;
    }
    // keep the spans of a tile's descriptors (input rows rlo .. rhi, output
    // rows of the strip) below 2^31 bytes; the entry points guarantee that
    // one row strip fits
    const int64_t LIM = ((int64_t)1 << 31) - 1;
    int64_t cap = (LIM - a.W) / a.ldI - a.h + 1;
    if (a.S1 != nullptr) cap = std::min(cap, (LIM / 4 - a.W) / a.ldS + 1);
    if (a.mean != nullptr) cap = std::min(cap, (LIM / 4 - a.W) / a.ldMS + 1);
    if (a.mask != nullptr) cap = std::min(cap, (LIM - a.W) / a.ldM + 1);
    if (strip > cap) strip = (int)std::max<int64_t>(cap, 1);
    a.strip = strip;
    a.nsy = (a.H + strip - 1) / strip;
}

hipError_t launch_box(const BoxJob &a, hipStream_t stream)
{
    const bool ms = a.mean != nullptr;
    switch (a.mode) {
    case MODE_SUMS: return launch_mode<MODE_SUMS, false>(a, stream);
    case MODE_MEANSTD: return launch_mode<MODE_MEANSTD, true>(a, stream);
    case MODE_SAUVOLA: return ms ? launch_mode<MODE_SAUVOLA, true>(a, stream) : launch_mode<MODE_SAUVOLA, false>(a, stream);
    case MODE_NIBLACK: return ms ? launch_mode<MODE_NIBLACK, true>(a, stream) : launch_mode<MODE_NIBLACK, false>(a, stream);
    case MODE_TABLE1:
        switch (a.rule) {
#define BZ_T1_CASE(RULE)                                                                              \
    case RULE:                                                                                        \
        return ms ? launch_mode<MODE_T1_BASE + RULE, true>(a, stream)                                 \
                  : launch_mode<MODE_T1_BASE + RULE, false>(a, stream);
            BZ_T1_CASE(T1_WOLF)
            BZ_T1_CASE(T1_FENG)
            BZ_T1_CASE(T1_RAIS)
            BZ_T1_CASE(T1_NICK)
            BZ_T1_CASE(T1_PHANSALKAR)
#undef BZ_T1_CASE
        default: return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
}

size_t batch_workspace_bytes(int count)
{
    const size_t raw = sizeof(BatchHeader) + (size_t)count * sizeof(BoxJob) + (size_t)(count + 1) * sizeof(int);
    return (raw + 255) & ~(size_t)255;
}

int batch_variant(const BoxJob *jobs, int count)
{
    // the unaligned row loader is correct for aligned rows as well, so a
    // batch that mixes the two runs the unaligned variant
    int v = -2;
    bool all_aligned = true;
    for (int i = 0; i < count; ++i) {
        const BoxJob &j = jobs[i];
        const int vi = (j.mode == MODE_NIBLACK ? 4 : 0) + (j.mean != nullptr ? 1 : 0);
        all_aligned = all_aligned && j.aligned;
        if (v == -2) v = vi;
        else if (v != vi) return -1;
    }
    return v < 0 ? -1 : v + (all_aligned ? 2 : 0);
}

namespace {
std::mutex g_batch_mu;
// kernel variant of each planned workspace (host side)
std::unordered_map<const void *, int> g_batch_variant;
// persistent grid size per device and variant
std::unordered_map<int64_t, int> g_batch_grid;
}  // namespace

void register_batch_variant(const void *workspace, int variant)
{
    std::lock_guard<std::mutex> lock(g_batch_mu);
    g_batch_variant[workspace] = variant;
}

int batch_grid(int variant)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) device = 0;
    const int64_t key = (int64_t)device * 16 + (variant + 1);
    std::lock_guard<std::mutex> lock(g_batch_mu);
    auto it = g_batch_grid.find(key);
    if (it != g_batch_grid.end()) return it->second;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    const size_t lds = (size_t)box_lds_words(BATCH_THREADS) * sizeof(uint32_t);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(variant), BATCH_THREADS, lds) !=
            hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    g_batch_grid[key] = cus * per_cu;
    return cus * per_cu;
}

hipError_t launch_box_batched(void *workspace, hipStream_t stream)
{
    int variant = -1;
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        auto it = g_batch_variant.find(workspace);
        if (it != g_batch_variant.end()) variant = it->second;
    }
    const size_t lds = (size_t)box_lds_words(BATCH_THREADS) * sizeof(uint32_t);
    BatchHeader *hdr = (BatchHeader *)workspace;
    void *args[] = {&hdr};
    return hipLaunchKernel(batch_kernel(variant), dim3(batch_grid(variant)), dim3(BATCH_THREADS), args, lds,
                           stream);
}

}  // namespace bz
