// Haar-like features (the rectangle features of Viola and Jones) of one
// template at every anchor where it fits, from sliding rectangle sums rather
// than an integral image (Section 3.4 names these features among the uses of
// recursive window sums).  The template is a kv x kh grid of a x b cells with
// signs; F[i][j] = sum of sign(m, n) * (sum of I over the cell anchored at
// (i + m a, j + n b)).
//
// Two or three launches over a caller workspace V of Hv = H - a + 1 rows:
//   k_haar_v       V[i][x] = sum of I over rows i .. i+a-1 of column x, slid
//                  down a strip: add the entering row, subtract the leaving
//                  one (the column recursion of Section 3.1), stored in 16
//                  bits (255 * 257 < 2^16, Section 3.3's bound);
//   k_haar_row     per output row, the kv rows of V it needs become inclusive
//                  prefixes along x in LDS (wrap-around uint32), and a cell's
//                  sum is a difference of two prefix entries, P_r[c + b - 1] -
//                  P_r[c - 1] (P_r[-1] = 0); F sums kv * kh of them;
//   (rows of more than 48 KiB for the kv prefixes: k_haar_prefix writes the
//   row prefixes of V to a uint32 field P after V, then k_haar_combine reads
//   them.)
// Every cell sum is below 2^32 (255 * 257 * 257), so the wrap-around
// differences are exact, and |F| <= 2 * 255 * 257 * 257 < 2^31.
//
// The five templates have alternating signs down and across (the checker is
// the product of the two), which allows a fused form of one launch and no
// workspace, k_haar_fused, used for 4-byte aligned rows and templates up to
// 256 columns wide:
//   G[i][x] = sum over m < kv of (-1)^m (sum of I over rows i + m a ..
//             i + m a + a - 1 of column x),
//   F[i][j] = sum over n < kh of (-1)^n (sum of G[i] over columns j + n b ..
//             j + n b + b - 1).
// Down a strip G slides with kv + 1 row reads per step (Section 3.1's column
// recursion over the signed stack of cells):
//   G[i+1][x] - G[i][x] = sum over j = 0 .. kv of c_j I[i + j a][x],
//   c_0 = -1, c_j = 2 (-1)^(j-1) for 0 < j < kv, c_kv = (-1)^(kv-1),
// and along the row F is a signed sum of kh + 1 entries of the inclusive
// prefix P of G[i] (P[-1] = 0), with the same coefficients:
//   F[i][j] = sum over n = 0 .. kh of c_n P[j + n b - 1].
#include "device.hpp"
#include "haar.hpp"

#include <stdlib.h>

#include <algorithm>

namespace bz {
namespace {

constexpr int HAAR_THREADS = HAAR_BLOCK;
constexpr int HAAR_STRIP = HAAR_ROWS;
// largest kv * W that k_haar_row keeps in LDS: 48 KiB of prefixes, three
// 4096-wide rows (measured faster than the two-launch path for them once each
// row is loaded whole before its scan)
constexpr int HAAR_ROW_ELEMS = 12288;
constexpr size_t HAAR_ROW_LDS = HAAR_ROW_ELEMS * sizeof(uint32_t);
// output rows per group of k_haar_fused: the next group's row loads are in
// flight while a group is processed.  Measured on the 4096 x 3072 page
// (edge_h and checker at 12, line_v and line_h at 48): one row per group
// 14.8, 16.9, 23.6 and 19.3 us; two 14.7, 17.1, 24.0, 19.9; four 15.4, 18.3,
// 24.9, 20.3; eight slower still (line_v 31.2).
constexpr int HAAR_GROUP = 1;
// priming rows of k_haar_fused loaded together (cells of 16 rows or more;
// measured on line_v at a = 48: 25 us against 29.8 us four rows at a time)
constexpr int HAAR_PRIME = 16;

// Workgroup (bx, sy): columns bx*256 .. +255, rows of V y0 = sy*S .. y0+S-1.
__global__ __launch_bounds__(HAAR_THREADS) void k_haar_v(const uint8_t *__restrict__ I, int64_t ld, int W, int a,
                                                         int Hv, int S, int nbx, uint16_t *__restrict__ V,
                                                         int64_t ldV)
{
    const int bx = blockIdx.x % nbx, sy = blockIdx.x / nbx;
    const int x = bx * HAAR_THREADS + threadIdx.x;
    const int y0 = sy * S;
    if (x >= W) return;
    const int y1 = min(y0 + S, Hv);
    const uint8_t *col = I + x;
    uint32_t c = 0;
#pragma unroll 8
    for (int r = 0; r < a; ++r) c += col[(int64_t)(y0 + r) * ld];  // y0 + a - 1 <= Hv - 1 + a - 1 = H - 1
    V[(int64_t)y0 * ldV + x] = (uint16_t)c;
#pragma unroll 8
    for (int y = y0 + 1; y < y1; ++y) {
        c += (uint32_t)col[(int64_t)(y + a - 1) * ld] - (uint32_t)col[(int64_t)(y - 1) * ld];
        V[(int64_t)y * ldV + x] = (uint16_t)c;
    }
}

// Inclusive prefix of src[0 .. W) into dst, by the whole
// workgroup, in chunks of 4 * 256 elements: a per-thread prefix of four, a
// wavefront scan of the thread totals, the wavefront totals through LDS, and
// the running total of the earlier chunks.
__device__ __forceinline__ void row_prefix(const uint16_t *src, uint32_t *dst, int W, uint32_t *wsum)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < W; base += 4 * HAAR_THREADS) {
        const int j = base + 4 * threadIdx.x;
        uint32_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = j + q < W ? (uint32_t)src[j + q] : 0u;
        v[1] += v[0];
        v[2] += v[1];
        v[3] += v[2];
        uint32_t s = v[3];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)s, d, 64);
            if (lane >= d) s += t;
        }
        if (lane == 63) wsum[wave] = s;
        __syncthreads();
        uint32_t before = carry, total = 0;
#pragma unroll
        for (int k = 0; k < HAAR_THREADS / 64; ++k) {
            if (k < wave) before += wsum[k];
            total += wsum[k];
        }
        __syncthreads();  // wsum is rewritten by the next chunk
        const uint32_t excl = before + s - v[3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (j + q < W) dst[j + q] = v[q] + excl;
        carry += total;
    }
}

// One output position j: the kv x kh cells from the prefixes P_m (row m of
// the template at P + m * step).  neg: bit m * kh + n set where cell (m, n)
// is negative.
__device__ __forceinline__ int32_t haar_at(const uint32_t *P, int64_t step, int j, int b, int kv, int kh,
                                           uint32_t neg)
{
    uint32_t f = 0;
    for (int m = 0; m < kv; ++m) {
        const uint32_t *row = P + m * step;
        uint32_t prev = j > 0 ? row[j - 1] : 0u;
        for (int n = 0; n < kh; ++n) {
            const uint32_t cur = row[j + (n + 1) * b - 1];  // <= Wf - 1 + kh b - 1 = W - 1
            const uint32_t cell = cur - prev;
            f += ((neg >> (m * kh + n)) & 1u) ? 0u - cell : cell;
            prev = cur;
        }
    }
    return (int32_t)f;
}

// Workgroup i: output row i.  Rows i, i + a, ... of V (one per row of the
// template) are read whole into registers first (KV * W <= 12288, so at most
// NCH chunks of 1024 per row, four elements per thread, one 8-byte load
// each), then turned into prefixes in LDS chunk by chunk, and the row's
// features are combined from LDS.  Reading V up to its padded row stride
// stays inside the workspace; elements past W are taken as 0.
template <int KV>
__global__ __launch_bounds__(HAAR_THREADS) void k_haar_row(const uint16_t *__restrict__ V, int64_t ldV, int W,
                                                           int a, int b, int kh, uint32_t neg, int Wf,
                                                           int32_t *__restrict__ F, int64_t ldF)
{
    constexpr int CH = 4 * HAAR_THREADS;
    constexpr int NCH = (HAAR_ROW_ELEMS / KV + CH - 1) / CH;
    extern __shared__ uint32_t P[];  // [KV][W]
    __shared__ uint32_t wsum[HAAR_THREADS / 64];
    const int i = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t v[KV][NCH][4];
#pragma unroll
    for (int m = 0; m < KV; ++m) {
        const uint16_t *row = V + (int64_t)(i + m * a) * ldV;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j = c * CH + 4 * threadIdx.x;
            ushort4 e = make_ushort4(0, 0, 0, 0);
            if (j < ldV) e = *(const ushort4 *)(row + j);  // ldV is a multiple of 64
            v[m][c][0] = j < W ? e.x : 0u;
            v[m][c][1] = j + 1 < W ? e.y : 0u;
            v[m][c][2] = j + 2 < W ? e.z : 0u;
            v[m][c][3] = j + 3 < W ? e.w : 0u;
        }
    }
#pragma unroll
    for (int m = 0; m < KV; ++m) {
        uint32_t carry = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (c * CH >= W) break;  // uniform
            const int j = c * CH + 4 * threadIdx.x;
            uint32_t *x = v[m][c];
            x[1] += x[0];
            x[2] += x[1];
            x[3] += x[2];
            uint32_t s = x[3];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t tt = (uint32_t)__shfl_up((int)s, d, 64);
                if (lane >= d) s += tt;
            }
            if (lane == 63) wsum[wave] = s;
            __syncthreads();
            uint32_t before = carry, total = 0;
#pragma unroll
            for (int k = 0; k < HAAR_THREADS / 64; ++k) {
                if (k < wave) before += wsum[k];
                total += wsum[k];
            }
            __syncthreads();
            const uint32_t excl = before + s - x[3];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j + q < W) P[m * W + j + q] = x[q] + excl;
            carry += total;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < Wf; j += HAAR_THREADS) F[(int64_t)i * ldF + j] = haar_at(P, W, j, b, KV, kh, neg);
}

// Rows too wide for k_haar_row's LDS: row r of P (uint32, same stride as V)
// becomes the prefix of row r of V (workgroup r), then k_haar_combine reads P.
__global__ __launch_bounds__(HAAR_THREADS) void k_haar_prefix(const uint16_t *__restrict__ V, uint32_t *__restrict__ P,
                                                              int64_t ldV, int W)
{
    __shared__ uint32_t wsum[HAAR_THREADS / 64];
    row_prefix(V + (int64_t)blockIdx.x * ldV, P + (int64_t)blockIdx.x * ldV, W, wsum);
}

// Workgroup (cx, i): outputs F[i][cx*256 .. +255] from the prefixes in P.
__global__ __launch_bounds__(HAAR_THREADS) void k_haar_combine(const uint32_t *__restrict__ P, int64_t ldP, int a,
                                                               int b, int kv, int kh, uint32_t neg, int Wf, int ncx,
                                                               int32_t *__restrict__ F, int64_t ldF)
{
    const int cx = blockIdx.x % ncx, i = blockIdx.x / ncx;
    const int j = cx * HAAR_THREADS + threadIdx.x;
    if (j >= Wf) return;
    F[(int64_t)i * ldF + j] = haar_at(P + (int64_t)i * ldP, (int64_t)a * ldP, j, b, kv, kh, neg);
}

// Coefficient c_j of the slide and of the prefix combination for a stack of
// k alternating cells (see the head of this file).
__host__ __device__ constexpr int haar_coef(int j, int k)
{
    return j == 0 ? -1 : j == k ? ((k - 1) & 1 ? -1 : 1) : ((j - 1) & 1 ? -2 : 2);
}

// Wavefront (tx, sy), one per 64-thread workgroup in XCD order: the tile of
// TWC = 256 NDW columns of G from x0 = tx * step (step <= TWC - (kh b - 1),
// a multiple of 4) gives the outputs x0 .. x0 + step - 1 of output rows
// i0 = sy * S .. min(i0 + S, Hf) - 1.  Lane t holds G of columns 4t .. 4t+3
// (+ 256 d for its d-th dword).  Rows are read through a descriptor per row
// from column x0 with (W - x0) bytes rounded up to a dword: the aligned dword
// holding the row's last byte is readable memory, and columns past W only
// reach prefix entries that no kept output reads (output j reads G columns up
// to j + kh b - 1 <= W - 1).  Per output row: the lane's inclusive prefix
// over its four columns, a wavefront scan of the lane totals, the row's
// prefix to LDS (P[c] at entry 4 + c, entry 3 the zero P[-1], so that a lane
// writes its four entries as one aligned 16-byte store), then lane t forms
// the outputs t + 64 k from LDS and stores them (the descriptor over the
// output row drops columns past Wf, and an offset past it those past the
// tile's step).  The stores take the default cache policy: tile rows start
// at any 4-byte offset of a cache line, and neighbouring tiles complete each
// other's partial lines in L2 (non-temporal stores measured 1.2 to 1.5x
// slower for 12 x 12 cells on the 4096 x 3072 page).  Two LDS buffers
// alternate by row, so one barrier per row suffices, and rows go in groups of
// HAAR_GROUP: the slide's row loads of the next group are issued before a
// group's work, so that their latency is hidden behind it (processing two rows
// per barrier, with their scans interleaved, measured slower).
template <int KV, int KH, int NDW>
__global__ __launch_bounds__(64) void k_haar_fused(const uint8_t *__restrict__ I, int64_t ldI, int W, int a, int b,
                                                   int Hf, int Wf, int step, int ntx, int S, int nsy,
                                                   int32_t *__restrict__ F, int64_t ldF)
{
    constexpr int TWC = 256 * NDW;
    constexpr int NC = 4 * NDW;  // columns per lane
    __shared__ __align__(16) uint32_t Q[2][TWC + 4];
    const int lane = threadIdx.x;
    const int L = xcd_remap(blockIdx.x, ntx * nsy);
    const int tx = L / nsy, sy = L - tx * nsy;
    const int x0 = tx * step;
    const int i0 = sy * S, i1 = min(i0 + S, Hf);
    const uint32_t nrec = (uint32_t)((W - x0 + 3) & ~3);
    const uint8_t *I0 = I + x0;
    auto row_rsrc = [&](int row) { return rsrc(I0 + (int64_t)row * ldI, nrec); };
    auto load = [&](const __amdgpu_buffer_rsrc_t &d, int q) {
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(d, 4 * lane + 256 * q, 0, 0);
    };

    // G of row i0: the signed sum of the kv a rows below it.  Each cell's a
    // rows are summed bytewise into 16-bit fields (even and odd bytes of a
    // dword apart; a <= 257 rows of at most 255 stay below 2^16), then
    // added to G with the cell's sign.
    uint32_t g[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) g[c] = 0u;
#pragma unroll
    for (int m = 0; m < KV; ++m) {
        const int r0 = i0 + m * a;
        uint32_t ev[NDW], od[NDW];
#pragma unroll
        for (int q = 0; q < NDW; ++q) ev[q] = od[q] = 0u;
        // the rows in chunks of HAAR_PRIME (all loads of a chunk in flight
        // together), then the rest four at a time
        int r = 0;
        for (; r + HAAR_PRIME <= a; r += HAAR_PRIME) {
            uint32_t v[HAAR_PRIME][NDW];
#pragma unroll
            for (int k = 0; k < HAAR_PRIME; ++k) {
                const __amdgpu_buffer_rsrc_t d = row_rsrc(r0 + r + k);
#pragma unroll
                for (int q = 0; q < NDW; ++q) v[k][q] = load(d, q);
            }
#pragma unroll
            for (int k = 0; k < HAAR_PRIME; ++k)
#pragma unroll
                for (int q = 0; q < NDW; ++q) {
                    ev[q] += v[k][q] & 0x00ff00ffu;
                    od[q] += __builtin_amdgcn_perm(0u, v[k][q], 0x0c030c01u);  // bytes 1, 3 into 0, 2
                }
        }
#pragma unroll 4
        for (; r < a; ++r) {
            const __amdgpu_buffer_rsrc_t d = row_rsrc(r0 + r);
#pragma unroll
            for (int q = 0; q < NDW; ++q) {
                const uint32_t v = load(d, q);
                ev[q] += v & 0x00ff00ffu;
                od[q] += __builtin_amdgcn_perm(0u, v, 0x0c030c01u);  // bytes 1, 3 into 0, 2
            }
        }
#pragma unroll
        for (int q = 0; q < NDW; ++q) {
            const uint32_t cs[4] = {ev[q] & 0xffffu, od[q] & 0xffffu, ev[q] >> 16, od[q] >> 16};
#pragma unroll
            for (int c = 0; c < 4; ++c) g[4 * q + c] = (m & 1) ? g[4 * q + c] - cs[c] : g[4 * q + c] + cs[c];
        }
    }

    const __amdgpu_buffer_rsrc_t none = rsrc(I, 0u);
    const uint32_t Fbytes = 4u * (uint32_t)(Wf - x0);
    // the slide's rows of a group of HAAR_GROUP output rows ig .. (row i's
    // rows for G[i+1]; none for the strip's last row or rows past it)
    uint32_t cur[HAAR_GROUP][KV + 1][NDW], nxt[HAAR_GROUP][KV + 1][NDW];
    auto load_group = [&](int ig, uint32_t(&sl)[HAAR_GROUP][KV + 1][NDW]) {
#pragma unroll
        for (int r = 0; r < HAAR_GROUP; ++r) {
            const bool in = ig + r + 1 < i1;
#pragma unroll
            for (int j = 0; j <= KV; ++j) {
                const __amdgpu_buffer_rsrc_t d = in ? row_rsrc(ig + r + j * a) : none;
#pragma unroll
                for (int q = 0; q < NDW; ++q) sl[r][j][q] = load(d, q);
            }
        }
    };
    load_group(i0, cur);
    int buf = 0;
    for (int ig = i0; ig < i1; ig += HAAR_GROUP) {
        load_group(ig + HAAR_GROUP, nxt);  // in flight during this group
#pragma unroll
        for (int r = 0; r < HAAR_GROUP; ++r) {
            const int i = ig + r;
            if (i >= i1) break;
            // prefix of G[i] over the tile into Q[buf][4 ..] (Q[buf][3] = 0)
            uint32_t carry = 0u;
#pragma unroll
            for (int q = 0; q < NDW; ++q) {
                uint32_t p[4];
                p[0] = g[4 * q];
#pragma unroll
                for (int c = 1; c < 4; ++c) p[c] = p[c - 1] + g[4 * q + c];
                const uint32_t incl = wave_scan(p[3]);
                const uint32_t excl = carry + incl - p[3];
                *(uint4 *)&Q[buf][4 + 256 * q + 4 * lane] = make_uint4(excl + p[0], excl + p[1], excl + p[2],
                                                                        excl + p[3]);
                carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            }
            if (lane == 0) Q[buf][3] = 0u;
            __syncthreads();
            // outputs t + 64 k of row i
            const __amdgpu_buffer_rsrc_t fo = rsrc(F + (int64_t)i * ldF + x0, Fbytes);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int col = lane + 64 * k;
                uint32_t f = 0u;
#pragma unroll
                for (int n = 0; n <= KH; ++n) f += (uint32_t)haar_coef(n, KH) * Q[buf][3 + min(col + n * b, TWC)];
                const uint32_t off = col < step ? 4u * (uint32_t)col : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b32(f, fo, (int)off, 0, 0);
            }
            buf ^= 1;
            // G[i+1]
#pragma unroll
            for (int j = 0; j <= KV; ++j) {
                const int cj = haar_coef(j, KV);
#pragma unroll
                for (int q = 0; q < NDW; ++q)
#pragma unroll
                    for (int c = 0; c < 4; ++c) g[4 * q + c] += (uint32_t)cj * ((cur[r][j][q] >> (8 * c)) & 0xffu);
            }
        }
#pragma unroll
        for (int r = 0; r < HAAR_GROUP; ++r)
#pragma unroll
            for (int j = 0; j <= KV; ++j)
#pragma unroll
                for (int q = 0; q < NDW; ++q) cur[r][j][q] = nxt[r][j][q];
    }
}

}  // namespace

int64_t haar_ld(int W) { return ((int64_t)W + 63) / 64 * 64; }

bool haar_fused(int W, int kv) { return (size_t)kv * (size_t)W * sizeof(uint32_t) <= HAAR_ROW_LDS; }

// V (uint16) first; for the two-launch path P (uint32) after it, 256-byte aligned.
static size_t haar_v_bytes(int H, int W, int a)
{
    return ((size_t)(H - a + 1) * (size_t)haar_ld(W) * sizeof(uint16_t) + 255) / 256 * 256;
}

size_t haar_workspace_bytes(int H, int W, int a, int kv)
{
    const size_t v = haar_v_bytes(H, W, a);
    return haar_fused(W, kv) ? v : v + (size_t)(H - a + 1) * (size_t)haar_ld(W) * sizeof(uint32_t);
}

// Negative cells of the alternating kv x kh template: (m + n) odd.
static uint32_t alternating(int kv, int kh)
{
    uint32_t neg = 0;
    for (int m = 0; m < kv; ++m)
        for (int n = 0; n < kh; ++n)
            if ((m + n) & 1) neg |= 1u << (m * kh + n);
    return neg;
}

template <int KV, int KH>
static void launch_fused(int ndw, dim3 grid, hipStream_t stream, const uint8_t *I, int64_t ldI, int W, int a, int b,
                         int Hf, int Wf, int step, int ntx, int S, int nsy, int32_t *F, int64_t ldF)
{
    if (ndw == 1)
        hipLaunchKernelGGL((k_haar_fused<KV, KH, 1>), grid, dim3(64), 0, stream, I, ldI, W, a, b, Hf, Wf, step, ntx,
                           S, nsy, F, ldF);
    else
        hipLaunchKernelGGL((k_haar_fused<KV, KH, 2>), grid, dim3(64), 0, stream, I, ldI, W, a, b, Hf, Wf, step, ntx,
                           S, nsy, F, ldF);
}

bool haar_fused_plan(const uint8_t *I, int64_t ldI, int H, int W, int a, int b, int kv, int kh, uint32_t neg,
                     HaarPlan &p)
{
    const char *e = getenv("BZ_HAAR_FUSED");
    if (e && atoi(e) == 0) return false;
    if (((uintptr_t)I & 3u) != 0 || (ldI & 3) != 0 || neg != alternating(kv, kh)) return false;
    if (!((kv == 1 && kh == 2) || (kv == 2 && kh == 1) || (kv == 1 && kh == 3) || (kv == 3 && kh == 1) ||
          (kv == 2 && kh == 2)))
        return false;
    const int halo = kh * b - 1;
    if (halo > 255) return false;
    p.Hf = H - kv * a + 1;
    p.Wf = W - kh * b + 1;
    p.ndw = halo <= 31 ? 1 : 2;
    e = getenv("BZ_HAAR_NDW");
    if (e && (atoi(e) == 1 || atoi(e) == 2) && 256 * atoi(e) - halo >= 4) p.ndw = atoi(e);
    p.step = (256 * p.ndw - halo) & ~3;
    p.ntx = (p.Wf + p.step - 1) / p.step;
    // strips: about an eighth of the kv a priming rows (8 to 64), halved
    // while the grid has fewer than 2048 wavefronts (down to 4 rows);
    // BZ_HAAR_STRIP overrides
    int S = std::min(64, std::max(8, (kv * a + 7) / 8));
    while (S > 4 && (int64_t)p.ntx * ((p.Hf + S - 1) / S) < 2048) S /= 2;
    e = getenv("BZ_HAAR_STRIP");
    if (e && atoi(e) > 0) S = atoi(e);
    p.S = std::min(S, p.Hf);
    p.nsy = (p.Hf + p.S - 1) / p.S;
    return (int64_t)p.ntx * p.nsy < ((int64_t)1 << 31) / 64;
}

hipError_t launch_haar(const uint8_t *I, int64_t ldI, int H, int W, int a, int b, int kv, int kh, uint32_t neg,
                       void *ws, int32_t *F, int64_t ldF, hipStream_t stream)
{
    HaarPlan fp;
    if (haar_fused_plan(I, ldI, H, W, a, b, kv, kh, neg, fp)) {
        const dim3 grid(fp.ntx * fp.nsy);
#define BZ_HAAR_FUSED(KV, KH)                                                                                   \
    launch_fused<KV, KH>(fp.ndw, grid, stream, I, ldI, W, a, b, fp.Hf, fp.Wf, fp.step, fp.ntx, fp.S, fp.nsy, F, \
                         ldF)
        if (kv == 1 && kh == 2) BZ_HAAR_FUSED(1, 2);
        else if (kv == 2 && kh == 1) BZ_HAAR_FUSED(2, 1);
        else if (kv == 1 && kh == 3) BZ_HAAR_FUSED(1, 3);
        else if (kv == 3 && kh == 1) BZ_HAAR_FUSED(3, 1);
        else BZ_HAAR_FUSED(2, 2);
#undef BZ_HAAR_FUSED
        return hipGetLastError();
    }
    const int Hv = H - a + 1, Hf = H - kv * a + 1, Wf = W - kh * b + 1;
    const int64_t ldV = haar_ld(W);
    uint16_t *V = (uint16_t *)ws;
    const int nbx = (W + HAAR_THREADS - 1) / HAAR_THREADS;
    const int nsy = (Hv + HAAR_STRIP - 1) / HAAR_STRIP;
    hipLaunchKernelGGL(k_haar_v, dim3(nbx * nsy), dim3(HAAR_THREADS), 0, stream, I, ldI, W, a, Hv, HAAR_STRIP, nbx,
                       V, ldV);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (haar_fused(W, kv)) {
        const size_t lds = (size_t)kv * (size_t)W * sizeof(uint32_t);
        if (kv == 1)
            hipLaunchKernelGGL(k_haar_row<1>, dim3(Hf), dim3(HAAR_THREADS), lds, stream, V, ldV, W, a, b, kh, neg,
                               Wf, F, ldF);
        else if (kv == 2)
            hipLaunchKernelGGL(k_haar_row<2>, dim3(Hf), dim3(HAAR_THREADS), lds, stream, V, ldV, W, a, b, kh, neg,
                               Wf, F, ldF);
        else
            hipLaunchKernelGGL(k_haar_row<3>, dim3(Hf), dim3(HAAR_THREADS), lds, stream, V, ldV, W, a, b, kh, neg,
                               Wf, F, ldF);
        return hipGetLastError();
    }
    uint32_t *P = (uint32_t *)((uint8_t *)ws + haar_v_bytes(H, W, a));
    hipLaunchKernelGGL(k_haar_prefix, dim3(Hv), dim3(HAAR_THREADS), 0, stream, V, P, ldV, W);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int ncx = (Wf + HAAR_THREADS - 1) / HAAR_THREADS;
    hipLaunchKernelGGL(k_haar_combine, dim3(ncx * Hf), dim3(HAAR_THREADS), 0, stream, P, ldV, a, b, kv, kh, neg, Wf,
                       ncx, F, ldF);
    return hipGetLastError();
}

}  // namespace bz
