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
#include "haar.hpp"

namespace bz {
namespace {

constexpr int HAAR_THREADS = HAAR_BLOCK;
constexpr int HAAR_STRIP = HAAR_ROWS;
// largest kv * W that k_haar_row keeps in LDS: 48 KiB of prefixes, three
// 4096-wide rows (measured faster than the two-launch path for them once each
// row is loaded whole before its scan)
constexpr int HAAR_ROW_ELEMS = 12288;
constexpr size_t HAAR_ROW_LDS = HAAR_ROW_ELEMS * sizeof(uint32_t);

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

hipError_t launch_haar(const uint8_t *I, int64_t ldI, int H, int W, int a, int b, int kv, int kh, uint32_t neg,
                       void *ws, int32_t *F, int64_t ldF, hipStream_t stream)
{
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
