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
// Three kernels: k_soft<FWD> (sums -> y), k_soft<BWD1> (sums -> G1, G2,
// delta/tau and per-workgroup partials of dL/dk, dL/dR), k_soft<ADJ> (adjoint
// sums of G1, G2 -> dL/dI), and k_soft_reduce (fixed-order reduction of the
// partials, so the k and R gradients are deterministic).  Nothing is saved by
// the forward: the backward recomputes m and s from I.
//
// Sums are binary64: vertical running sums per lane column (add the entering
// row, subtract the leaving row) and a row prefix per tile (DPP wave scan plus
// an LDS cross-wave combine), differenced at the window ends.
#include "../../include/binarize.h"
#include "internal.hpp"

#include <math.h>
#include <string.h>

namespace bz {
namespace {

enum Phase { FWD = 0, BWD1 = 1, ADJ = 2 };

constexpr int SOFT_THREADS = 256;
constexpr int SOFT_WAVES = SOFT_THREADS / 64;
constexpr int SR = 2;  // rows per barrier pair

struct SoftArgs {
    const float *I;     // B images, image b at I + b*H*ld
    const float *gy;    // upstream gradient (BWD1), same layout as I
    float *y;           // FWD output, layout of I
    float *G1, *G2, *dd;  // BWD1 outputs / ADJ inputs: B*H*W, row stride W
    float *gI;          // ADJ output, layout of I
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
};

__device__ __forceinline__ int xcd_remap_s(int b, int n)
{
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, i = b >> 3;
    return (x < rem) ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

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

__device__ __forceinline__ double wave_sum_f64(double v)
{
    // fixed-order reduction: the inclusive scan's last lane holds the total
    v = wave_scan_f64(v);
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// The four values X1 (and X2) of a lane's columns in one row.  FWD/BWD1 sum
// I and I^2; ADJ sums G1 and G2.  Out-of-image columns and rows are zero.
template <int PH>
__device__ __forceinline__ void row_vals(const SoftArgs &a, int b, int row, int cb, double x1[4],
                                         double x2[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + k;
        float v1 = 0.0f, v2 = 0.0f;
        if (c >= 0 && c < a.W) {
            if (PH == ADJ) {
                const int64_t off = ((int64_t)b * a.H + row) * a.W + c;
                v1 = a.G1[off];
                v2 = a.G2[off];
            } else {
                v1 = a.I[((int64_t)b * a.H + row) * a.ld + c];
            }
        }
        x1[k] = (double)v1;
        x2[k] = (PH == ADJ) ? (double)v2 : (double)v1 * (double)v1;  // exact square
    }
}

template <int PH>
__global__ __launch_bounds__(SOFT_THREADS) void k_soft(SoftArgs a)
{
    constexpr int NT = SOFT_THREADS;
    constexpr int NH = 4 * NT;
    constexpr int PS = NH + 4;
    __shared__ double P[SR][2][PS];
    __shared__ double Tot[SR][2][SOFT_WAVES];
    __shared__ double Red[2][SOFT_WAVES];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int L = xcd_remap_s(blockIdx.x, gridDim.x);
    const int per_img = a.ntx * a.nsy;
    const int b = L / per_img;
    const int rem = L - b * per_img;
    const int tx = rem / a.nsy, sy = rem - tx * a.nsy;
    const int x0 = tx * a.tile_w, x1 = min(x0 + a.tile_w, a.W);
    const int y0 = sy * a.strip, y1 = min(y0 + a.strip, a.H);
    const int xh = (tx == 0) ? 0 : x0 - a.halo_l;
    const int cb = xh + 4 * tid;
    const int H = a.H, W = a.W;

    if (tid < SR) {
        P[tid][0][0] = 0.0;
        P[tid][1][0] = 0.0;
    }
    int ai[4], bi[4];
    double ncd[4];
    bool valid[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = cb + k;
        valid[k] = (j >= x0) && (j < x1);
        const int ar = min(j + a.er, W - 1), bl = max(j - a.el, -1);
        ai[k] = valid[k] ? ar - xh + 1 : 0;
        bi[k] = valid[k] ? bl - xh + 1 : 0;
        // the forward count (the adjoint sums need none)
        ncd[k] = (double)(min(j + a.r, W - 1) - max(j - a.l, -1));
    }

    double kb = 0.0, R64 = 0.0;
    if (PH != ADJ) {
        kb = (double)a.k[b];
        R64 = (double)a.R[0];
    }
    const double tau = (double)a.tau;

    // priming: rows y0-eo .. y0+eu-1
    double C[4] = {0, 0, 0, 0}, D[4] = {0, 0, 0, 0};
    for (int row = max(y0 - a.eo, 0); row <= min(y0 + a.eu - 1, H - 1); ++row) {
        double x1v[4], x2v[4];
        row_vals<PH>(a, b, row, cb, x1v, x2v);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            C[k] += x1v[k];
            D[k] += x2v[k];
        }
    }

    double dk_acc = 0.0, dR_acc = 0.0;
    for (int yg = y0; yg < y1; yg += SR) {
        double pc[SR][4], pd[SR][4], sc[SR], sd[SR];
#pragma unroll
        for (int r = 0; r < SR; ++r) {
            const int y = yg + r;
            if (y < y1) {
                double e1[4], e2[4], l1[4], l2[4];
                const int ra = y + a.eu, rb = y - a.eo;
                if (ra < H) row_vals<PH>(a, b, ra, cb, e1, e2);
                else { for (int k = 0; k < 4; ++k) { e1[k] = 0.0; e2[k] = 0.0; } }
                if (rb >= 0) row_vals<PH>(a, b, rb, cb, l1, l2);
                else { for (int k = 0; k < 4; ++k) { l1[k] = 0.0; l2[k] = 0.0; } }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    C[k] = (C[k] + e1[k]) - l1[k];
                    D[k] = (D[k] + e2[k]) - l2[k];
                }
            }
            pc[r][0] = C[0]; pc[r][1] = pc[r][0] + C[1]; pc[r][2] = pc[r][1] + C[2]; pc[r][3] = pc[r][2] + C[3];
            pd[r][0] = D[0]; pd[r][1] = pd[r][0] + D[1]; pd[r][2] = pd[r][1] + D[2]; pd[r][3] = pd[r][2] + D[3];
            sc[r] = wave_scan_f64(pc[r][3]);
            sd[r] = wave_scan_f64(pd[r][3]);
            if (lane == 63) {
                Tot[r][0][wave] = sc[r];
                Tot[r][1][wave] = sd[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SR; ++r) {
            double oc = 0.0, od = 0.0;
            for (int w2 = 0; w2 < wave; ++w2) {  // fixed order
                oc += Tot[r][0][w2];
                od += Tot[r][1][w2];
            }
            const double ec = (sc[r] - pc[r][3]) + oc, ed = (sd[r] - pd[r][3]) + od;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                P[r][0][1 + 4 * tid + k] = pc[r][k] + ec;
                P[r][1][1 + 4 * tid + k] = pd[r][k] + ed;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SR; ++r) {
            const int y = yg + r;
            if (y >= y1) continue;
            const int nr = min(y + a.u, H - 1) - max(y - a.o, -1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!valid[k]) continue;
                const int j = cb + k;
                const double S1 = P[r][0][ai[k]] - P[r][0][bi[k]];
                const double S2 = P[r][1][ai[k]] - P[r][1][bi[k]];
                const int64_t pix = ((int64_t)b * H + y) * a.ld + j;
                if (PH == ADJ) {
                    const int64_t g = ((int64_t)b * H + y) * W + j;
                    a.gI[pix] = (float)((double)a.dd[g] + S1 + 2.0 * (double)a.I[pix] * S2);
                    continue;
                }
                const double n = (double)nr * ncd[k];
                const double m = S1 / n;
                double v = (n * S2 - S1 * S1) / (n * n);
                if (v < 0.0) v = 0.0;
                const double s = sqrt(v);
                const double q = s / R64 - 1.0;
                const double t = m * (1.0 + kb * q);
                const double Iv = (double)a.I[pix];
                const double z = (Iv - t) / tau;
                const double yv = 1.0 / (1.0 + exp(-z));
                if (PH == FWD) {
                    a.y[pix] = (float)yv;
                    continue;
                }
                const double delta = (double)a.gy[pix] * yv * (1.0 - yv);
                const double e = -delta / tau;
                dk_acc += e * m * q;
                dR_acc += e * (-kb * m * s / (R64 * R64));
                const double aa = e * (1.0 + kb * q);
                const double beta = e * kb * m / R64;
                double g1, g2;
                if (s > 0.0) {
                    g1 = aa / n - beta * m / (n * s);
                    g2 = beta / (2.0 * n * s);
                } else {
                    g1 = aa / n;
                    g2 = 0.0;
                }
                const int64_t g = ((int64_t)b * H + y) * W + j;
                a.G1[g] = (float)g1;
                a.G2[g] = (float)g2;
                a.dd[g] = (float)(delta / tau);
            }
        }
    }
    if (PH == BWD1) {
        const double wk = wave_sum_f64(dk_acc), wr = wave_sum_f64(dR_acc);
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

// gk[b] = sum of image b's partials, gR = sum of all, each in a fixed order.
__global__ __launch_bounds__(64) void k_soft_reduce(const double *part, int B, int per_img,
                                                    float *gk, float *gR)
{
    const int t = threadIdx.x;
    for (int b = t; b < B; b += 64) {
        double s = 0.0;
        for (int i = 0; i < per_img; ++i) s += part[2 * ((int64_t)b * per_img + i)];
        gk[b] = (float)s;
    }
    if (t == 0) {
        double s = 0.0;
        for (int64_t i = 0; i < (int64_t)B * per_img; ++i) s += part[2 * i + 1];
        gR[0] = (float)s;
    }
}

// Tiling shared by the three phases: one column tile when W fits a block,
// else tiles with a halo wide enough for either window orientation.
void plan_soft(SoftArgs &a)
{
    a.o = (a.h + 1) / 2;
    a.u = a.h / 2;
    a.l = (a.w + 1) / 2;
    a.r = a.w / 2;
    constexpr int NH = 4 * SOFT_THREADS;
    if (a.W <= NH) {
        a.tile_w = a.W;
        a.ntx = 1;
        a.halo_l = 0;
    } else {
        const int lmax = (a.l > a.r + 1) ? a.l : a.r + 1;   // forward l or adjoint r+1
        const int rmax = (a.r > a.l - 1) ? a.r : a.l - 1;   // forward r or adjoint l-1
        a.halo_l = ((lmax - 1) + 3) & ~3;
        a.tile_w = (NH - a.halo_l - rmax) & ~3;
        a.ntx = (a.W + a.tile_w - 1) / a.tile_w;
    }
    // about 4 workgroups per CU over the whole batch
    const long target = 1024;
    int strip = (int)(((long)a.B * a.H * a.ntx + target - 1) / target);
    if (strip < 2 * a.h) strip = 2 * a.h;
    if (strip > a.H) strip = a.H;
    a.strip = strip;
    a.nsy = (a.H + strip - 1) / strip;
}

size_t soft_fields_bytes(int B, int H, int W) { return (size_t)B * H * W * sizeof(float); }

}  // namespace

size_t soft_workspace_bytes(int B, int H, int W)
{
    // partial slots for any window: a column tile is at least 4*256 - 2*132
    // columns wide and a strip at least 2 rows tall
    const size_t tiles = (size_t)B * ((W + 759) / 760) * ((H + 1) / 2);
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
    a.eo = a.o;
    a.eu = a.u;
    a.el = a.l;
    a.er = a.r;
    const int blocks = B * a.ntx * a.nsy;
    hipLaunchKernelGGL(k_soft<FWD>, dim3(blocks), dim3(SOFT_THREADS), 0, st, a);
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
    hipLaunchKernelGGL(k_soft<BWD1>, dim3(blocks), dim3(SOFT_THREADS), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the reflected window: rows q-u .. q+o-1, columns q-r .. q+l-1
    a.eo = a.u + 1;
    a.eu = a.o - 1;
    a.el = a.r + 1;
    a.er = a.l - 1;
    hipLaunchKernelGGL(k_soft<ADJ>, dim3(blocks), dim3(SOFT_THREADS), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_reduce, dim3(1), dim3(64), 0, st, (const double *)a.part, B, per_img,
                       gk, gR);
    return hipGetLastError();
}

}  // namespace bz
