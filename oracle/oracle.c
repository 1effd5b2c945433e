/*
 * CPU oracle for local adaptive binarization statistics.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code with the HIP library.
 *
 * Everything here is written to be read against the paper (Chan, "Memory-
 * efficient and fast implementation of local adaptive binarization methods"):
 * plain loops, no blocking, no fusion.  Floating point is IEEE binary64 with
 * contraction disabled (built with -ffp-contract=off, no fast-math).
 *
 * Notation (Section 3.2, Algorithm 1):
 *   l = floor((w+1)/2), r = floor(w/2), o = floor((h+1)/2), u = floor(h/2);
 *   the window of pixel (i, j) is rows i-o < a <= i+u and columns
 *   j-l < b <= j+r (the bounds of the Introduction's mean formula), clipped to
 *   the image: elements outside the image count as zero (Section 3.2,
 *   assumptions) and the divisor is the in-bounds count n of Algorithm 1.
 *
 * Images are row-major uint8 with a row stride `ld` (elements).  Outputs are
 * dense H x W arrays (row stride W).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

/* Algorithm 1, first four assignments. */
static void extents(int h, int w, int *o, int *u, int *l, int *r)
{
    *l = (w + 1) / 2;
    *r = w / 2;
    *o = (h + 1) / 2;
    *u = h / 2;
}

/* Algorithm 1, the assignment to n: the number of window pixels inside the
 * image, (min{j+r,W-1} - max{j-l,-1}) * (min{i+u,H-1} - max{i-o,-1}). */
int64_t orc_count(int H, int W, int h, int w, int i, int j)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    int64_t nc = imin(j + r, W - 1) - imax(j - l, -1);
    int64_t nr = imin(i + u, H - 1) - imax(i - o, -1);
    return nc * nr;
}

/* The direct definition (Introduction): for every pixel add up I and I^2 over
 * the clipped window.  Theta(H W h w). */
void orc_sums_direct(const uint8_t *I, int H, int W, int64_t ld, int h, int w,
                     uint64_t *S1, uint64_t *S2)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            uint64_t s1 = 0, s2 = 0;
            for (int a = i - o + 1; a <= i + u; ++a) {
                if (a < 0 || a >= H) continue;
                for (int b = j - l + 1; b <= j + r; ++b) {
                    if (b < 0 || b >= W) continue;
                    uint64_t v = I[(int64_t)a * ld + b];
                    s1 += v;
                    s2 += v * v;
                }
            }
            S1[(int64_t)i * W + j] = s1;
            S2[(int64_t)i * W + j] = s2;
        }
    }
}

/* Same definition evaluated only at the listed pixels (for large images). */
void orc_sums_direct_at(const uint8_t *I, int H, int W, int64_t ld, int h, int w,
                        int npts, const int32_t *pi, const int32_t *pj,
                        uint64_t *S1, uint64_t *S2)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    for (int p = 0; p < npts; ++p) {
        int i = pi[p], j = pj[p];
        uint64_t s1 = 0, s2 = 0;
        for (int a = i - o + 1; a <= i + u; ++a) {
            if (a < 0 || a >= H) continue;
            for (int b = j - l + 1; b <= j + r; ++b) {
                if (b < 0 || b >= W) continue;
                uint64_t v = I[(int64_t)a * ld + b];
                s1 += v;
                s2 += v * v;
            }
        }
        S1[p] = s1;
        S2[p] = s2;
    }
}

/* Zero-extended pixel access (Section 3.2: undefined elements are zero). */
static uint32_t px(const uint8_t *I, int H, int W, int64_t ld, int i, int j)
{
    if (i < 0 || i >= H || j < 0 || j >= W) return 0;
    return I[(int64_t)i * ld + j];
}

/* Section 3.1's recurrences with the accumulator widths of Section 3.3.
 *
 * Both passes use one idea: a window sum at position p is the sum at p-1 plus
 * the element entering the window minus the element leaving it.  Each pass
 * starts from a window that lies wholly before the image (all zero under the
 * zero extension of Section 3.2, so its sum is 0 and no priming pass is
 * needed) and slides into the image one position at a time; outputs are
 * written only from position 0 on.
 *
 * Vertical: the column sums C_j (16 bits: at most 257 values of at most 255)
 * and D_j (32 bits) of the window rows i-o+1 .. i+u, slid from row -u-1
 * (rows -u-o .. -1, empty) down to row H-1.
 * Horizontal: for each row, c and d over columns j-l+1 .. j+r of C and D,
 * slid from column -r-1 to W-1 (32 bits: every window sum is below 2^32, so
 * the wrap-around differences are exact).
 * Requires h, w <= 257 (Section 3.3's range argument). */

/* Add the entering row and remove the leaving row of every column sum. */
static void slide_columns(const uint8_t *I, int H, int W, int64_t ld, int enter, int leave,
                          uint16_t *C, uint32_t *D)
{
    for (int j = 0; j < W; ++j) {
        uint32_t a = px(I, H, W, ld, enter, j);
        uint32_t b = px(I, H, W, ld, leave, j);
        C[j] = (uint16_t)(C[j] + a - b);
        D[j] = D[j] + a * a - b * b;
    }
}

/* The row window sums of one row of column sums: c and d slide along the row
 * (entering column j+r, leaving column j-l; columns outside the row are 0). */
static void slide_row(const uint16_t *C, const uint32_t *D, int W, int l, int r, uint32_t *S1,
                      uint32_t *S2)
{
    uint32_t c = 0, d = 0;
    for (int j = -r; j < W; ++j) {
        if (j + r < W) {
            c += C[j + r];
            d += D[j + r];
        }
        if (j - l >= 0) {
            c -= C[j - l];
            d -= D[j - l];
        }
        if (j >= 0) {
            S1[j] = c;
            S2[j] = d;
        }
    }
}

int orc_sums_recursive(const uint8_t *I, int H, int W, int64_t ld, int h, int w,
                       uint32_t *S1, uint32_t *S2)
{
    if (h > 257 || w > 257) return -1;
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    uint16_t *C = (uint16_t *)calloc((size_t)W, sizeof(uint16_t));
    uint32_t *D = (uint32_t *)calloc((size_t)W, sizeof(uint32_t));
    if (!C || !D) { free(C); free(D); return -2; }
    for (int i = -u; i < H; ++i) {
        slide_columns(I, H, W, ld, i + u, i - o, C, D);
        if (i >= 0) slide_row(C, D, W, l, r, S1 + (int64_t)i * W, S2 + (int64_t)i * W);
    }
    free(C);
    free(D);
    return 0;
}

/* Integral images (Section 2): J(i,j) = sum over a <= i, b <= j of f(I), and a
 * window sum is J(a1,b1) - J(a0,b1) - J(a1,b0) + J(a0,b0).  64-bit entries. */
int orc_sums_integral(const uint8_t *I, int H, int W, int64_t ld, int h, int w,
                      uint64_t *S1, uint64_t *S2)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    int64_t Wp = (int64_t)W + 1;
    int64_t *J1 = (int64_t *)calloc((size_t)((H + 1) * Wp), sizeof(int64_t));
    int64_t *J2 = (int64_t *)calloc((size_t)((H + 1) * Wp), sizeof(int64_t));
    if (!J1 || !J2) { free(J1); free(J2); return -2; }
    /* J[(i+1)*Wp + (j+1)] holds J(i, j); row/column 0 hold J(-1, .) = 0. */
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            int64_t v = I[(int64_t)i * ld + j];
            int64_t a = (int64_t)(i + 1) * Wp + (j + 1);
            J1[a] = J1[a - Wp] + J1[a - 1] - J1[a - Wp - 1] + v;
            J2[a] = J2[a - Wp] + J2[a - 1] - J2[a - Wp - 1] + v * v;
        }
    }
    for (int i = 0; i < H; ++i) {
        int a0 = imax(i - o, -1), a1 = imin(i + u, H - 1);
        for (int j = 0; j < W; ++j) {
            int b0 = imax(j - l, -1), b1 = imin(j + r, W - 1);
            int64_t p11 = (int64_t)(a1 + 1) * Wp + (b1 + 1);
            int64_t p01 = (int64_t)(a0 + 1) * Wp + (b1 + 1);
            int64_t p10 = (int64_t)(a1 + 1) * Wp + (b0 + 1);
            int64_t p00 = (int64_t)(a0 + 1) * Wp + (b0 + 1);
            S1[(int64_t)i * W + j] = (uint64_t)(J1[p11] - J1[p01] - J1[p10] + J1[p00]);
            S2[(int64_t)i * W + j] = (uint64_t)(J2[p11] - J2[p01] - J2[p10] + J2[p00]);
        }
    }
    free(J1);
    free(J2);
    return 0;
}

/* Method codes shared by the threshold routines. */
enum { ORC_MEANSTD = 0, ORC_SAUVOLA = 1, ORC_NIBLACK = 2 };

/* Moments and thresholds in the canonical binary64 sequence:
 *   n from Algorithm 1; Vn = n*S2 - S1^2 as an exact 64-bit integer (the
 *   population variance numerator, Introduction's s formula times n^2);
 *   m = S1 / n; v = Vn / (n*n); s = sqrt(v);
 *   Sauvola (Introduction; Table 1): t = m * (1 + k * (s / R - 1));
 *   Niblack (Table 1): t = m + k * s;
 *   mask = 1 iff I < t.
 * Every operation rounds to nearest once; nothing is fused.
 * m, s, t and mask may be NULL.  S1, S2 are dense H x W. */
void orc_threshold(const uint8_t *I, int H, int W, int64_t ld, int h, int w,
                   const uint64_t *S1, const uint64_t *S2, int method, float k, float R,
                   double *m_out, double *s_out, double *t_out, uint8_t *mask)
{
    const double k64 = (double)k, R64 = (double)R;
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            int64_t p = (int64_t)i * W + j;
            int64_t n = orc_count(H, W, h, w, i, j);
            int64_t s1 = (int64_t)S1[p], s2 = (int64_t)S2[p];
            int64_t Vn = n * s2 - s1 * s1;
            double nd = (double)n;
            double m = (double)s1 / nd;
            double v = (double)Vn / (nd * nd);
            double s = sqrt(v);
            double t = 0.0;
            if (method == ORC_SAUVOLA) {
                double q = s / R64;
                q = q - 1.0;
                q = k64 * q;
                q = 1.0 + q;
                t = m * q;
            } else if (method == ORC_NIBLACK) {
                double q = k64 * s;
                t = m + q;
            }
            if (m_out) m_out[p] = m;
            if (s_out) s_out[p] = s;
            if (t_out) t_out[p] = t;
            if (mask) mask[p] = ((double)I[(int64_t)i * ld + j] < t) ? 1 : 0;
        }
    }
}

/* Global statistics of an image, in Table 1's notation: L = minimum gray
 * level, M = mean and S = population standard deviation of all N = H W gray
 * levels.  The sums T1 = sum I and T2 = sum I^2 are exact integers and
 * N T2 - T1^2 is exact in 128 bits; then, each operation rounded once,
 * M = T1 / N and S = sqrt(VN / (N N)) with VN = N T2 - T1^2 rounded to
 * binary64.  out: L, the maximum, M, S; sums: N, T1, T2. */
void orc_global_stats(const uint8_t *I, int H, int W, int64_t ld, double out[4], uint64_t sums[3])
{
    uint64_t T1 = 0, T2 = 0;
    unsigned lo = 255, hi = 0;
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            const unsigned g = I[(int64_t)i * ld + j];
            T1 += g;
            T2 += (uint64_t)g * g;
            if (g < lo) lo = g;
            if (g > hi) hi = g;
        }
    }
    const uint64_t N = (uint64_t)H * (uint64_t)W;
    const unsigned __int128 VN = (unsigned __int128)N * T2 - (unsigned __int128)T1 * T1;
    const double Nd = (double)N;
    out[0] = (double)lo;
    out[1] = (double)hi;
    out[2] = (double)T1 / Nd;
    out[3] = sqrt((double)VN / (Nd * Nd));
    sums[0] = N;
    sums[1] = T1;
    sums[2] = T2;
}

/* The remaining thresholds of Table 1, each in one binary64 sequence (every
 * operation rounded once, nothing fused) from the canonical m, s of
 * orc_threshold and the global L, M, S of orc_global_stats:
 *   Wolf:       t = m - k (m - L) (1 - s/R)             p = {k, R}
 *   Feng:       t = a1 m + k1 (s/R)^(1+g) (m - L)
 *                    + k2 (s/R)^g L                       p = {a1, k1, k2, g, R}
 *   Rais:       t = m + 0.3 (m s - M S) / max{m s, M S} s (the fraction is
 *               taken as 0 where both products are 0)      p = {}
 *   Khurshid (NICK): t = m + k sqrt(s^2 + m^2 (n-1)/n), with the window's
 *               in-bounds count n in place of h w          p = {k}
 *   Phansalkar: t = m (1 + p e^(-q m) + k (s/R - 1))      p = {p, q, k, R}
 * mask = 1 iff I < t.  pow and exp are the C library's. */
enum { ORC_WOLF = 3, ORC_FENG = 4, ORC_RAIS = 5, ORC_NICK = 6, ORC_PHANSALKAR = 7 };

double orc_table1_t(int method, double m, double s, double n, const double *p, double L, double M,
                    double S)
{
    switch (method) {
    case ORC_WOLF: {
        double a = s / p[1];
        a = 1.0 - a;
        double b = m - L;
        b = p[0] * b;
        b = b * a;
        return m - b;
    }
    case ORC_FENG: {
        const double x = s / p[4];
        const double x1 = pow(x, 1.0 + p[3]);
        const double x0 = pow(x, p[3]);
        const double a = p[0] * m;
        double b = p[1] * x1;
        b = b * (m - L);
        double c = p[2] * x0;
        c = c * L;
        double t = a + b;
        return t + c;
    }
    case ORC_RAIS: {
        const double a = m * s, b = M * S;
        const double e = a > b ? a : b;
        double f = 0.0;
        if (e > 0.0) f = (a - b) / e;
        double g = 0.3 * f;
        g = g * s;
        return m + g;
    }
    case ORC_NICK: {
        const double a = s * s;
        double b = m * m;
        const double c = (n - 1.0) / n;
        b = b * c;
        const double r = sqrt(a + b);
        const double q = p[0] * r;
        return m + q;
    }
    case ORC_PHANSALKAR: {
        double e = p[1] * m;
        e = exp(-e);
        const double a = p[0] * e;
        double b = s / p[3];
        b = b - 1.0;
        b = p[2] * b;
        double c = 1.0 + a;
        c = c + b;
        return m * c;
    }
    default:
        return 0.0;
    }
}

/* Table 1 thresholds over an image: m, s as in orc_threshold (canonical
 * binary64), then orc_table1_t.  gstats: L, max, M, S from orc_global_stats.
 * t and mask may be NULL; S1, S2 dense H x W. */
void orc_table1(const uint8_t *I, int H, int W, int64_t ld, int h, int w, const uint64_t *S1,
                const uint64_t *S2, int method, const double *p, const double *gstats, double *t_out,
                uint8_t *mask)
{
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            const int64_t q = (int64_t)i * W + j;
            const int64_t n = orc_count(H, W, h, w, i, j);
            const int64_t s1 = (int64_t)S1[q], s2 = (int64_t)S2[q];
            const int64_t Vn = n * s2 - s1 * s1;
            const double nd = (double)n;
            const double m = (double)s1 / nd;
            const double v = (double)Vn / (nd * nd);
            const double s = sqrt(v);
            const double t = orc_table1_t(method, m, s, nd, p, gstats[0], gstats[2], gstats[3]);
            if (t_out) t_out[q] = t;
            if (mask) mask[q] = ((double)I[(int64_t)i * ld + j] < t) ? 1 : 0;
        }
    }
}

/* The square-root-free Sauvola decision of Section 3.2 (k >= 0), in binary64:
 * background (paper's output 0) iff I + m(k-1) <= 0 or
 * (I + m(k-1))^2 <= k^2 m^2 v / R^2.  Writes the paper's output bit I'. */
void orc_sauvola_sqrtfree(const uint8_t *I, int H, int W, int64_t ld, int h, int w,
                          const uint64_t *S1, const uint64_t *S2, float k, float R,
                          uint8_t *out)
{
    const double k64 = (double)k, R64 = (double)R;
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            int64_t p = (int64_t)i * W + j;
            int64_t n = orc_count(H, W, h, w, i, j);
            int64_t s1 = (int64_t)S1[p], s2 = (int64_t)S2[p];
            double nd = (double)n;
            double m = (double)s1 / nd;
            double v = (double)(n * s2 - s1 * s1) / (nd * nd);
            double a = (double)I[(int64_t)i * ld + j] + m * (k64 - 1.0);
            double rhs = (k64 * k64) * (m * m) * v / (R64 * R64);
            out[p] = (a <= 0.0 || a * a <= rhs) ? 0 : 1;
        }
    }
}

/* Windowed quantile, direct form: gather the clipped window, sort it, take the
 * rho-th smallest value with rho = max(1, ceil(q * n)) (q * n in binary64).
 * Q and mask (= 1 iff I < Q) are dense H x W; mask may be NULL. */
static int cmp_u8(const void *a, const void *b)
{
    return (int)(*(const uint8_t *)a) - (int)(*(const uint8_t *)b);
}

int64_t orc_rank(double q, int64_t n)
{
    double x = ceil(q * (double)n);
    int64_t rho = (int64_t)x;
    return rho < 1 ? 1 : rho;
}

void orc_quantile_sort(const uint8_t *I, int H, int W, int64_t ld, int h, int w, double q,
                       uint8_t *Q, uint8_t *mask)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    uint8_t *buf = (uint8_t *)malloc((size_t)h * (size_t)w);
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            int64_t n = 0;
            for (int a = imax(i - o + 1, 0); a <= imin(i + u, H - 1); ++a)
                for (int b = imax(j - l + 1, 0); b <= imin(j + r, W - 1); ++b)
                    buf[n++] = I[(int64_t)a * ld + b];
            qsort(buf, (size_t)n, 1, cmp_u8);
            int64_t rho = orc_rank(q, n);
            uint8_t val = buf[rho - 1];
            Q[(int64_t)i * W + j] = val;
            if (mask) mask[(int64_t)i * W + j] = (I[(int64_t)i * ld + j] < val) ? 1 : 0;
        }
    }
    free(buf);
}

/* Windowed quantile by a sliding 256-bin histogram (Section 3.4): along each
 * row the window histogram loses the leaving column and gains the entering
 * column; the quantile is the smallest gray level g whose cumulative count
 * reaches rho. */
void orc_quantile_hist(const uint8_t *I, int H, int W, int64_t ld, int h, int w, double q,
                       uint8_t *Q, uint8_t *mask)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    int64_t hist[256];
    for (int i = 0; i < H; ++i) {
        int a0 = imax(i - o + 1, 0), a1 = imin(i + u, H - 1);
        memset(hist, 0, sizeof(hist));
        /* columns 0 .. r-1 enter before the first pixel of the row */
        for (int b = 0; b < r && b < W; ++b)
            for (int a = a0; a <= a1; ++a) hist[I[(int64_t)a * ld + b]]++;
        for (int j = 0; j < W; ++j) {
            int bin = j + r, bout = j - l;
            if (bin < W)
                for (int a = a0; a <= a1; ++a) hist[I[(int64_t)a * ld + bin]]++;
            if (bout >= 0)
                for (int a = a0; a <= a1; ++a) hist[I[(int64_t)a * ld + bout]]--;
            int64_t n = orc_count(H, W, h, w, i, j);
            int64_t rho = orc_rank(q, n);
            int64_t cum = 0;
            int g = 0;
            for (g = 0; g < 256; ++g) {
                cum += hist[g];
                if (cum >= rho) break;
            }
            Q[(int64_t)i * W + j] = (uint8_t)g;
            if (mask) mask[(int64_t)i * W + j] = (I[(int64_t)i * ld + j] < g) ? 1 : 0;
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Differentiable (soft) Sauvola in binary64.                               */
/* Forward: window sums of a real-valued image, m, s and the Sauvola        */
/* threshold t as above, then y = 1 / (1 + exp(-(I - t) / tau)).            */
/* Backward for an upstream gradient g = dL/dy, by the chain rule through   */
/* t = m (1 + k (s/R - 1)), m = S1/n, s = sqrt(S2/n - m^2), and the window  */
/* sums S1 = sum I, S2 = sum I^2; a pixel q feeds every window containing   */
/* it, i.e. the pixels p of the reflected window rows q-u..q+o-1, columns   */
/* q-r..q+l-1.  Where v = 0 the derivative of s does not exist; there the   */
/* s-terms are dropped.                                                     */
/* ----------------------------------------------------------------------- */

/* Window sums of a float image over the clipped window, binary64, direct. */
static void fsum_direct(const float *I, int H, int W, int h, int w, int i, int j,
                        double *s1, double *s2)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    double a1 = 0.0, a2 = 0.0;
    for (int a = imax(i - o + 1, 0); a <= imin(i + u, H - 1); ++a)
        for (int b = imax(j - l + 1, 0); b <= imin(j + r, W - 1); ++b) {
            double v = (double)I[(int64_t)a * W + b];
            a1 += v;
            a2 += v * v;
        }
    *s1 = a1;
    *s2 = a2;
}

/* Per-pixel forward quantities at (i, j) of one image. */
static void soft_point(const float *I, int H, int W, int h, int w, double k, double R,
                       double tau, int i, int j, double *m, double *s, double *t, double *y,
                       double *n_out)
{
    double s1, s2;
    fsum_direct(I, H, W, h, w, i, j, &s1, &s2);
    double n = (double)orc_count(H, W, h, w, i, j);
    double mm = s1 / n;
    double v = (n * s2 - s1 * s1) / (n * n);
    if (v < 0.0) v = 0.0;
    double ss = sqrt(v);
    double tt = mm * (1.0 + k * (ss / R - 1.0));
    double z = ((double)I[(int64_t)i * W + j] - tt) / tau;
    *m = mm;
    *s = ss;
    *t = tt;
    *y = 1.0 / (1.0 + exp(-z));
    *n_out = n;
}

/* y for all pixels of B images (each H x W, contiguous); k has B entries. */
void orc_soft_fwd(const float *I, int B, int H, int W, int h, int w, const double *k,
                  double R, double tau, double *y, double *t)
{
    for (int b = 0; b < B; ++b) {
        const float *Ib = I + (int64_t)b * H * W;
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                double m, s, tt, yy, n;
                soft_point(Ib, H, W, h, w, k[b], R, tau, i, j, &m, &s, &tt, &yy, &n);
                int64_t p = (int64_t)b * H * W + (int64_t)i * W + j;
                y[p] = yy;
                if (t) t[p] = tt;
            }
    }
}

/* Box sum of a binary64 field over each pixel's clipped window (the
 * operator B of the window sums, direct form). */
void orc_box_f64(const double *x, int H, int W, int h, int w, double *out)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double acc = 0.0;
            for (int a = imax(i - o + 1, 0); a <= imin(i + u, H - 1); ++a)
                for (int b = imax(j - l + 1, 0); b <= imin(j + r, W - 1); ++b)
                    acc += x[(int64_t)a * W + b];
            out[(int64_t)i * W + j] = acc;
        }
}

/* The adjoint B* of the window sum: pixel q receives the sum of G over the
 * centres p whose window contains q.  From p-o < q <= p+u this is
 * q-u <= p <= q+o-1 for rows and q-r <= p <= q+l-1 for columns (the window
 * reflected through q), clipped to the image. */
void orc_box_adjoint(const double *G, int H, int W, int h, int w, double *out)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double acc = 0.0;
            for (int pi = imax(i - u, 0); pi <= imin(i + o - 1, H - 1); ++pi)
                for (int pj = imax(j - r, 0); pj <= imin(j + l - 1, W - 1); ++pj)
                    acc += G[(int64_t)pi * W + pj];
            out[(int64_t)i * W + j] = acc;
        }
}

/* Gradients of L = sum g * y with respect to I (all pixels), k (per image)
 * and R (shared).  Direct evaluation: first the per-pixel adjoint fields
 * G1 = dL/dS1 and G2 = dL/dS2 of every window, then for every pixel q the sum
 * of G1 + 2 I_q G2 over the windows that contain q. */
void orc_soft_bwd(const float *I, const double *g, int B, int H, int W, int h, int w,
                  const double *k, double R, double tau, double *gI, double *gk, double *gR)
{
    int o, u, l, r;
    extents(h, w, &o, &u, &l, &r);
    int64_t HW = (int64_t)H * W;
    double *G1 = (double *)malloc((size_t)HW * sizeof(double));
    double *G2 = (double *)malloc((size_t)HW * sizeof(double));
    double *dd = (double *)malloc((size_t)HW * sizeof(double));
    double *A1 = (double *)malloc((size_t)HW * sizeof(double));
    double *A2 = (double *)malloc((size_t)HW * sizeof(double));
    double gr = 0.0;
    for (int b = 0; b < B; ++b) {
        const float *Ib = I + (int64_t)b * HW;
        const double *gb = g + (int64_t)b * HW;
        double kb = k[b], gkb = 0.0;
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                int64_t p = (int64_t)i * W + j;
                double m, s, t, y, n;
                soft_point(Ib, H, W, h, w, kb, R, tau, i, j, &m, &s, &t, &y, &n);
                double delta = gb[p] * y * (1.0 - y); /* dL/dz */
                double e = -delta / tau;              /* dL/dt */
                /* t = m (1 + k (s/R - 1)) */
                gkb += e * m * (s / R - 1.0);
                gr += e * (-kb * m * s / (R * R));
                double dt_dm = 1.0 + kb * (s / R - 1.0);
                double dt_ds = kb * m / R;
                double a = e * dt_dm; /* dL/dm through t */
                double beta = e * dt_ds; /* dL/ds through t */
                /* m = S1/n: dm/dS1 = 1/n.  s = sqrt(S2/n - (S1/n)^2):
                 * ds/dS1 = -m / (n s), ds/dS2 = 1 / (2 n s). */
                if (s > 0.0) {
                    G1[p] = a / n - beta * m / (n * s);
                    G2[p] = beta / (2.0 * n * s);
                } else {
                    G1[p] = a / n;
                    G2[p] = 0.0;
                }
                dd[p] = delta / tau; /* direct path: dz/dI = 1/tau */
            }
        gk[b] = gkb;
        orc_box_adjoint(G1, H, W, h, w, A1);
        orc_box_adjoint(G2, H, W, h, w, A2);
        for (int64_t q = 0; q < HW; ++q)
            gI[(int64_t)b * HW + q] = dd[q] + A1[q] + 2.0 * (double)Ib[q] * A2[q];
    }
    *gR = gr;
    free(G1);
    free(G2);
    free(dd);
    free(A1);
    free(A2);
}
