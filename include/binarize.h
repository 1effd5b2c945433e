/*
 * binarize.h -- C ABI of the MI355X (gfx950) library for the sliding-window
 * statistics of local adaptive binarization (Chan, "Memory-efficient and fast
 * implementation of local adaptive binarization methods").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Images.  Row-major, element (i, j) at base[i * ld + j], 0 <= i < H rows,
 *   0 <= j < W columns; every `ld_*` is a row stride in ELEMENTS and must be
 *   >= W.  Gray levels are uint8 (0..255).
 * Window.  h rows by w columns.  With o = floor((h+1)/2), u = floor(h/2),
 *   l = floor((w+1)/2), r = floor(w/2) (Algorithm 1), the window of pixel
 *   (i, j) is rows i-o+1 .. i+u and columns j-l+1 .. j+r, i.e. the bounds
 *   i - h/2 < a <= i + h/2 of the Introduction's mean formula.  Windows are
 *   clipped to the image: out-of-image pixels are zero (Section 3.2) and the
 *   divisor is the in-bounds count n of Algorithm 1.  1 <= h, w <= 257: within
 *   that range the column sums fit 16 bits and the window sum of squares fits
 *   32 bits (Section 3.3).
 * Memory.  Every pointer is DEVICE memory owned by the caller unless stated
 *   otherwise.  The library never allocates or frees device memory.  A call
 *   enqueues its kernels on `stream` and returns without synchronising; the
 *   exceptions are the set-up call bz_batched_plan, which synchronises its
 *   stream once, and bz_binarize_streamed, whose image and mask live in host
 *   memory and which returns when the mask is complete.  Outputs must not overlap the input or each other (Section
 *   3.2's aliasing assumption); overlapping byte ranges are rejected with
 *   BZ_ERR_ALIAS.  32-bit outputs must be 4-byte aligned.
 * Stream.  `stream` is a hipStream_t (NULL = the null stream).
 * Errors.  Arguments are validated before any HIP call; an invalid call
 *   returns its status and enqueues nothing.  BZ_ERR_HIP reports a launch
 *   failure.  Output contents are undefined after an error.  Calls are
 *   re-entrant; calls on different streams may run concurrently.
 */
#ifndef BINARIZE_H
#define BINARIZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *bz_stream; /* hipStream_t */

typedef enum {
    BZ_OK = 0,
    BZ_ERR_INVALID = 1,   /* bad size, stride, pointer or parameter */
    BZ_ERR_RANGE = 2,     /* h or w above 257, sizes beyond 2^31, h rows of the
                             image (h * ld + W bytes) spanning 2^31 bytes or more,
                             or one float32 image of the soft calls spanning
                             ((H - 1) * ld + W) 2^29 elements or more */
    BZ_ERR_ALIAS = 3,     /* an output overlaps the input or another output */
    BZ_ERR_WORKSPACE = 4, /* caller workspace too small */
    BZ_ERR_HIP = 5        /* the HIP runtime reported an error */
} bz_status;

/* Human-readable name of a status code (static string). */
const char *bz_status_string(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int bz_version(void);

/* Largest accepted window side (257, Section 3.3). */
int bz_max_window(void);

/*
 * Window sums S1 = sum I and S2 = sum I^2 over each pixel's clipped window
 * (the quantity Algorithm 1 maintains in c and d; the Introduction's
 * definition).  S1, S2: uint32 H x W with row stride ld_S; both exact.
 */
bz_status bz_window_sums(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                         uint32_t *S1, uint32_t *S2, ptrdiff_t ld_S, bz_stream stream);

/*
 * Window mean m = S1/n and population standard deviation
 * s = sqrt(n S2 - S1^2) / n (Introduction, with Algorithm 1's divisor n).
 * n S2 - S1^2 is formed exactly (its terms are integers below 2^53, combined
 * by one binary64 fused multiply-add); m and s are float32, within 1e-6
 * relative of the binary64 values, and s == 0 exactly where the window is
 * constant.  mean, std: float H x W, row stride ld_out.
 */
bz_status bz_window_mean_std(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                             float *mean, float *std, ptrdiff_t ld_out, bz_stream stream);

/*
 * Sauvola binarization (Introduction; Table 1): t = m (1 + k (s/R - 1)) and
 * mask = 1 where I < t, else 0.  k >= 0 (Algorithm 1's input), R > 0.
 * mask: uint8 H x W, row stride ld_mask.  mean, std: optional float32 outputs
 * (NULL to skip), row stride ld_ms.  The mask equals that of the binary64
 * sequence m = S1/n, v = (n S2 - S1^2)/(n n), s = sqrt(v),
 * t = m * (1 + k * (s/R - 1)), each operation rounded once, with k and R
 * widened from float.
 */
bz_status bz_sauvola(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, float k,
                     float R, uint8_t *mask, ptrdiff_t ld_mask, float *mean, float *std,
                     ptrdiff_t ld_ms, bz_stream stream);

/*
 * Niblack binarization (Table 1): t = m + k s, any finite k; mask = 1 where
 * I < t.  Outputs as bz_sauvola; the binary64 sequence is t = m + k * s.
 */
bz_status bz_niblack(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, float k,
                     uint8_t *mask, ptrdiff_t ld_mask, float *mean, float *std,
                     ptrdiff_t ld_ms, bz_stream stream);

/*
 * Windowed quantile from sliding 256-bin gray-level histograms (Section 3.4):
 * Q = the rho-th smallest gray level of the clipped window, with
 * rho = max(1, ceil(q * n)) evaluated in binary64 (0 <= q <= 1; q = 0.5 is
 * the lower median, q = 1 the maximum).  Q: uint8 H x W (row stride ld_Q);
 * mask (optional, NULL to skip): 1 where I < Q, row stride ld_mask.
 */
bz_status bz_window_quantile(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                             double q, uint8_t *Q, ptrdiff_t ld_Q, uint8_t *mask,
                             ptrdiff_t ld_mask, bz_stream stream);

/* Workspace bytes of bz_window_minmax and bz_bernsen for an H x W image. */
size_t bz_extremes_workspace_size(int H, int W);

/*
 * Window minimum and maximum of the clipped window (in-bounds pixels only;
 * the paper's local extremes, which it keeps with deques).  Windows of at
 * most 64 x 64 run in one launch with both separable passes in on-chip
 * memory; larger ones take two passes through a 16-bit H x W field in
 * `workspace`.  The workspace (DEVICE memory of at least
 * bz_extremes_workspace_size(H, W) bytes, 4-byte aligned, overlapping no
 * input or output) is checked either way.  mn, mx: uint8 H x W, row stride
 * ld_out; exact.
 */
bz_status bz_window_minmax(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, uint8_t *mn,
                           uint8_t *mx, ptrdiff_t ld_out, void *workspace, size_t ws_bytes,
                           bz_stream stream);

/*
 * Bernsen's midrange rule (cited by the paper beside Table 1 as a method on
 * local extremes): with mn, mx the window minimum and maximum,
 * mask = 1 where mx - mn >= contrast_min (0 .. 256) and 2 I < mn + mx, else
 * 0 (windows of lower contrast are background).  mn and mx (row stride
 * ld_mm) are written as well; all integer, exact.  Workspace as for
 * bz_window_minmax.
 */
bz_status bz_bernsen(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int contrast_min,
                     uint8_t *mask, ptrdiff_t ld_mask, uint8_t *mn, uint8_t *mx, ptrdiff_t ld_mm,
                     void *workspace, size_t ws_bytes, bz_stream stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it): bz_bernsen without a workspace
 * argument.  The 16-bit field of the two passes (windows over 64 rows or
 * columns) lives in a device array of the library, fixed at 32 MiB per GPU
 * (held until the process ends), so
 * H W must not exceed bz_bernsen_noalloc_max_pixels() (16,777,216; larger
 * images return BZ_ERR_WORKSPACE).  The call allocates nothing; its first
 * call on a device looks up that device's array (BZ_ERR_HIP if the lookup
 * fails).  Every call on one GPU shares the array: calls that overlap in
 * time on one GPU (on different streams) race and give undefined outputs;
 * calls ordered on one stream do not.  No part of the array needs to start
 * at zero (the first pass writes every entry the second pass reads).
 * Arguments, validation and results are those of bz_bernsen.
 */
size_t bz_bernsen_noalloc_max_pixels(void);
bz_status bz_bernsen_noalloc(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int contrast_min,
                             uint8_t *mask, ptrdiff_t ld_mask, uint8_t *mn, uint8_t *mx, ptrdiff_t ld_mm,
                             bz_stream stream);

/* Thresholding rule of a batched item. */
enum { BZ_METHOD_SAUVOLA = 1, BZ_METHOD_NIBLACK = 2 };

/* The other rules of Table 1, for bz_threshold. */
enum {
    BZ_METHOD_WOLF = 3,
    BZ_METHOD_FENG = 4,
    BZ_METHOD_RAIS = 5,
    BZ_METHOD_NICK = 6, /* Khurshid et al. */
    BZ_METHOD_PHANSALKAR = 7
};

/*
 * Global statistics of one image (Table 1's notation: L the minimum gray
 * level, M the mean, S the population standard deviation), as written by
 * bz_global_stats into DEVICE memory (8-byte aligned, 48 bytes): n = H W,
 * sum and sumsq the exact sums of I and I^2, min and max, then
 * mean = sum / n and std = sqrt((n sumsq - sum^2) / (n n)) in binary64, with
 * n sumsq - sum^2 formed exactly and rounded once.
 */
typedef struct {
    uint64_t n, sum, sumsq;
    uint32_t min, max;
    double mean, std;
} bz_global;

/*
 * Compute the global statistics of I into `stats` (device).  Two small
 * kernels on `stream`: a reset, then an accumulation whose last workgroup
 * forms mean and std (meanwhile the record's n counts the finished
 * workgroups, so the record is complete only when the call's work is).  No
 * memset, so the call can be captured in a graph.  Deterministic (integer
 * atomics).
 */
bz_status bz_global_stats(const uint8_t *I, int H, int W, ptrdiff_t ld_I, bz_global *stats,
                          bz_stream stream);

/*
 * The other thresholding rules of Table 1, each deciding mask = 1 where
 * I < t in one binary64 sequence from the canonical m, s (as in bz_sauvola),
 * every operation rounded once:
 *   BZ_METHOD_WOLF        t = m - k (m - L)(1 - s/R)          params {k, R}
 *   BZ_METHOD_FENG        t = a1 m + k1 (s/R)^(1+g) (m - L)
 *                             + k2 (s/R)^g L                  params {a1, k1, k2, g, R}
 *   BZ_METHOD_RAIS        t = m + 0.3 (m s - M S) / max{m s, M S} s, the
 *                         fraction taken as 0 where both products are 0
 *                                                             params {} (NULL allowed)
 *   BZ_METHOD_NICK        t = m + k sqrt(s^2 + m^2 (n-1)/n), with the
 *                         window's in-bounds count n for h w  params {k}
 *   BZ_METHOD_PHANSALKAR  t = m (1 + p e^(-q m) + k (s/R - 1)) params {p, q, k, R}
 * `params` is a HOST array read during the call; every value must be finite
 * and R > 0.  `stats` is the DEVICE record of bz_global_stats for this image
 * (Wolf and Feng read L, Rais reads M and S; NULL allowed for NICK and
 * Phansalkar); it must be complete when the kernel runs (same stream, or
 * synchronised).  mask, mean, std as in bz_sauvola.  Feng's powers and
 * Phansalkar's exponential use the device's binary64 pow and exp, so near
 * exact ties a pixel's decision can differ from a C library's.
 */
bz_status bz_threshold(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int method,
                       const double *params, const bz_global *stats, uint8_t *mask,
                       ptrdiff_t ld_mask, float *mean, float *std, ptrdiff_t ld_ms,
                       bz_stream stream);

/* One image of a ragged batch; pointers are device memory, mean/std may be
 * NULL.  Each item has its own size, strides, window and parameters. */
typedef struct {
    const uint8_t *I;
    uint8_t *mask;
    float *mean;
    float *std;
    int H, W, h, w;
    ptrdiff_t ld_I, ld_mask, ld_ms;
    float k, R;
    int method; /* BZ_METHOD_SAUVOLA or BZ_METHOD_NIBLACK */
} bz_item;

/* Haar-like feature templates: a grid of a x b cells, signs row by row. */
enum {
    BZ_HAAR_EDGE_H = 1, /* [+ -]          1 x 2 cells */
    BZ_HAAR_EDGE_V = 2, /* [+ ; -]        2 x 1 */
    BZ_HAAR_LINE_H = 3, /* [+ - +]        1 x 3 */
    BZ_HAAR_LINE_V = 4, /* [+ ; - ; +]    3 x 1 */
    BZ_HAAR_CHECKER = 5 /* [+ - ; - +]    2 x 2 */
};

/* Workspace bytes of bz_haar_features for template `kind`: H - a + 1 rows of
 * W 16-bit column sums (row stride rounded up to 64; a column of at most 257
 * gray levels sums below 2^16, Section 3.3), plus as many 32-bit row prefixes
 * when kv * W > 12288 (kv: rows of cells); 0 for invalid arguments. */
size_t bz_haar_workspace_size(int H, int W, int a, int kind);

/*
 * Haar-like features (the rectangle features of Viola and Jones, which
 * Section 3.4 names as computable from recursive window sums instead of an
 * integral image) of one template at every anchor where the whole template
 * lies in the image: with kv x kh cells of a rows by b columns,
 * F[i * ld_F + j] = sum over cells (m, n) of sign(m, n) times the sum of I
 * over rows i + m a .. i + (m+1) a - 1 and columns j + n b .. j + (n+1) b - 1,
 * for 0 <= i < H - kv a + 1 and 0 <= j < W - kh b + 1 (exact int32).  The
 * cell sums come from sliding column sums (Section 3.1's recursion) and row
 * prefixes of them: in one launch, with the workspace unused, for 4-byte
 * aligned rows (I and ld_I) and kh b <= 256; otherwise in two or three
 * launches through the workspace.  1 <= a, b <= 257 (BZ_ERR_RANGE
 * above); a template larger than the image is BZ_ERR_INVALID.  F: int32,
 * 4-byte aligned, ld_F >= W - kh b + 1.  workspace: at least
 * bz_haar_workspace_size(H, W, a, kind) bytes, 256-byte aligned, overlapping
 * neither I nor F.
 */
bz_status bz_haar_features(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int a, int b, int kind, int32_t *F,
                           ptrdiff_t ld_F, void *workspace, size_t ws_bytes, bz_stream stream);

/* Sweep axis of bz_binarize_streamed. */
enum { BZ_AXIS_AUTO = 0, BZ_AXIS_ROWS = 1, BZ_AXIS_COLUMNS = 2 };

/* Device workspace bytes of bz_binarize_streamed (four band slots); 0 for
 * invalid arguments. */
size_t bz_stream_workspace_size(int H, int W, int h, int w, int band, int axis);

/*
 * Sauvola or Niblack (method BZ_METHOD_SAUVOLA or BZ_METHOD_NIBLACK, k and R
 * as for bz_sauvola / bz_niblack; R is ignored by Niblack) over an image in
 * HOST memory that need not fit on the device.  The image streams through the
 * device in bands of `band` lines, each computed with the window's halo
 * (h - 1 rows or w - 1 columns); the mask equals that of bz_sauvola /
 * bz_niblack on the whole image.
 * axis: BZ_AXIS_ROWS sweeps down the rows (bands of whole rows, each host
 * transfer a run of full rows); BZ_AXIS_COLUMNS sweeps across the columns
 * (bands of H rows by `band` columns), so that the resident part spans H
 * elements per line: with the axis of the smaller extent, min{H, W}, as in
 * Section 3.3.  BZ_AXIS_AUTO takes rows unless h + 1 rows of a row band
 * would span 2^31 bytes, then columns.  (Host-to-device copies of short
 * column segments run far below the copy engines' rate for whole rows.)
 * I and mask are HOST pointers, row strides ld_I and ld_mask in elements (no
 * device limit applies to them); page-locked memory (hipHostMalloc) lets the
 * copies run at full rate beside the kernels.  mask may be I itself with
 * ld_mask == ld_I: in-place binarization (Section 3.2).  The halo lines a
 * band shares with the previous band are kept on the device, so no gray
 * level is read after its line was overwritten; any other overlap of I and
 * mask is BZ_ERR_ALIAS.  workspace: DEVICE memory of at least
 * bz_stream_workspace_size(H, W, h, w, band, axis) bytes, 256-byte aligned.
 * Bands are double-buffered: host-to-device copies run on load_stream,
 * kernels and device copies on stream, device-to-host copies on store_stream,
 * so that loading one band, computing another and storing a third overlap
 * (any of the three may be the same stream, which serialises them).  Unlike
 * the device calls this call is SYNCHRONOUS: it returns once the whole mask
 * is in host memory.  BZ_ERR_RANGE also when h + 1 rows of a band's device
 * slot would span 2^31 bytes or more.
 */
bz_status bz_binarize_streamed(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int method,
                               float k, float R, uint8_t *mask, ptrdiff_t ld_mask, int band, int axis,
                               void *workspace, size_t ws_bytes, bz_stream stream,
                               bz_stream load_stream, bz_stream store_stream);

/*
 * Tiling of the single-image box-statistics calls (bz_sauvola, bz_niblack,
 * bz_window_mean_std, bz_window_sums, bz_threshold and the bands of
 * bz_binarize_streamed), for example from a table measured by an autotuner:
 * `rows` is a HOST array of `count` rows of four ints (largest h, largest W,
 * strip rows, threads per workgroup), copied during the call.  A call takes
 * the first row, in order of (largest h, largest W), whose class holds its
 * window height and image width; calls outside every class, or with
 * BZ_TILE_S or BZ_TILE_THREADS set in the environment (which win), keep the
 * built-in plan; a strip or threads of 0 in a row keeps the built-in choice
 * of that parameter.  Results do not depend on the tiling.  count = 0 removes
 * the table.  threads must be 0 or a multiple of 64 in [64, 1024], strip
 * non-negative and the class bounds positive, else BZ_ERR_INVALID and the
 * table is left unchanged.  The
 * table is process-wide; installing it while other threads make calls is
 * safe (each call reads it once).
 */
bz_status bz_set_tile_table(const int *rows, int count);

/* Workspace bytes that bz_sauvola_batched needs for `count` items. */
size_t bz_batched_workspace_size(int count);

/*
 * Binarize a ragged batch in ONE persistent kernel launch (bz_batched_plan
 * followed by bz_batched_run).  `items` is a HOST array of `count`
 * descriptors, read during the call; `workspace` is device memory of at least
 * bz_batched_workspace_size(count) bytes, 64-byte aligned, that must stay
 * untouched until the launch completes.  Each item's outputs equal those of
 * bz_sauvola / bz_niblack on that item alone.  No output may overlap another
 * item's output or input (the items run concurrently): such a batch is
 * rejected with BZ_ERR_ALIAS before any device work; inputs may overlap each
 * other.  Synchronises `stream` once, after the descriptor upload and before
 * the launch.
 */
bz_status bz_sauvola_batched(const bz_item *items, int count, void *workspace,
                             size_t ws_bytes, bz_stream stream);

/*
 * Two-step form of bz_sauvola_batched for callers that replay the same batch
 * (for example inside a captured HIP graph).  bz_batched_plan validates the
 * items, picks each image's tiling (strip_rows: optional HOST array of `count`
 * strip heights in rows, e.g. from an autotuner; NULL or entries < 1 select
 * the default of 2h rows, at least 32 and at most 128), orders the tiles
 * largest-first, uploads the descriptors into `workspace` and SYNCHRONISES
 * `stream` before returning (it is a set-up call, not part of the hot path).
 * It also records, for this workspace address, which kernel runs it: a batch
 * whose items all share the method and the presence of mean/std outputs runs
 * a kernel specialised to that choice (and to 4-byte aligned rows when every
 * item has them); a batch that mixes methods or outputs runs the general
 * kernel.  bz_batched_run launches the single
 * persistent kernel over a planned workspace and returns at once; it neither
 * copies nor synchronises, so it can be captured in a graph and replayed.  The
 * kernel leaves the workspace ready for the next run.  Runs of one workspace
 * must not overlap in time.
 */
bz_status bz_batched_plan(const bz_item *items, int count, const int *strip_rows,
                          void *workspace, size_t ws_bytes, bz_stream stream);
bz_status bz_batched_run(void *workspace, bz_stream stream);

/* Workspace bytes of the soft-Sauvola backward for B images of H x W. */
size_t bz_soft_workspace_size(int B, int H, int W);

/*
 * Differentiable ("soft") Sauvola forward: for B float32 images of H x W
 * (values nominally in [0, 255]; image b at I + b * H * ld, row stride ld),
 * window sums in binary64, m, s and t = m (1 + k_b (s/R - 1)) as above, and
 * y = 1 / (1 + exp(-(I - t) / tau)).  k: float[B] on the device, R: float[1]
 * on the device, tau > 0.  y: float32 with the same layout as I.
 */
bz_status bz_soft_sauvola_fwd(const float *I, int B, int H, int W, ptrdiff_t ld, int h, int w,
                              const float *k, const float *R, float tau, float *y,
                              bz_stream stream);

/*
 * Backward of bz_soft_sauvola_fwd for an upstream gradient gy = dL/dy (same
 * layout as I).  Recomputes the window statistics from I (nothing is saved
 * by the forward); the gradient reaching I through the window sums is the
 * adjoint window sum: pixel q collects from the centres p whose window holds
 * q (rows q-u .. q+o-1, columns q-r .. q+l-1, clipped).  Where s = 0 the
 * derivative of s does not exist and its terms are dropped.  Writes
 * gI (layout of I), gk (float[B]) and gR (float[1]); reductions are
 * deterministic (fixed order).  workspace: device memory of at least
 * bz_soft_workspace_size(B, H, W) bytes.
 */
bz_status bz_soft_sauvola_bwd(const float *I, const float *gy, int B, int H, int W, ptrdiff_t ld,
                              int h, int w, const float *k, const float *R, float tau,
                              float *gI, float *gk, float *gR, void *workspace, size_t ws_bytes,
                              bz_stream stream);

/*
 * The binary64 window sums S1 = sum I and S2 = sum I^2 that the soft calls
 * compute internally (Introduction's definition over the clipped window of
 * Algorithm 1), exported for testing.  The sums run down strips of at most
 * 32 rows, each primed afresh, so the add-and-subtract recurrence of Section
 * 3.1 never runs longer than one strip on real-valued data.  I: B float32
 * images as in bz_soft_sauvola_fwd; S1, S2: binary64, image b at
 * S + b * H * ld_S, row stride ld_S >= W, 8-byte aligned.  BZ_ERR_RANGE if
 * one output image spans 2^28 elements or more.
 */
bz_status bz_soft_window_sums(const float *I, int B, int H, int W, ptrdiff_t ld, int h, int w, double *S1,
                              double *S2, ptrdiff_t ld_S, bz_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BINARIZE_H */
