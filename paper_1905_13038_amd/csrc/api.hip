// C ABI of libbinarize: argument validation, aliasing checks and dispatch to
// the HIP kernels.  Everything here runs on the host; validation finishes
// before the first HIP call, so invalid calls have no device side effects.
#include "../../include/binarize.h"
#include "haar.hpp"
#include "internal.hpp"

#include <mutex>

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

using namespace bz;

namespace {

constexpr int MAX_WIN = 257;

struct Range {
    uintptr_t lo, hi;  // [lo, hi)
};

// Byte range touched by an H x W array of `esize`-byte elements, row stride ld.
Range span(const void *p, int H, int W, ptrdiff_t ld, size_t esize)
{
    const uintptr_t lo = (uintptr_t)p;
    const uintptr_t hi = lo + ((uintptr_t)(H - 1) * (uintptr_t)ld + (uintptr_t)W) * esize;
    return Range{lo, hi};
}

bool overlaps(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; }

// Test hook: BZ_FAULT_INJECT=launch makes every entry point report a HIP
// launch failure instead of launching (used to exercise error mapping).
bool inject_launch_fault()
{
    const char *e = getenv("BZ_FAULT_INJECT");
    return e != nullptr && strcmp(e, "launch") == 0;
}

bz_status hip_status(hipError_t e) { return e == hipSuccess ? BZ_OK : BZ_ERR_HIP; }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Common validation of an image and window.
bz_status check_image(const void *I, int H, int W, ptrdiff_t ld, int h, int w)
{
    if (I == nullptr) return BZ_ERR_INVALID;
    if (H < 1 || W < 1 || h < 1 || w < 1) return BZ_ERR_INVALID;
    if (ld < W) return BZ_ERR_INVALID;
    if (h > MAX_WIN || w > MAX_WIN) return BZ_ERR_RANGE;
    if ((int64_t)H * (int64_t)ld > ((int64_t)1 << 46)) return BZ_ERR_RANGE;
    // the rows one window spans must lie within 2^31 bytes (a kernel reads a
    // strip of rows through one buffer descriptor)
    if ((int64_t)h * (int64_t)ld + W >= ((int64_t)1 << 31)) return BZ_ERR_RANGE;
    return BZ_OK;
}

bz_status check_out(const void *p, int H, int W, ptrdiff_t ld, size_t esize)
{
    if (p == nullptr) return BZ_ERR_INVALID;
    if (ld < W) return BZ_ERR_INVALID;
    if (esize > 1 && !aligned(p, esize)) return BZ_ERR_INVALID;
    if ((int64_t)H * (int64_t)ld > ((int64_t)1 << 46)) return BZ_ERR_RANGE;
    return BZ_OK;
}

BoxJob make_job(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w)
{
    BoxJob j;
    memset(&j, 0, sizeof(j));
    j.I = I;
    j.ldI = ld_I;
    j.H = H;
    j.W = W;
    j.h = h;
    j.w = w;
    return j;
}

// Test and tuning hooks read from the environment at each call:
// BZ_TILE_S / BZ_TILE_THREADS override the strip height / block size, and
// BZ_FORCE_REFERENCE=1 decides every pixel with the binary64 reference
// sequence instead of only those inside the float32 guard.
int env_int(const char *name)
{
    const char *e = getenv(name);
    return e ? atoi(e) : 0;
}

// The tiling table installed by bz_set_tile_table: rows of (largest h,
// largest W, strip rows, threads), kept sorted by (h, W).
struct TileRule {
    int hmax, wmax, strip, threads;
};
std::mutex g_tile_mu;
std::vector<TileRule> g_tile_table;

// Strip and block size for a plain call: the environment's overrides, else
// the first table row whose class holds (h, W), else 0 (the built-in plan;
// a row's 0 also keeps the built-in choice of that parameter).
void tile_choice(int h, int W, int &strip, int &threads)
{
    strip = env_int("BZ_TILE_S");
    threads = env_int("BZ_TILE_THREADS");
    if (strip > 0 || threads > 0) return;
    std::lock_guard<std::mutex> lk(g_tile_mu);
    for (const TileRule &t : g_tile_table)
        if (h <= t.hmax && W <= t.wmax) {
            strip = t.strip;
            threads = t.threads;
            return;
        }
}

bz_status run_box(BoxJob &j, hipStream_t stream)
{
    int strip, threads;
    tile_choice(j.h, j.W, strip, threads);
    plan_box(j, strip, threads);
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_box(j, stream));
}

// Validate a Sauvola/Niblack call and fill its job (without tiling).
bz_status make_threshold_job(int mode, const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h,
                             int w, float k, float R, uint8_t *mask, ptrdiff_t ld_mask,
                             float *mean, float *stdv, ptrdiff_t ld_ms, BoxJob &j)
{
    bz_status st = check_image(I, H, W, ld_I, h, w);
    if (st != BZ_OK) return st;
    if (!isfinite(k)) return BZ_ERR_INVALID;
    if (mode == MODE_SAUVOLA && (!(k >= 0.0f) || !isfinite(R) || !(R > 0.0f))) return BZ_ERR_INVALID;
    if ((st = check_out(mask, H, W, ld_mask, 1)) != BZ_OK) return st;
    if ((mean == nullptr) != (stdv == nullptr)) return BZ_ERR_INVALID;
    const Range in = span(I, H, W, ld_I, 1);
    const Range rm = span(mask, H, W, ld_mask, 1);
    if (overlaps(in, rm)) return BZ_ERR_ALIAS;
    if (mean) {
        if ((st = check_out(mean, H, W, ld_ms, 4)) != BZ_OK) return st;
        if ((st = check_out(stdv, H, W, ld_ms, 4)) != BZ_OK) return st;
        const Range a = span(mean, H, W, ld_ms, 4), b = span(stdv, H, W, ld_ms, 4);
        if (overlaps(in, a) || overlaps(in, b) || overlaps(a, b) || overlaps(a, rm) ||
            overlaps(b, rm))
            return BZ_ERR_ALIAS;
    }
    j = make_job(I, H, W, ld_I, h, w);
    j.mode = mode;
    j.mask = mask;
    j.ldM = ld_mask;
    j.mean = mean;
    j.stdv = stdv;
    j.ldMS = mean ? ld_ms : 0;
    if (mode == MODE_SAUVOLA) {
        j.c0 = (float)(1.0 - (double)k);
        j.c1 = (float)((double)k / (double)R);
    } else {
        j.c0 = 0.0f;
        j.c1 = k;
    }
    j.kabs = fabsf(k);
    j.k64 = (double)k;
    j.R64 = (double)R;
    j.aligned = aligned(I, 4) && ld_I % 4 == 0 && W % 4 == 0;
    j.force_ref = env_int("BZ_FORCE_REFERENCE");
    return BZ_OK;
}

// Threshold entry shared by Sauvola and Niblack.
bz_status threshold_call(int mode, const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                         float k, float R, uint8_t *mask, ptrdiff_t ld_mask, float *mean,
                         float *stdv, ptrdiff_t ld_ms, bz_stream stream)
{
    BoxJob j;
    const bz_status st =
        make_threshold_job(mode, I, H, W, ld_I, h, w, k, R, mask, ld_mask, mean, stdv, ld_ms, j);
    if (st != BZ_OK) return st;
    return run_box(j, (hipStream_t)stream);
}

// Cross-item aliasing of a batch: no output byte range may overlap another
// output range or any input range (inputs may share memory).  The items run
// concurrently, so such an overlap would make the results depend on timing.
// Sorted sweep over the ranges: a range overlaps an earlier one exactly when
// it starts below that range's end.
bz_status check_batch_aliasing(const bz_item *items, int count)
{
    struct Tagged {
        Range r;
        bool out;
    };
    std::vector<Tagged> v;
    v.reserve((size_t)count * 4);
    for (int i = 0; i < count; ++i) {
        const bz_item &it = items[i];
        v.push_back({span(it.I, it.H, it.W, it.ld_I, 1), false});
        v.push_back({span(it.mask, it.H, it.W, it.ld_mask, 1), true});
        if (it.mean) {
            v.push_back({span(it.mean, it.H, it.W, it.ld_ms, 4), true});
            v.push_back({span(it.std, it.H, it.W, it.ld_ms, 4), true});
        }
    }
    std::sort(v.begin(), v.end(), [](const Tagged &x, const Tagged &y) { return x.r.lo < y.r.lo; });
    uintptr_t end_in = 0, end_out = 0;  // largest end so far of each kind
    for (const Tagged &x : v) {
        if (x.r.lo < end_out || (x.out && x.r.lo < end_in)) return BZ_ERR_ALIAS;
        if (x.out) end_out = std::max(end_out, x.r.hi);
        else end_in = std::max(end_in, x.r.hi);
    }
    return BZ_OK;
}

// Default strip height of a batched image: long enough that the h-1 priming
// rows stay a small part of a tile.
int default_batch_strip(int h)
{
    int s = 2 * h;
    if (s < 32) s = 32;
    if (s > 128) s = 128;
    return s;
}

// Banded binarization of an image in host memory (Section 3.3: the sweep can
// run along either axis, so the resident state can span min{H, W}; Section
// 3.2: in-place binarization keeps the window's rows above the current ones
// aside).  The image is cut into bands of `band` lines (rows or columns); band j's
// outputs are lines Y .. Y+B-1 and its input lines A .. E-1 with the halo
// A = Y - (before), E = Y + B + (after), clipped.  Inside the halo every window
// of the band is the window of the whole image, clipped where the image ends,
// so the band computed as an image of its own gives the whole image's results
// on its output lines.  Two input and two output slots alternate; the halo
// lines a band shares with the previous one come from that band's slot
// (device to device), so each host line is read once, before the lines above
// it are written back.
struct BandGeom {
    bool rows;             // bands of rows or of columns
    int len, cross;        // extent along the sweep axis and across it
    int before, after;     // window lines before and after its centre, along the sweep
    int band;              // output lines per band
    int64_t pitch;         // row stride of a device slot, bytes
    int slot_rows;         // rows of a device slot
    size_t slot_bytes;     // bytes of a slot, a multiple of 256
};

int64_t round_up64(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Slot rows of a band of rows at pitch round_up(W, 64) must keep h + 1 of
// them below 2^31 bytes (the device calls' window span).
bool rows_fit(int W, int h) { return (int64_t)(h + 1) * round_up64(W, 64) < ((int64_t)1 << 31); }

BandGeom band_geom(int H, int W, int h, int w, int band, int axis)
{
    BandGeom g;
    g.rows = axis == BZ_AXIS_ROWS || (axis == BZ_AXIS_AUTO && rows_fit(W, h));
    g.len = g.rows ? H : W;
    g.cross = g.rows ? W : H;
    const int win = g.rows ? h : w;
    g.before = (win + 1) / 2 - 1;
    g.after = win / 2;
    g.band = band < g.len ? band : g.len;
    const int64_t lines = std::min<int64_t>((int64_t)g.band + win - 1, g.len);
    g.pitch = g.rows ? round_up64(W, 64) : round_up64(lines, 64);
    g.slot_rows = g.rows ? (int)lines : H;
    g.slot_bytes = (size_t)round_up64(g.pitch * g.slot_rows, 256);
    return g;
}

// Address of line t of a band buffer: a row (rows) or a column.
template <typename T>
T *band_line(T *base, const BandGeom &g, int64_t t, int64_t ld)
{
    return base + (g.rows ? t * ld : t);
}

// Copy `count` lines of g.cross elements between two 2-D buffers.
hipError_t copy_lines(const BandGeom &g, void *dst, int64_t dld, const void *src, int64_t sld, int count,
                      hipMemcpyKind kind, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (g.rows) return hipMemcpy2DAsync(dst, (size_t)dld, src, (size_t)sld, (size_t)g.cross, (size_t)count, kind, s);
    return hipMemcpy2DAsync(dst, (size_t)dld, src, (size_t)sld, (size_t)count, (size_t)g.cross, kind, s);
}

bz_status stream_check(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int method, float k,
                       float R, const uint8_t *mask, ptrdiff_t ld_mask, int band, int axis)
{
    // host buffers: no device limit on their strides, only the size guard
    if (I == nullptr || mask == nullptr) return BZ_ERR_INVALID;
    if (H < 1 || W < 1 || h < 1 || w < 1 || band < 1) return BZ_ERR_INVALID;
    if (axis != BZ_AXIS_AUTO && axis != BZ_AXIS_ROWS && axis != BZ_AXIS_COLUMNS) return BZ_ERR_INVALID;
    if (ld_I < W || ld_mask < W) return BZ_ERR_INVALID;
    if (h > MAX_WIN || w > MAX_WIN) return BZ_ERR_RANGE;
    if ((int64_t)H * (int64_t)ld_I > ((int64_t)1 << 46) || (int64_t)H * (int64_t)ld_mask > ((int64_t)1 << 46))
        return BZ_ERR_RANGE;
    if (method != BZ_METHOD_SAUVOLA && method != BZ_METHOD_NIBLACK) return BZ_ERR_INVALID;
    if (!isfinite(k)) return BZ_ERR_INVALID;
    if (method == BZ_METHOD_SAUVOLA && (!(k >= 0.0f) || !isfinite(R) || !(R > 0.0f))) return BZ_ERR_INVALID;
    // in place (the same buffer and stride) or disjoint
    const bool same = (const void *)mask == (const void *)I && ld_mask == ld_I;
    if (!same && overlaps(span(I, H, W, ld_I, 1), span(mask, H, W, ld_mask, 1))) return BZ_ERR_ALIAS;
    // a band's slot, read as an image, must meet the device calls' limits
    // (h rows of it below 2^31 bytes)
    const BandGeom g = band_geom(H, W, h, w, band, axis);
    if ((int64_t)(h + 1) * g.pitch >= ((int64_t)1 << 31)) return BZ_ERR_RANGE;
    if (g.slot_bytes > ((size_t)1 << 46)) return BZ_ERR_RANGE;
    return BZ_OK;
}

}  // namespace

extern "C" {

const char *bz_status_string(int status)
{
    switch (status) {
    case BZ_OK: return "BZ_OK";
    case BZ_ERR_INVALID: return "BZ_ERR_INVALID";
    case BZ_ERR_RANGE: return "BZ_ERR_RANGE";
    case BZ_ERR_ALIAS: return "BZ_ERR_ALIAS";
    case BZ_ERR_WORKSPACE: return "BZ_ERR_WORKSPACE";
    case BZ_ERR_HIP: return "BZ_ERR_HIP";
    default: return "BZ_UNKNOWN";
    }
}

int bz_version(void) { return 100; }

int bz_max_window(void) { return MAX_WIN; }

bz_status bz_window_sums(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                         uint32_t *S1, uint32_t *S2, ptrdiff_t ld_S, bz_stream stream)
{
    bz_status st = check_image(I, H, W, ld_I, h, w);
    if (st != BZ_OK) return st;
    if ((st = check_out(S1, H, W, ld_S, 4)) != BZ_OK) return st;
    if ((st = check_out(S2, H, W, ld_S, 4)) != BZ_OK) return st;
    const Range in = span(I, H, W, ld_I, 1), a = span(S1, H, W, ld_S, 4), b = span(S2, H, W, ld_S, 4);
    if (overlaps(in, a) || overlaps(in, b) || overlaps(a, b)) return BZ_ERR_ALIAS;
    BoxJob j = make_job(I, H, W, ld_I, h, w);
    j.mode = MODE_SUMS;
    j.S1 = S1;
    j.S2 = S2;
    j.ldS = ld_S;
    j.aligned = aligned(I, 4) && ld_I % 4 == 0 && W % 4 == 0;
    return run_box(j, (hipStream_t)stream);
}

bz_status bz_window_mean_std(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                             float *mean, float *stdv, ptrdiff_t ld_out, bz_stream stream)
{
    bz_status st = check_image(I, H, W, ld_I, h, w);
    if (st != BZ_OK) return st;
    if ((st = check_out(mean, H, W, ld_out, 4)) != BZ_OK) return st;
    if ((st = check_out(stdv, H, W, ld_out, 4)) != BZ_OK) return st;
    const Range in = span(I, H, W, ld_I, 1), a = span(mean, H, W, ld_out, 4),
                b = span(stdv, H, W, ld_out, 4);
    if (overlaps(in, a) || overlaps(in, b) || overlaps(a, b)) return BZ_ERR_ALIAS;
    BoxJob j = make_job(I, H, W, ld_I, h, w);
    j.mode = MODE_MEANSTD;
    j.mean = mean;
    j.stdv = stdv;
    j.ldMS = ld_out;
    j.aligned = aligned(I, 4) && ld_I % 4 == 0 && W % 4 == 0;
    return run_box(j, (hipStream_t)stream);
}

bz_status bz_sauvola(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, float k,
                     float R, uint8_t *mask, ptrdiff_t ld_mask, float *mean, float *stdv,
                     ptrdiff_t ld_ms, bz_stream stream)
{
    return threshold_call(MODE_SAUVOLA, I, H, W, ld_I, h, w, k, R, mask, ld_mask, mean, stdv,
                          ld_ms, stream);
}

bz_status bz_niblack(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, float k,
                     uint8_t *mask, ptrdiff_t ld_mask, float *mean, float *stdv,
                     ptrdiff_t ld_ms, bz_stream stream)
{
    return threshold_call(MODE_NIBLACK, I, H, W, ld_I, h, w, k, 1.0f, mask, ld_mask, mean, stdv,
                          ld_ms, stream);
}

static_assert(sizeof(bz_global) == sizeof(GlobalStats), "bz_global layout");
static_assert(BZ_METHOD_WOLF == T1_WOLF && BZ_METHOD_FENG == T1_FENG && BZ_METHOD_RAIS == T1_RAIS &&
                  BZ_METHOD_NICK == T1_NICK && BZ_METHOD_PHANSALKAR == T1_PHANSALKAR,
              "Table 1 rule codes");

bz_status bz_global_stats(const uint8_t *I, int H, int W, ptrdiff_t ld_I, bz_global *stats,
                          bz_stream stream)
{
    const bz_status st = check_image(I, H, W, ld_I, 1, 1);
    if (st != BZ_OK) return st;
    if (stats == nullptr || !aligned(stats, 8)) return BZ_ERR_INVALID;
    const Range g{(uintptr_t)stats, (uintptr_t)stats + sizeof(bz_global)};
    if (overlaps(span(I, H, W, ld_I, 1), g)) return BZ_ERR_ALIAS;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_global_stats(I, H, W, ld_I, (GlobalStats *)stats, (hipStream_t)stream));
}

bz_status bz_threshold(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int method,
                       const double *params, const bz_global *stats, uint8_t *mask,
                       ptrdiff_t ld_mask, float *mean, float *stdv, ptrdiff_t ld_ms,
                       bz_stream stream)
{
    int np = 0, r_at = -1;     // parameters taken; index of R (must be > 0)
    bool needs_stats = false;  // the rule reads L, M or S
    switch (method) {
    case BZ_METHOD_WOLF: np = 2; r_at = 1; needs_stats = true; break;
    case BZ_METHOD_FENG: np = 5; r_at = 4; needs_stats = true; break;
    case BZ_METHOD_RAIS: needs_stats = true; break;
    case BZ_METHOD_NICK: np = 1; break;
    case BZ_METHOD_PHANSALKAR: np = 4; r_at = 3; break;
    default: return BZ_ERR_INVALID;
    }
    double p[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (np > 0 && params == nullptr) return BZ_ERR_INVALID;
    for (int i = 0; i < np; ++i) {
        if (!isfinite(params[i])) return BZ_ERR_INVALID;
        p[i] = params[i];
    }
    if (r_at >= 0 && !(p[r_at] > 0.0)) return BZ_ERR_INVALID;
    if (needs_stats && (stats == nullptr || !aligned(stats, 8))) return BZ_ERR_INVALID;
    BoxJob j;
    const bz_status st = make_threshold_job(MODE_TABLE1, I, H, W, ld_I, h, w, 0.0f, 1.0f, mask,
                                            ld_mask, mean, stdv, ld_ms, j);
    if (st != BZ_OK) return st;
    if (needs_stats) {
        const Range g{(uintptr_t)stats, (uintptr_t)stats + sizeof(bz_global)};
        if (overlaps(g, span(mask, H, W, ld_mask, 1))) return BZ_ERR_ALIAS;
        if (mean && (overlaps(g, span(mean, H, W, ld_ms, 4)) || overlaps(g, span(stdv, H, W, ld_ms, 4))))
            return BZ_ERR_ALIAS;
    }
    j.rule = method;
    memcpy(j.tp, p, sizeof(p));
    j.gs = needs_stats ? (const GlobalStats *)stats : nullptr;
    return run_box(j, (hipStream_t)stream);
}

bz_status bz_window_quantile(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                             double q, uint8_t *Q, ptrdiff_t ld_Q, uint8_t *mask,
                             ptrdiff_t ld_mask, bz_stream stream)
{
    bz_status st = check_image(I, H, W, ld_I, h, w);
    if (st != BZ_OK) return st;
    if (!isfinite(q) || q < 0.0 || q > 1.0) return BZ_ERR_INVALID;
    if ((st = check_out(Q, H, W, ld_Q, 1)) != BZ_OK) return st;
    const Range in = span(I, H, W, ld_I, 1), rq = span(Q, H, W, ld_Q, 1);
    if (overlaps(in, rq)) return BZ_ERR_ALIAS;
    if (mask) {
        if ((st = check_out(mask, H, W, ld_mask, 1)) != BZ_OK) return st;
        const Range rm = span(mask, H, W, ld_mask, 1);
        if (overlaps(in, rm) || overlaps(rq, rm)) return BZ_ERR_ALIAS;
    }
    QuantJob j;
    memset(&j, 0, sizeof(j));
    j.I = I;
    j.ldI = ld_I;
    j.H = H;
    j.W = W;
    j.h = h;
    j.w = w;
    j.o = (h + 1) / 2;
    j.u = h / 2;
    j.l = (w + 1) / 2;
    j.r = w / 2;
    j.q = q;
    j.Q = Q;
    j.ldQ = ld_Q;
    j.mask = mask;
    j.ldM = mask ? ld_mask : 0;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_quantile(j, (hipStream_t)stream));
}

namespace {
// Validate the extremes outputs (and the mask, when given) of a min/max call.
bz_status check_minmax(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, uint8_t *mn,
                       uint8_t *mx, ptrdiff_t ld_out, uint8_t *mask, ptrdiff_t ld_mask)
{
    bz_status st = check_image(I, H, W, ld_I, h, w);
    if (st != BZ_OK) return st;
    if ((st = check_out(mn, H, W, ld_out, 1)) != BZ_OK) return st;
    if ((st = check_out(mx, H, W, ld_out, 1)) != BZ_OK) return st;
    const Range in = span(I, H, W, ld_I, 1), a = span(mn, H, W, ld_out, 1), b = span(mx, H, W, ld_out, 1);
    if (overlaps(in, a) || overlaps(in, b) || overlaps(a, b)) return BZ_ERR_ALIAS;
    if (mask) {
        if ((st = check_out(mask, H, W, ld_mask, 1)) != BZ_OK) return st;
        const Range m = span(mask, H, W, ld_mask, 1);
        if (overlaps(in, m) || overlaps(a, m) || overlaps(b, m)) return BZ_ERR_ALIAS;
    }
    return BZ_OK;
}
}  // namespace

size_t bz_extremes_workspace_size(int H, int W)
{
    if (H < 1 || W < 1) return 0;
    return extremes_workspace_bytes(H, W);
}

namespace {
bz_status extremes_call(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int cmin, uint8_t *mask,
                        ptrdiff_t ld_mask, uint8_t *mn, uint8_t *mx, ptrdiff_t ld_mm, void *workspace,
                        size_t ws_bytes, bz_stream stream)
{
    const bz_status st = check_minmax(I, H, W, ld_I, h, w, mn, mx, ld_mm, mask, ld_mask);
    if (st != BZ_OK) return st;
    if (workspace == nullptr || !aligned(workspace, 4)) return BZ_ERR_INVALID;
    if (ws_bytes < extremes_workspace_bytes(H, W)) return BZ_ERR_WORKSPACE;
    const Range ws{(uintptr_t)workspace, (uintptr_t)workspace + extremes_workspace_bytes(H, W)};
    if (overlaps(ws, span(I, H, W, ld_I, 1)) || overlaps(ws, span(mn, H, W, ld_mm, 1)) ||
        overlaps(ws, span(mx, H, W, ld_mm, 1)) || (mask && overlaps(ws, span(mask, H, W, ld_mask, 1))))
        return BZ_ERR_ALIAS;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_extremes(I, ld_I, H, W, h, w, (uint16_t *)workspace, mn, mx, ld_mm, cmin, mask,
                                      mask ? ld_mask : 0, (hipStream_t)stream));
}
}  // namespace

bz_status bz_window_minmax(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, uint8_t *mn,
                           uint8_t *mx, ptrdiff_t ld_out, void *workspace, size_t ws_bytes, bz_stream stream)
{
    return extremes_call(I, H, W, ld_I, h, w, 0, nullptr, 0, mn, mx, ld_out, workspace, ws_bytes, stream);
}

bz_status bz_bernsen(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int contrast_min,
                     uint8_t *mask, ptrdiff_t ld_mask, uint8_t *mn, uint8_t *mx, ptrdiff_t ld_mm,
                     void *workspace, size_t ws_bytes, bz_stream stream)
{
    if (mask == nullptr) return BZ_ERR_INVALID;
    if (contrast_min < 0 || contrast_min > 256) return BZ_ERR_INVALID;
    return extremes_call(I, H, W, ld_I, h, w, contrast_min, mask, ld_mask, mn, mx, ld_mm, workspace, ws_bytes,
                         stream);
}

// ---- Bernsen's rule with no allocation and no workspace argument ----
// The field of the two passes lives in a file-scope device array of fixed
// size; its device address is looked up once per device, with that device
// current, on the first call there.  In host code the array's name is not a
// device address: only the looked-up pointer is passed to kernels.
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;  // 32 MiB: 16 Mpx of 16-bit field
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];  // per device, set once
}  // namespace
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
bz_status scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return BZ_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return BZ_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BZ_OK;
}
}  // namespace

size_t bz_bernsen_noalloc_max_pixels(void) { return NOALLOC_SCRATCH_BYTES / sizeof(uint16_t); }

bz_status bz_bernsen_noalloc(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int contrast_min,
                             uint8_t *mask, ptrdiff_t ld_mask, uint8_t *mn, uint8_t *mx, ptrdiff_t ld_mm,
                             bz_stream stream)
{
    if (mask == nullptr) return BZ_ERR_INVALID;
    if (contrast_min < 0 || contrast_min > 256) return BZ_ERR_INVALID;
    const bz_status st = check_minmax(I, H, W, ld_I, h, w, mn, mx, ld_mm, mask, ld_mask);
    if (st != BZ_OK) return st;
    if (extremes_workspace_bytes(H, W) > NOALLOC_SCRATCH_BYTES) return BZ_ERR_WORKSPACE;
    void *ws = nullptr;
    const bz_status sa = scratch_address(&ws);
    if (sa != BZ_OK) return sa;
    return extremes_call(I, H, W, ld_I, h, w, contrast_min, mask, ld_mask, mn, mx, ld_mm, ws,
                         NOALLOC_SCRATCH_BYTES, stream);
}

bz_status bz_set_tile_table(const int *rows, int count)
{
    if (count < 0 || (count > 0 && rows == nullptr) || count > 4096) return BZ_ERR_INVALID;
    std::vector<TileRule> t((size_t)count);
    for (int i = 0; i < count; ++i) {
        const int *r = rows + 4 * (size_t)i;
        if (r[0] < 1 || r[1] < 1 || r[2] < 0 || r[3] < 0 || r[3] > MAX_THREADS || r[3] % 64 != 0)
            return BZ_ERR_INVALID;
        t[(size_t)i] = TileRule{r[0], r[1], r[2], r[3]};
    }
    std::stable_sort(t.begin(), t.end(), [](const TileRule &a, const TileRule &b) {
        return a.hmax != b.hmax ? a.hmax < b.hmax : a.wmax < b.wmax;
    });
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile_table.swap(t);
    return BZ_OK;
}

size_t bz_batched_workspace_size(int count)
{
    if (count < 0) return 0;
    return batch_workspace_bytes(count);
}

bz_status bz_batched_plan(const bz_item *items, int count, const int *strip_rows, void *workspace,
                          size_t ws_bytes, bz_stream stream)
{
    if (count < 1 || items == nullptr || workspace == nullptr) return BZ_ERR_INVALID;
    if (!aligned(workspace, 64)) return BZ_ERR_INVALID;
    if (ws_bytes < batch_workspace_bytes(count)) return BZ_ERR_WORKSPACE;
    std::vector<BoxJob> jobs((size_t)count);
    std::vector<int64_t> work((size_t)count);
    for (int i = 0; i < count; ++i) {
        const bz_item &it = items[i];
        int mode;
        if (it.method == BZ_METHOD_SAUVOLA) mode = MODE_SAUVOLA;
        else if (it.method == BZ_METHOD_NIBLACK) mode = MODE_NIBLACK;
        else return BZ_ERR_INVALID;
        const bz_status st = make_threshold_job(mode, it.I, it.H, it.W, it.ld_I, it.h, it.w, it.k,
                                                it.R, it.mask, it.ld_mask, it.mean, it.std,
                                                it.ld_ms, jobs[(size_t)i]);
        if (st != BZ_OK) return st;
        int strip = (strip_rows != nullptr) ? strip_rows[i] : 0;
        if (strip < 1) strip = default_batch_strip(it.h);
        plan_box(jobs[(size_t)i], strip, BATCH_THREADS);
        const BoxJob &j = jobs[(size_t)i];
        // work of one tile: rows of the strip plus its priming rows, times
        // the lanes' columns (priming rows cost about a twelfth of a row)
        work[(size_t)i] = (int64_t)(12 * j.strip + j.h) * (int64_t)std::min(j.W, COLS_PER_LANE * BATCH_THREADS);
    }
    const bz_status alias = check_batch_aliasing(items, count);
    if (alias != BZ_OK) return alias;
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return work[(size_t)x] > work[(size_t)y]; });
    std::vector<char> blob(batch_workspace_bytes(count), 0);
    BatchHeader *hdr = (BatchHeader *)blob.data();
    hdr->next_tile = 0;
    hdr->done = 0;
    hdr->count = count;
    BoxJob *dj = (BoxJob *)(hdr + 1);
    int *prefix = (int *)(dj + count);
    int64_t total = 0;
    for (int i = 0; i < count; ++i) {
        const BoxJob &j = jobs[(size_t)order[(size_t)i]];
        dj[i] = j;
        prefix[i] = (int)total;
        total += (int64_t)j.ntx * j.nsy;
        if (total > (int64_t)1 << 30) return BZ_ERR_RANGE;
    }
    prefix[count] = (int)total;
    register_batch_variant(workspace, batch_variant(dj, count));
    if (inject_launch_fault()) return BZ_ERR_HIP;
    hipError_t e = hipMemcpyAsync(workspace, blob.data(), blob.size(), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    return hip_status(e);
}

bz_status bz_batched_run(void *workspace, bz_stream stream)
{
    if (workspace == nullptr || !aligned(workspace, 64)) return BZ_ERR_INVALID;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_box_batched(workspace, (hipStream_t)stream));
}

bz_status bz_sauvola_batched(const bz_item *items, int count, void *workspace, size_t ws_bytes,
                             bz_stream stream)
{
    const bz_status st = bz_batched_plan(items, count, nullptr, workspace, ws_bytes, stream);
    if (st != BZ_OK) return st;
    return bz_batched_run(workspace, stream);
}

size_t bz_soft_workspace_size(int B, int H, int W)
{
    if (B < 1 || H < 1 || W < 1) return 0;
    return soft_workspace_bytes(B, H, W);
}

namespace {

bz_status check_soft(const float *I, int B, int H, int W, ptrdiff_t ld, int h, int w,
                     const float *k, const float *R, float tau)
{
    if (I == nullptr || k == nullptr || R == nullptr) return BZ_ERR_INVALID;
    if (B < 1 || H < 1 || W < 1 || h < 1 || w < 1 || ld < W) return BZ_ERR_INVALID;
    if (h > MAX_WIN || w > MAX_WIN) return BZ_ERR_RANGE;
    if (!isfinite(tau) || !(tau > 0.0f)) return BZ_ERR_INVALID;
    if (!aligned(I, 4)) return BZ_ERR_INVALID;
    if ((int64_t)B * H * (int64_t)ld > ((int64_t)1 << 40)) return BZ_ERR_RANGE;
    // one image (and one dense H x W field) spans under 2^31 bytes
    if ((int64_t)(H - 1) * ld + W >= ((int64_t)1 << 29)) return BZ_ERR_RANGE;
    return BZ_OK;
}

}  // namespace

bz_status bz_soft_sauvola_fwd(const float *I, int B, int H, int W, ptrdiff_t ld, int h, int w,
                              const float *k, const float *R, float tau, float *y,
                              bz_stream stream)
{
    bz_status st = check_soft(I, B, H, W, ld, h, w, k, R, tau);
    if (st != BZ_OK) return st;
    if (y == nullptr || !aligned(y, 4)) return BZ_ERR_INVALID;
    const Range in = span(I, B * H, W, ld, 4), out = span(y, B * H, W, ld, 4);
    if (overlaps(in, out)) return BZ_ERR_ALIAS;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_soft_fwd(I, B, H, W, ld, h, w, k, R, tau, y, (hipStream_t)stream));
}

bz_status bz_soft_window_sums(const float *I, int B, int H, int W, ptrdiff_t ld, int h, int w, double *S1,
                              double *S2, ptrdiff_t ld_S, bz_stream stream)
{
    if (I == nullptr || S1 == nullptr || S2 == nullptr) return BZ_ERR_INVALID;
    if (B < 1 || H < 1 || W < 1 || h < 1 || w < 1 || ld < W || ld_S < W) return BZ_ERR_INVALID;
    if (h > MAX_WIN || w > MAX_WIN) return BZ_ERR_RANGE;
    if (!aligned(I, 4) || !aligned(S1, 8) || !aligned(S2, 8)) return BZ_ERR_INVALID;
    if ((int64_t)B * H * (int64_t)ld > ((int64_t)1 << 40) || (int64_t)B * H * (int64_t)ld_S > ((int64_t)1 << 40))
        return BZ_ERR_RANGE;
    // one float32 image spans under 2^31 bytes, and so does one binary64 output image
    if ((int64_t)(H - 1) * ld + W >= ((int64_t)1 << 29) || (int64_t)(H - 1) * ld_S + W >= ((int64_t)1 << 28))
        return BZ_ERR_RANGE;
    const Range in = span(I, B * H, W, ld, 4), a = span(S1, B * H, W, ld_S, 8), b = span(S2, B * H, W, ld_S, 8);
    if (overlaps(in, a) || overlaps(in, b) || overlaps(a, b)) return BZ_ERR_ALIAS;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_soft_sums(I, B, H, W, ld, h, w, S1, S2, ld_S, (hipStream_t)stream));
}

bz_status bz_soft_sauvola_bwd(const float *I, const float *gy, int B, int H, int W, ptrdiff_t ld,
                              int h, int w, const float *k, const float *R, float tau,
                              float *gI, float *gk, float *gR, void *workspace, size_t ws_bytes,
                              bz_stream stream)
{
    bz_status st = check_soft(I, B, H, W, ld, h, w, k, R, tau);
    if (st != BZ_OK) return st;
    if (gy == nullptr || gI == nullptr || gk == nullptr || gR == nullptr || workspace == nullptr)
        return BZ_ERR_INVALID;
    if (!aligned(gy, 4) || !aligned(gI, 4) || !aligned(gk, 4) || !aligned(gR, 4) ||
        !aligned(workspace, 256))
        return BZ_ERR_INVALID;
    if (ws_bytes < soft_workspace_bytes(B, H, W)) return BZ_ERR_WORKSPACE;
    const Range in = span(I, B * H, W, ld, 4), g = span(gy, B * H, W, ld, 4),
                out = span(gI, B * H, W, ld, 4), wsr = span(workspace, 1, (int)0, 0, 1);
    const Range wsr2{(uintptr_t)workspace, (uintptr_t)workspace + ws_bytes};
    (void)wsr;
    if (overlaps(in, out) || overlaps(g, out) || overlaps(wsr2, in) || overlaps(wsr2, g) ||
        overlaps(wsr2, out))
        return BZ_ERR_ALIAS;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_soft_bwd(I, gy, B, H, W, ld, h, w, k, R, tau, gI, gk, gR, workspace,
                                      (hipStream_t)stream));
}

size_t bz_stream_workspace_size(int H, int W, int h, int w, int band, int axis)
{
    if (H < 1 || W < 1 || h < 1 || w < 1 || h > MAX_WIN || w > MAX_WIN || band < 1) return 0;
    if (axis != BZ_AXIS_AUTO && axis != BZ_AXIS_ROWS && axis != BZ_AXIS_COLUMNS) return 0;
    return 4 * band_geom(H, W, h, w, band, axis).slot_bytes;
}

bz_status bz_binarize_streamed(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w, int method,
                               float k, float R, uint8_t *mask, ptrdiff_t ld_mask, int band, int axis,
                               void *workspace, size_t ws_bytes, bz_stream stream, bz_stream load_stream,
                               bz_stream store_stream)
{
    bz_status st = stream_check(I, H, W, ld_I, h, w, method, k, R, mask, ld_mask, band, axis);
    if (st != BZ_OK) return st;
    const BandGeom g = band_geom(H, W, h, w, band, axis);
    if (workspace == nullptr || !aligned(workspace, 256)) return BZ_ERR_INVALID;
    if (ws_bytes < 4 * g.slot_bytes) return BZ_ERR_WORKSPACE;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    const int mode = method == BZ_METHOD_SAUVOLA ? MODE_SAUVOLA : MODE_NIBLACK;
    hipStream_t cs = (hipStream_t)stream, ls = (hipStream_t)load_stream, ss = (hipStream_t)store_stream;
    uint8_t *slot[4];
    for (int i = 0; i < 4; ++i) slot[i] = (uint8_t *)workspace + (size_t)i * g.slot_bytes;
    // per slot: loaded (its input is in), freed (no longer read), computed
    // (its output is in), stored (its output is no longer read)
    hipEvent_t ev[4][2] = {};
    hipEvent_t(&loaded)[2] = ev[0], (&freed)[2] = ev[1], (&computed)[2] = ev[2], (&stored)[2] = ev[3];
    hipError_t e = hipSuccess;
    for (int i = 0; i < 8 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i / 2][i % 2], hipEventDisableTiming);
    // band arithmetic in 64 bits: Y + B + after may pass 2^31 near the size limit
    const int nb = (int)(((int64_t)g.len + g.band - 1) / g.band);
    auto first = [&](int j) { return (int)std::max<int64_t>((int64_t)j * g.band - g.before, 0); };  // A of band j
    auto last = [&](int j) {                                                                       // E of band j
        return (int)std::min<int64_t>((int64_t)j * g.band + g.band + g.after, g.len);
    };
    for (int j = 0; j < nb && e == hipSuccess && st == BZ_OK; ++j) {
        const int Y = (int)((int64_t)j * g.band), B = std::min(g.band, g.len - Y), s = j & 1;
        const int A = first(j), E = last(j);
        const int N0 = j == 0 ? A : last(j - 1);  // first line read from the host
        uint8_t *in = slot[s], *out = slot[2 + s];
        // load the new lines once band j-2's kernel and band j-1's carry have
        // read slot s; the lines a band shares with band j-1 arrive by the carry
        if (j >= 2) e = hipStreamWaitEvent(ls, freed[s], 0);
        if (e == hipSuccess)
            e = copy_lines(g, band_line(in, g, N0 - A, g.pitch), g.pitch, band_line(I, g, N0, ld_I), ld_I, E - N0,
                           hipMemcpyHostToDevice, ls);
        if (e == hipSuccess) e = hipEventRecord(loaded[s], ls);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, loaded[s], 0);
        if (e == hipSuccess && j >= 2) e = hipStreamWaitEvent(cs, stored[s], 0);
        if (e != hipSuccess) break;
        BoxJob job;
        const int Hb = g.rows ? E - A : H, Wb = g.rows ? W : E - A;
        st = make_threshold_job(mode, in, Hb, Wb, g.pitch, h, w, k, R, out, g.pitch, nullptr, nullptr, 0, job);
        if (st == BZ_OK) st = run_box(job, cs);
        if (st != BZ_OK) break;
        // the halo band j+1 shares with this band, into the other slot (its
        // previous reader, band j-1's kernel, precedes on this stream)
        if (j + 1 < nb)
            e = copy_lines(g, slot[s ^ 1], g.pitch, band_line(in, g, first(j + 1) - A, g.pitch), g.pitch,
                           E - first(j + 1), hipMemcpyDeviceToDevice, cs);
        if (e == hipSuccess) e = hipEventRecord(freed[s], cs);
        if (e == hipSuccess) e = hipEventRecord(computed[s], cs);
        if (e == hipSuccess) e = hipStreamWaitEvent(ss, computed[s], 0);
        if (e == hipSuccess)
            e = copy_lines(g, band_line(mask, g, Y, ld_mask), ld_mask, band_line(out, g, Y - A, g.pitch), g.pitch, B,
                           hipMemcpyDeviceToHost, ss);
        if (e == hipSuccess) e = hipEventRecord(stored[s], ss);
    }
    // the call returns with the host outputs complete
    const hipError_t e1 = hipStreamSynchronize(cs), e2 = hipStreamSynchronize(ls), e3 = hipStreamSynchronize(ss);
    for (int i = 0; i < 8; ++i)
        if (ev[i / 2][i % 2]) (void)hipEventDestroy(ev[i / 2][i % 2]);
    if (st != BZ_OK) return st;
    return (e != hipSuccess || e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) ? BZ_ERR_HIP : BZ_OK;
}
namespace {
// Cell grid and negative cells (bit m * kh + n) of a template; false if unknown.
bool haar_template(int kind, int &kv, int &kh, uint32_t &neg)
{
    switch (kind) {
    case BZ_HAAR_EDGE_H: kv = 1, kh = 2, neg = 2u; return true;
    case BZ_HAAR_EDGE_V: kv = 2, kh = 1, neg = 2u; return true;
    case BZ_HAAR_LINE_H: kv = 1, kh = 3, neg = 2u; return true;
    case BZ_HAAR_LINE_V: kv = 3, kh = 1, neg = 2u; return true;
    case BZ_HAAR_CHECKER: kv = 2, kh = 2, neg = 6u; return true;
    default: return false;
    }
}
}  // namespace

size_t bz_haar_workspace_size(int H, int W, int a, int kind)
{
    int kv, kh;
    uint32_t neg;
    if (H < 1 || W < 1 || a < 1 || a > H || !haar_template(kind, kv, kh, neg)) return 0;
    return haar_workspace_bytes(H, W, a, kv);
}

bz_status bz_haar_features(const uint8_t *I, int H, int W, ptrdiff_t ld_I, int a, int b, int kind, int32_t *F,
                           ptrdiff_t ld_F, void *workspace, size_t ws_bytes, bz_stream stream)
{
    if (I == nullptr || F == nullptr) return BZ_ERR_INVALID;
    if (H < 1 || W < 1 || a < 1 || b < 1 || ld_I < W) return BZ_ERR_INVALID;
    if (a > MAX_WIN || b > MAX_WIN) return BZ_ERR_RANGE;
    int kv, kh;
    uint32_t neg;  // bit m * kh + n: cell (m, n) negative
    if (!haar_template(kind, kv, kh, neg)) return BZ_ERR_INVALID;
    if ((int64_t)kv * a > H || (int64_t)kh * b > W) return BZ_ERR_INVALID;  // the template must fit
    const int Hf = H - kv * a + 1, Wf = W - kh * b + 1;
    bz_status st = check_out(F, Hf, Wf, ld_F, 4);
    if (st != BZ_OK) return st;
    if ((int64_t)H * (int64_t)ld_I > ((int64_t)1 << 46)) return BZ_ERR_RANGE;
    // each launch's grid, in threads, must stay below 2^32
    const int64_t Hv = H - a + 1, lim = (int64_t)1 << 32;
    if (Hv * HAAR_BLOCK >= lim || ((int64_t)W + HAAR_BLOCK - 1) / HAAR_BLOCK * ((Hv + HAAR_ROWS - 1) / HAAR_ROWS) *
                                          HAAR_BLOCK >= lim ||
        ((int64_t)Wf + HAAR_BLOCK - 1) / HAAR_BLOCK * Hf * HAAR_BLOCK >= lim)
        return BZ_ERR_RANGE;
    if (workspace == nullptr || !aligned(workspace, 256)) return BZ_ERR_INVALID;
    const size_t need = haar_workspace_bytes(H, W, a, kv);
    if (ws_bytes < need) return BZ_ERR_WORKSPACE;
    const Range in = span(I, H, W, ld_I, 1), out = span(F, Hf, Wf, ld_F, 4);
    const Range ws{(uintptr_t)workspace, (uintptr_t)workspace + need};
    if (overlaps(in, out) || overlaps(ws, in) || overlaps(ws, out)) return BZ_ERR_ALIAS;
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_haar(I, ld_I, H, W, a, b, kv, kh, neg, workspace, F, ld_F, (hipStream_t)stream));
}

}  // extern "C"
