// C ABI of libbinarize: argument validation, aliasing checks and dispatch to
// the HIP kernels.  Everything here runs on the host; validation finishes
// before the first HIP call, so invalid calls have no device side effects.
#include "../../include/binarize.h"
#include "internal.hpp"

#include <math.h>
#include <stdlib.h>
#include <string.h>

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
    j.rh = 1.0f / (float)h;
    return j;
}

int env_int(const char *name)
{
    const char *e = getenv(name);
    return e ? atoi(e) : 0;
}

bz_status run_box(BoxJob &j, hipStream_t stream)
{
    plan_box(j, env_int("BZ_TILE_S"), env_int("BZ_TILE_THREADS"));
    // Test hook: BZ_FORCE_REFERENCE=1 decides every pixel with the binary64
    // reference sequence instead of only those inside the float32 guard.
    j.force_ref = env_int("BZ_FORCE_REFERENCE");
    if (inject_launch_fault()) return BZ_ERR_HIP;
    return hip_status(launch_box(j, stream));
}

// Threshold entry shared by Sauvola and Niblack.
bz_status threshold_call(int mode, const uint8_t *I, int H, int W, ptrdiff_t ld_I, int h, int w,
                         float k, float R, uint8_t *mask, ptrdiff_t ld_mask, float *mean,
                         float *stdv, ptrdiff_t ld_ms, bz_stream stream)
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
    BoxJob j = make_job(I, H, W, ld_I, h, w);
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
    j.aligned = aligned(I, 4) && ld_I % 4 == 0 && aligned(mask, 4) && ld_mask % 4 == 0 &&
                (mean == nullptr || (aligned(mean, 16) && aligned(stdv, 16) && ld_ms % 4 == 0));
    return run_box(j, (hipStream_t)stream);
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
    j.aligned = aligned(I, 4) && ld_I % 4 == 0 && aligned(S1, 16) && aligned(S2, 16) && ld_S % 4 == 0;
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
    j.aligned = aligned(I, 4) && ld_I % 4 == 0 && aligned(mean, 16) && aligned(stdv, 16) &&
                ld_out % 4 == 0;
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

}  // extern "C"
