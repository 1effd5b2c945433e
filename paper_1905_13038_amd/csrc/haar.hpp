// Host-side entry of the Haar-like feature kernels (haar.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bz {

constexpr int HAAR_BLOCK = 256;  // threads per workgroup of every Haar kernel
constexpr int HAAR_ROWS = 32;    // rows of the vertical sums per workgroup

// Row stride, in elements, of the vertical-sum field for W columns.
int64_t haar_ld(int W);
// Workspace bytes for a template of kv rows of cells: H - a + 1 rows of
// haar_ld(W) uint16 column sums, and as many uint32 row prefixes when the kv
// prefixes of a row do not fit the row kernel's LDS.
size_t haar_workspace_bytes(int H, int W, int a, int kv);
// Launch shape of the fused single-launch form (k_haar_fused): dwords of
// columns per lane, outputs per tile, tiles, strip height and strips.
struct HaarPlan {
    int Hf, Wf, ndw, step, ntx, S, nsy;
};
// The fused form's plan, or false where it does not apply (unaligned rows, a
// template wider than 256 columns or with other signs); in the environment,
// BZ_HAAR_FUSED=0 turns it off and BZ_HAAR_NDW and BZ_HAAR_STRIP override its
// tile width and strip height.
bool haar_fused_plan(const uint8_t *I, int64_t ldI, int H, int W, int a, int b, int kv, int kh, uint32_t neg,
                     HaarPlan &p);
// Features of a kv x kh template of a x b cells (bit m * kh + n of neg set for
// a negative cell) into F, (H - kv a + 1) x (W - kh b + 1) at row stride ldF.
hipError_t launch_haar(const uint8_t *I, int64_t ldI, int H, int W, int a, int b, int kv, int kh, uint32_t neg,
                       void *ws, int32_t *F, int64_t ldF, hipStream_t stream);

}  // namespace bz
