// Internal declarations shared by the HIP translation units of libbinarize.
// Not part of the public C ABI (include/binarize.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bz {

// What the box-statistics kernel writes.
enum Mode : int {
    MODE_SUMS = 0,     // S1, S2 (uint32)
    MODE_MEANSTD = 1,  // m, s (float)
    MODE_SAUVOLA = 2,  // mask (+ optional m, s)
    MODE_NIBLACK = 3,  // mask (+ optional m, s)
    MODE_TABLE1 = 4    // mask by one of Table 1's other rules, decided in binary64
                       // (+ optional m, s)
};

// Table 1 rules of MODE_TABLE1 (the codes of the C ABI's bz_method).
enum Table1 : int { T1_WOLF = 3, T1_FENG = 4, T1_RAIS = 5, T1_NICK = 6, T1_PHANSALKAR = 7 };

// Global statistics of one image (layout of the C ABI's bz_global): exact
// integer sums, then the mean and population standard deviation in binary64.
struct GlobalStats {
    uint64_t n, sum, sumsq;
    uint32_t min, max;
    double mean, stdev;
};
static_assert(sizeof(GlobalStats) == 48, "bz_global layout");

// Columns owned by one lane in the box kernels (one dword of pixels).
constexpr int COLS_PER_LANE = 4;
// Largest block: 16 waves of 64 lanes.
constexpr int MAX_THREADS = 1024;
constexpr int MAX_WAVES = MAX_THREADS / 64;

// Per-image description of one box-statistics job, with its tiling.
struct BoxJob {
    const uint8_t *I;
    int64_t ldI;
    int H, W, h, w;
    int o, u, l, r;        // window extents (Algorithm 1)
    // outputs (unused ones are null)
    uint32_t *S1, *S2;
    int64_t ldS;
    float *mean, *stdv;
    int64_t ldMS;
    uint8_t *mask;
    int64_t ldM;
    // threshold parameters: float fast path and binary64 canonical path
    float c0, c1;          // Sauvola: 1 - k, k / R; Niblack: unused, c1 = k
    float kabs;            // |k| (Niblack guard)
    double k64, R64;
    int mode;
    // tiling: column tiles of tile_w outputs, row strips of `strip` rows
    int threads;           // block size (multiple of 64, <= 1024)
    int tile_w, ntx, halo_l;
    int strip, nsy;
    int aligned;           // all pointers/strides allow vector access
    int force_ref;         // decide every pixel with the binary64 sequence (testing)
    // MODE_TABLE1: the rule, its parameters and the image's global statistics
    // (device record; null for rules that use none)
    int rule;
    double tp[5];
    const GlobalStats *gs;
};

// Fill o,u,l,r and the tiling of `job` (threads, tile_w, ntx, halo_l, strip,
// nsy) for a stand-alone launch.  `strip_override` > 0 forces the strip
// height; `threads_override` > 0 forces the block size.
void plan_box(BoxJob &job, int strip_override, int threads_override);

// Enqueue the box-statistics kernel for one planned job.
hipError_t launch_box(const BoxJob &job, hipStream_t stream);

// LDS words one box tile uses with NT threads.
int box_lds_words(int NT);

// Ragged batches: one persistent launch over the tiles of many images.
// Workspace layout: BatchHeader, BoxJob jobs[count], int prefix[count + 1]
// (prefix[i] = first tile of job i, prefix[count] = total tiles).
constexpr int BATCH_THREADS = 256;
struct alignas(64) BatchHeader {
    unsigned int next_tile;  // tile counter (zero between launches)
    unsigned int done;       // finished workgroups (zero between launches)
    int count;               // number of jobs
    int pad[13];
};
size_t batch_workspace_bytes(int count);
// Kernel variant shared by all jobs (0..7: Niblack*4 + aligned*2 + mean/std),
// or -1 for a mixed batch.
int batch_variant(const BoxJob *jobs, int count);
// Remember the variant of a planned workspace; the launch picks the kernel
// from it (a workspace never registered runs the mixed-batch kernel).
void register_batch_variant(const void *workspace, int variant);
hipError_t launch_box_batched(void *workspace, hipStream_t stream);
int batch_grid(int variant);

// Global statistics of an image into a device record (three launches: reset,
// accumulate, finish).
hipError_t launch_global_stats(const uint8_t *I, int H, int W, int64_t ld, GlobalStats *out,
                               hipStream_t stream);

// Window extremes (two separable passes through a 16-bit H x W field V in
// caller memory), and Bernsen's decision when mask is not null.
size_t extremes_workspace_bytes(int H, int W);
hipError_t launch_extremes(const uint8_t *I, int64_t ldI, int H, int W, int h, int w, uint16_t *V, uint8_t *mn,
                           uint8_t *mx, int64_t ldE, int cmin, uint8_t *mask, int64_t ldM, hipStream_t stream);

// Windowed quantile (Section 3.4).
struct QuantJob {
    const uint8_t *I;
    int64_t ldI;
    int H, W, h, w;
    int o, u, l, r;
    double q;
    uint8_t *Q;
    int64_t ldQ;
    uint8_t *mask;
    int64_t ldM;
};
hipError_t launch_quantile(const QuantJob &job, hipStream_t stream);

// Differentiable Sauvola (binary64 window sums over float32 images).
size_t soft_workspace_bytes(int B, int H, int W);
hipError_t launch_soft_fwd(const float *I, int B, int H, int W, int64_t ld, int h, int w,
                           const float *k, const float *R, float tau, float *y, hipStream_t st);
// The binary64 window sums of the soft kernels (export for tests).
hipError_t launch_soft_sums(const float *I, int B, int H, int W, int64_t ld, int h, int w, double *S1,
                            double *S2, int64_t ldS, hipStream_t st);
hipError_t launch_soft_bwd(const float *I, const float *gy, int B, int H, int W, int64_t ld, int h,
                           int w, const float *k, const float *R, float tau, float *gI, float *gk,
                           float *gR, void *ws, hipStream_t st);

}  // namespace bz
