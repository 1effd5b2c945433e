// Device helpers shared by the kernels of libbinarize: raw buffer
// descriptors, the XCD-aware workgroup order and the DPP wavefront scan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bz {

// Raw buffer resources (base, num_records in bytes, stride 0).  Accesses at
// offsets at or beyond num_records read zero and drop stores in hardware, so
// image borders, out-of-image rows and lanes outside a tile need no per-lane
// branch or select.  The last descriptor word is the raw-buffer format value
// for gfx9-family chips.
constexpr int RSRC_FLAGS = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, RSRC_FLAGS);
}

// Workgroup b of n is placed on XCD (b mod 8).  The logical index returned
// gives every XCD a contiguous range of logical tiles, so that data shared by
// neighbouring tiles (the halo rows of vertically adjacent strips) stays in
// that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, i = b >> 3;
    return (x < rem) ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v)
{
    // lanes without a DPP source (or in rows masked off) read 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes of a wavefront (Hillis-Steele within
// rows of 16 lanes, then the row_bcast steps that carry row totals forward).
__device__ __forceinline__ uint32_t wave_scan(uint32_t v)
{
    v += dpp_or_zero<0x111, 0xf>(v);  // row_shr:1
    v += dpp_or_zero<0x112, 0xf>(v);  // row_shr:2
    v += dpp_or_zero<0x114, 0xf>(v);  // row_shr:4
    v += dpp_or_zero<0x118, 0xf>(v);  // row_shr:8
    v += dpp_or_zero<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v += dpp_or_zero<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

// Inclusive prefix sum over the first 16 lanes (row 0).
__device__ __forceinline__ uint32_t row_scan16(uint32_t v)
{
    v += dpp_or_zero<0x111, 0xf>(v);
    v += dpp_or_zero<0x112, 0xf>(v);
    v += dpp_or_zero<0x114, 0xf>(v);
    v += dpp_or_zero<0x118, 0xf>(v);
    return v;
}

}  // namespace bz
