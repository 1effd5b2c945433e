// Windowed quantiles from sliding 256-bin gray-level histograms (Section 3.4).
//
// Each wavefront works on its own tile; lane t owns output column x0 + t and
// slides its window histogram DOWN a strip of rows: per row it adds the w
// gray levels of the entering row and removes those of the leaving row (the
// Theta(max{h,w}) per-pixel cost the paper states).
//
// Histograms are private per lane and live in a 64 KB LDS array of 256 bin
// rows of 64 words, the bin as the major dimension: a lane's bin v is in row
// v at its slot, so each lane always hits its own bank.  When no count can
// exceed 65535 (h w <= 65535) the bins are 16 bits and two lanes share a
// slot: a workgroup holds two wavefronts, lane t of wave u has slot
// 32 u + (t mod 32) and the half t / 32 of it (four waves per CU); otherwise a
// workgroup is one wavefront and lane t has all of slot t (two per CU).  A
// bin's byte offset, 256 v + 4 slot, is then one byte permute of the gray
// level and the slot, and its increment (1 or 65536) a constant of the lane.
// Bin updates are fire-and-forget LDS atomics.
//
// Row data: the wave loads the bytes its 64 windows need from a row (at most
// 64 + w - 1 of them) as aligned dwords, one or two per lane, prefetched a
// row ahead; a lane takes its bytes four at a time from the lanes holding
// them (ds_bpermute) with a byte funnel shift.
//
// The quantile is tracked incrementally: the lane keeps its current answer Q
// and lt = #{window values < Q}, adjusts lt as values enter and leave, then
// walks Q down or up until lt < rho <= lt + hist[Q].
#include "device.hpp"
#include "internal.hpp"

#include <math.h>
#include <stdlib.h>

namespace bz {
namespace {

constexpr int QLANES = 64;

// The bytes of one row the wave needs, [cs, cs + nb), held as aligned dwords
// from the dword containing byte cs: lane t holds dwords t and 64 + t.
// sh = offset of byte cs in its dword.  Bytes past the row read as zero or
// as the next row's (never used: lanes only take bytes of their windows).
template <bool TWO>
struct RowBytes {
    uint32_t d0 = 0, d1 = 0;
    int sh = 0;
    __device__ __forceinline__ void load(const uint8_t *rowp, int nb, int lane)
    {
        const uintptr_t p = (uintptr_t)rowp;
        const uint8_t *ap = (const uint8_t *)(p & ~(uintptr_t)3);
        sh = (int)(p & 3);
        // whole dwords only: a dword crossing the descriptor end reads zero,
        // and the aligned dword holding the last byte is readable memory
        const uint32_t bytes = (uint32_t)((sh + nb + 3) & ~3);
        const __amdgpu_buffer_rsrc_t d = rsrc(ap, bytes);
        d0 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(d, 4 * lane, 0, 0);
        d1 = TWO ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(d, 4 * lane + 256, 0, 0) : 0u;
    }
    // dword i (0 <= i < 128) of the row's span
    __device__ __forceinline__ uint32_t dword(int i) const
    {
        const int a = (i & 63) << 2;
        const uint32_t v0 = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)d0);
        if (!TWO) return v0;
        const uint32_t v1 = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)d1);
        return i < 64 ? v0 : v1;
    }
};

// A lane's place in the histogram array: its slot's byte offset in a bin row
// (s4 = 4 slot, at most 252), the increment of one count (1, or 65536 for the
// high half of a shared slot) and the shift of its half.
struct Slot {
    uint32_t s4, inc, sh;
};

// The count of a bin from its word.
template <bool PACK>
__device__ __forceinline__ int bin_of(uint32_t wd, const Slot &slot)
{
    return PACK ? (int)((wd >> slot.sh) & 0xffffu) : (int)wd;
}

// Byte offset of the bin of byte q of val in the lane's histogram,
// 256 byte + s4 (one permute: byte 0 from s4, byte 1 from val), and the
// signed increment of its count.
template <int q, int SIGN>
__device__ __forceinline__ void bin_slot(uint32_t val, const Slot &slot, uint32_t &off, uint32_t &inc)
{
    off = __builtin_amdgcn_perm(slot.s4, val, 0x0c0c0004u | ((uint32_t)q << 8));
    inc = SIGN > 0 ? slot.inc : 0u - slot.inc;
}

// Adds inc (already signed) to the word at byte offset off.
__device__ __forceinline__ void lds_add(uint32_t *hist, uint32_t off, uint32_t inc)
{
    atomicAdd((uint32_t *)((char *)hist + off), inc);
}

// Number of the four bytes of val that are >= Q, in two 8-bit fields (bits
// 8..15 and 24..31): with K = 0x01000100 - Q (0x00010001), each 16-bit half
// of (byte + K) carries into its bit 8 exactly when byte >= Q.
__device__ __forceinline__ uint32_t ge_fields(uint32_t val, uint32_t K)
{
    const uint32_t ev = val & 0x00ff00ffu;
    const uint32_t od = __builtin_amdgcn_perm(0u, val, 0x0c030c01u);  // bytes 1, 3 into 0, 2
    return ((ev + K) & 0x01000100u) + ((od + K) & 0x01000100u);
}

constexpr int GROUP = 8;  // dwords of row bytes per group (32 window columns)

// Byte q of the entering (ve) and leaving (vl) dwords at window column c0 + q.
template <bool PACK, bool FULL, bool BOTH, int LSIGN, int q>
__device__ __forceinline__ void group_bytes(uint32_t *hist, const Slot &slot, uint32_t ve, uint32_t vl, bool has_e,
                                            bool has_l, int c0, int wmax, int nc, int Q, int &lt)
{
    const int c = c0 + q;
    const bool ok = FULL || (c < wmax && c < nc);
    uint32_t off, inc;
    bin_slot<q, 1>(ve, slot, off, inc);
    const bool oke = FULL || (ok && has_e);
    lds_add(hist, off, oke ? inc : 0u);
    if (BOTH) {
        const bool okl = FULL || (ok && has_l);
        bin_slot<q, LSIGN>(vl, slot, off, inc);
        lds_add(hist, off, okl ? inc : 0u);
        if (!FULL && LSIGN < 0) {
            const uint32_t v_e = (ve >> (8 * q)) & 0xffu, v_l = (vl >> (8 * q)) & 0xffu;
            lt += (int)(oke && v_e < (uint32_t)Q) - (int)(okl && v_l < (uint32_t)Q);
        }
    }
}

// The updates of one group: the window columns kbase .. kbase + 4 GROUP - 1
// of the lane, from GROUP + 1 dwords of each row span (funnel-shifted by the
// span's byte offset).  FULL: every column is inside every lane's window and
// both rows exist, so no byte needs a check, and lt is updated from the
// group's byte counts; otherwise each byte is checked (a byte outside adds
// zero) and compared.  BOTH false: only e is added, to the first window,
// built with Q = 0 (no value lies below it).  LSIGN +1: l is added too (two
// rows of the first window per round trip; lt stays 0).
template <bool PACK, bool FULL, bool BOTH, int LSIGN>
__device__ __forceinline__ void group_update(uint32_t *hist, const Slot &slot, const uint32_t *de, const uint32_t *dl,
                                             int se, int sl, bool has_e, bool has_l, int kbase, int wmax, int nc,
                                             int Q, int &lt)
{
    const uint32_t K = 0x01000100u - (uint32_t)Q * 0x00010001u;
    uint32_t ge_e = 0, ge_l = 0;
#pragma unroll
    for (int t = 0; t < GROUP; ++t) {
        const uint32_t ve = __builtin_amdgcn_alignbyte(de[t + 1], de[t], se);
        const uint32_t vl = BOTH ? __builtin_amdgcn_alignbyte(dl[t + 1], dl[t], sl) : 0u;
        if (FULL && BOTH && LSIGN < 0) {
            ge_e += ge_fields(ve, K);
            ge_l += ge_fields(vl, K);
        }
        group_bytes<PACK, FULL, BOTH, LSIGN, 0>(hist, slot, ve, vl, has_e, has_l, kbase + 4 * t, wmax, nc, Q, lt);
        group_bytes<PACK, FULL, BOTH, LSIGN, 1>(hist, slot, ve, vl, has_e, has_l, kbase + 4 * t, wmax, nc, Q, lt);
        group_bytes<PACK, FULL, BOTH, LSIGN, 2>(hist, slot, ve, vl, has_e, has_l, kbase + 4 * t, wmax, nc, Q, lt);
        group_bytes<PACK, FULL, BOTH, LSIGN, 3>(hist, slot, ve, vl, has_e, has_l, kbase + 4 * t, wmax, nc, Q, lt);
    }
    if (FULL && BOTH && LSIGN < 0) {
        // bytes below Q: entering minus leaving = (32 - ge_e) - (32 - ge_l)
        lt += (int)(((ge_l >> 8) & 0xffu) + (ge_l >> 24)) - (int)(((ge_e >> 8) & 0xffu) + (ge_e >> 24));
    }
}

// The row step of the lane's histogram: the bytes [rel, rel + nc) of the
// entering row span e are added and those of the leaving row span l
// removed (has_e / has_l false: that row lies outside the image).  All
// ds_bpermutes of a group are issued together, so the LDS round trips are
// per group, not per dword.  clip: some lane's window is clipped by the
// image border (nc < w).  BOTH false: only e is added (the first window);
// LSIGN +1: e and l are both added (two rows of the first window).
template <bool PACK, bool TWO, bool BOTH, int LSIGN = -1>
__device__ __forceinline__ void slide_rows(uint32_t *hist, const Slot &slot, const RowBytes<TWO> &e, const RowBytes<TWO> &l, bool has_e,
                                           bool has_l, int rel, int nc, int wmax, bool clip, int Q, int &lt)
{
    const int be = e.sh + rel, bl = l.sh + rel;
    const int se = be & 3, sl = bl & 3;
    const int ie = be >> 2, il = bl >> 2;
    const bool fast = has_e && (has_l || !BOTH) && !clip;
    for (int k = 0; k < wmax; k += 4 * GROUP) {
        // dword indices past the lane's bytes wrap or read the other half:
        // those bytes are never counted
        uint32_t de[GROUP + 1], dl[GROUP + 1];
#pragma unroll
        for (int t = 0; t <= GROUP; ++t) {
            de[t] = e.dword(ie + k / 4 + t);
            dl[t] = BOTH ? l.dword(il + k / 4 + t) : 0u;
        }
        if (fast && k + 4 * GROUP <= wmax)
            group_update<PACK, true, BOTH, LSIGN>(hist, slot, de, dl, se, sl, has_e, has_l, k, wmax, nc, Q, lt);
        else
            group_update<PACK, false, BOTH, LSIGN>(hist, slot, de, dl, se, sl, has_e, has_l, k, wmax, nc, Q, lt);
    }
}

// Four rows of the first window per round trip: the bytes of rows a, b, c
// and d are fetched before any of their atomics (every row exists).
template <bool PACK, bool TWO>
__device__ __forceinline__ void build_rows4(uint32_t *hist, const Slot &slot, const RowBytes<TWO> &a,
                                            const RowBytes<TWO> &b, const RowBytes<TWO> &c, const RowBytes<TWO> &d,
                                            int rel, int nc, int wmax, bool clip, int Q, int &lt)
{
    const int ba = a.sh + rel, bb = b.sh + rel, bc = c.sh + rel, bd = d.sh + rel;
    for (int k = 0; k < wmax; k += 4 * GROUP) {
        uint32_t da[GROUP + 1], db[GROUP + 1], dc[GROUP + 1], dd[GROUP + 1];
#pragma unroll
        for (int t = 0; t <= GROUP; ++t) {
            da[t] = a.dword((ba >> 2) + k / 4 + t);
            db[t] = b.dword((bb >> 2) + k / 4 + t);
            dc[t] = c.dword((bc >> 2) + k / 4 + t);
            dd[t] = d.dword((bd >> 2) + k / 4 + t);
        }
        if (!clip && k + 4 * GROUP <= wmax) {
            group_update<PACK, true, true, 1>(hist, slot, da, db, ba & 3, bb & 3, true, true, k, wmax, nc, Q, lt);
            group_update<PACK, true, true, 1>(hist, slot, dc, dd, bc & 3, bd & 3, true, true, k, wmax, nc, Q, lt);
        } else {
            group_update<PACK, false, true, 1>(hist, slot, da, db, ba & 3, bb & 3, true, true, k, wmax, nc, Q, lt);
            group_update<PACK, false, true, 1>(hist, slot, dc, dd, bc & 3, bd & 3, true, true, k, wmax, nc, Q, lt);
        }
    }
}

// Walk Q to the rho-th smallest window value: down while lt >= rho, up while
// lt + hist[Q] < rho (Q stays in [0, 255] whatever the counts hold).  The
// common case, Q unchanged, costs one LDS read; otherwise each round trip
// reads WALK_WORDS bins, issued together, so that a quantile that jumps
// across an edge costs a few round trips instead of one per bin.  hb: the
// lane's slot in bin row 0.
constexpr int WALK_WORDS = 8;
template <bool PACK>
__device__ __forceinline__ void walk(const uint32_t *hb, const Slot &slot, int rho, int &Q, int &lt)
{
    if (lt < rho && (Q >= 255 || lt + bin_of<PACK>(hb[Q * QLANES], slot) >= rho)) return;
    // each step below is a select, so the lanes of a chunk stay converged
    while (lt >= rho && Q > 0) {
        // bins Q-1 and the WALK_WORDS-1 below it (from 0 at the bottom)
        const int base = Q - WALK_WORDS > 0 ? Q - WALK_WORDS : 0;
        uint32_t wd[WALK_WORDS];
#pragma unroll
        for (int t = 0; t < WALK_WORDS; ++t) wd[t] = hb[(base + t) * QLANES];
#pragma unroll
        for (int t = WALK_WORDS - 1; t >= 0; --t) {
            const int g = base + t;
            const bool step = g == Q - 1 && lt >= rho;
            lt = step ? lt - bin_of<PACK>(wd[t], slot) : lt;
            Q = step ? g : Q;
        }
    }
    bool found = Q >= 255;
    while (!found) {
        // bin Q and the WALK_WORDS-1 above it (base < Q only at the top,
        // where bins below Q are skipped and the walk stops at bin 255)
        const int base = Q < 256 - WALK_WORDS ? Q : 256 - WALK_WORDS;
        uint32_t wd[WALK_WORDS];
#pragma unroll
        for (int t = 0; t < WALK_WORDS; ++t) wd[t] = hb[(base + t) * QLANES];
        const int q0 = Q;
#pragma unroll
        for (int t = 0; t < WALK_WORDS; ++t) {
            const int g = base + t;
            const int cnt = bin_of<PACK>(wd[t], slot);
            const bool live = !found && g >= q0;
            const bool hit = live && (g >= 255 || lt + cnt >= rho);
            lt = (live && !hit) ? lt + cnt : lt;
            Q = hit ? g : Q;
            found = found || hit;
        }
        Q = found ? Q : base + WALK_WORDS;
    }
}

// Software-pipelined row step for windows of at most 4 PGROUP columns.  The
// walk of row y reads the histogram after row y's atomics; an LDS read waits
// for every earlier LDS operation of the wave, so the atomics are followed
// by VALU work that needs no LDS: decoding row y+1 (from bytes fetched
// before the atomics) into LDS offsets and increments.
constexpr int PGROUP = 8;
struct PipeRow {
    uint32_t off[2][4 * PGROUP], inc[2][4 * PGROUP];  // [entering, leaving] updates
    uint32_t raw[2][PGROUP];                          // their bytes (255 where not counted)
    bool full;  // every update counts: inc unused, the lane's constant increments apply
};

// The row span dwords of a lane's window bytes: GROUP + 1 per row; se, sl:
// the byte offsets of the first window byte in its dword.
template <bool TWO>
__device__ __forceinline__ void fetch_rows(uint32_t *de, uint32_t *dl, int &se, int &sl, const RowBytes<TWO> &e,
                                           const RowBytes<TWO> &l, int rel)
{
    const int be = e.sh + rel, bl = l.sh + rel;
    se = be & 3;
    sl = bl & 3;
#pragma unroll
    for (int t = 0; t <= PGROUP; ++t) {
        de[t] = e.dword((be >> 2) + t);
        dl[t] = l.dword((bl >> 2) + t);
    }
}

template <bool PACK, bool FULL, int q>
__device__ __forceinline__ void decode_byte(PipeRow &S, int t, uint32_t ve, uint32_t vl, uint32_t me, uint32_t ml,
                                            const Slot &slot)
{
    uint32_t off, inc;
    bin_slot<q, 1>(ve, slot, off, inc);
    S.off[0][4 * t + q] = off;
    if (!FULL) S.inc[0][4 * t + q] = ((me >> (8 * q)) & 1u) == 0u ? inc : 0u;
    bin_slot<q, -1>(vl, slot, off, inc);
    S.off[1][4 * t + q] = off;
    if (!FULL) S.inc[1][4 * t + q] = ((ml >> (8 * q)) & 1u) == 0u ? inc : 0u;
}

// Offsets and increments of a row's updates.  FULL: all 4 PGROUP columns are
// in every lane's window and both rows exist; otherwise a byte outside the
// lane's window (or of a missing row) gets increment 0 and reads as 255,
// which no rank count takes as below Q.
template <bool PACK, bool FULL>
__device__ __forceinline__ void decode_rows(PipeRow &S, const uint32_t *de, const uint32_t *dl, int se, int sl,
                                            bool has_e, bool has_l, int wmax, int nc, const Slot &slot)
{
    S.full = FULL;
#pragma unroll
    for (int t = 0; t < PGROUP; ++t) {
        uint32_t ve = __builtin_amdgcn_alignbyte(de[t + 1], de[t], se);
        uint32_t vl = __builtin_amdgcn_alignbyte(dl[t + 1], dl[t], sl);
        uint32_t me = 0, ml = 0;
        if (!FULL) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 4 * t + q;
                const bool ok = c < wmax && c < nc;
                me |= (ok && has_e) ? 0u : (0xffu << (8 * q));
                ml |= (ok && has_l) ? 0u : (0xffu << (8 * q));
            }
            ve |= me;
            vl |= ml;
        }
        S.raw[0][t] = ve;
        S.raw[1][t] = vl;
        decode_byte<PACK, FULL, 0>(S, t, ve, vl, me, ml, slot);
        decode_byte<PACK, FULL, 1>(S, t, ve, vl, me, ml, slot);
        decode_byte<PACK, FULL, 2>(S, t, ve, vl, me, ml, slot);
        decode_byte<PACK, FULL, 3>(S, t, ve, vl, me, ml, slot);
    }
}

__device__ __forceinline__ void apply_rows(uint32_t *hist, const PipeRow &S, const Slot &slot)
{
    if (S.full) {
        const uint32_t ie = slot.inc, il = 0u - slot.inc;
#pragma unroll
        for (int i = 0; i < 4 * PGROUP; ++i) {
            lds_add(hist, S.off[0][i], ie);
            lds_add(hist, S.off[1][i], il);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4 * PGROUP; ++i) {
            lds_add(hist, S.off[0][i], S.inc[0][i]);
            lds_add(hist, S.off[1][i], S.inc[1][i]);
        }
    }
}

// lt += (entering bytes below Q) - (leaving bytes below Q); bytes not
// counted read 255 in both rows.
__device__ __forceinline__ void count_below(const PipeRow &S, int Q, int &lt)
{
    const uint32_t K = 0x01000100u - (uint32_t)Q * 0x00010001u;
    uint32_t ge_e = 0, ge_l = 0;
#pragma unroll
    for (int t = 0; t < PGROUP; ++t) {
        ge_e += ge_fields(S.raw[0][t], K);
        ge_l += ge_fields(S.raw[1][t], K);
    }
    lt += (int)(((ge_l >> 8) & 0xffu) + (ge_l >> 24)) - (int)(((ge_e >> 8) & 0xffu) + (ge_e >> 24));
}

// Wavefronts of a workgroup: two sharing the slots of 16-bit bins, or one.
template <bool PACK>
constexpr int qwaves() { return PACK ? 2 : 1; }

// Workgroup b: wavefront u works on tile qwaves() * b + u (in XCD order) of
// the ntiles = ntx * nsy tiles, with no barrier between the wavefronts.
template <bool PACK, bool TWO>
__global__ __launch_bounds__(qwaves<PACK>() * QLANES) void k_quantile(QuantJob a, int seg, int nsy, int ntiles)
{
    __shared__ uint32_t hist[256 * QLANES];  // 256 bin rows of 64 slots (64 KB)
    const int lane = threadIdx.x & (QLANES - 1);
    const int u = PACK ? (int)(threadIdx.x >> 6) : 0;
    const int L = qwaves<PACK>() * xcd_remap(blockIdx.x, gridDim.x) + u;
    if (L >= ntiles) return;  // the second wavefront of the last workgroup
    const int tx = L / nsy;
    const int sy = L - tx * nsy;
    const int x0 = tx * QLANES;
    const int j = x0 + lane;
    const bool active = j < a.W;
    const int y0 = sy * seg;
    const int y1 = min(y0 + seg, a.H);
    const int H = a.H, W = a.W;

    const uint32_t sidx = PACK ? 32u * (uint32_t)u + (uint32_t)(lane & 31) : (uint32_t)lane;
    Slot slot;
    slot.s4 = 4u * sidx;
    slot.inc = (PACK && lane >= 32) ? 65536u : 1u;
    slot.sh = (PACK && lane >= 32) ? 16u : 0u;
    uint32_t *hb = hist + sidx;
    // clear the lane's bins (a shared slot by its low-half lane, before any
    // update: one wavefront's LDS operations take effect in order)
    if (!PACK || lane < 32) {
#pragma unroll 8
        for (int b = 0; b < 256; ++b) hb[b * QLANES] = 0u;
    }

    // bytes any lane of the wave needs: columns cs .. ce
    const int cs = max(x0 - a.l + 1, 0);
    const int ce = min(x0 + QLANES - 1 + a.r, W - 1);
    const int nb = ce - cs + 1;
    // clipped window columns of this lane, relative to cs
    const int c0 = max(j - a.l + 1, 0);
    const int c1 = active ? min(j + a.r, W - 1) : c0 - 1;
    const int nc = max(c1 - c0 + 1, 0);
    const int rel = c0 - cs;
    const int wmax = a.w;
    // some window of the wave clipped by the image border (wave-uniform)
    const bool clip = __builtin_amdgcn_ballot_w64(nc < wmax) != 0;

    auto rowp = [&](int row) { return a.I + (int64_t)row * a.ldI + cs; };

    int Q = 0;   // current answer
    int lt = 0;  // number of window values below Q
    // histogram of the window of row y0.  Windows wider than 32 columns take
    // four rows per pass (the bytes of all four are fetched before any of
    // their atomics), narrower ones two (four measured slower there); the
    // next rows are loaded ahead, and the last one to three rows go in a
    // pair and singly
    {
        const int r0 = max(y0 - a.o + 1, 0), r1 = min(y0 + a.u, H - 1);
        const bool quads = wmax > 4 * PGROUP;  // wave-uniform
        RowBytes<TWO> ra, rb, rc, rd;
        if (r0 <= r1) ra.load(rowp(r0), nb, lane);
        if (r0 + 1 <= r1) rb.load(rowp(r0 + 1), nb, lane);
        if (quads && r0 + 2 <= r1) rc.load(rowp(r0 + 2), nb, lane);
        if (quads && r0 + 3 <= r1) rd.load(rowp(r0 + 3), nb, lane);
        int row = r0;
        if (quads) {
            for (; row + 3 <= r1; row += 4) {
                const RowBytes<TWO> ca = ra, cb = rb, cc = rc, cd = rd;
                if (row + 4 <= r1) ra.load(rowp(row + 4), nb, lane);
                if (row + 5 <= r1) rb.load(rowp(row + 5), nb, lane);
                if (row + 6 <= r1) rc.load(rowp(row + 6), nb, lane);
                if (row + 7 <= r1) rd.load(rowp(row + 7), nb, lane);
                build_rows4<PACK, TWO>(hist, slot, ca, cb, cc, cd, rel, nc, wmax, clip, Q, lt);
            }
            // rows row .. r1 (at most three) are in ra, rb, rc
            if (row + 1 <= r1) {
                slide_rows<PACK, TWO, true, 1>(hist, slot, ra, rb, true, true, rel, nc, wmax, clip, Q, lt);
                if (row + 2 <= r1)
                    slide_rows<PACK, TWO, false>(hist, slot, rc, rc, true, false, rel, nc, wmax, clip, Q, lt);
            } else if (row <= r1) {
                slide_rows<PACK, TWO, false>(hist, slot, ra, ra, true, false, rel, nc, wmax, clip, Q, lt);
            }
        } else {
            for (; row <= r1; row += 2) {
                const RowBytes<TWO> ca = ra, cb = rb;
                if (row + 2 <= r1) ra.load(rowp(row + 2), nb, lane);
                if (row + 3 <= r1) rb.load(rowp(row + 3), nb, lane);
                if (row + 1 <= r1)
                    slide_rows<PACK, TWO, true, 1>(hist, slot, ca, cb, true, true, rel, nc, wmax, clip, Q, lt);
                else
                    slide_rows<PACK, TWO, false>(hist, slot, ca, ca, true, false, rel, nc, wmax, clip, Q, lt);
            }
        }
    }

    auto pixel = [&](int y) {  // the lane's own pixel of row y (for the mask)
        const __amdgpu_buffer_rsrc_t d = rsrc(a.I + (int64_t)y * a.ldI + x0, (uint32_t)(W - x0));
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(d, lane, 0, 0);
    };
    auto finish = [&](int y, uint32_t iv) {  // walk to row y's quantile and store it
        if (!active) return;
        const int nr = min(y + a.u, H - 1) - max(y - a.o, -1);
        const int n = nr * nc;  // at most 257 * 257
        int rho = (int)ceil(a.q * (double)n);
        if (rho < 1) rho = 1;
        walk<PACK>(hb, slot, rho, Q, lt);
        a.Q[(int64_t)y * a.ldQ + j] = (uint8_t)Q;
        if (a.mask) a.mask[(int64_t)y * a.ldM + j] = (iv < (uint32_t)Q) ? 1 : 0;
    };

    if (!TWO && wmax <= 4 * PGROUP) {
        // rows entering and leaving the window of row y (y + u and y - o)
        // and the pixels: A holds row y+1's, B row y+2's (two rows ahead)
        RowBytes<TWO> eA, lA, eB, lB;
        uint32_t pxA = 0, pxB = 0;
        auto load_rows = [&](int y, RowBytes<TWO> &e, RowBytes<TWO> &l) {
            if (y + a.u < H) e.load(rowp(y + a.u), nb, lane);
            if (y - a.o >= 0) l.load(rowp(y - a.o), nb, lane);
        };
        uint32_t px = pixel(y0);
        if (y0 + 1 < y1) {
            load_rows(y0 + 1, eA, lA);
            pxA = pixel(y0 + 1);
        }
        if (y0 + 2 < y1) {
            load_rows(y0 + 2, eB, lB);
            pxB = pixel(y0 + 2);
        }
        PipeRow S;
        uint32_t de[PGROUP + 1], dl[PGROUP + 1];
        for (int y = y0; y < y1; ++y) {
            if (y > y0) count_below(S, Q, lt);  // S: row y's updates
            const int yn = y + 1;
            if (yn < y1) {
                int se, sl;
                fetch_rows(de, dl, se, sl, eA, lA, rel);  // before this row's atomics
                if (y > y0) apply_rows(hist, S, slot);
                const bool has_e = yn + a.u < H, has_l = yn - a.o >= 0;
                if (has_e && has_l && !clip && wmax == 4 * PGROUP)
                    decode_rows<PACK, true>(S, de, dl, se, sl, has_e, has_l, wmax, nc, slot);
                else
                    decode_rows<PACK, false>(S, de, dl, se, sl, has_e, has_l, wmax, nc, slot);
            } else if (y > y0) {
                apply_rows(hist, S, slot);
            }
            const uint32_t iv = px;
            // advance the load pipeline: A <- B, B <- row y + 3
            px = pxA;
            eA = eB;
            lA = lB;
            pxA = pxB;
            if (y + 3 < y1) {
                load_rows(y + 3, eB, lB);
                pxB = pixel(y + 3);
            }
            finish(y, iv);
        }
        return;
    }

    // rows entering and leaving the window of row y: y + u and y - o; with
    // them the lane's own pixel of row y (for the mask), one row ahead
    RowBytes<TWO> ne, nl;
    uint32_t npx = 0;
    auto load_row = [&](int y) {
        if (y > y0) {
            if (y + a.u < H) ne.load(rowp(y + a.u), nb, lane);
            if (y - a.o >= 0) nl.load(rowp(y - a.o), nb, lane);
        }
        npx = pixel(y);
    };
    load_row(y0);
    for (int y = y0; y < y1; ++y) {
        const RowBytes<TWO> e = ne, l = nl;
        const uint32_t iv = npx;
        if (y + 1 < y1) load_row(y + 1);
        if (y > y0) {
            const bool has_e = y + a.u < H, has_l = y - a.o >= 0;
            slide_rows<PACK, TWO, true>(hist, slot, e, l, has_e, has_l, rel, nc, wmax, clip, Q, lt);
        }
        finish(y, iv);
    }
}

template <bool PACK, bool TWO>
void launch_variant(const QuantJob &a, int ntiles, int seg, int nsy, hipStream_t stream)
{
    constexpr int nw = qwaves<PACK>();
    hipLaunchKernelGGL((k_quantile<PACK, TWO>), dim3((ntiles + nw - 1) / nw), dim3(nw * QLANES), 0, stream, a, seg,
                       nsy, ntiles);
}

}  // namespace

// Workgroups of `lds` bytes of LDS that stay resident on the device at
// once.  Measured on MI355X: four 32 KB workgroups fit on a CU but not five
// (five fit at 31 KB), so the usable LDS per CU is taken as 158 KB.
static int resident_groups(size_t lds)
{
    int device = 0, cus = 0;
    if (hipGetDevice(&device) != hipSuccess) device = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    const int per_cu = (int)((160u * 1024u - 2048u) / lds);
    return cus * (per_cu > 0 ? per_cu : 1);
}

hipError_t launch_quantile(const QuantJob &a, hipStream_t stream)
{
    const int ntx = (a.W + QLANES - 1) / QLANES;
    const bool pack = (int64_t)a.h * a.w <= 65535;
    // strips: one resident round of waves (a wave more would run in a
    // second round), and at least h/2 rows (building the first window
    // costs h w updates against 2 w per row of the slide)
    const long target = (long)resident_groups(256 * QLANES * sizeof(uint32_t)) * (pack ? 2 : 1);
    int seg = (int)(((long)a.H * ntx + target - 1) / target);
    if (seg < (a.h + 1) / 2) seg = (a.h + 1) / 2;
    if (seg < 8) seg = 8;
    const char *e = getenv("BZ_QUANTILE_STRIP");  // tuning override
    if (e && atoi(e) > 0) seg = atoi(e);
    if (seg > a.H) seg = a.H;
    const int nsy = (a.H + seg - 1) / seg;
    // dwords a lane reads from the row span: from (sh + rel) / 4 <= 16 to
    // 16 + (w - 1) / 4 + 1; one dword per lane holds dwords 0 .. 63
    const bool two = 16 + (a.w - 1) / 4 + 1 >= QLANES;
    const int ntiles = ntx * nsy;
    if (pack) {
        if (two) launch_variant<true, true>(a, ntiles, seg, nsy, stream);
        else launch_variant<true, false>(a, ntiles, seg, nsy, stream);
    } else {
        if (two) launch_variant<false, true>(a, ntiles, seg, nsy, stream);
        else launch_variant<false, false>(a, ntiles, seg, nsy, stream);
    }
    return hipGetLastError();
}

}  // namespace bz
