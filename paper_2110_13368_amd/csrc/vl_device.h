// vl_device.h -- device helpers shared by the sweep and adjoint kernels:
// tile lookup, Dirichlet face selection, raw buffer access and the unrolled
// loops over a half line held in VGPRs.  Internal.
#pragma once

#include "vl_internal.h"

namespace vl {

// Workgroup b runs on XCD b % 8; give each XCD a contiguous range of tiles so
// that tiles sharing cache lines meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    const int x = bid & 7, q = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return (x < rem) ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
}

// Largest k in [0, count) with prefix[k] <= tile.
__device__ __forceinline__ int find_slot(const int *__restrict__ prefix, int count, int tile)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Highest-numbered face whose bit is set in both masks, -1 if none.
__device__ __forceinline__ int top_face(int mask)
{
    return mask ? 31 - __builtin_clz(mask) : -1;
}

__device__ __forceinline__ float face_value(const float (&d)[6], int f)
{
    float v = d[0];
    v = (f == 1) ? d[1] : v;
    v = (f == 2) ? d[2] : v;
    v = (f == 3) ? d[3] : v;
    v = (f == 4) ? d[4] : v;
    v = (f == 5) ? d[5] : v;
    return v;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw buffer access: the lane part of an offset stays in a VGPR, the
// wave-uniform row part goes in an SGPR, so walking a line costs no vector
// address arithmetic.  Offsets are in bytes from the resource base.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float *base, long long elems)
{
    const long long bytes = elems * 4;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), 0,
                                             (int)min(bytes, (long long)0x7fffffff), 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, soff, 0);
}
// The same with a cache policy (the instruction's aux bits): kNonTemporal
// marks streaming accesses whose lines will not be touched again soon.
constexpr int kNonTemporal = 2;
template <int POL>
__device__ __forceinline__ float bload_p(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, POL));
}
template <int POL>
__device__ __forceinline__ void bstore_p(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, soff, POL);
}
typedef unsigned vl_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned vl_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, float4 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(vl_u32x4, v), r, (int)voff, soff, 0);
}

// Runs BODY for t = 0..CAP-1 with t < cnt, cnt wave-uniform: whole groups
// of 8 without per-element tests.  Written as macros so that every register
// index is a constant after unrolling (the array must never leave VGPRs).
#define VL_FOR_UP(CAP_, cnt, t, BODY)                                                  \
    _Pragma("unroll") for (int g_ = 0; g_ < (CAP_); g_ += 8)                           \
    {                                                                                  \
        if (g_ + 8 <= (cnt)) {                                                         \
            _Pragma("unroll") for (int j_ = 0; j_ < 8; ++j_)                           \
            {                                                                          \
                const int t = g_ + j_;                                                 \
                if (t < (CAP_)) { BODY }                                               \
            }                                                                          \
        } else if (g_ < (cnt)) {                                                       \
            _Pragma("unroll") for (int j_ = 0; j_ < 8; ++j_)                           \
            {                                                                          \
                const int t = g_ + j_;                                                 \
                if (t < (CAP_) && t < (cnt)) { BODY }                                  \
            }                                                                          \
        }                                                                              \
    }
// Same, t descending.
#define VL_FOR_DOWN(CAP_, cnt, t, BODY)                                                \
    _Pragma("unroll") for (int g_ = ((CAP_) + 7) / 8 * 8 - 8; g_ >= 0; g_ -= 8)        \
    {                                                                                  \
        if (g_ + 8 <= (cnt)) {                                                         \
            _Pragma("unroll") for (int j_ = 7; j_ >= 0; --j_)                          \
            {                                                                          \
                const int t = g_ + j_;                                                 \
                if (t < (CAP_)) { BODY }                                               \
            }                                                                          \
        } else if (g_ < (cnt)) {                                                       \
            _Pragma("unroll") for (int j_ = 7; j_ >= 0; --j_)                          \
            {                                                                          \
                const int t = g_ + j_;                                                 \
                if (t < (CAP_) && t < (cnt)) { BODY }                                  \
            }                                                                          \
        }                                                                              \
    }

// LDS of one tile.  The x sweep needs a 64x64 staging block per wave (rows
// padded to 65 floats, or 16 blocks of 4 rows padded to 260 floats: the same
// size); the others only the exchange slots and the pivot table.  The
// forward sweeps keep both in FP64 (their recurrences run in FP64), the
// adjoint's reverse solves in FP32.
template <int CAP, bool XSTAGE, typename PIV = double2, typename XCH = double, int SX = 65>
struct TileLds {
    XCH xch[2][kWave];
    PIV piv[CAP];
    __attribute__((aligned(16))) float stage[XSTAGE ? 2 * 64 * SX : 1];
};

// Chunks of the forward split x sweep's stage: a wave holds at most CAP
// columns of its 64 rows, so lines of up to 65 voxels (CAP 32) move 32
// columns at a time through a 64 x 33 block per wave, half the LDS of the
// 64 x 65 block the longer lines use (which lets twice as many workgroups
// share a CU).
template <int CAP>
struct XStage {
    static constexpr int W = CAP <= 32 ? 32 : 64;  // columns per chunk
    static constexpr int SX = W + 1;                // row stride in floats (odd: no bank conflicts)
};
template <int CAP, bool XSTAGE>
using FwdLds = TileLds<CAP, XSTAGE, double2, double, XStage<CAP>::SX>;

// ---------------------------------------------------------------------------
// x lines with 16-byte transfers (long lines, CAP >= 160).  A 64-row x
// 64-column chunk of the tile moves with 16 LDS-DMA instructions of 1 KB
// (lane i: row 4k + i/16, one group of 4 columns) and 16 stores of 1 KB.
// In the stage, block k holds rows 4k..4k+3 (64 floats each, block stride
// 260 floats); row q's column group g sits in 16-byte slot (g + 4(q%4)) % 16.
// With that rotation a lane's 16-byte read of 4 columns of its own row hits
// distinct banks across any 16 consecutive lanes, and the DMA / store side
// moves contiguous 16-byte slots.  Fewer VGPRs than the 4-byte path, so the
// long-line classes run two waves per SIMD.
constexpr int kXBlk = 260;
template <int CAP>
struct XWide {
    static constexpr bool value = CAP >= 160;
};

// Loads this wave's half lines into v (top: columns 0..nel-1 in order; bottom:
// columns n-1 downwards).  For CAP >= 64 every needed chunk starts at a
// column >= 0 and ends at <= n-1, so only the top wave's unneeded groups past
// n-4 are clamped.
// Position in the stage of row q's column c of the chunk (0 <= c < 64).
__device__ __forceinline__ int x_wide_slot(int q, int c)
{
    return (q >> 2) * kXBlk + (q & 3) * 64 + 4 * (((c >> 2) + 4 * (q & 3)) & 15) + (c & 3);
}

// on_chunk(c, cbase) runs once per chunk after the chunk has landed in the
// stage and before it is read back (the cell sources carried into the x
// solve are applied there).
template <int CAP, typename F>
__device__ __forceinline__ void x_load_wide(float (&v)[CAP], __amdgpu_buffer_rsrc_t rs, float *stw, bool top,
                                            int n, int nel, int row_b, int xrows_left, int lane, F &&on_chunk)
{
    constexpr int kChunks = (CAP + 63) / 64;
    const int rb = lane >> 4;
    const int gq = ((lane & 15) - 4 * rb) & 15;
    const float *rowp = stw + (lane >> 2) * kXBlk + (lane & 3) * 64;
    const int rot = 4 * (lane & 3);
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        if (c * 64 < nel) {
            const int cbase = top ? c * 64 : n - 64 * (c + 1);
            const int col = top ? min(cbase + 4 * gq, n - 4) : cbase + 4 * gq;
            // the previous chunk's stage reads complete before the DMA reuses
            // the stage (LDS-DMA writes are not ordered after earlier LDS reads)
            if (c > 0) __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
            for (int k = 0; k < 16; ++k)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (__attribute__((address_space(3))) void *)(stw + k * kXBlk), 16,
                    min(4 * k + rb, xrows_left - 1) * row_b + col * 4, 0, 0, 0);
            __builtin_amdgcn_s_waitcnt(0);
            wave_sync_lds();
            on_chunk(c, cbase);
#pragma unroll
            for (int h = 0; h < 16; ++h) {
                if (c * 64 + 4 * h < CAP && c * 64 + 4 * h < nel) {
                    const int gh = top ? h : 15 - h;
                    const float4 q4 = *reinterpret_cast<const float4 *>(rowp + 4 * ((gh + rot) & 15));
                    const float e4[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (c * 64 + 4 * h + e < CAP) v[c * 64 + 4 * h + e] = top ? e4[e] : e4[3 - e];
                }
            }
            wave_sync_lds();
        }
    }
}

// Stores this wave's half lines from v (the middle row is stored by the
// caller).  Column groups wholly owned by the wave go out as 16-byte stores;
// the one group per row that straddles the wave's first/last owned column is
// written element by element by the lane that owns the row.
template <int CAP>
__device__ __forceinline__ void x_store_wide(const float (&v)[CAP], __amdgpu_buffer_rsrc_t rs, float *stw, bool top,
                                             int n, int nel, int row_b, int xrows_left, int lane, unsigned lane_b,
                                             bool line_ok)
{
    constexpr int kChunks = (CAP + 63) / 64;
    const int rb = lane >> 4;
    const int gq = ((lane & 15) - 4 * rb) & 15;
    float *rowp = stw + (lane >> 2) * kXBlk + (lane & 3) * 64;
    const int rot = 4 * (lane & 3);
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        if (c * 64 < nel) {
#pragma unroll
            for (int h = 0; h < 16; ++h) {
                if (c * 64 + 4 * h < CAP && c * 64 + 4 * h < nel) {
                    const int gh = top ? h : 15 - h;
                    float e4[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int idx = c * 64 + 4 * h + (top ? e : 3 - e);
                        e4[e] = (idx < CAP) ? v[idx < CAP ? idx : 0] : 0.f;
                    }
                    *reinterpret_cast<float4 *>(rowp + 4 * ((gh + rot) & 15)) =
                        make_float4(e4[0], e4[1], e4[2], e4[3]);
                }
            }
            wave_sync_lds();
            const int own = nel - c * 64;  // columns of this chunk the wave owns
            const int cbase = top ? c * 64 : n - 64 * (c + 1);
            const bool full = top ? (4 * gq + 3 < own) : (4 * gq >= 64 - own);
            const unsigned col4 = (unsigned)(cbase + 4 * gq) * 4u;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (full && 4 * k + rb < xrows_left)
                    bstore4(rs, col4, (4 * k + rb) * row_b, *reinterpret_cast<const float4 *>(stw + k * kXBlk + 4 * lane));
            if (own < 64) {
                const int first = top ? 0 : 64 - own;  // owned chunk columns [first, last)
                const int last = top ? own : 64;
                const int gp = first == 0 ? (own >> 2) : (first >> 2);
                const bool partial = top ? (own & 3) != 0 : (first & 3) != 0;
                if (partial && line_ok) {
                    const float *src = rowp + 4 * ((gp + rot) & 15);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int tc = 4 * gp + e;
                        if (tc >= first && tc < last) bstore(rs, lane_b + (unsigned)(cbase + tc) * 4u, 0, src[e]);
                    }
                }
            }
            wave_sync_lds();
        }
    }
}

}  // namespace vl
