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

// LDS of one tile.  The x sweep needs the 64x65 staging block per wave; the
// others only the exchange slots and the pivot table.
template <int CAP, bool XSTAGE>
struct TileLds {
    float xch[2][kWave];
    float2 piv[CAP];
    float stage[XSTAGE ? 2 * 64 * 65 : 1];
};

}  // namespace vl
