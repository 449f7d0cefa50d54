// vl_copy.hip -- a plain device copy, the practical bandwidth ceiling that
// the sweeps are measured against.  Each sweep reads and writes every element
// once, so a copy of the same bytes is the fastest a sweep can be on this
// memory system; the variants here (4-, 8- or 16-byte accesses per lane,
// ordinary or non-temporal loads and stores) show which access shapes reach
// it.  With the destination equal to the source the buffer is rewritten in
// place, which is how the sweeps move their field (each element read and
// written back where it lies).  Also the kernel of known traffic (bytes read
// = bytes written = size) that scales the HBM byte counters.
#include "vl_internal.h"

namespace vl {

namespace {

typedef unsigned cp_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned cp_u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;  // accesses in flight per thread

template <typename T, bool NTL, bool NTS>
__global__ void __launch_bounds__(kCopyThreads)
copy_probe_kernel(const T *__restrict__ src, T *__restrict__ dst, size_t n)
{
    const size_t base = (size_t)blockIdx.x * (kCopyThreads * kCopyUnroll) + threadIdx.x;
    T r[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + (size_t)u * kCopyThreads;
        if (i < n) r[u] = NTL ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + (size_t)u * kCopyThreads;
        if (i < n) {
            if (NTS)
                __builtin_nontemporal_store(r[u], dst + i);
            else
                dst[i] = r[u];
        }
    }
}

// In place: every element read and then written back unchanged by the same
// thread (no restrict: source and destination are one buffer).
template <typename T, bool NTL, bool NTS>
__global__ void __launch_bounds__(kCopyThreads) rewrite_probe_kernel(T *buf, size_t n)
{
    const size_t base = (size_t)blockIdx.x * (kCopyThreads * kCopyUnroll) + threadIdx.x;
    T r[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + (size_t)u * kCopyThreads;
        if (i < n) r[u] = NTL ? __builtin_nontemporal_load(buf + i) : buf[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + (size_t)u * kCopyThreads;
        if (i < n) {
            if (NTS)
                __builtin_nontemporal_store(r[u], buf + i);
            else
                buf[i] = r[u];
        }
    }
}

// Tiles of kTileThreads x kTileItems 16-byte values (64 KiB) per workgroup,
// each read whole into registers before any of it is written: the access
// shape of a sweep tile, which loads its lines, solves, then stores them.
// Source and destination may be the same buffer (each thread writes back
// only what it read).
constexpr int kTileThreads = 256;
constexpr int kTileItems = 16;

__global__ void __launch_bounds__(kTileThreads) tile_probe_kernel(const cp_u32x4 *src, cp_u32x4 *dst, size_t n)
{
    const size_t base = (size_t)blockIdx.x * (kTileThreads * kTileItems) + threadIdx.x;
    cp_u32x4 r[kTileItems];
#pragma unroll
    for (int u = 0; u < kTileItems; ++u) {
        const size_t i = base + (size_t)u * kTileThreads;
        if (i < n) r[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kTileItems; ++u) {
        const size_t i = base + (size_t)u * kTileThreads;
        if (i < n) dst[i] = r[u];
    }
}

template <typename T>
hipError_t launch_typed(const void *src, void *dst, size_t bytes, int nt, hipStream_t st)
{
    const size_t n = bytes / sizeof(T);
    const size_t per = (size_t)kCopyThreads * kCopyUnroll;
    const dim3 grid((unsigned)((n + per - 1) / per)), block(kCopyThreads);
    const T *s = (const T *)src;
    T *d = (T *)dst;
    if (src == dst) {
        switch (nt & 3) {
        case 0: hipLaunchKernelGGL((rewrite_probe_kernel<T, false, false>), grid, block, 0, st, d, n); break;
        case 1: hipLaunchKernelGGL((rewrite_probe_kernel<T, true, false>), grid, block, 0, st, d, n); break;
        case 2: hipLaunchKernelGGL((rewrite_probe_kernel<T, false, true>), grid, block, 0, st, d, n); break;
        default: hipLaunchKernelGGL((rewrite_probe_kernel<T, true, true>), grid, block, 0, st, d, n); break;
        }
        return hipGetLastError();
    }
    switch (nt & 3) {
    case 0: hipLaunchKernelGGL((copy_probe_kernel<T, false, false>), grid, block, 0, st, s, d, n); break;
    case 1: hipLaunchKernelGGL((copy_probe_kernel<T, true, false>), grid, block, 0, st, s, d, n); break;
    case 2: hipLaunchKernelGGL((copy_probe_kernel<T, false, true>), grid, block, 0, st, s, d, n); break;
    default: hipLaunchKernelGGL((copy_probe_kernel<T, true, true>), grid, block, 0, st, s, d, n); break;
    }
    return hipGetLastError();
}

}  // namespace

// width: bytes per lane access (4, 8 or 16); nt: bit 0 non-temporal loads,
// bit 1 non-temporal stores, or 4 for 64 KiB tiles loaded whole before they
// are stored (width 16); src == dst rewrites the buffer in place.  bytes is a multiple of 16 and below 2^32 *
// (kCopyThreads * kCopyUnroll) * width (checked by the caller).
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, int width, int nt, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    if (nt == 4) {
        const size_t n = bytes / 16;
        const size_t per = (size_t)kTileThreads * kTileItems;
        hipLaunchKernelGGL(tile_probe_kernel, dim3((unsigned)((n + per - 1) / per)), dim3(kTileThreads), 0, st,
                           (const cp_u32x4 *)src, (cp_u32x4 *)dst, n);
        return hipGetLastError();
    }
    if (width == 4) return launch_typed<unsigned>(src, dst, bytes, nt, st);
    if (width == 8) return launch_typed<cp_u32x2>(src, dst, bytes, nt, st);
    return launch_typed<cp_u32x4>(src, dst, bytes, nt, st);
}

}  // namespace vl
