// vl_kernels.hip -- coefficient precompute, the plain FP64 path, cell binning,
// cell sources and diagnostics for gfx950.
//
// arXiv:2110.13368: Eq. (1) defines the model; section "Elements of
// Parallelism" keeps the field and the auxiliary arrays resident on the
// device, solves direction by direction with elimination/back-substitution and
// applies Dirichlet conditions in a function of their own; section "Future
// Work" names cell secretion/uptake as the next part to move onto the device.
#include "vl_internal.h"

namespace vl {

// ---------------------------------------------------------------------------
// a1: line-solve coefficients, FP64 recurrences, one thread per (volume, axis).
//
// Line matrix tridiag(-c, b, -c) with zero-flux ends: b_end = 1 + c + sigma,
// b_in = 1 + 2c + sigma, and 1 + sigma for a one-voxel line.
//  * full-line table (FP64 plain path): d_0 = b_0, d_i = b_i - c^2/d_{i-1};
//    entries (1/d_i, c/d_i), i < n.
//  * half-line table (split solve of the FP32 path): pivots from one end,
//    d_0 = b_end, d_t = b_in - c^2/d_{t-1}, t < cb = n - 1 - m with
//    m = (n-1)/2; entries (f/d_t, c/d_t) where f is the decay factor folded
//    into the x solve.  Stored twice: in FP64 for the forward sweeps, whose
//    recurrences run in FP64, and in FP32 for the adjoint's reverse solves.
//    Middle row m: gamma = b_m - c^2/d_{m-1} [m>0] - c^2/d_{cb-1} [cb>0],
//    x_m = r_m f/gamma + (c/gamma) (y_{m-1} + z_{m+1}).
__global__ void coefficients_kernel(SubDev *subs, int nsubs, float2 *coef32, double2 *coefh, double2 *coef64)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nsubs * 3) return;
    SubDev &S = subs[id / 3];
    const int a = id % 3;
    const int n = S.n[a];
    const double c = S.c[a];
    const double sg = S.sigma;
    const double f = (a == 0) ? S.fdec : 1.0;
    const double b_in = 1.0 + 2.0 * c + sg;
    const double b_end = (n == 1) ? 1.0 + sg : 1.0 + c + sg;

    if (coef64) {
        double2 *t64 = coef64 + S.coef64[a];
        double d = b_end;
        for (int i = 0; i < n; ++i) {
            if (i > 0) d = ((i == n - 1) ? b_end : b_in) - c * c / d;
            t64[i] = make_double2(1.0 / d, c / d);
        }
    }
    if (coef32) {
        float2 *t32 = coef32 + S.coef32[a];
        double2 *th = coefh ? coefh + S.coef32[a] : nullptr;
        const int m = (n - 1) / 2;
        const int cb = n - 1 - m;
        double d = b_end, d_m1 = 0.0, d_cb1 = 0.0;
        for (int t = 0; t < cb; ++t) {
            if (t > 0) d = b_in - c * c / d;
            t32[t] = make_float2((float)(f / d), (float)(c / d));
            if (th) th[t] = make_double2(f / d, c / d);
            if (t == m - 1) d_m1 = d;
            if (t == cb - 1) d_cb1 = d;
        }
        const double b_m = (n == 1) ? 1.0 + sg : (n == 2 ? 1.0 + c + sg : b_in);
        double gamma = b_m;
        if (m > 0) gamma -= c * c / d_m1;
        if (cb > 0) gamma -= c * c / d_cb1;
        S.mid32[a][0] = (float)(f / gamma);
        S.mid32[a][1] = (float)(c / gamma);
        S.mid64[a][0] = f / gamma;
        S.mid64[a][1] = c / gamma;
    }
}

hipError_t launch_coefficients(const SubDev *, int nsubs, float2 *coef32, double2 *coefh, double2 *coef64,
                               SubDev *subs_rw, hipStream_t st)
{
    const int threads = nsubs * 3;
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(coefficients_kernel, dim3((threads + 127) / 128), dim3(128), 0, st,
                       subs_rw, nsubs, coef32, coefh, coef64);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain FP64 path: one thread per line, Thomas elimination writing y into the
// field, back-substitution reading it back (the paper's per-direction loops).

__device__ __forceinline__ int find_slot_ll(const long long *__restrict__ prefix, int count,
                                            long long x)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int AXIS>
__global__ void sweep_plain_kernel(const SubDev *__restrict__ subs, int nsubs,
                                   const long long *__restrict__ lines_prefix,
                                   long long total, const double2 *__restrict__ coef,
                                   double *__restrict__ field)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int k = find_slot_ll(lines_prefix, nsubs, g);
    const SubDev &S = subs[k];
    const long long L = g - lines_prefix[k];
    const long long nx = S.n[0], ny = S.n[1];
    const int n = S.n[AXIS];
    long long start, stride;
    if (AXIS == 0) {
        start = L * nx;
        stride = 1;
    } else if (AXIS == 1) {
        start = (L % nx) + nx * ny * (L / nx);
        stride = nx;
    } else {
        start = L;
        stride = nx * ny;
    }
    double *p = field + S.base + start;
    const double2 *cf = coef + S.coef64[AXIS];
    const double c = S.c[AXIS];
    double y = p[0] * cf[0].x;
    p[0] = y;
    for (int i = 1; i < n; ++i) {
        y = (p[i * stride] + c * y) * cf[i].x;
        p[i * stride] = y;
    }
    double x = y;
    for (int i = n - 2; i >= 0; --i) {
        x = p[i * stride] + cf[i].y * x;
        p[i * stride] = x;
    }
}

hipError_t launch_sweep_plain(int axis, const SubDev *subs, int nsubs,
                              const long long *lines_prefix, long long total_lines,
                              const double2 *coef, double *field, hipStream_t st)
{
    if (total_lines <= 0) return hipSuccess;
    const dim3 grid((unsigned)((total_lines + 255) / 256)), block(256);
    if (axis == 0)
        hipLaunchKernelGGL(sweep_plain_kernel<0>, grid, block, 0, st, subs, nsubs, lines_prefix, total_lines, coef, field);
    else if (axis == 1)
        hipLaunchKernelGGL(sweep_plain_kernel<1>, grid, block, 0, st, subs, nsubs, lines_prefix, total_lines, coef, field);
    else
        hipLaunchKernelGGL(sweep_plain_kernel<2>, grid, block, 0, st, subs, nsubs, lines_prefix, total_lines, coef, field);
    return hipGetLastError();
}

// P_D over the Dirichlet faces.  faces[q] = (volume, face, 0, 0); one thread
// per voxel of a face; every thread writes the value of the highest-numbered
// active face containing its voxel, so voxels shared by faces get the same
// value from every thread that touches them.
__global__ void dirichlet_plain_kernel(const SubDev *__restrict__ subs, const int4 *__restrict__ faces,
                                       int nfaces, const long long *__restrict__ face_prefix,
                                       long long total, double *__restrict__ field)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int q = find_slot_ll(face_prefix, nfaces, g);
    const int4 F = faces[q];
    const SubDev &S = subs[F.x];
    const int f = F.y;
    const int a = f / 2;
    const int au = (a == 0) ? 1 : 0, aw = (a == 2) ? 1 : 2;
    const long long u_w = g - face_prefix[q];
    int c[3];
    c[a] = (f & 1) ? S.n[a] - 1 : 0;
    c[au] = (int)(u_w % S.n[au]);
    c[aw] = (int)(u_w / S.n[au]);
    int best = -1;
    for (int ff = 0; ff < 6; ++ff) {
        const int aa = ff / 2;
        const int layer = (ff & 1) ? S.n[aa] - 1 : 0;
        if (((S.dir_mask >> ff) & 1) && c[aa] == layer) best = ff;
    }
    const long long v = c[0] + (long long)S.n[0] * (c[1] + (long long)S.n[1] * c[2]);
    field[S.base + v] = S.dval64[best];
}

hipError_t launch_dirichlet_plain(const SubDev *subs, const int4 *faces, int nfaces,
                                  const long long *face_prefix, long long total,
                                  double *field, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(dirichlet_plain_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, subs, faces, nfaces, face_prefix, total, field);
    return hipGetLastError();
}

// F: rho <- rho / (1 + lambda dt), elementwise.
__global__ void decay_plain_kernel(const SubDev *__restrict__ subs, int nsubs,
                                   const long long *__restrict__ vox_prefix, long long total,
                                   double *__restrict__ field)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int k = find_slot_ll(vox_prefix, nsubs, g);
    const SubDev &S = subs[k];
    double *p = field + S.base + (g - vox_prefix[k]);
    *p = *p * S.fdec;
}

hipError_t launch_decay_plain(const SubDev *subs, int nsubs, const long long *vox_prefix,
                              long long total, double *field, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(decay_plain_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       subs, nsubs, vox_prefix, total, field);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a2: cell binning.  Keys are (voxel << 24) | cell index, so sorting them
// orders cells by voxel and, inside a voxel, by upload order; cells outside
// the grid get the largest key and sort last.

constexpr unsigned long long kNoVoxel = ~0ull;

__global__ void cell_keys_kernel(const double *__restrict__ pos, int n, int nx, int ny, int nz,
                                 double x0, double y0, double z0, double dx, double dy, double dz,
                                 unsigned long long *__restrict__ keys, int *n_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {x0, y0, z0}, h[3] = {dx, dy, dz};
    const int nn[3] = {nx, ny, nz};
    long long idx[3];
    bool inside = true;
    for (int a = 0; a < 3; ++a) {
        const double t = floor((pos[3 * (size_t)i + a] - lo[a]) / h[a]);
        if (!(t >= 0.0) || !(t < (double)nn[a])) inside = false;
        idx[a] = inside ? (long long)t : 0;
    }
    if (!inside) {
        keys[i] = kNoVoxel;
        atomicAdd(n_out, 1);
        return;
    }
    const unsigned long long v = idx[0] + (long long)nx * (idx[1] + (long long)ny * idx[2]);
    keys[i] = (v << 24) | (unsigned long long)i;
}

hipError_t launch_cell_keys(const double *pos, int n, int nx, int ny, int nz, double x0, double y0,
                            double z0, double dx, double dy, double dz, unsigned long long *keys,
                            int *n_out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(cell_keys_kernel, dim3((n + 255) / 256), dim3(256), 0, st, pos, n, nx, ny,
                       nz, x0, y0, z0, dx, dy, dz, keys, n_out);
    return hipGetLastError();
}

// Stable LSD radix sort of 64-bit keys on bits [lo, lo + 4*passes): least
// significant digit first, each pass a stable counting sort of one 4-bit digit
// (Knuth, The Art of Computer Programming vol. 3, section 5.2.5).  Blocks of
// kRsTile consecutive keys: per-block digit counts, one exclusive scan over
// (digit, block) in digit-major order, then each block writes its keys to
// their places in key order, which keeps equal digits in their input order.
// The key count is read on the device (*n_dev, at most n_cap, which sizes the
// grids), so a count produced by an earlier kernel needs no trip to the host.
constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsRadix = 16;

__global__ void __launch_bounds__(kRsThreads)
rs_hist_kernel(const unsigned long long *__restrict__ keys, const int *__restrict__ n_dev, int shift,
               unsigned *__restrict__ hist, int nblocks)
{
    __shared__ unsigned cnt[kRsRadix];
    const int n = *n_dev;
    if (threadIdx.x < kRsRadix) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRsTile;
    for (int i = threadIdx.x; i < kRsTile; i += kRsThreads) {
        const int g = base + i;
        if (g < n) atomicAdd(&cnt[(unsigned)(keys[g] >> shift) & (kRsRadix - 1)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kRsRadix) hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// In-place exclusive scan of a[0..m) by one workgroup of 1024 threads, in
// rounds of kScanChunk entries: each round is read into LDS with coalesced
// loads, thread t scans its eight consecutive entries, the thread sums are
// scanned within each wave by shuffles and across the 16 waves through LDS,
// and the round goes back with coalesced stores, offset by the earlier
// rounds' sum.  *total (if given) receives the sum of all entries.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanThreads * kScanPer;

__global__ void __launch_bounds__(kScanThreads) scan_small_kernel(unsigned *__restrict__ a, int m, int *total)
{
    __shared__ unsigned buf[kScanChunk];
    __shared__ unsigned wsum[kScanThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    unsigned carry = 0;  // sum of the earlier rounds
    for (int c0 = 0; c0 < m; c0 += kScanChunk) {
        const int len = min(kScanChunk, m - c0);
        for (int i = t; i < len; i += kScanThreads) buf[i] = a[c0 + i];
        __syncthreads();
        unsigned v[kScanPer];
        unsigned sum = 0;
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int i = kScanPer * t + j;
            v[j] = i < len ? buf[i] : 0u;
            sum += v[j];
        }
        unsigned x = sum;  // inclusive scan of the thread sums within the wave
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const unsigned y = __shfl_up(x, off, kWave);
            if (lane >= off) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        if (t < kWave) {  // inclusive scan of the wave sums
            unsigned q = t < kScanThreads / kWave ? wsum[t] : 0u;
#pragma unroll
            for (int off = 1; off < kScanThreads / kWave; off <<= 1) {
                const unsigned y = __shfl_up(q, off, kWave);
                if (t >= off) q += y;
            }
            if (t < kScanThreads / kWave) wsum[t] = q;
        }
        __syncthreads();
        unsigned run = carry + (w ? wsum[w - 1] : 0u) + (x - sum);
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int i = kScanPer * t + j;
            if (i < len) buf[i] = run;
            run += v[j];
        }
        carry += wsum[kScanThreads / kWave - 1];
        __syncthreads();
        for (int i = t; i < len; i += kScanThreads) a[c0 + i] = buf[i];
        __syncthreads();  // buf and wsum are refilled by the next round
    }
    if (total && t == 0) *total = (int)carry;
}

// c[d][t]: thread t's count of digit d on entry, its exclusive prefix over the
// block's threads on exit (16 digits x 16 segments of 16 threads: each thread
// sums one segment, one thread per digit scans the segment sums).
__device__ __forceinline__ void rs_block_prefix(unsigned (&c)[kRsRadix][kRsThreads],
                                                unsigned (&seg)[kRsRadix][kRsThreads / kRsRadix])
{
    constexpr int kSeg = kRsThreads / kRsRadix;
    const int t = threadIdx.x;
    const int r = t / kSeg, q = t % kSeg;
    unsigned sum = 0;
    for (int j = 0; j < kSeg; ++j) sum += c[r][q * kSeg + j];
    seg[r][q] = sum;
    __syncthreads();
    if (t < kRsRadix) {
        unsigned run = 0;
        for (int j = 0; j < kSeg; ++j) {
            const unsigned v = seg[t][j];
            seg[t][j] = run;
            run += v;
        }
    }
    __syncthreads();
    unsigned run = seg[r][q];
    for (int j = 0; j < kSeg; ++j) {
        const unsigned v = c[r][q * kSeg + j];
        c[r][q * kSeg + j] = run;
        run += v;
    }
    __syncthreads();
}

// Thread t holds keys t*kRsItems .. of its block's tile, in order; the keys of
// one digit land after those of earlier blocks and earlier threads.
__global__ void __launch_bounds__(kRsThreads)
rs_scatter_kernel(const unsigned long long *__restrict__ in, unsigned long long *__restrict__ out,
                  const int *__restrict__ n_dev, int shift, const unsigned *__restrict__ offs, int nblocks)
{
    __shared__ unsigned c[kRsRadix][kRsThreads];
    __shared__ unsigned seg[kRsRadix][kRsThreads / kRsRadix];
    const int n = *n_dev;
    const int t = threadIdx.x;
    const int base = blockIdx.x * kRsTile + t * kRsItems;
    for (int d = 0; d < kRsRadix; ++d) c[d][t] = 0;
    unsigned long long k[kRsItems];
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int g = base + j;
        k[j] = g < n ? in[g] : 0ull;
        if (g < n) ++c[(unsigned)(k[j] >> shift) & (kRsRadix - 1)][t];
    }
    __syncthreads();
    rs_block_prefix(c, seg);
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        if (base + j < n) {
            const unsigned d = (unsigned)(k[j] >> shift) & (kRsRadix - 1);
            out[offs[d * nblocks + blockIdx.x] + c[d][t]++] = k[j];
        }
    }
}

int radix_hist_entries(int n_cap) { return kRsRadix * ((max(n_cap, 1) + kRsTile - 1) / kRsTile); }

hipError_t launch_radix_sort(unsigned long long *keys, unsigned long long *alt, int n_cap, const int *n_dev, int lo_bit,
                             int bits, unsigned *hist, hipStream_t st)
{
    if (n_cap <= 0 || bits <= 0) return hipSuccess;
    const int passes = (bits + 3) / 4;
    if (lo_bit < 0 || lo_bit + 4 * passes > 64) return hipErrorInvalidValue;
    const int nb = (n_cap + kRsTile - 1) / kRsTile;
    unsigned long long *src = keys, *dst = alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = lo_bit + 4 * p;
        hipLaunchKernelGGL(rs_hist_kernel, dim3(nb), dim3(kRsThreads), 0, st, src, n_dev, shift, hist, nb);
        hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(1024), 0, st, hist, kRsRadix * nb, (int *)nullptr);
        hipLaunchKernelGGL(rs_scatter_kernel, dim3(nb), dim3(kRsThreads), 0, st, src, dst, n_dev, shift, hist, nb);
        unsigned long long *tmp = src;
        src = dst;
        dst = tmp;
    }
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    // after an odd number of passes the sorted keys are in alt (the first
    // *n_dev of them matter; n_cap bounds them)
    if (passes & 1) return hipMemcpyAsync(keys, alt, sizeof(unsigned long long) * (size_t)n_cap,
                                          hipMemcpyDeviceToDevice, st);
    return hipSuccess;
}

// Occupied voxels of the sorted keys (the first n_in, counts[2], are inside
// the grid): each key that starts a new voxel is flagged, and the flags are
// numbered by an exclusive scan over blocks of kRsTile keys (block counts, one
// scan of the block counts, then each block's own scan), so segment ids, the
// occupied-voxel list and each segment's first key come out in ascending
// voxel order; counts[1] receives the number of occupied voxels.
__device__ __forceinline__ unsigned new_voxel(const unsigned long long *__restrict__ keys, int p, int n)
{
    return p < n && (p == 0 || (keys[p] >> 24) != (keys[p - 1] >> 24));
}

__global__ void __launch_bounds__(kRsThreads) n_in_kernel(int n, int *counts)
{
    if (threadIdx.x == 0) counts[2] = n - counts[0];
}

// The counts of an upload: out of domain, occupied voxels and inside (filled
// in by the kernels that follow) start at zero; counts[4] = n keys to sort.
__global__ void upload_counts_kernel(int *counts, int n)
{
    if (threadIdx.x == 0) {
        counts[0] = 0;
        counts[1] = 0;
        counts[2] = 0;
        counts[4] = n;
    }
}

hipError_t launch_upload_counts(int *counts, int n, hipStream_t st)
{
    hipLaunchKernelGGL(upload_counts_kernel, dim3(1), dim3(64), 0, st, counts, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kRsThreads)
seg_count_kernel(const unsigned long long *__restrict__ keys, const int *__restrict__ counts,
                 unsigned *__restrict__ bsum)
{
    __shared__ unsigned red[kRsThreads];
    const int n = counts[2];
    const int base = blockIdx.x * kRsTile;
    unsigned c = 0;
    for (int i = threadIdx.x; i < kRsTile; i += kRsThreads) c += new_voxel(keys, base + i, n);
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = kRsThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kRsThreads)
seg_write_kernel(const unsigned long long *__restrict__ keys, const int *__restrict__ counts,
                 const unsigned *__restrict__ boff, int *__restrict__ seg_id, int *__restrict__ occ_vox,
                 int *__restrict__ seg_start)
{
    __shared__ unsigned tsum[kRsThreads];
    const int n = counts[2];
    const int t = threadIdx.x;
    const int base = blockIdx.x * kRsTile + t * kRsItems;
    unsigned f[kRsItems], c = 0;
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        f[j] = new_voxel(keys, base + j, n);
        c += f[j];
    }
    tsum[t] = c;
    __syncthreads();
    for (int o = 1; o < kRsThreads; o <<= 1) {
        const unsigned v = t >= o ? tsum[t - o] : 0u;
        __syncthreads();
        tsum[t] += v;
        __syncthreads();
    }
    unsigned run = boff[blockIdx.x] + (t ? tsum[t - 1] : 0u);
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int p = base + j;
        if (p < n) {
            run += f[j];
            const int sid = (int)run - 1;
            seg_id[p] = sid;
            if (f[j]) {
                occ_vox[sid] = (int)(keys[p] >> 24);
                seg_start[sid] = p;
            }
        }
    }
    if (blockIdx.x == 0 && t == 0) seg_start[counts[1]] = n;
}

hipError_t launch_segments(const unsigned long long *keys, int n_cap, int n, int *seg_id, int *occ_vox,
                           int *seg_start, int *counts, unsigned *scratch, hipStream_t st)
{
    const int nb = (max(n_cap, 1) + kRsTile - 1) / kRsTile;
    hipLaunchKernelGGL(n_in_kernel, dim3(1), dim3(kRsThreads), 0, st, n, counts);
    hipLaunchKernelGGL(seg_count_kernel, dim3(nb), dim3(kRsThreads), 0, st, keys, counts, scratch);
    hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(1024), 0, st, scratch, nb, counts + 1);
    hipLaunchKernelGGL(seg_write_kernel, dim3(nb), dim3(kRsThreads), 0, st, keys, counts, scratch, seg_id, occ_vox,
                       seg_start);
    return hipGetLastError();
}

// FP32 path: occupied voxels re-ordered by z-line (i, j) then k, so that the
// voxels of 64 consecutive z-lines form one contiguous range.  Keys are
// (line << 32) | (index in voxel order), sorted stably on the line bits.  The
// number of occupied voxels is counts[1] (on the device), at most n_cap.
__global__ void zline_keys_kernel(const int *__restrict__ occ_vox_v, const int *__restrict__ counts, int n_cap,
                                  int nxy, int nz, unsigned long long *__restrict__ zkeys)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_cap || p >= counts[1]) return;
    // the list is in voxel order, i.e. by (k, line): a stable sort on the
    // line alone leaves each line's voxels in k order
    const int v = occ_vox_v[p];
    zkeys[p] = ((unsigned long long)(unsigned)(v % nxy) << 32) | (unsigned)p;
}

// After sorting the z keys: pos[voxel-order index] = z-order index, the
// occupied voxel list in z order, and line_start[L] = first z-order entry of
// z-line L (line_start[nxy] = n_occ).  Each entry fills the starts of the
// lines between its predecessor's line and its own.
__global__ void zline_scatter_kernel(const unsigned long long *__restrict__ zkeys, const int *__restrict__ counts,
                                     int n_cap, int nxy, int nz, const int *__restrict__ occ_vox_v,
                                     int *__restrict__ occ_vox, int *__restrict__ pos, int *__restrict__ line_start)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_occ = counts[1];
    if (p >= n_cap || p >= n_occ) return;
    const unsigned long long key = zkeys[p];
    const int q = (int)(key & 0xffffffffull);
    pos[q] = p;
    occ_vox[p] = occ_vox_v[q];
    const int L = (int)(key >> 32);
    const int Lprev = (p == 0) ? -1 : (int)(zkeys[p - 1] >> 32);
    for (int l = Lprev + 1; l <= L; ++l) line_start[l] = p;
    if (p == n_occ - 1)
        for (int l = L + 1; l <= nxy; ++l) line_start[l] = n_occ;
}

static int bit_length(unsigned long long x)
{
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

hipError_t launch_zline_order(const int *occ_vox_v, const int *counts, int n_cap, int nxy, int nz,
                              unsigned long long *zkeys, unsigned long long *zalt, unsigned *hist, int *occ_vox,
                              int *pos, int *line_start, hipStream_t st)
{
    if (n_cap <= 0) return hipSuccess;
    const dim3 grid((n_cap + 255) / 256), block(256);
    hipLaunchKernelGGL(zline_keys_kernel, grid, block, 0, st, occ_vox_v, counts, n_cap, nxy, nz, zkeys);
    // the line part of a key is below nxy
    hipError_t e = launch_radix_sort(zkeys, zalt, n_cap, counts + 1, 32, bit_length((unsigned long long)nxy), hist, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(zline_scatter_kernel, grid, block, 0, st, zkeys, counts, n_cap, nxy, nz, occ_vox_v, occ_vox,
                       pos, line_start);
    return hipGetLastError();
}

// Per occupied voxel and substrate, walk its cells in upload order (FP64):
//   a_i = k_i S_i rho*_i,  b_i = 1 + k_i (S_i + U_i),  k_i = dt V_i / V_vox.
// Applying the cells one after another maps rho to rho R + P with
//   R <- R / b_i,  P <- (P + a_i) / b_i  (from R = 1, P = 0),
// i.e. R = 1/B and P = A/B of the composite (rho + A)/B, A = sum a_i prod_{j<i}
// b_j, B = prod b_i.  Both stay bounded whatever the number of cells:
// 0 < R <= 1 and P lies between 0 and the largest rho*_i, where A and B
// themselves grow without bound (B passes the FP32 range after about 150
// fast cells).  FP32 path: (P, R), applied as fmaf(rho, R, P); FP64 path: the
// per-cell (a_i, b_i) in sorted order.
__global__ void composites_kernel(const unsigned long long *__restrict__ keys,
                                  const int *__restrict__ seg_start, const int *__restrict__ counts, int ns,
                                  const double *__restrict__ V, const double *__restrict__ S,
                                  const double *__restrict__ U, const double *__restrict__ RS,
                                  double dt, double vvox, const int *__restrict__ pos,
                                  float2 *__restrict__ comp32, float2 *__restrict__ comp32_v, int v_stride,
                                  double2 *__restrict__ ab64, double *__restrict__ krs,
                                  double *__restrict__ kcell, int *__restrict__ cell_of)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)counts[1] * ns) return;
    const int seg = (int)(g / ns), s = (int)(g % ns);
    const int out = pos ? pos[seg] : seg;
    double P = 0.0, R = 1.0;
    for (int p = seg_start[seg]; p < seg_start[seg + 1]; ++p) {
        const int i = (int)(keys[p] & 0xFFFFFFull);
        const double k = dt * V[i] / vvox;
        const size_t q = (size_t)i * ns + s;
        const double a = k * S[q] * RS[q];
        const double b = 1.0 + k * (S[q] + U[q]);
        if (ab64) ab64[(size_t)p * ns + s] = make_double2(a, b);
        if (krs) krs[(size_t)p * ns + s] = k * RS[q];
        if (s == 0 && kcell) kcell[p] = k;
        if (s == 0 && cell_of) cell_of[p] = i;
        P = (P + a) / b;
        R = R / b;
    }
    const float2 c32 = make_float2((float)P, (float)R);
    if (comp32) comp32[(size_t)out * ns + s] = c32;
    if (comp32_v) comp32_v[(size_t)s * v_stride + seg] = c32;  // substrate-major
}

hipError_t launch_composites(const unsigned long long *keys, const int *seg_start, const int *counts, int n_cap,
                             int ns, const double *V, const double *S, const double *U, const double *RS,
                             double dt, double vvox, const int *pos, float2 *comp32, float2 *comp32_v,
                             int v_stride, double2 *ab64, double *krs, double *kcell, int *cell_of, hipStream_t st)
{
    const long long total = (long long)n_cap * ns;  // counts[1] * ns of them work
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(composites_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, keys,
                       seg_start, counts, ns, V, S, U, RS, dt, vvox, pos, comp32, comp32_v, v_stride, ab64, krs,
                       kcell, cell_of);
    return hipGetLastError();
}

// The end of a simulation's upload, on the device so that the host need not
// read the counts back: its occupied-voxel count (counts[1], none without
// counts) into its entry of the cell tables, whether its sources can be
// carried into the next x solve (only with occupied voxels), and the
// exclusive prefix of the occupied voxels over the simulations, which the
// sources kernels search and whose last entry bounds them.  One thread; the
// kernels launched after it on the stream see the new tables.
__global__ void finish_upload_kernel(const int *__restrict__ counts, SimCells *__restrict__ cells, int sim,
                                     int nsims, int xs_base, int *__restrict__ occ_prefix)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int n_occ = counts ? counts[1] : 0;
    cells[sim].n_occ = n_occ;
    cells[sim].xs_base = n_occ > 0 ? xs_base : -1;
    int acc = 0;
    occ_prefix[0] = 0;
    for (int k = 0; k < nsims; ++k) {
        acc += cells[k].n_occ;
        occ_prefix[k + 1] = acc;
    }
}

hipError_t launch_finish_upload(const int *counts, SimCells *cells, int sim, int nsims, int xs_base, int *occ_prefix,
                                hipStream_t st)
{
    hipLaunchKernelGGL(finish_upload_kernel, dim3(1), dim3(64), 0, st, counts, cells, sim, nsims, xs_base, occ_prefix);
    return hipGetLastError();
}

// First entry of every x-line (j + ny k) in the occupied voxels listed in
// voxel order: the lower bound of the line's first voxel index.
__global__ void xline_starts_kernel(const int *__restrict__ occ_vox_v, const int *__restrict__ counts, int nx,
                                    int nlines, int *__restrict__ line_start)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > nlines) return;
    const long long v0 = (long long)l * nx;
    int lo = 0, hi = counts[1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)occ_vox_v[mid] < v0)
            lo = mid + 1;
        else
            hi = mid;
    }
    line_start[l] = lo;
}

hipError_t launch_xline_starts(const int *occ_vox_v, const int *counts, int nx, int nlines, int *line_start,
                               hipStream_t st)
{
    if (nlines < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xline_starts_kernel, dim3((nlines + 1 + 255) / 256), dim3(256), 0, st, occ_vox_v, counts,
                       nx, nlines, line_start);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sources (C), after the last Dirichlet projection of the step.

__device__ __forceinline__ int find_slot_i(const int *__restrict__ prefix, int count, int x)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The composite of occupied voxel jl (of simulation C) on substrate s:
// rho <- rho R + P, one fused multiply-add (the same operation wherever the
// sources are applied, so every placement gives the same bits), for the
// jl-th occupied voxel in voxel order and its substrate-major composite
// (stride occ_cap): neighbouring threads update neighbouring voxels.
__device__ __forceinline__ void apply_composite(const SimCells &C, int jl, int s, const SubDev *__restrict__ subs,
                                                const int *__restrict__ occ_vox_v, const float2 *__restrict__ comp_v,
                                                float *__restrict__ field)
{
    const int v = occ_vox_v[C.occ_base + jl];
    const float2 ab = comp_v[C.comp_base + (size_t)s * C.occ_cap + jl];
    float *p = field + subs[C.sub0 + s].base + v;
    *p = fmaf(*p, ab.y, ab.x);
}

// FP32: one thread per (occupied voxel, substrate), the voxels in voxel order.
__global__ void sources_f32_kernel(const SimCells *__restrict__ cells, int nsims,
                                   const int *__restrict__ occ_prefix, int occ_bound,
                                   const SubDev *__restrict__ subs, const int *__restrict__ occ_vox_v,
                                   const float2 *__restrict__ comp_v, float *__restrict__ field, int only_carried)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= occ_bound || j >= occ_prefix[nsims]) return;  // past the occupied voxels
    const int sim = find_slot_i(occ_prefix, nsims, j);
    const SimCells &C = cells[sim];
    if (s >= C.ns || (only_carried && C.xs_base < 0)) return;
    apply_composite(C, j - occ_prefix[sim], s, subs, occ_vox_v, comp_v, field);
}

// The same update for the simulations one voxel thick in z, whose z solve is
// the identity when the decay is applied once and is therefore not launched:
// no z tile applies their sources, so this pass does, after the y solve's
// stores (which already hold the last Dirichlet projection).  skip_carried:
// leave those whose sources the next x solve applies.
__global__ void sources_thin_f32_kernel(const SimCells *__restrict__ cells, int nsims,
                                        const int *__restrict__ occ_prefix, int occ_bound,
                                        const SubDev *__restrict__ subs, const int *__restrict__ occ_vox_v,
                                        const float2 *__restrict__ comp_v, float *__restrict__ field, int skip_carried)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= occ_bound || j >= occ_prefix[nsims]) return;  // past the occupied voxels
    const int sim = find_slot_i(occ_prefix, nsims, j);
    const SimCells &C = cells[sim];
    if (s >= C.ns || subs[C.sub0].n[2] != 1 || (skip_carried && C.xs_base >= 0)) return;
    apply_composite(C, j - occ_prefix[sim], s, subs, occ_vox_v, comp_v, field);
}

hipError_t launch_sources_thin_f32(const SimCells *cells, int nsims, const int *occ_prefix, int occ_bound,
                                   int max_ns, const SubDev *subs, const int *occ_vox_v, const float2 *comp_v,
                                   float *field, int skip_carried, hipStream_t st)
{
    if (occ_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(sources_thin_f32_kernel, dim3((unsigned)((occ_bound + 255LL) / 256), max_ns), dim3(256), 0, st,
                       cells, nsims, occ_prefix, occ_bound, subs, occ_vox_v, comp_v, field, skip_carried);
    return hipGetLastError();
}

hipError_t launch_sources_f32(const SimCells *cells, int nsims, const int *occ_prefix, int occ_bound,
                              int max_ns, const SubDev *subs, const int *occ_vox_v, const float2 *comp_v,
                              float *field, int only_carried, hipStream_t st)
{
    if (occ_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(sources_f32_kernel, dim3((unsigned)((occ_bound + 255LL) / 256), max_ns), dim3(256), 0, st,
                       cells, nsims, occ_prefix, occ_bound, subs, occ_vox_v, comp_v, field, only_carried);
    return hipGetLastError();
}

// FP64 plain path: one thread per occupied voxel, cells applied one after
// another in upload order: rho <- (rho + a_i) / b_i.
__global__ void sources_plain_kernel(const SimCells *__restrict__ cells, int nsims,
                                     const int *__restrict__ occ_prefix, int occ_bound,
                                     const SubDev *__restrict__ subs, const int *__restrict__ occ_vox,
                                     const int *__restrict__ seg_start, const double2 *__restrict__ ab,
                                     double *__restrict__ field)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= occ_bound || j >= occ_prefix[nsims]) return;  // past the occupied voxels
    const int sim = find_slot_i(occ_prefix, nsims, j);
    const SimCells &C = cells[sim];
    const int jl = j - occ_prefix[sim];
    const int v = occ_vox[C.occ_base + jl];
    const int p0 = seg_start[C.occ_base + jl], p1 = seg_start[C.occ_base + jl + 1];
    for (int s = 0; s < C.ns; ++s) {
        double *p = field + subs[C.sub0 + s].base + v;
        double r = *p;
        for (int q = p0; q < p1; ++q) {
            const double2 e = ab[C.ab_base + (size_t)q * C.ns + s];
            r = (r + e.x) / e.y;
        }
        *p = r;
    }
}

hipError_t launch_sources_plain(const SimCells *cells, int nsims, const int *occ_prefix, int occ_bound,
                                const SubDev *subs, const int *occ_vox, const int *seg_start,
                                const double2 *ab, double *field, hipStream_t st)
{
    if (occ_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(sources_plain_kernel, dim3((unsigned)((occ_bound + 255LL) / 256)), dim3(256), 0, st, cells,
                       nsims, occ_prefix, occ_bound, subs, occ_vox, seg_start, ab, field);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a7: mass.  Fixed grid of kMassBlocks blocks, each summing a fixed strided
// set of voxels and reducing in a fixed tree; a second one-block pass adds
// the partials in block order.  The result does not depend on timing.

template <typename T>
__global__ void __launch_bounds__(256) mass_partial_kernel(const T *__restrict__ field, long long base,
                                                           long long vol, double *__restrict__ partials)
{
    __shared__ double red[256];
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < vol; v += stride)
        acc += (double)field[base + v];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void mass_final_kernel(const double *__restrict__ partials, int n, double *out)
{
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += partials[i];
    *out = acc;
}

hipError_t launch_mass(const void *field, int is_f64, long long base, long long vol,
                       double *partials, double *out, hipStream_t st)
{
    if (is_f64)
        hipLaunchKernelGGL(mass_partial_kernel<double>, dim3(kMassBlocks), dim3(256), 0, st,
                           (const double *)field, base, vol, partials);
    else
        hipLaunchKernelGGL(mass_partial_kernel<float>, dim3(kMassBlocks), dim3(256), 0, st,
                           (const float *)field, base, vol, partials);
    hipLaunchKernelGGL(mass_final_kernel, dim3(1), dim3(64), 0, st, partials, kMassBlocks, out);
    return hipGetLastError();
}

template <typename T>
__global__ void nonfinite_kernel(const T *__restrict__ field, const SubDev *__restrict__ subs,
                                 unsigned long long *count)
{
    const SubDev &S = subs[blockIdx.y];
    unsigned long long bad = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < S.vol; v += stride) {
        const double x = (double)field[S.base + v];
        bad += !isfinite(x);
    }
    if (bad) atomicAdd(count, bad);
}

hipError_t launch_count_nonfinite(const void *field, int is_f64, const SubDev *subs, int nsubs,
                                  unsigned long long *count, hipStream_t st)
{
    if (nsubs <= 0) return hipSuccess;
    const dim3 grid(128, nsubs);
    if (is_f64)
        hipLaunchKernelGGL(nonfinite_kernel<double>, grid, dim3(256), 0, st, (const double *)field, subs, count);
    else
        hipLaunchKernelGGL(nonfinite_kernel<float>, grid, dim3(256), 0, st, (const float *)field, subs, count);
    return hipGetLastError();
}

// AoS [v][s] <-> the SoA volumes of one simulation (inverse = 1: SoA -> AoS).
template <typename T>
__global__ void aos_soa_kernel(const T *__restrict__ src, T *__restrict__ field, long long base,
                               long long vol_stride, long long vol, int ns, int inverse)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= vol * ns) return;
    const long long v = g / ns;
    const int s = (int)(g % ns);
    if (!inverse)
        field[base + s * vol_stride + v] = src[g];
    else
        const_cast<T *>(src)[g] = field[base + s * vol_stride + v];
}

hipError_t launch_aos_to_soa(const void *src, void *field, int is_f64, long long base,
                             long long vol_stride, long long vol, int ns, int inverse, hipStream_t st)
{
    const long long total = vol * ns;
    if (total <= 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (is_f64)
        hipLaunchKernelGGL(aos_soa_kernel<double>, grid, block, 0, st, (const double *)src, (double *)field,
                           base, vol_stride, vol, ns, inverse);
    else
        hipLaunchKernelGGL(aos_soa_kernel<float>, grid, block, 0, st, (const float *)src, (float *)field,
                           base, vol_stride, vol, ns, inverse);
    return hipGetLastError();
}

// Checks cell arrays that are already on the device before an upload uses
// them: bit 0 of *bad for a volume that is not finite and > 0, bit 1 for a
// negative or non-finite rate, bit 2 for a non-finite target density.  The
// flags are combined with atomic OR in global memory.
__global__ void check_cells_kernel(int n, int ns, const double *__restrict__ V, const double *__restrict__ S,
                                   const double *__restrict__ U, const double *__restrict__ RS, int *__restrict__ bad)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)n * ns) return;
    const int i = (int)(g / ns);
    int b = 0;
    if (g % ns == 0 && !(V[i] > 0.0 && isfinite(V[i]))) b |= 1;
    if (!(S[g] >= 0.0 && isfinite(S[g])) || !(U[g] >= 0.0 && isfinite(U[g]))) b |= 2;
    if (!isfinite(RS[g])) b |= 4;
    if (b) atomicOr(bad, b);
}

hipError_t launch_check_cells(int n, int ns, const double *V, const double *S, const double *U, const double *RS,
                              int *bad, hipStream_t st)
{
    const long long total = (long long)n * ns;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(check_cells_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, ns, V, S, U, RS,
                       bad);
    return hipGetLastError();
}

}  // namespace vl
