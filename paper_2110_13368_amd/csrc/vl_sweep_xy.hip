// vl_sweep_xy.hip -- the x and the y solve of one z-plane in one workgroup.
//
// Every x-line and every y-line of the plane k lies in that plane, and the
// plane is one contiguous run of nx*ny voxels.  When it fits in LDS, one
// workgroup DMA-loads it from HBM, solves its x-lines in LDS (with the
// Dirichlet projection before and after, and the decay folded into the x
// table), then solves its y-lines reading LDS and stores the result to HBM:
// the two sweeps cost one read and one write of the field instead of two of
// each.
//
// The solves run in place in LDS: the elimination overwrites each right-hand
// side with its eliminated value, the back-substitution overwrites those with
// the solution (the y solve sends it to HBM instead).  No per-lane register
// array, so one kernel serves every line length.  Same tables, same
// operations in the same order as the separate x and y kernels, so the field
// is bitwise the same.
#include "vl_device.h"

namespace vl {

constexpr int kXYBlock = 16;  // rows per block of LDS reads in the in-place solves

// One x (AXIS 0) or y (AXIS 1) solve of the lines of one plane held in LDS
// at P (row j at P + j*SX).  Lines are handled 64 at a time by each of the
// four wave pairs (wave 0 of a pair takes the first half of each line, wave 1
// the second, as in the split solve of the sweep kernels); every wave runs
// the same rounds so that the workgroup barriers line up.
template <int AXIS>
__device__ __forceinline__ void plane_solve(const SubDev &S, int k, float *P, int SX, const double2 *piv,
                                            double *xchg, __amdgpu_buffer_rsrc_t rp)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int pair = wave >> 1;
    const bool top = (wave & 1) == 0;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int n = S.n[AXIS];
    const int nlines = AXIS == 0 ? ny : nx;  // lines of this axis in the plane
    const int m = (n - 1) >> 1;
    const int cb = n - 1 - m;
    const int nel = top ? m : cb;
    const double g1 = S.mid64[AXIS][0];
    const double g2 = S.mid64[AXIS][1];
    const int dmask = S.dir_mask;
    const int lo_f = (dmask >> (2 * AXIS)) & 1 ? 2 * AXIS : -1;
    const int hi_f = (dmask >> (2 * AXIS + 1)) & 1 ? 2 * AXIS + 1 : -1;
    const int on_z = (k == 0 ? 1 << 4 : 0) | (k == nz - 1 ? 1 << 5 : 0);
    // this pair's exchange slot per lane: the second-half wave leaves its last
    // eliminated value there, the first-half wave reads it and puts the middle
    // unknown in its place (the barriers separate the three accesses)
    double *xs = xchg + pair * kWave;
    // element t of this wave's half line: e_first + t*e_step from the line's
    // origin (x: along the row; y: down the column)
    const int unit = AXIS == 0 ? 1 : SX;
    const int e_first = top ? 0 : (n - 1) * unit;
    const int e_step = top ? unit : -unit;
    const int e_mid = m * unit;
    // HBM byte offsets of the y solve's rows (wave-uniform)
    const int g_first = top ? 0 : (n - 1) * nx * 4;
    const int g_step = (top ? 1 : -1) * nx * 4;

    const int ntiles = (nlines + kTileLines - 1) / kTileLines;
    const int rounds = (ntiles + 3) / 4;
    for (int rd = 0; rd < rounds; ++rd) {
        const int tt = rd * 4 + pair;
        const bool active = tt < ntiles;  // wave-uniform
        const int line = min(tt * kTileLines + lane, nlines - 1);
        const bool valid = active && tt * kTileLines + lane < nlines;
        int on = on_z;
        if (AXIS == 0)
            on |= (line == 0 ? 1 << 2 : 0) | (line == ny - 1 ? 1 << 3 : 0);
        else
            on |= (line == 0 ? 1 : 0) | (line == nx - 1 ? 2 : 0);
        const int wface = top_face(dmask & on);
        const bool whole = wface >= 0;
        const float wv = whole ? face_value(S.dval32, wface) : 0.f;
        const int f_first = max(wface, max(lo_f, n == 1 ? hi_f : -1));
        const int f_last = max(wface, hi_f);
        float *L0 = P + (AXIS == 0 ? line * SX : line);

        // ---- elimination from this wave's end towards the middle (x: the
        //      end row takes its Dirichlet value first), in blocks of
        //      kXYBlock rows: the block's reads are issued together, the
        //      recurrence runs in registers, then the block is written back.
        //      Element t sits at E0[t * e_step]; full blocks carry no
        //      per-row tests, only the last (partial) block does ----
        float *E0 = L0 + e_first;
        const int nfull = nel / kXYBlock;
        double prev = 0.0;  // FP64 recurrences, as in the sweep kernels
        if (active) {
            const bool end_d = AXIS == 0 && (top ? lo_f : hi_f) >= 0;
            const float end_v = end_d ? S.dval32[top ? lo_f : hi_f] : 0.f;
            for (int b = 0; b < nfull; ++b) {
                const int t0 = b * kXYBlock;
                float r[kXYBlock];
#pragma unroll
                for (int e = 0; e < kXYBlock; ++e) r[e] = E0[(t0 + e) * e_step];
                if (b == 0 && end_d) r[0] = end_v;
#pragma unroll
                for (int e = 0; e < kXYBlock; ++e) {
                    const double2 c = piv[t0 + e];
                    prev = fma(c.y, prev, (double)r[e] * c.x);
                    r[e] = (float)prev;
                }
                if (valid) {
#pragma unroll
                    for (int e = 0; e < kXYBlock; ++e) E0[(t0 + e) * e_step] = r[e];
                }
            }
            const int t0 = nfull * kXYBlock;
            if (t0 < nel) {
                float r[kXYBlock];
#pragma unroll
                for (int e = 0; e < kXYBlock; ++e)
                    if (t0 + e < nel) r[e] = E0[(t0 + e) * e_step];
                if (t0 == 0 && end_d) r[0] = end_v;
#pragma unroll
                for (int e = 0; e < kXYBlock; ++e) {
                    if (t0 + e < nel) {
                        const double2 c = piv[t0 + e];
                        prev = fma(c.y, prev, (double)r[e] * c.x);
                        r[e] = (float)prev;
                    }
                }
                if (valid) {
#pragma unroll
                    for (int e = 0; e < kXYBlock; ++e)
                        if (t0 + e < nel) E0[(t0 + e) * e_step] = r[e];
                }
            }
            if (!top) xs[lane] = prev;  // z_{m+1} (0 when the line has one row)
        }
        __syncthreads();
        // ---- middle row (the first-half wave keeps it in a register) ----
        double xm = 0.0;
        if (active && top) {
            float rm = L0[e_mid];
            if (AXIS == 0 && m == 0) {
                const int f0 = max(lo_f, n == 1 ? hi_f : -1);
                if (f0 >= 0) rm = S.dval32[f0];
            }
            xm = fma(g2, prev + xs[lane], (double)rm * g1);
            xs[lane] = xm;
        }
        __syncthreads();
        // ---- back-substitution from the middle outwards (the partial block
        //      first), then the Dirichlet projection of the solve's output;
        //      x writes back to LDS, y stores to HBM with the row offset in
        //      a scalar register ----
        if (active) {
            if (!top) xm = xs[lane];
            double nxt = xm;
            const unsigned col_b = (unsigned)line * 4u;
            if (top && valid) {
                float out = whole ? wv : (float)xm;
                if (m == 0 && f_first >= 0) out = face_value(S.dval32, f_first);
                if (AXIS == 0)
                    L0[e_mid] = out;
                else
                    bstore(rp, col_b, m * nx * 4, out);
            }
            const float end_out = face_value(S.dval32, top ? f_first : f_last);
            const bool end_p = (top ? f_first : f_last) >= 0;
            {
                const int t0 = nfull * kXYBlock;
                if (t0 < nel) {
                    float y[kXYBlock];
#pragma unroll
                    for (int e = 0; e < kXYBlock; ++e)
                        if (t0 + e < nel) y[e] = E0[(t0 + e) * e_step];
#pragma unroll
                    for (int e = kXYBlock - 1; e >= 0; --e) {
                        if (t0 + e < nel) {
                            nxt = fma(piv[t0 + e].y, nxt, (double)y[e]);
                            y[e] = whole ? wv : (float)nxt;
                        }
                    }
                    if (t0 == 0 && end_p) y[0] = end_out;
                    if (valid) {
#pragma unroll
                        for (int e = 0; e < kXYBlock; ++e) {
                            if (t0 + e < nel) {
                                if (AXIS == 0)
                                    E0[(t0 + e) * e_step] = y[e];
                                else
                                    bstore(rp, col_b, g_first + (t0 + e) * g_step, y[e]);
                            }
                        }
                    }
                }
            }
            for (int b = nfull - 1; b >= 0; --b) {
                const int t0 = b * kXYBlock;
                float y[kXYBlock];
#pragma unroll
                for (int e = 0; e < kXYBlock; ++e) y[e] = E0[(t0 + e) * e_step];
#pragma unroll
                for (int e = kXYBlock - 1; e >= 0; --e) {
                    nxt = fma(piv[t0 + e].y, nxt, (double)y[e]);
                    y[e] = whole ? wv : (float)nxt;
                }
                if (b == 0 && end_p) y[0] = end_out;
                if (valid) {
#pragma unroll
                    for (int e = 0; e < kXYBlock; ++e) {
                        if (AXIS == 0)
                            E0[(t0 + e) * e_step] = y[e];
                        else
                            bstore(rp, col_b, g_first + (t0 + e) * g_step, y[e]);
                    }
                }
            }
        }
    }
}

__global__ void __launch_bounds__(kXYThreads)
sweep_xy_plane(SweepLaunch L, const SubDev *__restrict__ subs, const double2 *__restrict__ coef,
               float *__restrict__ field)
{
    extern __shared__ __attribute__((aligned(16))) float xy_lds[];
    const int plane = blockIdx.x;
    const int slot = find_slot(L.tile_prefix, L.count, plane);
    const int k = plane - L.tile_prefix[slot];
    const SubDev &S = subs[L.sub_ids[slot]];
    const int nx = S.n[0], ny = S.n[1];
    const int SX = xy_row_stride(nx);
    const int cbx = nx - 1 - (nx - 1) / 2, cby = ny - 1 - (ny - 1) / 2;
    // LDS: x and y pivot tables, one exchange slot per lane of each wave
    // pair, then the plane (sized by xy_lds_bytes)
    double2 *pivx = reinterpret_cast<double2 *>(xy_lds);
    double2 *pivy = pivx + cbx;
    double *xchg = reinterpret_cast<double *>(pivy + cby);
    float *P = reinterpret_cast<float *>(xchg + (kXYThreads / 2));
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const long long pbase = S.base + (long long)k * nx * ny;
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(field + pbase, (long long)nx * ny);

    // the plane into LDS, row j at P + j*SX: 64 columns per DMA instruction,
    // lanes past the row's end switched off
    for (int j = wave; j < ny; j += kXYThreads / kWave)
        for (int c = 0; c * kWave < nx; ++c)
            if (c * kWave + lane < nx)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rp, (__attribute__((address_space(3))) void *)(P + j * SX + c * kWave), 4,
                    (j * nx + c * kWave + lane) * 4, 0, 0, 0);
    {
        const double2 *__restrict__ cfx = coef + S.coef32[0];
        const double2 *__restrict__ cfy = coef + S.coef32[1];
        for (int t = threadIdx.x; t < cbx; t += kXYThreads) pivx[t] = cfx[t];
        for (int t = threadIdx.x; t < cby; t += kXYThreads) pivy[t] = cfy[t];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    plane_solve<0>(S, k, P, SX, pivx, xchg, rp);
    __syncthreads();
    plane_solve<1>(S, k, P, SX, pivy, xchg, rp);
}

hipError_t prepare_sweep_xy(size_t lds_bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_xy_plane),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_sweep_xy(const SweepLaunch &L, size_t lds_bytes, const SubDev *subs, const double2 *coef,
                           float *field, hipStream_t st)
{
    if (L.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(sweep_xy_plane, dim3(L.total_tiles), dim3(kXYThreads), (unsigned)lds_bytes, st, L, subs,
                       coef, field);
    return hipGetLastError();
}

}  // namespace vl
