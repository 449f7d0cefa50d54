// vl_adjoint.hip -- adjoint of the LOD step (FP32 storage, FP64 reductions).
//
// For a scalar loss L of the field after n steps, the reverse of one step
//   rho <- C . P_D . S_z . P_D . S_y . P_D . F . S_x . P_D (rho)
// is, with w the adjoint of the step's output,
//   w <- C^T w;  P_D^T;  S_z^T;  P_D^T;  S_y^T;  P_D^T;  F^T;  S_x^T;  P_D^T
// P_D^T zeroes w at Dirichlet voxels (their forward value does not depend on
// the input).  Every line matrix T is symmetric, so S_a^T is the same split
// Thomas solve as the forward sweep; the decay factor f folded into the x
// table makes the x kernel apply (F S_x)^T = f T^-1 directly.  Parameter
// derivatives, with T = (1 + sigma) I - c K (K the zero-flux second
// difference) and y the forward solve's output:
//   dL/dc     +=  w_out^T K y  = - sum_i (w_{i+1} - w_i)(y_{i+1} - y_i)
//   dL/dsigma += -w_out^T y
//   dL/dlambda (decay once) += -dt f^2 w_in^T y_x
// summed in a fixed order (per lane, per wave, per tile over the reverse
// steps, then the tiles of a volume in order), so results are deterministic.
#include "vl_device.h"

namespace vl {

__device__ __forceinline__ double wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <int AXIS, int CAP>
__device__ __forceinline__ void adjoint_tile(const SubDev &S, int local, int tile,
                                             const float2 *__restrict__ coef, float *__restrict__ w,
                                             const float *__restrict__ raw, double *__restrict__ part,
                                             TileLds<CAP, AXIS == 0, float2, float> &sh)
{
    constexpr int kChunks = (CAP + 63) / 64;
    float(&xch)[2][kWave] = sh.xch;
    float2 *cs_lds = sh.piv;
    float *stage = sh.stage;
    __shared__ double red[2][3];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const bool top = (wave == 0);
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int n = S.n[AXIS];
    const int m = (n - 1) >> 1;
    const int cb = n - 1 - m;
    const int nel = top ? m : cb;
    const float g1 = S.mid32[AXIS][0];
    const float g2 = S.mid32[AXIS][1];
    const int dmask = S.dir_mask;
    {
        const float2 *__restrict__ cf = coef + S.coef32[AXIS];
        for (int t = threadIdx.x; t < cb && t < CAP; t += 128) cs_lds[t] = cf[t];
    }

    int on = 0;
    long long base = 0;
    unsigned lane_b = 0;
    int row_b = 0;
    int xrows_left = 0;
    bool valid;
    if (AXIS == 0) {
        const int nrows = ny * nz;
        const int r0 = local * kTileLines;
        const int r = min(r0 + lane, nrows - 1);
        valid = r0 + lane < nrows;
        const int j = r % ny, k = r / ny;
        on = (j == 0 ? 1 << 2 : 0) | (j == ny - 1 ? 1 << 3 : 0) |
             (k == 0 ? 1 << 4 : 0) | (k == nz - 1 ? 1 << 5 : 0);
        base = S.base + (long long)r0 * nx;
        lane_b = (unsigned)(r - r0) * (unsigned)nx * 4u;
        row_b = nx * 4;
        xrows_left = nrows - r0;
    } else {
        const int no = (AXIS == 1) ? nz : ny;
        const int nlines = nx * no;
        const int L0 = local * kTileLines;
        const int L = min(L0 + lane, nlines - 1);
        valid = L0 + lane < nlines;
        const int i = L % nx, o = L / nx;
        on = (i == 0 ? 1 : 0) | (i == nx - 1 ? 2 : 0);
        long long start, start0;
        if (AXIS == 1) {
            on |= (o == 0 ? 1 << 4 : 0) | (o == nz - 1 ? 1 << 5 : 0);
            start = i + (long long)o * nx * ny;
            start0 = (L0 % nx) + (long long)(L0 / nx) * nx * ny;
            row_b = nx * 4;
        } else {
            on |= (o == 0 ? 1 << 2 : 0) | (o == ny - 1 ? 1 << 3 : 0);
            start = L;
            start0 = L0;
            row_b = nx * ny * 4;
        }
        base = S.base + start0;
        lane_b = (unsigned)(start - start0) * 4u;
    }
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(w + base, S.base + S.vol - base);
    const __amdgpu_buffer_rsrc_t ry = make_rsrc(raw + base, S.base + S.vol - base);
    const int wface = top_face(dmask & on);
    const int lo_f = (dmask >> (2 * AXIS)) & 1 ? 2 * AXIS : -1;
    const int hi_f = (dmask >> (2 * AXIS + 1)) & 1 ? 2 * AXIS + 1 : -1;
    const bool d_first = max(wface, max(lo_f, n == 1 ? hi_f : -1)) >= 0;  // row 0 is Dirichlet
    const bool d_last = max(wface, hi_f) >= 0;                            // row n-1 is Dirichlet
    const bool whole = wface >= 0;
    const bool any_whole = __builtin_amdgcn_ballot_w64(whole) != 0;
    // byte offset of local index t in this wave's direction, and of row m
    // (x: along the lane's own line; y, z: wave-uniform row offsets)
    const int step_b = (AXIS == 0) ? (top ? 4 : -4) : (top ? row_b : -row_b);
    const int first_b = top ? 0 : (n - 1) * ((AXIS == 0) ? 4 : row_b);
    const int mid_b = m * ((AXIS == 0) ? 4 : row_b);

    float v[CAP];

    // ---- load w (same paths as the forward sweep) ----
    if (AXIS == 0) {
        float *st = stage + wave * 64 * 65;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (c * 64 < nel) {
                const int cs = top ? c * 64 : n - 64 * (c + 1);
                const int col = top ? min(cs + lane, nel - 1) : max(cs + lane, n - cb);
                const unsigned cb4 = (unsigned)col * 4u;
                // the previous chunk's stage reads complete before the DMA
                // reuses the stage (LDS-DMA writes are not ordered after
                // earlier LDS reads)
                if (c > 0) __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
                for (int q = 0; q < 64; ++q)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void *)(st + q * 65), 4, (int)cb4,
                        min(q, xrows_left - 1) * row_b, 0, 0);
                __builtin_amdgcn_s_waitcnt(0);
                wave_sync_lds();
                if (top) {
#pragma unroll
                    for (int jj = 0; jj < 64; ++jj)
                        if (c * 64 + jj < CAP && c * 64 + jj < nel) v[c * 64 + jj] = st[lane * 65 + jj];
                } else {
#pragma unroll
                    for (int jj = 0; jj < 64; ++jj)
                        if (c * 64 + jj < CAP && c * 64 + jj < nel) v[c * 64 + jj] = st[lane * 65 + 63 - jj];
                }
                wave_sync_lds();
            }
        }
    } else {
        VL_FOR_UP(CAP, nel, t, v[t] = bload(rs, lane_b, first_b + t * step_b);)
    }
    __syncthreads();  // pivot table visible

    // ---- P_D^T on the input ----
    if (any_whole) VL_FOR_UP(CAP, nel, t, v[t] = whole ? 0.f : v[t];)
    if (top && m >= 1 && d_first) v[0] = 0.f;
    if (!top && cb >= 1 && d_last) v[0] = 0.f;

    double s_lam = 0.0, s_k = 0.0, s_sig = 0.0;
    // decay term of the x sweep: w_in^T y over this wave's rows
    if (AXIS == 0) VL_FOR_UP(CAP, nel, t, s_lam += (double)v[t] * (double)bload(ry, lane_b, first_b + t * step_b);)

    // ---- the solve (identical to the forward one) ----
    float prev = 0.f;
    VL_FOR_UP(CAP, nel, t, {
        const float2 c = cs_lds[t];
        prev = fmaf(c.y, prev, v[t] * c.x);
        v[t] = prev;
    })
    float xm = 0.f;
    if (!top) xch[0][lane] = prev;
    __syncthreads();
    if (top) {
        float rm = bload(rs, lane_b, mid_b);
        const bool d_mid = whole || (m == 0 && d_first);
        if (d_mid) rm = 0.f;
        if (AXIS == 0) s_lam += (double)rm * (double)bload(ry, lane_b, mid_b);
        xm = fmaf(g2, prev + xch[0][lane], rm * g1);
        xch[1][lane] = xm;
    }
    __syncthreads();
    if (!top) xm = xch[1][lane];
    float nxt = xm;
    VL_FOR_DOWN(CAP, nel, t, {
        nxt = fmaf(cs_lds[t].y, nxt, v[t]);
        v[t] = nxt;
    })

    // ---- parameter sums with the forward output y ----
    {
        const float ym = bload(ry, lane_b, mid_b);
        float yp = 0.f, wp = 0.f;  // previous local element
        VL_FOR_UP(CAP, nel, t, {
            const float yt = bload(ry, lane_b, first_b + t * step_b);
            s_sig -= (double)v[t] * (double)yt;
            if (t > 0) s_k -= ((double)v[t] - (double)wp) * ((double)yt - (double)yp);
            yp = yt;
            wp = v[t];
        })
        if (nel > 0) s_k -= ((double)xm - (double)wp) * ((double)ym - (double)yp);  // pair (last, middle)
        if (top) s_sig -= (double)xm * (double)ym;
    }

    // ---- P_D^T on the output, store ----
    if (any_whole) VL_FOR_UP(CAP, nel, t, v[t] = whole ? 0.f : v[t];)
    if (top) {
        if (m >= 1 && d_first) v[0] = 0.f;
        if (whole || (m == 0 && d_first)) xm = 0.f;
    } else if (cb >= 1 && d_last) {
        v[0] = 0.f;
    }
    if (top) bstore(rs, lane_b, mid_b, xm);
    VL_FOR_UP(CAP, nel, t, bstore(rs, lane_b, first_b + t * step_b, v[t]);)

    // ---- per-tile sums: clamped duplicate lanes do not count ----
    if (!valid) {
        s_lam = 0.0;
        s_k = 0.0;
        s_sig = 0.0;
    }
    s_k = wave_sum(s_k);
    s_sig = wave_sum(s_sig);
    s_lam = wave_sum(s_lam);
    if (lane == 0) {
        red[wave][0] = s_k;
        red[wave][1] = s_sig;
        red[wave][2] = s_lam;
    }
    __syncthreads();
    // each tile owns its slots and the reverse steps run in stream order, so
    // the running sum over steps needs no atomics
    if (threadIdx.x < 3) part[3 * (size_t)tile + threadIdx.x] += red[0][threadIdx.x] + red[1][threadIdx.x];
}

template <int AXIS, int CAP>
__global__ void __launch_bounds__(128)
adjoint_sweep(SweepLaunch L, const SubDev *__restrict__ subs, const float2 *__restrict__ coef,
              float *__restrict__ w, const float *__restrict__ raw, double *__restrict__ part)
{
    __shared__ TileLds<CAP, AXIS == 0, float2, float> sh;
    const int tile = blockIdx.x;
    const int slot = find_slot(L.tile_prefix, L.count, tile);
    const int local = tile - L.tile_prefix[slot];
    adjoint_tile<AXIS, CAP>(subs[L.sub_ids[slot]], local, tile, coef, w, raw, part, sh);
}

template <int AXIS>
static hipError_t launch_adj_axis(int cap_idx, const SweepLaunch &L, const SubDev *subs,
                                  const float2 *coef, float *w, const float *raw, double *part,
                                  hipStream_t st)
{
    const dim3 grid(L.total_tiles), block(128);
    switch (cap_idx) {
    case 0: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[0]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 1: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[1]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 2: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[2]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 3: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[3]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 4: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[4]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 5: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[5]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 6: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[6]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    case 7: hipLaunchKernelGGL((adjoint_sweep<AXIS, kCaps[7]>), grid, block, 0, st, L, subs, coef, w, raw, part); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_sweep(int axis, int cap_idx, const SweepLaunch &L, const SubDev *subs,
                                const float2 *coef, float *w, const float *raw, double *partials,
                                hipStream_t st)
{
    if (L.total_tiles <= 0) return hipSuccess;
    if (axis == 0) return launch_adj_axis<0>(cap_idx, L, subs, coef, w, raw, partials, st);
    if (axis == 1) return launch_adj_axis<1>(cap_idx, L, subs, coef, w, raw, partials, st);
    if (axis == 2) return launch_adj_axis<2>(cap_idx, L, subs, coef, w, raw, partials, st);
    return hipErrorInvalidValue;
}

// One thread per (volume of the launch, sum k): adds its tiles in order.
__global__ void reduce_partials_kernel(SweepLaunch L, int axis, const double *__restrict__ part,
                                       double *__restrict__ totals)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 3 * L.count) return;
    const int slot = g / 3, k = g % 3;
    double acc = 0.0;
    for (int t = L.tile_prefix[slot]; t < L.tile_prefix[slot + 1]; ++t) acc += part[3 * (size_t)t + k];
    totals[3 * (3 * (size_t)L.sub_ids[slot] + axis) + k] += acc;
}

hipError_t launch_reduce_partials(const SweepLaunch &L, int axis, const double *partials,
                                  double *totals, hipStream_t st)
{
    if (L.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((3 * L.count + 127) / 128), dim3(128), 0, st, L, axis,
                       partials, totals);
    return hipGetLastError();
}

// C^T at one occupied voxel and substrate.  The forward values after each
// cell are rebuilt from the value before the sources (rho) and recovered on
// the way back as rho_{i-1} = rho_i b_i - a_i.  For cell i, with w the
// adjoint of the value after it:
//   abar = w/b_i,  bbar = -w rho_i/b_i,  w <- w/b_i,
//   dS_i += abar (k_i rho*_i) + k_i bbar,  dU_i += k_i bbar
// (a = k S rho*, b = 1 + k (S + U)).  Each cell is in one voxel, so one
// thread owns each dS/dU entry.
__device__ __forceinline__ int find_slot_int(const int *__restrict__ prefix, int count, int x)
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

__global__ void sources_adjoint_kernel(const SimCells *__restrict__ cells, int nsims,
                                       const int *__restrict__ occ_prefix, int occ_bound,
                                       const SubDev *__restrict__ subs, const int *__restrict__ occ_vox_v,
                                       const int *__restrict__ seg_start, const double2 *__restrict__ ab,
                                       const double *__restrict__ krs, const double *__restrict__ kcell,
                                       const int *__restrict__ cell_of, const float *__restrict__ rho,
                                       float *__restrict__ w, const int *__restrict__ out_base,
                                       double *__restrict__ dS, double *__restrict__ dU)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= occ_bound || j >= occ_prefix[nsims]) return;  // past the occupied voxels
    const int sim = find_slot_int(occ_prefix, nsims, j);
    const SimCells &C = cells[sim];
    if (s >= C.ns) return;
    const int jl = j - occ_prefix[sim];
    const int v = occ_vox_v[C.occ_base + jl];
    const int p0 = seg_start[C.occ_base + jl], p1 = seg_start[C.occ_base + jl + 1];
    const long long at = subs[C.sub0 + s].base + v;
    double r = rho[at];
    for (int p = p0; p < p1; ++p) {
        const double2 e = ab[C.ab_base + (size_t)p * C.ns + s];
        r = (r + e.x) / e.y;
    }
    double wb = w[at];
    for (int p = p1 - 1; p >= p0; --p) {
        const double2 e = ab[C.ab_base + (size_t)p * C.ns + s];
        const double abar = wb / e.y;
        const double bbar = -wb * r / e.y;
        const double k = kcell[C.cell_base + p];
        const size_t o = (size_t)out_base[sim] + (size_t)cell_of[C.cell_base + p] * C.ns + s;
        dS[o] += abar * krs[C.ab_base + (size_t)p * C.ns + s] + k * bbar;
        dU[o] += k * bbar;
        wb = wb / e.y;
        r = r * e.y - e.x;
    }
    w[at] = (float)wb;
}

hipError_t launch_sources_adjoint(const SimCells *cells, int nsims, const int *occ_prefix, int occ_bound,
                                  int max_ns, const SubDev *subs, const int *occ_vox_v,
                                  const int *seg_start, const double2 *ab, const double *krs,
                                  const double *kcell, const int *cell_of, const float *rho, float *w,
                                  const int *cell_out_base, double *dS, double *dU, hipStream_t st)
{
    if (occ_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(sources_adjoint_kernel, dim3((unsigned)((occ_bound + 127LL) / 128), max_ns), dim3(128), 0, st, cells,
                       nsims, occ_prefix, occ_bound, subs, occ_vox_v, seg_start, ab, krs, kcell, cell_of, rho, w,
                       cell_out_base, dS, dU);
    return hipGetLastError();
}

}  // namespace vl
