// vl_sweep_xl.hip -- the x solve with lanes along the line.
//
// x-lines are contiguous, so instead of transposing 64 lines through LDS (one
// line per lane, as the split sweep does), lane l of a wave holds K
// consecutive voxels of ONE line (K = 4 for lines of 129-256 voxels, 8 up to
// 512, 9 for 513), loaded and stored with wide, fully coalesced buffer
// instructions.  The line matrix T = tridiag(-c, b, -c)
// is solved by substructuring:
//   * the last voxel of each lane's run is a separator; the voxels before it
//     form the lane's interval, eliminated locally (x_int = u + al*x_left +
//     be*x_own, u = T_int^-1 r_int, al/be = T_int^-1 of the couplings c);
//   * the separators satisfy a tridiagonal system over the lanes, A x_{l-1} +
//     B x_l + C x_{l+1} = r_sep + c*u_last + c*u_first(next lane), whose matrix
//     depends only on n, c and sigma: parallel cyclic reduction with
//     precomputed multipliers solves it in six levels of two lane shuffles;
//   * the intervals are completed from the separators.
// The result equals the line solve up to rounding (it is the same linear
// system; the order of operations differs from the split Thomas sweep).
// Decay (once per step) multiplies the solution by f; the Dirichlet projection
// before and after is applied as in the other sweeps.
#include <type_traits>

#include "vl_device.h"

namespace vl {

// ---------------------------------------------------------------------------
// Tables, FP64 arithmetic: one workgroup of 64 threads per volume, thread l =
// lane l.

__device__ __forceinline__ double xl_bdiag(int n, int row, double c, double sg)
{
    if (n == 1) return 1.0 + sg;
    return (row == 0 || row == n - 1) ? 1.0 + c + sg : 1.0 + 2.0 * c + sg;
}

__global__ void __launch_bounds__(64) xl_tables_kernel(const SubDev *__restrict__ subs, float *__restrict__ xl32,
                                                       double *__restrict__ xl64)
{
    __shared__ double sa[64], sb[64], sc[64];
    __shared__ double alf[64], ber[64];  // first al, first be of each lane's interval
    __shared__ int mm[64];
    const SubDev &S = subs[blockIdx.x];
    const int l = threadIdx.x;
    const int n = S.n[0];
    if (S.xlane < 0) return;  // uniform per block
    const int K = xl_k(n);
    const int P = (n + K - 1) / K;
    const double c = S.c[0], sg = S.sigma;
    float *T = xl32 + S.xlane;
    double *T64 = xl64 + S.xlane;
    const int nf = xl_fields(K);
    const bool act = l < P;
    const int s0 = K * l;
    const int e0 = act ? min(K * l + K - 1, n - 1) : 0;
    const int m = act ? e0 - s0 : 0;

    double inv[kXLaneMaxK - 1], ee[kXLaneMaxK - 1], al[kXLaneMaxK - 1], be[kXLaneMaxK - 1];
    for (int t = 0; t < kXLaneMaxK - 1; ++t) inv[t] = ee[t] = al[t] = be[t] = 0.0;
    double d = 0.0;
    for (int t = 0; t < m; ++t) {
        const double bt = xl_bdiag(n, s0 + t, c, sg);
        d = (t == 0) ? bt : bt - c * c / d;
        inv[t] = 1.0 / d;
        ee[t] = c / d;
    }
    // responses of the interval to a unit coupling c at its first / last row
    for (int pass = 0; pass < 2; ++pass) {
        if (m == 0 || (pass == 0 && l == 0)) continue;  // lane 0's interval has no left separator
        double y[kXLaneMaxK - 1];
        double prev = 0.0;
        for (int t = 0; t < m; ++t) {
            const double rhs = (pass == 0 ? t == 0 : t == m - 1) ? c : 0.0;
            prev = (rhs + c * prev) * inv[t];
            y[t] = prev;
        }
        double nxt = 0.0;
        for (int t = m - 1; t >= 0; --t) {
            nxt = y[t] + ee[t] * nxt;
            (pass == 0 ? al : be)[t] = nxt;
        }
    }
    mm[l] = m;
    alf[l] = al[0];
    ber[l] = be[0];
    __syncthreads();
    // the reduced system of the separators
    double A = 0.0, B = 1.0, C = 0.0;
    if (act) {
        const int mn = (l + 1 < P) ? mm[l + 1] : 0;
        B = xl_bdiag(n, e0, c, sg);
        if (e0 >= 1) {
            if (m > 0) {
                B -= c * be[m - 1];
                A = (l > 0) ? -c * al[m - 1] : 0.0;
            } else {
                A = -c;  // the row before is the previous separator
            }
        }
        if (e0 <= n - 2) {
            if (mn > 0) {
                B -= c * alf[l + 1];
                C = -c * ber[l + 1];
            } else {
                C = -c;
            }
        }
        T[(4 * (K - 1) + 2 * kXLaneLevels + 1) * 64 + l] = (m > 0) ? (float)c : 0.f;   // cprev
        T[(4 * (K - 1) + 2 * kXLaneLevels + 2) * 64 + l] = (mn > 0) ? (float)c : 0.f;  // cnext
        T64[(4 * (K - 1) + 2 * kXLaneLevels + 1) * 64 + l] = (m > 0) ? c : 0.0;
        T64[(4 * (K - 1) + 2 * kXLaneLevels + 2) * 64 + l] = (mn > 0) ? c : 0.0;
    } else {
        T[(4 * (K - 1) + 2 * kXLaneLevels + 1) * 64 + l] = 0.f;
        T[(4 * (K - 1) + 2 * kXLaneLevels + 2) * 64 + l] = 0.f;
        T64[(4 * (K - 1) + 2 * kXLaneLevels + 1) * 64 + l] = 0.0;
        T64[(4 * (K - 1) + 2 * kXLaneLevels + 2) * 64 + l] = 0.0;
    }
    for (int t = 0; t < K - 1; ++t) {
        T[(0 * (K - 1) + t) * 64 + l] = (float)inv[t];
        T[(1 * (K - 1) + t) * 64 + l] = (float)ee[t];
        T[(2 * (K - 1) + t) * 64 + l] = (float)al[t];
        T[(3 * (K - 1) + t) * 64 + l] = (float)be[t];
        T64[(0 * (K - 1) + t) * 64 + l] = inv[t];
        T64[(1 * (K - 1) + t) * 64 + l] = ee[t];
        T64[(2 * (K - 1) + t) * 64 + l] = al[t];
        T64[(3 * (K - 1) + t) * 64 + l] = be[t];
    }
    // parallel cyclic reduction: level v eliminates the couplings at distance 2^v
    sa[l] = A;
    sb[l] = B;
    sc[l] = C;
    __syncthreads();
    for (int v = 0; v < kXLaneLevels; ++v) {
        const int s = 1 << v;
        double k1 = 0.0, k2 = 0.0, na = 0.0, nb = sb[l], nc = 0.0;
        if (act) {
            if (l - s >= 0) {
                k1 = sa[l] / sb[l - s];
                na = -k1 * sa[l - s];
                nb -= k1 * sc[l - s];
            }
            if (l + s < P) {
                k2 = sc[l] / sb[l + s];
                nc = -k2 * sc[l + s];
                nb -= k2 * sa[l + s];
            }
        }
        __syncthreads();
        sa[l] = na;
        sb[l] = nb;
        sc[l] = nc;
        T[(4 * (K - 1) + 2 * v) * 64 + l] = (float)k1;
        T[(4 * (K - 1) + 2 * v + 1) * 64 + l] = (float)k2;
        T64[(4 * (K - 1) + 2 * v) * 64 + l] = k1;
        T64[(4 * (K - 1) + 2 * v + 1) * 64 + l] = k2;
        __syncthreads();
    }
    T[(4 * (K - 1) + 2 * kXLaneLevels) * 64 + l] = act ? (float)(1.0 / sb[l]) : 0.f;
    T64[(4 * (K - 1) + 2 * kXLaneLevels) * 64 + l] = act ? 1.0 / sb[l] : 0.0;
    (void)nf;
}

hipError_t launch_xl_tables(const SubDev *subs, int nsubs, const float2 *, float *xl32, double *xl64, hipStream_t st)
{
    if (nsubs <= 0 || !xl32 || !xl64) return hipSuccess;
    hipLaunchKernelGGL(xl_tables_kernel, dim3(nsubs), dim3(64), 0, st, subs, xl32, xl64);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The sweep.  The launch covers tiles of 64 x-lines (the split sweep's
// tiling); 16 / lpw workgroups of four waves share a tile, and each wave
// solves lpw consecutive lines one after another, with the loads of the next
// three lines issued before the current line is solved.  Fewer lines per wave
// make more, shorter-lived workgroups (a shorter tail at the end of the
// launch); more lines per wave hide more load latency within a wave.

template <int K>
__device__ __forceinline__ void xl_load(float (&r)[K], __amdgpu_buffer_rsrc_t rs, unsigned voff)
{
    int t = 0;
#pragma unroll
    for (; t + 4 <= K; t += 4) {
        const vl_u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(voff + 4u * t), 0, 0);
        r[t] = __uint_as_float(q.x);
        r[t + 1] = __uint_as_float(q.y);
        r[t + 2] = __uint_as_float(q.z);
        r[t + 3] = __uint_as_float(q.w);
    }
    if (t + 2 <= K) {
        const vl_u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(voff + 4u * t), 0, 0);
        r[t] = __uint_as_float(q.x);
        r[t + 1] = __uint_as_float(q.y);
        t += 2;
    }
    if (t < K) r[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(voff + 4u * t), 0, 0));
}

template <int K>
__device__ __forceinline__ void xl_store(const float (&o)[K], __amdgpu_buffer_rsrc_t rs, unsigned voff, int cnt)
{
    if (cnt == K) {
        int t = 0;
#pragma unroll
        for (; t + 4 <= K; t += 4)
            __builtin_amdgcn_raw_buffer_store_b128(
                vl_u32x4{__float_as_uint(o[t]), __float_as_uint(o[t + 1]), __float_as_uint(o[t + 2]),
                         __float_as_uint(o[t + 3])},
                rs, (int)(voff + 4u * t), 0, 0);
        if (t + 2 <= K) {
            __builtin_amdgcn_raw_buffer_store_b64(vl_u32x2{__float_as_uint(o[t]), __float_as_uint(o[t + 1])}, rs,
                                                  (int)(voff + 4u * t), 0, 0);
            t += 2;
        }
        if (t < K) bstore(rs, voff + 4u * t, 0, o[t]);
    } else {
#pragma unroll
        for (int t = 0; t < K; ++t)
            if (t < cnt) bstore(rs, voff + 4u * t, 0, o[t]);
    }
}

constexpr int kXlAhead = 3;

template <int K, bool CARRY>
__global__ void __launch_bounds__(256)
sweep_xl(SweepLaunch L, int lpw, const SubDev *__restrict__ subs, const double *__restrict__ xl64,
         float *__restrict__ field, float *__restrict__ raw, CarriedSources carry)
{
    // per wave: which of a lane's voxels receive a carried source, and the
    // composites by voxel of the line
    __shared__ unsigned cs_mask[4][CARRY ? 64 : 1];
    __shared__ float2 cs_ab[4][CARRY ? 64 * K : 1];
    // the volume's interval tables (FP64), field-major, three columns: lane
    // 0, the middle lanes, the last active lane
    __shared__ double xl_int[K > 1 ? 4 * (K - 1) * 3 : 1];
    constexpr int KM = K > 1 ? K - 1 : 1;
    const int parts = (kTileLines / 4) / lpw;  // workgroups per tile
    const int blk = L.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int tile = blk / parts, part = blk - tile * parts;
    const int slot = find_slot(L.tile_prefix, L.count, tile);
    const int local = tile - L.tile_prefix[slot];
    const SubDev &S = subs[L.sub_ids[slot]];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int n = nx;
    const int P = (n + K - 1) / K;
    const bool act = lane < P;
    const int m = act ? min(K * lane + K - 1, n - 1) - K * lane : 0;  // interval length
    const int cnt = act ? m + 1 : 0;                                   // voxels of this lane
    const int nrows = ny * nz;
    const int row0 = local * kTileLines + (part * 4 + wave) * lpw;
    const int dmask = S.dir_mask;
    const int lo_f = (dmask & 1) ? 0 : -1;
    const int hi_f = (dmask & 2) ? 1 : -1;
    const double fdec = S.fdec;

    // The solve's arithmetic is FP64 (tables included); only the line's
    // values and the interval results it keeps between phases are FP32:
    // rounding inside FP32 recurrences is coherent across neighbouring lines
    // and steps and accumulates like a bias.  The interval tables (4(K-1)
    // FP64 values per lane) live in LDS, read per line, which keeps the
    // kernel at four waves per SIMD; the reduction's multipliers stay in
    // registers.  Lanes 1 .. P-2 each hold an interval of K-1 inner rows of
    // the line, so their tables are equal; only lane 0 (whose interval starts
    // at the line's first row) and lane P-1 (whose interval is shorter when n
    // is not a multiple of K) differ.  So LDS keeps three columns and every
    // table read is a near-broadcast (three addresses per wave).
    const double *__restrict__ T = xl64 + S.xlane;
    for (int e = threadIdx.x; e < 4 * (K - 1) * 3; e += 256) {
        const int col = e % 3;
        xl_int[e] = T[(e / 3) * 64 + (col == 0 ? 0 : col == 1 ? min(1, P - 1) : P - 1)];
    }
    __syncthreads();
    const int tcol = lane == 0 ? 0 : (lane < P - 1 ? 1 : 2);
    // Read at each use: the column index carries a per-line term that is
    // zero (line indices stay below 2^28) but that the compiler cannot prove
    // zero, so the reads are not hoisted out of the line loop into registers.
    auto inv = [&](int tl, int t) { return K > 1 ? xl_int[(0 * (K - 1) + t) * 3 + tl] : 0.0; };
    auto ee = [&](int tl, int t) { return K > 1 ? xl_int[(1 * (K - 1) + t) * 3 + tl] : 0.0; };
    auto al = [&](int tl, int t) { return K > 1 ? xl_int[(2 * (K - 1) + t) * 3 + tl] : 0.0; };
    auto be = [&](int tl, int t) { return K > 1 ? xl_int[(3 * (K - 1) + t) * 3 + tl] : 0.0; };
    double k1[kXLaneLevels], k2[kXLaneLevels];
#pragma unroll
    for (int v = 0; v < kXLaneLevels; ++v) {
        k1[v] = T[(4 * (K - 1) + 2 * v) * 64 + lane];
        k2[v] = T[(4 * (K - 1) + 2 * v + 1) * 64 + lane];
    }
    const double binv = T[(4 * (K - 1) + 2 * kXLaneLevels) * 64 + lane];
    const double cprev = T[(4 * (K - 1) + 2 * kXLaneLevels + 1) * 64 + lane];
    const double cnext = T[(4 * (K - 1) + 2 * kXLaneLevels + 2) * 64 + lane];

    const __amdgpu_buffer_rsrc_t rs = make_rsrc(field + S.base, S.vol);
    const __amdgpu_buffer_rsrc_t rr = make_rsrc(raw ? raw + S.base : field + S.base, S.vol);
    const unsigned lane_b = (unsigned)(K * lane) * 4u;

    // Dirichlet values and which lanes they go to, fixed for the launch, so
    // that the per-line code below has no divergent branches
    const float fv0 = S.dval32[0], fv1 = S.dval32[1], fv2 = S.dval32[2], fv3 = S.dval32[3], fv4 = S.dval32[4],
                fv5 = S.dval32[5];
    auto fval = [&](int f) {  // value of face f (uniform), 0 <= f < 6
        return f == 5 ? fv5 : f == 4 ? fv4 : f == 3 ? fv3 : f == 2 ? fv2 : f == 1 ? fv1 : fv0;
    };
    const int f_in_lo = n == 1 ? max(lo_f, hi_f) : lo_f;  // before the solve, first voxel
    const float v_in_lo = fval(f_in_lo);
    const bool set_in_lo = lane == 0 && f_in_lo >= 0;
    const bool set_in_hi = n > 1 && hi_f >= 0 && lane == P - 1;  // before the solve, last voxel
    const float v_in_hi = fv1;
    const bool last_lane = n > 1 && lane == P - 1;

    // A lane's byte offset of a line, or one past any buffer when the line is
    // not to be touched: buffer loads there return 0 and stores are dropped
    // by the hardware's range check, so no lane needs a branch around them.
    constexpr unsigned kOff = 0x80000000u;
    auto line_off = [&](int row, bool want) -> unsigned {
        return (want && act) ? (unsigned)row * (unsigned)nx * 4u + lane_b : kOff;
    };

    // Lane addresses of the shuffles, fixed for the launch; as with
    // __shfl_up / __shfl_down, a lane with no source lane reads its own value.
    int a_up[kXLaneLevels], a_dn[kXLaneLevels];
#pragma unroll
    for (int v = 0; v < kXLaneLevels; ++v) {
        const int s = 1 << v;
        a_up[v] = (lane >= s ? lane - s : lane) << 2;
        a_dn[v] = (lane + s < 64 ? lane + s : lane) << 2;
    }
    auto from_lane = [](int addr, float x) {
        return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
    };
    auto from_lane_d = [](int addr, double x) {
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
        const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    };
    // cell sources of the previous step carried into this solve (uniform):
    // each x-line's range [e0, e1) of the voxel-ordered occupied voxels, the
    // voxels, and their FP32 composites (P, R) of this substrate (one
    // contiguous run per substrate)
    const SimCells *CC = CARRY ? &carry.cells[S.sim] : nullptr;
    const bool carried = CC != nullptr && CC->xs_base >= 0;
    const int c_occ = carried ? CC->n_occ : 0;
    const __amdgpu_buffer_rsrc_t xs_r =
        make_rsrc(carried ? (const float *)(carry.xline_start + CC->xs_base) : field, carried ? nrows + 1 : 0);
    const __amdgpu_buffer_rsrc_t ov_r =
        make_rsrc(carried ? (const float *)(carry.occ_vox_v + CC->occ_base) : field, c_occ);
    const __amdgpu_buffer_rsrc_t ab_r =
        make_rsrc(carried ? (const float *)(carry.comp_v + CC->comp_base + (size_t)S.sub * CC->occ_cap) : field,
                  2LL * c_occ);
    // a line's range (0, 0 for a line not to be touched)
    auto load_range = [&](int row, bool want) -> vl_u32x2 {
        return __builtin_amdgcn_raw_buffer_load_b64(xs_r, (int)(want ? (unsigned)row * 4u : kOff), 0, 0);
    };
    // this lane's entry of the chunk starting at c0 (voxel, composite)
    auto load_entry = [&](int c0, int e1, int &vox, float2 &ab) {
        const int e = c0 + lane;
        const bool ok = e < e1;
        vox = (int)__builtin_amdgcn_raw_buffer_load_b32(ov_r, (int)(ok ? (unsigned)e * 4u : kOff), 0, 0);
        const vl_u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(ab_r, (int)(ok ? (unsigned)e * 8u : kOff), 0, 0);
        ab = make_float2(__uint_as_float(q.x), __uint_as_float(q.y));
    };
    // rho <- rho R + P on the occupied voxels of the chunk: each
    // entry's lane writes its composite to the wave's LDS slot of that voxel
    // and marks the voxel in its owner lane's mask; owners then update their
    // registers.  Lanes talk through LDS here: the wavefront-scope fences keep
    // the compiler from moving these accesses across the phases (or
    // forwarding a lane's own cleared mask to its read); the wave's LDS
    // operations themselves execute in order.
    auto apply_chunk = [&](bool ok, int i, float2 ab, float (&r)[K]) {
        cs_mask[wave][lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (ok) {
            atomicOr(&cs_mask[wave][i / K], 1u << (i % K));
            cs_ab[wave][i] = ab;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const unsigned mk = cs_mask[wave][lane];
#pragma unroll
        for (int t = 0; t < K; ++t)
            if (mk & (1u << t)) {
                const float2 q = cs_ab[wave][K * lane + t];
                r[t] = fmaf(r[t], q.y, q.x);
            }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    // the line's carried sources: the first 64 entries were loaded ahead with
    // the line, any further ones are loaded here
    auto carry_in = [&](const int row, float (&r)[K], vl_u32x2 rg, int vox0, float2 ab0) {
        const int e0 = __builtin_amdgcn_readfirstlane((int)rg.x), e1 = __builtin_amdgcn_readfirstlane((int)rg.y);
        if (e1 <= e0) return;  // uniform
        apply_chunk(e0 + lane < e1, vox0 - row * nx, ab0, r);
        for (int c0 = e0 + 64; c0 < e1; c0 += 64) {  // uniform
            int vox;
            float2 ab;
            load_entry(c0, e1, vox, ab);
            apply_chunk(c0 + lane < e1, vox - row * nx, ab, r);
        }
    };

    // faces of the first and last voxel of a line on no y/z Dirichlet face
    const int f_first0 = max(lo_f, n == 1 ? hi_f : -1), f_last0 = hi_f;
    const float v_first0 = fval(f_first0), v_last0 = fval(f_last0);

    // One line.  With FULL (n a multiple of K) every active lane holds K
    // voxels, so the per-lane interval length is the constant K - 1.
    auto solve_line = [&](auto full_c, auto carry_c, const int row, const int j, const int k, float (&r)[K],
                          vl_u32x2 rg, int vox0, float2 ab0) {
        constexpr bool FULL = decltype(full_c)::value;
        const int mm = FULL ? K - 1 : m;
        const int tl = tcol + ((row >> 30) << 2);  // the table column
        if (decltype(carry_c)::value) carry_in(row, r, rg, vox0, ab0);
        // Dirichlet projection before the solve: the end voxels of the line
        r[0] = set_in_lo ? v_in_lo : r[0];
#pragma unroll
        for (int t = 0; t < K; ++t) r[t] = (set_in_hi && t == mm) ? v_in_hi : r[t];

        // the lane's interval: u = T_int^-1 r_int (FP64 recurrences; the
        // eliminated values and u are kept in FP32)
        float u[KM];
        {
            float y[KM];
            double prev = 0.0;
#pragma unroll
            for (int t = 0; t < K - 1; ++t) {
                prev = fma(ee(tl, t), prev, (double)r[t] * inv(tl, t));
                y[t] = t < mm ? (float)prev : 0.f;
            }
            double nxt = 0.0;
#pragma unroll
            for (int t = K - 2; t >= 0; --t) {
                nxt = t < mm ? fma(ee(tl, t), nxt, (double)y[t]) : 0.0;
                u[t] = (float)nxt;
            }
            if (K == 1) u[0] = 0.f;
        }
        // the separator's right-hand side
        float rsep = r[0], ulast = 0.f;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if (t == mm) rsep = r[t];
#pragma unroll
        for (int t = 0; t < K - 1; ++t)
            if (t == mm - 1) ulast = u[t];
        const float ufirst_next = from_lane(a_dn[0], u[0]);
        double d = act ? fma(cnext, (double)ufirst_next, fma(cprev, (double)ulast, (double)rsep)) : 0.0;
        // parallel cyclic reduction over the lanes (a level whose distance
        // reaches past the last lane has zero multipliers)
#pragma unroll
        for (int v = 0; v < kXLaneLevels; ++v) {
            const double dl = from_lane_d(a_up[v], d);
            const double dr = from_lane_d(a_dn[v], d);
            d = fma(-k2[v], dr, fma(-k1[v], dl, d));
        }
        const double xs = d * binv;
        const double xl = from_lane_d(a_up[0], xs);
        // the lane's voxels; decay once per step after the x solve
        float o[K];
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double xi = (t < K - 1 && t < mm)
                                  ? fma(be(tl, t < KM ? t : 0), xs, fma(al(tl, t < KM ? t : 0), xl, (double)u[t < KM ? t : 0]))
                                  : xs;
            o[t] = (float)(xi * fdec);
        }
        const unsigned voff = line_off(row, true);
        if (raw) {  // uniform
            if (FULL) xl_store<K>(o, rr, voff, K);
            else if (act) xl_store<K>(o, rr, voff, cnt);
        }
        // Dirichlet projection after the solve: whole line on a y/z face, then
        // the ends on the x faces (the last active face in x-, x+, y-, y+, z-,
        // z+ order wins); the faces are uniform across the wave
        const int on = (j == 0 ? 1 << 2 : 0) | (j == ny - 1 ? 1 << 3 : 0) | (k == 0 ? 1 << 4 : 0) |
                       (k == nz - 1 ? 1 << 5 : 0);
        const int wface = top_face(dmask & on);
        int f_first = f_first0, f_last = f_last0;
        float v_first = v_first0, v_last = v_last0;
        if (wface >= 0) {  // uniform
            const float wv = fval(wface);
#pragma unroll
            for (int t = 0; t < K; ++t) o[t] = wv;
            f_first = max(wface, f_first0);
            f_last = max(wface, f_last0);
            v_first = fval(f_first);
            v_last = fval(f_last);
        }
        o[0] = (lane == 0 && f_first >= 0) ? v_first : o[0];
#pragma unroll
        for (int t = 0; t < K; ++t) o[t] = (last_lane && f_last >= 0 && t == mm) ? v_last : o[t];
        if (FULL) xl_store<K>(o, rs, voff, K);
        else if (act) xl_store<K>(o, rs, voff, cnt);
    };

    // A ring of kXlAhead + 1 line slots, unrolled so that every slot has
    // fixed registers: before line l is solved, the load of line
    // l + kXlAhead goes into the slot that line l - 1 used (free by then), so
    // kXlAhead loads stay in flight behind every solve.  Lanes with no voxels
    // load from past the buffer and read zeros.  With carried sources a slot
    // also holds its line's entry range (loaded with the line) and this
    // lane's first entry (loaded one line later, once the range is in).
    auto run = [&](auto full_c, auto carry_c) {
        constexpr bool CL = decltype(carry_c)::value;
        constexpr int NS = kXlAhead + 1;
        const int kLines = lpw;
        int j = row0 % ny, k = row0 / ny;  // the line being solved
        float rn[NS][K];
        vl_u32x2 rg[NS];
        int ev[NS];
        float2 eab[NS];
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            rg[a] = vl_u32x2{0u, 0u};
            ev[a] = 0;
            eab[a] = make_float2(0.f, 1.f);
        }
#pragma unroll
        for (int a = 0; a < kXlAhead; ++a) {
            const bool want = a < kLines && row0 + a < nrows;
            xl_load<K>(rn[a], rs, line_off(row0 + a, want));
            if (CL) rg[a] = load_range(row0 + a, want);
        }
        if (CL)
#pragma unroll
            for (int a = 0; a + 1 < kXlAhead; ++a) load_entry((int)rg[a].x, (int)rg[a].y, ev[a], eab[a]);
        for (int g = 0; g < kLines; g += NS) {
#pragma unroll
            for (int a = 0; a < NS; ++a) {
                const int row = row0 + g + a;
                const int nrow = row + kXlAhead;
                const bool want = g + a + kXlAhead < kLines && nrow < nrows;
                xl_load<K>(rn[(a + kXlAhead) % NS], rs, line_off(nrow, want));
                if (CL) {
                    rg[(a + kXlAhead) % NS] = load_range(nrow, want);
                    const int sm = (a + kXlAhead - 1) % NS;  // the line after this one
                    load_entry((int)rg[sm].x, (int)rg[sm].y, ev[sm], eab[sm]);
                }
                if (g + a < kLines && row < nrows) {  // wave-uniform
                    solve_line(full_c, carry_c, row, j, k, rn[a], rg[a], ev[a], eab[a]);
                    if (++j == ny) {
                        j = 0;
                        ++k;
                    }
                }
            }
        }
    };
    if constexpr (CARRY) {
        if (carried) {
            if (n % K == 0) run(std::true_type{}, std::true_type{});
            else run(std::false_type{}, std::true_type{});
            return;
        }
    }
    if (n % K == 0) run(std::true_type{}, std::false_type{});
    else run(std::false_type{}, std::false_type{});
}

hipError_t launch_sweep_xl(int K, int lpw, const SweepLaunch &L, const SubDev *subs, const double *xl64,
                           float *field, float *raw, const CarriedSources &carry, hipStream_t st)
{
    if (L.total_tiles <= 0) return hipSuccess;
    if (lpw < 1 || lpw > kTileLines / 4 || (kTileLines / 4) % lpw != 0) return hipErrorInvalidValue;
    const long long blocks = (long long)L.total_tiles * ((kTileLines / 4) / lpw);
    if (blocks >= (1ll << 31)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(256);
    switch (K) {
#define VL_XL_CASE(k)                                                                                  \
    case k:                                                                                            \
        if (carry.enabled)                                                                             \
            hipLaunchKernelGGL((sweep_xl<k, true>), grid, block, 0, st, L, lpw, subs, xl64, field, raw, carry); \
        else                                                                                           \
            hipLaunchKernelGGL((sweep_xl<k, false>), grid, block, 0, st, L, lpw, subs, xl64, field, raw, carry); \
        break;
        VL_XL_CASE(1)
        VL_XL_CASE(2)
        VL_XL_CASE(4)
        VL_XL_CASE(8)
        VL_XL_CASE(9)
#undef VL_XL_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vl
