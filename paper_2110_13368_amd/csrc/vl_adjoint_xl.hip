// vl_adjoint_xl.hip -- the reverse x solve of the adjoint with the lanes of a
// wave along the line.
//
// The reverse of F S_x P_D is P_D^T (f T^-1) P_D^T: T is symmetric, so the
// transposed solve is the forward one (the substructured solve of
// vl_sweep_xl.hip: each lane eliminates its run of K voxels, the runs' last
// voxels form a tridiagonal system over the lanes solved by parallel cyclic
// reduction with the same FP64-built multipliers), followed by the decay
// factor f.  Alongside, with y the forward x solve's output as the replay
// stored it (f included, before its Dirichlet store), each lane sums in FP64
//   s_k   -= (w_{i+1} - w_i)(y_{i+1} - y_i)   over neighbouring pairs,
//   s_sig -= w_out . y,     s_lam += w_in . y,
// the pair that straddles two lanes taken by the left lane.  One workgroup
// takes one tile of 64 lines (16 per wave) and adds its sums to the tile's
// partial slots, as the split reverse kernel does, so the per-volume totals
// are reduced the same way and stay deterministic.
#include "vl_device.h"

namespace vl {

namespace {

constexpr unsigned kOob = 0x80000000u;  // offset past any buffer: loads read 0, stores are dropped

template <int K>
__device__ __forceinline__ void axl_load(float (&r)[K], __amdgpu_buffer_rsrc_t rs, unsigned voff)
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
__device__ __forceinline__ void axl_store(const float (&o)[K], __amdgpu_buffer_rsrc_t rs, unsigned voff, int cnt,
                                          bool full)
{
    if (full) {
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

__device__ __forceinline__ double axl_wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

}  // namespace

template <int K>
__global__ void __launch_bounds__(256)
adjoint_xl(SweepLaunch L, const SubDev *__restrict__ subs, const float *__restrict__ xl32, float *__restrict__ w,
           const float *__restrict__ raw, double *__restrict__ part)
{
    constexpr int KM = K > 1 ? K - 1 : 1;
    constexpr int kLines = kTileLines / 4;  // lines per wave: one workgroup per tile
    __shared__ double red[4][3];
    const int tile = (int)blockIdx.x;
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
    const bool full = n % K == 0;
    const int nrows = ny * nz;
    const int row0 = local * kTileLines + wave * kLines;
    const int dmask = S.dir_mask;
    const int lo_f = (dmask & 1) ? 0 : -1;
    const int hi_f = (dmask & 2) ? 1 : -1;
    const float fdec = (float)S.fdec;
    // x-face ends that P_D^T zeroes (a whole line on a y/z face is zeroed too)
    const bool zero_first = lane == 0 && max(lo_f, n == 1 ? hi_f : -1) >= 0;
    const bool zero_last = n > 1 && hi_f >= 0 && lane == P - 1;
    const bool pair_next = lane + 1 < P;  // this lane's last voxel has a right neighbour

    const float *__restrict__ T = xl32 + S.xlane;
    float inv[KM], ee[KM], al[KM], be[KM], k1[kXLaneLevels], k2[kXLaneLevels];
#pragma unroll
    for (int t = 0; t < KM; ++t) {
        inv[t] = K > 1 ? T[(0 * (K - 1) + t) * 64 + lane] : 0.f;
        ee[t] = K > 1 ? T[(1 * (K - 1) + t) * 64 + lane] : 0.f;
        al[t] = K > 1 ? T[(2 * (K - 1) + t) * 64 + lane] : 0.f;
        be[t] = K > 1 ? T[(3 * (K - 1) + t) * 64 + lane] : 0.f;
    }
#pragma unroll
    for (int v = 0; v < kXLaneLevels; ++v) {
        k1[v] = T[(4 * (K - 1) + 2 * v) * 64 + lane];
        k2[v] = T[(4 * (K - 1) + 2 * v + 1) * 64 + lane];
    }
    const float binv = T[(4 * (K - 1) + 2 * kXLaneLevels) * 64 + lane];
    const float cprev = T[(4 * (K - 1) + 2 * kXLaneLevels + 1) * 64 + lane];
    const float cnext = T[(4 * (K - 1) + 2 * kXLaneLevels + 2) * 64 + lane];
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

    const __amdgpu_buffer_rsrc_t rw = make_rsrc(w + S.base, S.vol);
    const __amdgpu_buffer_rsrc_t ry = make_rsrc(raw + S.base, S.vol);
    const unsigned lane_b = (unsigned)(K * lane) * 4u;
    auto line_off = [&](int row, bool want) -> unsigned {
        return (want && act) ? (unsigned)row * (unsigned)nx * 4u + lane_b : kOob;
    };

    double s_k = 0.0, s_sig = 0.0, s_lam = 0.0;
    auto reverse_line = [&](const int row, const int j, const int k, float (&r)[K], const float (&y)[K]) {
        // P_D^T on the input
        const int on = (j == 0 ? 1 << 2 : 0) | (j == ny - 1 ? 1 << 3 : 0) | (k == 0 ? 1 << 4 : 0) |
                       (k == nz - 1 ? 1 << 5 : 0);
        const bool whole = (dmask & on) != 0;  // uniform
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const bool z = whole || (t == 0 && zero_first) || (t == m && zero_last);
            r[t] = z ? 0.f : r[t];
        }
#pragma unroll
        for (int t = 0; t < K; ++t)
            if (t < cnt) s_lam += (double)r[t] * (double)y[t];

        // the solve (as the forward x solve)
        float u[KM];
        {
            float yy[KM];
            float prev = 0.f;
#pragma unroll
            for (int t = 0; t < K - 1; ++t) {
                prev = fmaf(ee[t], prev, r[t] * inv[t]);
                yy[t] = t < m ? prev : 0.f;
            }
            float nxt = 0.f;
#pragma unroll
            for (int t = K - 2; t >= 0; --t) {
                nxt = t < m ? fmaf(ee[t], nxt, yy[t]) : 0.f;
                u[t] = nxt;
            }
            if (K == 1) u[0] = 0.f;
        }
        float rsep = r[0], ulast = 0.f;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if (t == m) rsep = r[t];
#pragma unroll
        for (int t = 0; t < K - 1; ++t)
            if (t == m - 1) ulast = u[t];
        const float ufirst_next = from_lane(a_dn[0], u[0]);
        float d = act ? fmaf(cnext, ufirst_next, fmaf(cprev, ulast, rsep)) : 0.f;
#pragma unroll
        for (int v = 0; v < kXLaneLevels; ++v) {
            const float dl = from_lane(a_up[v], d);
            const float dr = from_lane(a_dn[v], d);
            d = fmaf(-k2[v], dr, fmaf(-k1[v], dl, d));
        }
        const float xs = d * binv;
        const float xl = from_lane(a_up[0], xs);
        float o[K];
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const float xi =
                (t < K - 1 && t < m) ? fmaf(be[t < KM ? t : 0], xs, fmaf(al[t < KM ? t : 0], xl, u[t < KM ? t : 0]))
                                     : xs;
            o[t] = act ? xi * fdec : 0.f;
        }

        // parameter sums with the forward output y
        const float o_next = from_lane(a_dn[0], o[0]);
        const float y_next = from_lane(a_dn[0], y[0]);
#pragma unroll
        for (int t = 0; t < K; ++t) {
            if (t < cnt) s_sig -= (double)o[t] * (double)y[t];
            if (t + 1 < K && t < m) s_k -= ((double)o[t + 1] - (double)o[t]) * ((double)y[t + 1] - (double)y[t]);
            if (t == m && pair_next) s_k -= ((double)o_next - (double)o[t]) * ((double)y_next - (double)y[t]);
        }

        // P_D^T on the output, store
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const bool z = whole || (t == 0 && zero_first) || (t == m && zero_last);
            o[t] = z ? 0.f : o[t];
        }
        axl_store<K>(o, rw, line_off(row, true), cnt, full);
    };
    // A ring of three line slots (w and y), unrolled so that each slot has
    // fixed registers: before line l is reversed, the loads of line l + 2 go
    // into the slot that line l - 1 used.
    constexpr int kAhead = 2, NS = kAhead + 1;
    int j = row0 % ny, k = row0 / ny;
    float rw_[NS][K], ry_[NS][K];
#pragma unroll
    for (int a = 0; a < kAhead; ++a) {
        const bool want = a < kLines && row0 + a < nrows;
        axl_load<K>(rw_[a], rw, line_off(row0 + a, want));
        axl_load<K>(ry_[a], ry, line_off(row0 + a, want));
    }
    for (int g = 0; g < kLines; g += NS) {
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const int row = row0 + g + a;
            const int nrow = row + kAhead;
            const bool want = g + a + kAhead < kLines && nrow < nrows;
            axl_load<K>(rw_[(a + kAhead) % NS], rw, line_off(nrow, want));
            axl_load<K>(ry_[(a + kAhead) % NS], ry, line_off(nrow, want));
            if (g + a < kLines && row < nrows) {  // wave-uniform
                reverse_line(row, j, k, rw_[a], ry_[a]);
                if (++j == ny) {
                    j = 0;
                    ++k;
                }
            }
        }
    }

    s_k = axl_wave_sum(s_k);
    s_sig = axl_wave_sum(s_sig);
    s_lam = axl_wave_sum(s_lam);
    if (lane == 0) {
        red[wave][0] = s_k;
        red[wave][1] = s_sig;
        red[wave][2] = s_lam;
    }
    __syncthreads();
    // each tile owns its slots and the reverse steps run in stream order
    if (threadIdx.x < 3)
        part[3 * (size_t)tile + threadIdx.x] +=
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

hipError_t launch_adjoint_xl(int K, const SweepLaunch &L, const SubDev *subs, const float *xl32, float *w,
                             const float *raw, double *part, hipStream_t st)
{
    if (L.total_tiles <= 0) return hipSuccess;
    const dim3 grid(L.total_tiles), block(256);
    switch (K) {
    case 1: hipLaunchKernelGGL((adjoint_xl<1>), grid, block, 0, st, L, subs, xl32, w, raw, part); break;
    case 2: hipLaunchKernelGGL((adjoint_xl<2>), grid, block, 0, st, L, subs, xl32, w, raw, part); break;
    case 4: hipLaunchKernelGGL((adjoint_xl<4>), grid, block, 0, st, L, subs, xl32, w, raw, part); break;
    case 8: hipLaunchKernelGGL((adjoint_xl<8>), grid, block, 0, st, L, subs, xl32, w, raw, part); break;
    case 9: hipLaunchKernelGGL((adjoint_xl<9>), grid, block, 0, st, L, subs, xl32, w, raw, part); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vl
