// vl_sweep_f32.hip -- FP32 line solves of the LOD step for gfx950.
//
// arXiv:2110.13368, section "Elements of Parallelism": the implicit
// diffusion-decay update is solved direction by direction (x, then y, then z),
// every grid line of every substrate being a constant-coefficient tridiagonal
// system solved by elimination (the paper's axpy) and back-substitution (its
// naxpy); Dirichlet conditions are applied by their own function around the
// solves.  Here the Dirichlet projection and the decay factor are folded into
// the solve's loads and stores, so each sweep reads and writes every element
// once.
//
// Split solve.  The line matrix T = tridiag(-c, b, -c) has the same end
// diagonal at both ends, so it is persymmetric: eliminating from the last row
// upwards meets the same pivots d_t as eliminating from the first row
// downwards.  A line of n rows is split at its middle row m = (n-1)/2:
//   wave 0 eliminates rows 0..m-1 downwards   y_t = r_t/d_t + (c/d_t) y_{t-1}
//   wave 1 eliminates rows n-1..m+1 upwards   z_t likewise, from the other end
//   the middle row gives x_m = (r_m + c y_{m-1} + c z_{m+1}) / gamma
//   both waves back-substitute outwards       x_t = y_t + (c/d_t) x_{t+1}.
// This is Gaussian elimination without pivoting on a reordered system (an
// exact factorisation, as is the plain Thomas algorithm); both waves use the
// same pivot table, indexed by the distance from their end.
//
// Mapping.  A workgroup is two waves and owns a tile of 64 lines; lane l of
// both waves works on line l.  Each wave walks its rows in one direction with
// a wave-uniform row offset, so y- and z-lines (stride nx, nx*ny) are read and
// written as 256-byte rows of 64 neighbouring x values.  x-lines are
// contiguous: they are moved through a 64x65 LDS block per 64 columns (64x33
// per 32 columns for lines of up to 65 voxels), loaded
// with lanes along x and read back with lanes along the lines.  The half line
// a lane owns stays in VGPRs (CAP values).
#include <climits>

#include "vl_device.h"

namespace vl {

// z tiles apply their cells' sources while they store, from a stage of up to
// kZSrcStage occupied voxels, in the classes of up to kZSrcMaxCap values per
// lane: lines that short leave L2 before a pass after the stores could
// re-read them (on the 256-grid batch that pass read 1.46x the field; the
// 100-value class on a 128 MB field, which the Infinity Cache holds, was
// faster with the pass after the stores)
constexpr int kZSrcStage = 1024;
constexpr int kZSrcMaxCap = 64;


// One tile of one sweep: 64 lines of volume S, tile index `local` within the
// volume's tiles of this axis.  Called by every thread of a 128-thread
// workgroup (it contains workgroup barriers).
template <int AXIS, int CAP, bool XSTAGE, bool NT = false>
__device__ __forceinline__ void sweep_tile(const SubDev &S, int local, const double2 *__restrict__ coef,
                                           float *__restrict__ field, float *__restrict__ raw,
                                           const FusedSources &src, const CarriedSources &carry,
                                           FwdLds<CAP, XSTAGE> &sh)
{
    constexpr int kW = XStage<CAP>::W;    // stage columns per chunk
    constexpr int kSX = XStage<CAP>::SX;  // stage row stride
    constexpr int kChunks = (CAP + kW - 1) / kW;
    // x with 32-column chunks (lines of up to 65 voxels): each LDS-DMA load
    // and each store instruction moves two rows of the tile (lanes 0-31 row
    // 2p, lanes 32-63 row 2p+1), where one row per instruction would leave
    // half the lanes idle.  Row q sits at (q/2)*kPS + (q%2)*32 in the stage,
    // and lane l solves row xrow(l) = 2(l mod 32) + l/32, so that the 32
    // lanes of each half read their own rows without bank conflicts.
    constexpr bool kPair = AXIS == 0 && kW == 32;
    constexpr int kPS = 2 * kW + 1;
    // NT (z launches of long lines whose tiles re-read no voxel after their
    // stores): the rows lie a plane apart and each 256-byte row is read and
    // written once, so the loads and stores are non-temporal (5 % faster on
    // 400^3 x 8; y, whose rows are neighbours, was not faster, nor were
    // shorter z-lines, and a z tile that applies cell sources after its
    // stores would lose those lines)
    constexpr int kPol = NT ? kNonTemporal : 0;
    double(&xch)[2][kWave] = sh.xch;
    double2 *cs_lds = sh.piv;
    float *stage = sh.stage;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const bool top = (wave == 0);
    const int xrow = kPair ? 2 * (lane & 31) + (lane >> 5) : lane;  // this lane's row of an x tile
    const int xcol = kPair ? (lane & 31) : lane;                    // the chunk column a lane moves
    auto srow = [&](int q) { return kPair ? (q >> 1) * kPS + (q & 1) * 32 : q * kSX; };

    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int n = S.n[AXIS];
    const int m = (n - 1) >> 1;    // middle row
    const int cb = n - 1 - m;      // rows below the middle (m or m + 1)
    const int nel = top ? m : cb;  // rows this wave eliminates and holds
    const double g1 = S.mid64[AXIS][0];
    const double g2 = S.mid64[AXIS][1];
    const int dmask = S.dir_mask;

    // pivot table (inv_d_t, c/d_t), t < cb, FP64, staged once per workgroup
    {
        const double2 *__restrict__ cf = coef + S.coef32[AXIS];
        for (int t = threadIdx.x; t < cb && t < CAP; t += 128) cs_lds[t] = cf[t];
    }

    // Geometry of this lane's line: faces of the other axes it lies on, and a
    // buffer resource plus offsets to address its rows.
    int on = 0;
    long long base = 0;      // element offset of the resource base
    unsigned lane_b = 0;     // per-lane byte offset (y, z: along x; x: row start)
    int row_b = 0;           // bytes between rows (y, z) / between x-lines (x)
    int xrows_left = 0;      // x-lines of the tile that exist
    bool line_ok = true;     // this lane's line exists (x: not a clamped copy; a copy's
                             // values differ once carried sources are applied, so it
                             // must not store)
    if (AXIS == 0) {
        const int nrows = ny * nz;
        const int r0 = local * kTileLines;
        const int r = min(r0 + xrow, nrows - 1);
        line_ok = r0 + xrow < nrows;
        const int j = r % ny, k = r / ny;
        on = (j == 0 ? 1 << 2 : 0) | (j == ny - 1 ? 1 << 3 : 0) |
             (k == 0 ? 1 << 4 : 0) | (k == nz - 1 ? 1 << 5 : 0);
        base = S.base + (long long)r0 * nx;
        lane_b = (unsigned)(r - r0) * (unsigned)nx * 4u;
        row_b = nx * 4;
        xrows_left = nrows - r0;
    } else {
        // y-lines (i, k) and z-lines (i, j) numbered L = i + nx*o; a tile is 64
        // consecutive lines, so no lane idles except in a volume's last tile.
        const int no = (AXIS == 1) ? nz : ny;
        const int nlines = nx * no;
        const int L0 = local * kTileLines;
        const int L = min(L0 + lane, nlines - 1);
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
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(field + base, S.base + S.vol - base);
    const int wface = top_face(dmask & on);  // whole line Dirichlet

    // x: cell sources of the previous step carried into this solve (as in the
    // x solve with lanes along the line): the occupied voxels of the tile's
    // x-lines form one range of the simulation's voxel-ordered list, each
    // applied (rho R + P, the update of every other placement) to the staged
    // line values before the Dirichlet projection that opens the step
    const SimCells *CC = (AXIS == 0 && carry.enabled) ? &carry.cells[S.sim] : nullptr;
    const bool carried = CC != nullptr && CC->xs_base >= 0;  // uniform
    const int *__restrict__ c_xs = carried ? carry.xline_start + CC->xs_base : nullptr;
    const int *__restrict__ c_vox = carried ? carry.occ_vox_v + CC->occ_base : nullptr;
    const float2 *__restrict__ c_ab =
        carried ? carry.comp_v + CC->comp_base + (size_t)S.sub * CC->occ_cap : nullptr;
    const int c_r0 = local * kTileLines;
    const int c_e0 = carried ? c_xs[c_r0] : 0;
    const int c_e1 = carried ? c_xs[min(c_r0 + kTileLines, S.n[1] * S.n[2])] : 0;
    // the entries whose columns this wave holds in [cs, cs + width) of the
    // stage, 64 at a time; slot(q, c) is row q's column cs + c in the stage
    auto carry_chunk = [&](int cs, int width, auto slot) {
        if (!carried) return;
        for (int eb = c_e0; eb < c_e1; eb += kWave) {  // uniform
            const int e = eb + lane;
            if (e < c_e1) {
                const int vox = c_vox[e];
                const int q = vox / nx - c_r0;
                const int i = vox - (q + c_r0) * nx;
                const bool own = top ? i < m : i > m;
                if (own && i >= cs && i < cs + width) {
                    float *pq = slot(q, i - cs);
                    const float2 ab = c_ab[e];
                    *pq = fmaf(*pq, ab.y, ab.x);
                }
            }
        }
        wave_sync_lds();
    };
    const int lo_f = (dmask >> (2 * AXIS)) & 1 ? 2 * AXIS : -1;
    const int hi_f = (dmask >> (2 * AXIS + 1)) & 1 ? 2 * AXIS + 1 : -1;
    const int f_first = max(wface, max(lo_f, n == 1 ? hi_f : -1));  // row 0
    const int f_last = max(wface, hi_f);                            // row n-1

    float v[CAP];

    // ---- load the half line (local t: wave 0 row t, wave 1 row n-1-t) ----
    if (AXIS == 0 && XWide<CAP>::value) {
        float *stw = stage + wave * 64 * kSX;
        x_load_wide<CAP>(v, rs, stw, top, n, nel, row_b, xrows_left, lane, [&](int, int cbase) {
            carry_chunk(cbase, 64, [&](int q, int c) { return stw + x_wide_slot(q, c); });
        });
    } else if (AXIS == 0) {
        float *st = stage + wave * 64 * kSX;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (c * kW < nel) {
                const int cs = top ? c * kW : n - kW * (c + 1);
                const int col = top ? min(cs + xcol, nel - 1) : max(cs + xcol, n - cb);
                const unsigned cb4 = (unsigned)col * 4u;
                // the previous chunk's reads of the stage must be complete
                // before this chunk's DMA overwrites it: LDS-DMA writes are
                // ordered after the wave's earlier LDS reads neither by the
                // compiler nor by the hardware
                if (c > 0) __builtin_amdgcn_s_waitcnt(0);
                // DMA straight into LDS: lane j's value of row q lands in
                // st[q*kSX + j]; no VGPR staging, all 64 rows in flight.  The
                // DMA writes lane j at the instruction's base + j, so with
                // 32-column chunks lanes 32-63 land on the pair's second row.
                if (kPair) {
#pragma unroll
                    for (int p = 0; p < 32; ++p)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(
                            rs, (__attribute__((address_space(3))) void *)(st + p * kPS), 4,
                            (int)(cb4 + (unsigned)(min(2 * p + (lane >> 5), xrows_left - 1) * row_b)), 0, 0, 0);
                } else {
#pragma unroll
                    for (int q = 0; q < 64; ++q)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(
                            rs, (__attribute__((address_space(3))) void *)(st + q * kSX), 4, (int)cb4,
                            min(q, xrows_left - 1) * row_b, 0, 0);
                }
                __builtin_amdgcn_s_waitcnt(0);
                wave_sync_lds();
                carry_chunk(cs, kW, [&](int q, int cc) { return st + srow(q) + cc; });
                if (top) {
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj)
                        if (c * kW + jj < CAP && c * kW + jj < nel) v[c * kW + jj] = st[srow(xrow) + jj];
                } else {
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj)
                        if (c * kW + jj < CAP && c * kW + jj < nel) v[c * kW + jj] = st[srow(xrow) + kW - 1 - jj];
                }
                wave_sync_lds();
            }
        }
    } else {
        // Every row of the capacity is loaded, the rows past this wave's
        // half from an offset beyond the buffer (they read 0 and touch no
        // memory): with no branch around the loads the waits before the
        // elimination can be for the first rows only.
        const int row0 = top ? 0 : (n - 1) * row_b;
        const int step = top ? row_b : -row_b;
#pragma unroll
        for (int t = 0; t < CAP; ++t) {
            const unsigned oob = (unsigned)((nel - 1 - t) >> 31) & 0x80000000u;  // uniform
            v[t] = bload_p<kPol>(rs, lane_b | oob, oob ? 0 : row0 + t * step);
        }
    }

    __syncthreads();  // pivot table visible

    // ---- Dirichlet projection before the x solve: only the end rows matter,
    //      whole-line Dirichlet lines are overwritten after the solve ----
    if (AXIS == 0) {
        if (!top && cb >= 1 && hi_f >= 0) v[0] = S.dval32[hi_f];
        if (top && m >= 1 && lo_f >= 0) v[0] = S.dval32[lo_f];
    }

    // ---- elimination from this wave's end towards the middle ----
    // The recurrences run in FP64 and only the values they store are rounded
    // to FP32: rounding inside an FP32 recurrence is the same for
    // neighbouring lines of a smooth field and from one step to the next, so
    // it accumulates like a bias (a drift of the mean of about 3 ulp per 100
    // steps), while rounding the stored values does not.
    double prev = 0.0;
    VL_FOR_UP(CAP, nel, t, {
        const double2 c = cs_lds[t];
        prev = fma(c.y, prev, (double)v[t] * c.x);
        v[t] = (float)prev;
    })

    // ---- middle row ----
    double xm = 0.0;
    if (!top) xch[0][lane] = prev;  // z_{m+1} (0 when the line has one row)
    __syncthreads();
    if (top) {
        float rm;
        if (AXIS == 0) {
            rm = bload(rs, lane_b + (unsigned)m * 4u, 0);
            if (carried && line_ok) {  // the middle column's source, if any, from this lane's own x-line
                const int r = c_r0 + xrow;
                const int want = r * nx + m;
                for (int e = c_xs[r]; e < c_xs[r + 1]; ++e) {
                    const int vox = c_vox[e];
                    if (vox >= want) {
                        if (vox == want) {
                            const float2 ab = c_ab[e];
                            rm = fmaf(rm, ab.y, ab.x);
                        }
                        break;
                    }
                }
            }
            if (m == 0) {
                const int f0 = max(lo_f, n == 1 ? hi_f : -1);
                if (f0 >= 0) rm = S.dval32[f0];
            }
        } else {
            rm = bload(rs, lane_b, m * row_b);
        }
        xm = fma(g2, prev + xch[0][lane], (double)rm * g1);
        xch[1][lane] = xm;
    }
    __syncthreads();
    if (!top) xm = xch[1][lane];

    // ---- back-substitution from the middle outwards ----
    double nxt = xm;
    VL_FOR_DOWN(CAP, nel, t, {
        nxt = fma(cs_lds[t].y, nxt, (double)v[t]);
        v[t] = (float)nxt;
    })
    float xm32 = (float)xm;

    // ---- raw solve output before the Dirichlet projection (adjoint replay) ----
    if (raw != nullptr) {
        const __amdgpu_buffer_rsrc_t rr = make_rsrc(raw + base, S.base + S.vol - base);
        if (AXIS == 0 && XWide<CAP>::value) {
            if (top && line_ok) bstore(rr, lane_b + (unsigned)m * 4u, 0, xm32);
            x_store_wide<CAP>(v, rr, stage + wave * 64 * kSX, top, n, nel, row_b, xrows_left, lane, lane_b, line_ok);
        } else if (AXIS == 0) {
            // through the LDS stage, like the field store below
            float *st = stage + wave * 64 * kSX;
            if (top && line_ok) bstore(rr, lane_b + (unsigned)m * 4u, 0, xm32);
#pragma unroll
            for (int c = 0; c < kChunks; ++c) {
                if (c * kW < nel) {
                    if (top) {
#pragma unroll
                        for (int jj = 0; jj < kW; ++jj)
                            if (c * kW + jj < CAP && c * kW + jj < nel) st[srow(xrow) + jj] = v[c * kW + jj];
                    } else {
#pragma unroll
                        for (int jj = 0; jj < kW; ++jj)
                            if (c * kW + jj < CAP && c * kW + jj < nel) st[srow(xrow) + kW - 1 - jj] = v[c * kW + jj];
                    }
                    wave_sync_lds();
                    const int cs = top ? c * kW : n - kW * (c + 1);
                    const int col = top ? min(cs + xcol, nel - 1) : max(cs + xcol, n - cb);
                    const int so = col - cs;
                    const unsigned cb4 = (unsigned)col * 4u;
                    if (kPair) {
#pragma unroll 16
                        for (int p = 0; p < 32; ++p) {
                            const int q = 2 * p + (lane >> 5);
                            if (q < xrows_left) bstore(rr, cb4 + (unsigned)(q * row_b), 0, st[srow(q) + so]);
                        }
                    } else {
#pragma unroll 16
                        for (int q = 0; q < 64; ++q)
                            if (q < xrows_left) bstore(rr, cb4, q * row_b, st[q * kSX + so]);
                    }
                    wave_sync_lds();
                }
            }
        } else {
            if (top) bstore(rr, lane_b, m * row_b, xm32);
            const int row0 = top ? 0 : (n - 1) * row_b;
            const int step = top ? row_b : -row_b;
            VL_FOR_UP(CAP, nel, t, bstore(rr, lane_b, row0 + t * step, v[t]);)
        }
    }

    // ---- Dirichlet projection after the solve ----
    if (__builtin_amdgcn_ballot_w64(wface >= 0) != 0) {
        const float wv = face_value(S.dval32, wface);
        const bool whole = wface >= 0;
        VL_FOR_UP(CAP, nel, t, v[t] = whole ? wv : v[t];)
        xm32 = whole ? wv : xm32;
    }
    if (top) {
        if (f_first >= 0) {
            const float ev = face_value(S.dval32, f_first);
            if (m >= 1)
                v[0] = ev;
            else
                xm32 = ev;
        }
    } else if (cb >= 1 && f_last >= 0) {
        v[0] = face_value(S.dval32, f_last);
    }

    // ---- cell sources of this tile's z-lines, applied as it stores (the
    //      classes up to kZSrcMaxCap values; a tile with more than
    //      kZSrcStage occupied voxels, and the longer classes, apply them
    //      after their stores instead) ----
    // The occupied voxels of the tile's 64 z-lines are one run of the
    // z-line-ordered list, sorted by (line, k) within it.  Staged in LDS,
    // each lane walks its own line's entries upwards (top wave: rows 0 ..
    // m - 1, then the middle row) or downwards (bottom wave: rows n - 1 ..
    // m + 1) while it stores its rows, and stores rho R + P where the row
    // matches: the same fmaf on the same FP32 value as the pass after the
    // stores.
    [[maybe_unused]] bool src_walk = false;  // uniform
    [[maybe_unused]] int zp = 0, zk = 0, za = 0, zb = 0;  // this lane's walk: position, its row, range [za, zb)
    [[maybe_unused]] const int *zs = nullptr;       // the staged entries' rows
    [[maybe_unused]] const float2 *zc = nullptr;    // and their composites (P, R)
    if constexpr (AXIS == 2 && CAP <= kZSrcMaxCap) {
        __shared__ int zs_k[kZSrcStage];
        __shared__ float2 zs_c[kZSrcStage];
        if (src.enabled && src.while_storing) {
            const SimCells &C = src.cells[S.sim];
            if (C.zl_base >= 0 && !(src.skip_carried && C.xs_base >= 0)) {
                const int nxy = nx * ny;
                const int L0 = local * kTileLines;
                const int *ls = src.line_start + C.zl_base;
                const int e0 = ls[L0], e1 = ls[min(L0 + kTileLines, nxy)];
                if (e1 - e0 <= kZSrcStage) {
                    for (int e = e0 + (int)threadIdx.x; e < e1; e += 2 * kWave) {
                        zs_k[e - e0] = src.occ_vox[C.occ_base + e] / nxy;
                        zs_c[e - e0] = src.comp[C.comp_base + (size_t)e * C.ns + S.sub];
                    }
                    __syncthreads();
                    // this lane's line (past the volume's last line: a copy of
                    // it, which then stores the same values)
                    const int L = min(L0 + lane, nxy - 1);
                    za = ls[L] - e0;
                    zb = ls[L + 1] - e0;
                    zp = top ? za : zb - 1;
                    zk = top ? (zp < zb ? zs_k[zp] : INT_MAX) : (zp >= za ? zs_k[zp] : -1);
                    zs = zs_k;
                    zc = zs_c;
                    src_walk = true;
                }
            }
        }
    }

    // ---- store ----
    if (AXIS == 0 && XWide<CAP>::value) {
        if (top && line_ok) bstore(rs, lane_b + (unsigned)m * 4u, 0, xm32);
        x_store_wide<CAP>(v, rs, stage + wave * 64 * kSX, top, n, nel, row_b, xrows_left, lane, lane_b, line_ok);
    } else if (AXIS == 0) {
        float *st = stage + wave * 64 * kSX;
        if (top && line_ok) bstore(rs, lane_b + (unsigned)m * 4u, 0, xm32);
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (c * kW < nel) {
                if (top) {
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj)
                        if (c * kW + jj < CAP && c * kW + jj < nel) st[srow(xrow) + jj] = v[c * kW + jj];
                } else {
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj)
                        if (c * kW + jj < CAP && c * kW + jj < nel) st[srow(xrow) + kW - 1 - jj] = v[c * kW + jj];
                }
                wave_sync_lds();
                const int cs = top ? c * kW : n - kW * (c + 1);
                const int col = top ? min(cs + xcol, nel - 1) : max(cs + xcol, n - cb);
                const int so = col - cs;
                const unsigned cb4 = (unsigned)col * 4u;
                if (kPair) {
#pragma unroll 16
                    for (int p = 0; p < 32; ++p) {
                        const int q = 2 * p + (lane >> 5);
                        if (q < xrows_left) bstore(rs, cb4 + (unsigned)(q * row_b), 0, st[srow(q) + so]);
                    }
                } else {
#pragma unroll 16
                    for (int q = 0; q < 64; ++q)
                        if (q < xrows_left) bstore(rs, cb4, q * row_b, st[q * kSX + so]);
                }
                wave_sync_lds();
            }
        }
    } else {
        bool stored = false;
        if constexpr (AXIS == 2 && CAP <= kZSrcMaxCap) {
            if (src_walk) {  // uniform
                const int row0 = top ? 0 : (n - 1) * row_b;
                const int step = top ? row_b : -row_b;
                if (top) {
                    VL_FOR_UP(CAP, nel, t, {
                        float val = v[t];
                        if (t == zk) {
                            const float2 q = zc[zp];
                            val = fmaf(val, q.y, q.x);
                            ++zp;
                            zk = zp < zb ? zs[zp] : INT_MAX;
                        }
                        bstore_p<kPol>(rs, lane_b, row0 + t * step, val);
                    })
                    if (zk == m) {
                        const float2 q = zc[zp];
                        xm32 = fmaf(xm32, q.y, q.x);
                    }
                    bstore_p<kPol>(rs, lane_b, m * row_b, xm32);
                } else {
                    VL_FOR_UP(CAP, nel, t, {
                        float val = v[t];
                        if (n - 1 - t == zk) {
                            const float2 q = zc[zp];
                            val = fmaf(val, q.y, q.x);
                            --zp;
                            zk = zp >= za ? zs[zp] : -1;
                        }
                        bstore_p<kPol>(rs, lane_b, row0 + t * step, val);
                    })
                }
                stored = true;
            }
        }
        if (!stored) {
            if (top) bstore_p<kPol>(rs, lane_b, m * row_b, xm32);
            const int row0 = top ? 0 : (n - 1) * row_b;
            const int step = top ? row_b : -row_b;
            VL_FOR_UP(CAP, nel, t, bstore_p<kPol>(rs, lane_b, row0 + t * step, v[t]);)
        }

        // ---- cell sources of this tile's z-lines (after the last P_D) ----
        if (AXIS == 2 && src.enabled && !(CAP <= kZSrcMaxCap && src_walk)) {
            const SimCells &C = src.cells[S.sim];
            if (C.zl_base >= 0 && !(src.skip_carried && C.xs_base >= 0)) {
                const int nlines = nx * ny;
                const int L0 = local * kTileLines;
                const int *ls = src.line_start + C.zl_base;
                const int e0 = ls[L0], e1 = ls[min(L0 + kTileLines, nlines)];
                if (e1 > e0) {
                    // both waves' stores of this tile complete and visible
                    __builtin_amdgcn_s_waitcnt(0);
                    __syncthreads();
                    const __amdgpu_buffer_rsrc_t rv = make_rsrc(field + S.base, S.vol);
                    for (int e = e0 + (int)threadIdx.x; e < e1; e += 128) {
                        const int vox = src.occ_vox[C.occ_base + e];
                        const float2 ab = src.comp[C.comp_base + (size_t)e * C.ns + S.sub];
                        const unsigned off = (unsigned)vox * 4u;
                        const float r = bload(rv, off, 0);
                        bstore(rv, off, 0, fmaf(r, ab.y, ab.x));
                    }
                }
            }
        }
    }
}

template <int AXIS, int CAP, bool NT>
__global__ void __launch_bounds__(128)
sweep_f32(SweepLaunch L, const SubDev *__restrict__ subs, const double2 *__restrict__ coef,
          float *__restrict__ field, float *__restrict__ raw, FusedSources src, CarriedSources carry)
{
    __shared__ FwdLds<CAP, AXIS == 0> sh;
    const int tile = L.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int slot = find_slot(L.tile_prefix, L.count, tile);
    const int local = tile - L.tile_prefix[slot];
    sweep_tile<AXIS, CAP, AXIS == 0, NT>(subs[L.sub_ids[slot]], local, coef, field, raw, src, carry, sh);
}

// The whole step in one launch.  Workgroups take tiles from one queue in the
// order: every x tile, then every y tile, then every z tile (volume by
// volume).  A y (z) tile of a volume first waits until all x (y) tiles of
// that volume are done.  Those tiles were taken earlier by workgroups that
// are running and never wait on later tiles, so the waits always end,
// whatever the grid size.  A wait that exceeds Q.wait_ticks sets *error and
// gives up (the step is then wrong, but every wave exits); every later wait
// of the launch sees the error and gives up at once, so the limit bounds the
// launch, not each of its tiles.  The last workgroup to leave resets the
// counters for the next launch.
template <int CAP>
__global__ void __launch_bounds__(128)
sweep_step_persistent(StepQueue Q, const SubDev *__restrict__ subs, const double2 *__restrict__ coef,
                      float *__restrict__ field, FusedSources src)
{
    __shared__ FwdLds<CAP, true> sh;
    __shared__ int s_tile;
    const CarriedSources nocarry{nullptr, nullptr, nullptr, nullptr, 0};
    unsigned *head = Q.counters;
    unsigned *exited = Q.counters + 1;
    unsigned *done = Q.counters + 2;  // [phase][slot]
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= Q.phase_start[3]) break;
        const int phase = t < Q.phase_start[1] ? 0 : (t < Q.phase_start[2] ? 1 : 2);
        const int tp = t - Q.phase_start[phase];
        const int *prefix = Q.prefix + phase * (Q.count + 1);
        const int slot = find_slot(prefix, Q.count, tp);
        const int local = tp - prefix[slot];
        if (phase > 0) {
            if (threadIdx.x == 0) {
                const int *pp = Q.prefix + (phase - 1) * (Q.count + 1);
                const unsigned need = (unsigned)(pp[slot + 1] - pp[slot]);
                unsigned *d = done + (phase - 1) * Q.count + slot;
                // The counter is read with an atomic read-modify-write: each
                // XCD has its own L2, and a plain load may keep returning a
                // stale line of it; RMW atomics act at the coherence point.
                // Q.zero (0, but not a constant here) keeps the compiler from
                // turning the idempotent add into a load.
                // A launch in which a wait has already given up waits no more.
                auto gave_up = [&]() {
                    return __hip_atomic_fetch_add(Q.error, (int)Q.zero, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) != 0;
                };
                if (__hip_atomic_fetch_add(d, Q.zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need &&
                    !gave_up()) {
                    const unsigned long long t0 = wall_clock64();
                    unsigned polls = 0;
                    while (__hip_atomic_fetch_add(d, Q.zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        __builtin_amdgcn_s_sleep(2);
                        if (wall_clock64() - t0 > Q.wait_ticks || ((++polls & 63u) == 0 && gave_up())) {
                            atomicOr(Q.error, 1);
                            break;
                        }
                    }
                }
                // see the other tiles' stores: invalidates this CU's L1 and this XCD's L2
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
        }
        const SubDev &S = subs[Q.sub_ids[slot]];
        if (phase == 0)
            sweep_tile<0, CAP, true>(S, local, coef, field, nullptr, src, nocarry, sh);
        else if (phase == 1)
            sweep_tile<1, CAP, true>(S, local, coef, field, nullptr, src, nocarry, sh);
        else
            sweep_tile<2, CAP, true>(S, local, coef, field, nullptr, src, nocarry, sh);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(done + phase * Q.count + slot, 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_exchange(head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int i = 0; i < 3 * Q.count; ++i)
                __hip_atomic_exchange(done + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_exchange(exited, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int AXIS, bool NT>
static hipError_t launch_axis(int cap_idx, const SweepLaunch &L, const SubDev *subs, const double2 *coef,
                              float *field, float *raw, const FusedSources &src, const CarriedSources &carry,
                              hipStream_t st)
{
    const dim3 grid(L.total_tiles), block(128);
    switch (cap_idx) {
#define VL_CAP_CASE(i)                                                                                            \
    case i:                                                                                                       \
        hipLaunchKernelGGL((sweep_f32<AXIS, kCaps[i], NT>), grid, block, 0, st, L, subs, coef, field, raw, src,  \
                           carry);                                                                                \
        break;
        VL_CAP_CASE(0)
        VL_CAP_CASE(1)
        VL_CAP_CASE(2)
        VL_CAP_CASE(3)
        VL_CAP_CASE(4)
        VL_CAP_CASE(5)
        VL_CAP_CASE(6)
        VL_CAP_CASE(7)
#undef VL_CAP_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step_persistent(int cap_idx, int grid, const StepQueue &Q, const SubDev *subs,
                                  const double2 *coef, float *field, const FusedSources &src,
                                  hipStream_t st)
{
    if (Q.phase_start[3] <= 0 || grid <= 0) return hipSuccess;
    const dim3 g(grid), b(128);
    switch (cap_idx) {
    case 0: hipLaunchKernelGGL(sweep_step_persistent<kCaps[0]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 1: hipLaunchKernelGGL(sweep_step_persistent<kCaps[1]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 2: hipLaunchKernelGGL(sweep_step_persistent<kCaps[2]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 3: hipLaunchKernelGGL(sweep_step_persistent<kCaps[3]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 4: hipLaunchKernelGGL(sweep_step_persistent<kCaps[4]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 5: hipLaunchKernelGGL(sweep_step_persistent<kCaps[5]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 6: hipLaunchKernelGGL(sweep_step_persistent<kCaps[6]>, g, b, 0, st, Q, subs, coef, field, src); break;
    case 7: hipLaunchKernelGGL(sweep_step_persistent<kCaps[7]>, g, b, 0, st, Q, subs, coef, field, src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t persistent_blocks_per_cu(int cap_idx, int *blocks)
{
    switch (cap_idx) {
    case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[0]>, 128, 0);
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[1]>, 128, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[2]>, 128, 0);
    case 3: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[3]>, 128, 0);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[4]>, 128, 0);
    case 5: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[5]>, 128, 0);
    case 6: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[6]>, 128, 0);
    case 7: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_step_persistent<kCaps[7]>, 128, 0);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_f32(int axis, int cap_idx, const SweepLaunch &L, const SubDev *subs,
                            const double2 *coef, float *field, float *raw, const FusedSources &src,
                            const CarriedSources &carry, bool nontemporal, hipStream_t st)
{
    if (L.total_tiles <= 0) return hipSuccess;
    const CarriedSources none{nullptr, nullptr, nullptr, nullptr, 0};
    if (axis == 0) return launch_axis<0, false>(cap_idx, L, subs, coef, field, raw, src, carry, st);
    if (axis == 1) return launch_axis<1, false>(cap_idx, L, subs, coef, field, raw, src, none, st);
    if (axis == 2)
        return nontemporal ? launch_axis<2, true>(cap_idx, L, subs, coef, field, raw, src, none, st)
                           : launch_axis<2, false>(cap_idx, L, subs, coef, field, raw, src, none, st);
    return hipErrorInvalidValue;
}

}  // namespace vl
