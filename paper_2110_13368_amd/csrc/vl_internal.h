// vl_internal.h -- device-visible descriptors shared by the host runtime and
// the gfx950 kernels of the LOD diffusion-decay library.  Internal: not part of
// the C ABI (include/voxlod.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vl {

// Lines per tile of the FP32 sweeps.  A tile is solved by one workgroup of two
// waves: wave 0 eliminates the first half of each line top-down, wave 1 the
// second half bottom-up; lane l of both waves owns line l of the tile.
constexpr int kTileLines = 64;
constexpr int kWave = 64;

// Per-lane capacities (elements of one half line held in VGPRs) compiled for
// the FP32 sweeps.  A sweep class uses the smallest one >= ceil((n-1)/2).
// 100 serves lines of 194-201 voxels (200 is a common grid edge) without the
// 28 spare registers and rows of the 128 class.
constexpr int kNumCaps = 8;
constexpr int kCaps[kNumCaps] = {32, 64, 96, 100, 128, 160, 200, 256};

// x and y solves of one z-plane per workgroup (volumes whose plane fits in
// LDS): four wave pairs; plane rows padded to an odd stride so that 64 lanes
// walking 64 consecutive rows hit 64 different banks.
constexpr int kXYThreads = 512;
constexpr size_t kXYMaxLds = 160 * 1024;
__host__ __device__ constexpr int xy_row_stride(int nx) { return nx | 1; }
// dynamic LDS of that kernel: pivot tables of both axes (FP64 pairs), one
// FP64 exchange slot per lane of each wave pair, the plane
inline size_t xy_lds_bytes(int nx, int ny)
{
    const size_t cbx = (size_t)(nx - 1 - (nx - 1) / 2), cby = (size_t)(ny - 1 - (ny - 1) / 2);
    return (cbx + cby) * 16 + (size_t)(kXYThreads / 2) * 8 + (size_t)ny * xy_row_stride(nx) * 4;
}

// One (simulation, substrate) volume.
struct SubDev {
    long long base;      // element offset of voxel (0,0,0) in the field
    long long vol;       // voxels in the volume (nx*ny*nz)
    int n[3];            // nx, ny, nz
    int sim;             // owning simulation
    int sub;             // substrate index within the simulation
    int dir_mask;        // bit f set: face f (x-, x+, y-, y+, z-, z+) is Dirichlet
    int coef32[3];       // per axis: first float2 of the half-line table
    int coef64[3];       // per axis: first double2 of the full-line table
    float dval32[6];     // Dirichlet values (FP32 path)
    float mid32[3][2];   // per axis: (g1, g2) of the middle row of the split solve
    double dval64[6];    // Dirichlet values (FP64 path)
    double mid64[3][2];  // per axis: (g1, g2) of the middle row, FP64 (FP32 path's recurrences)
    double c[3];         // dt*D/h_a^2 per axis
    double sigma;        // diagonal shift lambda*dt/3 (decay split over the solves) or 0
    double fdec;         // decay factor 1/(1 + lambda*dt) applied after the x solve, or 1
    int xlane;           // first float of the lanes-along-the-line x table (FP32 path)
    int pad_;
};

// x solve with lanes along the line (FP32 path, option): lane l of a wave
// holds K = ceil(nx/64) consecutive voxels of one x-line.  The last voxel of
// each lane's run is a separator; the voxels before it (the lane's interval)
// are eliminated locally, the separators form a tridiagonal system over the
// lanes whose matrix does not depend on the data, solved by parallel cyclic
// reduction with precomputed multipliers.  Per volume a table of
// xl_fields(K) rows of 64 floats (row-major by field, one column per lane):
//   inv[t], e[t]     t < K-1   interval pivots (1/d_t, c/d_t)
//   al[t], be[t]     t < K-1   interval response to the left / own separator
//   k1[v], k2[v]     v < 6     multipliers of reduction level v (distance 2^v)
//   binv                       1 / reduced diagonal after the last level
//   cprev, cnext               c where the lane's / the next lane's interval
//                              is not empty, else 0
constexpr int kXLaneMaxK = 9;  // lines of up to 576 voxels
constexpr int kXLaneLevels = 6;
constexpr int kXLaneMinN = 129;       // shorter lines keep the split solve (few voxels per lane)
constexpr int kXLaneMinNShort = 65;   // the same with two voxels per lane (VL_OPT_X_LANES 2)
__host__ __device__ constexpr int xl_fields(int K) { return 4 * (K - 1) + 2 * kXLaneLevels + 3; }
// voxels per lane: whole 16-byte pieces where the line allows
__host__ __device__ constexpr int xl_k(int n) { return n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : n <= 512 ? 8 : 9; }

// One launch of an FP32 sweep over a group of volumes sharing a capacity
// class: tiles of the listed volumes are numbered consecutively.
struct SweepLaunch {
    const int *sub_ids;      // volumes in this launch
    const int *tile_prefix;  // count+1 exclusive prefix of their tile counts
    int count;
    int total_tiles;
    int xcd_order;           // 1: give each XCD a contiguous range of tiles
};

// Per-simulation cell tables (all offsets in elements of their arrays).
struct SimCells {
    int sub0;        // index of the simulation's first SubDev (substrate 0)
    int ns;          // substrates
    int n_occ;       // occupied voxels
    int occ_base;    // first entry in occ_vox / seg_start
    int cell_base;   // first entry of the sorted per-cell arrays
    int comp_base;   // first float2 of the FP32 composites (n_occ x ns)
    int ab_base;     // first double2 of the sorted per-cell (a, b) (n_cells x ns)
    int zl_base;     // first entry of the z-line starts (nx*ny + 1), -1 without cells
    int xs_base;     // first entry of the x-line starts (ny*nz + 1) when this simulation's sources
                     // can be carried into the next x solve (FP32, x-lines solved with the lanes
                     // along the line, cells present), else -1
    int occ_cap;     // occupied voxels the tables have room for (the voxel-ordered composites
                     // are substrate-major with this stride)
};

// Cell sources applied by the z sweep after its stores (FP32 path).  The
// occupied voxels of a simulation are listed by z-line then k; line_start
// gives each z-line's first entry.
struct FusedSources {
    const SimCells *cells;
    const int *line_start;
    const int *occ_vox;
    const float2 *comp;
    int enabled;
    int skip_carried;  // leave simulations with xs_base >= 0 to the next x solve
    int while_storing;  // short-line z tiles apply them as they store (else in a pass after)
};

// Cell sources of the previous step applied by the x solve (lanes along the
// line) to each line as it is loaded, before the Dirichlet projection: the
// occupied voxels in voxel order, each x-line's first entry (xs_base), their
// FP32 composites in the same order, substrate-major (stride occ_cap).
struct CarriedSources {
    const SimCells *cells;
    const int *xline_start;
    const int *occ_vox_v;
    const float2 *comp_v;
    int enabled;
};

// One launch for a whole step: tiles of all three sweeps in one queue.
struct StepQueue {
    const int *sub_ids;     // volumes (count)
    const int *prefix;      // 3 x (count + 1) exclusive tile prefixes, one row per axis
    int count;
    int phase_start[4];     // first queue index of the x, y, z tiles; [3] = total
    unsigned *counters;     // [0] queue head, [1] workgroups done, [2..] done tiles per (axis, volume)
    int *error;             // set to 1 when a wait gives up
    unsigned long long wait_ticks;  // wall-clock ticks a wait may take before giving up
    unsigned zero;          // always 0: the operand of the atomic reads of the counters
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files, called by the runtime).

// a1: coefficients.  One thread per (volume, axis), FP64 recurrences.
// coefh receives the half-line table in FP64 (same indexing as coef32): the
// forward FP32 sweeps run their recurrences in FP64 from it.
hipError_t launch_coefficients(const SubDev *subs, int nsubs, float2 *coef32, double2 *coefh,
                               double2 *coef64, SubDev *subs_rw, hipStream_t st);

// a3+a4 for volumes whose z-plane fits in LDS: x then y solve of one plane per
// workgroup (tile_prefix counts planes); lds_bytes as from xy_lds_bytes.
// prepare_sweep_xy raises the kernel's dynamic-LDS limit (once per device).
hipError_t prepare_sweep_xy(size_t lds_bytes);
hipError_t launch_sweep_xy(const SweepLaunch &L, size_t lds_bytes, const SubDev *subs, const double2 *coef,
                           float *field, hipStream_t st);

// a3 with lanes along the line: tables (one 64-thread workgroup per volume,
// FP64 arithmetic) and the sweep for lines of K voxels per lane (tiles of 64
// x-lines as for the split sweep).  raw as for launch_sweep_f32.
// The tables are written twice: in FP64 (xl64) for the forward solve, whose
// arithmetic is FP64, and in FP32 (xl32) for the adjoint's reverse solve.
hipError_t launch_xl_tables(const SubDev *subs, int nsubs, const float2 *coef_unused, float *xl32, double *xl64,
                            hipStream_t st);
hipError_t launch_sweep_xl(int K, int lpw, const SweepLaunch &L, const SubDev *subs, const double *xl64, float *field,
                           float *raw, const CarriedSources &carry, hipStream_t st);

// a3-a5, FP32 split-Thomas sweeps along axis (0, 1, 2) for capacity class cap_idx.
// carry (x only): the previous step's cell sources applied to the staged lines.
// raw (may be null, same layout as the field) receives each solve's output
// before the Dirichlet projection, for the adjoint's replay.  nontemporal (z
// only): stream the rows with non-temporal loads and stores, for launches
// none of whose tiles applies cell sources after its stores.
hipError_t launch_sweep_f32(int axis, int cap_idx, const SweepLaunch &L,
                            const SubDev *subs, const double2 *coef, float *field, float *raw,
                            const FusedSources &src, const CarriedSources &carry, bool nontemporal,
                            hipStream_t st);

// a9: adjoint sweep along axis, in place on w (same layout as the field).  The
// Dirichlet adjoint (zero at Dirichlet voxels) is applied on load and store;
// raw holds the forward solve's output.  Per tile, partials[3*tile + k] get
// k = 0: w_out^T K y, 1: -w_out^T y, 2: w_in^T y (x sweep only).
hipError_t launch_adjoint_sweep(int axis, int cap_idx, const SweepLaunch &L, const SubDev *subs,
                                const float2 *coef, float *w, const float *raw, double *partials,
                                hipStream_t st);
// totals[3*(3*q + axis) + k] += the partials of volume q's tiles, in tile order.
hipError_t launch_reduce_partials(const SweepLaunch &L, int axis, const double *partials,
                                  double *totals, hipStream_t st);
// Adjoint of the sources of every simulation (FP64 arithmetic): w at occupied
// voxels walks back through each voxel's cells; dS, dU (per cell and
// substrate, in upload order) accumulate.
hipError_t launch_sources_adjoint(const SimCells *cells, int nsims, const int *occ_prefix,
                                  int occ_bound, int max_ns, const SubDev *subs,
                                  const int *occ_vox_v, const int *seg_start,
                                  const double2 *ab, const double *krs, const double *kcell,
                                  const int *cell_of, const float *rho, float *w,
                                  const int *cell_out_base, double *dS, double *dU,
                                  hipStream_t st);

// a8: the whole step as one persistent launch of `grid` workgroups.
hipError_t launch_step_persistent(int cap_idx, int grid, const StepQueue &Q, const SubDev *subs,
                                  const double2 *coef, float *field, const FusedSources &src,
                                  hipStream_t st);
hipError_t persistent_blocks_per_cu(int cap_idx, int *blocks);

// FP64 plain path: one thread per line, Thomas with the intermediate kept in
// the field itself.  lines_prefix has nsubs+1 entries.
hipError_t launch_sweep_plain(int axis, const SubDev *subs, int nsubs,
                              const long long *lines_prefix, long long total_lines,
                              const double2 *coef, double *field, hipStream_t st);
hipError_t launch_dirichlet_plain(const SubDev *subs, const int4 *faces, int nfaces,
                                  const long long *face_prefix, long long total,
                                  double *field, hipStream_t st);
hipError_t launch_decay_plain(const SubDev *subs, int nsubs, const long long *vox_prefix,
                              long long total, double *field, hipStream_t st);

// a2: cell binning.  The counts of an upload live on the device (counts[0]
// out of domain, [1] occupied voxels, [2] inside, [4] cells), so the binning
// kernels run back to back without reading counts on the host; n_cap (the
// upload's cell count) bounds them and sizes the grids.
hipError_t launch_upload_counts(int *counts, int n, hipStream_t st);
hipError_t launch_cell_keys(const double *pos, int n, int nx, int ny, int nz, double x0,
                            double y0, double z0, double dx, double dy, double dz,
                            unsigned long long *keys, int *n_out, hipStream_t st);
// Stable radix sort of *n_dev (<= n_cap) keys on bits [lo_bit, lo_bit + bits)
// (rounded up to whole pairs of 4-bit digits), ping-ponging with alt; hist
// holds radix_hist_entries(n_cap) entries.
int radix_hist_entries(int n_cap);
hipError_t launch_radix_sort(unsigned long long *keys, unsigned long long *alt, int n_cap, const int *n_dev,
                             int lo_bit, int bits, unsigned *hist, hipStream_t st);
// scratch: radix_hist_entries(n_cap) entries (the sort's hist serves)
hipError_t launch_segments(const unsigned long long *keys, int n_cap, int n, int *seg_id, int *occ_vox,
                           int *seg_start, int *counts, unsigned *scratch, hipStream_t st);
hipError_t launch_composites(const unsigned long long *keys, const int *seg_start, const int *counts, int n_cap,
                             int ns, const double *V, const double *S, const double *U, const double *RS,
                             double dt, double vvox, const int *pos, float2 *comp32, float2 *comp32_v,
                             int v_stride, double2 *ab64, double *krs, double *kcell, int *cell_of, hipStream_t st);
hipError_t launch_xline_starts(const int *occ_vox_v, const int *counts, int nx, int nlines, int *line_start,
                               hipStream_t st);
// the upload's occupied-voxel count into the cell tables and the prefix over
// the simulations (counts null: no cells)
hipError_t launch_finish_upload(const int *counts, SimCells *cells, int sim, int nsims, int xs_base, int *occ_prefix,
                                hipStream_t st);
hipError_t launch_zline_order(const int *occ_vox_v, const int *counts, int n_cap, int nxy, int nz,
                              unsigned long long *zkeys, unsigned long long *zalt, unsigned *hist, int *occ_vox,
                              int *pos, int *line_start, hipStream_t st);

// a5/a6: sources over the occupied voxels of every simulation.
hipError_t launch_sources_f32(const SimCells *cells, int nsims, const int *occ_prefix,
                              int occ_bound, int max_ns, const SubDev *subs,
                              const int *occ_vox, const float2 *comp, float *field,
                              int only_carried, hipStream_t st);
hipError_t launch_sources_plain(const SimCells *cells, int nsims, const int *occ_prefix,
                                int occ_bound, const SubDev *subs, const int *occ_vox,
                                const int *seg_start, const double2 *ab, double *field,
                                hipStream_t st);

// a7: FP64 mass of one volume; partials has kMassBlocks entries.
constexpr int kMassBlocks = 256;
hipError_t launch_mass(const void *field, int is_f64, long long base, long long vol,
                       double *partials, double *out, hipStream_t st);
// The same sums for nvols volumes of vol elements, vol_stride apart from
// field, into out_dev[0..nvols), with the partial sums in the library's static
// per-device array (vl_noalloc.hip) instead of a workspace.
constexpr int kNoallocMaxVolumes = 64;
hipError_t mass_noalloc(const void *field, int is_f64, long long vol, long long vol_stride, int nvols,
                        double *out_dev, hipStream_t st);
hipError_t launch_count_nonfinite(const void *field, int is_f64, const SubDev *subs,
                                  int nsubs, unsigned long long *count, hipStream_t st);

// AoS <-> SoA on the device for one simulation.
hipError_t launch_aos_to_soa(const void *src, void *field, int is_f64, long long base,
                             long long vol_stride, long long vol, int ns, int inverse,
                             hipStream_t st);

}  // namespace vl
