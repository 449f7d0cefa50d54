/*
 * voxlod.h -- C ABI of the MI355X (gfx950) library for the locally
 * one-dimensional (LOD) diffusion-decay step with cell secretion/uptake.
 *
 * Method: Stack, Macklin, Searles, Chandrasekaran, "OpenACC Acceleration of an
 * Agent-Based Biological Simulation Framework", arXiv:2110.13368.
 *   Eq. (1)  d(rho)/dt = D lap(rho) - lambda rho
 *                        + sum_i delta(x - x_i) V_i (S_i (rho*_i - rho) - U_i rho)
 *   Section "Elements of Parallelism": the diffusion-decay part is solved
 *   direction by direction (x, y, z), each direction as independent line
 *   solves built from an elimination and a back-substitution over the
 *   substrate vector, with Dirichlet conditions applied by their own function;
 *   the field and the auxiliary arrays stay resident on the device.
 *   Section "Future Work": cell secretion/uptake moved onto the device.
 *
 * One step, for every simulation and substrate s (c = dt*D_s/h_a^2):
 *   rho <- C . P_D . S_z . P_D . S_y . P_D . F . S_x . P_D (rho)
 *   S_a  solves tridiag(-c, b, -c) x = r on every line along axis a, with
 *        zero-flux ends: b = 1 + c + sigma at both ends, 1 + 2c + sigma inside,
 *        1 + sigma for a line of one voxel;
 *   F    divides by (1 + lambda*dt) (VL_DECAY_ONCE, sigma = 0), or is the
 *        identity with sigma = lambda*dt/3 in every S_a (VL_DECAY_THIRDS);
 *   P_D  overwrites the outermost voxel layer of every Dirichlet face; on
 *        edges and corners the last active face in the order x-, x+, y-, y+,
 *        z-, z+ wins;
 *   C    applies every cell, in the order it was uploaded, to the voxel that
 *        holds it: rho <- (rho + k S rho*) / (1 + k (S + U)), k = dt V/V_vox.
 *        A cell at x lies in voxel floor((x - x0)/dx) (per axis, half-open
 *        grid); cells outside are skipped and counted.
 *
 * Memory.  The library never allocates device memory.  The caller allocates
 * the field and a workspace of the sizes vl_finalize reports (normally as
 * torch tensors) and passes raw device pointers to vl_bind; the caller keeps
 * ownership and must keep both alive until vl_destroy.  Host arrays passed to
 * any call are copied before the call returns.  Streams are borrowed
 * (hipStream_t passed as void*).
 *
 * Field layout (device): per simulation, per substrate, a volume
 * [z][y][x] with x fastest (structure of arrays), elements of the context's
 * precision (float for VL_F32, double for VL_F64).  Every volume starts on a
 * 256-byte boundary; vl_field_offset gives the element offset of a
 * simulation's first volume and vl_volume_stride the distance between its
 * substrates.
 *
 * Errors.  Every call returns VL_OK (0) or a negative VL_E_* code; the message
 * of the last failure on the calling thread is returned by vl_last_error()
 * (valid until the next call on that thread).  Kernel faults surface at the
 * next synchronising call (vl_sync, vl_mass, vl_get_field, vl_check_finite).
 * A context is not thread-safe; distinct contexts are independent.
 */
#ifndef VOXLOD_H
#define VOXLOD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VL_ABI_VERSION 1

/* status codes */
#define VL_OK 0
#define VL_E_ARG (-1)       /* an argument is out of range or inconsistent   */
#define VL_E_STATE (-2)     /* call not allowed in the context's current state */
#define VL_E_SHAPE (-3)     /* sizes do not fit the reserved layout          */
#define VL_E_HIP (-4)       /* the HIP runtime reported an error             */
#define VL_E_NONFINITE (-5) /* a non-finite value was found                  */

/* precision of field storage and of the line solves */
#define VL_F32 0 /* FP32 field; coefficients computed in FP64 on the device */
#define VL_F64 1 /* FP64 field, plain one-line-per-thread kernels           */

/* placement of the decay term */
#define VL_DECAY_ONCE 0   /* F = 1/(1 + lambda dt) after the x solve (default) */
#define VL_DECAY_THIRDS 1 /* sigma = lambda dt / 3 on every direction         */

/* boundary kinds, faces 0..5 = x-, x+, y-, y+, z-, z+ */
#define VL_NEUMANN 0
#define VL_DIRICHLET 1

/* host-side field layouts for vl_set_field / vl_get_field */
#define VL_SOA 0 /* [s][z][y][x]  */
#define VL_AOS 1 /* [z][y][x][s]  (the paper's voxel-major order) */

/* kernel kinds reported by vl_kernel_stats */
#define VL_K_SWEEP_X 0
#define VL_K_SWEEP_Y 1
#define VL_K_SWEEP_Z 2
#define VL_K_SOURCES 3
#define VL_K_DIRICHLET 4
#define VL_K_DECAY 5
#define VL_K_STEP 6 /* the one-launch step (VL_MODE_PERSISTENT) */
/* inside vl_adjoint (its forward steps count as the kinds above) */
#define VL_K_REPLAY_X 7 /* forward solves that also keep their raw output */
#define VL_K_REPLAY_Y 8
#define VL_K_REPLAY_Z 9
#define VL_K_ADJ_X 10 /* reverse solves with the parameter partial sums */
#define VL_K_ADJ_Y 11
#define VL_K_ADJ_Z 12
#define VL_K_ADJ_SOURCES 13
#define VL_K_ADJ_REDUCE 14
#define VL_K_ADJ_COPY 15 /* checkpoint and state copies */
#define VL_K_SWEEP_XY 16  /* x and y solves of one z-plane per workgroup */
#define VL_K_COUNT 17

typedef struct vl_ctx vl_ctx;

/* Library plumbing (no passage of the paper defines these): the ABI version
 * this header describes, and the message of the calling thread's last
 * failure. */
int vl_abi_version(void);
const char *vl_last_error(void);

/* Lifecycle.  n_sims >= 1 independent simulations share one context and are
 * stepped together (each launch covers all of them).  Each simulation is one
 * instance of Eq. (1) on its own voxel grid; running many at once serves the
 * exploration and calibration runs of section "Introduction and Motivation"
 * (many independent simulations of one model).  precision VL_F32 or VL_F64
 * (section "Methods of Validation for Data Integrity", Method 2: the paper's
 * field is double precision); decay_split VL_DECAY_ONCE or VL_DECAY_THIRDS
 * (where the decay term of Eq. (1) enters the direction-by-direction solve,
 * which the paper does not state).  *out receives the context; VL_E_ARG on
 * a null out or a value out of range.  vl_destroy frees the host state
 * (device memory stays the caller's); a null context is accepted. */
int vl_create(vl_ctx **out, int n_sims, int precision, int decay_split);
int vl_destroy(vl_ctx *ctx);

/* Per-simulation setup (before vl_finalize; VL_E_STATE after it, VL_E_ARG
 * for a simulation index out of range or a value out of its limits).
 * vl_set_grid (Eq. (1) discretised on a uniform voxel grid, section "Elements
 * of Parallelism": one substrate vector per voxel; section "Input Datasets":
 * a cube domain of voxels): nx, ny, nz >= 1 voxels of edges dx, dy, dz > 0 (um), lower
 *   corner (x0, y0, z0).  Each volume must hold fewer than 2^28 voxels;
 *   the FP32 path takes lines of at most 513 voxels.
 * vl_set_substrates (the diffusion coefficient D and decay rate lambda of
 *   each substrate in Eq. (1)): n_sub >= 1, D[s] >= 0 (um^2/min),
 *   lambda[s] >= 0 (1/min); the host arrays hold n_sub values each and are
 *   copied.  All faces start zero-flux.
 * vl_set_boundary (section "Elements of Parallelism": Dirichlet conditions
 *   are applied by a function of their own around the direction solves;
 *   section "Methods of Validation for Data Integrity", Method 3, where a
 *   mistake in that function's index range showed in the images): face
 *   0..5 = x-, x+, y-, y+, z-, z+ of substrate sub becomes VL_NEUMANN (zero
 *   flux) or VL_DIRICHLET with a finite value, which overwrites the outermost
 *   voxel layer of that face before the x solve and after each solve.
 * vl_reserve_cells (the cells i of Eq. (1)'s source sum): capacity for
 *   vl_upload_cells (default 0, max 2^24); it sizes the cell tables of the
 *   workspace. */
int vl_set_grid(vl_ctx *ctx, int sim, int nx, int ny, int nz, double dx, double dy,
                double dz, double x0, double y0, double z0);
int vl_set_substrates(vl_ctx *ctx, int sim, int n_sub, const double *D,
                      const double *lambda);
int vl_set_boundary(vl_ctx *ctx, int sim, int sub, int face, int kind, double value);
int vl_reserve_cells(vl_ctx *ctx, int sim, int max_cells);

/* Change one simulation's cell capacity after vl_finalize (the cells i of
 * Eq. (1)'s source sum, for agent populations that grow past the capacity
 * reserved at set-up; the paper's hybrid model adds and removes cells as it
 * runs).  Waits for the bound stream, lays the workspace out again for the
 * new capacities and reports its size in *workspace_bytes (may be NULL); the
 * field layout does not change.  The context is then unbound: call vl_bind
 * again, with the same field (its values are kept) and a workspace of that
 * size, and upload every simulation's cells again (vl_bind clears them).
 * The old workspace is the caller's to free once vl_bind returns.
 * VL_E_STATE before vl_finalize or while a snapshot is in flight; VL_E_ARG
 * for max_cells outside [0, 2^24]. */
int vl_resize_cells(vl_ctx *ctx, int sim, int max_cells, size_t *workspace_bytes);

/* Fix the layout for time step dt > 0 and report the sizes the caller must
 * allocate: *field_elems elements of the context's precision and
 * *workspace_bytes bytes (256-byte aligned device memory).  Section
 * "Elements of Parallelism": the arrays the diffusion solves need besides the
 * densities are set up once and stay on the device; here they are the line
 * solve pivots, the launch tables and the cell tables, all placed in the one
 * workspace.  Host-only: no device call.  VL_E_STATE if a simulation lacks a
 * grid or substrates or the context is already finalized; VL_E_SHAPE if
 * lines are too long for the FP32 path or the tables overflow. */
int vl_finalize(vl_ctx *ctx, double dt, size_t *field_elems, size_t *workspace_bytes);

/* Attach device memory and a stream.  Computes the line-solve coefficients
 * on the device (FP64 arithmetic) and uploads the launch tables (section
 * "Elements of Parallelism": the densities and the auxiliary arrays are
 * copied to the device once and stay resident; the elimination constants of
 * the line solves depend only on dt, D, lambda and the grid).  field_dev and
 * workspace_dev are device pointers of the sizes vl_finalize reported,
 * 256-byte aligned and owned by the caller (VL_E_ARG otherwise).  The field
 * contents are left as they are.  Synchronises the stream.  May be called
 * again to move to other buffers or another stream; the workspace is then
 * re-initialised and cells must be uploaded again.  stream may be NULL
 * (the null stream; steps are then launched without a graph). */
int vl_bind(vl_ctx *ctx, void *field_dev, void *workspace_dev, void *stream);

/* Change one simulation's D and lambda after vl_bind (n_sub values each, same
 * limits as vl_set_substrates; n_sub must equal the count set before
 * vl_finalize).  Recomputes that context's line-solve coefficients on the
 * bound stream, ordered after work already queued there; the tile tables and
 * cells are unchanged.  This is what a parameter-fitting loop calls between
 * a gradient step and the next forward run. */
int vl_update_substrates(vl_ctx *ctx, int sim, int n_sub, const double *D,
                         const double *lambda);

/* Where one simulation's volumes lie in the field (section "Elements of
 * Parallelism" ports the paper's per-voxel density vectors to flat arrays;
 * here each substrate is a volume of its own, x fastest): the element offset
 * of substrate 0 and the element distance between substrates.  Host-only;
 * VL_E_STATE before vl_finalize. */
int vl_field_offset(vl_ctx *ctx, int sim, size_t *elem_offset);
int vl_volume_stride(vl_ctx *ctx, int sim, size_t *elems);

/* Copy one simulation's field in or out.  src/dst hold n_sub*nz*ny*nx elements
 * of the context's precision, host or device memory, in layout VL_SOA or
 * VL_AOS (VL_AOS is the paper's voxel-major order of section "Elements of
 * Parallelism"; reading the whole field back is how section "Methods of
 * Validation for Data Integrity", Method 2, compares GPU and CPU results
 * voxel by voxel).  Both synchronise the stream; the caller keeps src/dst. */
int vl_set_field(vl_ctx *ctx, int sim, const void *src, int src_is_device, int layout);
int vl_get_field(vl_ctx *ctx, int sim, void *dst, int dst_is_device, int layout);

/* Snapshots of one simulation's field while stepping goes on (section
 * "GPU-accelerated Long-time Simulations": long runs that save the full data
 * at fixed simulated-time intervals).  vl_snapshot enqueues, on the bound
 * stream after the work already queued there, a copy of simulation sim's
 * field into the caller's device buffer stage_dev, then a copy from there
 * into host_dst on a copy stream of the library's own, so the steps enqueued
 * afterwards run while the transfer goes on.  Both buffers hold
 * n_sub*nz*ny*nx elements of the context's precision in layout VL_SOA
 * (substrate-major, x fastest), the caller owns them, and they stay in use
 * until vl_snapshot_wait returns.  host_dst should be pinned (hipHostMalloc)
 * for the transfer to overlap the steps; with pageable memory the transfer
 * may complete before the call returns.  Each call orders its staging copy
 * after the previous call's transfer, so one staging buffer can serve every
 * snapshot.  vl_snapshot_wait blocks until every snapshot enqueued so far is
 * in host memory.  Not for use under stream capture.
 * Errors: VL_E_ARG (sim out of range, null buffer), VL_E_STATE (not bound),
 * VL_E_HIP. */
int vl_snapshot(vl_ctx *ctx, int sim, void *stage_dev, void *host_dst);
int vl_snapshot_wait(vl_ctx *ctx);

/* The cells of Eq. (1)'s source sum, whose secretion/uptake section "Future
 * Work" names as the next part to run on the device.
 * Upload n cells of one simulation (host arrays, row-major): pos n x 3 (um),
 * V n (um^3, > 0), S, U n x n_sub (1/min, >= 0), rho_star n x n_sub.  The
 * order is the order of application.  On the device: voxel of each cell
 * (FP64), stable sort by voxel, per occupied voxel the composite of its cells
 * (FP64 arithmetic).  *n_out_of_domain (may be NULL) receives the number of
 * cells outside the grid.  Synchronises the stream.  n = 0 removes all cells.
 * VL_E_SHAPE if n exceeds vl_reserve_cells' capacity; VL_E_ARG for a
 * volume <= 0, a negative rate or a non-finite value (nothing changes then). */
int vl_upload_cells(vl_ctx *ctx, int sim, int n, const double *pos, const double *V,
                    const double *S, const double *U, const double *rho_star,
                    int *n_out_of_domain);
/* The same upload from arrays that are already in device memory (same
 * layouts; the caller keeps ownership and the arrays are only read on the
 * bound stream during the call), for cells that move or change between
 * steps: the agents' mechanics can update them on the device and the
 * re-binning (voxel index, sort, composites; the same kernels as above)
 * needs no host copy.  The arrays are checked on the device first (volumes
 * finite and > 0, rates finite and >= 0, targets finite), which waits for
 * the stream once; on a failed check it returns VL_E_ARG and the previous
 * cells stay.  With n_out_of_domain NULL nothing else waits: the binning is
 * queued on the bound stream and reads the arrays there after the call
 * returns, so the caller leaves them unchanged until the stream has passed
 * the upload (the next vl_sync, or stream-ordered work); a non-null
 * n_out_of_domain reads the count back and synchronises the stream.  The
 * step graphs of vl_step survive uploads that keep every simulation's cell
 * count.  Cells come from the moving agents of the paper's hybrid model
 * (Eq. 1, section "Future Work" on moving cell secretion/uptake to the
 * device). */
int vl_upload_cells_dev(vl_ctx *ctx, int sim, int n, const double *pos, const double *V,
                        const double *S, const double *U, const double *rho_star,
                        int *n_out_of_domain);

/* Advance every simulation by n_steps steps of Eq. (1), asynchronously on the
 * bound stream: per step the x, y and z line solves of section "Elements of
 * Parallelism" (each line a tridiagonal elimination and back-substitution,
 * with the Dirichlet function around them), then the cells' secretion/uptake
 * (section "Future Work").  VL_E_STATE before vl_bind; n_steps < 0 is
 * VL_E_ARG.  Faults of the launched kernels surface at vl_sync.  With a
 * non-null stream the step is captured once into a hipGraph and replayed; the
 * graph is rebuilt after a change of binding or options, or an upload that
 * changes a simulation's number of cells (the cell tables themselves are
 * read from the workspace at every replay). */
int vl_step(vl_ctx *ctx, int n_steps);
/* Wait for the work queued on the bound stream (plumbing).  VL_E_HIP carries
 * a kernel fault; VL_E_STATE reports a one-launch step whose tile gave up
 * waiting. */
int vl_sync(vl_ctx *ctx);

/* Diagnostics (synchronising).  vl_mass: out[s] = sum over voxels of rho (FP64
 * accumulation, deterministic order); with zero-flux faces and lambda = 0 the
 * diffusion part of Eq. (1) conserves it, which is what the validation of
 * section "Methods of Validation for Data Integrity" relies on.
 * vl_check_finite: *bad = number of non-finite field values (status
 * VL_E_NONFINITE when > 0).  out holds n_sub doubles (host, caller's). */
int vl_mass(vl_ctx *ctx, int sim, double *out);
int vl_check_finite(vl_ctx *ctx, long long *bad);

/* Options.  VL_OPT_FUSE_SOURCES (FP32 path, default 1): 1 applies the cell
 * sources inside the z sweep, right after each tile's stores (the occupied
 * voxels of 64 z-lines form one contiguous range of a per-simulation list
 * ordered by z-line); 0 applies them with a separate kernel over all occupied
 * voxels; 2 carries a step's sources into the next step's x solve (each
 * line gets them as it is loaded, before the Dirichlet projection that opens
 * the step; both kinds of x solve do this), and one pass at the end of every
 * vl_step call applies the last step's, so the field is whole whenever
 * vl_step returns (with x and y solved per z-plane, 2 acts as 1).  All three
 * give bitwise identical fields; vl_tune times them. */
#define VL_OPT_FUSE_SOURCES 1
/* VL_OPT_STEP_MODE (FP32 path): VL_MODE_LAUNCHES (default) launches one
 * kernel per sweep and capacity class, each covering every simulation;
 * VL_MODE_PERSISTENT runs the whole step as one launch whose workgroups take
 * tiles from a single queue (all x tiles, then y, then z) and start a volume's
 * y (z) tiles once its x (y) tiles are done, so ragged batches need no global
 * barrier.  VL_OPT_PERSISTENT_GRID: workgroups of that launch (0 = as many
 * as fit on the device at once).  VL_OPT_WAIT_LIMIT_US: microseconds a tile
 * may wait for the previous sweep of its volume before it gives up (default
 * 2000000); once one wait has given up, every later wait of the same launch
 * gives up at once, so the limit bounds the launch.  Giving up makes the next
 * vl_sync fail with VL_E_STATE, so a step can never hang (the limit exists
 * for tests of that path). */
#define VL_OPT_STEP_MODE 2
#define VL_OPT_PERSISTENT_GRID 3
#define VL_OPT_WAIT_LIMIT_US 4
#define VL_MODE_LAUNCHES 0
#define VL_MODE_PERSISTENT 1
/* VL_OPT_XCD_ORDER (default 1): workgroup b of a sweep runs on XCD b mod 8;
 * with 1 each XCD gets a contiguous range of tiles (neighbouring tiles share
 * an L2), with 0 tiles follow the workgroup index. */
#define VL_OPT_XCD_ORDER 5
/* VL_OPT_FUSE_XY (FP32 path, default 0): 1 solves x and y of every z-plane
 * that fits in LDS (160 KiB: up to 199 x 199 voxels) in one workgroup, which
 * reads and writes the field once for both solves; volumes with larger
 * planes keep the separate x and y sweeps.  Fields are bitwise identical
 * either way.  One plane per workgroup leaves its load, solve and store
 * phases unoverlapped, so on the grids measured so far the separate sweeps
 * are as fast or faster; vl_tune times both.  Without the device's support
 * for that much LDS per workgroup the option has no effect. */
#define VL_OPT_FUSE_XY 6
/* VL_OPT_X_LANES (FP32 path, default 1): 1 solves x-lines of 129 or more
 * voxels with the lanes of a wave along one line (each lane 4 consecutive
 * voxels for lines up to 256, 8 up to 512, 9 beyond; wide coalesced loads and
 * stores, no LDS transpose): each lane eliminates its run locally and the
 * runs' last voxels form a tridiagonal system over the lanes, solved by
 * parallel cyclic reduction with multipliers computed in FP64 when the
 * coefficients are (vl_bind, vl_update_substrates).  The same linear system
 * as the split solve, to rounding.  Shorter lines keep the split solve.
 * 2 does the same for lines of 65 or more voxels (2 per lane below 129),
 * which pays on large grids with such lines and not on batches of small
 * ones.  Used when x and y are not solved per plane; the adjoint's replay
 * follows it.  0 uses the split solve for every line; vl_tune times them. */
#define VL_OPT_X_LANES 7
/* VL_OPT_X_LANE_LINES (FP32 path, default 8): x-lines each wave of that
 * solve takes one after another: 1, 2, 4, 8 or 16.  A workgroup is four
 * waves, so a launch has (lines / (4 * value)) workgroups: small values give
 * many short workgroups (a short tail when the grid is only a few rounds of
 * the device), large ones keep more loads in flight per wave.  Fields do not
 * depend on it; vl_tune times the candidates. */
#define VL_OPT_X_LANE_LINES 8
/* VL_OPT_ADJOINT_TABLES (FP32 path, default 1): a cell upload also writes the
 * per-cell tables that only vl_adjoint reads (each cell's a_i, b_i, k_i
 * rho*_i and k_i, in voxel order; about 24 bytes per cell and substrate).
 * 0 skips them, for callers that only step forward: the fields do not
 * change, and vl_adjoint returns VL_E_STATE while any simulation holds cells
 * uploaded without them.  It applies to the uploads that follow. */
#define VL_OPT_ADJOINT_TABLES 9
/* VL_OPT_Z_SOURCES_STORING (FP32 path, default -1): where the z sweep of
 * lines of up to 129 voxels applies the cell sources when they are applied
 * in the z sweep: 1 while each tile stores its rows (its occupied voxels
 * staged in LDS, up to 1024 per tile), 0 in a pass over them after the
 * tile's stores, -1 (auto) the first when the field is larger than the 256
 * MB Infinity Cache, where that pass would re-read lines from HBM.  Fields
 * are bitwise the same either way. */
#define VL_OPT_Z_SOURCES_STORING 10
/* Launch-shape options (no passage of the paper defines them; fields do not
 * depend on them beyond rounding, and the placements of the sources and the
 * x+y-per-plane option give bitwise equal fields).  Unknown options and
 * values out of range are VL_E_ARG.
 * Selecting VL_MODE_PERSISTENT currently fails with VL_E_STATE: the one-launch
 * step is switched off until a hang seen in its first GPU runs is explained. */
int vl_set_option(vl_ctx *ctx, int option, int value);
int vl_get_option(vl_ctx *ctx, int option, int *value);

/* Autotuner (launch shapes only; no passage of the paper defines it, and it
 * never changes results beyond rounding): times the candidate launch configurations (x+y per z-plane or
 * separate sweeps, x lanes along the line or the split x solve and its lines
 * per wave, XCD tile order on or off, sources fused into the z sweep or
 * separate) on the bound buffers, a
 * few steps each (which overwrite the field), and keeps the fastest.  With a
 * non-NULL cache_path the choice is read from / appended to that text file,
 * keyed by precision, decay split and every volume's shape, so a second call
 * for the same shapes does no timing.  No-op for VL_F64. */
int vl_tune(vl_ctx *ctx, const char *cache_path);

/* Adjoint of n_steps steps (FP32 contexts; for VL_F64 both return VL_E_STATE):
 * the transpose of the step of vl_step, for fitting the parameters of
 * Eq. (1) (D, lambda per substrate; S_i, U_i per cell) to observed fields, the
 * calibration use that section "Introduction and Motivation" motivates.
 * For a scalar loss L whose gradient with respect to the field after n_steps
 * steps is grad_final (device, field layout, field_elems floats), computes
 *   grad_rho0 (device, field layout; may be NULL)  dL/d(field now),
 *   dD, dlambda (host, one double per volume, simulations in order and their
 *     substrates in order; may be NULL)            dL/dD_s, dL/dlambda_s,
 *   dS, dU (device doubles, per simulation its cells in upload order, each
 *     cell's substrates in order; required when cells exist) dL/dS_is, dL/dU_is
 *     (zero for cells outside the grid).
 * The forward run starts from the current field, keeps a checkpoint every
 * ckpt_every steps and replays each segment; the field is restored on return.
 * Reverse of a step: the adjoint of the sources (cells walked backwards per
 * voxel, FP64), then of the z, y and x solves in that order (the line matrices
 * are symmetric, so each is the same split solve) with the Dirichlet adjoint
 * folded in; parameter sums are FP64 and taken in a fixed order.
 * The caller allocates the adjoint workspace of vl_adjoint_workspace's size
 * (256-byte aligned device memory).  Synchronises the stream. */
int vl_adjoint_workspace(vl_ctx *ctx, int n_steps, int ckpt_every, size_t *bytes);
int vl_adjoint(vl_ctx *ctx, int n_steps, int ckpt_every, void *adj_workspace,
               const void *grad_final, void *grad_rho0, double *dD, double *dlambda,
               double *dS, double *dU);

/* Per-kernel timing (the per-function profile of section "Profiling;
 * Identifying Hot Spots", which found the diffusion solves to be about two
 * thirds of the run time).  While enabled, vl_step launches without a graph and
 * brackets every kernel with HIP events on the bound stream; so does
 * vl_adjoint.
 * vl_kernel_stats synchronises and reports, for one VL_K_* kind, the number
 * of launches and their summed duration since profiling was enabled. */
int vl_set_profiling(vl_ctx *ctx, int enable);
int vl_kernel_stats(vl_ctx *ctx, int kind, long long *launches, double *total_ms);

/* Copy probe (measurement plumbing; no passage of the paper defines it):
 * copies bytes from src to dst, both device memory, 16-byte aligned, either
 * the same buffer (dst == src: every element read and written back in place,
 * the way a sweep updates its field) or not overlapping at all, bytes a
 * multiple of 16, with width-byte accesses per lane (4, 8 or 16) and, per
 * bit of nontemporal (0 to 3), non-temporal loads (bit 0) and stores (bit 1);
 * nontemporal 4 (width 16) copies in 64 KiB tiles instead, each workgroup
 * loading its whole tile before storing it, the access shape of a sweep
 * tile.  Asynchronous on stream (hipStream_t as void*, NULL = the null
 * stream).  Each sweep of vl_step reads and writes every element once,
 * so a copy of the field's bytes is the practical ceiling a sweep is measured
 * against; it is also the kernel of known traffic that scales the HBM byte
 * counters.  The caller owns both buffers.  VL_E_ARG for a bad argument
 * (including buffers that overlap without being the same), VL_E_HIP if the
 * launch fails. */
int vl_copy_probe(void *dst, const void *src, size_t bytes, int width, int nontemporal, void *stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): the FP64 sums of
 * vl_mass without a context or workspace.  out_dev[q] (device memory, n_vols
 * doubles) receives the sum of the n_vox elements starting at element
 * q*vol_stride of field_dev (device memory of the given precision, VL_F32 or
 * VL_F64), for q < n_vols; with vl_field_offset and vl_volume_stride this is
 * one simulation's per-substrate mass.  Same kernels and summation order as
 * vl_mass, so the sums are bitwise equal.  Asynchronous on stream (NULL = the
 * null stream); no allocation and no synchronisation.  The partial sums live
 * in a static array of the library on each GPU (64 volumes x 256 doubles,
 * 128 KiB, held until the process ends), shared by every call on that GPU:
 * calls that overlap on one GPU race.  The caller owns field_dev and
 * out_dev.  VL_E_SHAPE for more than 64 volumes; VL_E_ARG for a null or
 * misaligned buffer, n_vox < 1, or vol_stride < n_vox with several volumes;
 * VL_E_HIP if a launch fails. */
int vl_mass_noalloc(const void *field_dev, int precision, long long n_vox, int n_vols,
                    long long vol_stride, double *out_dev, void *stream);

#ifdef __cplusplus
}
#endif
#endif
