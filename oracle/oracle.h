/*
 * oracle.h -- plain FP64 CPU reference for the locally-one-dimensional (LOD)
 * diffusion-decay step with cell secretion/uptake.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests and the
 * benchmark's CPU-baseline leg can check and time the GPU library.  No product
 * code may link, load or call it, and it shares no source with the GPU path.
 *
 * What it computes (Stack, Macklin, Searles, Chandrasekaran, "OpenACC
 * Acceleration of an Agent-Based Biological Simulation Framework",
 * arXiv:2110.13368):
 *
 *   Eq. (1):  d(rho)/dt = D lap(rho) - lambda rho
 *                         + sum_i delta(x - x_i) V_i ( S_i (rho*_i - rho) - U_i rho )
 *
 *   discretised on a uniform voxel grid.  Section "Elements of Parallelism"
 *   states that the diffusion part is solved direction by direction (x, y and
 *   z in 3-D), that each direction is a set of line solves built from an
 *   elimination (axpy) and a back-substitution (naxpy) over the substrate
 *   vector, and that Dirichlet conditions are applied by a separate function.
 *   Everything below that the paper leaves open is a documented reading:
 *
 *   - line matrix T = tridiag(-c, b, -c), c = dt*D_s/h_a^2, zero-flux ends:
 *     b_0 = b_{n-1} = 1 + c + sigma, interior b = 1 + 2c + sigma; n = 1 gives
 *     b_0 = 1 + sigma;
 *   - decay: ORC_DECAY_ONCE divides by (1 + lambda*dt) once per step, right
 *     after the x solve (sigma = 0); ORC_DECAY_THIRDS puts sigma = lambda*dt/3
 *     on the diagonal of every direction;
 *   - Dirichlet projection P_D overwrites the outermost voxel layer of every
 *     Dirichlet face; on edges and corners the last active face in the order
 *     x-, x+, y-, y+, z-, z+ wins;
 *   - one step is  C . P_D . S_z . P_D . S_y . P_D . F . S_x . P_D
 *     where S_a is the set of line solves along axis a, F the decay factor
 *     and C the cell sources;
 *   - C visits the cells in index order; cell i, inside voxel v, does for
 *     every substrate s
 *         rho[v][s] <- (rho[v][s] + a_is) / b_is,
 *         k_i  = dt * V_i / V_vox,
 *         a_is = k_i * S_is * rho*_is,
 *         b_is = 1 + k_i * (S_is + U_is),
 *     which is the backward-Euler step of the delta term of Eq. (1) with the
 *     delta function replaced by 1/V_vox on the voxel holding x_i;
 *   - a cell at x belongs to voxel floor((x - x0)/dx) per axis on the
 *     half-open box; cells outside are skipped and counted.
 *
 * Storage is the paper's voxel-major layout (section "Elements of
 * Parallelism": one substrate vector per voxel): rho[v*n_sub + s] with
 * v = i + nx*(j + ny*k).  All arithmetic is IEEE double, divisions are true
 * divisions, and the library is compiled without FMA contraction.
 *
 * Error handling: functions returning int give 0 on success and -1 on a bad
 * argument; they never abort.  The caller owns every array it passes; the
 * library copies what it keeps.  A handle is not thread-safe; the library
 * itself uses OpenMP over independent lines, which does not change any result.
 */
#ifndef VOXLOD_ORACLE_H
#define VOXLOD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NEUMANN 0
#define ORC_DIRICHLET 1

#define ORC_DECAY_ONCE 0
#define ORC_DECAY_THIRDS 1

#define ORC_LAYOUT_AOS 0 /* rho[v][s] */
#define ORC_LAYOUT_SOA 1 /* rho[s][v] */

typedef struct orc_sim orc_sim;

/* Create a grid of nx*ny*nz voxels of size dx*dy*dz whose lower corner is
 * (x0, y0, z0), with n_sub substrates of diffusion coefficients D[s] and decay
 * rates lambda[s], diffusion time step dt and decay placement decay_mode.
 * All faces start as zero-flux; the field starts at 0.  NULL on bad input. */
orc_sim *orc_create(int nx, int ny, int nz, double dx, double dy, double dz,
                    double x0, double y0, double z0, int n_sub,
                    const double *D, const double *lambda, double dt,
                    int decay_mode);
void orc_destroy(orc_sim *sim);

/* face: 0..5 = x-, x+, y-, y+, z-, z+; kind ORC_NEUMANN or ORC_DIRICHLET. */
int orc_set_boundary(orc_sim *sim, int s, int face, int kind, double value);

/* Copy the whole field in or out (n_vox*n_sub doubles) in either layout. */
int orc_set_field(orc_sim *sim, const double *src, int layout);
int orc_get_field(const orc_sim *sim, double *dst, int layout);

/* Register n cells (replacing any earlier set).  pos is n x 3, V is n,
 * S, U, rho_star are n x n_sub, all row-major.  The order of the arrays is the
 * order in which C applies the cells.  *n_out receives the number of cells
 * outside the grid (may be NULL). */
int orc_upload_cells(orc_sim *sim, int n, const double *pos, const double *V,
                     const double *S, const double *U, const double *rho_star,
                     int *n_out);
/* Voxel index of each registered cell, -1 when outside (n entries). */
int orc_cell_voxels(const orc_sim *sim, long long *out);

/* Advance n_steps full LOD steps. */
int orc_step(orc_sim *sim, int n_steps);

/* The single operators of one step, for tests. */
int orc_sweep(orc_sim *sim, int axis);  /* S_a */
int orc_decay(orc_sim *sim);            /* F (identity for ORC_DECAY_THIRDS) */
int orc_dirichlet(orc_sim *sim);        /* P_D */
int orc_sources(orc_sim *sim);          /* C */

/* M_s = sum over voxels of rho[v][s], summed in voxel order (n_sub doubles). */
int orc_mass(const orc_sim *sim, double *out);

/* Solve T x = r for one line of length n with off-diagonal -c and diagonal
 * shift sigma by the Thomas algorithm (elimination, then back-substitution). */
int orc_thomas_line(int n, double c, double sigma, const double *r, double *x);

/* Adjoint of n_steps steps started from the current field.  The forward run is
 * replayed internally (the current field is left unchanged).  g_final is the
 * gradient of a scalar loss with respect to the field after the last step
 * (SoA, n_sub*n_vox).  Outputs: g_rho0 (SoA, n_sub*n_vox) with respect to the
 * starting field, dD and dlambda (n_sub each), dS and dU (n_cells x n_sub,
 * zero for cells outside the grid).  Any output pointer may be NULL. */
int orc_adjoint(const orc_sim *sim, int n_steps, const double *g_final,
                double *g_rho0, double *dD, double *dlambda, double *dS,
                double *dU);

/* OpenMP thread count used by the line loops (<= 0 leaves the default). */
void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
