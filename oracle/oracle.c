/*
 * oracle.c -- plain FP64 CPU reference for the LOD diffusion-decay step with
 * cell secretion/uptake (arXiv:2110.13368, Eq. (1) and section "Elements of
 * Parallelism").  TEST INFRASTRUCTURE ONLY: see oracle.h for the readings of
 * the paper that this file implements and for the API contract.
 *
 * Every operator works on the whole field in the paper's voxel-major layout
 * rho[v*n_sub + s], v = i + nx*(j + ny*k).  Lines are independent, so the line
 * loops are OpenMP-parallel; each line is solved by the same serial code, so
 * the result does not depend on the thread count.  Sums that feed gradients
 * are formed per line and then added in line order, for the same reason.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_sim {
    int n[3];
    double h[3];
    double lo[3];
    long long nvox;
    int ns;
    double *D;
    double *lambda;
    double dt;
    int decay_mode;
    int *bc_kind;     /* [s*6 + face] */
    double *bc_value; /* [s*6 + face] */
    double *rho;      /* [v*ns + s] */
    int ncell;
    long long *cell_vox; /* voxel of cell i, -1 when outside */
    double *cell_k;      /* k_i = dt * V_i / V_vox */
    double *cell_S;      /* [i*ns + s] */
    double *cell_U;
    double *cell_rs;     /* rho*_is */
    double *cell_a;      /* a_is = k_i S_is rho*_is */
    double *cell_b;      /* b_is = 1 + k_i (S_is + U_is) */
};

/* ------------------------------------------------------------------------ */
/* Line geometry.                                                           */

static long long stride_of(const orc_sim *sim, int axis)
{
    if (axis == 0) return 1;
    if (axis == 1) return sim->n[0];
    return (long long)sim->n[0] * sim->n[1];
}

/* First voxel of line L along axis (lines are numbered by the two other
 * coordinates, lower axis fastest). */
static long long line_start(const orc_sim *sim, int axis, long long L)
{
    long long nx = sim->n[0], ny = sim->n[1];
    if (axis == 0) return L * nx;              /* L = j + ny*k */
    if (axis == 1) return (L % nx) + nx * ny * (L / nx); /* L = i + nx*k */
    return L;                                  /* L = i + nx*j */
}

/* c = dt*D_s/h_a^2, the off-diagonal magnitude of the implicit line system. */
static double line_c(const orc_sim *sim, int axis, int s)
{
    return sim->dt * sim->D[s] / (sim->h[axis] * sim->h[axis]);
}

/* Diagonal shift: lambda*dt/3 per direction when decay is split over the
 * three solves, else 0 (decay is then the separate factor F). */
static double line_sigma(const orc_sim *sim, int s)
{
    if (sim->decay_mode == ORC_DECAY_THIRDS) return sim->lambda[s] * sim->dt / 3.0;
    return 0.0;
}

/* Main diagonal of row i of the zero-flux line matrix. */
static double line_diag(int n, int i, double c, double sigma)
{
    if (n == 1) return 1.0 + sigma;
    if (i == 0 || i == n - 1) return 1.0 + c + sigma;
    return 1.0 + 2.0 * c + sigma;
}

/* Thomas algorithm (Thomas 1949; Golub & Van Loan, Matrix Computations,
 * sec. 4.3) for tridiag(-c, b_i, -c) x = r.  d holds n doubles of scratch.
 * Elimination:        d_0 = b_0,  d_i = b_i - c^2/d_{i-1},
 *                     y_0 = r_0/d_0,  y_i = (r_i + c y_{i-1})/d_i
 * Back-substitution:  x_{n-1} = y_{n-1},  x_i = y_i + (c/d_i) x_{i+1}.
 * x may alias r. */
static void thomas(int n, double c, double sigma, const double *r, double *x,
                   double *d)
{
    d[0] = line_diag(n, 0, c, sigma);
    x[0] = r[0] / d[0];
    for (int i = 1; i < n; ++i) {
        d[i] = line_diag(n, i, c, sigma) - c * c / d[i - 1];
        x[i] = (r[i] + c * x[i - 1]) / d[i];
    }
    for (int i = n - 2; i >= 0; --i) x[i] = x[i] + (c / d[i]) * x[i + 1];
}

int orc_thomas_line(int n, double c, double sigma, const double *r, double *x)
{
    if (n < 1 || !r || !x) return -1;
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    if (!d) return -1;
    thomas(n, c, sigma, r, x, d);
    free(d);
    return 0;
}

/* (K y)_i with K = tridiag(1, -2, 1) and zero-flux ends, so that the line
 * matrix is T = (1 + sigma) I - c K. */
static double lap_row(int n, int i, const double *y)
{
    if (n == 1) return 0.0;
    if (i == 0) return y[1] - y[0];
    if (i == n - 1) return y[n - 2] - y[n - 1];
    return y[i - 1] - 2.0 * y[i] + y[i + 1];
}

/* ------------------------------------------------------------------------ */
/* Forward operators on an arbitrary field buffer.                          */

/* S_a: solve every line along axis for every substrate. */
static void sweep_buf(const orc_sim *sim, double *rho, int axis)
{
    const int n = sim->n[axis];
    const int ns = sim->ns;
    const long long stride = stride_of(sim, axis);
    const long long nlines = sim->nvox / n;
    for (int s = 0; s < ns; ++s) {
        const double c = line_c(sim, axis, s);
        const double sigma = line_sigma(sim, s);
#pragma omp parallel
        {
            double *r = (double *)malloc(sizeof(double) * (size_t)n);
            double *d = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
            for (long long L = 0; L < nlines; ++L) {
                const long long v0 = line_start(sim, axis, L);
                for (int t = 0; t < n; ++t) r[t] = rho[(v0 + t * stride) * ns + s];
                thomas(n, c, sigma, r, r, d);
                for (int t = 0; t < n; ++t) rho[(v0 + t * stride) * ns + s] = r[t];
            }
            free(r);
            free(d);
        }
    }
}

/* F: implicit decay rho <- rho / (1 + lambda dt), once per step. */
static void decay_buf(const orc_sim *sim, double *rho)
{
    if (sim->decay_mode != ORC_DECAY_ONCE) return;
    const int ns = sim->ns;
#pragma omp parallel for schedule(static)
    for (long long v = 0; v < sim->nvox; ++v)
        for (int s = 0; s < ns; ++s)
            rho[v * ns + s] = rho[v * ns + s] / (1.0 + sim->lambda[s] * sim->dt);
}

/* Visit every voxel of one face (the layer i_a = 0 or n_a - 1 of axis
 * a = face/2): runs body with v set to each voxel of that layer. */
#define FOR_FACE_VOXELS(sim, face, v, body)                                     \
    do {                                                                        \
        const int ax_ = (face) / 2;                                             \
        const long long layer_ = ((face) % 2) ? (sim)->n[ax_] - 1 : 0;          \
        const int au_ = ax_ == 0 ? 1 : 0;                                       \
        const int aw_ = ax_ == 2 ? 1 : 2;                                       \
        for (long long w_ = 0; w_ < (sim)->n[aw_]; ++w_)                        \
            for (long long u_ = 0; u_ < (sim)->n[au_]; ++u_) {                  \
                long long c_[3];                                                \
                c_[ax_] = layer_;                                               \
                c_[au_] = u_;                                                   \
                c_[aw_] = w_;                                                   \
                const long long v = c_[0] + (sim)->n[0] * (c_[1] + (long long)(sim)->n[1] * c_[2]); \
                body;                                                           \
            }                                                                   \
    } while (0)

/* P_D: overwrite the outermost layer of every Dirichlet face, faces taken in
 * the order x-, x+, y-, y+, z-, z+ so that the last active face wins. */
static void dirichlet_buf(const orc_sim *sim, double *rho)
{
    const int ns = sim->ns;
    for (int face = 0; face < 6; ++face)
        for (int s = 0; s < ns; ++s) {
            if (sim->bc_kind[s * 6 + face] != ORC_DIRICHLET) continue;
            const double g = sim->bc_value[s * 6 + face];
            FOR_FACE_VOXELS(sim, face, v, rho[v * ns + s] = g);
        }
}

/* Adjoint of P_D: the output at a Dirichlet voxel does not depend on the
 * input, so the adjoint is zeroed there. */
static void dirichlet_adj(const orc_sim *sim, double *w)
{
    const int ns = sim->ns;
    for (int face = 0; face < 6; ++face)
        for (int s = 0; s < ns; ++s) {
            if (sim->bc_kind[s * 6 + face] != ORC_DIRICHLET) continue;
            FOR_FACE_VOXELS(sim, face, v, w[v * ns + s] = 0.0);
        }
}

/* C: the cells in index order; each one applies the backward-Euler update of
 * its delta source to the voxel that holds it.  When after != NULL the value
 * just after cell i is recorded in after[i*ns + s]. */
static void sources_buf(const orc_sim *sim, double *rho, double *after)
{
    const int ns = sim->ns;
    for (int i = 0; i < sim->ncell; ++i) {
        const long long v = sim->cell_vox[i];
        if (v < 0) continue;
        for (int s = 0; s < ns; ++s) {
            double *p = &rho[v * ns + s];
            *p = (*p + sim->cell_a[(size_t)i * ns + s]) / sim->cell_b[(size_t)i * ns + s];
            if (after) after[(size_t)i * ns + s] = *p;
        }
    }
}

/* One full step. */
static void step_buf(const orc_sim *sim, double *rho)
{
    dirichlet_buf(sim, rho);
    sweep_buf(sim, rho, 0);
    decay_buf(sim, rho);
    dirichlet_buf(sim, rho);
    sweep_buf(sim, rho, 1);
    dirichlet_buf(sim, rho);
    sweep_buf(sim, rho, 2);
    dirichlet_buf(sim, rho);
    sources_buf(sim, rho, NULL);
}

/* ------------------------------------------------------------------------ */
/* Public forward API.                                                      */

static int valid_num(double x) { return isfinite(x); }

orc_sim *orc_create(int nx, int ny, int nz, double dx, double dy, double dz,
                    double x0, double y0, double z0, int n_sub,
                    const double *D, const double *lambda, double dt,
                    int decay_mode)
{
    if (nx < 1 || ny < 1 || nz < 1 || n_sub < 1 || !D || !lambda) return NULL;
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !(dt > 0)) return NULL;
    if (!valid_num(dx) || !valid_num(dy) || !valid_num(dz) || !valid_num(dt)) return NULL;
    if (!valid_num(x0) || !valid_num(y0) || !valid_num(z0)) return NULL;
    if (decay_mode != ORC_DECAY_ONCE && decay_mode != ORC_DECAY_THIRDS) return NULL;
    for (int s = 0; s < n_sub; ++s)
        if (!(D[s] >= 0) || !(lambda[s] >= 0) || !valid_num(D[s]) || !valid_num(lambda[s]))
            return NULL;
    orc_sim *sim = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!sim) return NULL;
    sim->n[0] = nx; sim->n[1] = ny; sim->n[2] = nz;
    sim->h[0] = dx; sim->h[1] = dy; sim->h[2] = dz;
    sim->lo[0] = x0; sim->lo[1] = y0; sim->lo[2] = z0;
    sim->nvox = (long long)nx * ny * nz;
    sim->ns = n_sub;
    sim->dt = dt;
    sim->decay_mode = decay_mode;
    sim->D = (double *)malloc(sizeof(double) * n_sub);
    sim->lambda = (double *)malloc(sizeof(double) * n_sub);
    sim->bc_kind = (int *)calloc((size_t)n_sub * 6, sizeof(int));
    sim->bc_value = (double *)calloc((size_t)n_sub * 6, sizeof(double));
    sim->rho = (double *)calloc((size_t)sim->nvox * n_sub, sizeof(double));
    if (!sim->D || !sim->lambda || !sim->bc_kind || !sim->bc_value || !sim->rho) {
        orc_destroy(sim);
        return NULL;
    }
    memcpy(sim->D, D, sizeof(double) * n_sub);
    memcpy(sim->lambda, lambda, sizeof(double) * n_sub);
    return sim;
}

static void free_cells(orc_sim *sim)
{
    free(sim->cell_vox); free(sim->cell_k); free(sim->cell_S); free(sim->cell_U);
    free(sim->cell_rs); free(sim->cell_a); free(sim->cell_b);
    sim->cell_vox = NULL; sim->cell_k = NULL; sim->cell_S = NULL; sim->cell_U = NULL;
    sim->cell_rs = NULL; sim->cell_a = NULL; sim->cell_b = NULL;
    sim->ncell = 0;
}

void orc_destroy(orc_sim *sim)
{
    if (!sim) return;
    free(sim->D); free(sim->lambda); free(sim->bc_kind); free(sim->bc_value);
    free(sim->rho);
    free_cells(sim);
    free(sim);
}

int orc_set_boundary(orc_sim *sim, int s, int face, int kind, double value)
{
    if (!sim || s < 0 || s >= sim->ns || face < 0 || face > 5) return -1;
    if (kind != ORC_NEUMANN && kind != ORC_DIRICHLET) return -1;
    if (!valid_num(value)) return -1;
    sim->bc_kind[s * 6 + face] = kind;
    sim->bc_value[s * 6 + face] = value;
    return 0;
}

int orc_set_field(orc_sim *sim, const double *src, int layout)
{
    if (!sim || !src) return -1;
    const int ns = sim->ns;
    if (layout == ORC_LAYOUT_AOS) {
        memcpy(sim->rho, src, sizeof(double) * (size_t)sim->nvox * ns);
    } else if (layout == ORC_LAYOUT_SOA) {
        for (int s = 0; s < ns; ++s)
            for (long long v = 0; v < sim->nvox; ++v)
                sim->rho[v * ns + s] = src[(size_t)s * sim->nvox + v];
    } else {
        return -1;
    }
    return 0;
}

int orc_get_field(const orc_sim *sim, double *dst, int layout)
{
    if (!sim || !dst) return -1;
    const int ns = sim->ns;
    if (layout == ORC_LAYOUT_AOS) {
        memcpy(dst, sim->rho, sizeof(double) * (size_t)sim->nvox * ns);
    } else if (layout == ORC_LAYOUT_SOA) {
        for (int s = 0; s < ns; ++s)
            for (long long v = 0; v < sim->nvox; ++v)
                dst[(size_t)s * sim->nvox + v] = sim->rho[v * ns + s];
    } else {
        return -1;
    }
    return 0;
}

/* Voxel of a point on the half-open grid, -1 when outside (or not finite). */
static long long voxel_of(const orc_sim *sim, const double *p)
{
    long long idx[3];
    for (int a = 0; a < 3; ++a) {
        const double t = floor((p[a] - sim->lo[a]) / sim->h[a]);
        if (!(t >= 0.0) || !(t < (double)sim->n[a])) return -1;
        idx[a] = (long long)t;
    }
    return idx[0] + (long long)sim->n[0] * (idx[1] + (long long)sim->n[1] * idx[2]);
}

int orc_upload_cells(orc_sim *sim, int n, const double *pos, const double *V,
                     const double *S, const double *U, const double *rho_star,
                     int *n_out)
{
    if (!sim || n < 0) return -1;
    if (n > 0 && (!pos || !V || !S || !U || !rho_star)) return -1;
    const int ns = sim->ns;
    for (int i = 0; i < n; ++i) {
        if (!(V[i] > 0) || !valid_num(V[i])) return -1;
        for (int s = 0; s < ns; ++s) {
            const size_t q = (size_t)i * ns + s;
            if (!(S[q] >= 0) || !(U[q] >= 0) || !valid_num(S[q]) || !valid_num(U[q]) ||
                !valid_num(rho_star[q]))
                return -1;
        }
    }
    free_cells(sim);
    if (n == 0) {
        if (n_out) *n_out = 0;
        return 0;
    }
    sim->cell_vox = (long long *)malloc(sizeof(long long) * n);
    sim->cell_k = (double *)malloc(sizeof(double) * n);
    sim->cell_S = (double *)malloc(sizeof(double) * (size_t)n * ns);
    sim->cell_U = (double *)malloc(sizeof(double) * (size_t)n * ns);
    sim->cell_rs = (double *)malloc(sizeof(double) * (size_t)n * ns);
    sim->cell_a = (double *)malloc(sizeof(double) * (size_t)n * ns);
    sim->cell_b = (double *)malloc(sizeof(double) * (size_t)n * ns);
    if (!sim->cell_vox || !sim->cell_k || !sim->cell_S || !sim->cell_U || !sim->cell_rs ||
        !sim->cell_a || !sim->cell_b) {
        free_cells(sim);
        return -1;
    }
    sim->ncell = n;
    const double vvox = sim->h[0] * sim->h[1] * sim->h[2];
    int outside = 0;
    for (int i = 0; i < n; ++i) {
        sim->cell_vox[i] = voxel_of(sim, &pos[3 * (size_t)i]);
        if (sim->cell_vox[i] < 0) ++outside;
        const double k = sim->dt * V[i] / vvox;
        sim->cell_k[i] = k;
        for (int s = 0; s < ns; ++s) {
            const size_t q = (size_t)i * ns + s;
            sim->cell_S[q] = S[q];
            sim->cell_U[q] = U[q];
            sim->cell_rs[q] = rho_star[q];
            sim->cell_a[q] = k * S[q] * rho_star[q];
            sim->cell_b[q] = 1.0 + k * (S[q] + U[q]);
        }
    }
    if (n_out) *n_out = outside;
    return 0;
}

int orc_cell_voxels(const orc_sim *sim, long long *out)
{
    if (!sim || (!out && sim->ncell > 0)) return -1;
    for (int i = 0; i < sim->ncell; ++i) out[i] = sim->cell_vox[i];
    return 0;
}

int orc_step(orc_sim *sim, int n_steps)
{
    if (!sim || n_steps < 0) return -1;
    for (int t = 0; t < n_steps; ++t) step_buf(sim, sim->rho);
    return 0;
}

int orc_sweep(orc_sim *sim, int axis)
{
    if (!sim || axis < 0 || axis > 2) return -1;
    sweep_buf(sim, sim->rho, axis);
    return 0;
}

int orc_decay(orc_sim *sim)
{
    if (!sim) return -1;
    decay_buf(sim, sim->rho);
    return 0;
}

int orc_dirichlet(orc_sim *sim)
{
    if (!sim) return -1;
    dirichlet_buf(sim, sim->rho);
    return 0;
}

int orc_sources(orc_sim *sim)
{
    if (!sim) return -1;
    sources_buf(sim, sim->rho, NULL);
    return 0;
}

int orc_mass(const orc_sim *sim, double *out)
{
    if (!sim || !out) return -1;
    const int ns = sim->ns;
    for (int s = 0; s < ns; ++s) {
        double m = 0.0;
        for (long long v = 0; v < sim->nvox; ++v) m += sim->rho[v * ns + s];
        out[s] = m;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint.                                                                 */

/* Adjoint of S_a.  On entry w is the adjoint of the sweep output y; on exit it
 * is the adjoint of the sweep input, T^{-T} w = T^{-1} w because every line
 * matrix is symmetric.  With T = (1 + sigma) I - c K, the derivative of the
 * loss with respect to c is  w_in^T K y  and with respect to sigma it is
 * -w_in^T y, summed over the lines of each substrate into gc[s], gsig[s]. */
static void sweep_adj(const orc_sim *sim, double *w, const double *y, int axis,
                      double *gc, double *gsig)
{
    const int n = sim->n[axis];
    const int ns = sim->ns;
    const long long stride = stride_of(sim, axis);
    const long long nlines = sim->nvox / n;
    double *part_c = (double *)malloc(sizeof(double) * (size_t)nlines);
    double *part_s = (double *)malloc(sizeof(double) * (size_t)nlines);
    for (int s = 0; s < ns; ++s) {
        const double c = line_c(sim, axis, s);
        const double sigma = line_sigma(sim, s);
#pragma omp parallel
        {
            double *r = (double *)malloc(sizeof(double) * (size_t)n);
            double *yy = (double *)malloc(sizeof(double) * (size_t)n);
            double *d = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
            for (long long L = 0; L < nlines; ++L) {
                const long long v0 = line_start(sim, axis, L);
                for (int t = 0; t < n; ++t) {
                    r[t] = w[(v0 + t * stride) * ns + s];
                    yy[t] = y[(v0 + t * stride) * ns + s];
                }
                thomas(n, c, sigma, r, r, d);
                double pc = 0.0, ps = 0.0;
                for (int t = 0; t < n; ++t) {
                    pc += r[t] * lap_row(n, t, yy);
                    ps -= r[t] * yy[t];
                }
                part_c[L] = pc;
                part_s[L] = ps;
                for (int t = 0; t < n; ++t) w[(v0 + t * stride) * ns + s] = r[t];
            }
            free(r);
            free(yy);
            free(d);
        }
        for (long long L = 0; L < nlines; ++L) {
            gc[s] += part_c[L];
            gsig[s] += part_s[L];
        }
    }
    free(part_c);
    free(part_s);
}

/* Adjoint of C.  rho_after holds, per cell, the value just after that cell was
 * applied in the forward pass.  Walking the cells in reverse index order, with
 * w the adjoint of the value after cell i:  abar = w/b,  bbar = -w*after_i/b,
 * w <- w/b;  then dS += k (abar rho* + bbar) and dU += k bbar because
 * a = k S rho* and b = 1 + k (S + U). */
static void sources_adj(const orc_sim *sim, double *w, const double *rho_after,
                        double *dS, double *dU)
{
    const int ns = sim->ns;
    for (int i = sim->ncell - 1; i >= 0; --i) {
        const long long v = sim->cell_vox[i];
        if (v < 0) continue;
        const double k = sim->cell_k[i];
        for (int s = 0; s < ns; ++s) {
            const size_t q = (size_t)i * ns + s;
            const double b = sim->cell_b[q];
            const double wv = w[v * ns + s];
            const double abar = wv / b;
            const double bbar = -wv * rho_after[q] / b;
            w[v * ns + s] = wv / b;
            if (dS) dS[q] += k * (abar * sim->cell_rs[q] + bbar);
            if (dU) dU[q] += k * bbar;
        }
    }
}

/* Adjoint of one step that started from rho_t.  The step is replayed to get
 * the intermediates; w enters as the adjoint of the step's output and leaves
 * as the adjoint of rho_t.  gc[a][s], gsig[a][s], glam[s] accumulate. */
static int step_adj(const orc_sim *sim, const double *rho_t, double *w,
                    double *gc, double *gsig, double *glam, double *dS, double *dU)
{
    const size_t nf = (size_t)sim->nvox * sim->ns;
    const int ns = sim->ns;
    double *y_x = (double *)malloc(sizeof(double) * nf); /* S_x output */
    double *y_y = (double *)malloc(sizeof(double) * nf); /* S_y output */
    double *y_z = (double *)malloc(sizeof(double) * nf); /* S_z output */
    double *r = (double *)malloc(sizeof(double) * nf);
    double *after = (double *)malloc(sizeof(double) * ((size_t)sim->ncell * ns + 1));
    if (!y_x || !y_y || !y_z || !r || !after) {
        free(y_x); free(y_y); free(y_z); free(r); free(after);
        return -1;
    }
    /* replay: r0 -> P_D -> S_x (y_x) -> F -> P_D -> S_y (y_y) -> P_D -> S_z (y_z)
     *         -> P_D -> C */
    memcpy(r, rho_t, sizeof(double) * nf);
    dirichlet_buf(sim, r);
    sweep_buf(sim, r, 0);
    memcpy(y_x, r, sizeof(double) * nf);
    decay_buf(sim, r);
    dirichlet_buf(sim, r);
    sweep_buf(sim, r, 1);
    memcpy(y_y, r, sizeof(double) * nf);
    dirichlet_buf(sim, r);
    sweep_buf(sim, r, 2);
    memcpy(y_z, r, sizeof(double) * nf);
    dirichlet_buf(sim, r);
    sources_buf(sim, r, after);

    /* reverse */
    sources_adj(sim, w, after, dS, dU);
    dirichlet_adj(sim, w);
    sweep_adj(sim, w, y_z, 2, gc + 2 * ns, gsig + 2 * ns);
    dirichlet_adj(sim, w);
    sweep_adj(sim, w, y_y, 1, gc + 1 * ns, gsig + 1 * ns);
    dirichlet_adj(sim, w);
    if (sim->decay_mode == ORC_DECAY_ONCE) {
        /* F: out = in / (1 + lambda dt);  d out / d lambda = -dt in / (1+lambda dt)^2 */
        for (int s = 0; s < ns; ++s) {
            const double q = 1.0 + sim->lambda[s] * sim->dt;
            double acc = 0.0;
            for (long long v = 0; v < sim->nvox; ++v) {
                acc += w[v * ns + s] * y_x[v * ns + s];
                w[v * ns + s] = w[v * ns + s] / q;
            }
            glam[s] += -sim->dt * acc / (q * q);
        }
    }
    sweep_adj(sim, w, y_x, 0, gc + 0 * ns, gsig + 0 * ns);
    dirichlet_adj(sim, w);
    free(y_x); free(y_y); free(y_z); free(r); free(after);
    return 0;
}

int orc_adjoint(const orc_sim *sim, int n_steps, const double *g_final,
                double *g_rho0, double *dD, double *dlambda, double *dS,
                double *dU)
{
    if (!sim || n_steps < 0 || !g_final) return -1;
    const int ns = sim->ns;
    const size_t nf = (size_t)sim->nvox * ns;
    const size_t nc = (size_t)sim->ncell * ns;
    double *w = (double *)malloc(sizeof(double) * nf);
    double *gc = (double *)calloc(3 * (size_t)ns, sizeof(double));
    double *gsig = (double *)calloc(3 * (size_t)ns, sizeof(double));
    double *glam = (double *)calloc((size_t)ns, sizeof(double));
    double *gS = (double *)calloc(nc + 1, sizeof(double));
    double *gU = (double *)calloc(nc + 1, sizeof(double));
    /* checkpoints every K steps, K ~ sqrt(n); each segment is replayed */
    int K = 1;
    while ((long long)K * K < n_steps) ++K;
    const int nck = n_steps / K + 1;
    double *ck = (double *)malloc(sizeof(double) * nf * (size_t)nck);
    double *seg = (double *)malloc(sizeof(double) * nf * (size_t)K);
    int rc = 0;
    if (!w || !gc || !gsig || !glam || !gS || !gU || !ck || !seg) {
        rc = -1;
        goto done;
    }
    /* adjoint input: g_final is SoA */
    for (int s = 0; s < ns; ++s)
        for (long long v = 0; v < sim->nvox; ++v) w[v * ns + s] = g_final[(size_t)s * sim->nvox + v];
    memcpy(ck, sim->rho, sizeof(double) * nf);
    for (int c = 1; c < nck; ++c) {
        memcpy(ck + nf * c, ck + nf * (c - 1), sizeof(double) * nf);
        for (int t = 0; t < K; ++t) step_buf(sim, ck + nf * c);
    }
    for (int c = nck - 1; c >= 0; --c) {
        const int t0 = c * K;
        int t1 = t0 + K;
        if (t1 > n_steps) t1 = n_steps;
        if (t1 <= t0) continue;
        memcpy(seg, ck + nf * c, sizeof(double) * nf);
        for (int t = t0 + 1; t < t1; ++t) {
            memcpy(seg + nf * (t - t0), seg + nf * (t - t0 - 1), sizeof(double) * nf);
            step_buf(sim, seg + nf * (t - t0));
        }
        for (int t = t1 - 1; t >= t0; --t)
            if (step_adj(sim, seg + nf * (t - t0), w, gc, gsig, glam, gS, gU) != 0) {
                rc = -1;
                goto done;
            }
    }
    if (g_rho0)
        for (int s = 0; s < ns; ++s)
            for (long long v = 0; v < sim->nvox; ++v) g_rho0[(size_t)s * sim->nvox + v] = w[v * ns + s];
    for (int s = 0; s < ns; ++s) {
        /* c_a = dt D / h_a^2;  sigma = lambda dt / 3 when split over the solves */
        double d = 0.0, l = glam[s];
        for (int a = 0; a < 3; ++a) {
            d += gc[a * ns + s] * (sim->dt / (sim->h[a] * sim->h[a]));
            if (sim->decay_mode == ORC_DECAY_THIRDS) l += gsig[a * ns + s] * (sim->dt / 3.0);
        }
        if (dD) dD[s] = d;
        if (dlambda) dlambda[s] = l;
    }
    if (dS) memcpy(dS, gS, sizeof(double) * nc);
    if (dU) memcpy(dU, gU, sizeof(double) * nc);
done:
    free(w); free(gc); free(gsig); free(glam); free(gS); free(gU); free(ck); free(seg);
    return rc;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
