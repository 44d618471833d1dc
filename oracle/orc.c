/*
 * Reference (oracle) solver for the staggered-grid Poisson and Helmholtz
 * problems of the fractional-step method (paper eqs. e and f of the
 * Runge-Kutta sub-step, Section 2.1; linear systems, Section 2.3.3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct CPU definition that the GPU library is checked against.  It is
 * used by tests/, by the smoke check and by the benchmark's CPU-baseline
 * leg; the GPU library never links, loads or calls it, and it shares no
 * code with the GPU library.
 *
 * What it does, in FP64 (long double only where stated):
 *   - builds the (optionally tanh-stretched) staggered grid in y;
 *   - applies the staggered divergence D and gradient G (second-order
 *     central differences on a staggered grid, Section 2.1), periodic in
 *     x and z, walls in y;
 *   - assembles the 7-point operators L_p = D G (pressure), L_c (velocity
 *     components stored at cell-centre height, Dirichlet wall by a mirror
 *     ghost: Appendix B, alpha = 2) and L_f (wall-normal velocity on the
 *     y faces, Dirichlet wall value: Appendix B, alpha = 1) as CSR, in the
 *     symmetric weighted form S = W(-L_p) or S = W(I - cL);
 *   - solves S x = f by Jacobi-preconditioned conjugate gradients to a
 *     true relative residual of 1e-14, then polishes with a few steps of
 *     iterative refinement whose residual b - A x is evaluated from the
 *     flux form of the stencil in long double;
 *   - for the pressure problem, projects the right-hand side onto the
 *     compatible subspace (Neumann compatibility: weighted mean of b is
 *     zero) and returns the solution with zero volume-weighted mean (the
 *     null mode is fixed; the paper fixes it by a zero mean in the triply
 *     periodic solver, Section 2.3.3, item S2).
 *
 * Array layout: C order [z][y][x] (x fastest).  Cell fields and the x- and
 * z-face velocities are [nz][ny][nx]; the y-face velocity v is
 * [nz][ny+1][nx], faces j = 0 and j = ny being the walls (ignored on input,
 * written as zero on output).
 *
 * Triply periodic variant (geometry flag py; the paper's 3-periodic branch,
 * Section 2.3.3, items S1 and S2): y wraps like x and z, every operator uses
 * its interior formula everywhere (the distance across the wrap,
 * (Delta_0 + Delta_{ny-1})/2, is delta_0 = delta_ny), v has ny faces
 * ([nz][ny][nx], face ny being face 0), and the pressure's null mode is
 * fixed by the same zero weighted mean.
 *
 * Walls in x (geometry flag wx; the non-periodic direction of the paper's
 * inflow-outflow example, Section 3.2, as walls): the faces x = 0 and
 * x = lx bound the domain.  The x-face velocity u is Dirichlet there (zero
 * on both wall faces) and keeps the [nz][ny][nx] layout: slot i holds face
 * i, slot 0 being the wall face x = 0 (ignored on input, written as zero on
 * output; the wall face x = lx is not stored), so its unknowns are faces
 * 1..nx-1.  v and w (cell centres in x) take the mirror-ghost Dirichlet
 * row, as u and w do at the y walls; the pressure takes homogeneous Neumann
 * (zero flux through the walls), so its null mode is again the constant.
 * Walls in z (flag wz) are the same construction along z: w's plane k holds
 * the face z = k hz, plane 0 being the wall face (unknowns: planes
 * 1..nz-1); u and v take the mirror-ghost row, the pressure zero flux.
 * A wall-bounded x or z may be stretched (dxc/dxf, dzc/dzf): its rows are
 * then the flux forms with the local widths, as the y rows are, and the
 * weights W carry the local widths too.
 *
 * Operator codes: 0 = pressure Poisson (A = L_p), 1 = u Helmholtz,
 * 2 = v Helmholtz, 3 = w Helmholtz (A = I - c L).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, nz;
    double hx, hz;
    const double *dyc; /* [ny]    cell heights Delta_j                  */
    const double *dyf; /* [ny+1]  centre-to-centre distances delta_j,   */
                       /*         valid for j = 1..ny-1 (periodic y:    */
                       /*         also j = 0 and ny, the distance       */
                       /*         across the wrap)                      */
    int py;            /* 1: y periodic too (the triply periodic        */
                       /*    branch, Section 2.3.3, items S1/S2): no    */
                       /*    walls, v has ny faces [nz][ny][nx]         */
    int wx;            /* 1: walls at x = 0 and x = lx instead of the   */
                       /*    periodic x (see the header comment)        */
    int wz;            /* 1: walls at z = 0 and z = lz, the same way    */
                       /*    (w's plane 0 is the wall face z = 0)       */
    const double *dxc; /* NULL, or with walls in x the cell widths      */
                       /*    Delta^x_i [nx] of a stretched x            */
    const double *dxf; /*    and the centre distances delta^x_i [nx+1]  */
                       /*    (valid for i = 1..nx-1)                    */
    const double *dzc; /* the same for a stretched z with walls         */
    const double *dzf;
} orc_geom;

typedef struct {
    int iters;          /* CG iterations of the main solve            */
    int polish_steps;   /* refinement steps after the main solve      */
    int polish_iters;   /* CG iterations spent in refinement          */
    int stagnated;      /* 1 if the main CG stalled above tolerance   */
    double rel_residual;    /* ||b - A x|| / ||b|| (long double, final) */
    double removed_mean;    /* weighted mean removed from b (Poisson)  */
} orc_info;

/* ------------------------------------------------------------------ */
/* Grid (uniform x, z; tanh-stretched y).                              */
/* ------------------------------------------------------------------ */

/* Face positions y_f[j] = (ly/2) (1 + tanh(beta (2j/ny - 1)) / tanh(beta)),
 * j = 0..ny; beta = 0 gives the uniform grid of Section 2.1.  If yf_in is
 * non-NULL it is copied instead.  Outputs: centres yc[ny], heights
 * dyc[ny] = yf[j+1]-yf[j], distances dyf[ny+1] with dyf[j] = yc[j]-yc[j-1]
 * for j = 1..ny-1 and dyf[0] = dyf[ny] = 0. */
int orc_grid(int ny, double ly, double beta, const double *yf_in, double *yf,
             double *yc, double *dyc, double *dyf)
{
    if (ny < 1) return -1;
    for (int j = 0; j <= ny; ++j) {
        if (yf_in) {
            yf[j] = yf_in[j];
        } else if (beta == 0.0) {
            yf[j] = ly * (double)j / (double)ny;
        } else {
            double t = tanh(beta * (2.0 * (double)j / (double)ny - 1.0));
            yf[j] = 0.5 * ly * (1.0 + t / tanh(beta));
        }
    }
    for (int j = 0; j < ny; ++j) {
        yc[j] = 0.5 * (yf[j] + yf[j + 1]);
        dyc[j] = yf[j + 1] - yf[j];
        if (!(dyc[j] > 0.0)) return -2;
    }
    dyf[0] = 0.0;
    dyf[ny] = 0.0;
    for (int j = 1; j < ny; ++j) dyf[j] = yc[j] - yc[j - 1];
    return 0;
}

static inline int64_t cidx(const orc_geom *g, int i, int j, int k)
{
    return ((int64_t)k * g->ny + j) * g->nx + i;
}
static inline int vrows(const orc_geom *g) { return g->py ? g->ny : g->ny + 1; }
static inline int64_t vidx(const orc_geom *g, int i, int j, int k)
{
    return ((int64_t)k * vrows(g) + j) * g->nx + i;
}
static inline int wrap(int i, int n) { return (i % n + n) % n; }
/* local widths: cell width and centre distance in x and z (uniform: h) */
static inline double DX(const orc_geom *g, int i) { return g->dxc ? g->dxc[i] : g->hx; }
static inline double DXF(const orc_geom *g, int i) { return g->dxf ? g->dxf[i] : g->hx; }
static inline double DZ(const orc_geom *g, int k) { return g->dzc ? g->dzc[k] : g->hz; }
static inline double DZF(const orc_geom *g, int k) { return g->dzf ? g->dzf[k] : g->hz; }

/* ------------------------------------------------------------------ */
/* Divergence and gradient (Section 2.1; kernels E2 and E3).           */
/* ------------------------------------------------------------------ */

/* b = scale * D(u,v,w) on cells:
 * (u_{i+1}-u_i)/hx + (v_{j+1}-v_j)/Delta_j + (w_{k+1}-w_k)/hz. */
void orc_divergence(const orc_geom *g, const double *u, const double *v,
                    const double *w, double scale, double *b)
{
#pragma omp parallel for collapse(2)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                /* x walls: u = 0 on the wall faces 0 and nx */
                double ue = (g->wx && i + 1 == g->nx) ? 0.0 : u[cidx(g, wrap(i + 1, g->nx), j, k)];
                double uw = (g->wx && i == 0) ? 0.0 : u[cidx(g, i, j, k)];
                double du = (ue - uw) / DX(g, i);
                /* z walls: w = 0 on the wall faces 0 and nz */
                double wt = (g->wz && k + 1 == g->nz) ? 0.0 : w[cidx(g, i, j, wrap(k + 1, g->nz))];
                double wb = (g->wz && k == 0) ? 0.0 : w[cidx(g, i, j, k)];
                int jt = (g->py && j + 1 == g->ny) ? 0 : j + 1;   /* face ny = face 0 */
                double dv = (v[vidx(g, i, jt, k)] - v[vidx(g, i, j, k)]) / g->dyc[j];
                double dw = (wt - wb) / DZ(g, k);
                b[cidx(g, i, j, k)] = scale * (du + dv + dw);
            }
}

/* Components of G(phi): (phi_i - phi_{i-1})/hx on x-faces (zero on the
 * wall face 0 with x walls), (phi_j - phi_{j-1})/delta_j on interior
 * y-faces (zero on the wall faces: homogeneous Neumann), (phi_k -
 * phi_{k-1})/hz on z-faces. */
void orc_gradient(const orc_geom *g, const double *phi, double *gu, double *gv,
                  double *gw)
{
#pragma omp parallel for collapse(2)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < vrows(g); ++j)
            for (int i = 0; i < g->nx; ++i) {
                if (g->py) {
                    /* every face is interior; face 0 lies between cells
                     * ny-1 and 0, dyf[0] apart */
                    gu[cidx(g, i, j, k)] = (g->wx && i == 0) ? 0.0 :
                        (phi[cidx(g, i, j, k)] - phi[cidx(g, wrap(i - 1, g->nx), j, k)]) / DXF(g, i);
                    gw[cidx(g, i, j, k)] = (g->wz && k == 0) ? 0.0 :
                        (phi[cidx(g, i, j, k)] - phi[cidx(g, i, j, wrap(k - 1, g->nz))]) / DZF(g, k);
                    gv[vidx(g, i, j, k)] =
                        (phi[cidx(g, i, j, k)] - phi[cidx(g, i, wrap(j - 1, g->ny), k)]) / g->dyf[j];
                    continue;
                }
                if (j < g->ny) {
                    gu[cidx(g, i, j, k)] = (g->wx && i == 0) ? 0.0 :
                        (phi[cidx(g, i, j, k)] - phi[cidx(g, wrap(i - 1, g->nx), j, k)]) / DXF(g, i);
                    gw[cidx(g, i, j, k)] = (g->wz && k == 0) ? 0.0 :
                        (phi[cidx(g, i, j, k)] - phi[cidx(g, i, j, wrap(k - 1, g->nz))]) / DZF(g, k);
                }
                if (j == 0 || j == g->ny)
                    gv[vidx(g, i, j, k)] = 0.0;
                else
                    gv[vidx(g, i, j, k)] =
                        (phi[cidx(g, i, j, k)] - phi[cidx(g, i, j - 1, k)]) / g->dyf[j];
            }
}

/* ------------------------------------------------------------------ */
/* Unknown numbering.                                                  */
/* ------------------------------------------------------------------ */

/* y unknowns per column: v has the interior faces 1..ny-1 with walls, all
 * ny faces when y is periodic; cell fields have ny */
static int ny_unknowns(const orc_geom *g, int op)
{
    return (op == 2 && !g->py) ? g->ny - 1 : g->ny;
}
static int first_y(const orc_geom *g, int op) { return (op == 2 && !g->py) ? 1 : 0; }
/* x unknowns per row: u has the interior faces 1..nx-1 with x walls */
static int nx_unknowns(const orc_geom *g, int op)
{
    return (op == 1 && g->wx) ? g->nx - 1 : g->nx;
}
static int first_x(const orc_geom *g, int op) { return (op == 1 && g->wx) ? 1 : 0; }
/* z planes of unknowns: w has the interior faces 1..nz-1 with z walls */
static int nz_unknowns(const orc_geom *g, int op)
{
    return (op == 3 && g->wz) ? g->nz - 1 : g->nz;
}
static int first_z(const orc_geom *g, int op) { return (op == 3 && g->wz) ? 1 : 0; }
static int64_t n_unknowns(const orc_geom *g, int op)
{
    return (int64_t)nx_unknowns(g, op) * ny_unknowns(g, op) * nz_unknowns(g, op);
}
/* (i, j, k) of unknown number r; for op 2 with walls, j is the face index
 * 1..ny-1; for op 1 with x walls, i is the face index 1..nx-1 */
static void unknown_ijk(const orc_geom *g, int op, int64_t r, int *i, int *j,
                        int *k)
{
    int nyu = ny_unknowns(g, op), nxu = nx_unknowns(g, op);
    *i = (int)(r % nxu) + first_x(g, op);
    int64_t t = r / nxu;
    *j = (int)(t % nyu) + first_y(g, op);
    *k = (int)(t / nyu) + first_z(g, op);
}
static int64_t unknown_id(const orc_geom *g, int op, int i, int j, int k)
{
    int nyu = ny_unknowns(g, op), nxu = nx_unknowns(g, op);
    int jj = j - first_y(g, op), ii = i - first_x(g, op), kk = k - first_z(g, op);
    return ((int64_t)kk * nyu + jj) * nxu + ii;
}
/* position of unknown r in the caller's full array layout */
static int64_t unknown_to_array(const orc_geom *g, int op, int64_t r)
{
    int i, j, k;
    unknown_ijk(g, op, r, &i, &j, &k);
    return (op == 2) ? vidx(g, i, j, k) : cidx(g, i, j, k);
}
/* weight W of unknown r: the volume of its control cell, Delta^x Delta_j
 * Delta^z for cells, with delta_j for y faces, delta^x for x faces and
 * delta^z for z faces (uniform x, z: hx, hz) */
static double unknown_weight(const orc_geom *g, int op, int64_t r)
{
    int i, j, k;
    unknown_ijk(g, op, r, &i, &j, &k);
    const double wxi = (op == 1) ? DXF(g, i) : DX(g, i);
    const double wzk = (op == 3) ? DZF(g, k) : DZ(g, k);
    return wxi * wzk * ((op == 2) ? g->dyf[j] : g->dyc[j]);
}

/* ------------------------------------------------------------------ */
/* Stencil of the unweighted Laplacian L for unknown (i,j,k).          */
/* Up to 7 (column, value) pairs, duplicates merged.                   */
/* ------------------------------------------------------------------ */
static int add_entry(int64_t *cols, double *vals, int n, int64_t c, double v)
{
    for (int q = 0; q < n; ++q)
        if (cols[q] == c) { vals[q] += v; return n; }
    cols[n] = c;
    vals[n] = v;
    return n + 1;
}

static int laplacian_row(const orc_geom *g, int op, int i, int j, int k,
                         int64_t *cols, double *vals)
{
    int n = 0;
    const double ax = 1.0 / (g->hx * g->hx), az = 1.0 / (g->hz * g->hz);
    int64_t me = unknown_id(g, op, i, j, k);
    if (!g->wz) { /* periodic z: (f_{k+1} - 2 f_k + f_{k-1}) / h^2 */
        n = add_entry(cols, vals, n, me, -2.0 * az);
        n = add_entry(cols, vals, n, unknown_id(g, op, i, j, wrap(k - 1, g->nz)), az);
        n = add_entry(cols, vals, n, unknown_id(g, op, i, j, wrap(k + 1, g->nz)), az);
    } else if (op == 3) { /* z faces 1..nz-1, wall values w_0 = w_nz = 0:
                           * ((w_{k+1}-w_k)/Dz_k - (w_k-w_{k-1})/Dz_{k-1}) / dz_k */
        const double at = 1.0 / (DZ(g, k) * DZF(g, k)), ab = 1.0 / (DZ(g, k - 1) * DZF(g, k));
        n = add_entry(cols, vals, n, me, -at - ab);
        if (k + 1 <= g->nz - 1) n = add_entry(cols, vals, n, unknown_id(g, op, i, j, k + 1), at);
        if (k - 1 >= 1) n = add_entry(cols, vals, n, unknown_id(g, op, i, j, k - 1), ab);
    } else { /* cell centres in z: Neumann (pressure) or mirror ghost (u, v) */
        const double D = DZ(g, k);
        if (k + 1 < g->nz) {
            const double a = 1.0 / (DZF(g, k + 1) * D);
            n = add_entry(cols, vals, n, me, -a);
            n = add_entry(cols, vals, n, unknown_id(g, op, i, j, k + 1), a);
        } else if (op != 0) {
            n = add_entry(cols, vals, n, me, -2.0 / (D * D));
        }
        if (k > 0) {
            const double a = 1.0 / (DZF(g, k) * D);
            n = add_entry(cols, vals, n, me, -a);
            n = add_entry(cols, vals, n, unknown_id(g, op, i, j, k - 1), a);
        } else if (op != 0) {
            n = add_entry(cols, vals, n, me, -2.0 / (D * D));
        }
    }
    if (!g->wx) { /* periodic x: the same */
        n = add_entry(cols, vals, n, me, -2.0 * ax);
        n = add_entry(cols, vals, n, unknown_id(g, op, wrap(i - 1, g->nx), j, k), ax);
        n = add_entry(cols, vals, n, unknown_id(g, op, wrap(i + 1, g->nx), j, k), ax);
    } else if (op == 1) { /* x faces 1..nx-1, wall values u_0 = u_nx = 0:
                           * ((u_{i+1}-u_i)/Dx_i - (u_i-u_{i-1})/Dx_{i-1}) / dx_i */
        const double ae = 1.0 / (DX(g, i) * DXF(g, i)), aw = 1.0 / (DX(g, i - 1) * DXF(g, i));
        n = add_entry(cols, vals, n, me, -ae - aw);
        if (i + 1 <= g->nx - 1) n = add_entry(cols, vals, n, unknown_id(g, op, i + 1, j, k), ae);
        if (i - 1 >= 1) n = add_entry(cols, vals, n, unknown_id(g, op, i - 1, j, k), aw);
    } else { /* cell centres in x: interior flux over delta^x, or at a wall
              * zero flux (pressure, Neumann) or the mirror-ghost flux
              * -2 f/Dx (v, w); divided by Dx_i */
        const double D = DX(g, i);
        if (i + 1 < g->nx) {
            const double a = 1.0 / (DXF(g, i + 1) * D);
            n = add_entry(cols, vals, n, me, -a);
            n = add_entry(cols, vals, n, unknown_id(g, op, i + 1, j, k), a);
        } else if (op != 0) {
            n = add_entry(cols, vals, n, me, -2.0 / (D * D));
        }
        if (i > 0) {
            const double a = 1.0 / (DXF(g, i) * D);
            n = add_entry(cols, vals, n, me, -a);
            n = add_entry(cols, vals, n, unknown_id(g, op, i - 1, j, k), a);
        } else if (op != 0) {
            n = add_entry(cols, vals, n, me, -2.0 / (D * D));
        }
    }
    const int ny = g->ny;
    if (g->py) {
        /* periodic y: the same interior formulas everywhere, neighbours
         * wrapping (cells: fluxes over delta; faces: over Delta) */
        int jn = wrap(j + 1, ny), js = wrap(j - 1, ny);
        double au, al;
        if (op == 2) {
            double d = g->dyf[j];
            au = 1.0 / (g->dyc[j] * d);
            al = 1.0 / (g->dyc[js] * d);
        } else {
            double D = g->dyc[j];
            au = 1.0 / (g->dyf[j + 1] * D);
            al = 1.0 / (g->dyf[j] * D);
        }
        n = add_entry(cols, vals, n, me, -au - al);
        n = add_entry(cols, vals, n, unknown_id(g, op, i, jn, k), au);
        n = add_entry(cols, vals, n, unknown_id(g, op, i, js, k), al);
        return n;
    }
    if (op == 0 || op == 1 || op == 3) {
        /* cell-centre height: (F_{j+1/2} - F_{j-1/2}) / Delta_j */
        double D = g->dyc[j];
        if (j + 1 < ny) { /* interior upper flux (f_{j+1}-f_j)/delta_{j+1} */
            double a = 1.0 / (g->dyf[j + 1] * D);
            n = add_entry(cols, vals, n, unknown_id(g, op, i, j + 1, k), a);
            n = add_entry(cols, vals, n, me, -a);
        } else if (op != 0) { /* wall above: mirror ghost, flux -2 f/Delta */
            n = add_entry(cols, vals, n, me, -2.0 / (D * D));
        } /* Poisson: homogeneous Neumann, zero flux */
        if (j > 0) {
            double a = 1.0 / (g->dyf[j] * D);
            n = add_entry(cols, vals, n, unknown_id(g, op, i, j - 1, k), a);
            n = add_entry(cols, vals, n, me, -a);
        } else if (op != 0) {
            n = add_entry(cols, vals, n, me, -2.0 / (D * D));
        }
    } else {
        /* y faces j = 1..ny-1: ((v_{j+1}-v_j)/Delta_j - (v_j-v_{j-1})/Delta_{j-1}) / delta_j,
         * wall values v_0 = v_ny = 0 */
        double d = g->dyf[j];
        double au = 1.0 / (g->dyc[j] * d), al = 1.0 / (g->dyc[j - 1] * d);
        n = add_entry(cols, vals, n, me, -au - al);
        if (j + 1 <= ny - 1) n = add_entry(cols, vals, n, unknown_id(g, op, i, j + 1, k), au);
        if (j - 1 >= 1) n = add_entry(cols, vals, n, unknown_id(g, op, i, j - 1, k), al);
    }
    return n;
}

/* Assemble the unweighted operator A (op 0: L_p; else I - cL) as CSR over
 * the unknowns.  rowptr has n+1 entries, col/val up to 7n.  Returns n. */
int64_t orc_assemble(const orc_geom *g, int op, double c, int64_t *rowptr,
                     int64_t *col, double *val)
{
    int64_t n = n_unknowns(g, op);
    rowptr[0] = 0;
    for (int64_t r = 0; r < n; ++r) {
        int i, j, k;
        int64_t cols[8];
        double vals[8];
        unknown_ijk(g, op, r, &i, &j, &k);
        int m = laplacian_row(g, op, i, j, k, cols, vals);
        if (op != 0) {
            for (int q = 0; q < m; ++q) vals[q] = -c * vals[q];
            m = add_entry(cols, vals, m, r, 1.0);
        }
        /* sort columns (insertion sort, m <= 7) */
        for (int a = 1; a < m; ++a)
            for (int b = a; b > 0 && cols[b - 1] > cols[b]; --b) {
                int64_t tc = cols[b]; cols[b] = cols[b - 1]; cols[b - 1] = tc;
                double tv = vals[b]; vals[b] = vals[b - 1]; vals[b - 1] = tv;
            }
        for (int q = 0; q < m; ++q) {
            col[rowptr[r] + q] = cols[q];
            val[rowptr[r] + q] = vals[q];
        }
        rowptr[r + 1] = rowptr[r] + m;
    }
    return n;
}

int64_t orc_num_unknowns(const orc_geom *g, int op) { return n_unknowns(g, op); }

/* weights W of all unknowns, in unknown order */
void orc_weights(const orc_geom *g, int op, double *w)
{
    int64_t n = n_unknowns(g, op);
    for (int64_t r = 0; r < n; ++r) w[r] = unknown_weight(g, op, r);
}

/* ------------------------------------------------------------------ */
/* Residual r = b - A x in long double, straight from the flux form.   */
/* x, b, r in the caller's full array layout.  Returns ||r||_2 and     */
/* ||b||_2 (over the unknowns) through norms[0], norms[1].             */
/* ------------------------------------------------------------------ */
/* lo, hi: wall data of column (i, k) at y = 0 and y = ly ([nz][nx] arrays,
 * NULL = homogeneous).  Poisson: the prescribed flux d(phi)/dy on the wall
 * face (Neumann).  u, w: the wall value of the velocity, imposed through
 * the mirror ghost f_ghost = 2 g - f_0, i.e. the wall flux
 * (f_0 - g)/(Delta_0/2) (Appendix B, alpha = 2).  v: the value of the wall
 * face itself (alpha = 1). */
static long double wall_at(const double *data, const orc_geom *g, int i, int k)
{
    return data ? (long double)data[(int64_t)k * g->nx + i] : 0.0L;
}

static long double flux_apply_bc_ld(const orc_geom *g, int op, int i, int j, int k,
                                    const double *x, const double *lo, const double *hi);
static long double flux_apply_ld(const orc_geom *g, int op, int i, int j, int k,
                                 const double *x)
{
    return flux_apply_bc_ld(g, op, i, j, k, x, NULL, NULL);
}

static long double flux_apply_bc_ld(const orc_geom *g, int op, int i, int j, int k,
                                    const double *x, const double *lo, const double *hi)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    long double hx = g->hx, hz = g->hz;
    int64_t (*at)(const orc_geom *, int, int, int) = (op == 2) ? vidx : cidx;
    long double xc = x[at(g, i, j, k)];
    long double ft, fb;   /* z fluxes through the top and bottom sides */
    if (!g->wz) {
        ft = ((long double)x[at(g, i, j, wrap(k + 1, nz))] - xc) / hz;
        fb = (xc - (long double)x[at(g, i, j, wrap(k - 1, nz))]) / hz;
    } else if (op == 3) { /* faces: wall values w_0 = w_nz = 0 */
        long double xt = (k + 1 <= nz - 1) ? (long double)x[at(g, i, j, k + 1)] : 0.0L;
        long double xb = (k - 1 >= 1) ? (long double)x[at(g, i, j, k - 1)] : 0.0L;
        ft = (xt - xc) / (long double)DZ(g, k);
        fb = (xc - xb) / (long double)DZ(g, k - 1);
        hz = DZF(g, k);
    } else { /* cells: Neumann (pressure) or mirror ghost (u, v) at a wall */
        const long double D = DZ(g, k);
        ft = (k + 1 < nz) ? ((long double)x[at(g, i, j, k + 1)] - xc) / (long double)DZF(g, k + 1)
                          : (op == 0 ? 0.0L : -xc / (D / 2.0L));
        fb = (k > 0) ? (xc - (long double)x[at(g, i, j, k - 1)]) / (long double)DZF(g, k)
                     : (op == 0 ? 0.0L : xc / (D / 2.0L));
        hz = D;
    }
    long double fe, fw;   /* x fluxes through the east and west sides */
    if (!g->wx) {
        fe = ((long double)x[at(g, wrap(i + 1, nx), j, k)] - xc) / hx;
        fw = (xc - (long double)x[at(g, wrap(i - 1, nx), j, k)]) / hx;
    } else if (op == 1) { /* faces: wall values u_0 = u_nx = 0 */
        long double xe = (i + 1 <= nx - 1) ? (long double)x[at(g, i + 1, j, k)] : 0.0L;
        long double xw = (i - 1 >= 1) ? (long double)x[at(g, i - 1, j, k)] : 0.0L;
        fe = (xe - xc) / (long double)DX(g, i);
        fw = (xc - xw) / (long double)DX(g, i - 1);
        hx = DXF(g, i);
    } else { /* cells: Neumann (pressure) or mirror ghost (v, w) at a wall */
        const long double D = DX(g, i);
        fe = (i + 1 < nx) ? ((long double)x[at(g, i + 1, j, k)] - xc) / (long double)DXF(g, i + 1)
                          : (op == 0 ? 0.0L : -xc / (D / 2.0L));
        fw = (i > 0) ? (xc - (long double)x[at(g, i - 1, j, k)]) / (long double)DXF(g, i)
                     : (op == 0 ? 0.0L : xc / (D / 2.0L));
        hx = D;
    }
    long double lap = (fe - fw) / hx + (ft - fb) / hz;
    if (g->py) {
        int jn = wrap(j + 1, ny), js = wrap(j - 1, ny);
        long double xn = x[at(g, i, jn, k)], xs = x[at(g, i, js, k)];
        if (op == 2) {
            long double fu = (xn - xc) / (long double)g->dyc[j];
            long double fl = (xc - xs) / (long double)g->dyc[js];
            lap += (fu - fl) / (long double)g->dyf[j];
        } else {
            long double fu = (xn - xc) / (long double)g->dyf[j + 1];
            long double fl = (xc - xs) / (long double)g->dyf[j];
            lap += (fu - fl) / (long double)g->dyc[j];
        }
        return lap;
    }
    if (op != 2) {
        long double D = g->dyc[j];
        long double fu, fl;
        if (j + 1 < ny) fu = ((long double)x[at(g, i, j + 1, k)] - xc) / (long double)g->dyf[j + 1];
        else fu = (op == 0) ? wall_at(hi, g, i, k) : (wall_at(hi, g, i, k) - xc) / (D / 2.0L);
        if (j > 0) fl = (xc - (long double)x[at(g, i, j - 1, k)]) / (long double)g->dyf[j];
        else fl = (op == 0) ? wall_at(lo, g, i, k) : (xc - wall_at(lo, g, i, k)) / (D / 2.0L);
        lap += (fu - fl) / D;
    } else {
        long double vu = (j + 1 <= ny - 1) ? (long double)x[vidx(g, i, j + 1, k)] : wall_at(hi, g, i, k);
        long double vl = (j - 1 >= 1) ? (long double)x[vidx(g, i, j - 1, k)] : wall_at(lo, g, i, k);
        long double fu = (vu - xc) / (long double)g->dyc[j];
        long double fl = (xc - vl) / (long double)g->dyc[j - 1];
        lap += (fu - fl) / (long double)g->dyf[j];
    }
    return lap;
}

void orc_residual_bc_ld(const orc_geom *g, int op, double c, const double *x,
                        const double *b, const double *lo, const double *hi,
                        double *r, double *norms);
void orc_residual_ld(const orc_geom *g, int op, double c, const double *x,
                     const double *b, double *r, double *norms)
{
    orc_residual_bc_ld(g, op, c, x, b, NULL, NULL, r, norms);
}

/* As orc_residual_ld, with inhomogeneous wall data lo, hi (see wall_at):
 * r = b - A(x; lo, hi), the operator applied with the wall fluxes or
 * values the data prescribe. */
void orc_residual_bc_ld(const orc_geom *g, int op, double c, const double *x,
                        const double *b, const double *lo, const double *hi,
                        double *r, double *norms)
{
    int64_t n = n_unknowns(g, op);
    long double rr = 0.0L, bb = 0.0L;
#pragma omp parallel for reduction(+ : rr, bb)
    for (int64_t q = 0; q < n; ++q) {
        int i, j, k;
        unknown_ijk(g, op, q, &i, &j, &k);
        int64_t a = unknown_to_array(g, op, q);
        long double lap = flux_apply_bc_ld(g, op, i, j, k, x, lo, hi);
        long double ax = (op == 0) ? lap : (long double)x[a] - (long double)c * lap;
        long double res = (long double)b[a] - ax;
        r[a] = (double)res;
        rr += res * res;
        bb += (long double)b[a] * (long double)b[a];
    }
    if (op == 2 && !g->py) {
        for (int k = 0; k < g->nz; ++k)
            for (int i = 0; i < g->nx; ++i) {
                r[vidx(g, i, 0, k)] = 0.0;
                r[vidx(g, i, g->ny, k)] = 0.0;
            }
    }
    if (op == 1 && g->wx) { /* the wall face x = 0 */
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j) r[cidx(g, 0, j, k)] = 0.0;
    }
    if (op == 3 && g->wz) { /* the wall face z = 0 */
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) r[cidx(g, i, j, 0)] = 0.0;
    }
    if (norms) {
        norms[0] = sqrt((double)rr);
        norms[1] = sqrt((double)bb);
    }
}

/* y = A x (unweighted, CSR), unknown ordering */
static void csr_mv(int64_t n, const int64_t *rp, const int64_t *ci, const double *v,
                   const double *x, double *y)
{
#pragma omp parallel for
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t q = rp[r]; q < rp[r + 1]; ++q) s += v[q] * x[ci[q]];
        y[r] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s)
    for (int64_t q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}

/* weighted mean sum(w x)/sum(w) */
static double wmean(int64_t n, const double *w, const double *x)
{
    long double s = 0.0L, t = 0.0L;
    for (int64_t q = 0; q < n; ++q) {
        s += (long double)w[q] * x[q];
        t += w[q];
    }
    return (double)(s / t);
}

/* Jacobi-preconditioned CG on the symmetric weighted system S x = f,
 * S = sgn * diag(w) * A (sgn = -1 for the pressure operator so that S is
 * positive semidefinite).  The true residual f - S x is recomputed every
 * 50 iterations and at the stop; stop when ||f - S x|| <= tol ||f||.
 * For the pressure problem the residual and the iterate are projected
 * onto the zero-weighted-mean subspace at each recomputation. */
static int pcg(int64_t n, const int64_t *rp, const int64_t *ci, const double *av,
               const double *w, double sgn, int proj, const double *f, double *x,
               double tol, int maxit, int *stagnated)
{
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    double *dinv = malloc(n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double dii = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] == i) dii = av[e];
        dinv[i] = 1.0 / (sgn * w[i] * dii);
    }
    double fn = sqrt(dot(n, f, f));
    if (fn == 0.0) {
        memset(x, 0, n * sizeof(double));
        free(r); free(z); free(p); free(q); free(dinv);
        return 0;
    }
    /* r = f - S x */
    csr_mv(n, rp, ci, av, x, q);
    for (int64_t i = 0; i < n; ++i) r[i] = f[i] - sgn * w[i] * q[i];
    for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    memcpy(p, z, n * sizeof(double));
    double rz = dot(n, r, z);
    int it = 0;
    double best = INFINITY;
    int since_best = 0;
    *stagnated = 0;
    for (it = 1; it <= maxit; ++it) {
        csr_mv(n, rp, ci, av, p, q);
#pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) q[i] *= sgn * w[i];
        double pq = dot(n, p, q);
        if (!(pq > 0.0)) break;
        double alpha = rz / pq;
#pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        if (it % 50 == 0) {
            if (proj) {
                double m = wmean(n, w, x);
                for (int64_t i = 0; i < n; ++i) x[i] -= m;
            }
            csr_mv(n, rp, ci, av, x, q);
#pragma omp parallel for
            for (int64_t i = 0; i < n; ++i) r[i] = f[i] - sgn * w[i] * q[i];
            double rn = sqrt(dot(n, r, r));
            if (rn <= tol * fn) break;
            if (rn < 0.999 * best) { best = rn; since_best = 0; }
            else if (++since_best >= 20) { *stagnated = 1; break; }
        }
#pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rz1 = dot(n, r, z);
        double beta = rz1 / rz;
        rz = rz1;
#pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        if (it % 50 != 0 && sqrt(dot(n, r, r)) <= tol * fn) {
            /* confirm on the true residual */
            csr_mv(n, rp, ci, av, x, q);
            for (int64_t i = 0; i < n; ++i) r[i] = f[i] - sgn * w[i] * q[i];
            if (sqrt(dot(n, r, r)) <= tol * fn) break;
        }
    }
    free(r); free(z); free(p); free(q); free(dinv);
    return it;
}

/* Solve A x = b for operator op (Helmholtz coefficient c ignored for
 * op 0).  b and x in the caller's full layout.  Returns 0 on success. */
int orc_solve(const orc_geom *g, int op, double c, const double *b_in, double *x_out,
              double tol, int maxit, orc_info *info)
{
    if (op < 0 || op > 3) return -1;
    if (op == 2 && g->ny < 2) return -1;
    int64_t n = n_unknowns(g, op);
    int64_t *rp = malloc((n + 1) * sizeof(int64_t));
    int64_t *ci = malloc(7 * n * sizeof(int64_t));
    double *av = malloc(7 * n * sizeof(double));
    double *w = malloc(n * sizeof(double));
    double *b = malloc(n * sizeof(double)), *f = malloc(n * sizeof(double));
    double *x = calloc(n, sizeof(double)), *d = malloc(n * sizeof(double));
    double *full_r = NULL;
    orc_assemble(g, op, c, rp, ci, av);
    orc_weights(g, op, w);
    for (int64_t q = 0; q < n; ++q) b[q] = b_in[unknown_to_array(g, op, q)];
    double sgn = (op == 0) ? -1.0 : 1.0;
    int proj = (op == 0);
    double removed = 0.0;
    if (proj) { /* Neumann compatibility: remove the weighted mean of b */
        removed = wmean(n, w, b);
        for (int64_t q = 0; q < n; ++q) b[q] -= removed;
    }
    for (int64_t q = 0; q < n; ++q) f[q] = sgn * w[q] * b[q];
    int stag = 0;
    int iters = pcg(n, rp, ci, av, w, sgn, proj, f, x, tol, maxit, &stag);
    if (proj) {
        double m = wmean(n, w, x);
        for (int64_t q = 0; q < n; ++q) x[q] -= m;
    }
    /* write out, evaluate the long double residual of the projected b */
    int64_t nfull = (op == 2) ? (int64_t)g->nx * vrows(g) * g->nz
                              : (int64_t)g->nx * g->ny * g->nz;
    double *full_b = calloc(nfull, sizeof(double));
    full_r = calloc(nfull, sizeof(double));
    memset(x_out, 0, nfull * sizeof(double));
    for (int64_t q = 0; q < n; ++q) {
        x_out[unknown_to_array(g, op, q)] = x[q];
        full_b[unknown_to_array(g, op, q)] = b[q];
    }
    double norms[2];
    orc_residual_ld(g, op, c, x_out, full_b, full_r, norms);
    /* polish: x += A^{-1} r with r from the long double flux residual */
    int psteps = 0, piters = 0;
    double prev = norms[0];
    for (int s = 0; s < 6 && norms[0] > 0.0; ++s) {
        for (int64_t q = 0; q < n; ++q) d[q] = full_r[unknown_to_array(g, op, q)];
        if (proj) {
            double m = wmean(n, w, d);
            for (int64_t q = 0; q < n; ++q) d[q] -= m;
        }
        for (int64_t q = 0; q < n; ++q) f[q] = sgn * w[q] * d[q];
        memset(d, 0, n * sizeof(double));
        int st2 = 0;
        piters += pcg(n, rp, ci, av, w, sgn, proj, f, d, 1e-12, maxit, &st2);
        for (int64_t q = 0; q < n; ++q) x[q] += d[q];
        if (proj) {
            double m = wmean(n, w, x);
            for (int64_t q = 0; q < n; ++q) x[q] -= m;
        }
        for (int64_t q = 0; q < n; ++q) x_out[unknown_to_array(g, op, q)] = x[q];
        orc_residual_ld(g, op, c, x_out, full_b, full_r, norms);
        ++psteps;
        if (!(norms[0] < 0.5 * prev)) break;
        prev = norms[0];
    }
    if (info) {
        info->iters = iters;
        info->polish_steps = psteps;
        info->polish_iters = piters;
        info->stagnated = stag;
        info->rel_residual = norms[1] > 0.0 ? norms[0] / norms[1] : 0.0;
        info->removed_mean = removed;
    }
    free(rp); free(ci); free(av); free(w); free(b); free(f); free(x); free(d);
    free(full_b); free(full_r);
    return 0;
}

/* Weighted mean sum(W x)/sum(W) of a field in full layout (x over the
 * unknowns of op). */
double orc_weighted_mean(const orc_geom *g, int op, const double *x)
{
    int64_t n = n_unknowns(g, op);
    long double s = 0.0L, t = 0.0L;
    for (int64_t q = 0; q < n; ++q) {
        double wq = unknown_weight(g, op, q);
        s += (long double)wq * x[unknown_to_array(g, op, q)];
        t += wq;
    }
    return (double)(s / t);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
