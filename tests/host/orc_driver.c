/* Host driver of the oracle for the sanitizer build: grids with walls or
 * periodic y, periodic x/z or walls in x and/or z (uniform or stretched),
 * every operator, inhomogeneous wall data, solves. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nx, ny, nz;
    double hx, hz;
    const double *dyc, *dyf;
    int py, wx, wz;
    const double *dxc, *dxf, *dzc, *dzf;
} orc_geom;
typedef struct {
    int iters, polish_steps, polish_iters, stagnated;
    double rel_residual, removed_mean;
} orc_info;
int orc_grid(int ny, double ly, double beta, const double *yf_in, double *yf, double *yc, double *dyc,
             double *dyf);
void orc_residual_bc_ld(const orc_geom *g, int op, double c, const double *x, const double *b,
                        const double *lo, const double *hi, double *r, double *norms);
int orc_solve(const orc_geom *g, int op, double c, const double *b, double *x, double tol, int maxit,
              orc_info *info);

int main(void)
{
    int bad = 0;
    for (int cfg = 0; cfg < 12; ++cfg) {
        /* 0..7: periodic y, walls in x, walls in z on the bits; 8..11: a
         * duct with stretched x, and z stretched too on bit 1 */
        const int py = cfg & 1;
        const int wx = cfg >= 8 ? 1 : (cfg >> 1) & 1, wz = cfg >= 8 ? 1 : (cfg >> 2) & 1;
        const int sx = cfg >= 8, sz = cfg >= 8 && ((cfg >> 1) & 1);
        const int nx = 6, ny = 7, nz = 5;
        double yf[8], yc[7], dyc[7], dyf[8];
        double xf[7], xc[6], dxc[6], dxf[7], zf[6], zc[5], dzc[5], dzf[6];
        if (orc_grid(ny, 1.0, 1.5, NULL, yf, yc, dyc, dyf)) return 1;
        if (orc_grid(nx, 1.0, 1.2, NULL, xf, xc, dxc, dxf)) return 1;
        if (orc_grid(nz, 1.0, 0.9, NULL, zf, zc, dzc, dzf)) return 1;
        if (py) dyf[0] = dyf[ny] = 0.5 * (dyc[0] + dyc[ny - 1]);
        orc_geom g = {nx, ny, nz, 1.0 / nx, 1.0 / nz, dyc, dyf, py, wx, wz,
                      sx ? dxc : NULL, sx ? dxf : NULL, sz ? dzc : NULL, sz ? dzf : NULL};
        const int nfull = nx * (ny + 1) * nz;
        double *b = calloc(nfull, sizeof(double)), *x = calloc(nfull, sizeof(double));
        double *r = calloc(nfull, sizeof(double)), *lo = calloc(nx * nz, sizeof(double));
        double *hi = calloc(nx * nz, sizeof(double));
        for (int q = 0; q < nfull; ++q) b[q] = sin(0.37 * q) + 0.1 * cos(1.3 * q);
        for (int q = 0; q < nx * nz; ++q) { lo[q] = 0.5 * sin(q); hi[q] = cos(q); }
        for (int op = 0; op < 4; ++op) {
            orc_info info;
            double norms[2];
            if (orc_solve(&g, op, op ? 1e-2 : 0.0, b, x, 1e-14, 100000, &info)) ++bad;
            orc_residual_bc_ld(&g, op, op ? 1e-2 : 0.0, x, b, py ? NULL : lo, py ? NULL : hi, r, norms);
            printf("py %d wx %d wz %d sx %d sz %d op %d iters %d rel %.3g\n", py, wx, wz, sx, sz, op,
                   info.iters, info.rel_residual);
            if (!(info.rel_residual < 1e-12)) ++bad;
        }
        free(b); free(x); free(r); free(lo); free(hi);
    }
    return bad;
}
