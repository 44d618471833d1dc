/* Host driver of the oracle for the sanitizer build: grids with walls or
 * periodic y, periodic x/z or walls in x and/or z, every operator,
 * inhomogeneous wall data, solves. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nx, ny, nz;
    double hx, hz;
    const double *dyc, *dyf;
    int py, wx, wz;
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
    for (int cfg = 0; cfg < 8; ++cfg) {
        const int py = cfg & 1, wx = (cfg >> 1) & 1, wz = (cfg >> 2) & 1;
        const int nx = 6, ny = 7, nz = 5;
        double yf[8], yc[7], dyc[7], dyf[8];
        if (orc_grid(ny, 1.0, 1.5, NULL, yf, yc, dyc, dyf)) return 1;
        if (py) dyf[0] = dyf[ny] = 0.5 * (dyc[0] + dyc[ny - 1]);
        orc_geom g = {nx, ny, nz, 1.0 / nx, 1.0 / nz, dyc, dyf, py, wx, wz};
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
            printf("py %d wx %d wz %d op %d iters %d rel %.3g\n", py, wx, wz, op, info.iters, info.rel_residual);
            if (!(info.rel_residual < 1e-12)) ++bad;
        }
        free(b); free(x); free(r); free(lo); free(hi);
    }
    return bad;
}
