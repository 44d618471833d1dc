// Multi-grid batches: the device job table of the stage kernels
// (k_multigrid.hip) and the host builder's view of it.
#pragma once
#include "ibs_internal.h"

namespace ibs {

// One field (a Poisson solve, or one Helmholtz component) of a multi-grid
// batch, as the stage kernels read it from device memory.  in: the rhs
// ([nz][rows][nx]); out: the solution (also the buffer of the transformed
// field between the z transforms); work: a field-sized scratch array.
struct MgField {
    const double *in;
    double *out;
    double *work;
    double *cpt;                 // the pencils' forward factors [nz][rows][nx] (library-owned, built once)
    const double *xfwd, *xinv;   // swizzled nx x nx B operands: Q, G^T
    const double *zfwd, *zinv;   // swizzled nz x nz A operands: Q^T, G
    const double *lam_x, *lam_z; // eigenvalues of the field's x / z kinds
    const double *lo, *di, *up;  // y rows of the field's kind [rows]
    const double *wy;            // Delta_j [ny]
    ibs_solve_info *info;        // or null
    double c;                    // Helmholtz coefficient (Poisson: 0)
    double inv_sqrt_nxnz;
    int nx, ny, nz, rows, kind, poisson;
};

enum { MG_X_FWD = 0, MG_Z_FWD, MG_TRI, MG_Z_INV, MG_X_INV, MG_STAGES };
constexpr int MG_FACTOR = MG_STAGES;  // set-up launch: the pencils' factors into cpt (tridiagonal work list)
constexpr int MG_MAX_BLOCKS = 2048;   // persistent grid: at most 8 blocks per CU
constexpr int MG_WM = 2;              // transform tiles: 16 MG_WM rows x 64 columns per wave

hipError_t launch_multigrid_stage(int stage, const MgField *fields, const int4 *items, int nitems,
                                  hipStream_t s);

// Swizzled plain (unfolded) transform table of a plan's x or z kind, built
// from its host bases: x forward Q, x inverse G^T (B operands), z forward
// Q^T, z inverse G (A operands).
void plain_transform_table(const Plan &p, bool z_axis, int kind, bool inverse, std::vector<double> &out);

}  // namespace ibs
