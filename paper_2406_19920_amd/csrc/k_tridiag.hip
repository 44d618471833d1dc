// Tridiagonal solves along y: launch-shape selection and the entry points
// (the kernel and its per-shape launcher are in tridiag.h; the cyclic
// shapes of the triply periodic branch are instantiated in
// k_tridiag_cyc.hip).
#include "tridiag.h"

namespace ibs {

template <typename T, typename R>
static hipError_t launch_by_rows(const JobSet &js, const TriParams &tp, int n, hipStream_t s)
{
    // lanes per pencil and rows per lane: short chunks keep the per-lane
    // arrays in registers
    if (n <= 48) return launch_pm<T, R, 16, 3>(js, tp, s);
    if (n <= 80) return launch_pm<T, R, 16, 5>(js, tp, s);
    if (n <= 112) return launch_pm<T, R, 16, 7>(js, tp, s);
    if (n <= 144) return launch_pm<T, R, 16, 9>(js, tp, s);
    if (n <= 224) return launch_pm<T, R, 32, 7>(js, tp, s);
    if (n <= 256) return launch_pm<T, R, 32, 8>(js, tp, s);
    if (n <= 288) return launch_pm<T, R, 32, 9>(js, tp, s);
    if (n <= 352) return launch_pm<T, R, 32, 11>(js, tp, s);
    if (n <= 416) return launch_pm<T, R, 32, 13>(js, tp, s);
    if (n <= 544) return launch_pm<T, R, 32, 17>(js, tp, s);
    if (n <= 672) return launch_pm<T, R, 32, 21>(js, tp, s);
    if (n <= 800) return launch_pm<T, R, 32, 25>(js, tp, s);
    return hipErrorInvalidValue;
}

// Upper bound on the condition number of every Helmholtz pencil matrix
// (1 - c s) I - c T_kind of the jobs: its eigenvalues lie in
// [1, 1 + c (max|s| + Gershgorin bound of -T)].
static double helmholtz_kappa(const JobSet &js, const Plan &p)
{
    double smax = 0.0;
    for (int xk = 0; xk < NUM_XK; ++xk)
        for (double v : p.lam_x[xk]) smax = std::max(smax, -v);
    double szmax = 0.0;
    for (int zk = 0; zk < NUM_XK; ++zk)
        for (double v : p.lam_z[zk]) szmax = std::max(szmax, -v);
    double kap = 1.0;
    for (int q = 0; q < js.n; ++q) {
        const int kd = js.j[q].kind;
        double g = 0.0;
        for (size_t j = 0; j < p.di[kd].size(); ++j)
            g = std::max(g, std::fabs(p.lo[kd][j]) + std::fabs(p.di[kd][j]) + std::fabs(p.up[kd][j]));
        kap = std::max(kap, 1.0 + std::fabs(js.j[q].c) * (smax + szmax + g));
    }
    return kap;
}

// Launch shape by system size: padded partitions, or (periodic y) the
// cyclic shapes, which need the exact row count.
template <typename T, typename R>
static hipError_t launch_rows(const Plan &p, const JobSet &js, const TriParams &tp, int n, hipStream_t s)
{
    if (p.py) {
        if constexpr (sizeof(T) == 8) return launch_cyclic_dd(js, tp, n, s);
        else if constexpr (sizeof(R) == 8) return launch_cyclic_fd(js, tp, n, s);
        else return launch_cyclic_ff(js, tp, n, s);
    }
    return launch_by_rows<T, R>(js, tp, n, s);
}

template <typename T>
static hipError_t launch_tridiag(const JobSet &js, const Plan &p, const State &st, bool poisson, int pass,
                                 hipStream_t s)
{
    TriParams tp;
    for (int xk = 0; xk < NUM_XK; ++xk) tp.lam_x[xk] = blob_ptr(p, p.lay.lam_x[xk]);
    for (int zk = 0; zk < NUM_XK; ++zk) tp.lam_z[zk] = blob_ptr(p, p.lay.lam_z[zk]);
    for (int kd = 0; kd < NUM_KINDS; ++kd) {
        tp.lo[kd] = blob_ptr(p, p.lay.lo[kd]);
        tp.di[kd] = blob_ptr(p, p.lay.di[kd]);
        tp.up[kd] = blob_ptr(p, p.lay.up[kd]);
    }
    tp.wy = blob_ptr(p, p.lay.wy);
    tp.bmean = st.bmean;
    tp.xsum = nullptr;
    tp.record_mean = 1;
    tp.skip = nullptr;
    tp.wsum_y = 0.0;
    for (int j = 0; j < p.ny; ++j) tp.wsum_y += p.dyc[j];
    tp.nx = p.nx;
    tp.nz = p.nz;
    tp.poisson = poisson ? 1 : 0;
    tp.nxsum = residual_tiles(p);
    if (pass > 0) {
        tp.record_mean = 0;
        tp.xsum = st.xsum;
    }
    if (pass >= 2) tp.skip = st.done;
    tp.inv_sqrt_nxnz = 1.0 / std::sqrt((double)p.nx * (double)p.nz);
    tp.lane_mask = nullptr;
    tp.lane_list = nullptr;
    tp.lane_len = 0;
    tp.lane_mode = 0;
    // refined path (FP32 data): the first pass records the partial maxima
    // the residual scale is taken from; later passes steer in its units
    tp.bmax = (sizeof(T) == 4 && pass == 0) ? st.bmax : nullptr;
    tp.scale = (sizeof(T) == 4 && pass > 0) ? st.scale : nullptr;
    int n = 0;
    for (int q = 0; q < js.n; ++q) {
        const int rows = js.j[q].rows - skip_first_row(js.j[q].kind);   // system rows
        n = rows > n ? rows : n;
    }
    // FP32 arithmetic where its rounding is far below what refinement
    // removes anyway: FP32 data (refined path), Helmholtz, and pencil
    // condition numbers bounded by FP32_KAPPA.
    if constexpr (sizeof(T) == 4) {
        if (!poisson && helmholtz_kappa(js, p) <= FP32_KAPPA) return launch_rows<T, float>(p, js, tp, n, s);
        if (poisson && p.lane_len > 0) {
            // pressure pencils: FP32 arithmetic on every tile but the FP64
            // lane's, then FP64 arithmetic on the lane's tiles (disjoint
            // pencils; the lane holds the singular (0,0) pencil and every
            // pencil whose condition bound exceeds LANE64_KAPPA)
            tp.lane_mask = reinterpret_cast<const unsigned *>(blob_ptr(p, p.lay.lane_mask));
            tp.lane_list = reinterpret_cast<const int *>(blob_ptr(p, p.lay.lane_list));
            tp.lane_len = p.lane_len;
            tp.lane_mode = 1;
            hipError_t e = launch_rows<T, float>(p, js, tp, n, s);
            if (e != hipSuccess) return e;
            tp.lane_mode = 2;
            return launch_rows<T, double>(p, js, tp, n, s);
        }
    }
    return launch_rows<T, double>(p, js, tp, n, s);
}

hipError_t launch_tridiag_f64(const JobSet &js, const Plan &p, const State &st, bool poisson, hipStream_t s)
{
    return launch_tridiag<double>(js, p, st, poisson, 0, s);
}

hipError_t launch_tridiag_f32(const JobSet &js, const Plan &p, const State &st, bool poisson, int pass,
                              hipStream_t s)
{
    return launch_tridiag<float>(js, p, st, poisson, pass, s);
}

}  // namespace ibs
