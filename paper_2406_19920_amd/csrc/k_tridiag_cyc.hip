// Cyclic tridiagonal pencils of the triply periodic branch (Section 2.3.3,
// items S1 and S2 with y periodic too): the partitioned solve of
// tridiag.h with CYC = true, one shape per supported row count (the P
// chunks of M rows must hold the system exactly, since a cyclic system has
// no end at which padding rows could sit).
#include "tridiag.h"

namespace ibs {

template <typename T, typename R>
static hipError_t launch_cyclic(const JobSet &js, const TriParams &tp, int n, hipStream_t s)
{
    switch (n) {
    case 48: return launch_pm<T, R, 16, 3, true>(js, tp, s);
    case 64: return launch_pm<T, R, 16, 4, true>(js, tp, s);
    case 80: return launch_pm<T, R, 16, 5, true>(js, tp, s);
    case 96: return launch_pm<T, R, 32, 3, true>(js, tp, s);
    case 128: return launch_pm<T, R, 32, 4, true>(js, tp, s);
    case 160: return launch_pm<T, R, 32, 5, true>(js, tp, s);
    case 192: return launch_pm<T, R, 32, 6, true>(js, tp, s);
    case 256: return launch_pm<T, R, 32, 8, true>(js, tp, s);
    case 320: return launch_pm<T, R, 32, 10, true>(js, tp, s);
    case 384: return launch_pm<T, R, 32, 12, true>(js, tp, s);
    case 512: return launch_pm<T, R, 32, 16, true>(js, tp, s);
    default: return hipErrorInvalidValue;
    }
}

// cyclic_rows_supported() (the sizes above) is defined with the plan
// builder (host code).

hipError_t launch_cyclic_dd(const JobSet &js, const TriParams &tp, int n, hipStream_t s)
{
    return launch_cyclic<double, double>(js, tp, n, s);
}
hipError_t launch_cyclic_fd(const JobSet &js, const TriParams &tp, int n, hipStream_t s)
{
    return launch_cyclic<float, double>(js, tp, n, s);
}
hipError_t launch_cyclic_ff(const JobSet &js, const TriParams &tp, int n, hipStream_t s)
{
    return launch_cyclic<float, float>(js, tp, n, s);
}

}  // namespace ibs
