// Host-only driver of the plan builder for the sanitizer build (address and
// undefined-behaviour checks): builds plans for valid and invalid grids of
// both precisions, both y conditions and periodic or wall-bounded x and z
// (uniform or stretched), and walks every table.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "ibs_internal.h"

namespace ibs {
ibs_status build_plan(const ibs_grid_desc &d, Plan *&out);
void set_error(const std::string &msg) { (void)msg; }
}  // namespace ibs

using namespace ibs;

int main()
{
    struct Case { int nx, ny, nz; double beta; int prec, py, expect_ok, wx = 0, wz = 0, st = 0; };
    const std::vector<Case> cases = {
        {32, 24, 16, 2.0, IBS_FP64, 0, 1},  {64, 64, 64, 0.0, IBS_REFINED_BF16X3, 0, 1},
        {96, 33, 32, 3.0, IBS_REFINED_BF16X3, 0, 1}, {48, 2, 80, 1.0, IBS_FP64, 0, 1},
        {64, 48, 32, 0.0, IBS_REFINED_BF16X3, 1, 1}, {32, 160, 64, 2.0, IBS_FP64, 1, 1},
        {512, 5, 64, 2.0, IBS_REFINED_BF16X3, 0, 1}, {16, 2, 16, 0.0, IBS_FP64, 0, 1},
        {24, 16, 32, 0.0, IBS_FP64, 0, 0},  {32, 100, 32, 0.0, IBS_FP64, 1, 0},
        {48, 16, 64, 0.0, IBS_REFINED_BF16X3, 0, 0}, {32, 1, 32, 0.0, IBS_FP64, 0, 0},
        {64, 40, 32, 1.5, IBS_FP64, 0, 1, 1, 0}, {96, 24, 64, 2.0, IBS_REFINED_BF16X3, 0, 1, 0, 1},
        {64, 48, 64, 0.0, IBS_REFINED_BF16X3, 1, 1, 1, 1}, {48, 17, 80, 1.0, IBS_FP64, 0, 1, 1, 1},
        // stretched x (st bit 0) and z (bit 1); the last one along a periodic x
        {64, 20, 32, 1.5, IBS_FP64, 0, 1, 1, 0, 1}, {96, 24, 64, 2.0, IBS_REFINED_BF16X3, 0, 1, 1, 1, 3},
        {32, 16, 32, 0.0, IBS_FP64, 0, 0, 0, 1, 1}};
    int bad = 0;
    for (const Case &c : cases) {
        ibs_grid_desc d{};
        d.nx = c.nx; d.ny = c.ny; d.nz = c.nz; d.beta = c.beta;
        d.bc_x = c.wx ? IBS_DIRICHLET : IBS_PERIODIC;
        d.bc_z = c.wz ? IBS_DIRICHLET : IBS_PERIODIC;
        d.bc_y_vel = c.py ? IBS_PERIODIC : IBS_DIRICHLET;
        d.bc_y_p = c.py ? IBS_PERIODIC : IBS_NEUMANN;
        d.precision = c.prec;
        // tanh-graded faces of a stretched axis
        auto faces = [](int n, double beta) {
            std::vector<double> f(n + 1);
            for (int i = 0; i <= n; ++i)
                f[i] = 0.5 * (1.0 + std::tanh(beta * (2.0 * i / n - 1.0)) / std::tanh(beta));
            return f;
        };
        const std::vector<double> xf = faces(c.nx, 1.3), zf = faces(c.nz, 0.9);
        if (c.st & 1) d.x_faces = xf.data();
        if (c.st & 2) d.z_faces = zf.data();
        Plan *p = nullptr;
        const ibs_status st = build_plan(d, p);
        if ((st == IBS_OK) != (c.expect_ok != 0)) {
            std::printf("unexpected status %d for %dx%dx%d\n", (int)st, c.nx, c.ny, c.nz);
            ++bad;
        }
        if (p) {
            double sum = 0.0;
            for (unsigned char b : p->blob) sum += b;
            for (int k = 0; k < NUM_KINDS; ++k)
                for (size_t j = 0; j < p->di[k].size(); ++j) sum += p->lo[k][j] + p->di[k][j] + p->up[k][j];
            std::printf("plan %dx%dx%d blob %zu bytes, lane %d, checksum %.6g\n", c.nx, c.ny, c.nz,
                        p->blob.size(), p->lane_len, sum);
            delete p;
        }
    }
    return bad;
}
