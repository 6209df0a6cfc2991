// Host construction of the uniform scatterer grid (counting sort by cell).
#include "scatter_grid.h"

#include <algorithm>

#ifndef UR_GRID_ITEMS_PER_CELL
#define UR_GRID_ITEMS_PER_CELL 2.0   // mean scatterers per cell (before the capture-ball overlap); the walk
                                     // tests a cell's items four at a time, so fuller cells pay off
#endif

namespace ur {

ScatterGrid build_scatter_grid(const double *box, const double *scat, long n_scat, double r_s, double margin,
                               const RxCone *rx) {
    ScatterGrid g;
    const double r = r_s + margin;
    // the scatterers kept and the bounding box of their grown capture balls
    std::vector<char> keep((size_t)n_scat, 1);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long i = 0; i < n_scat; ++i) {
        const double *p = scat + 4 * i;
        if (rx && !rx_may_hear(*rx, p, r)) {
            keep[(size_t)i] = 0;
            continue;
        }
        ++g.kept;
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k] - r - margin);
            hi[k] = std::max(hi[k], p[k] + r + margin);
        }
    }
    double ext[3], vol = 1.0;
    for (int k = 0; k < 3; ++k) {
        lo[k] = std::max(lo[k], box[k] - margin);
        hi[k] = std::min(hi[k], box[3 + k] + margin);
        if (!(hi[k] > lo[k])) {   // nothing kept: one empty cell over the box
            lo[k] = box[k];
            hi[k] = box[3 + k];
        }
        ext[k] = hi[k] - lo[k];
        vol *= ext[k];
    }
    const double rho = g.kept > 0 ? (double)g.kept / vol : 1.0 / vol;
    const double h_min = std::max(4.0 * r_s, std::cbrt(vol / (double)(1 << 24)) * 1.0001);
    double h = std::max(std::cbrt(UR_GRID_ITEMS_PER_CELL / rho), h_min);
    // The kept scatterers may fill only part of their bounding box (a convex
    // array hears a thin curved slab): then the cells they occupy hold many
    // more than the mean.  Cells shrink until the occupied ones hold about
    // UR_GRID_ITEMS_PER_CELL registrations on average.
    for (int pass = 0; pass < 4 && g.kept > 0 && h > h_min; ++pass) {
        int n[3];
        for (int k = 0; k < 3; ++k) n[k] = std::max(1, (int)std::ceil(ext[k] / h));
        std::vector<int> count((size_t)n[0] * n[1] * n[2], 0);
        long regs = 0, occupied = 0;
        for (long i = 0; i < n_scat; ++i) {
            if (!keep[(size_t)i]) continue;
            const double *p = scat + 4 * i;
            int a[3], b[3];
            for (int k = 0; k < 3; ++k) {
                a[k] = std::max(0, (int)std::floor((p[k] - r - lo[k]) / h));
                b[k] = std::min(n[k] - 1, (int)std::floor((p[k] + r - lo[k]) / h));
            }
            for (int z = a[2]; z <= b[2]; ++z)
                for (int y = a[1]; y <= b[1]; ++y)
                    for (int x = a[0]; x <= b[0]; ++x) {
                        occupied += count[((size_t)z * n[1] + y) * n[0] + x]++ == 0;
                        ++regs;
                    }
        }
        const double mean = occupied > 0 ? (double)regs / (double)occupied : 0.0;
        if (!(mean > 1.5 * UR_GRID_ITEMS_PER_CELL)) break;
        h = std::max(h_min, h * std::cbrt(UR_GRID_ITEMS_PER_CELL / mean));
    }
    for (int k = 0; k < 3; ++k) {
        g.info.lo[k] = lo[k];
        g.info.n[k] = std::max(1, (int)std::ceil(ext[k] / h));
    }
    g.info.h = h;
    g.info.inv_h = 1.0 / h;
    // Every cone of a linear array lies in the wedge |y| <= z tan(alpha_c):
    // its axis is +z through a point with y = 0.  A convex array's cones have
    // tilted axes in the xz-plane, so each lies in the slab
    // |y| <= tan(alpha_c) (s - R), s the distance of the point from the centre
    // of curvature: |y| <= |q - c| sin(alpha) <= tan(alpha) (q - c).n
    // <= tan(alpha_c) (s - R), with (q - c).n = (x, z + R).n - R <= s - R.
    // The walks are clipped to the wedge (wy_b) or the slab (cv_r, cv_tan);
    // the 10 um margin wy_a dwarfs the rounding of a capture point and of the
    // clip itself.
    g.info.wy_a = 1e-5;
    g.info.wy_b = rx && rx->radius == 0.0 && rx->alpha_c < 80.0 * M_PI / 180.0
                      ? std::tan(rx->alpha_c) * (1.0 + 1e-9) : -1.0;
    g.info.cv_r = rx && rx->radius > 0.0 && rx->alpha_c < 80.0 * M_PI / 180.0 ? rx->radius : 0.0;
    g.info.cv_tan = g.info.cv_r > 0.0 ? std::tan(rx->alpha_c) * (1.0 + 1e-9) : 0.0;
    const long cells = (long)g.info.n[0] * g.info.n[1] * g.info.n[2];
    g.cell_start.assign(cells + 1, 0);
    auto range = [&](const double *p, int k, int &a, int &b) {
        a = (int)std::floor((p[k] - r - g.info.lo[k]) * g.info.inv_h);
        b = (int)std::floor((p[k] + r - g.info.lo[k]) * g.info.inv_h);
        a = std::max(a, 0);
        b = std::min(b, g.info.n[k] - 1);
    };
    auto for_cells = [&](const double *p, auto &&fn) {
        int a[3], b[3];
        for (int k = 0; k < 3; ++k) range(p, k, a[k], b[k]);
        for (int z = a[2]; z <= b[2]; ++z)
            for (int y = a[1]; y <= b[1]; ++y)
                for (int x = a[0]; x <= b[0]; ++x) fn((long)(z * g.info.n[1] + y) * g.info.n[0] + x);
    };
    for (long i = 0; i < n_scat; ++i)
        if (keep[(size_t)i]) for_cells(scat + 4 * i, [&](long c) { ++g.cell_start[c + 1]; });
    for (long c = 0; c < cells; ++c) g.cell_start[c + 1] += g.cell_start[c];
    g.items.resize(g.cell_start[cells]);
    std::vector<int> fill(g.cell_start.begin(), g.cell_start.end() - 1);
    for (long i = 0; i < n_scat; ++i)
        if (keep[(size_t)i]) for_cells(scat + 4 * i, [&](long c) { g.items[fill[c]++] = (int)i; });
    return g;
}

}  // namespace ur
