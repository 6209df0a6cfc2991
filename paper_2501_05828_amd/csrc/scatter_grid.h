// Uniform grid over the scene box for scatterer capture queries, and the
// 3D digital-differential-analyser walk (Amanatides & Woo, 1987) along a
// ray segment.  Plain C++ usable from host code and from HIP device code.
//
// Each scatterer is registered in every cell that its capture ball, grown by
// a small margin, overlaps.  The walk hands each pierced cell the interval
// [ta, tb) of ray parameters spent in it; consecutive intervals share their
// end points, so the intervals partition [0, t_end) exactly and a capture
// whose projection parameter s lies in [ta, tb) is reported in that cell
// only -- every capture is found exactly once.
#pragma once
#include <cmath>
#include <vector>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define UR_HD __host__ __device__ __forceinline__
#else
#define UR_HD inline
#endif

namespace ur {

struct GridInfo {
    double lo[3];       // grid origin (box minimum)
    double h, inv_h;    // cell edge [m]
    int n[3];           // cells per axis
};

// Visits the cells pierced by o + t d for t in [0, t_end) in order.  visit
// returns false to stop early.  Returns the number of cells visited.  Axis
// state is kept in scalars (no dynamically indexed arrays) so that device
// code keeps it in registers.
template <class F>
UR_HD int dda_walk(const GridInfo &g, const double *o, const double *d, double t_end, F &&visit) {
    const double h = g.h;
    int cx = (int)floor((o[0] - g.lo[0]) * g.inv_h);
    int cy = (int)floor((o[1] - g.lo[1]) * g.inv_h);
    int cz = (int)floor((o[2] - g.lo[2]) * g.inv_h);
    cx = cx < 0 ? 0 : (cx > g.n[0] - 1 ? g.n[0] - 1 : cx);
    cy = cy < 0 ? 0 : (cy > g.n[1] - 1 ? g.n[1] - 1 : cy);
    cz = cz < 0 ? 0 : (cz > g.n[2] - 1 ? g.n[2] - 1 : cz);
    const int sx = d[0] > 0.0 ? 1 : (d[0] < 0.0 ? -1 : 0);
    const int sy = d[1] > 0.0 ? 1 : (d[1] < 0.0 ? -1 : 0);
    const int sz = d[2] > 0.0 ? 1 : (d[2] < 0.0 ? -1 : 0);
    const double ix = sx ? 1.0 / d[0] : 0.0, iy = sy ? 1.0 / d[1] : 0.0, iz = sz ? 1.0 / d[2] : 0.0;
    // parameter at which the ray crosses the next cell face on each axis
    double tmx = sx ? (g.lo[0] + (double)(cx + (sx > 0)) * h - o[0]) * ix : INFINITY;
    double tmy = sy ? (g.lo[1] + (double)(cy + (sy > 0)) * h - o[1]) * iy : INFINITY;
    double tmz = sz ? (g.lo[2] + (double)(cz + (sz > 0)) * h - o[2]) * iz : INFINITY;
    const int nx = g.n[0], nxy = g.n[0] * g.n[1];
    int cell = cz * nxy + cy * nx + cx;
    const int limit = g.n[0] + g.n[1] + g.n[2] + 3;
    double ta = 0.0;
    int visited = 0;
    while (true) {
        const bool ax = tmx <= tmy && tmx <= tmz;
        const bool ay = !ax && tmy <= tmz;
        const double tn = ax ? tmx : (ay ? tmy : tmz);
        const double tb = tn < t_end ? tn : t_end;
        ++visited;
        if (tb > ta && !visit(cell, ta, tb)) break;
        if (tb >= t_end || visited >= limit) break;
        if (ax) {
            cx += sx;
            if (cx < 0 || cx >= g.n[0]) break;
            cell += sx;
            tmx = (g.lo[0] + (double)(cx + (sx > 0)) * h - o[0]) * ix;
        } else if (ay) {
            cy += sy;
            if (cy < 0 || cy >= g.n[1]) break;
            cell += sy * nx;
            tmy = (g.lo[1] + (double)(cy + (sy > 0)) * h - o[1]) * iy;
        } else {
            cz += sz;
            if (cz < 0 || cz >= g.n[2]) break;
            cell += sz * nxy;
            tmz = (g.lo[2] + (double)(cz + (sz > 0)) * h - o[2]) * iz;
        }
        if (tb > ta) ta = tb;
    }
    return visited;
}

// Host build: cell edge chosen for about half a scatterer per cell (never
// below four capture radii), at most 2^24 cells.
struct ScatterGrid {
    GridInfo info;
    std::vector<int> cell_start;   // [cells + 1]
    std::vector<int> items;        // scatterer indices, grouped by cell
};

ScatterGrid build_scatter_grid(const double *box, const double *scat, long n_scat, double r_s, double margin);

}  // namespace ur
