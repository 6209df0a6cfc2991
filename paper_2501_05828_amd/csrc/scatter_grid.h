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

// Cell-by-cell walker.  After init(), the ray is in cell `cell` for the
// parameter interval [ta, bound(t_end)); step() moves to the next pierced
// cell (false once the ray leaves the grid).  Axis state is kept in scalars
// (no dynamically indexed arrays) so device code keeps it in registers.
struct DdaIter {
    int cx, cy, cz, sx, sy, sz, cell;
    double ix, iy, iz, tmx, tmy, tmz, ta;

    UR_HD void init(const GridInfo &g, const double *o, const double *d) {
        cx = (int)floor((o[0] - g.lo[0]) * g.inv_h);
        cy = (int)floor((o[1] - g.lo[1]) * g.inv_h);
        cz = (int)floor((o[2] - g.lo[2]) * g.inv_h);
        cx = cx < 0 ? 0 : (cx > g.n[0] - 1 ? g.n[0] - 1 : cx);
        cy = cy < 0 ? 0 : (cy > g.n[1] - 1 ? g.n[1] - 1 : cy);
        cz = cz < 0 ? 0 : (cz > g.n[2] - 1 ? g.n[2] - 1 : cz);
        sx = d[0] > 0.0 ? 1 : (d[0] < 0.0 ? -1 : 0);
        sy = d[1] > 0.0 ? 1 : (d[1] < 0.0 ? -1 : 0);
        sz = d[2] > 0.0 ? 1 : (d[2] < 0.0 ? -1 : 0);
        ix = sx ? 1.0 / d[0] : 0.0;
        iy = sy ? 1.0 / d[1] : 0.0;
        iz = sz ? 1.0 / d[2] : 0.0;
        // parameter at which the ray crosses the next cell face on each axis
        tmx = sx ? (g.lo[0] + (double)(cx + (sx > 0)) * g.h - o[0]) * ix : INFINITY;
        tmy = sy ? (g.lo[1] + (double)(cy + (sy > 0)) * g.h - o[1]) * iy : INFINITY;
        tmz = sz ? (g.lo[2] + (double)(cz + (sz > 0)) * g.h - o[2]) * iz : INFINITY;
        cell = (cz * g.n[1] + cy) * g.n[0] + cx;
        ta = 0.0;
    }
    UR_HD double bound(double t_end) const {
        const double tn = fmin(tmx, fmin(tmy, tmz));
        return tn < t_end ? tn : t_end;
    }
    // Moves to the next cell; the interval start becomes the previous bound.
    UR_HD bool step(const GridInfo &g, const double *o, double tb) {
        if (tmx <= tmy && tmx <= tmz) {
            cx += sx;
            if (cx < 0 || cx >= g.n[0]) return false;
            cell += sx;
            tmx = (g.lo[0] + (double)(cx + (sx > 0)) * g.h - o[0]) * ix;
        } else if (tmy <= tmz) {
            cy += sy;
            if (cy < 0 || cy >= g.n[1]) return false;
            cell += sy * g.n[0];
            tmy = (g.lo[1] + (double)(cy + (sy > 0)) * g.h - o[1]) * iy;
        } else {
            cz += sz;
            if (cz < 0 || cz >= g.n[2]) return false;
            cell += sz * g.n[0] * g.n[1];
            tmz = (g.lo[2] + (double)(cz + (sz > 0)) * g.h - o[2]) * iz;
        }
        if (tb > ta) ta = tb;
        return true;
    }
};

// Visits the cells pierced by o + t d for t in [0, t_end) in order, with
// the interval [ta, tb) spent in each (empty intervals skipped).  visit
// returns false to stop early.  Returns the number of cells stepped through.
template <class F>
UR_HD int dda_walk(const GridInfo &g, const double *o, const double *d, double t_end, F &&visit) {
    DdaIter it;
    it.init(g, o, d);
    const int limit = g.n[0] + g.n[1] + g.n[2] + 3;
    int visited = 0;
    while (true) {
        const double tb = it.bound(t_end);
        ++visited;
        if (tb > it.ta && !visit(it.cell, it.ta, tb)) break;
        if (tb >= t_end || visited >= limit) break;
        if (!it.step(g, o, tb)) break;
    }
    return visited;
}

// Host build: cell edge chosen for about two scatterers per cell (never
// below four capture radii), at most 2^24 cells.
struct ScatterGrid {
    GridInfo info;
    std::vector<int> cell_start;   // [cells + 1]
    std::vector<int> items;        // scatterer indices, grouped by cell
};

ScatterGrid build_scatter_grid(const double *box, const double *scat, long n_scat, double r_s, double margin);

}  // namespace ur
