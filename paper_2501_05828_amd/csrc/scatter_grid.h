// Uniform grid for scatterer capture queries, and the 3D digital-
// differential-analyser walk (Amanatides & Woo, 1987) along a ray segment.
// Plain C++ usable from host code and from HIP device code.
//
// Each scatterer is registered in every cell that its capture ball, grown by
// a small margin, overlaps.  The grid covers the bounding box of the
// registered balls only; a segment is first clipped to that box (no capture
// point lies outside it).  The walk hands each pierced cell the interval
// [ta, tb) of ray parameters spent in it; consecutive intervals share their
// end points, so the intervals partition the clipped segment exactly and a
// capture whose projection parameter s lies in [ta, tb) is reported in that
// cell only -- every capture is found exactly once.
//
// Scatterers that no receiving element can hear (Eq. 13 is zero for every
// point of their capture ball and every element) may be left out of the grid:
// each of their captures would yield a zero-valued secondary ray, and a
// capture changes nothing else on the path.  For the same reason the walk may
// be clipped to a wedge around the acceptance cones: a capture point outside
// every cone yields a zero-valued secondary ray too.
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
    // acceptance wedge |y| <= wy_a + wy_b z that holds every point some
    // element can hear (the walk is clipped to it); wy_b < 0: no wedge
    double wy_a, wy_b;
    // convex array (cv_r > 0): a point at distance s from the centre of
    // curvature (0, 0, -cv_r) that some element hears has
    // |y| <= wy_a + cv_tan (s - cv_r); s is convex along a segment, so each
    // walk is clipped to |y| <= wy_a + cv_tan (max of s at its ends - cv_r)
    double cv_r, cv_tan;
};

// Receiving aperture for the audibility cull: element centres on the x axis
// within [x_lo, x_hi] at y = z = 0, normals +z, or on a convex arc, and the
// acceptance half-angle alpha_c (Eq. 13 is zero beyond it).
struct RxCone {
    double x_lo, x_hi, alpha_c;       // linear array: element centres on [x_lo, x_hi] of the x axis, facing +z
    double radius = 0.0;              // convex array: arc radius (centre of curvature (0, 0, -radius)) ...
    double phi_lo = 0.0, phi_hi = 0.0; // ... and the angles of its end elements' centres
};

// Whether some point within distance r of p lies in the acceptance cone of an
// element centred anywhere on [x_lo, x_hi] (a superset of the elements, so a
// false answer is final).  The distance from p to the cone with apex a is
// that of the point (axial h, radial rho) to the half-line at angle alpha_c
// from the axis, and rho is smallest at the apex nearest in x.
//
// Convex array: apexes on the arc at angle phi in [phi_lo, phi_hi], axes
// radial.  For a point at distance s > R from the centre of curvature and at
// angle psi about it, both the angle to the axis of the apex at phi and the
// distance to that apex grow with |psi - phi| (d/dc of (s c - R) / |q - a| is
// s (s (s - R c) + y^2) / |q - a|^3 > 0, c = cos(psi - phi)), so the nearest
// cone is the one whose apex angle is nearest psi.  Points within r + R of
// the centre are kept.
inline bool rx_may_hear(const RxCone &rx, const double *p, double r) {
    if (!(rx.alpha_c < 0.5 * M_PI)) return true;
    const double ca = std::cos(rx.alpha_c), sa = std::sin(rx.alpha_c);
    double h, rho;
    if (rx.radius > 0.0) {
        const double R = rx.radius, zc = p[2] + R;
        if (std::hypot(p[0], zc) <= R + r) return true;
        double ph = std::atan2(p[0], zc);
        ph = ph < rx.phi_lo ? rx.phi_lo : (ph > rx.phi_hi ? rx.phi_hi : ph);
        const double sp = std::sin(ph), cp = std::cos(ph);
        const double vx = p[0] - R * sp, vz = zc - R * cp;
        h = vx * sp + vz * cp;
        rho = std::hypot(vx * cp - vz * sp, p[1]);
    } else {
        const double xa = p[0] < rx.x_lo ? rx.x_lo : (p[0] > rx.x_hi ? rx.x_hi : p[0]);
        rho = std::hypot(p[0] - xa, p[1]);
        h = p[2];
    }
    if (h * ca + rho * sa >= 0.0) return rho * ca - h * sa <= r;
    return std::hypot(h, rho) <= r;
}

// Cell-by-cell walker.  After init(), the ray is in cell `cell` for the
// parameter interval [ta, bound(t_end)); step() moves to the next pierced
// cell (false once the ray leaves the grid).  Axis state is kept in scalars
// (no dynamically indexed arrays) so device code keeps it in registers.
struct DdaIter {
    int cx, cy, cz, sx, sy, sz, cell;
    double ix, iy, iz, tmx, tmy, tmz, ta;

    // Clips [0, t_end) to the grid box and enters the cell of the entry
    // point; false if the segment misses the box.  t_hi receives the end of
    // the clipped interval, ta its start.
    UR_HD bool init(const GridInfo &g, const double *o, const double *d, double t_end, double &t_hi) {
        sx = d[0] > 0.0 ? 1 : (d[0] < 0.0 ? -1 : 0);
        sy = d[1] > 0.0 ? 1 : (d[1] < 0.0 ? -1 : 0);
        sz = d[2] > 0.0 ? 1 : (d[2] < 0.0 ? -1 : 0);
        ix = sx ? 1.0 / d[0] : 0.0;
        iy = sy ? 1.0 / d[1] : 0.0;
        iz = sz ? 1.0 / d[2] : 0.0;
        double t0 = 0.0, t1 = t_end;
        const int s3[3] = {sx, sy, sz};
        const double i3[3] = {ix, iy, iz};
        for (int k = 0; k < 3; ++k) {
            const double lo = g.lo[k], hi = g.lo[k] + (double)g.n[k] * g.h;
            if (s3[k]) {
                const double a = (lo - o[k]) * i3[k], b = (hi - o[k]) * i3[k];
                t0 = fmax(t0, fmin(a, b));
                t1 = fmin(t1, fmax(a, b));
            } else if (!(o[k] >= lo && o[k] <= hi)) {
                return false;
            }
        }
        if (g.wy_b >= 0.0 || g.cv_r > 0.0) {
            // the two half-spaces +-y - wb z - wa <= 0 along the ray: the
            // linear array's wedge, or the convex array's slab of this segment
            double wa = g.wy_a, wb = g.wy_b;
            if (g.cv_r > 0.0) {
                if (!(t0 < t1)) return false;
                const double za = o[2] + g.cv_r + t0 * d[2], zb = o[2] + g.cv_r + t1 * d[2];
                const double xa = o[0] + t0 * d[0], xb = o[0] + t1 * d[0];
                const double s = fmax(sqrt(xa * xa + za * za), sqrt(xb * xb + zb * zb));
                wa += g.cv_tan * fmax(0.0, s - g.cv_r);
                wb = 0.0;
            }
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double c0 = (double)sgn * o[1] - wb * o[2] - wa;
                const double c1 = (double)sgn * d[1] - wb * d[2];
                if (c1 > 0.0) t1 = fmin(t1, -c0 / c1);
                else if (c1 < 0.0) t0 = fmax(t0, -c0 / c1);
                else if (c0 > 0.0) return false;
            }
        }
        if (!(t0 < t1)) return false;
        t_hi = t1;
        const double px = o[0] + t0 * d[0], py = o[1] + t0 * d[1], pz = o[2] + t0 * d[2];
        cx = (int)floor((px - g.lo[0]) * g.inv_h);
        cy = (int)floor((py - g.lo[1]) * g.inv_h);
        cz = (int)floor((pz - g.lo[2]) * g.inv_h);
        cx = cx < 0 ? 0 : (cx > g.n[0] - 1 ? g.n[0] - 1 : cx);
        cy = cy < 0 ? 0 : (cy > g.n[1] - 1 ? g.n[1] - 1 : cy);
        cz = cz < 0 ? 0 : (cz > g.n[2] - 1 ? g.n[2] - 1 : cz);
        // parameter at which the ray crosses the next cell face on each axis
        tmx = sx ? (g.lo[0] + (double)(cx + (sx > 0)) * g.h - o[0]) * ix : INFINITY;
        tmy = sy ? (g.lo[1] + (double)(cy + (sy > 0)) * g.h - o[1]) * iy : INFINITY;
        tmz = sz ? (g.lo[2] + (double)(cz + (sz > 0)) * g.h - o[2]) * iz : INFINITY;
        cell = (cz * g.n[1] + cy) * g.n[0] + cx;
        ta = t0;
        return true;
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

// Visits the cells pierced by o + t d for t in [0, t_end) (clipped to the
// grid box) in order, with the interval [ta, tb) spent in each (empty
// intervals skipped).  visit returns false to stop early.  Returns the number
// of cells stepped through.
template <class F>
UR_HD int dda_walk(const GridInfo &g, const double *o, const double *d, double t_end, F &&visit) {
    DdaIter it;
    double t_hi;
    if (!it.init(g, o, d, t_end, t_hi)) return 0;
    const int limit = g.n[0] + g.n[1] + g.n[2] + 3;
    int visited = 0;
    while (true) {
        const double tb = it.bound(t_hi);
        ++visited;
        if (tb > it.ta && !visit(it.cell, it.ta, tb)) break;
        if (tb >= t_hi || visited >= limit) break;
        if (!it.step(g, o, tb)) break;
    }
    return visited;
}

// Host build over the bounding box of the registered capture balls (within
// the scene box grown by the margin): cell edge chosen for about two
// registered scatterers per cell (never below four capture radii), at most
// 2^24 cells.  With rx, scatterers whose capture ball (grown by the margin)
// no element can hear are left out, and walks are clipped to the wedge
// |y| <= z tan(alpha_c) + 10 um around the acceptance cones (alpha_c < 80
// degrees).
struct ScatterGrid {
    GridInfo info;
    std::vector<int> cell_start;   // [cells + 1]
    std::vector<int> items;        // scatterer indices, grouped by cell
    long kept = 0;                 // scatterers registered
};

ScatterGrid build_scatter_grid(const double *box, const double *scat, long n_scat, double r_s, double margin,
                               const RxCone *rx = nullptr);

}  // namespace ur
