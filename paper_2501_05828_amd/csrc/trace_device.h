// Device-side geometry and sampling shared by the trace kernel and the
// path-replay adjoint: RNG draws, FP32 conservative box culling, FP64
// primitive tests, interface fractions, receive directivity, the emission
// map and ray emission.
#pragma once
#include "philox.h"
#include "ur_internal.h"

namespace ur {
namespace dev {

// counter = (ray, element | tx << 16, segment | purpose << 16, k); with the
// synthetic-aperture scheme every transmit draws as transmit 0
__device__ __forceinline__ void draw(const TraceParams &P, uint32_t ray, int e, int tx, int seg, uint32_t purpose,
                                     uint32_t k, uint32_t out[4]) {
    const uint32_t txr = P.sa ? 0u : (uint32_t)tx;
    philox4x32_10(ray, (uint32_t)e | (txr << 16), (uint32_t)seg | (purpose << 16), k, P.key0, P.key1, out);
}

__device__ __forceinline__ double u01(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

__device__ __forceinline__ double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ------------------------------------------------------------- FP32 culling
struct CullRay {
    float ox, oy, oz, ix, iy, iz;
};

// FP32 reciprocal for the culling slab tests: the hardware estimate (about
// 1 ulp).  Over a 0.3 m scene it moves a slab plane along the ray by under
// 0.1 um, far inside the 1 um dilation of the boxes.
__device__ __forceinline__ float safe_inv(double d) {
    const float a = fabs(d) < 1e-20 ? copysignf(1e-20f, (float)d) : (float)d;
    return __builtin_amdgcn_rcpf(a);
}

// Attenuation factor of a ray weight.  Weights decide nothing (every
// decision uses positions, times and random numbers), so the factor is
// evaluated in FP32: relative error ~1e-7 per factor against the 1e-4
// tolerance of the channel data.
__device__ __forceinline__ double atten(double x) { return (double)expf((float)x); }

__device__ __forceinline__ CullRay make_cull(const double *o, const double *d) {
    CullRay c;
    c.ox = (float)o[0];
    c.oy = (float)o[1];
    c.oz = (float)o[2];
    c.ix = safe_inv(d[0]);
    c.iy = safe_inv(d[1]);
    c.iz = safe_inv(d[2]);
    return c;
}

// conservative upper bound of an FP64 ray parameter for the FP32 box test
__device__ __forceinline__ float cull_tmax(double t) { return (float)(t * (1.0 + 1e-6) + 1e-6); }

struct Node {
    float4 lo, hi;
};

__device__ __forceinline__ Node load_node(const BvhNode *nodes, int i) {
    const float4 *p = reinterpret_cast<const float4 *>(nodes + i);
    return Node{p[0], p[1]};
}

__device__ __forceinline__ bool slab(const Node &n, const CullRay &r, float tmax) {
    const float tx0 = (n.lo.x - r.ox) * r.ix, tx1 = (n.hi.x - r.ox) * r.ix;
    const float ty0 = (n.lo.y - r.oy) * r.iy, ty1 = (n.hi.y - r.oy) * r.iy;
    const float tz0 = (n.lo.z - r.oz) * r.iz, tz1 = (n.hi.z - r.oz) * r.iz;
    const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
    return tn <= tf;
}

__device__ __forceinline__ int node_skip(const Node &n) { return __float_as_int(n.lo.w); }
__device__ __forceinline__ int node_leaf(const Node &n) { return __float_as_int(n.hi.w); }

// ---------------------------------------------------------- FP64 primitives
// Moller-Trumbore with precomputed edges e1 = v1 - v0, e2 = v2 - v0.  The
// barycentric tests compare the numerators against the determinant (sign
// aware), so only accepted hits pay for the division.
__device__ __forceinline__ bool tri_isect(const double *tr, const double *o, const double *d, double &t) {
    const double *v0 = tr, *e1 = tr + 3, *e2 = tr + 6;
    const double p0 = d[1] * e2[2] - d[2] * e2[1];
    const double p1 = d[2] * e2[0] - d[0] * e2[2];
    const double p2 = d[0] * e2[1] - d[1] * e2[0];
    const double det = e1[0] * p0 + e1[1] * p1 + e1[2] * p2;
    if (det == 0.0) return false;
    const double t0 = o[0] - v0[0], t1 = o[1] - v0[1], t2 = o[2] - v0[2];
    const double un = t0 * p0 + t1 * p1 + t2 * p2;
    // the bounds tests for either sign of det, as one test on the values
    // multiplied by sign(det) (exact), so lanes of both signs share one path
    const double sg = det > 0.0 ? 1.0 : -1.0, ad = fabs(det), us = un * sg;
    if (us < 0.0 || us > ad) return false;
    const double q0 = t1 * e1[2] - t2 * e1[1];
    const double q1 = t2 * e1[0] - t0 * e1[2];
    const double q2 = t0 * e1[1] - t1 * e1[0];
    const double vn = d[0] * q0 + d[1] * q1 + d[2] * q2;
    const double vs = vn * sg;
    if (vs < 0.0 || (un + vn) * sg > ad) return false;
    t = (e2[0] * q0 + e2[1] * q1 + e2[2] * q2) / det;
    return true;
}

// Elements a transducer-sampling target is drawn from for capture point q
// (Sec. 2.3): all E, or with the cone-restricted choice the K whose centre
// x_e = (e - (E-1)/2) pitch satisfies |x_e - q_x| <= rho, rho^2 = q_z^2
// tan^2(alpha_c) - q_y^2 (Eq. 13 is zero for the others), the interval
// widened by a relative 1e-9 so that rounding never drops an element.
// Convex array: q at distance s > R from the centre of curvature, at angle
// psi about it and elevation y.  The cosine of the angle between q - c(phi)
// and the normal at phi grows with c = cos(psi - phi) (c >= R/s) and equals
// cos(alpha_c) at c* = (R sin^2 alpha_c + cos alpha_c sqrt(s^2 + y^2 -
// R^2 sin^2 alpha_c)) / s, so the elements that can hear q have
// |phi_e - psi| <= acos(c*) (none if c* > 1), widened the same way.
// Returns false when no element is left.
template <bool CONVEX = true>
__device__ __forceinline__ bool elem_range(const TraceParams &P, double qx, double qy, double qz, int &e_lo,
                                           int &n_e) {
    e_lo = 0;
    n_e = P.E;
    if (P.elem_choice != UR_ELEMENT_CONE) return true;
    const double half = 0.5 * (double)(P.E - 1);
    double lo, hi;
    if (CONVEX && P.convex) {
        const double R = P.radius, zc = qz + P.radius;
        const double sq = sqrt(qx * qx + zc * zc), sa = P.sin_alpha_c, ca = P.cos_alpha_c;
        if (!(sq > R)) return false;
        const double cs = (R * sa * sa + ca * sqrt(sq * sq + qy * qy - R * R * sa * sa)) / sq;
        if (!(cs <= 1.0)) return false;
        const double dl = acos(cs) * (1.0 + 1e-9) + 1e-12, psi = atan2(qx, zc);
        lo = ceil((psi - dl) / P.dphi + half);
        hi = floor((psi + dl) / P.dphi + half);
    } else {
        const double tc = P.tan_alpha_c;
        const double rho2 = qz * qz * tc * tc - qy * qy;
        if (!(qz > 0.0 && rho2 >= 0.0)) return false;
        const double rho = sqrt(rho2) * (1.0 + 1e-9) + 1e-12;
        lo = ceil((qx - rho) / P.pitch + half);
        hi = floor((qx + rho) / P.pitch + half);
    }
    lo = lo < 0.0 ? 0.0 : lo;
    hi = hi > (double)(P.E - 1) ? (double)(P.E - 1) : hi;
    if (hi < lo) return false;
    e_lo = (int)lo;
    n_e = (int)hi - e_lo + 1;
    return true;
}

// Rough boundaries (Eq. 12).  Orthonormal basis (t, b) completing a unit n:
// the branch-free construction of Duff et al., "Building an Orthonormal
// Basis, Revisited" (JCGT 6(1), 2017).
__device__ __forceinline__ void onb(const double *n, double *t, double *b) {
    const double sg = copysign(1.0, n[2]);
    const double a = -1.0 / (sg + n[2]);
    const double c = n[0] * n[1] * a;
    t[0] = 1.0 + sg * n[0] * n[0] * a;
    t[1] = sg * c;
    t[2] = -sg * n[0];
    b[0] = c;
    b[1] = sg + n[1] * n[1] * a;
    b[2] = -n[1];
}

// Microfacet normal about n with density D(h) (n.h), D the GGX distribution
// of Eq. 12: tan^2(theta_h) = alpha^2 xi1 / (1 - xi1), phi_h = 2 pi xi2
// (Walter et al. 2007, Eqs. 35-36).
__device__ __forceinline__ void ggx_sample(const double *n, double alpha, double xi1, double xi2, double *h) {
    double t[3], b[3];
    onb(n, t, b);
    const double q = 1.0 - xi1 + alpha * alpha * xi1;
    const double ct = sqrt((1.0 - xi1) / q), st = alpha * sqrt(xi1 / q);
    double sp, cp;
    sincos(2.0 * M_PI * xi2, &sp, &cp);
    for (int i = 0; i < 3; ++i) h[i] = st * cp * t[i] + st * sp * b[i] + ct * n[i];
}

// Smith masking of the GGX distribution at cos(theta_v) = v.n > 0 (Walter et
// al. 2007, Eq. 34).
__device__ __forceinline__ double ggx_g1(double alpha, double cv) {
    const double tan2 = (1.0 - cv * cv) / (cv * cv);
    return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));
}

// A rough boundary's scattering toward direction o as implied by the
// sampler of after_hit (transducer sampling at rough boundaries).  wi = -d,
// n the normal on the incident side, z1 incident and z2 far impedance,
// eta = z1 / z2.  The microfacet normal sending wi to o is wi + o when o is
// on the incident side (reflection), else +-(eta wi + o) (refraction about
// it, Eq. 9), normalised with n.h > 0.  The sampler draws h with density
// D(h) (n.h) (Eq. 12), reflects with the Fresnel probability R_h of Eq. 11
// about h and maps h to o with |dh/do| = 1 / (4 |o.h|) or
// |o.h| / (eta wi.h + o.h)^2 (Walter et al. 2007).  pdf receives the
// direction density D (n.h) P J (P = R_h or 1 - R_h); the result,
// f |n.o| = (wi.h) G1(wi) G1(o) D P J / (n.wi), is the sampler's weight
// times pdf.  Zero for directions the sampler cannot produce.
__device__ __forceinline__ double rough_fcos(const double *wi, const double *n, double z1, double z2, double alpha,
                                             const double *o, double &pdf) {
    pdf = 0.0;
    const double cni = dot3(wi, n), cno = dot3(o, n), eta = z1 / z2;
    if (!(cni > 0.0) || cno == 0.0) return 0.0;
    const bool refl = cno > 0.0;
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = refl ? wi[k] + o[k] : eta * wi[k] + o[k];
    const double hl = sqrt(dot3(h, h));
    if (!(hl > 0.0)) return 0.0;
    const double sg = dot3(h, n) < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) h[k] = h[k] * sg / hl;
    const double ci = dot3(wi, h), co = dot3(o, h), chn = dot3(h, n);
    if (!(ci > 0.0) || !(chn > 0.0)) return 0.0;
    if (refl ? !(co > 0.0) : !(co < 0.0)) return 0.0;
    const double rad = 1.0 - eta * eta * (1.0 - ci * ci);
    double Rh = 1.0;
    if (rad >= 0.0) {
        const double ct = sqrt(rad), den = z1 * ci + z2 * ct;
        if (den != 0.0) {
            const double A = (z1 * ci - z2 * ct) / den;
            Rh = A * A;
        }
    }
    const double Pl = refl ? Rh : 1.0 - Rh;
    double J;
    if (refl) {
        J = 1.0 / (4.0 * co);
    } else {
        const double den = eta * ci + co;
        if (den == 0.0) return 0.0;
        J = -co / (den * den);
    }
    const double a2 = alpha * alpha, q = chn * chn * (a2 - 1.0) + 1.0;
    const double D = a2 / (M_PI * q * q);
    pdf = D * chn * Pl * J;
    return ci * ggx_g1(alpha, cni) * ggx_g1(alpha, fabs(cno)) * D * Pl * J / cni;
}

// Unit geometric normal of triangle k, computed once on the host in FP64
__device__ __forceinline__ void tri_normal(const TraceParams &P, int64_t k, double *n) {
    const double4 v = P.tri_n[k];
    n[0] = v.x;
    n[1] = v.y;
    n[2] = v.z;
}

__device__ __forceinline__ bool sph_roots(const double *s, const double *o, const double *d, double &t0,
                                          double &t1) {
    const double oc[3] = {o[0] - s[0], o[1] - s[1], o[2] - s[2]};
    const double b = dot3(oc, d);
    const double c = dot3(oc, oc) - s[3] * s[3];
    const double disc = b * b - c;
    if (disc < 0.0) return false;
    const double sq = sqrt(disc);
    t0 = -b - sq;
    t1 = -b + sq;
    return true;
}

__device__ __forceinline__ bool pln_isect(const double *p, const double *o, const double *d, double &t) {
    const double den = dot3(p, d);
    if (den == 0.0) return false;
    t = (p[3] - dot3(p, o)) / den;
    return true;
}

// Transmitted intensity fraction 1 - A_r^2 (Eqs. 8, 11) of a straight crossing.
__device__ __forceinline__ double transmit_fraction(double z1, double z2, double cos_r) {
    const double eta = z1 / z2;
    const double rad = 1.0 - eta * eta * (1.0 - cos_r * cos_r);
    if (rad < 0.0) return 0.0;
    const double cos_t = sqrt(rad);
    const double den = z1 * cos_r + z2 * cos_t;
    if (den == 0.0) return 0.0;
    const double A = (z1 * cos_r - z2 * cos_t) / den;
    return 1.0 - A * A;
}

// Receive directivity, Eq. 13.
__device__ __forceinline__ double directivity(double al, double am, double ac) {
    al = fabs(al);
    if (al > ac) return 0.0;
    if (al <= am) return 1.0;
    return (ac - al) / (ac - am);
}

// sin and cos of |x| <= pi/4 by their Taylor series in x^2 through x^17 and
// x^16 (truncation below 1e-17 relative on this range), Horner form.
__device__ __forceinline__ void sincos_quarter(double x, double &sn, double &cs) {
    const double y = x * x;
    double ps = 1.0 / 355687428096000.0;               //  1/17!
    ps = fma(ps, y, -1.0 / 1307674368000.0);           // -1/15!
    ps = fma(ps, y, 1.0 / 6227020800.0);               //  1/13!
    ps = fma(ps, y, -1.0 / 39916800.0);                // -1/11!
    ps = fma(ps, y, 1.0 / 362880.0);                   //  1/9!
    ps = fma(ps, y, -1.0 / 5040.0);                    // -1/7!
    ps = fma(ps, y, 1.0 / 120.0);                      //  1/5!
    ps = fma(ps, y, -1.0 / 6.0);                       // -1/3!
    sn = fma(ps * y, x, x);
    double pc = 1.0 / 20922789888000.0;                //  1/16!
    pc = fma(pc, y, -1.0 / 87178291200.0);             // -1/14!
    pc = fma(pc, y, 1.0 / 479001600.0);                //  1/12!
    pc = fma(pc, y, -1.0 / 3628800.0);                 // -1/10!
    pc = fma(pc, y, 1.0 / 40320.0);                    //  1/8!
    pc = fma(pc, y, -1.0 / 720.0);                     // -1/6!
    pc = fma(pc, y, 1.0 / 24.0);                       //  1/4!
    pc = fma(pc, y, -0.5);                             // -1/2!
    cs = fma(pc, y, 1.0);
}

// Equal-area square -> hemisphere map: Shirley-Chiu concentric disk, then
// the area-preserving lift z = 1 - r^2, xy scaled by sqrt(2 - r^2).  The disk
// angle is (pi/4) u or pi/2 - (pi/4) u with |u| <= 1.
__device__ __forceinline__ void hemisphere(double a, double b, double *d) {
    const double sa = 2.0 * a - 1.0, sb = 2.0 * b - 1.0;
    if (sa == 0.0 && sb == 0.0) {
        d[0] = 0.0;
        d[1] = 0.0;
        d[2] = 1.0;
        return;
    }
    // one quotient and one polynomial pair for either half of the square, so
    // the lanes of a wavefront do not run both
    const bool xa = fabs(sa) > fabs(sb);
    const double r = xa ? sa : sb, q = xa ? sb : sa;
    double s1, c1;
    sincos_quarter((M_PI / 4.0) * (q / r), s1, c1);
    const double sp = xa ? s1 : c1, cp = xa ? c1 : s1;   // cos(pi/2 - x) = sin x
    const double r2 = r * r, sc = sqrt(2.0 - r2);
    d[0] = r * cp * sc;
    d[1] = r * sp * sc;
    d[2] = 1.0 - r2;
}

// Emission (Eqs. 4 and 6): origin uniform on the element face, direction from
// the uniform or tabulated proposal on the equal-area map, weight
// cos(theta) / (rays per transmit * pdf).  On a convex array the face is the
// element's arc, angle phi = (e - (E-1)/2 + u0 - 1/2) dphi about the centre
// of curvature (0, 0, -R), and the direction is drawn in the frame of the
// outward normal there: tangent (cos phi, 0, -sin phi), y, normal
// (sin phi, 0, cos phi).  CONVEX = false: a kernel variant for linear arrays.
template <bool CONVEX = true>
__device__ __forceinline__ void emit(const TraceParams &P, int tx, int e, uint32_t ray, double *o, double *d,
                                     double &w, int &cell_out) {
    uint32_t x[4];
    draw(P, ray, e, tx, 0, 0, 0, x);
    const double u0 = u01(x[0]), u1 = u01(x[1]), u2 = u01(x[2]), u3 = u01(x[3]);
    double sp = 0.0, cp = 1.0;
    if (CONVEX && P.convex) {
        const double ph = ((double)e - 0.5 * (double)(P.E - 1) + (u0 - 0.5)) * P.dphi, h = sin(0.5 * ph);
        sincos(ph, &sp, &cp);
        o[0] = P.radius * sp;
        o[2] = -2.0 * P.radius * h * h;
    } else {
        o[0] = P.xe[e] + (u0 - 0.5) * P.pitch;
        o[2] = 0.0;
    }
    o[1] = (u1 - 0.5) * P.elev;
    double ca, cb, pdf;
    if (!P.proposal) {
        ca = u2;
        cb = u3;
        pdf = 1.0 / (2.0 * M_PI);
        cell_out = (int)((x[3] >> 27) * 32u + (x[2] >> 27));   // floor(32 u3) * 32 + floor(32 u2)
    } else {
        uint32_t y[4];
        draw(P, ray, e, tx, 0, 3, 0, y);
        const double uc = u01(y[0]);
        const int64_t row = ((int64_t)tx * P.E + e) * kCells;
        const float *cdf = P.cdf + row;
        int lo = 0, hi = kCells;                 // first cell with uc <= cdf[cell]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (uc <= (double)cdf[mid]) hi = mid;
            else lo = mid + 1;
        }
        const int cell = lo < kCells ? lo : kCells - 1;
        cell_out = cell;
        ca = ((double)(cell % 32) + u2) / 32.0;
        cb = ((double)(cell / 32) + u3) / 32.0;
        pdf = (double)P.pdf[row + cell] * (double)kCells / (2.0 * M_PI);
    }
    hemisphere(ca, cb, d);
    w = d[2] / (P.n_per_tx * pdf);
    if (CONVEX && P.convex) {
        const double hx = d[0], hz = d[2];
        d[0] = hx * cp + hz * sp;
        d[2] = hz * cp - hx * sp;
    }
}

}  // namespace dev
}  // namespace ur
